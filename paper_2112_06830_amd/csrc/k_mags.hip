// Fused magnitudes: SED tile = W . SSP on MFMA, then attenuation and the
// redshifted filter integrals in registers (Section 2.1 Eqs. cspdeftheta and
// full_mdf; Section 3.4 Eqs. attenuation-uvbump; Section 2.2.1 Eq. restmag).
// The SED never reaches memory: each workgroup reduces its 128 x 128
// (wavelength x galaxy) tile straight into per-galaxy band sums.
//
// GEMM orientation: rows (M) are rest wavelengths, columns (N) are galaxies,
// the contraction (K) runs over (metallicity, age) bins.  With this choice an
// MFMA output lane holds one galaxy and 16 wavelengths, so per-galaxy dust and
// redshift parameters sit in registers and the wavelength reduction is mostly
// lane-local.  Both operands are K-contiguous rows in memory (ST[l][k] and
// W[g][k]); each lane feeds MFMA from one 16-byte LDS read per operand per
// k-run.
//
// Exactness of the tiling: a galaxy's sums do not depend on which galaxies
// share its tile.  K blocks skipped for the tile are zero for every member,
// wavelength chunks outside a galaxy's window have zero transmission, and
// chunk boundaries are fixed on the global wavelength grid, so every galaxy
// sees the same floating-point operations in the same order.
#include "gemm_core.hpp"

namespace dsps {


// Blocks are dispatched round-robin over the 8 XCDs by linear id.  All
// wavelength groups of one galaxy tile go to the same XCD (its W tile then
// stays in that XCD's L2): block b runs on XCD b % 8 and takes tile
// (b / 8 / G) * 8 + b % 8, group (b / 8) % G.
__device__ __forceinline__ void xcd_tile_group(int b, int groups, int &tile, int &group) {
  const int xcd = b & 7, slot = b >> 3;
  tile = (slot / groups) * 8 + xcd;
  group = slot % groups;
}

// Per-galaxy sums of one chunk, reduced over the two lane halves and the two
// row-waves of each column block, written to the chunk's partial slot.
__device__ __forceinline__ void write_chunk_partial(float (&num)[2][DSPS_MAX_BAND],
                                                   float (&den)[2][DSPS_MAX_BAND], int n_band,
                                                   float *s_red, int wr, int wc, int lane,
                                                   int nvalid, float *out_base, int stride) {
  const int h = lane >> 5;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int b = 0; b < DSPS_MAX_BAND; ++b) {
      num[nb][b] += __shfl_xor(num[nb][b], 32, 64);
      den[nb][b] += __shfl_xor(den[nb][b], 32, 64);
    }
  // Lane half h finishes column block nb = h.  Every array index below is a
  // compile-time constant (a runtime-selected index would move the
  // accumulators to scratch memory).
  const int col = h * 32 + (lane & 31);
  float *red = s_red + (wc * 64 + col) * (2 * DSPS_MAX_BAND);
  if (wr == 1) {
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      if (h == nb) {
#pragma unroll
        for (int b = 0; b < DSPS_MAX_BAND; ++b) {
          red[b] = num[nb][b];
          red[DSPS_MAX_BAND + b] = den[nb][b];
        }
      }
    }
  }
  __syncthreads();
  if (wr == 0) {
    const int tcol = wc * 64 + col;
    if (tcol < nvalid) {
      float *out = out_base + (size_t)tcol * stride;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        if (h == nb) {
#pragma unroll
          for (int b = 0; b < DSPS_MAX_BAND; ++b) {
            if (b < n_band) {
              out[b] = num[nb][b] + red[b];
              out[n_band + b] = den[nb][b] + red[DSPS_MAX_BAND + b];
            }
          }
        }
      }
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(GEMM_THREADS, 2) void k_mags_gemm(MagsLaunch a) {
  using C = GemmCfg<PREC>;
  using elem = typename C::elem;
  __shared__ GemmSmem<PREC> sm;
  __shared__ float4 s_lc[TILE_L];
  __shared__ float s_q[TILE_L];
  __shared__ float s_red[2 * 64 * 2 * DSPS_MAX_BAND];
  __shared__ int s_tile[4];   // window lo, window hi, metallicity-row mask, age hi
  extern __shared__ float s_filt[];   // [n_band * n_pts]

  int tile, group;
  xcd_tile_group(blockIdx.x, a.n_groups, tile, group);
  const int n_tiles = (a.s_count + TILE_G - 1) / TILE_G;
  if (tile >= n_tiles) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int h = lane >> 5;
  const SspView P = a.ssp;        // by value: a reference into the kernel
  const FilterView F = a.flt;     // argument would force a private-memory copy
  const int n_band = F.n_band, n_pts = F.n_pts;
  const int g0 = tile * TILE_G;                 // first batch-local galaxy of the tile
  const int nvalid = min(TILE_G, a.s_count - g0);

  // ---- tile union of windows and non-zero weight blocks
  if (threadIdx.x == 0) { s_tile[0] = 1 << 30; s_tile[1] = 0; s_tile[2] = 0; s_tile[3] = 0; }
  __syncthreads();
  if (threadIdx.x < nvalid) {
    const GalaxyRange r = a.range[a.s_begin + g0 + threadIdx.x];
    atomicMin(&s_tile[0], r.win_lo);
    atomicMax(&s_tile[1], r.win_hi);
    if (r.age_hi > 0) {
      const int jl = r.met_lo_hi & 0xFFFF, jh = r.met_lo_hi >> 16;
      atomicOr(&s_tile[2], (int)(((1u << (jh + 1)) - 1u) & ~((1u << jl) - 1u)));
      atomicMax(&s_tile[3], r.age_hi);
    }
  }
  __syncthreads();
  const int win_lo = s_tile[0], win_hi = s_tile[1];
  const unsigned met_mask = (unsigned)s_tile[2];
  const int age_hi = s_tile[3];
  const int c_first = win_lo / TILE_L;
  const int c_last = max((win_hi + TILE_L - 1) / TILE_L, c_first);   // exclusive
  if (group == 0 && threadIdx.x == 0) a.tile_chunks[tile] = make_int2(c_first, c_last);
  // groups are aligned to the tile's own window: all but the last are full
  const int c_begin = c_first + group * CHUNKS_PER_GROUP;
  const int c_end = min(c_begin + CHUNKS_PER_GROUP, c_last);
  if (c_begin >= c_end) return;

  // ---- filters into LDS
  for (int i = threadIdx.x; i < n_band * n_pts; i += GEMM_THREADS) s_filt[i] = F.trans[i];

  // ---- per-galaxy parameters of this lane's two columns
  float zp1[2], da[2], dl[2], bp[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = wc * 64 + nb * 32 + (lane & 31);
    if (col < nvalid) {
      const GalaxyMeta m = a.meta[a.s_begin + g0 + col];
      zp1[nb] = m.zp1; da[nb] = m.dust_a; dl[nb] = m.delta; bp[nb] = m.bump;
    } else {
      zp1[nb] = 1.0f; da[nb] = 0.0f; dl[nb] = 0.0f; bp[nb] = 0.0f;
    }
  }
  float fw0[DSPS_MAX_BAND], finv[DSPS_MAX_BAND];
#pragma unroll
  for (int b = 0; b < DSPS_MAX_BAND; ++b) {
    if (b < n_band) { const float2 gr = F.grid[b]; fw0[b] = gr.x; finv[b] = gr.y; }
    else { fw0[b] = 0.0f; finv[b] = 0.0f; }
  }

  // ---- K steps: metallicity rows in met_mask x age blocks below age_hi
  const int n_ab = (age_hi + C::KT - 1) / C::KT;
  const int nk = __builtin_popcount(met_mask) * n_ab;
  const int j_first = met_mask ? __builtin_ctz(met_mask) : 0;
  const elem *st = PREC == DSPS_FP32 ? (const elem *)P.st32 : (const elem *)P.st16;
  const elem *w = (const elem *)a.w_pad;
  const int n_comp = 2 * n_band;
  float *part_tile = a.partial + (size_t)g0 * a.n_chunks * n_comp;

  for (int c = c_begin; c < c_end; ++c) {
    const int l0 = c * TILE_L;
    __syncthreads();
    if (threadIdx.x < TILE_L) {
      s_lc[threadIdx.x] = P.lconst[l0 + threadIdx.x];
      s_q[threadIdx.x] = P.qweight[l0 + threadIdx.x];
    }
    f32x16 acc[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

    StageRegs<PREC> regs;
    int j_cur = j_first, ab_cur = 0;    // K block of the stage held in regs
    if (nk > 0) load_stage<PREC>(regs, st, P.k_pad, l0, w, g0, a.s_count, j_cur * AGE_PAD);
    for (int ks = 0; ks < nk; ++ks) {
      __syncthreads();
      store_stage<PREC>(regs, sm);
      __syncthreads();
      if (ks + 1 < nk) {
        if (++ab_cur == n_ab) {
          ab_cur = 0;
          j_cur = __builtin_ctz(met_mask & ~((2u << j_cur) - 1u));
        }
        load_stage<PREC>(regs, st, P.k_pad, l0, w, g0, a.s_count, j_cur * AGE_PAD + ab_cur * C::KT);
      }
      mma_stage(sm, wr, wc, lane, acc);
    }
    __syncthreads();   // s_lc / s_q / filters visible

    // ---- epilogue: attenuation x resampled transmission, lane-local sums
    float num[2][DSPS_MAX_BAND], den[2][DSPS_MAX_BAND];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int b = 0; b < DSPS_MAX_BAND; ++b) { num[nb][b] = 0.0f; den[nb][b] = 0.0f; }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const float4 lc = s_lc[row];   // (lambda, log2(lambda/5500), k0, drude shape)
        const float q = s_q[row];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const float powl = exp2f(dl[nb] * lc.y);
          const float att = exp2f(da[nb] * (lc.z * powl + bp[nb] * lc.w));
          const float lq = acc[mb][nb][r] * att * q;
          const float lobs = zp1[nb] * lc.x;
#pragma unroll
          for (int b = 0; b < DSPS_MAX_BAND; ++b) {
            if (b < n_band) {
              const float t = filter_at(s_filt + b * n_pts, n_pts, (lobs - fw0[b]) * finv[b]);
              num[nb][b] += t * lq;
              den[nb][b] += t * q;
            }
          }
        }
      }
    }
    write_chunk_partial(num, den, n_band, s_red, wr, wc, lane, nvalid,
                        part_tile + (size_t)c * n_comp, a.n_chunks * n_comp);
  }
}

int launch_mags_gemm(const MagsLaunch &a, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  const int n_tiles = (a.s_count + TILE_G - 1) / TILE_G;
  const int blocks = (n_tiles + 7) / 8 * 8 * a.n_groups;
  const size_t lds = sizeof(float) * a.flt.n_band * a.flt.n_pts;
  ProfScope prof(DSPS_KERNEL_MAGS_GEMM, stream);
  if (a.precision == DSPS_BF16)
    hipLaunchKernelGGL(k_mags_gemm<DSPS_BF16>, dim3(blocks), dim3(GEMM_THREADS), lds, stream, a);
  else
    hipLaunchKernelGGL(k_mags_gemm<DSPS_FP32>, dim3(blocks), dim3(GEMM_THREADS), lds, stream, a);
  return hip_fail(hipGetLastError(), "k_mags_gemm launch");
}

// Sum the per-chunk partial band sums in chunk order and form magnitudes
// m = -2.5 log10(num / (AB0 den)) + [D_mod(z) - 2.5 log10(1+z)] in float64.
__global__ void k_mags_finalize(FinalizeLaunch a) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= a.s_count) return;
  const int s = a.s_begin + local;
  const int g = a.perm ? a.perm[s] : s;
  const int nb = a.n_band, nc = 2 * nb;
  const int2 cr = a.tile_chunks[local / TILE_G];
  const float *p = a.partial + (size_t)local * a.n_chunks * nc;
  const double offset = a.mag_offset[s];
  for (int b = 0; b < nb; ++b) {
    float num = 0.0f, den = 0.0f;
    for (int c = cr.x; c < cr.y; ++c) {
      num += p[c * nc + b];
      den += p[c * nc + nb + b];
    }
    double m;
    if (den == 0.0f) m = __builtin_nan("");
    else m = -2.5 * log10((double)num / (AB_ZERO_POINT * (double)den)) + offset;
    a.mags[(size_t)g * nb + b] = (float)m;
    if (a.bands) {
      a.bands[(size_t)g * nc + b] = num;
      a.bands[(size_t)g * nc + nb + b] = den;
    }
  }
}

int launch_mags_finalize(const FinalizeLaunch &a, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  ProfScope prof(DSPS_KERNEL_MAGS_FINALIZE, stream);
  hipLaunchKernelGGL(k_mags_finalize, dim3((a.s_count + 255) / 256), dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "k_mags_finalize launch");
}

}  // namespace dsps
