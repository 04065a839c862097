// Unfused composite SED: L[g, l] = sum_k W[g, k] L_SSP[k, l] (Section 2.1,
// Eqs. cspdeftheta and full_mdf), optionally times the attenuation F_att
// (Section 3.4, Eq. attenuation), written to memory in the rest frame.  With
// the ionization axis (NEB; Section 3.3, Eq. nebsed) the sum also runs over
// the ionization points the tile's galaxies reach, each galaxy's weight row
// scaled by its weight of the point as it is staged; with ion_tangent the
// weights are replaced by their derivatives in the distribution's centre or
// width, which gives the SED's derivative (the sum is linear in them).
//
// AGED (Section 3.4.1, Eq. agedep_dust_csp): the age-major table and weight
// rows, the stage list grouped by the ages that share dust parameters, and
// the attenuation folded after each group (AgeFold), so the output is already
// attenuated.
//
// Galaxies come in the ordering sort's order, so a tile's members share few
// metallicity rows and ages: the K loop runs over the tile's stage list (the
// weight blocks non-zero for some member), as in the fused kernel.  Skipped
// blocks are zero for every member, so a galaxy's result does not depend on
// its tile.
#include "gemm_core.hpp"

namespace dsps {

template <int PREC, bool NEB = false, bool AGED = false>
__global__ __launch_bounds__(GEMM_THREADS, 2) void k_sed_gemm(SedLaunch a) {
  using C = GemmCfg<PREC>;
  using elem = typename C::elem;
  static_assert(!(NEB || AGED) || PREC == DSPS_FP32, "float32 only");
  static_assert(!(NEB && AGED), "not both");
  __shared__ float4 s_lc[AGED ? TILE_L : 1];
  __shared__ GemmSmem<PREC> sm[2];
  __shared__ float s_pn[NEB ? DSPS_MAX_ION * TILE_G : 1];
  // byte offsets (A, B) of each thread's 16-byte piece of every stage
  __shared__ int2 s_piece[4 * (AGED ? MAX_AGED_UNITS : MAX_UNITS) / GemmCfg<PREC>::UNITS];
  const int chunk = a.n_sel ? a.chunk_list[blockIdx.x] : (int)blockIdx.x;
  const int tile = blockIdx.y;
  const int live = live_in_range(a.n_live, a.g_begin, a.g_count);
  if (tile * TILE_G >= live) return;   // the whole workgroup: no barrier has run
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave & 1, wc = wave >> 1, h = lane >> 5;
  const SspView P = a.ssp;
  const int l0 = chunk * TILE_L;
  const int g0 = tile * TILE_G;
  const elem *st = AGED ? (const elem *)P.sa32
                        : (PREC == DSPS_FP32 ? (const elem *)P.st32 : (const elem *)P.st16);
  const int k_cols = AGED ? AGE_K : P.k_pad;
  const int a_stride = NEB ? P.k_row : k_cols;
  const int nvalid = min(TILE_G, live - g0);
  const GemmOps<PREC> ops =
      gemm_ops<PREC>(st, (size_t)P.n_wave_pad * a_stride, a_stride, linear_rows<PREC>(l0),
                     (const elem *)a.w_pad + (size_t)g0 * k_cols, nvalid, k_cols);
  const int ucol = stage_col();
  auto unit = [&](int s) {
    const int2 p = s_piece[STAGE_UNITS * s + ucol];
    return UnitSrc{p.x, p.y, nullptr};
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const TilePlan *pl = a.plan + tile;
  const int nk = pl->nk;
  for (int t = threadIdx.x; t < STAGE_UNITS * nk; t += blockDim.x)
    s_piece[t] = piece_bytes<PREC>(unit_piece<PREC>(pl->koff, t / STAGE_UNITS, t % STAGE_UNITS));
  if constexpr (NEB) {
    // every member's weight of each of the tile's ionization points
    const int u_lo = pl->u_lo, n_uu = pl->u_hi - pl->u_lo + 1;
    for (int t = threadIdx.x; t < n_uu * TILE_G; t += blockDim.x) {
      const int uu = t / TILE_G, col = t - uu * TILE_G;
      float f = 0.0f;
      if (col < nvalid) {
        const GalaxyIon gi = a.ion[a.g_begin + g0 + col];
        const int u = u_lo + uu;
        const double c = gi.lgu, sg = gi.sigma_u;
        f = (float)(a.ion_tangent == 1   ? ion_weight_d<1>(P.ion_edges, u, c, sg)
                    : a.ion_tangent == 2 ? ion_weight_d<2>(P.ion_edges, u, c, sg)
                                         : ion_weight(P.ion_edges, u, c, sg));
      }
      s_pn[t] = f;
    }
    __syncthreads();
    const int kp = P.k_pad;
    gemm_kloop<PREC>(sm, ops, nk * n_uu,
                     [&](int s) {
                       const int uu = s / nk;
                       const int2 p = s_piece[STAGE_UNITS * (s - uu * nk) + ucol];
                       return UnitSrc{(u_lo + uu) * kp * (int)sizeof(elem) + p.x, p.y,
                                      s_pn + uu * TILE_G};
                     },
                     wr, wc, lane, acc);
  } else if constexpr (AGED) {
    if (threadIdx.x < TILE_L) s_lc[threadIdx.x] = P.lconst[l0 + threadIdx.x];
    AgeFold af{pl->tag, a.age_young, a.age_old, a.dust_pivot, a.dust_width, P.lg_age, {}, {}, {}, {}, {}};
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int col = wc * 64 + nb * 32 + (lane & 31);
      float v[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      if (col < nvalid) {
        const int s = a.g_begin + g0 + col;
        const GalaxyMeta m = a.meta[s];
        const GalaxyDustOld d = a.dust_old[s];
        v[0] = m.dust_a; v[1] = m.delta; v[2] = d.dust_a; v[3] = d.delta; v[4] = m.bump;
      }
      af.da_y[nb] = v[0]; af.dl_y[nb] = v[1]; af.da_o[nb] = v[2]; af.dl_o[nb] = v[3];
      af.bp[nb] = v[4];
    }
    f32x16 sed[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) sed[mb][nb][r] = 0.0f;
    __syncthreads();
    gemm_kloop<PREC>(sm, ops, nk, unit, wr, wc, lane, acc,
                     [&](int ks) { af(ks, sed, acc, s_lc, wr, h); });
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = sed[mb][nb];
  } else {
    __syncthreads();
    gemm_kloop<PREC, PREC == DSPS_FP32>(sm, ops, nk, unit, wr, wc, lane, acc);
  }

#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = wc * 64 + nb * 32 + (lane & 31);
    if (col >= nvalid) continue;
    const int s = a.g_begin + g0 + col;     // sorted position
    float da = 0.0f, dl = 0.0f, bp = 0.0f;
    if (a.apply_dust && !AGED) {   // AGED: the folds attenuated already
      const GalaxyMeta m = a.meta[s];
      da = m.dust_a; dl = m.delta; bp = m.bump;
    }
    // out[l] is grid point l of the galaxy's row (full rows), or of its
    // slot of the selected chunks
    float *out = a.n_sel ? a.sed + (size_t)(g0 + col) * a.out_stride + blockIdx.x * TILE_L - l0
                         : a.sed + (size_t)a.perm[s] * P.n_wave;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int l = l0 + wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (!a.n_sel && l >= P.n_wave) continue;
        float v = acc[mb][nb][r];
        if (a.apply_dust && !AGED) {
          const float4 lc = P.lconst[l];
          v *= exp2f(da * (lc.z * exp2f(dl * lc.y) + bp * lc.w));
        }
        out[l] = v;
      }
    }
  }
}

int launch_sed_gemm(const SedLaunch &a, hipStream_t stream) {
  if (a.g_count <= 0) return DSPS_OK;
  const dim3 grid(a.n_sel ? a.n_sel : a.ssp.n_wave_pad / TILE_L, (a.g_count + TILE_G - 1) / TILE_G);
  ProfScope prof(DSPS_KERNEL_SED_GEMM, stream);
  if (a.age_dust) {
    if (a.precision != DSPS_FP32 || !a.ssp.sa32 || a.ion || !a.apply_dust) return DSPS_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((k_sed_gemm<DSPS_FP32, false, true>), grid, dim3(GEMM_THREADS), 0, stream, a);
  } else if (a.ion) {
    if (a.precision != DSPS_FP32 || !a.ssp.st32) return DSPS_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((k_sed_gemm<DSPS_FP32, true>), grid, dim3(GEMM_THREADS), 0, stream, a);
  } else if (a.precision == DSPS_BF16) {
    hipLaunchKernelGGL(k_sed_gemm<DSPS_BF16>, grid, dim3(GEMM_THREADS), 0, stream, a);
  } else {
    hipLaunchKernelGGL(k_sed_gemm<DSPS_FP32>, grid, dim3(GEMM_THREADS), 0, stream, a);
  }
  return hip_fail(hipGetLastError(), "k_sed_gemm launch");
}

}  // namespace dsps
