// Fused magnitudes: SED tile = W . SSP on MFMA, then attenuation and the
// redshifted filter integrals in registers (Section 2.1 Eqs. cspdeftheta and
// full_mdf; Section 3.4 Eqs. attenuation-uvbump; Section 2.2.1 Eq. restmag),
// optionally with age-dependent attenuation (Section 3.4.1) or over the
// nebular ionization axis (Section 3.3, Eq. nebsed).
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


// Most band slots evaluated together in one epilogue pass (a pass takes as
// many of the chunk's remaining bands as it can, up to this).
constexpr int NSLOT = 3;
// Rows of the accumulator whose filter lookups are scheduled together.
constexpr int EPI_ROWS = 2;

// Per-galaxy sums of one chunk for bands base .. base + NS - 1, NCOMP
// components each, reduced over the two lane halves and the two row-waves of
// each column block and stored to (or, with add, added to) the chunk's
// partial slot (component c of band b at c * n_band + b).  s_red aliases the operand staging area: the
// leading barrier orders these writes after every wave's last MFMA read and
// after the previous pass's reads.
template <int NCOMP, int NS>
__device__ __forceinline__ void write_band_slots(float (&sum)[NCOMP][2][NS], int base, int n_band,
                                                 float *s_red, int wr, int wc, int lane, int nvalid,
                                                 float *out_base, int stride, bool add) {
  const int h = lane >> 5;
#pragma unroll
  for (int c = 0; c < NCOMP; ++c)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int k = 0; k < NS; ++k) sum[c][nb][k] += __shfl_xor(sum[c][nb][k], 32, 64);
  // Lane half h finishes column block nb = h.  Every array index below is a
  // compile-time constant (a runtime-selected index would move the
  // accumulators to scratch memory).
  const int col = h * 32 + (lane & 31);
  float *red = s_red + (wc * 64 + col) * (NCOMP * NS);
  __syncthreads();
  if (wr == 1) {
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      if (h == nb) {
#pragma unroll
        for (int c = 0; c < NCOMP; ++c)
#pragma unroll
          for (int k = 0; k < NS; ++k) red[c * NS + k] = sum[c][nb][k];
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
          for (int k = 0; k < NS; ++k)
#pragma unroll
            for (int c = 0; c < NCOMP; ++c) {
              const float v = sum[c][nb][k] + red[c * NS + k];
              float *o = out + c * n_band + base + k;
              *o = add ? *o + v : v;
            }
        }
      }
    }
  }
}

// Per-lane state of the epilogue: the lane's two galaxy columns.
struct EpiLane {
  float zp1[2], da[2], dl[2], bp[2];
};

// One epilogue pass over bands base .. base + NS - 1 of a chunk.  Without the
// moments (MOM false) acc already holds the attenuated SED times the
// trapezoid weight, e = L F_att q; with them acc holds L and e and the three
// moment integrands are formed here.  Sums, per band: num += T e,
// den += T q and, with MOM, T e k_lambda, T e k0 (lambda/5500)^delta
// log2(lambda/5500) and T e D(lambda).
template <bool MOM, int NCOMP, int NS, bool INSIDE>
__device__ __forceinline__ void band_pass(const f32x16 (&acc)[2][2], const EpiLane &E,
                                          const FilterView &F, const float *s_tr,
                                          const float4 *s_lc, const float *s_q, int base, int wr,
                                          int h, float (&sum)[NCOMP][2][NS]) {
  const int n_int = F.n_pts - 1;
  const float *tab[NS];
  float nw0[NS], wi[NS];   // u = lambda_obs * wi - w0 * wi
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const float2 gr = F.grid[base + k];
    tab[k] = s_tr + (base + k) * filter_stride(F.n_pts);
    wi[k] = gr.y;
    nw0[k] = -gr.x * gr.y;
  }
#pragma unroll
  for (int c = 0; c < NCOMP; ++c)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int k = 0; k < NS; ++k) sum[c][nb][k] = 0.0f;
  // An offset the compiler cannot see through keeps the per-row LDS reads
  // below inside the pass (hoisted out of it they would pin 64 registers).
  int zero;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
  const float4 *lcp = s_lc + zero;
  const float *qp = s_q + zero;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      const float4 lc = lcp[row];   // (lambda, log2(lambda/5500), k0, drude shape)
      const float q = qp[row];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const float lobs = E.zp1[nb] * lc.x;
        float e = acc[mb][nb][r];
        float x[3];
        if (MOM) {
          const float k0x = __fmul_rn(lc.z, __builtin_amdgcn_exp2f(E.dl[nb] * lc.y));
          const float kl = fmaf(E.bp[nb], lc.w, k0x);
          e = e * __builtin_amdgcn_exp2f(E.da[nb] * kl) * q;
          x[0] = e * kl; x[1] = e * k0x * lc.y; x[2] = e * lc.w;
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const float u = fmaf(lobs, wi[k], nw0[k]);
          const float t = INSIDE ? filter_table_inside(tab[k], u) : filter_table_at(tab[k], n_int, u);
          sum[0][nb][k] += t * e;
          sum[1][nb][k] += t * q;
          if (MOM) {
            sum[2 % NCOMP][nb][k] += t * x[0];
            sum[3 % NCOMP][nb][k] += t * x[1];
            sum[4 % NCOMP][nb][k] += t * x[2];
          }
        }
      }
      // bound the scheduler's look-ahead: batching the lookups of a few
      // rows hides LDS latency, batching all of them spills registers
      if ((r & (EPI_ROWS - 1)) == EPI_ROWS - 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Three workgroups per CU (at most 168 VGPRs); with the dust moments (MOM),
// whose extra sums need more registers, or with age-dependent attenuation
// (AGED), which keeps a second accumulator, two.  The cross-wave reduction
// buffer of the epilogue reuses the operand staging area, which is idle by
// then.
//
// AGED (Section 3.4.1, Eq. agedep_dust_csp): the K units are halves of an
// age's 16 metallicity slots in the age-major table, those some member holds
// a weight in, and the attenuation, which depends on age, is applied per group
// of stages sharing one set of dust parameters: the young-star ages as one
// group, each age of the transition on its own, the old-star ages as one
// group (no stage mixes two groups).  After a group's last stage every wave
// folds the group's partial SED into a second accumulator,
// sed += F_att(group) * acc, and restarts acc.
//
// NEB (Section 3.3, Eq. nebsed): the table rows hold one (metallicity, age)
// block per ionization point, and the K loop runs over the tile's stages once
// per ionization point some member reaches.  A galaxy's weight row is the
// same for every point; it is multiplied by the galaxy's weight of the point
// as each stage is staged into LDS, so the accumulator sums the cells of all
// three axes.
enum { MAGS_PLAIN = 0, MAGS_AGED = 1, MAGS_NEB = 2 };
template <int PREC, bool MOM, int VAR = MAGS_PLAIN>
__global__ __launch_bounds__(GEMM_THREADS, (MOM || VAR == MAGS_AGED) ? 2 : 3) void k_mags_gemm(MagsLaunch a) {
  using C = GemmCfg<PREC>;
  using elem = typename C::elem;
  constexpr bool AGED = VAR == MAGS_AGED, NEB = VAR == MAGS_NEB;
  static_assert(!(AGED || NEB) || PREC == DSPS_FP32, "float32 only");
  static_assert(!(AGED && MOM), "no dust moments with the age-dependent attenuation");
  constexpr int NCOMP = MOM ? 5 : 2;
  static_assert(2 * sizeof(GemmSmem<PREC>) >= sizeof(float) * 128 * NCOMP * NSLOT, "reduction alias");
  __shared__ GemmSmem<PREC> sm[2];
  __shared__ float4 s_lc[TILE_L];
  __shared__ float s_q[TILE_L];
  // byte offsets (A, B) of each thread's 16-byte piece of every stage of the
  // tile's unit list (age-major: its piece list), by stage and piece
  __shared__ int2 s_piece[4 * (AGED ? MAX_AGED_UNITS : MAX_UNITS) / GemmCfg<PREC>::UNITS];
  // dynamic: filter transmissions [n_band][n_pts + 1], then with NEB the
  // members' ionization weights [point - u_lo][column] (n_u points at most)
  extern __shared__ float s_tr[];
  float *s_pn = s_tr + a.flt.n_band * filter_stride(a.flt.n_pts);
  float *s_red = reinterpret_cast<float *>(&sm[0]);

  int tile, group;
  xcd_tile_group(blockIdx.x, a.n_groups, tile, group);
  const int live = live_in_range(a.n_live, a.s_begin, a.s_count);
  const int n_tiles = (live + TILE_G - 1) / TILE_G;
  if (tile >= n_tiles) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int h = lane >> 5;
  const SspView P = a.ssp;        // by value: a reference into the kernel
  const FilterView F = a.flt;     // argument would force a private-memory copy
  const int n_band = F.n_band;
  const int g0 = tile * TILE_G;                 // first batch-local galaxy of the tile
  const int nvalid = min(TILE_G, live - g0);

  // ---- the tile's plan.  A workgroup takes a group of CPG chunks of the
  // tile's window.  Where a partial slot holds a whole group (PCG = CPG),
  // groups are CPG whole chunks from a multiple of CPG, clipped to the
  // window: a slot's sum (its chunks in order; chunks outside a galaxy's own
  // window add exact zeros) is then the same in any tile.  Otherwise groups
  // start at the window's first chunk.  Workgroup `group` takes the tile's
  // group-th group; the grid holds a host bound on one galaxy's window, and
  // a tile whose members' windows spread further hands every remaining chunk
  // to its last workgroup.
  const TilePlan *pl = a.plan + tile;
  const int c_first = pl->c_first, c_last = pl->c_last;
  constexpr int CPG = chunks_per_group(PREC), PCG = partial_chunks(PREC);
  static_assert(PCG == 1 || PCG == CPG, "a slot holds one chunk or a whole group");
  const int c_base = PCG > 1 ? c_first / CPG * CPG : c_first;
  const int c_begin = max(c_base + group * CPG, c_first);
  const int c_end = group == a.n_groups - 1 ? c_last : min(c_base + (group + 1) * CPG, c_last);
  if (c_begin >= c_end) return;
  const int nk = pl->nk;
  const float zp1_min = pl->zp1_min, zp1_max = pl->zp1_max;
  for (int t = threadIdx.x; t < STAGE_UNITS * nk; t += blockDim.x)
    s_piece[t] = piece_bytes<PREC>(unit_piece<PREC>(pl->koff, t / STAGE_UNITS, t % STAGE_UNITS));
  int u_lo = 0, n_uu = 1;
  if constexpr (NEB) {
    u_lo = pl->u_lo;
    n_uu = pl->u_hi - pl->u_lo + 1;
    for (int t = threadIdx.x; t < n_uu * TILE_G; t += blockDim.x) {
      const int uu = t / TILE_G, col = t - uu * TILE_G;
      float f = 0.0f;
      if (col < nvalid) {
        const GalaxyIon gi = a.ion[a.s_begin + g0 + col];
        const int u = u_lo + uu;
        const double c = gi.lgu, sg = gi.sigma_u;
        f = (float)(a.ion_tangent == 1   ? ion_weight_d<1>(P.ion_edges, u, c, sg)
                    : a.ion_tangent == 2 ? ion_weight_d<2>(P.ion_edges, u, c, sg)
                                         : ion_weight(P.ion_edges, u, c, sg));
      }
      s_pn[t] = f;
    }
  }

  // ---- filter tables into LDS
  fill_filter_table(F, s_tr);

  // ---- per-galaxy parameters of this lane's two columns
  EpiLane E;
  float da_old[2] = {0.0f, 0.0f}, dl_old[2] = {0.0f, 0.0f};   // AGED: old-star dust
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = wc * 64 + nb * 32 + (lane & 31);
    if (col < nvalid) {
      const GalaxyMeta m = a.meta[a.s_begin + g0 + col];
      E.zp1[nb] = m.zp1; E.da[nb] = m.dust_a; E.dl[nb] = m.delta; E.bp[nb] = m.bump;
      if (AGED) {
        const GalaxyDustOld d = a.dust_old[a.s_begin + g0 + col];
        da_old[nb] = d.dust_a; dl_old[nb] = d.delta;
      }
    } else {
      // padding columns: zero weights; 1 + z inside the tile's range keeps
      // their filter lookups inside the tables
      E.zp1[nb] = zp1_min; E.da[nb] = 0.0f; E.dl[nb] = 0.0f; E.bp[nb] = 0.0f;
    }
  }

  // ---- K steps: the tile's non-zero weight units (s_piece), or with AGED
  // its ages
  const elem *st = AGED ? (const elem *)P.sa32
                        : (PREC == DSPS_FP32 ? (const elem *)P.st32 : (const elem *)P.st16);
  const int k_cols = AGED ? AGE_K : P.k_pad;
  const int a_stride = NEB ? P.k_row : k_cols;     // table row length
  const size_t a_elems = (size_t)P.n_wave_pad * a_stride;
  const elem *w_tile = (const elem *)a.w_pad + (size_t)g0 * k_cols;
  const int n_comp = NCOMP * n_band;
  const int ucol = stage_col();
  // this thread's unit of stage s from the tile's unit list (-1: zeros)
  auto unit = [&](int s) {
    const int2 p = s_piece[STAGE_UNITS * s + ucol];
    return UnitSrc{p.x, p.y, nullptr};
  };

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
    const GemmOps<PREC> ops =
        gemm_ops<PREC>(st, a_elems, a_stride, linear_rows<PREC>(l0), w_tile, nvalid, k_cols);

    if constexpr (AGED) {
      f32x16 sed[2][2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int r = 0; r < 16; ++r) sed[mb][nb][r] = 0.0f;
      AgeFold af{pl->tag, a.age_young, a.age_old, a.dust_pivot, a.dust_width, P.lg_age, {}, {}, {}, {}, {}};
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        af.da_y[nb] = E.da[nb]; af.dl_y[nb] = E.dl[nb];
        af.da_o[nb] = da_old[nb]; af.dl_o[nb] = dl_old[nb];
        af.bp[nb] = E.bp[nb];
      }
      auto fold = [&](int ks) { af(ks, sed, acc, s_lc, wr, h); };
      gemm_kloop<PREC>(sm, ops, nk, unit, wr, wc, lane, acc, fold);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = sed[mb][nb];
    } else if constexpr (NEB) {
      // stage s: ionization point u_lo + s / nk, units of stage s % nk
      gemm_kloop<PREC>(sm, ops, nk * n_uu,
                       [&](int s) {
                         const int uu = s / nk;
                         const int2 p = s_piece[STAGE_UNITS * (s - uu * nk) + ucol];
                         return UnitSrc{(u_lo + uu) * k_cols * (int)sizeof(elem) + p.x, p.y,
                                        s_pn + uu * TILE_G};
                       },
                       wr, wc, lane, acc);
    } else {
      gemm_kloop<PREC, PREC == DSPS_FP32>(sm, ops, nk, unit, wr, wc, lane, acc);
    }
    // (the loop's closing barrier makes s_lc, s_q and the filter tables visible)

    // ---- epilogue: attenuated SED x resampled transmission, summed over the
    // bands that can see this chunk
    // (wavelengths of the chunk are non-decreasing; padding repeats the last)
    const float o_lo = zp1_min * s_lc[0].x, o_hi = zp1_max * s_lc[TILE_L - 1].x;
    const unsigned bmask = __builtin_amdgcn_readfirstlane(active_bands(F, o_lo, o_hi));
    // bands every element of the chunk sees inside its table (every column's
    // 1 + z lies in the tile's range, padding columns included)
    const unsigned imask = __builtin_amdgcn_readfirstlane(interior_bands(F, o_lo, o_hi));
    const int b_lo = bmask ? __builtin_ctz(bmask) : 0;
    const int b_hi = bmask ? 31 - __builtin_clz(bmask) : -1;   // inclusive
    // partials are slot-major, [slot][galaxy][component]: a slot's first
    // chunk stores, each later one adds its sums in chunk order
    float *part = a.partial + ((size_t)(c / PCG) * a.part_rows + g0) * n_comp;
    const bool add = c != c_begin && c % PCG != 0;
    const int stride = n_comp;
    if (AGED && b_lo <= b_hi) {
      // the attenuation is in already: e = L_att q
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float q = s_q[wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) acc[mb][nb][r] *= q;
        }
    } else if (!MOM && b_lo <= b_hi) {
      // e = L F_att q in place, once for all passes.  Rounding is fixed
      // explicitly, so that both instantiations agree bit for bit whatever
      // the compiler contracts.  The hardware exp2 is within 1 ulp; its only
      // difference from the library exp2f is that results below 2^-126
      // (attenuation beyond ~380 mag) flush to zero.
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
          const float4 lc = s_lc[row];
          const float q = s_q[row];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            const float k0x = __fmul_rn(lc.z, __builtin_amdgcn_exp2f(E.dl[nb] * lc.y));  // k0 (lambda/5500)^delta
            const float kl = fmaf(E.bp[nb], lc.w, k0x);                                 // k_lambda
            acc[mb][nb][r] = acc[mb][nb][r] * __builtin_amdgcn_exp2f(E.da[nb] * kl) * q;
          }
        }
    }
    for (int base = b_lo; base <= b_hi;) {
      const int rem = b_hi - base + 1;
      // a pass whose bands are all interior takes the lookup without clamp
      if (rem >= 3) {
        float sum[NCOMP][2][3];
        if (((imask >> base) & 7u) == 7u)
          band_pass<MOM, NCOMP, 3, true>(acc, E, F, s_tr, s_lc, s_q, base, wr, h, sum);
        else
          band_pass<MOM, NCOMP, 3, false>(acc, E, F, s_tr, s_lc, s_q, base, wr, h, sum);
        write_band_slots<NCOMP, 3>(sum, base, n_band, s_red, wr, wc, lane, nvalid, part, stride, add);
        base += 3;
      } else if (rem == 2) {
        float sum[NCOMP][2][2];
        if (((imask >> base) & 3u) == 3u)
          band_pass<MOM, NCOMP, 2, true>(acc, E, F, s_tr, s_lc, s_q, base, wr, h, sum);
        else
          band_pass<MOM, NCOMP, 2, false>(acc, E, F, s_tr, s_lc, s_q, base, wr, h, sum);
        write_band_slots<NCOMP, 2>(sum, base, n_band, s_red, wr, wc, lane, nvalid, part, stride, add);
        base += 2;
      } else {
        float sum[NCOMP][2][1];
        if ((imask >> base) & 1u)
          band_pass<MOM, NCOMP, 1, true>(acc, E, F, s_tr, s_lc, s_q, base, wr, h, sum);
        else
          band_pass<MOM, NCOMP, 1, false>(acc, E, F, s_tr, s_lc, s_q, base, wr, h, sum);
        write_band_slots<NCOMP, 1>(sum, base, n_band, s_red, wr, wc, lane, nvalid, part, stride, add);
        base += 1;
      }
    }
    // bands that see none of this chunk contribute exact zeros: stored by the
    // slot's first chunk, nothing to add for a later one
    if (wr == 0 && !add) {
      const int tcol = wc * 64 + h * 32 + (lane & 31);
      if (tcol < nvalid) {
        float *out = part + (size_t)tcol * stride;
        for (int b = 0; b < n_band; ++b) {
          if (b < b_lo || b > b_hi) {
#pragma unroll
            for (int c = 0; c < NCOMP; ++c) out[c * n_band + b] = 0.0f;
          }
        }
      }
    }
  }
}

// One workgroup of TILE_G threads per tile: union of the members' windows,
// redshifts and non-zero weight blocks, then the unit list, ascending in K:
// a float32 unit is one 4-age block of a row and a bfloat16 unit two (16
// bytes of the weight row either way), kept when it holds a weight for some
// member, padded with -1 (zero units) to whole stages.  The age-major layout
// lists the halves of an age's metallicity slots that some member holds a
// weight in, attenuation group by group, each group padded to whole stages
// and its last stage tagged with one of its ages.
template <int PREC>
__global__ __launch_bounds__(TILE_G) void k_tile_plan(MagsLaunch a) {
  // per wave: window lo, window hi, min and max of (1+z) as float bits
  // (positive floats order like their bit patterns), highest non-zero age
  // (age-major stages), first and last ionization point, then the block mask
  constexpr int NV = 7;
  __shared__ int s_wave[TILE_G / 64][NV + KBLOCK_WORDS];
  __shared__ int s_tile[NV];
  __shared__ unsigned s_kblk[KBLOCK_WORDS];
  const int tile = blockIdx.x;
  const int g0 = tile * TILE_G;
  const int nvalid = min(TILE_G, live_in_range(a.n_live, a.s_begin, a.s_count) - g0);
  if (nvalid <= 0) return;   // past the live galaxies: no reader looks at this plan
  // each wave reduces its members (lanes past the tile's last galaxy hold
  // the identities), the two waves' results are joined in LDS: no atomics
  {
    const int wave = threadIdx.x >> 6;
    const bool live = (int)threadIdx.x < nvalid;
    GalaxyRange r;
    int zbits = 0x7f7fffff, zhi = 0, u_lo = 1 << 30, u_hi = 0;
    if (live) {
      r = a.range[a.s_begin + g0 + threadIdx.x];
      zbits = zhi = __float_as_int(a.meta[a.s_begin + g0 + threadIdx.x].zp1);
      if (a.ion) {
        const GalaxyIon gi = a.ion[a.s_begin + g0 + threadIdx.x];
        u_lo = gi.u_lo;
        u_hi = gi.u_hi;
      }
    } else {
      r.win_lo = 1 << 30;
      r.win_hi = 0;
      r.age_hi = 0;
#pragma unroll
      for (int w = 0; w < KBLOCK_WORDS; ++w) r.kblk[w] = 0u;
    }
    int v[NV + KBLOCK_WORDS];
    v[0] = wave_join<WAVE_MIN>(r.win_lo);
    v[1] = wave_join<WAVE_MAX>(r.win_hi);
    v[2] = wave_join<WAVE_MIN>(zbits);
    v[3] = wave_join<WAVE_MAX>(zhi);
    v[4] = wave_join<WAVE_MAX>(r.age_hi);
    v[5] = a.ion ? wave_join<WAVE_MIN>(u_lo) : 0;
    v[6] = a.ion ? wave_join<WAVE_MAX>(u_hi) : 0;
#pragma unroll
    for (int w = 0; w < KBLOCK_WORDS; ++w) v[NV + w] = wave_join<WAVE_OR>((int)r.kblk[w]);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV + KBLOCK_WORDS; ++k)
      if (lane == k) s_wave[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;   // wave 0 joins the waves and writes the plan
  const int lane = threadIdx.x;
  static_assert(TILE_G == 128, "two waves per plan block");
  if (lane < NV + KBLOCK_WORDS) {
    const int x = s_wave[0][lane], y = s_wave[1][lane];
    const bool is_min = lane == 0 || lane == 2 || lane == 5;
    const int j = lane < NV ? (is_min ? min(x, y) : max(x, y)) : (x | y);
    if (lane < NV) s_tile[lane] = j; else s_kblk[lane - NV] = (unsigned)j;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  TilePlan *pl = a.plan + tile;
  const int n_met = a.ssp.n_met;
  if (a.age_dust) {
    // groups of ages [a0, a1): all young ages, one transition age, all old
    // ages, up to the tile's highest age with a weight; candidate unit c is
    // half c % 2 of age c / 2: mask bits 2c and 2c + 1
    using C32 = GemmCfg<DSPS_FP32>;             // the age-major layout is float32
    static_assert(AGED_PIECES_PER_AGE == 4 && AGE_MET_SLOTS == 2 * C32::UNIT_K,
                  "two units of two pieces per age");
    constexpr int UPS = C32::UNITS;             // units per stage
    const int age_hi = min(s_tile[4], AGE_PAD);
    int n = 0;
    for (int a0 = 0; a0 < age_hi;) {
      const int a1 = a0 < a.age_young ? min(a.age_young, age_hi)
                                      : (a0 < a.age_old ? a0 + 1 : age_hi);
      const int n_start = n;
      for (int base = 2 * a0; base < 2 * a1; base += 64) {
        const int c = base + lane;
        const bool keep = c < 2 * a1 && ((s_kblk[(2 * c) >> 5] >> ((2 * c) & 31)) & 3u);
        const unsigned long long m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (keep) pl->koff[n + before] = AGE_MET_SLOTS * (c / 2) + C32::UNIT_K * (c % 2);
        n += __popcll(m);
      }
      if (n > n_start) {
        const int n_pad = (n + UPS - 1) / UPS * UPS;
        if (n + lane < n_pad) pl->koff[n + lane] = -1;
        for (int q = n_start / UPS + lane; q < n_pad / UPS; q += 64)
          pl->tag[q] = q == n_pad / UPS - 1 ? (short)(a1 - 1) : (short)-1;
        n = n_pad;
      }
      a0 = a1;
    }
    if (lane == 0) {
      const int c_first = s_tile[0] / TILE_L;
      pl->c_first = c_first;
      pl->c_last = max((s_tile[1] + TILE_L - 1) / TILE_L, c_first);   // exclusive
      pl->nk = n / UPS;
      pl->n_units = n;
      pl->zp1_min = __int_as_float(s_tile[2]);
      pl->zp1_max = __int_as_float(s_tile[3]);
      pl->u_lo = 0;
      pl->u_hi = 0;
    }
    return;
  }
  // candidate unit c: float32 (row c / 12, 8 ages from 8 (c % 12): 4-age
  // blocks 2 (c % 12) and + 1, both in mask word c % 12); bfloat16 (row
  // c / 6, 16 ages from 16 (c % 6): mask words 2 (c % 6) and + 1)
  constexpr int UNITS_PER_ROW = AGE_PAD / GemmCfg<PREC>::UNIT_K;   // 12 or 6
  const int n_cand = n_met * UNITS_PER_ROW;
  int n = 0;
  for (int base = 0; base < n_cand; base += 64) {
    const int c = base + lane;
    bool keep = false;
    int koff = 0;
    if (c < n_cand) {
      if (PREC == DSPS_BF16) {
        const int j = c / UNITS_PER_ROW, q = c % UNITS_PER_ROW;
        const unsigned m2 = s_kblk[2 * q] | s_kblk[2 * q + 1];
        keep = ((m2 >> j) | (m2 >> (16 + j))) & 1u;
        koff = j * AGE_PAD + 16 * q;
      } else {
        const int j = c / UNITS_PER_ROW, q = c % UNITS_PER_ROW;
        keep = ((s_kblk[q] >> j) | (s_kblk[q] >> (16 + j))) & 1u;
        koff = j * AGE_PAD + 8 * q;
      }
    }
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (keep) pl->koff[n + before] = koff;
    n += __popcll(m);
  }
  constexpr int UPS = GemmCfg<PREC>::UNITS;     // units per stage
  const int n_pad = (n + UPS - 1) / UPS * UPS;
  if (n + lane < n_pad) pl->koff[n + lane] = -1;
  if (lane == 0) {
    const int c_first = s_tile[0] / TILE_L;
    pl->c_first = c_first;
    pl->c_last = max((s_tile[1] + TILE_L - 1) / TILE_L, c_first);   // exclusive
    pl->nk = n_pad / UPS;
    pl->n_units = n;
    pl->zp1_min = __int_as_float(s_tile[2]);
    pl->zp1_max = __int_as_float(s_tile[3]);
    pl->u_lo = s_tile[5];
    pl->u_hi = s_tile[6];
  }
}

int launch_tile_plan(const MagsLaunch &a, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  const int n_tiles = (a.s_count + TILE_G - 1) / TILE_G;
  if (a.precision == DSPS_BF16)
    hipLaunchKernelGGL(k_tile_plan<DSPS_BF16>, dim3(n_tiles), dim3(TILE_G), 0, stream, a);
  else
    hipLaunchKernelGGL(k_tile_plan<DSPS_FP32>, dim3(n_tiles), dim3(TILE_G), 0, stream, a);
  return hip_fail(hipGetLastError(), "k_tile_plan launch");
}

int launch_mags_gemm(const MagsLaunch &a, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  const int n_tiles = (a.s_count + TILE_G - 1) / TILE_G;
  const int blocks = (n_tiles + 7) / 8 * 8 * a.n_groups;
  size_t lds = sizeof(float) * a.flt.n_band * filter_stride(a.flt.n_pts);
  if (int rc = launch_tile_plan(a, stream)) return rc;
  ProfScope prof(DSPS_KERNEL_MAGS_GEMM, stream);
  if (a.age_dust) {
    if (a.precision != DSPS_FP32 || a.moments || !a.ssp.sa32 || a.ion) return DSPS_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((k_mags_gemm<DSPS_FP32, false, MAGS_AGED>), dim3(blocks), dim3(GEMM_THREADS),
                       lds, stream, a);
  } else if (a.ion) {
    if (a.precision != DSPS_FP32 || !a.ssp.st32) return DSPS_ERR_UNSUPPORTED;
    lds += sizeof(float) * a.ssp.n_u * TILE_G;
    if (a.moments)
      hipLaunchKernelGGL((k_mags_gemm<DSPS_FP32, true, MAGS_NEB>), dim3(blocks), dim3(GEMM_THREADS),
                         lds, stream, a);
    else
      hipLaunchKernelGGL((k_mags_gemm<DSPS_FP32, false, MAGS_NEB>), dim3(blocks), dim3(GEMM_THREADS),
                         lds, stream, a);
  } else if (a.precision == DSPS_BF16) {
    if (a.moments) return DSPS_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((k_mags_gemm<DSPS_BF16, false>), dim3(blocks), dim3(GEMM_THREADS), lds, stream, a);
  } else if (a.moments) {
    hipLaunchKernelGGL((k_mags_gemm<DSPS_FP32, true>), dim3(blocks), dim3(GEMM_THREADS), lds, stream, a);
  } else {
    hipLaunchKernelGGL((k_mags_gemm<DSPS_FP32, false>), dim3(blocks), dim3(GEMM_THREADS), lds, stream, a);
  }
  return hip_fail(hipGetLastError(), "k_mags_gemm launch");
}

// Sum the per-chunk partial band sums in chunk order and form magnitudes
// m = -2.5 log10(num / (AB0 den)) + [D_mod(z) - 2.5 log10(1+z)] in float64.
// One workgroup per 128-galaxy tile: the tile's partial rows of one chunk are
// contiguous, so consecutive threads sum consecutive (galaxy, component)
// entries over the tile's chunks (each entry in chunk order) into LDS; then
// one thread per galaxy forms its magnitudes.
constexpr int FINALIZE_THREADS = 256;
__global__ __launch_bounds__(FINALIZE_THREADS) void k_mags_finalize(FinalizeLaunch a) {
  __shared__ float s_sum[TILE_G * 5 * DSPS_MAX_BAND];
  const int tile = blockIdx.x;
  const int g0 = tile * TILE_G;
  const int nvalid = min(TILE_G, live_in_range(a.n_live, a.s_begin, a.s_count) - g0);
  if (nvalid <= 0) return;   // the whole workgroup, before any barrier
  const int nb = a.n_band, ncomp = mags_components(a.moments), nc = ncomp * nb;
  const TilePlan &pl = a.plan[tile];
  // the partial slots of the tile's window (see k_mags_gemm); none if it is
  // empty
  const int q_first = pl.c_first / a.pcg;
  const int q_last = pl.c_last > pl.c_first ? (pl.c_last - 1) / a.pcg + 1 : q_first;
  const int n_el = nvalid * nc;
  // each thread sums up to FIN_ELEMS elements FINALIZE_THREADS apart, taking
  // FIN_SLOTS slots at a time: all their loads are issued before the first
  // add, and every element's sum still runs in slot order
  constexpr int FIN_ELEMS = 8, FIN_SLOTS = 8;
  for (int e0 = threadIdx.x; e0 < n_el; e0 += FINALIZE_THREADS * FIN_ELEMS) {
    float v[FIN_ELEMS];
#pragma unroll
    for (int i = 0; i < FIN_ELEMS; ++i) v[i] = 0.0f;
    for (int q0 = q_first; q0 < q_last; q0 += FIN_SLOTS) {
      float x[FIN_SLOTS][FIN_ELEMS];
#pragma unroll
      for (int k = 0; k < FIN_SLOTS; ++k) {
        const float *p = a.partial + ((size_t)(q0 + k) * a.part_rows + g0) * nc + e0;
#pragma unroll
        for (int i = 0; i < FIN_ELEMS; ++i)
          x[k][i] = q0 + k < q_last && e0 + i * FINALIZE_THREADS < n_el ? p[i * FINALIZE_THREADS] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < FIN_SLOTS; ++k)
        if (q0 + k < q_last)
#pragma unroll
          for (int i = 0; i < FIN_ELEMS; ++i) v[i] += x[k][i];
    }
#pragma unroll
    for (int i = 0; i < FIN_ELEMS; ++i)
      if (e0 + i * FINALIZE_THREADS < n_el) s_sum[e0 + i * FINALIZE_THREADS] = v[i];
  }
  __syncthreads();
  if ((int)threadIdx.x >= nvalid) return;
  const int local = g0 + threadIdx.x;
  const int s = a.s_begin + local;
  const int g = a.perm ? a.perm[s] : s;
  const float *acc = s_sum + threadIdx.x * nc;   // component k of band b at k * nb + b
  const double offset = a.mag_offset[s];
  for (int b = 0; b < nb; ++b) {
    const float num = acc[b], den = acc[nb + b];
    double m;
    if (a.tangent_bands) {
      // d(-2.5 log10 num) = -2.5 / ln 10 dnum / num
      const float num_fwd = a.tangent_bands[(size_t)g * 2 * nb + b];
      m = -1.0857362047581294 * (double)num / (double)num_fwd;
    } else if (den == 0.0f) {
      m = __builtin_nan("");
    } else {
      m = -2.5 * log10((double)num / (AB_ZERO_POINT * (double)den)) + offset;
    }
    a.mags[(size_t)g * nb + b] = (float)m;
    if (a.bands) {
      a.bands[(size_t)g * 2 * nb + b] = num;
      a.bands[(size_t)g * 2 * nb + nb + b] = den;
    }
    if (a.mom)
      for (int k = 0; k < 3; ++k) a.mom[(size_t)g * 3 * nb + k * nb + b] = acc[(2 + k) * nb + b];
  }
}

int launch_mags_finalize(const FinalizeLaunch &a, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  ProfScope prof(DSPS_KERNEL_MAGS_FINALIZE, stream);
  hipLaunchKernelGGL(k_mags_finalize, dim3((a.s_count + TILE_G - 1) / TILE_G),
                     dim3(FINALIZE_THREADS), 0, stream, a);
  return hip_fail(hipGetLastError(), "k_mags_finalize launch");
}

}  // namespace dsps
