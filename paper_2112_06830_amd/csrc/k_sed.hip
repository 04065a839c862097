// Unfused composite SED: L[g, l] = sum_k W[g, k] L_SSP[k, l] (Section 2.1,
// Eqs. cspdeftheta and full_mdf), optionally times the attenuation F_att
// (Section 3.4, Eq. attenuation), written to memory in the rest frame.  With
// the ionization axis (NEB; Section 3.3, Eq. nebsed) the sum also runs over
// the ionization points the tile's galaxies reach, each galaxy's weight row
// scaled by its weight of the point as it is staged; with ion_tangent the
// weights are replaced by their derivatives in the distribution's centre or
// width, which gives the SED's derivative (the sum is linear in them).
//
// Galaxies come in the ordering sort's order, so a tile's members share few
// metallicity rows and ages: the K loop runs over the tile's stage list (the
// weight blocks non-zero for some member), as in the fused kernel.  Skipped
// blocks are zero for every member, so a galaxy's result does not depend on
// its tile.
#include "gemm_core.hpp"

namespace dsps {

template <int PREC, bool NEB = false>
__global__ __launch_bounds__(GEMM_THREADS, 2) void k_sed_gemm(SedLaunch a) {
  using C = GemmCfg<PREC>;
  using elem = typename C::elem;
  static_assert(!NEB || PREC == DSPS_FP32, "the ionization axis is float32 only");
  __shared__ GemmSmem<PREC> sm[2];
  __shared__ float s_pn[NEB ? DSPS_MAX_ION * TILE_G : 1];
  __shared__ int s_koff[DSPS_MAX_MET * KBLOCKS_PER_ROW];   // K offset of each stage
  const int chunk = a.n_sel ? a.chunk_list[blockIdx.x] : (int)blockIdx.x;
  const int tile = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave & 1, wc = wave >> 1, h = lane >> 5;
  const SspView P = a.ssp;
  const int l0 = chunk * TILE_L;
  const int g0 = tile * TILE_G;
  const elem *st = PREC == DSPS_FP32 ? (const elem *)P.st32 : (const elem *)P.st16;
  const elem *w = (const elem *)a.w_pad;

  f32x16 acc[2][2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const TilePlan *pl = a.plan + tile;
  const int nk = pl->nk;
  for (int t = threadIdx.x; t < nk; t += blockDim.x) s_koff[t] = pl->koff[t];
  if constexpr (NEB) {
    // every member's weight of each of the tile's ionization points
    const int nvalid = min(TILE_G, a.g_count - g0);
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
    gemm_kloop_ab<PREC>(sm, st, P.k_row, l0, w, kp, g0, a.g_count, nk * n_uu,
                        [&](int s) {
                          const int uu = s / nk;
                          const int k = s_koff[s - uu * nk];
                          return StageSrc{(u_lo + uu) * kp + k, k, s_pn + uu * TILE_G};
                        },
                        wr, wc, lane, acc);
  } else {
    __syncthreads();
    gemm_kloop<PREC>(sm, st, P.k_pad, l0, w, g0, a.g_count, nk, [&](int ks) { return s_koff[ks]; },
                     wr, wc, lane, acc);
  }

#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = wc * 64 + nb * 32 + (lane & 31);
    if (g0 + col >= a.g_count) continue;
    const int s = a.g_begin + g0 + col;     // sorted position
    float da = 0.0f, dl = 0.0f, bp = 0.0f;
    if (a.apply_dust) {
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
        if (a.apply_dust) {
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
  if (a.ion) {
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
