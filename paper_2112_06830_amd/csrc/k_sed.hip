// Unfused composite SED: L[g, l] = sum_k W[g, k] L_SSP[k, l] (Section 2.1,
// Eqs. cspdeftheta and full_mdf), optionally times the attenuation F_att
// (Section 3.4, Eq. attenuation), written to memory in the rest frame.
#include "gemm_core.hpp"

namespace dsps {

template <int PREC>
__global__ __launch_bounds__(GEMM_THREADS, 2) void k_sed_gemm(SedLaunch a) {
  using C = GemmCfg<PREC>;
  using elem = typename C::elem;
  __shared__ GemmSmem<PREC> sm[2];
  const int chunk = blockIdx.x, tile = blockIdx.y;
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

  const int nk = P.k_pad / C::KT;
  gemm_kloop<PREC>(sm, st, P.k_pad, l0, w, g0, a.g_count, nk, [](int ks) { return ks * C::KT; },
                   wr, wc, lane, acc);

#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = wc * 64 + nb * 32 + (lane & 31);
    if (g0 + col >= a.g_count) continue;
    const int g = a.g_begin + g0 + col;
    float da = 0.0f, dl = 0.0f, bp = 0.0f;
    if (a.apply_dust) {
      const GalaxyMeta m = a.meta[g];
      da = m.dust_a; dl = m.delta; bp = m.bump;
    }
    float *out = a.sed + (size_t)g * P.n_wave;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int l = l0 + wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (l >= P.n_wave) continue;
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
  const dim3 grid(a.ssp.n_wave_pad / TILE_L, (a.g_count + TILE_G - 1) / TILE_G);
  ProfScope prof(DSPS_KERNEL_SED_GEMM, stream);
  if (a.precision == DSPS_BF16)
    hipLaunchKernelGGL(k_sed_gemm<DSPS_BF16>, grid, dim3(GEMM_THREADS), 0, stream, a);
  else
    hipLaunchKernelGGL(k_sed_gemm<DSPS_FP32>, grid, dim3(GEMM_THREADS), 0, stream, a);
  return hip_fail(hipGetLastError(), "k_sed_gemm launch");
}

}  // namespace dsps
