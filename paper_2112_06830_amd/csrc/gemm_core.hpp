// MFMA GEMM core shared by the fused-magnitude, SED and adjoint kernels.
//
// A workgroup of four wave64s computes a 128 x 128 output tile in a 2 x 2
// arrangement of 64 x 64 wave tiles (2 x 2 MFMA 32x32 blocks per wave).  Both
// operands are K-contiguous rows in memory; each K stage is staged through
// registers into LDS rows padded to a 16-byte-aligned, bank-conflict-free
// pitch, and every lane feeds MFMA from 16-byte LDS reads.
#pragma once

#include "dsps_internal.hpp"

namespace dsps {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// Native 16-byte vector for staging (HIP's uint4 is a struct wrapper that the
// optimiser does not always keep in registers).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct GemmCfg;
// K per LDS stage divides AGE_PAD.  Row pitches keep 16-byte alignment and
// put the eight rows read by one 8-lane group of a 16-byte LDS read on
// distinct bank quads.  The FP32 stage is kept short so that the fused kernel
// fits three workgroups per CU in registers and LDS.
template <> struct GemmCfg<DSPS_FP32> {
  using elem = float;
  static constexpr int KT = 16;
  static constexpr int PITCH = 20;
};
template <> struct GemmCfg<DSPS_BF16> {
  using elem = uint16_t;
  static constexpr int KT = 32;
  static constexpr int PITCH = 40;
};


template <int PREC>
struct GemmSmem {
  using C = GemmCfg<PREC>;
  typename C::elem a[TILE_L * C::PITCH];
  typename C::elem b[TILE_G * C::PITCH];
};

// Stage one KT-wide slice of 128 rows from a K-contiguous matrix into
// registers (vectors of 16 bytes).
template <int PREC>
struct StageRegs {
  using C = GemmCfg<PREC>;
  static constexpr int VPR = C::KT * (int)sizeof(typename C::elem) / 16;  // vectors per row
  static constexpr int NV = TILE_L * VPR / GEMM_THREADS;                  // vectors per thread
  u32x4 a[NV];
  u32x4 b[NV];
};

template <int PREC>
__device__ __forceinline__ void load_stage(StageRegs<PREC> &r, const typename GemmCfg<PREC>::elem *st,
                                           int k_pad, int l0, const typename GemmCfg<PREC>::elem *w,
                                           int g0, int g_count, int kofs) {
  using S = StageRegs<PREC>;
  constexpr int EPV = 16 / sizeof(typename GemmCfg<PREC>::elem);  // elements per vector
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    const int idx = threadIdx.x + v * GEMM_THREADS;
    const int row = idx / S::VPR, col = idx % S::VPR;
    r.a[v] = *reinterpret_cast<const u32x4 *>(st + (size_t)(l0 + row) * k_pad + kofs + col * EPV);
    u32x4 bv = {0u, 0u, 0u, 0u};
    if (g0 + row < g_count)
      bv = *reinterpret_cast<const u32x4 *>(w + (size_t)(g0 + row) * k_pad + kofs + col * EPV);
    r.b[v] = bv;
  }
}

template <int PREC>
__device__ __forceinline__ void store_stage(const StageRegs<PREC> &r, GemmSmem<PREC> &sm) {
  using S = StageRegs<PREC>;
  using C = GemmCfg<PREC>;
  constexpr int EPV = 16 / sizeof(typename C::elem);
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    const int idx = threadIdx.x + v * GEMM_THREADS;
    const int row = idx / S::VPR, col = idx % S::VPR;
    *reinterpret_cast<u32x4 *>(&sm.a[row * C::PITCH + col * EPV]) = r.a[v];
    *reinterpret_cast<u32x4 *>(&sm.b[row * C::PITCH + col * EPV]) = r.b[v];
  }
}

// acc[mb][nb] += A[rows of mb] . B[cols of nb] over one KT stage.
__device__ __forceinline__ void mma_stage(const GemmSmem<DSPS_FP32> &sm, int wr, int wc, int lane,
                                          f32x16 (&acc)[2][2]) {
  using C = GemmCfg<DSPS_FP32>;
  constexpr int HALF = C::KT / 2;      // contraction indices owned by one lane half
  const int h = lane >> 5, c = lane & 31;
  // Lane half h supplies contraction index HALF*h + 8u + t at MFMA step
  // (u, t), for A and B alike; each lane reads 8 contiguous values per
  // operand block and sub-step.
#pragma unroll
  for (int u = 0; u < HALF / 8; ++u) {
    float av[2][8], bv[2][8];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const float *p = &sm.a[(wr * 64 + mb * 32 + c) * C::PITCH + HALF * h + 8 * u];
      const float4 x0 = *reinterpret_cast<const float4 *>(p);
      const float4 x1 = *reinterpret_cast<const float4 *>(p + 4);
      av[mb][0] = x0.x; av[mb][1] = x0.y; av[mb][2] = x0.z; av[mb][3] = x0.w;
      av[mb][4] = x1.x; av[mb][5] = x1.y; av[mb][6] = x1.z; av[mb][7] = x1.w;
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const float *p = &sm.b[(wc * 64 + nb * 32 + c) * C::PITCH + HALF * h + 8 * u];
      const float4 x0 = *reinterpret_cast<const float4 *>(p);
      const float4 x1 = *reinterpret_cast<const float4 *>(p + 4);
      bv[nb][0] = x0.x; bv[nb][1] = x0.y; bv[nb][2] = x0.z; bv[nb][3] = x0.w;
      bv[nb][4] = x1.x; bv[nb][5] = x1.y; bv[nb][6] = x1.z; bv[nb][7] = x1.w;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[mb][t], bv[nb][t], acc[mb][nb], 0, 0, 0);
  }
}

__device__ __forceinline__ void mma_stage(const GemmSmem<DSPS_BF16> &sm, int wr, int wc, int lane,
                                          f32x16 (&acc)[2][2]) {
  using C = GemmCfg<DSPS_BF16>;
  const int h = lane >> 5, c = lane & 31;
#pragma unroll
  for (int t = 0; t < C::KT / 16; ++t) {
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
      av[mb] = *reinterpret_cast<const bf16x8 *>(&sm.a[(wr * 64 + mb * 32 + c) * C::PITCH + 16 * t + 8 * h]);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
      bv[nb] = *reinterpret_cast<const bf16x8 *>(&sm.b[(wc * 64 + nb * 32 + c) * C::PITCH + 16 * t + 8 * h]);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
  }
}

// Bands whose support meets the observed wavelengths [o_lo, o_hi] (with a
// relative margin far above float rounding): any band left out has zero
// transmission for every element of the chunk, so skipping it is exact.
__device__ __forceinline__ unsigned active_bands(const FilterView &F, float o_lo, float o_hi) {
  unsigned m = 0;
  for (int b = 0; b < F.n_band; ++b) {
    const float2 gr = F.grid[b];
    const float lo = gr.x, hi = gr.x + (float)(F.n_pts - 1) / gr.y;
    if (o_hi * 1.0001f >= lo && o_lo * 0.9999f <= hi) m |= 1u << b;
  }
  return m;
}

// Filter transmission as (T[i], T[i+1] - T[i]) per grid interval, so that an
// interpolation is one aligned 8-byte LDS read and one FMA.  Whole workgroup.
__device__ __forceinline__ void fill_filter_pairs(const FilterView &F, float2 *s_pair) {
  const int n_int = F.n_pts - 1;
  for (int i = threadIdx.x; i < F.n_band * n_int; i += blockDim.x) {
    const int b = i / n_int, k = i - b * n_int;
    const float t0 = F.trans[b * F.n_pts + k], t1 = F.trans[b * F.n_pts + k + 1];
    s_pair[i] = make_float2(t0, t1 - t0);
  }
}

// Transmission of one band at grid coordinate u = (lambda - first) / spacing:
// linear interpolation between grid points, zero outside [0, n_int].  Matches
// filter_at below bit for bit.
__device__ __forceinline__ float filter_pair_at(const float2 *tab, int n_int, float u) {
  const float uc = __builtin_amdgcn_fmed3f(u, 0.0f, (float)n_int);
  const int i = min((int)uc, n_int - 1);
  const float2 pr = tab[i];
  const float t = fmaf(uc - (float)i, pr.y, pr.x);
  return u == uc ? t : 0.0f;
}

// Linear interpolation of a uniformly gridded filter, zero outside.
__device__ __forceinline__ float filter_at(const float *tr, int n_pts, float u) {
  if (!(u >= 0.0f) || !(u <= (float)(n_pts - 1))) return 0.0f;
  int i = (int)u;
  i = i > n_pts - 2 ? n_pts - 2 : i;
  const float f = u - (float)i;
  const float t0 = tr[i];
  return t0 + f * (tr[i + 1] - t0);
}

}  // namespace dsps
