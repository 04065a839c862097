// MFMA GEMM core shared by the fused-magnitude, SED and adjoint kernels.
//
// A workgroup of four wave64s computes a 128 x 128 output tile in a 2 x 2
// arrangement of 64 x 64 wave tiles (2 x 2 MFMA 32x32 blocks per wave).  Both
// operands are K-contiguous rows in memory.  A K stage is one 64-byte slice of
// every operand row (16 FP32 or 32 BF16 values); it travels through registers
// into one of two LDS stage buffers, and every lane feeds MFMA from 16-byte
// LDS reads.
#pragma once

#include <type_traits>

#include "dsps_internal.hpp"

namespace dsps {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// Native 16-byte vector for staging (HIP's uint4 is a struct wrapper that the
// optimiser does not always keep in registers).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct GemmCfg;
// KT: K elements per stage.  A stage is UNITS units of UNIT_K consecutive K
// elements each, from anywhere in K: the stage lists of the fused kernels
// skip units that are zero for every member of a tile.  A unit is what one
// MFMA step takes from each operand row (float32: two steps), so a galaxy's
// sum adds its own units in ascending K order whatever else its tile holds,
// and units of zeros add exact zeros.
template <> struct GemmCfg<DSPS_FP32> {
  using elem = float;
  static constexpr int KT = 16;
  static constexpr int UNITS = 2, UNIT_K = 8;
};
template <> struct GemmCfg<DSPS_BF16> {
  using elem = uint16_t;
  static constexpr int KT = 32;
  static constexpr int UNITS = 2, UNIT_K = 16;
};
constexpr int STAGE_UNITS = 4;   // 16-byte units per operand row and stage

// LDS position of unit j of stage row r.  The XOR of row bits 1..3 into the
// unit index puts the rows read together by one 16-byte LDS access (8 or 16
// consecutive rows, one unit) and the units written together (4 units of 2
// or 4 consecutive rows) on distinct 4-bank groups, without padding.
__device__ __forceinline__ int stage_unit(int row, int j) {
  return row * STAGE_UNITS + (j ^ (((row >> 1) ^ (row >> 2)) & 3));
}

template <int PREC>
struct GemmSmem {
  static_assert(GemmCfg<PREC>::KT * sizeof(typename GemmCfg<PREC>::elem) == 16 * STAGE_UNITS,
                "one stage row is four 16-byte units");
  u32x4 a[TILE_L * STAGE_UNITS];
  u32x4 b[TILE_G * STAGE_UNITS];
};

// Stage one K slice of 128 rows from a K-contiguous matrix into registers
// (vectors of 16 bytes).
template <int PREC>
struct StageRegs {
  static constexpr int NV = TILE_L * STAGE_UNITS / GEMM_THREADS;   // vectors per thread
  u32x4 a[NV];
  u32x4 b[NV];
};

// Blocks are dispatched round-robin over the 8 XCDs by linear id.  All
// groups of one galaxy tile go to the same XCD (the tile's operand rows then
// stay in that XCD's L2): block b runs on XCD b % 8 and takes tile
// (b / 8 / G) * 8 + b % 8, group (b / 8) % G.  A grid of
// ceil(tiles / 8) * 8 * G blocks covers every (tile, group).
__device__ __forceinline__ void xcd_tile_group(int b, int groups, int &tile, int &group) {
  const int xcd = b & 7, slot = b >> 3;
  tile = (slot / groups) * 8 + xcd;
  group = slot % groups;
}

// The A rows this thread stages, one per staging vector: vector v of thread
// t holds unit (t + 256 v) % 4 of tile row (t + 256 v) / 4, read from A row
// r[v] (l0 + the tile row for a contiguous block of rows).
template <int PREC>
struct ARows {
  int r[StageRegs<PREC>::NV];
};
template <int PREC>
__device__ __forceinline__ ARows<PREC> linear_rows(int l0) {
  ARows<PREC> a;
#pragma unroll
  for (int v = 0; v < StageRegs<PREC>::NV; ++v)
    a.r[v] = l0 + (int)(threadIdx.x + v * GEMM_THREADS) / STAGE_UNITS;
  return a;
}
// Tile row of staging vector v of this thread.
template <int PREC>
__device__ __forceinline__ int stage_row(int v) {
  return (int)(threadIdx.x + v * GEMM_THREADS) / STAGE_UNITS;
}

// The operands of a K loop as buffer resources, plus this thread's row byte
// offsets (one per staging vector).  A buffer load outside its resource's
// range returns zeros: B rows past the tile's last galaxy, and units of
// zeros, cost no branch.
template <int PREC>
struct GemmOps {
  __amdgpu_buffer_rsrc_t a, b;
  int ra[StageRegs<PREC>::NV], rb[StageRegs<PREC>::NV];
};
// Raw buffer resource over n_bytes from p (dword 3 of the gfx9 family).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, size_t n_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n_bytes, 0x00020000);
}
// A: a matrix of a_elems elements in rows of a_stride, this thread's rows ar;
// B: the tile's rows from b_tile (its first galaxy), b_stride apart, of which
// the first b_valid hold data.
template <int PREC>
__device__ __forceinline__ GemmOps<PREC> gemm_ops(const typename GemmCfg<PREC>::elem *a_base,
                                                  size_t a_elems, int a_stride, const ARows<PREC> &ar,
                                                  const typename GemmCfg<PREC>::elem *b_tile,
                                                  int b_valid, int b_stride) {
  using elem = typename GemmCfg<PREC>::elem;
  GemmOps<PREC> o;
  o.a = buffer_rsrc(a_base, a_elems * sizeof(elem));
  o.b = buffer_rsrc(b_tile, (size_t)max(b_valid, 0) * b_stride * sizeof(elem));
#pragma unroll
  for (int v = 0; v < StageRegs<PREC>::NV; ++v) {
    o.ra[v] = ar.r[v] * a_stride * (int)sizeof(elem);
    o.rb[v] = stage_row<PREC>(v) * b_stride * (int)sizeof(elem);
  }
  return o;
}

// Where this thread's 16 bytes of a K stage come from: byte offsets in its A
// and B rows (ZERO_UNIT_BYTES in B: zeros) and, float32 only, factors of the
// B rows applied as the stage is written to LDS (or null).  Thread t stages LDS
// unit c = t % 4 of each of its rows: in float32 piece c / 2 of K unit c % 2
// (MFMA step s pairs LDS units s / 4 and 2 + s / 4), in bfloat16 piece c % 2
// of K unit c / 2 (MFMA step s takes LDS units 2s and 2s + 1).
struct UnitSrc {
  int a, b;
  const float *bscale;
};
__device__ __forceinline__ int stage_col() { return (int)(threadIdx.x % STAGE_UNITS); }
// This thread's piece of stage s from a list of K units (-1: a unit of zeros).
template <int PREC>
__device__ __forceinline__ int unit_piece(const int *units, int s, int col) {
  using C = GemmCfg<PREC>;
  constexpr int EPP = 16 / (int)sizeof(typename C::elem);   // elements per piece
  const int v = PREC == DSPS_FP32 ? col & 1 : col >> 1;
  const int q = PREC == DSPS_FP32 ? col >> 1 : col & 1;
  const int k = units[C::UNITS * s + v];
  return k < 0 ? -1 : k + q * EPP;
}
// The same for K units of a contiguous range from k0: unit v of stage s
// starts at k0 + KT s + UNIT_K v.
template <int PREC>
__device__ __forceinline__ int contiguous_piece(int k0, int s, int col) {
  using C = GemmCfg<PREC>;
  constexpr int EPP = 16 / (int)sizeof(typename C::elem);
  const int v = PREC == DSPS_FP32 ? col & 1 : col >> 1;
  const int q = PREC == DSPS_FP32 ? col >> 1 : col & 1;
  return k0 + C::KT * s + C::UNIT_K * v + q * EPP;
}
// An offset past the end of every B resource (tile rows stay far below it).
constexpr int ZERO_UNIT_BYTES = 0x40000000;

// Byte offsets of a 16-byte piece at element offset k of both operands
// (k < 0: a piece of zeros, read from the start of A and past the end of B).
template <int PREC>
__device__ __forceinline__ int2 piece_bytes(int k) {
  constexpr int ES = (int)sizeof(typename GemmCfg<PREC>::elem);
  return make_int2(max(k, 0) * ES, k < 0 ? ZERO_UNIT_BYTES : k * ES);
}

template <int PREC>
__device__ __forceinline__ void load_units(StageRegs<PREC> &r, const GemmOps<PREC> &o, UnitSrc u) {
#pragma unroll
  for (int v = 0; v < StageRegs<PREC>::NV; ++v) {
    r.a[v] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(o.a, o.ra[v] + u.a, 0, 0));
    r.b[v] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(o.b, o.rb[v] + u.b, 0, 0));
  }
}

// A thread's 16 bytes go to LDS unit t % 4 of their row.
template <int PREC>
__device__ __forceinline__ void store_stage(const StageRegs<PREC> &r, GemmSmem<PREC> &sm) {
  using S = StageRegs<PREC>;
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    const int idx = threadIdx.x + v * GEMM_THREADS;
    const int u = stage_unit(idx / STAGE_UNITS, idx % STAGE_UNITS);
    sm.a[u] = r.a[v];
    sm.b[u] = r.b[v];
  }
}

// B rows times per-row factors (float32 stages): row r of the staged B slice
// is multiplied by scale[r], rounded once per element.
__device__ __forceinline__ void scale_stage_b(StageRegs<DSPS_FP32> &r, const float *scale) {
  using S = StageRegs<DSPS_FP32>;
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    const float f = scale[(threadIdx.x + v * GEMM_THREADS) / STAGE_UNITS];
    r.b[v].x = __float_as_uint(__uint_as_float(r.b[v].x) * f);
    r.b[v].y = __float_as_uint(__uint_as_float(r.b[v].y) * f);
    r.b[v].z = __float_as_uint(__uint_as_float(r.b[v].z) * f);
    r.b[v].w = __float_as_uint(__uint_as_float(r.b[v].w) * f);
  }
}

__device__ __forceinline__ float4 as_float4(u32x4 v) {
  return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                     __uint_as_float(v.w));
}

// acc[mb][nb] += A[rows of mb] . B[cols of nb] over one K stage.
__device__ __forceinline__ void mma_stage(const GemmSmem<DSPS_FP32> &sm, int wr, int wc, int lane,
                                          f32x16 (&acc)[2][2]) {
  const int h = lane >> 5, c = lane & 31;
  // Lane half h supplies LDS row position 8h + t at MFMA step t, for A and B
  // alike: each lane reads units 2h and 2h + 1 of its rows.  With K unit v's
  // two 16-byte pieces in LDS units v and v + 2 (unit_piece), step t takes
  // elements t % 4 and 4 + t % 4 of K unit t / 4.
  float av[2][8], bv[2][8];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const int row = wr * 64 + mb * 32 + c;
    const float4 x0 = as_float4(sm.a[stage_unit(row, 2 * h)]);
    const float4 x1 = as_float4(sm.a[stage_unit(row, 2 * h + 1)]);
    av[mb][0] = x0.x; av[mb][1] = x0.y; av[mb][2] = x0.z; av[mb][3] = x0.w;
    av[mb][4] = x1.x; av[mb][5] = x1.y; av[mb][6] = x1.z; av[mb][7] = x1.w;
  }
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int row = wc * 64 + nb * 32 + c;
    const float4 x0 = as_float4(sm.b[stage_unit(row, 2 * h)]);
    const float4 x1 = as_float4(sm.b[stage_unit(row, 2 * h + 1)]);
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

__device__ __forceinline__ void mma_stage(const GemmSmem<DSPS_BF16> &sm, int wr, int wc, int lane,
                                          f32x16 (&acc)[2][2]) {
  const int h = lane >> 5, c = lane & 31;
  // MFMA step t takes contraction indices 16t .. 16t + 15; lane half h holds
  // 16t + 8h .. 16t + 8h + 7, which is unit 2t + h.
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
      av[mb] = __builtin_bit_cast(bf16x8, sm.a[stage_unit(wr * 64 + mb * 32 + c, 2 * t + h)]);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
      bv[nb] = __builtin_bit_cast(bf16x8, sm.b[stage_unit(wc * 64 + nb * 32 + c, 2 * t + h)]);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
  }
}

// One half of a float32 stage's MFMA operands: half j holds LDS units 2h + j
// of the lane's A and B rows (steps 4j .. 4j + 3 of mma_stage).
struct HalfStage {
  float4 a[2], b[2];
};
__device__ __forceinline__ void read_half(const GemmSmem<DSPS_FP32> &sm, int j, int wr, int wc,
                                          int lane, HalfStage &f) {
  const int h = lane >> 5, c = lane & 31;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) f.a[mb] = as_float4(sm.a[stage_unit(wr * 64 + mb * 32 + c, 2 * h + j)]);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) f.b[nb] = as_float4(sm.b[stage_unit(wc * 64 + nb * 32 + c, 2 * h + j)]);
}
// Steps 4j .. 4j + 3 of mma_stage, in its order for every accumulator.
__device__ __forceinline__ void mma_half(const HalfStage &f, f32x16 (&acc)[2][2]) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[mb][t], f.b[nb][t], acc[mb][nb], 0, 0, 0);
}

// The K loop of one output tile over nk stages; unit(s) says where this
// thread's unit of stage s comes from (a UnitSrc).  Two LDS stage buffers:
// while stage s feeds MFMA, stage s + 1 is written to the other buffer and
// stage s + 2 is loaded into registers, with one barrier per stage.  On
// entry no wave may still read sm; on return every wave has passed a barrier
// after its last read of it.  after(ks) runs in every wave right after the
// MFMAs of stage ks (register work on the accumulators only).
struct NoStageHook {
  __device__ void operator()(int) const {}
};
//
// SPLIT (float32): the barrier sits between the two halves of a stage's
// MFMAs, and the first half of the next stage's operands is read from LDS
// right after it, while the second half runs, so that no stage starts by
// waiting on its LDS reads.  Every accumulator takes the same steps in the
// same order as without it.
template <int PREC, bool SPLIT = false, typename UnitFn, typename StageHook = NoStageHook>
__device__ __forceinline__ void gemm_kloop(GemmSmem<PREC> *sm, const GemmOps<PREC> &ops, int nk,
                                           UnitFn unit, int wr, int wc, int lane,
                                           f32x16 (&acc)[2][2], StageHook after = StageHook()) {
  static_assert(!SPLIT || PREC == DSPS_FP32, "split stages are float32 only");
  StageRegs<PREC> regs;
  const float *pending = nullptr;   // B factors of the stage held in regs
  auto load = [&](int s) {
    const UnitSrc u = unit(s);
    load_units<PREC>(regs, ops, u);
    pending = u.bscale;
  };
  auto store = [&](GemmSmem<PREC> &buf) {
    if constexpr (PREC == DSPS_FP32) {
      if (pending) scale_stage_b(regs, pending);
    }
    store_stage(regs, buf);
  };
  if (nk > 0) {
    load(0);
    store(sm[0]);
    if (nk > 1) load(1);
  }
  __syncthreads();
  if constexpr (SPLIT) {
    HalfStage f0, f1;
    if (nk > 0) read_half(sm[0], 0, wr, wc, lane, f0);
    for (int ks = 0; ks < nk; ++ks) {
      read_half(sm[ks & 1], 1, wr, wc, lane, f1);
      mma_half(f0, acc);
      if (ks + 1 < nk) {
        // the other buffer's last reads (stage ks - 1) ended before the
        // previous barrier
        store(sm[(ks + 1) & 1]);
        if (ks + 2 < nk) load(ks + 2);
      }
      __syncthreads();
      if (ks + 1 < nk) read_half(sm[(ks + 1) & 1], 0, wr, wc, lane, f0);
      mma_half(f1, acc);
      after(ks);
    }
    // every read of sm, the last stage's second half included, ended before
    // the last iteration's barrier
  } else {
    for (int ks = 0; ks < nk; ++ks) {
      mma_stage(sm[ks & 1], wr, wc, lane, acc);
      after(ks);
      if (ks + 1 < nk) {
        store(sm[(ks + 1) & 1]);
        if (ks + 2 < nk) load(ks + 2);
      }
      __syncthreads();
    }
  }
}

// Age-dependent attenuation (Section 3.4.1, Eq. agedep_dust_csp) over an
// age-major K loop of metallicity pieces grouped by attenuation group: ages
// [0, age_young) share the young-star dust, ages [age_old, ...) the old-star
// dust, each age between has its own transition value, and no stage mixes
// two groups.  After the last stage of a group (tag >= 0: an age of the
// group) every wave folds the group's partial SED into sed += F_att(group)
// acc and restarts acc; lc holds the tile's per-row (lambda, log2(lambda/5500), k0,
// bump shape) constants.  Per column block nb: the young and old dust
// exponents and slopes and the bump amplitude.
struct AgeFold {
  const short *tag;    // per stage: an age of the group to fold after it, or -1
  int age_young, age_old;
  double pivot, width;
  const double *lg_age;
  float da_y[2], dl_y[2], da_o[2], dl_o[2], bp[2];

  __device__ __forceinline__ void operator()(int ks, f32x16 (&sed)[2][2], f32x16 (&acc)[2][2],
                                             const float4 *lc, int wr, int h) const {
    const int age = tag[ks];
    if (age < 0) return;
    const bool young = age < age_young, old = age >= age_old;
    // the group's transition weight: 0 young, 1 old, T_erf in between
    const float t = young ? 0.0f
                          : (old ? 1.0f : (float)mdf_transition(lg_age[age], pivot, width));
    float da[2], dl[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      da[nb] = t == 1.0f ? da_o[nb] : da_y[nb] + (da_o[nb] - da_y[nb]) * t;
      dl[nb] = t == 1.0f ? dl_o[nb] : dl_y[nb] + (dl_o[nb] - dl_y[nb]) * t;
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const float4 c = lc[row];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const float k0x = __fmul_rn(c.z, __builtin_amdgcn_exp2f(dl[nb] * c.y));
          const float kl = fmaf(bp[nb], c.w, k0x);
          sed[mb][nb][r] = fmaf(__builtin_amdgcn_exp2f(da[nb] * kl), acc[mb][nb][r], sed[mb][nb][r]);
          acc[mb][nb][r] = 0.0f;
        }
      }
  }
};

// A wave's reduction of one int per lane (bitwise or, minimum or maximum),
// left in lane 63 and read from there: prefix steps within rows of 16 lanes,
// then row broadcasts.  A lane whose source is outside its row keeps its own
// value, which every operation leaves unchanged.  Every lane of the wave must
// be active.
enum { WAVE_OR, WAVE_MIN, WAVE_MAX };
template <int OP>
__device__ __forceinline__ int wave_join_op(int x, int y) {
  return OP == WAVE_OR ? (x | y) : (OP == WAVE_MIN ? min(x, y) : max(x, y));
}
template <int OP, int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int wave_join_step(int x) {
  return wave_join_op<OP>(x, __builtin_amdgcn_update_dpp(x, x, CTRL, ROW_MASK, 0xf, false));
}
template <int OP>
__device__ __forceinline__ int wave_join(int x) {
  x = wave_join_step<OP, 0x111>(x);         // row_shr:1
  x = wave_join_step<OP, 0x112>(x);         // row_shr:2
  x = wave_join_step<OP, 0x114>(x);         // row_shr:4
  x = wave_join_step<OP, 0x118>(x);         // row_shr:8
  x = wave_join_step<OP, 0x142, 0xa>(x);    // row_bcast:15
  x = wave_join_step<OP, 0x143, 0xc>(x);    // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
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

// Bands whose table covers the observed wavelengths [o_lo, o_hi] with a
// relative margin far above float rounding: every lookup of such a band lands
// inside its table, so the clamp and the outside test can be left out.
__device__ __forceinline__ unsigned interior_bands(const FilterView &F, float o_lo, float o_hi) {
  unsigned m = 0;
  for (int b = 0; b < F.n_band; ++b) {
    const float2 gr = F.grid[b];
    const float lo = gr.x, hi = gr.x + (float)(F.n_pts - 1) / gr.y;
    if (o_lo >= lo * 1.00002f && o_hi <= hi * 0.99998f) m |= 1u << b;
  }
  return m;
}

// Filter transmission tables in LDS: band b at b * filter_stride(n_pts), its
// n_pts points followed by one pad entry repeating the last, so that an
// interpolation at the table's upper end needs no index clamp.
__host__ __device__ inline int filter_stride(int n_pts) { return n_pts + 1; }

// Whole workgroup.
__device__ __forceinline__ void fill_filter_table(const FilterView &F, float *s_tr) {
  const int stride = filter_stride(F.n_pts);
  for (int i = threadIdx.x; i < F.n_band * stride; i += blockDim.x) {
    const int b = i / stride, k = min(i - b * stride, F.n_pts - 1);
    s_tr[i] = F.trans[b * F.n_pts + k];
  }
}

// Transmission of one band (padded table tr, n_int + 1 points) at grid
// coordinate u = (lambda - first) / spacing, passed as u = lambda * (1 /
// spacing) - first / spacing: linear interpolation between grid points, zero
// outside [0, n_int].  The two points come from one paired LDS read.
__device__ __forceinline__ float filter_table_at(const float *tr, int n_int, float u) {
  const float uc = __builtin_amdgcn_fmed3f(u, 0.0f, (float)n_int);
  const int i = (int)uc;                          // <= n_int: the pad covers i + 1
  const float t0 = tr[i], t1 = tr[i + 1];
  const float t = fmaf(__builtin_amdgcn_fractf(uc), t1 - t0, t0);
  return u == uc ? t : 0.0f;
}
// The same for a u known to lie in [0, n_int] (an interior band): equal to
// filter_table_at there, without the clamp and the outside test.
__device__ __forceinline__ float filter_table_inside(const float *tr, float u) {
  const int i = (int)u;
  const float t0 = tr[i], t1 = tr[i + 1];
  return fmaf(__builtin_amdgcn_fractf(u), t1 - t0, t0);
}

}  // namespace dsps
