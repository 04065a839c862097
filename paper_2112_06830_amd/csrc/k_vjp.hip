// Reverse mode of the fused magnitudes (Section 2.1: with the SSP block
// fixed, the gradient of the SED flows through the weights; Section 3.4: the
// attenuation is differentiated analytically).
//
// For the magnitude cotangent g_b of galaxy g,
//   gamma_b   = -2.5 g_b / (ln 10 num_b)                      (d m_b / d num_b)
//   G(l)      = sum_b gamma_b T_b((1+z) l) q_l                (cotangent of F L)
//   Lbar(l)   = G(l) F(l)                                     (cotangent of the SED)
//   Wbar[k]   = sum_l Lbar(l) L_SSP[k, l]                     (transposed contraction)
//   A_V, delta, bump: sum_l G L dF/dtheta with F = 10^(-0.4 A_V k_lambda / 4.05)
// then Wbar -> (metallicity weights -> lgmet, sigma_Z) and (age-bin masses ->
// cumulative mass -> SFR table -> parametric SFH) in float64.
//
// Kernels: k_vjp_gamma (per galaxy), k_vjp_gemm (the forward tile recomputed
// on MFMA, never stored; its epilogue writes Lbar and the three dust sums),
// k_vjp_wbar (Lbar . SSP^T on MFMA), k_vjp_weights (one wave per galaxy).
#include "gemm_core.hpp"

namespace dsps {

constexpr float LN10_F = 2.302585092994046f;
constexpr double LN2_D = 0.69314718055994530942;
constexpr double LN10_D = 2.30258509299404568402;

__global__ void k_vjp_gamma(VjpLaunch a) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= a.s_count) return;
  const int s = a.s_begin + local;
  const int g = a.perm[s];
  const int nb = a.n_band;
  for (int b = 0; b < nb; ++b) {
    const float num = a.bands[(size_t)g * 2 * nb + b];
    const float bar = a.mags_bar[(size_t)g * nb + b];
    // a zero cotangent contributes nothing, also for a band with num = 0
    a.gamma[(size_t)s * nb + b] = bar == 0.0f ? 0.0f : -2.5f * bar / (LN10_F * num);
  }
}

// Forward tile recomputed; epilogue forms Lbar and the dust-gradient sums.
__global__ __launch_bounds__(GEMM_THREADS, 2) void k_vjp_gemm(VjpLaunch a) {
  using C = GemmCfg<DSPS_FP32>;
  __shared__ GemmSmem<DSPS_FP32> sm;
  __shared__ float4 s_lc[TILE_L];
  __shared__ float s_q[TILE_L];
  __shared__ float s_red[2][64][3];
  __shared__ float s_gam[TILE_G * DSPS_MAX_BAND];
  __shared__ float2 s_grid[DSPS_MAX_BAND];
  // window lo, window hi, metallicity-row mask, age hi, min and max of (1+z)
  // as float bits
  __shared__ int s_tile[6];
  extern __shared__ float2 s_pair[];   // [n_band][n_pts - 1] filter intervals

  const int group = blockIdx.x, tile = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave & 1, wc = wave >> 1, h = lane >> 5;
  const SspView P = a.ssp;
  const FilterView F = a.flt;
  const int n_band = F.n_band, n_pts = F.n_pts;
  const int g0 = tile * TILE_G;
  const int nvalid = min(TILE_G, a.s_count - g0);

  if (threadIdx.x == 0) {
    s_tile[0] = 1 << 30; s_tile[1] = 0; s_tile[2] = 0; s_tile[3] = 0;
    s_tile[4] = 0x7f7fffff; s_tile[5] = 0;
  }
  __syncthreads();
  if (threadIdx.x < nvalid) {
    const GalaxyRange r = a.range[a.s_begin + g0 + threadIdx.x];
    const int zbits = __float_as_int(a.meta[a.s_begin + g0 + threadIdx.x].zp1);
    atomicMin(&s_tile[0], r.win_lo);
    atomicMax(&s_tile[1], r.win_hi);
    atomicMin(&s_tile[4], zbits);
    atomicMax(&s_tile[5], zbits);
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
  const float zp1_min = __int_as_float(s_tile[4]), zp1_max = __int_as_float(s_tile[5]);
  const int c_first = win_lo / TILE_L;
  const int c_last = (win_hi + TILE_L - 1) / TILE_L;
  const int c_begin = max(group * CHUNKS_PER_GROUP, c_first);
  const int c_end = min((group + 1) * CHUNKS_PER_GROUP, c_last);

  if (c_begin >= c_end) {
    for (int idx = threadIdx.x; idx < nvalid * 3; idx += GEMM_THREADS) {
      const int gl = idx / 3, v = idx % 3;
      a.partial[((size_t)(g0 + gl) * a.n_groups + group) * 3 + v] = 0.0f;
    }
    return;
  }
  const int n_int = n_pts - 1;
  fill_filter_pairs(F, s_pair);

  // Per-galaxy gamma and the filter grids are read from LDS with a runtime
  // band index (per-band registers for 64 elements per lane would exhaust
  // the register file).
  for (int i = threadIdx.x; i < TILE_G * n_band; i += GEMM_THREADS) {
    const int col = i / n_band, b = i % n_band;
    s_gam[col * DSPS_MAX_BAND + b] =
        col < nvalid ? a.gamma[(size_t)(a.s_begin + g0 + col) * n_band + b] : 0.0f;
  }
  if (threadIdx.x < n_band) s_grid[threadIdx.x] = F.grid[threadIdx.x];
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
  float s_k[2] = {0.0f, 0.0f}, s_pw[2] = {0.0f, 0.0f}, s_d[2] = {0.0f, 0.0f};

  const int n_ab = (age_hi + C::KT - 1) / C::KT;
  const int nk = __builtin_popcount(met_mask) * n_ab;
  const int j_first = met_mask ? __builtin_ctz(met_mask) : 0;
  const float *st = P.st32;
  const float *w = (const float *)a.w_pad;
  const int nwp = P.n_wave_pad;

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
    StageRegs<DSPS_FP32> regs;
    int j_cur = j_first, ab_cur = 0;
    if (nk > 0) load_stage<DSPS_FP32>(regs, st, P.k_pad, l0, w, g0, a.s_count, j_cur * AGE_PAD);
    for (int ks = 0; ks < nk; ++ks) {
      __syncthreads();
      store_stage<DSPS_FP32>(regs, sm);
      __syncthreads();
      if (ks + 1 < nk) {
        if (++ab_cur == n_ab) {
          ab_cur = 0;
          j_cur = __builtin_ctz(met_mask & ~((2u << j_cur) - 1u));
        }
        load_stage<DSPS_FP32>(regs, st, P.k_pad, l0, w, g0, a.s_count, j_cur * AGE_PAD + ab_cur * C::KT);
      }
      mma_stage(sm, wr, wc, lane, acc);
    }
    __syncthreads();

    // Bands that can see this chunk for some galaxy of the tile (the others
    // add exact zeros to every sum below).  For each group of four rows (one
    // 16-byte Lbar store per column) the band loop runs outside the elements,
    // so the lookups of the group issue together.
    const unsigned bmask = __builtin_amdgcn_readfirstlane(
        active_bands(F, zp1_min * s_lc[0].x, zp1_max * s_lc[TILE_L - 1].x));
    const int b_lo = bmask ? __builtin_ctz(bmask) : 0;
    const int n_act = bmask ? 32 - __builtin_clz(bmask) - b_lo : 0;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int row0 = wr * 64 + mb * 32 + 8 * r4 + 4 * h;
        float lobs[4][2], gs[4][2];
#pragma unroll
        for (int r1 = 0; r1 < 4; ++r1) {
          const float lam = s_lc[row0 + r1].x;
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) { lobs[r1][nb] = zp1[nb] * lam; gs[r1][nb] = 0.0f; }
        }
        // G = sum_b gamma_b T_b in ascending band order
        for (int k = 0; k < n_act; ++k) {
          const int b = b_lo + k;
          const float2 gr = s_grid[b];
          const float2 *tab = s_pair + b * n_int;
          float gam[2];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) gam[nb] = s_gam[(wc * 64 + nb * 32 + (lane & 31)) * DSPS_MAX_BAND + b];
#pragma unroll
          for (int r1 = 0; r1 < 4; ++r1)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              gs[r1][nb] += gam[nb] * filter_pair_at(tab, n_int, (lobs[r1][nb] - gr.x) * gr.y);
        }
        float out4[2][4];
#pragma unroll
        for (int r1 = 0; r1 < 4; ++r1) {
          const int r = 4 * r4 + r1;
          const float4 lc = s_lc[row0 + r1];
          const float q = s_q[row0 + r1];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            const float powl = exp2f(dl[nb] * lc.y);
            const float kl = lc.z * powl + bp[nb] * lc.w;      // k_lambda
            const float att = exp2f(da[nb] * kl);
            const float gsum = gs[r1][nb] * q;
            acc[mb][nb][r] *= gsum * att;                      // e = G F L
            out4[nb][r1] = gsum * att;
          }
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const int col = wc * 64 + nb * 32 + (lane & 31);
          if (col < nvalid)
            *reinterpret_cast<float4 *>(a.lbar + (size_t)(g0 + col) * nwp + l0 + row0) =
                make_float4(out4[nb][0], out4[nb][1], out4[nb][2], out4[nb][3]);
        }
      }
    }
    // second pass: dust-gradient sums over e = G F L (the per-row factors are
    // recomputed; holding them from the first pass exhausts the registers)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 64 + mb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const float4 lc = s_lc[row];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const float e = acc[mb][nb][r];
          const float k0x = lc.z * exp2f(dl[nb] * lc.y);    // k0 (lambda/5500)^delta
          s_k[nb] += e * (k0x + bp[nb] * lc.w);
          s_pw[nb] += e * k0x * lc.y;
          s_d[nb] += e * lc.w;
        }
      }
    }
  }

#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    s_k[nb] += __shfl_xor(s_k[nb], 32, 64);
    s_pw[nb] += __shfl_xor(s_pw[nb], 32, 64);
    s_d[nb] += __shfl_xor(s_d[nb], 32, 64);
  }
  __syncthreads();
  const int my_nb = h;
  const int col = my_nb * 32 + (lane & 31);
  const float v0 = my_nb ? s_k[1] : s_k[0];
  const float v1 = my_nb ? s_pw[1] : s_pw[0];
  const float v2 = my_nb ? s_d[1] : s_d[0];
  if (wr == 1) { s_red[wc][col][0] = v0; s_red[wc][col][1] = v1; s_red[wc][col][2] = v2; }
  __syncthreads();
  if (wr == 0) {
    const int tcol = wc * 64 + col;
    if (tcol < nvalid) {
      float *out = a.partial + ((size_t)(g0 + tcol) * a.n_groups + group) * 3;
      out[0] = v0 + s_red[wc][col][0];
      out[1] = v1 + s_red[wc][col][1];
      out[2] = v2 + s_red[wc][col][2];
    }
  }
}

// Wbar[s, k] = sum_l Lbar[s, l] L_SSP[k, l] over the tile's wavelength window.
// Rows (M) are SSP rows k, columns (N) galaxies, reduction over wavelength.
__global__ __launch_bounds__(GEMM_THREADS, 2) void k_vjp_wbar(VjpLaunch a) {
  using C = GemmCfg<DSPS_FP32>;
  __shared__ GemmSmem<DSPS_FP32> sm;
  __shared__ int s_tile[2];
  const int kblk = blockIdx.x, tile = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave & 1, wc = wave >> 1, h = lane >> 5;
  const SspView P = a.ssp;
  const int g0 = tile * TILE_G;
  const int nvalid = min(TILE_G, a.s_count - g0);
  const int nwp = P.n_wave_pad;

  if (threadIdx.x == 0) { s_tile[0] = 1 << 30; s_tile[1] = 0; }
  __syncthreads();
  if (threadIdx.x < nvalid) {
    const GalaxyRange r = a.range[a.s_begin + g0 + threadIdx.x];
    atomicMin(&s_tile[0], r.win_lo);
    atomicMax(&s_tile[1], r.win_hi);
  }
  __syncthreads();
  const int l_begin = (s_tile[0] / TILE_L) * TILE_L;
  const int l_end = ((s_tile[1] + TILE_L - 1) / TILE_L) * TILE_L;
  const int k0 = kblk * TILE_L;

  f32x16 acc[2][2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.0f;

  const int nk = l_end > l_begin ? (l_end - l_begin) / C::KT : 0;
  StageRegs<DSPS_FP32> regs;
  if (nk > 0) load_stage<DSPS_FP32>(regs, P.sk32, nwp, k0, a.lbar, g0, a.s_count, l_begin);
  for (int ks = 0; ks < nk; ++ks) {
    __syncthreads();
    store_stage<DSPS_FP32>(regs, sm);
    __syncthreads();
    if (ks + 1 < nk)
      load_stage<DSPS_FP32>(regs, P.sk32, nwp, k0, a.lbar, g0, a.s_count, l_begin + (ks + 1) * C::KT);
    mma_stage(sm, wr, wc, lane, acc);
  }

  const int kp = P.k_pad;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = wc * 64 + nb * 32 + (lane & 31);
    if (col >= nvalid) continue;
    float *out = a.wbar + (size_t)(g0 + col) * kp + k0;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int row0 = wr * 64 + mb * 32 + 8 * r4 + 4 * h;
        if (k0 + row0 >= kp) continue;      // padding rows of the K-major table
        *reinterpret_cast<float4 *>(out + row0) =
            make_float4(acc[mb][nb][4 * r4], acc[mb][nb][4 * r4 + 1], acc[mb][nb][4 * r4 + 2],
                        acc[mb][nb][4 * r4 + 3]);
      }
  }
}

// ----------------------------------------------------------------- weights
__device__ __forceinline__ void wave_sync_v() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double sfr_base(double t, double a, double tau, double alpha) {
  const double x = t / tau;
  return a * exp(alpha * log(x) - x);
}

// Cosmic time t(z): LCDM closed form, else wave-cooperative quadrature (the
// same forms as the forward kernel).
__device__ double vjp_age_at_z(double z, const CosmoArgs &c, const GaussLegendre &gl, int lane) {
  if (c.lcdm) {
    if (c.ol <= 0.0) return (2.0 / 3.0) * c.hubble_time_gyr * pow(1.0 + z, -1.5) / sqrt(c.om0);
    return (2.0 / (3.0 * sqrt(c.ol))) * c.hubble_time_gyr * asinh(sqrt(c.ol / c.om0) * pow(1.0 + z, -1.5));
  }
  const double s_hi = sqrt(1.0 / (1.0 + z));
  const int panel = lane / GL_N, node = lane % GL_N;
  const double hh = s_hi * 0.25;
  const double s = hh * (panel + 0.5) + 0.5 * hh * gl.x[node];
  const double f = 2.0 * s * s / sqrt(c.om0 + c.ol * pow(s, -6.0 * c.w0));
  return c.hubble_time_gyr * wave_sum(0.5 * hh * gl.w[node] * f);
}

__device__ __forceinline__ int bracket(double t, const double *tt, int n_t) {
  int lo = 0, hi = n_t - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tt[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_vjp_weights(VjpLaunch a) {
  extern __shared__ double lds[];
  const int n_t = a.n_t;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *tt = lds;
  double *wbase = lds + n_t + wave * (2 * n_t + 3 * AGE_PAD + 2);
  double *buf = wbase;                 // SFR values, then the cumulative-mass cotangent
  double *mc = wbase + n_t;            // cumulative mass
  double *em = wbase + 2 * n_t;        // [n_age + 1] mass at the edges
  double *mage = em + AGE_PAD + 1;     // [n_age]
  double *mbar = mage + AGE_PAD;       // [n_age] age-mass cotangent (+1 pad)

  for (int n = threadIdx.x; n < n_t; n += blockDim.x) tt[n] = a.t_table[n];
  __syncthreads();
  const int local = blockIdx.x * WEIGHT_WAVES + wave;
  if (local >= a.s_count) return;
  const int s = a.s_begin + local;
  const int g = a.perm[s];
  const SspView P = a.ssp;
  const int n_age = P.n_age, n_met = P.n_met;
  const double z = (double)a.z[g];
  const double t_obs = vjp_age_at_z(z, a.cosmo, a.gl, lane);

  double pa = 0, ptau = 0, palpha = 0, pq = 0, ptq = 0;
  if (a.sfr) {
    const double *row = a.sfr + (size_t)g * n_t;
    for (int n = lane; n < n_t; n += 64) buf[n] = row[n];
  } else {
    pa = a.sfh_params[g]; ptau = a.sfh_params[a.n_gal + g]; palpha = a.sfh_params[2 * a.n_gal + g];
    pq = a.sfh_params[3 * a.n_gal + g]; ptq = a.sfh_params[4 * a.n_gal + g];
    for (int n = lane; n < n_t; n += 64) {
      const double v = (tt[n] - ptq) * (1.0 / QUENCH_WIDTH);
      buf[n] = sfr_base(tt[n], pa, ptau, palpha) * (1.0 - pq * 0.5 * erfc(-v * 0.70710678118654752440));
    }
  }
  wave_sync_v();
  if (lane == 0) mc[0] = 0.0;
  for (int m = lane; m < n_t - 1; m += 64)
    mc[m + 1] = 0.5 * (buf[m] + buf[m + 1]) * (tt[m + 1] - tt[m]) * YEARS_PER_GYR;
  wave_sync_v();
  {
    const int len = n_t - 1, per = (len + 63) / 64;
    const int b0 = 1 + lane * per, b1 = min(1 + (lane + 1) * per, n_t);
    double run = 0.0;
    for (int n = b0; n < b1; ++n) run += mc[n];
    double incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double up = __shfl_up(incl, off, 64);
      if (lane >= off) incl += up;
    }
    double acc = incl - run;
    for (int n = b0; n < b1; ++n) { acc += mc[n]; mc[n] = acc; }
  }
  wave_sync_v();
  for (int e = lane; e <= n_age; e += 64) {
    const double t = t_obs - P.age_edges[e];
    double m = 0.0;
    if (t > tt[0]) {
      if (t >= tt[n_t - 1]) m = mc[n_t - 1];
      else {
        const int lo = bracket(t, tt, n_t);
        const double f = (t - tt[lo]) / (tt[lo + 1] - tt[lo]);
        m = mc[lo] + f * (mc[lo + 1] - mc[lo]);
      }
    }
    em[e] = m;
  }
  wave_sync_v();
  for (int i = lane; i < n_age; i += 64) mage[i] = em[i] - em[i + 1];
  wave_sync_v();

  // ---- Wbar -> metallicity-weight and age-mass cotangents
  const double lgmet = (double)a.lgmet[g];
  const double sig = (double)a.sigma_z[g];
  const double inv_sig = 1.0 / sig;
  const float *wb = a.wbar + (size_t)local * P.k_pad;
  double d_lgmet = 0.0, d_sig = 0.0;
  // wb holds Y[j] = Wbar[j] - Wbar[j-1] (Y[0] = Wbar[0]) from the
  // metallicity-differenced table.  Bin j spans edges j and j+1,
  // P_j = C(u_{j+1}) - C(u_j); the cotangent of the CDF at an interior edge j
  // is Pbar_{j-1} - Pbar_j = -m_age Y[j], and m_age_bar = sum_j Wbar[j] P_j.
  for (int i = lane; i < n_age; i += 64) {
    const double mu = lgmet + a.slope * (P.lg_age[i] - a.pivot);
    const double m_i = mage[i];
    double mb = 0.0, wcum = 0.0;
    double c_lo = 0.0, u_lo = 0.0;    // CDF and u at edge j (the lower edge of bin j)
    for (int j = 0; j < n_met; ++j) {
      const double y = (double)wb[j * AGE_PAD + i];
      wcum += y;                       // Wbar[j]
      if (j >= 1) {
        const double ubar = -m_i * y * triweight_pdf(u_lo);
        d_lgmet -= ubar * inv_sig;
        d_sig -= ubar * u_lo * inv_sig;
      }
      double c_hi = 1.0, u_hi = 0.0;   // upper edge of the last bin is +inf
      if (j + 1 < n_met) {
        u_hi = (P.met_edges[j + 1] - mu) * inv_sig;
        c_hi = triweight_cdf(u_hi);
      }
      mb += wcum * (c_hi - c_lo);
      c_lo = c_hi;
      u_lo = u_hi;
    }
    mbar[i] = mb;
  }
  d_lgmet = wave_sum(d_lgmet);
  d_sig = wave_sum(d_sig);
  wave_sync_v();

  // ---- age-mass cotangent -> mass at the edges -> cumulative nodes
  double *mcb = buf;   // SFR values are no longer needed
  for (int n = lane; n < n_t; n += 64) mcb[n] = 0.0;
  wave_sync_v();
  for (int e = lane; e <= n_age; e += 64) {
    const double ebar = (e < n_age ? mbar[e] : 0.0) - (e > 0 ? mbar[e - 1] : 0.0);
    const double t = t_obs - P.age_edges[e];
    if (!(t > tt[0]) || ebar == 0.0) continue;
    if (t >= tt[n_t - 1]) { atomicAdd(&mcb[n_t - 1], ebar); continue; }
    const int lo = bracket(t, tt, n_t);
    const double f = (t - tt[lo]) / (tt[lo + 1] - tt[lo]);
    atomicAdd(&mcb[lo], (1.0 - f) * ebar);
    atomicAdd(&mcb[lo + 1], f * ebar);
  }
  wave_sync_v();
  // suffix sums Suf[n] = sum_{m >= n} mcb[m] (blocked, in place)
  {
    const int per = (n_t + 63) / 64;
    const int b0 = lane * per, b1 = min((lane + 1) * per, n_t);
    double run = 0.0;
    for (int n = b0; n < b1; ++n) run += mcb[n];
    double incl = run;   // inclusive suffix over lanes >= this lane
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double dn = __shfl_down(incl, off, 64);
      if (lane + off < 64) incl += dn;
    }
    double acc = incl - run;   // sum over later lanes
    for (int n = b1 - 1; n >= b0; --n) { acc += mcb[n]; mcb[n] = acc; }
  }
  wave_sync_v();

  // ---- SFR cotangent and the parametric-history pull-back
  double dp[5] = {0, 0, 0, 0, 0};
  for (int n = lane; n < n_t; n += 64) {
    double sb = 0.0;
    if (n >= 1) sb += (tt[n] - tt[n - 1]) * mcb[n];
    if (n + 1 < n_t) sb += (tt[n + 1] - tt[n]) * mcb[n + 1];
    sb *= 0.5 * YEARS_PER_GYR;
    if (a.sfr_bar) a.sfr_bar[(size_t)g * n_t + n] = sb;
    if (!a.sfr) {
      const double t = tt[n];
      const double base = sfr_base(t, pa, ptau, palpha);
      const double v = (t - ptq) * (1.0 / QUENCH_WIDTH);
      const double phi = 0.5 * erfc(-v * 0.70710678118654752440);
      const double pdf = exp(-0.5 * v * v) * 0.39894228040143267794;
      const double quench = 1.0 - pq * phi;
      const double sv = base * quench;
      dp[0] += sb * base * quench / pa;
      dp[1] += sb * sv * (-palpha / ptau + t / (ptau * ptau));
      dp[2] += sb * sv * log(t / ptau);
      dp[3] += sb * (-base * phi);
      dp[4] += sb * base * pq * pdf / QUENCH_WIDTH;
    }
  }
  if (!a.sfr && a.sfh_params_bar) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double v = wave_sum(dp[k]);
      if (lane == 0) a.sfh_params_bar[(size_t)k * a.n_gal + g] = v;
    }
  }

  if (lane == 0) {
    if (a.lgmet_bar) a.lgmet_bar[g] = (float)d_lgmet;
    if (a.sigma_bar) a.sigma_bar[g] = (float)d_sig;
    double sk = 0.0, spw = 0.0, sd = 0.0;
    const float *p = a.partial + (size_t)local * a.n_groups * 3;
    for (int gr = 0; gr < a.n_groups; ++gr) {
      sk += p[3 * gr];
      spw += p[3 * gr + 1];
      sd += p[3 * gr + 2];
    }
    // dF/dA_V = F (-0.4 ln10 / 4.05) k;  dF/d delta = F (-0.4 ln10 A_V / 4.05)
    // k0 (l/5500)^delta ln(l/5500);  dF/d bump = F (-0.4 ln10 A_V / 4.05) D
    const double c1 = -0.4 * LN10_D / DUST_RV;
    const double av = (double)a.av[g];
    if (a.av_bar) a.av_bar[g] = (float)(c1 * sk);
    if (a.delta_bar) a.delta_bar[g] = (float)(c1 * av * LN2_D * spw);
    if (a.bump_bar) a.bump_bar[g] = (float)(c1 * av * sd);
  }
}

int launch_vjp(const VjpLaunch &a, int stage, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  const int tiles = (a.s_count + TILE_G - 1) / TILE_G;
  if (stage == 0) {
    hipLaunchKernelGGL(k_vjp_gamma, dim3((a.s_count + 255) / 256), dim3(256), 0, stream, a);
  } else if (stage == 1) {
    ProfScope prof(DSPS_KERNEL_VJP_GEMM, stream);
    const size_t lds = sizeof(float2) * a.flt.n_band * (a.flt.n_pts - 1);
    hipLaunchKernelGGL(k_vjp_gemm, dim3(a.n_groups, tiles), dim3(GEMM_THREADS), lds, stream, a);
  } else if (stage == 2) {
    ProfScope prof(DSPS_KERNEL_VJP_WBAR, stream);
    hipLaunchKernelGGL(k_vjp_wbar, dim3(a.ssp.sk_rows / TILE_L, tiles), dim3(GEMM_THREADS), 0, stream, a);
  } else {
    const size_t lds = sizeof(double) * (a.n_t + WEIGHT_WAVES * (2 * a.n_t + 3 * AGE_PAD + 2));
    if (lds > 65536) {
      const int rc = hip_fail(hipFuncSetAttribute((const void *)k_vjp_weights,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                              "k_vjp_weights LDS attribute");
      if (rc) return rc;
    }
    ProfScope prof(DSPS_KERNEL_VJP_WEIGHTS, stream);
    hipLaunchKernelGGL(k_vjp_weights, dim3((a.s_count + WEIGHT_WAVES - 1) / WEIGHT_WAVES),
                       dim3(64 * WEIGHT_WAVES), lds, stream, a);
  }
  return hip_fail(hipGetLastError(), "vjp launch");
}

}  // namespace dsps
