// SSP weights: parametric SFH table, cumulative mass formed, age-bin masses,
// age-dependent metallicity weights, plus the redshift ordering sort and the
// preparation kernels of the resident SSP block.
//
// One wave64 owns one galaxy in the weights kernel.  Lanes first locate the
// age-bin edges on the time grid (block-shared in LDS), then stream the SFR
// row in batches of coalesced loads while a float64 wave scan accumulates the
// trapezoid round by round, picking up the mass at each edge on the fly;
// finally lanes split the (metallicity, age) weights, which leave as
// coalesced rows in the GEMM's padded K layout.
#include "dsps_internal.hpp"

#include <cmath>

namespace dsps {

// SFR(t) = A (t/tau)^alpha exp(-t/tau) (1 - q Phi((t - t_q)/0.5 Gyr)), the
// parametric stand-in for the Diffstar history (Section 3.1, Eq. diffstar).
__device__ __forceinline__ double sfr_param(double t, double a, double tau, double alpha,
                                            double q, double tq) {
  const double x = t / tau;
  const double base = a * exp(alpha * log(x) - x);
  const double v = (t - tq) * (1.0 / QUENCH_WIDTH);
  const double phi = 0.5 * erfc(-v * 0.70710678118654752440);
  return base * (1.0 - q * phi);
}

__global__ void k_sfh_table(const double *__restrict__ t_table, int n_t,
                            const double *__restrict__ params, int n_gal,
                            double *__restrict__ sfr) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)n_gal * n_t;
  if (idx >= total) return;
  const int g = (int)(idx / n_t);
  const int n = (int)(idx - (long long)g * n_t);
  sfr[idx] = sfr_param(t_table[n], params[g], params[n_gal + g], params[2 * n_gal + g],
                       params[3 * n_gal + g], params[4 * n_gal + g]);
}

int launch_sfh_table(const double *t_table, int n_t, const double *params, int n_gal,
                     double *sfr, hipStream_t stream) {
  const long long total = (long long)n_gal * n_t;
  if (total == 0) return DSPS_OK;
  const int threads = 256;
  const long long blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(k_sfh_table, dim3((unsigned)blocks), dim3(threads), 0, stream, t_table,
                     n_t, params, n_gal, sfr);
  return hip_fail(hipGetLastError(), "k_sfh_table launch");
}

// Cosmic time t(z) in Gyr: closed form for LCDM, else Gauss-Legendre (4
// panels of 16 nodes) in s = sqrt(a), where t = t_H int_0^{a_z} da / (a E(a))
// becomes t_H int_0^{sqrt(a_z)} 2 s^2 / sqrt(Om + OL s^(-6 w)) ds.  One thread.
__device__ double age_at_z(double z, const CosmoArgs &c, const GaussLegendre &gl) {
  if (c.lcdm) {
    const double zp1 = 1.0 + z;
    const double a32 = 1.0 / (zp1 * sqrt(zp1));   // (1+z)^(-3/2)
    if (c.ol <= 0.0) return (2.0 / 3.0) * c.hubble_time_gyr * a32 / sqrt(c.om0);
    return (2.0 / (3.0 * sqrt(c.ol))) * c.hubble_time_gyr * asinh(sqrt(c.ol / c.om0) * a32);
  }
  const double h = sqrt(1.0 / (1.0 + z)) * 0.25;
  double sum = 0.0;
  for (int k = 0; k < 4 * GL_N; ++k) {
    const int panel = k / GL_N, node = k % GL_N;
    const double s = h * (panel + 0.5) + 0.5 * h * gl.x[node];
    sum += 0.5 * h * gl.w[node] * (2.0 * s * s / sqrt(c.om0 + c.ol * pow(s, -6.0 * c.w0)));
  }
  return c.hubble_time_gyr * sum;
}

// Distance modulus 5 log10(d_L / 10 pc), d_L = (1+z) (c/H0) int_0^z dz'/E(z'),
// Gauss-Legendre with 4 panels of 16 nodes.  One thread.
__device__ double distance_modulus(double z, const CosmoArgs &c, const GaussLegendre &gl) {
  const double h = z * 0.25;
  double sum = 0.0;
  for (int k = 0; k < 4 * GL_N; ++k) {
    const int panel = k / GL_N, node = k % GL_N;
    const double zp1 = 1.0 + (h * (panel + 0.5) + 0.5 * h * gl.x[node]);
    const double de = c.lcdm ? c.ol : c.ol * pow(zp1, 3.0 * (1.0 + c.w0));   // dark energy term
    sum += 0.5 * h * gl.w[node] / sqrt(c.om0 * zp1 * zp1 * zp1 + de);
  }
  return 5.0 * log10((1.0 + z) * c.hubble_dist_mpc * sum) + 25.0;
}

// First index i in [0, n) with x[i] >= v (STRICT: x[i] > v) over an ascending
// array; n if none.
template <bool STRICT>
__device__ int first_index(const double *x, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool ok = STRICT ? x[mid] > v : x[mid] >= v;
    if (ok) hi = mid; else lo = mid + 1;
  }
  return lo;
}
// The same from a first guess: the index a log-uniform grid would hold v at
// (lx0 = ln x[0], inv_lspan = 1 / (ln x[n-1] - ln x[0])) is checked against
// its neighbour, which on such a grid settles it in one round of loads;
// otherwise a bisection finishes on the side the guess leaves.  The index is
// the same either way (the predicate is monotone over the ascending array).
template <bool STRICT>
__device__ int first_index_guess(const double *x, int n, double v, double lx0, double inv_lspan) {
  if (n <= 2 || !(v > 0.0)) return first_index<STRICT>(x, n, v);
  const double f = (log(v) - lx0) * inv_lspan * (double)(n - 1);
  const int g = (int)fmin(fmax(f, 0.0), (double)(n - 2));
  const bool ok_g = STRICT ? x[g] > v : x[g] >= v;
  const bool ok_next = STRICT ? x[g + 1] > v : x[g + 1] >= v;
  if (!ok_g && ok_next) return g + 1;
  int lo = ok_g ? 0 : g + 2, hi = ok_g ? g : n;   // the first index lies in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool ok = STRICT ? x[mid] > v : x[mid] >= v;
    if (ok) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Per-galaxy scalars, one thread per galaxy of the sorted range: cosmic time
// at z for the weights kernel, the GEMM's constants (1 + z and the dust
// parameters), the magnitude offset, the rest-wavelength window and, with the
// ionization axis, the first and last grid points of non-zero weight.  The
// window's non-zero weight blocks start as "all" and are narrowed by the
// weights kernel when it runs.
__global__ __launch_bounds__(256) void k_galaxy_scalars(WeightsLaunch a) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= live_in_range(a.n_live, a.s_begin, a.s_count)) return;
  const int s = a.s_begin + local;
  const int g = a.perm ? a.perm[s] : s;
  const double z = (double)a.z[g];
  if (a.t_obs) a.t_obs[s] = age_at_z(z, a.cosmo, a.gl);
  if (a.meta) {
    GalaxyMeta m;
    m.zp1 = (float)(1.0 + z);
    // F = 10^(-0.4 A_V/4.05 k) = 2^(dust_a k)
    m.dust_a = (float)(-0.4 * 3.32192809488736234787 * (double)a.av[g] / DUST_RV);
    m.delta = a.delta[g];
    m.bump = a.bump[g];
    a.meta[s] = m;
  }
  if (a.ion) {
    GalaxyIon gi;
    gi.lgu = a.lgu[g];
    gi.sigma_u = a.sigma_u[g];
    int lo = -1, hi = 0;
    for (int u = 0; u < a.ssp.n_u; ++u) {
      if (ion_weight(a.ssp.ion_edges, u, gi.lgu, gi.sigma_u) != 0.0) {
        if (lo < 0) lo = u;
        hi = u;
      }
    }
    gi.u_lo = lo < 0 ? 0 : lo;
    gi.u_hi = lo < 0 ? 0 : hi;
    a.ion[s] = gi;
  }
  if (a.dust_old) {
    GalaxyDustOld d;
    d.dust_a = (float)(-0.4 * 3.32192809488736234787 * (double)a.av_old[g] / DUST_RV);
    d.delta = a.delta_old[g];
    a.dust_old[s] = d;
  }
  // absolute magnitudes at z = 0 (Eq. restmag); distance terms beyond
  if (a.mag_offset)
    a.mag_offset[s] = z > 0.0 ? distance_modulus(z, a.cosmo, a.gl) - 2.5 * log10(1.0 + z) : 0.0;
  if (a.range) {
    // rest wavelengths whose redshifted value can meet a filter: [lo, hi)
    // with wave[lo] >= obs_lo/(1+z) and wave[hi-1] <= obs_hi/(1+z), padded
    // by two grid points on each side (points outside contribute exact
    // zeros; the padding covers float32 rounding of (1+z) lambda)
    const int n_wave = a.ssp.n_wave;
    const double lx0 = log(a.ssp.wave[0]);
    const double inv_lspan = 1.0 / (log(a.ssp.wave[n_wave - 1]) - lx0);
    const int lo = first_index_guess<false>(a.ssp.wave, n_wave, a.obs_lo / (1.0 + z), lx0, inv_lspan);
    const int hi = first_index_guess<true>(a.ssp.wave, n_wave, a.obs_hi / (1.0 + z), lx0, inv_lspan);
    GalaxyRange r;
    r.win_lo = max(lo - 2, 0);
    r.win_hi = min(hi + 2, n_wave);
#pragma unroll
    for (int w = 0; w < KBLOCK_WORDS; ++w) r.kblk[w] = ~0u;
    r.age_hi = AGE_PAD;
    a.range[s] = r;
  }
}

// Consecutive time-grid segments each lane takes per scan round (a round
// covers 64 * SFR_PER_LANE segments).
constexpr int SFR_PER_LANE = 4;
constexpr int SFR_ROUND = 64 * SFR_PER_LANE;
// Per-wave LDS: cumulative mass at a round's SFR_ROUND + 1 nodes.  Node
// 4 l + k (lane l's k-th) sits at k * SFR_PRE_K + l, so that the lanes' writes
// of one k fall on consecutive words; the round's last node sits at 64.
constexpr int SFR_PRE_K = 65;
constexpr int SFR_PRE = SFR_PER_LANE * SFR_PRE_K;
__device__ __forceinline__ int pre_slot(int n) { return (n & 3) * SFR_PRE_K + (n >> 2); }
// Scan rounds over a time grid of n_t nodes (n_t - 1 segments).
__host__ __device__ inline int sfr_rounds(int n_t) { return (n_t - 1 + SFR_ROUND - 1) / SFR_ROUND; }

// A double moved across lanes by one DPP control (GFX9 encodings), both
// halves alike; lanes whose row is masked off or whose source lies outside
// the row or wave receive +0.  Every lane of the wave must be active.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_ROW_SHR = 0x110;     // + shift 1..15, within rows of 16 lanes
constexpr int DPP_ROW_BCAST15 = 0x142; // lane 15 of each row to the next row
constexpr int DPP_ROW_BCAST31 = 0x143; // lane 31 to rows 2 and 3
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane i takes lane i + 1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane i takes lane i - 1

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ double wave_inclusive_sum(double x) {
  x += dpp_f64<DPP_ROW_SHR + 1>(x);
  x += dpp_f64<DPP_ROW_SHR + 2>(x);
  x += dpp_f64<DPP_ROW_SHR + 4>(x);
  x += dpp_f64<DPP_ROW_SHR + 8>(x);
  x += dpp_f64<DPP_ROW_BCAST15, 0xa>(x);
  x += dpp_f64<DPP_ROW_BCAST31, 0xc>(x);
  return x;
}

__device__ __forceinline__ double lane63_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned x) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, true);
}

// One lane's part of the metallicity weights: ages i0 and i0 + 1 (i0 even),
// their age-bin masses and MDF centres.
struct MdfLane {
  const double *medge;   // [n_met + 1] metallicity bin edges (LDS)
  const float *ks;       // [k_pad] bf16 row scales (LDS)
  int n_met, n_age, i0;
  double mu0, mu1, inv_sig, mage0, mage1;   // mage0, mage1 are 0 past the last age
  bool real0, real1;
  double mu_lo, mu_hi;   // the galaxy's smallest and largest centre over ages
  // interior edges 1 .. n_zero have CDF exactly 0 for every age, edges from
  // first_one on exactly 1 (mdf_edge_regions)
  int n_zero, first_one;
};

// An edge at least 3 sigma (plus a margin far above rounding) above every
// age's centre has CDF exactly 1 for all of them, one as far below exactly
// 0.  The edges are ascending, so the all-zero edges are a prefix and the
// all-one edges a suffix of the interior ones: one test per edge for the
// whole wave (lane k takes edge k + 1) gives both as counts the wave shares.
__device__ __forceinline__ void mdf_edge_regions(MdfLane &L, int lane) {
  const double margin = 3.0 + 1e-9;
  const int ne = L.n_met - 1;
  const double e = lane < ne ? L.medge[lane + 1] : 0.0;
  const bool z = lane < ne && (e - L.mu_lo) * L.inv_sig <= -margin;
  const bool o = lane < ne && (e - L.mu_hi) * L.inv_sig >= margin;
  const unsigned long long zm = __ballot(z), om = __ballot(o);
  L.n_zero = __popcll(zm);
  L.first_one = om ? __builtin_ctzll(om) + 1 : L.n_met;
}

// CDF of the MDF at interior edge j (value e) for the lane's two ages, c0
// and c1; the polynomial only between the all-zero and all-one edges.
__device__ __forceinline__ void mdf_edge_cdf(const MdfLane &L, int j, double e, double &c0,
                                             double &c1) {
  if (j >= L.first_one) {
    c0 = c1 = 1.0;
  } else if (j <= L.n_zero) {
    c0 = c1 = 0.0;
  } else {
    c0 = triweight_cdf((e - L.mu0) * L.inv_sig);
    c1 = triweight_cdf((e - L.mu1) * L.inv_sig);
  }
}
// W[j][i] = m_i (CDF(e_{j+1}) - CDF(e_j)) for the lane's two ages over every
// metallicity row j, in float64 and rounded once, into the natural layout
// [n_met][n_age] (the weights the library hands out); returns the rows in
// which either weight is non-zero (as stored).
__device__ __forceinline__ unsigned mdf_rows_user(const MdfLane &L, float *out) {
  unsigned nzr = 0u;
  double c_prev0 = 0.0, c_prev1 = 0.0;  // CDF at the lower edge of metallicity bin 0 (-inf)
  for (int j = 0; j < L.n_met; ++j) {
    float w0f = 0.0f, w1f = 0.0f;
    // a row whose upper edge is all-zero, or whose lower edge is all-one, has
    // equal CDFs at both edges: its weights are exactly 0
    if (j + 1 <= L.n_zero || j >= L.first_one) {
      c_prev0 = c_prev1 = j + 1 <= L.n_zero ? 0.0 : 1.0;
    } else {
      double c_next0 = 1.0, c_next1 = 1.0;  // upper edge of the last bin is +inf
      if (j < L.n_met - 1) mdf_edge_cdf(L, j + 1, L.medge[j + 1], c_next0, c_next1);
      // mage is 0 past the last age, and the CDF difference is finite and >= 0
      w0f = (float)(L.mage0 * (c_next0 - c_prev0));
      w1f = (float)(L.mage1 * (c_next1 - c_prev1));
      c_prev0 = c_next0;
      c_prev1 = c_next1;
    }
    if (L.real0) out[j * L.n_age + L.i0] = w0f;
    if (L.real1) out[j * L.n_age + L.i0 + 1] = w1f;
    nzr |= (w0f != 0.0f || w1f != 0.0f ? 1u : 0u) << j;
  }
  return nzr;
}

// The triweight CDF in float32 (the same polynomial as triweight_cdf), exactly
// 0 and 1 from +-3 on.
__device__ __forceinline__ float triweight_cdf_f32(float z) {
  const float z2 = z * z;
  float p = fmaf(-5.0f / 69984.0f, z2, 7.0f / 2592.0f);
  p = fmaf(p, z2, -35.0f / 864.0f);
  p = fmaf(p, z2, 35.0f / 96.0f);
  const float c = fmaf(z, p, 0.5f);
  return z <= -3.0f ? 0.0f : (z >= 3.0f ? 1.0f : c);
}

// The same W rows in the GEMM's padded layouts (BF16 with the row scales,
// or float32), with the CDF differences in float32.  The float32 CDF differs
// from the float64 one by about 1e-7.  BF16 rows round to 8 significant bits
// next: far coarser for every weight above 1e-4 of its age's mass, and the
// smaller ones carry a correspondingly small share of the light.  For float32
// rows the difference moves a band sum by about 1e-7 of the light (1e-7 mag),
// three orders below the path's 1e-4 mag target.
template <bool BF16>
__device__ __forceinline__ unsigned mdf_rows_pad(const MdfLane &L, void *out) {
  const bool active = L.i0 < AGE_PAD;
  const float mu0 = (float)L.mu0, mu1 = (float)L.mu1, inv_sig = (float)L.inv_sig;
  const float mage0 = (float)L.mage0, mage1 = (float)L.mage1;
  unsigned nzr = 0u;
  float c_prev0 = 0.0f, c_prev1 = 0.0f;  // CDF at the lower edge of metallicity bin 0 (-inf)
  for (int j = 0; j < L.n_met; ++j) {
    float w0 = 0.0f, w1 = 0.0f;
    if (j + 1 <= L.n_zero || j >= L.first_one) {
      // upper edge all-zero or lower edge all-one: equal CDFs, weights 0
      c_prev0 = c_prev1 = j + 1 <= L.n_zero ? 0.0f : 1.0f;
    } else {
      float c_next0 = 1.0f, c_next1 = 1.0f;  // upper edge of the last bin is +inf
      if (j + 1 < L.first_one) {             // (then j + 1 < n_met as well)
        const float e = (float)L.medge[j + 1];
        c_next0 = triweight_cdf_f32((e - mu0) * inv_sig);
        c_next1 = triweight_cdf_f32((e - mu1) * inv_sig);
      }
      w0 = mage0 * (c_next0 - c_prev0);
      w1 = mage1 * (c_next1 - c_prev1);
      c_prev0 = c_next0;
      c_prev1 = c_next1;
    }
    bool nz;
    if (BF16) {
      const float2 ks = active ? *reinterpret_cast<const float2 *>(&L.ks[j * AGE_PAD + L.i0])
                               : make_float2(0.0f, 0.0f);
      // the row scales are powers of two; both values round to nearest even
      // in one packed conversion (finite inputs: the same bits as
      // f32_to_bf16_rne)
      typedef float f32x2_t __attribute__((ext_vector_type(2)));
      typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
      const f32x2_t v = {w0 * ks.x, w1 * ks.y};
      const uint32_t q = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
      if (active) *reinterpret_cast<uint32_t *>((uint16_t *)out + j * AGE_PAD + L.i0) = q;
      nz = (q & 0x7FFF7FFFu) != 0u;
    } else {
      if (active) *reinterpret_cast<float2 *>((float *)out + j * AGE_PAD + L.i0) = make_float2(w0, w1);
      nz = w0 != 0.0f || w1 != 0.0f;
    }
    nzr |= (nz ? 1u : 0u) << j;
  }
  return nzr;
}

// Age-major float32 rows (age-dependent attenuation): each of the lane's two
// ages becomes 16 metallicity slots (zeros past n_met) written as four
// 16-byte stores.  Returns the lane's highest age with a non-zero weight plus
// one (0 if none); pieces gets bit 4 q + p set when slots 4 p .. 4 p + 3 of
// age i0 + q hold a non-zero weight.  The CDF differences are taken in
// float32, as for the padded rows (mdf_rows_pad): these rows feed only the
// float32 contraction.
__device__ __forceinline__ int mdf_rows_age(const MdfLane &L, float *out, unsigned &pieces) {
  float w0[AGE_MET_SLOTS], w1[AGE_MET_SLOTS];
  const float mu0 = (float)L.mu0, mu1 = (float)L.mu1, inv_sig = (float)L.inv_sig;
  const float mage0 = (float)L.mage0, mage1 = (float)L.mage1;   // 0 past the last age
  float c_prev0 = 0.0f, c_prev1 = 0.0f;
#pragma unroll
  for (int j = 0; j < AGE_MET_SLOTS; ++j) {
    float v0 = 0.0f, v1 = 0.0f;
    if (j < L.n_met) {
      float c_next0 = 1.0f, c_next1 = 1.0f;   // all-one edges and the last bin's +inf
      if (j + 1 < L.first_one) {               // (then j + 1 < n_met as well)
        if (j + 1 <= L.n_zero) {
          c_next0 = c_next1 = 0.0f;
        } else {
          const float e = (float)L.medge[j + 1];
          c_next0 = triweight_cdf_f32((e - mu0) * inv_sig);
          c_next1 = triweight_cdf_f32((e - mu1) * inv_sig);
        }
      }
      v0 = L.real0 ? mage0 * (c_next0 - c_prev0) : 0.0f;
      v1 = L.real1 ? mage1 * (c_next1 - c_prev1) : 0.0f;
      c_prev0 = c_next0;
      c_prev1 = c_next1;
    }
    w0[j] = v0;
    w1[j] = v1;
  }
  unsigned pm = 0u;
#pragma unroll
  for (int j = 0; j < AGE_MET_SLOTS; ++j) {
    if (w0[j] != 0.0f) pm |= 1u << (j / 4);
    if (w1[j] != 0.0f) pm |= 1u << (AGED_PIECES_PER_AGE + j / 4);
  }
  pieces = L.i0 < AGE_PAD ? pm : 0u;
  const bool nz0 = (pm & 0xfu) != 0u, nz1 = (pm >> AGED_PIECES_PER_AGE) != 0u;
  if (L.i0 < AGE_PAD) {
    float4 *p0 = reinterpret_cast<float4 *>(out + (size_t)L.i0 * AGE_MET_SLOTS);
#pragma unroll
    for (int q = 0; q < AGE_MET_SLOTS / 4; ++q) {
      p0[q] = make_float4(w0[4 * q], w0[4 * q + 1], w0[4 * q + 2], w0[4 * q + 3]);
      p0[q + AGE_MET_SLOTS / 4] = make_float4(w1[4 * q], w1[4 * q + 1], w1[4 * q + 2], w1[4 * q + 3]);
    }
  }
  return nz1 ? L.i0 + 2 : (nz0 ? L.i0 + 1 : 0);
}

// Orders one wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-shared LDS of the weights kernel, in doubles.
__host__ __device__ inline size_t weights_lds_doubles(int n_t, int n_age, int n_met, int k_pad) {
  return (size_t)n_t + (size_t)sfr_rounds(n_t) * SFR_ROUND + 1 + (n_age + 1) + n_age +
         (n_met + 1) + (k_pad + 1) / 2 + (size_t)WEIGHTS_FWD_WAVES * SFR_PRE;
}

// TABULATED: the SFR arrives as a table row per galaxy; otherwise it is
// evaluated from the parametric history at the time-grid nodes.
template <bool TABULATED>
__global__ __launch_bounds__(64 * WEIGHTS_FWD_WAVES) void k_weights(WeightsLaunch a) {
  const SspView P = a.ssp;
  const int n_t = a.n_t, n_age = P.n_age, n_met = P.n_met;
  // block-shared: time grid, SSP grid constants, row scales
  extern __shared__ double lds[];
  const int n_seg = n_t - 1;
  const int n_round = sfr_rounds(n_t);
  double *tt = lds;                                   // [n_t]
  double *s_segw = tt + n_t;                          // [n_round * SFR_ROUND]
  double *s_per_node = s_segw + n_round * SFR_ROUND;  // [1]
  double *s_aedge = s_per_node + 1;                   // [n_age + 1]
  double *s_lgage = s_aedge + n_age + 1;              // [n_age]
  double *s_medge = s_lgage + n_age;                  // [n_met + 1]
  float *s_ks = (float *)(s_medge + n_met + 1);       // [k_pad]
  // one galaxy per wave.  With a tabulated SFR the wave's index is made
  // uniform, which keeps the galaxy's scalars and its row's base address in
  // scalar registers; the parametric history's five float64 parameters would
  // not fit there beside the rest and stay in vector registers.
  const int wave = TABULATED ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  // per wave: cumulative mass at the SFR_ROUND + 1 nodes of a round
  double *s_pre = (double *)(s_ks + ((P.k_pad + 1) & ~1)) + wave * SFR_PRE;
  for (int n = threadIdx.x; n < n_t; n += blockDim.x) tt[n] = a.t_table[n];
  // trapezoid weight of every segment, (t_{m+1} - t_m) / 2 in years, in the
  // order the scan reads it: round r, lane l, k-th segment of the lane at
  // r * SFR_ROUND + 64 k + l; 0 past the last segment, which masks those out
  for (int i = threadIdx.x; i < n_round * SFR_ROUND; i += blockDim.x) {
    const int w = i & (SFR_ROUND - 1);
    const int m = (i - w) + SFR_PER_LANE * (w & 63) + (w >> 6);
    s_segw[i] = m < n_seg ? (a.t_table[m + 1] - a.t_table[m]) * (0.5 * YEARS_PER_GYR) : 0.0;
  }
  // the node a uniform grid would put a time at, from the mean spacing
  if (threadIdx.x == 0) s_per_node[0] = (double)n_seg / (a.t_table[n_seg] - a.t_table[0]);
  for (int n = threadIdx.x; n <= n_age; n += blockDim.x) s_aedge[n] = P.age_edges[n];
  for (int n = threadIdx.x; n < n_age; n += blockDim.x) s_lgage[n] = P.lg_age[n];
  for (int n = threadIdx.x; n <= n_met; n += blockDim.x) s_medge[n] = P.met_edges[n];
  if (a.w_pad_bf16)
    for (int n = threadIdx.x; n < P.k_pad; n += blockDim.x) s_ks[n] = P.kscale[n];
  __syncthreads();

  const int local = blockIdx.x * WEIGHTS_FWD_WAVES + wave;
  // whole wave leaves; no block barrier follows
  if (local >= live_in_range(a.n_live, a.s_begin, a.s_count)) return;
  const int s = a.s_begin + local;
  const int g = a.perm ? a.perm[s] : s;

  // every per-galaxy load is issued before the first use of any of them
  const double t_obs = a.t_obs[s];
  const float lgmet_f = a.lgmet[g], sig_f = a.sigma_z[g];
  const bool transition = a.lgmet_old != nullptr;
  const double lgmet_old = transition ? (double)a.lgmet_old[g] : 0.0;
  const double *row = TABULATED ? a.sfr + (size_t)g * n_t : nullptr;
  // SFR at nodes nb + SFR_PER_LANE lane + k of the next round to be summed
  // and at the first node of the round after it (a tabulated row's first
  // round is loaded up front, each later one while its predecessor is
  // summed).  A whole round reads no node past its own last one; in the
  // round that reaches past the row's end, those nodes only enter segments
  // of weight 0 and read the last node in their place.
  double vn[SFR_PER_LANE], vn_end = 0.0;
  auto load_round = [&](int nb) {
    if (nb + SFR_ROUND <= n_t - 1) {
      const double *r = row + nb + SFR_PER_LANE * lane;
#pragma unroll
      for (int k = 0; k < SFR_PER_LANE; ++k) vn[k] = r[k];
      vn_end = row[nb + SFR_ROUND];
    } else {
#pragma unroll
      for (int k = 0; k < SFR_PER_LANE; ++k) vn[k] = row[min(nb + SFR_PER_LANE * lane + k, n_t - 1)];
      vn_end = row[min(nb + SFR_ROUND, n_t - 1)];
    }
  };
  if (TABULATED) load_round(0);


  // ---- age-bin edges: lane owns edges e = 2 lane and 2 lane + 1.  The mass
  // formed by cosmic time t is 0 at or before t_table[0], the total after the
  // last node, and otherwise the cumulative trapezoid interpolated linearly
  // between nodes lo and lo + 1, where t_table[lo] <= t < t_table[lo + 1].
  int kind[2], lo[2];            // kind: 0 none formed, 1 inside the grid, 2 all formed
  double fe[2];
  {
    double te[2];
    int hi[2];
    const double t_first = tt[0], t_last = tt[n_t - 1];
    const double per_node = s_per_node[0];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = 2 * lane + q;
      te[q] = e <= n_age ? t_obs - s_aedge[e] : -1.0 / 0.0;
      kind[q] = !(te[q] > t_first) ? 0 : (te[q] >= t_last ? 2 : 1);
      lo[q] = 0;
      hi[q] = kind[q] == 1 ? n_t - 1 : 1;   // only an edge inside the grid searches
      if (kind[q] == 1) {
        // check the guess against the two nodes around it: on a (near)
        // uniform grid it brackets t, otherwise it narrows the bisection
        const int g = min(max((int)((te[q] - t_first) * per_node), 0), n_t - 2);
        if (tt[g] <= te[q]) {
          lo[q] = g;
          if (te[q] < tt[g + 1]) hi[q] = g + 1;
          else lo[q] = g + 1;
        } else {
          hi[q] = g;
        }
      }
    }
    // bisection of both edges together (tt[lo] <= t < tt[hi] for kind 1)
    while (hi[0] - lo[0] > 1 || hi[1] - lo[1] > 1) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (hi[q] - lo[q] > 1) {
          const int mid = (lo[q] + hi[q]) >> 1;
          if (tt[mid] <= te[q]) lo[q] = mid; else hi[q] = mid;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
      fe[q] = kind[q] == 1 ? (te[q] - tt[lo[q]]) / (tt[lo[q] + 1] - tt[lo[q]]) : 0.0;
  }

  // ---- cumulative trapezoid of the SFR row, one round of SFR_ROUND segments
  // at a time: segment m joins nodes m and m + 1; lane l holds segments
  // base + 4 l .. base + 4 l + 3, sums them locally and joins the wave's
  // exclusive scan of the lane totals.  The cumulative mass at the round's
  // nodes goes to the wave's LDS buffer, where every age-bin edge whose
  // interval lies in the round interpolates it linearly.
  double pa = 0, ptau = 1, palpha = 0, pq = 0, ptq = 0;
  if (!TABULATED) {
    pa = a.sfh_params[g]; ptau = a.sfh_params[a.n_gal + g];
    palpha = a.sfh_params[2 * a.n_gal + g]; pq = a.sfh_params[3 * a.n_gal + g];
    ptq = a.sfh_params[4 * a.n_gal + g];
  }
  static_assert(SFR_PER_LANE == 4, "pre_slot assumes four segments per lane");
  // an edge inside the grid interpolates in the round holding its interval
  // [lo, lo + 1], between the same two buffer slots whichever round it is
  int e_round[2], e_slot0[2], e_slot1[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int src = lo[q] & (SFR_ROUND - 1);
    e_round[q] = kind[q] == 1 ? lo[q] / SFR_ROUND : -1;
    e_slot0[q] = pre_slot(src);
    e_slot1[q] = pre_slot(src + 1);
  }
  double carry = 0.0;
  double em[2] = {0.0, 0.0};
  for (int base = 0, round = 0; base < n_seg; base += SFR_ROUND, ++round) {
    double v[SFR_PER_LANE], v_end;
    if (TABULATED) {
#pragma unroll
      for (int k = 0; k < SFR_PER_LANE; ++k) v[k] = vn[k];
      v_end = vn_end;
      if (base + SFR_ROUND < n_seg) load_round(base + SFR_ROUND);
    } else {
      // the round's nodes inside the grid, evaluated node-major (lane l takes
      // nodes base + l + 64 q, so a short grid costs few evaluations) into
      // the wave's buffer, then read back in the scan's order
      const int n_here = min(SFR_ROUND + 1, n_t - base);
      for (int q = 0; q * 64 < n_here; ++q) {
        const int j = q * 64 + lane;
        if (j < n_here) s_pre[pre_slot(j)] = sfr_param(tt[base + j], pa, ptau, palpha, pq, ptq);
      }
      wave_sync();
#pragma unroll
      for (int k = 0; k < SFR_PER_LANE; ++k)
        v[k] = SFR_PER_LANE * lane + k < n_here ? s_pre[k * SFR_PRE_K + lane] : 0.0;
      v_end = SFR_ROUND < n_here ? s_pre[pre_slot(SFR_ROUND)] : 0.0;
    }
    double after = dpp_f64<DPP_WAVE_SHL1>(v[0]);      // SFR at the next lane's first node
    if (lane == 63) after = v_end;
    const double *w = s_segw + base + lane;           // the lane's segment weights
    double part[SFR_PER_LANE];                        // local inclusive sums
#pragma unroll
    for (int k = 0; k < SFR_PER_LANE; ++k) {
      const double right = k + 1 < SFR_PER_LANE ? v[k + 1 < SFR_PER_LANE ? k + 1 : k] : after;
      const double seg = (v[k] + right) * w[64 * k];
      part[k] = k == 0 ? seg : part[k > 0 ? k - 1 : 0] + seg;
    }
    const double incl = wave_inclusive_sum(part[SFR_PER_LANE - 1]);
    const double before = carry + dpp_f64<DPP_WAVE_SHR1>(incl);   // lane 0 takes +0
    s_pre[lane] = before;                             // node n0 (pre_slot(4 lane))
#pragma unroll
    for (int k = 1; k < SFR_PER_LANE; ++k) s_pre[k * SFR_PRE_K + lane] = before + part[k - 1];
    if (lane == 63) s_pre[pre_slot(SFR_ROUND)] = before + part[SFR_PER_LANE - 1];
    wave_sync();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (e_round[q] == round) {
        const double m0 = s_pre[e_slot0[q]];
        em[q] = m0 + fe[q] * (s_pre[e_slot1[q]] - m0);
      }
    }
    carry += lane63_f64(incl);
    wave_sync();                                      // buffer reused by the next round
  }
#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (kind[q] == 2) em[q] = carry;

  // ---- bin masses m_i = M(t_obs - edge_i) - M(t_obs - edge_{i+1}) in float64;
  // lane l holds ages 2l and 2l + 1
  const double em_next = dpp_f64<DPP_WAVE_SHL1>(em[0]);   // edge 2l + 2
  const int i0 = 2 * lane;
  const bool real0 = i0 < n_age, real1 = i0 + 1 < n_age;
  const double mage0 = real0 ? em[0] - em[1] : 0.0;
  const double mage1 = real1 ? em[1] - em_next : 0.0;
  if (a.mstar && lane == 0) a.mstar[g] = em[0];

  // ---- metallicity weights and W = m_age * P: lane l writes ages 2l, 2l + 1
  // of every metallicity row as one 4-byte (bf16) or 8-byte (float32) store
  const double lgmet = (double)lgmet_f;
  const double inv_sig = 1.0 / (double)sig_f;
  const double mu0 = real0 ? mdf_centre(s_lgage[i0], lgmet, transition, lgmet_old, a.slope,
                                        a.pivot, a.mdf_width) : 0.0;
  const double mu1 = real1 ? mdf_centre(s_lgage[i0 + 1], lgmet, transition, lgmet_old, a.slope,
                                        a.pivot, a.mdf_width) : 0.0;
  // the centre is monotone in age: its extremes sit at the first and last age
  const double mu_a = mdf_centre(s_lgage[0], lgmet, transition, lgmet_old, a.slope, a.pivot,
                                 a.mdf_width);
  const double mu_b = mdf_centre(s_lgage[n_age - 1], lgmet, transition, lgmet_old, a.slope,
                                 a.pivot, a.mdf_width);
  MdfLane L{s_medge, s_ks, n_met, n_age, i0, mu0, mu1, inv_sig, mage0, mage1, real0, real1,
            fmin(mu_a, mu_b), fmax(mu_a, mu_b), 0, 0};
  mdf_edge_regions(L, lane);
  if (a.w_pad && a.w_pad_age) {
    // age-major rows: the contraction needs the highest non-zero age and the
    // pieces holding a weight
    unsigned pieces;
    const int hi = mdf_rows_age(L, (float *)a.w_pad + (size_t)local * AGE_K, pieces);
    const unsigned long long any = __ballot(hi > 0);
    const int top = any ? 63 - __builtin_clzll(any) : 0;
    const int age_hi = any ? __builtin_amdgcn_readlane(hi, top) : 0;
    if (a.range) {
      if (lane == 0) a.range[s].age_hi = age_hi;
      // lane l holds bits 8 l .. 8 l + 7 of the piece mask (ages 2 l, 2 l + 1):
      // word w gathers lanes 4 w .. 4 w + 3
      unsigned long long bit[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) bit[k] = __ballot((pieces >> k) & 1u);
      if (lane < KBLOCK_WORDS) {
        unsigned word = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int k = 0; k < 8; ++k)
            word |= (unsigned)((bit[k] >> (4 * lane + q)) & 1ull) << (8 * q + k);
        a.range[s].kblk[lane] = word;
      }
    }
    return;
  }
  unsigned nzr;   // metallicity rows in which either of the lane's ages has a non-zero weight
  if (a.w_pad && a.w_pad_bf16)
    nzr = mdf_rows_pad<true>(L, (uint16_t *)a.w_pad + (size_t)local * P.k_pad);
  else if (a.w_pad)
    nzr = mdf_rows_pad<false>(L, (float *)a.w_pad + (size_t)local * P.k_pad);
  else
    nzr = mdf_rows_user(L, a.w_user + (size_t)g * n_met * n_age);
  // non-zero (4-age block, row) mask: block b holds the ages of lanes 2b and
  // 2b + 1, so after one shifted OR lane 2b + 1 holds its rows; word w packs
  // blocks 2w (low half) and 2w + 1 (high half), which lane 4w + 3 joins
  // from lane 4w + 1 and itself and stores
  nzr |= dpp_u32<DPP_ROW_SHR + 1>(nzr);
  const unsigned low = dpp_u32<DPP_ROW_SHR + 2>(nzr);
  if (a.range && (lane & 3) == 3 && (lane >> 2) < KBLOCK_WORDS)
    a.range[s].kblk[lane >> 2] = (low & 0xffffu) | (nzr << 16);
}

int launch_weights(const WeightsLaunch &a, hipStream_t stream) {
  if (a.s_count <= 0) return DSPS_OK;
  ProfScope prof(DSPS_KERNEL_WEIGHTS, stream);
  if (a.t_obs || a.meta || a.range || a.mag_offset) {
    hipLaunchKernelGGL(k_galaxy_scalars, dim3((a.s_count + 255) / 256), dim3(256), 0, stream, a);
    const int rc = hip_fail(hipGetLastError(), "k_galaxy_scalars launch");
    if (rc) return rc;
  }
  // the weights kernel runs when weight rows are asked for, padded or in the
  // natural layout (the windows' block masks then narrow from "all" to the
  // exact union)
  if (!a.w_pad && !a.w_user) {
    if (!a.mstar) return DSPS_OK;
    set_error("internal: the mass formed needs the weight rows");
    return DSPS_ERR_ARG;
  }
  if (!a.t_obs || (a.w_pad && a.w_user)) {
    set_error("internal: weight rows need the cosmic-time workspace and one output layout");
    return DSPS_ERR_ARG;
  }
  const int blocks = (a.s_count + WEIGHTS_FWD_WAVES - 1) / WEIGHTS_FWD_WAVES;
  const size_t lds = sizeof(double) * weights_lds_doubles(a.n_t, a.ssp.n_age, a.ssp.n_met,
                                                          a.ssp.k_pad);
  const void *fn = a.sfr ? (const void *)k_weights<true> : (const void *)k_weights<false>;
  if (lds > 65536) {
    const int rc = hip_fail(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                            "k_weights LDS attribute");
    if (rc) return rc;
  }
  if (a.sfr)
    hipLaunchKernelGGL(k_weights<true>, dim3(blocks), dim3(64 * WEIGHTS_FWD_WAVES), lds, stream, a);
  else
    hipLaunchKernelGGL(k_weights<false>, dim3(blocks), dim3(64 * WEIGHTS_FWD_WAVES), lds, stream, a);
  return hip_fail(hipGetLastError(), "k_weights launch");
}

// ------------------------------------------------------------ ordering sort
// Key = (lowest and highest metallicity row the galaxy's MDF can reach,
// redshift bucket of 1/16 in log2(1+z)).  Galaxies of one 128-galaxy tile then
// share their non-zero metallicity rows and, within a row range, a narrow
// redshift span, hence a rest-wavelength window and the age blocks below the
// lookback time; the rows come first because a mismatch there costs whole
// K rows for every wavelength of the tile.  The order never changes a
// galaxy's result (the kernels' tiling is exact), only the work.
//
// With an ionization axis a tile's K stages run once per ionization point in
// the union of its members' supports, so the key leads with that support
// (first point, 3 bits, and extent, 2 bits), then the lowest metallicity row
// and a redshift bucket of 1/8 in log2(1+z): 13 bits as before.
__device__ __forceinline__ int sort_key(const SortLaunch &a, int g) {
  const float z = a.z[g];
  int zb = 0;
  if (z > 0.0f) {
    const float v = log2f(1.0f + z) * 16.0f;
    zb = v >= 31.0f ? 31 : (int)v;
  }
  const double lgmet = (double)a.lgmet[g], three_sig = 3.0 * (double)a.sigma_z[g];
  // the centre is monotone in age under both models: its extremes sit at the
  // youngest and oldest ages
  const bool transition = a.lgmet_old != nullptr;
  const double old = transition ? (double)a.lgmet_old[g] : 0.0;
  const double m0 = mdf_centre(a.lg_age_first, lgmet, transition, old, a.slope, a.pivot, a.mdf_width);
  const double m1 = mdf_centre(a.lg_age_last, lgmet, transition, old, a.slope, a.pivot, a.mdf_width);
  const double lo = fmin(m0, m1) - three_sig, hi = fmax(m0, m1) + three_sig;
  int jlo = 0, jhi = 0;
  for (int j = 1; j < a.n_met; ++j) {       // bin j starts at interior edge j
    jlo += a.met_edges[j] <= lo;
    jhi += a.met_edges[j] <= hi;
  }
  if (a.lgu) {
    // the same support the per-galaxy scalar pass finds
    const double c = (double)a.lgu[g], sg = (double)a.sigma_u[g];
    int ulo = -1, uhi = 0;
    for (int u = 0; u < a.n_u; ++u) {
      if (ion_weight(a.ion_edges, u, c, sg) != 0.0) {
        if (ulo < 0) ulo = u;
        uhi = u;
      }
    }
    if (ulo < 0) ulo = uhi = 0;
    return (min(ulo, 7) << 10) | (min(uhi - ulo, 3) << 8) | (min(jlo, 15) << 4) | (zb >> 1);
  }
  return (min(jlo, 15) << 9) | (min(jhi, 15) << 5) | zb;
}

__global__ void k_fill_int(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Galaxies per sort workgroup (1024 threads, 4 each).  Counts are aggregated
// in LDS first, so a key shared by many galaxies (a narrow redshift range, or
// the inert padding of a server batch) costs one global atomic per workgroup
// instead of one per galaxy.
constexpr int SORT_CHUNK = 4096;
constexpr int SORT_PER_THREAD = SORT_CHUNK / 1024;

__global__ __launch_bounds__(1024) void k_sort_hist(SortLaunch a) {
  __shared__ int cnt[SORT_BINS];
  for (int i = threadIdx.x; i < SORT_BINS; i += 1024) cnt[i] = 0;
  __syncthreads();
  const int g0 = blockIdx.x * SORT_CHUNK + threadIdx.x;
  const int live = live_in_range(a.n_live, 0, a.n_gal);
#pragma unroll
  for (int k = 0; k < SORT_PER_THREAD; ++k) {
    const int g = g0 + k * 1024;
    if (g < live) atomicAdd(&cnt[sort_key(a, g)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SORT_BINS; i += 1024)
    if (cnt[i]) atomicAdd(&a.hist[i], cnt[i]);
}

// Exclusive scan of SORT_BINS counters by one 1024-thread block, in place.
__global__ __launch_bounds__(1024) void k_sort_scan(int *hist) {
  constexpr int PER = SORT_BINS / 1024;
  __shared__ int part[1024];
  const int t = threadIdx.x;
  int v[PER], sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) { v[i] = hist[PER * t + i]; sum += v[i]; }
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int u = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  int run = part[t] - sum;
#pragma unroll
  for (int i = 0; i < PER; ++i) { hist[PER * t + i] = run; run += v[i]; }
}

// Each workgroup ranks its galaxies per key in LDS, reserves one range per
// key it holds from the scanned offsets, then writes the permutation.  The
// order inside a key is arbitrary (it never changes a galaxy's result).
__global__ __launch_bounds__(1024) void k_sort_scatter(SortLaunch a) {
  __shared__ int cnt[SORT_BINS];
  __shared__ int base[SORT_BINS];
  for (int i = threadIdx.x; i < SORT_BINS; i += 1024) cnt[i] = 0;
  __syncthreads();
  const int g0 = blockIdx.x * SORT_CHUNK + threadIdx.x;
  const int live = live_in_range(a.n_live, 0, a.n_gal);
  int key[SORT_PER_THREAD], rank[SORT_PER_THREAD];
#pragma unroll
  for (int k = 0; k < SORT_PER_THREAD; ++k) {
    const int g = g0 + k * 1024;
    key[k] = 0;
    rank[k] = 0;
    if (g < live) {
      key[k] = sort_key(a, g);
      rank[k] = atomicAdd(&cnt[key[k]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SORT_BINS; i += 1024)
    if (cnt[i]) base[i] = atomicAdd(&a.hist[i], cnt[i]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SORT_PER_THREAD; ++k) {
    const int g = g0 + k * 1024;
    if (g < live)
      a.perm[base[key[k]] + rank[k]] = g;
    else if (g < a.n_gal)
      a.perm[g] = g;       // padding keeps its place after the live galaxies
  }
}

int launch_sort(const SortLaunch &a, hipStream_t stream) {
  static_assert(SORT_BINS % 1024 == 0 && SORT_BINS >= (16 << 9), "key range");
  if (a.n_gal <= 0) return DSPS_OK;
  ProfScope prof(DSPS_KERNEL_ZSORT, stream);
  hipLaunchKernelGGL(k_fill_int, dim3(SORT_BINS / 256), dim3(256), 0, stream, a.hist, SORT_BINS, 0);
  const int blocks = (a.n_gal + SORT_CHUNK - 1) / SORT_CHUNK;
  hipLaunchKernelGGL(k_sort_hist, dim3(blocks), dim3(1024), 0, stream, a);
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, stream, a.hist);
  hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(1024), 0, stream, a);
  return hip_fail(hipGetLastError(), "ordering sort launch");
}

// ------------------------------------------------------------ BF16 quantiser
__global__ __launch_bounds__(256) void k_quantize_bf16(const float *__restrict__ x, int cols,
                                                       uint16_t *__restrict__ q,
                                                       float *__restrict__ scale) {
  __shared__ float red[4];
  const size_t row = blockIdx.x;
  const float *xr = x + row * cols;
  float m = 0.0f;
  for (int c = threadIdx.x; c < cols; c += blockDim.x) m = fmaxf(m, xr[c]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float s = pow2_ceil(m);
  if (threadIdx.x == 0) scale[row] = s;
  uint16_t *qr = q + row * cols;
  // x / s is exact for a power-of-two s except where it lands in the
  // subnormal range, where the correctly rounded division decides.
  for (int c = threadIdx.x; c < cols; c += blockDim.x) qr[c] = f32_to_bf16_rne(xr[c] / s);
}

int launch_quantize_bf16(const float *x, int rows, int cols, uint16_t *q, float *scale,
                         hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return DSPS_OK;
  hipLaunchKernelGGL(k_quantize_bf16, dim3(rows), dim3(256), 0, stream, x, cols, q, scale);
  return hip_fail(hipGetLastError(), "k_quantize_bf16 launch");
}

// ------------------------------------------------------------ table packing
// lum rows (met * n_age + age) x n_wave  ->  ST[l][met * 96 + age], zero padded.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_table(const T *__restrict__ src, int n_age,
                                                    int n_wave, int n_wave_pad, int k_pad,
                                                    int dst_stride, T *__restrict__ dst) {
  __shared__ T tile[32][33];
  const int k0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, l = l0 + tx;
    const int met = k / AGE_PAD, age = k - met * AGE_PAD;
    T v = T(0);
    if (age < n_age && l < n_wave) v = src[((size_t)met * n_age + age) * n_wave + l];
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int l = l0 + r, k = k0 + tx;
    if (l < n_wave_pad && k < k_pad) dst[(size_t)l * dst_stride + k] = tile[tx][r];
  }
}

// lum rows -> metallicity-differenced K-major table for the adjoint:
// SK[met * 96 + age][l] = L[met, age, l] - L[met - 1, age, l] (L[-1] = 0),
// formed in float64 and rounded once.  The transposed contraction against it
// returns Wbar[0] and the differences Wbar[j] - Wbar[j-1] directly, which are
// what the metallicity-weight gradients need (adjacent metallicity rows are
// nearly equal, so differencing Wbar afterwards would cancel in float32).
// Rows are padded to sk_rows and wavelengths to n_wave_pad with zeros.  With
// differenced == 0 the rows are the plain L[met, age, l] (the adjoint starts
// each galaxy's sum at the lowest row of its metallicity support from there).
__global__ void k_pack_table_kmajor(const float *__restrict__ src, int n_age, int n_wave,
                                    int n_wave_pad, int k_pad, int sk_rows, int differenced,
                                    float *__restrict__ dst) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)sk_rows * n_wave_pad) return;
  const int k = (int)(idx / n_wave_pad), l = (int)(idx % n_wave_pad);
  const int met = k / AGE_PAD, age = k - met * AGE_PAD;
  double v = 0.0;
  if (k < k_pad && age < n_age && l < n_wave) {
    v = (double)src[((size_t)met * n_age + age) * n_wave + l];
    if (differenced && met > 0) v -= (double)src[((size_t)(met - 1) * n_age + age) * n_wave + l];
  }
  dst[idx] = (float)v;
}

// lum rows -> age-major table for the age-dependent attenuation:
// SA[l][age * 16 + met] = L[met, age, l], zero for met >= n_met, age >= n_age
// or l >= n_wave.  One thread per element of the table.
__global__ void k_pack_table_age(const float *__restrict__ src, int n_met, int n_age, int n_wave,
                                 int n_wave_pad, float *__restrict__ dst) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n_wave_pad * AGE_K) return;
  const int l = (int)(idx / AGE_K), k = (int)(idx % AGE_K);
  const int age = k / AGE_MET_SLOTS, met = k % AGE_MET_SLOTS;
  float v = 0.0f;
  if (met < n_met && age < n_age && l < n_wave) v = src[((size_t)met * n_age + age) * n_wave + l];
  dst[idx] = v;
}

int launch_pack_table_age(const float *lum_rows, int n_met, int n_age, int n_wave, int n_wave_pad,
                          float *sa32, hipStream_t stream) {
  const size_t total = (size_t)n_wave_pad * AGE_K;
  hipLaunchKernelGGL(k_pack_table_age, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                     lum_rows, n_met, n_age, n_wave, n_wave_pad, sa32);
  return hip_fail(hipGetLastError(), "k_pack_table_age launch");
}

int launch_pack_table_kmajor(const float *lum_rows, int n_age, int n_wave, int n_wave_pad,
                             int k_pad, int sk_rows, int differenced, float *sk32,
                             hipStream_t stream) {
  const size_t total = (size_t)sk_rows * n_wave_pad;
  hipLaunchKernelGGL(k_pack_table_kmajor, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     stream, lum_rows, n_age, n_wave, n_wave_pad, k_pad, sk_rows, differenced, sk32);
  return hip_fail(hipGetLastError(), "k_pack_table_kmajor launch");
}

int launch_pack_table(const float *lum_rows, const uint16_t *q_rows, int n_met, int n_age,
                      int n_wave, int n_wave_pad, int k_pad, int dst_stride, float *st32,
                      uint16_t *st16, hipStream_t stream) {
  (void)n_met;
  const dim3 grid(k_pad / 32, n_wave_pad / 32);
  if (st32) hipLaunchKernelGGL(k_pack_table<float>, grid, dim3(256), 0, stream, lum_rows, n_age,
                               n_wave, n_wave_pad, k_pad, dst_stride, st32);
  if (st16) hipLaunchKernelGGL(k_pack_table<uint16_t>, grid, dim3(256), 0, stream, q_rows, n_age,
                               n_wave, n_wave_pad, k_pad, dst_stride, st16);
  return hip_fail(hipGetLastError(), "k_pack_table launch");
}

}  // namespace dsps
