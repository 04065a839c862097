// Internal definitions shared by the libdsps translation units.
//
// Layout decisions for gfx950 (see the design notes in the repository):
//  * The SSP block is stored wavelength-major, ST[l][k] with k = met * 96 + age
//    (ages zero-padded to 96 so that every 16- or 64-wide K block stays inside
//    one metallicity row).  With the nebular ionization axis each table row
//    holds one such block per ionization point, ST[l][u * k_pad + k].  Both GEMM operands are then K-contiguous rows, which
//    load as 16-byte vectors and feed MFMA fragments straight from LDS.
//  * Galaxies are processed in redshift order so that a 128-galaxy tile shares
//    one rest-frame wavelength window; per-galaxy scalars live in SoA arrays
//    indexed by sorted position.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/dsps.h"

namespace dsps {

// ----------------------------------------------------------------- limits
constexpr int AGE_PAD = 96;        // ages per metallicity row in the padded K axis
constexpr int TILE_G = 128;        // galaxies per GEMM tile (N of the MFMA tile)
constexpr int TILE_L = 128;        // wavelengths per chunk (M of the MFMA tile)
// Wavelength chunks one workgroup of the fused contraction walks, which
// amortises the per-workgroup set-up against load balance: two for float32
// (measured: 1.5% faster than one, three no better, four slower), four for
// bfloat16, whose chunks are cheaper.  The adjoint's Lbar kernel groups
// LBAR_CHUNKS chunks per workgroup.
__host__ __device__ constexpr int chunks_per_group(int precision) {
  return precision == DSPS_BF16 ? 4 : 2;
}
// Chunks whose band sums one partial slot holds: the workgroup's whole group
// in float32 (each later chunk adds its sums to the slot, and groups start at
// multiples of their size, so a slot does not depend on the tile); one in
// bfloat16, whose VALU-bound epilogue measured 13% slower waiting on the
// slot's read.
__host__ __device__ constexpr int partial_chunks(int precision) {
  return precision == DSPS_BF16 ? 1 : chunks_per_group(precision);
}
constexpr int LBAR_CHUNKS = 4;
constexpr int SORT_BINS = 8192;    // keys of the ordering sort (4+4-bit rows, 5-bit z bucket)
constexpr int GEMM_THREADS = 256;  // 4 wave64s in a 2 x 2 arrangement
constexpr int WEIGHT_WAVES = 4;    // galaxies per adjoint weights workgroup (one per wave)
// galaxies per forward weights workgroup: its grid tables are filled once per
// workgroup, so more waves share the fill
constexpr int WEIGHTS_FWD_WAVES = 8;

// ------------------------------------------------------------- constants
// AB zero point of a source at 10 pc, L_sun/Hz (Section 2.2.1).
constexpr double AB_ZERO_POINT = 1.13492e-13;
// Attenuation: A_lambda = A_V / 4.05 * k_lambda, k0 normalised at 5500 A;
// Drude bump centre 2175 A and width 350 A (Section 3.4).
constexpr double DUST_RV = 4.05;
constexpr double DUST_LAMBDA_V = 5500.0;
constexpr double DUST_SWITCH_ANGSTROM = 1500.0;
constexpr double BUMP_CENTRE = 2175.0;
constexpr double BUMP_WIDTH = 350.0;
// Mpc / (km/s) expressed in Gyr, and c in km/s.
constexpr double GYR_PER_MPC_S_KM = 977.7922216807891;
constexpr double LIGHT_KM_S = 299792.458;
constexpr double YEARS_PER_GYR = 1.0e9;
constexpr double QUENCH_WIDTH = 0.5;   // Gyr, parametric SFH transition width

// ------------------------------------------------------------- handles
// Device-side view of the resident SSP block, passed to kernels by value.
struct SspView {
  int n_met, n_age, n_wave;
  int n_wave_pad;                  // multiple of TILE_L
  int k_pad;                       // n_met * AGE_PAD
  int n_u;                         // ionization points (1 without the axis)
  int k_row;                       // columns of st32: n_u * k_pad
  const double *ion_edges;         // [n_u + 1] log10 U_s: -inf, midpoints, +inf
  const double *wave;              // [n_wave] rest Angstrom (float64)
  const double *age_edges;         // [n_age + 1] Gyr: 0, midpoints, +inf
  const double *met_edges;         // [n_met + 1] log10 Z: -inf, midpoints, +inf
  const double *lg_age;            // [n_age]
  const float *st32;               // [n_wave_pad][k_row] or null
  const uint16_t *st16;            // [n_wave_pad][k_pad] bf16 of lum / scale, or null
  const float *kscale;             // [k_pad] power-of-two row scales (1 on padding)
  const float4 *lconst;            // [n_wave_pad] (lambda, log2(lambda/5500), k0, drude shape)
  const float *qweight;            // [n_wave_pad] trapezoid weight in dlambda/lambda
  // [n_u][sk_rows][n_wave_pad] K-major, metallicity-differenced (adjoint),
  // one block per ionization point; without the ionization axis followed by
  // the plain K-major rows [sk_rows][n_wave_pad] (row sk_rows + k is L[k])
  const float *sk32;
  int sk_rows;                     // k_pad rounded up to a multiple of TILE_L
  // [n_wave_pad][AGE_K] age-major float32 (age-dependent attenuation) or null:
  // column age * 16 + met, zero for met >= n_met or age >= n_age
  const float *sa32;
};
// Columns of the age-major table and weight rows: 16 metallicity slots per age.
constexpr int AGE_MET_SLOTS = 16;
constexpr int AGE_K = AGE_PAD * AGE_MET_SLOTS;   // 1536

struct SspHandle {
  int device = -1;
  int precisions = 0;
  int k0_reading = 0;
  double lg_age_first = 0, lg_age_last = 0;
  std::vector<double> lg_age_host;  // SSP log10 ages (host copy, for launch set-up)
  SspView v{};
  std::vector<double> wave_host;   // rest wavelengths (host copy, for launch sizing)
  void *alloc = nullptr;           // single device allocation backing every array
};

struct FilterView {
  int n_band, n_pts;
  const float *trans;              // [n_band][n_pts]
  const float2 *grid;              // [n_band] (first wavelength, 1 / spacing)
};

struct FiltersHandle {
  int device = -1;
  FilterView v{};
  double obs_lo = 0, obs_hi = 0;   // union of the filter supports
  void *alloc = nullptr;
};

// Per-galaxy scalars written by the weights kernel, indexed by sorted position.
struct GalaxyMeta {
  float zp1;       // 1 + z
  float dust_a;    // -0.4 log2(10) A_V / 4.05: F = exp2(dust_a * k_lambda)
  float delta;
  float bump;
};
// Blocks of KBLOCK_AGES consecutive (padded) ages in one metallicity row:
// the unit in which the contraction skips all-zero weights (one 16-byte unit
// of a float32 weight row; two blocks make a bfloat16 unit).
constexpr int KBLOCK_AGES = 4;
constexpr int KBLOCKS_PER_ROW = AGE_PAD / KBLOCK_AGES;                  // 24
constexpr int KBLOCK_WORDS = (DSPS_MAX_MET * KBLOCKS_PER_ROW + 31) / 32;  // 12
static_assert(DSPS_MAX_MET <= 16 && KBLOCKS_PER_ROW == 2 * KBLOCK_WORDS, "block-major mask layout");
// K units of a tile's stage list: 8 ages of a row for float32 (two 4-age
// blocks), 16 for bfloat16.
constexpr int MAX_UNITS = DSPS_MAX_MET * KBLOCKS_PER_ROW / 2;           // 192
static_assert(MAX_UNITS % 2 == 0, "unit list size");
// The age-major layout's units are the two halves of an age's 16
// metallicity slots (unit u of age i: slots 8u .. 8u + 7, which is what one
// MFMA step pair reduces, so a galaxy's sums do not depend on its tile), the
// tile's non-zero ones grouped by attenuation group (all young ages, each
// transition age, all old ages) and each group padded to whole stages, so
// that no stage mixes two groups.  A galaxy's mask has bit 4 i + p of the
// same twelve words (KBLOCK_WORDS) set when slots 4p .. 4p + 3 of age i hold
// a weight.
constexpr int AGED_PIECES_PER_AGE = AGE_MET_SLOTS / 4;                   // 4
static_assert(AGED_PIECES_PER_AGE * AGE_PAD == 32 * KBLOCK_WORDS, "age-major piece mask");
// two units per age plus at most one of padding per group (at most
// AGE_PAD + 1 groups)
constexpr int MAX_AGED_UNITS = (2 * AGE_PAD + (AGE_PAD + 1) + 15) / 16 * 16;   // 304
constexpr int MAX_PLAN_K = MAX_AGED_UNITS > MAX_UNITS ? MAX_AGED_UNITS : MAX_UNITS;
constexpr int MAX_AGED_STAGES = MAX_AGED_UNITS / 2;

struct GalaxyRange {
  int win_lo, win_hi;            // rest-wavelength index window [lo, hi) that any filter sees
  // bit 16 (a % 2) + j of word a / 2 set when metallicity row j has a
  // non-zero weight at some age in [4 a, 4 a + 4); in the age-major layout,
  // bit c % 32 of word c / 32 set when piece c (age c / 4, slots 4 (c % 4) ..)
  // holds a non-zero weight
  unsigned kblk[KBLOCK_WORDS];
  int age_hi;    // ages >= age_hi carry no weight (AGE_PAD when unknown)
};
// Old-star attenuation of the age-dependent model, by sorted position.
struct GalaxyDustOld {
  float dust_a;  // as GalaxyMeta::dust_a, for av_old
  float delta;
};
// Ionization distribution of a galaxy (nebular axis), by sorted position:
// centre, width and the grid points [u_lo, u_hi] its triweight reaches.
struct GalaxyIon {
  float lgu, sigma_u;
  int u_lo, u_hi;
};

// ------------------------------------------------------------- device math
__device__ __forceinline__ double triweight_cdf(double z) {
  // Integral of 35/96 (1 - z^2/9)^3 from -3: 0 below -3, 1 above +3.
  if (z <= -3.0) return 0.0;
  if (z >= 3.0) return 1.0;
  const double z2 = z * z;
  double p = -5.0 / 69984.0;
  p = p * z2 + 7.0 / 2592.0;
  p = p * z2 - 35.0 / 864.0;
  p = p * z2 + 35.0 / 96.0;
  return 0.5 + z * p;
}

// MDF centre at log10 age a (Section 3.2.2, Eq. agedep_mdf): linear in log
// age, or, given an old-age centre, the cumulative-triweight transition from
// the young value lgmet to it over +-3 widths around the pivot.
__device__ __forceinline__ double mdf_transition(double a, double pivot, double width) {
  return triweight_cdf((a - pivot) / width);
}
// young + (old - young) t, taken as old where t is exactly 1, so that both
// asymptotes, and an unchanged value, come out exactly.
__device__ __forceinline__ double triweight_blend(double young, double old, double t) {
  return t == 1.0 ? old : young + (old - young) * t;
}
__device__ __forceinline__ double mdf_centre(double a, double lgmet, bool transition,
                                             double lgmet_old, double slope, double pivot,
                                             double width) {
  return transition ? triweight_blend(lgmet, lgmet_old, mdf_transition(a, pivot, width))
                    : lgmet + slope * (a - pivot);
}

// Weight of ionization point u (Section 3.3, Eq. nebsed): the triweight mass
// of the galaxy's distribution inside the point's bin.
__device__ __forceinline__ double ion_weight(const double *ion_edges, int u, double centre,
                                             double sigma) {
  const double inv = 1.0 / sigma;
  return triweight_cdf((ion_edges[u + 1] - centre) * inv) - triweight_cdf((ion_edges[u] - centre) * inv);
}

__device__ __forceinline__ double triweight_pdf(double z) {
  if (z <= -3.0 || z >= 3.0) return 0.0;
  const double u = 1.0 - z * z * (1.0 / 9.0);
  return (35.0 / 96.0) * u * u * u;
}

// Derivative of ion_weight with respect to the centre (WRT 1) or the width
// (WRT 2): with z_e = (e - centre)/sigma and T the triweight density,
// -(T(z_{u+1}) - T(z_u))/sigma and -(z_{u+1} T(z_{u+1}) - z_u T(z_u))/sigma;
// the infinite outer edges contribute nothing.  WRT 0 is the weight itself.
template <int WRT>
__device__ __forceinline__ double ion_weight_d(const double *ion_edges, int u, double centre,
                                               double sigma) {
  if (WRT == 0) return ion_weight(ion_edges, u, centre, sigma);
  const double inv = 1.0 / sigma;
  double t[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double e = ion_edges[u + s];
    const double z = (e - centre) * inv;
    const double d = triweight_pdf(z);
    t[s] = isinf(e) ? 0.0 : (WRT == 1 ? d : z * d);
  }
  return -(t[1] - t[0]) * inv;
}

// Round-to-nearest-even float32 -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

// Smallest power of two >= m (m > 0 finite), 1 for m == 0.
__device__ __forceinline__ float pow2_ceil(float m) {
  if (!(m > 0.0f)) return 1.0f;
  int e;
  float mant = frexpf(m, &e);  // m = mant * 2^e, mant in [0.5, 1)
  if (mant == 0.5f) e -= 1;
  return ldexpf(1.0f, e);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// ------------------------------------------------------------- host helpers
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

// Brackets one kernel launch with HIP events on `stream` while
// instrumentation is enabled (dsps_profile_enable); a no-op otherwise.
class ProfScope {
 public:
  ProfScope(int kernel_id, hipStream_t stream);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  int kid_;
  hipStream_t stream_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
};

// While an instance lives, ProfScope records nothing on this thread (for
// entry points that must not create events).
class ProfQuiet {
 public:
  ProfQuiet();
  ~ProfQuiet();
  ProfQuiet(const ProfQuiet &) = delete;
  ProfQuiet &operator=(const ProfQuiet &) = delete;
};

// Cosmology parameters passed by value to kernels.
struct CosmoArgs {
  double om0, ol, w0, hubble_time_gyr, hubble_dist_mpc;
  int lcdm;
};
CosmoArgs make_cosmo(const dsps_cosmo &c);

// Gauss-Legendre nodes on [-1, 1], 16 points, filled once on the host.
constexpr int GL_N = 16;
struct GaussLegendre {
  double x[GL_N];
  double w[GL_N];
};
const GaussLegendre &gauss_legendre16();

// ------------------------------------------------------------- launchers
// Defined in k_weights.hip.
// Live galaxies of a launch's range [begin, begin + count) of sorted
// positions.  With a device-side count (a server's padded batch) the ordering
// sort puts the galaxies at and past it last, in their own order, and every
// kernel stops there: their inputs are not read and their outputs not
// written.  Grids stay sized by the host's count; the extra blocks leave.
__device__ __forceinline__ int live_in_range(const int *n_live, int begin, int count) {
  return n_live ? min(count, max(0, *n_live - begin)) : count;
}

struct WeightsLaunch {
  // inputs
  const double *t_table;
  const double *sfr;         // [n_gal][n_t] or null
  const double *sfh_params;  // [5][n_gal] or null
  const float *z, *lgmet, *sigma_z, *av, *delta, *bump;
  int n_gal, n_t;
  double slope, pivot;
  const float *lgmet_old;    // transition MDF (old-age centre), or null (linear model)
  double mdf_width;
  const float *av_old, *delta_old;   // age-dependent attenuation, or null
  const float *lgu, *sigma_u;        // ionization distribution (n_u > 1), or null
  CosmoArgs cosmo;
  GaussLegendre gl;
  SspView ssp;
  // ordering: sorted position s -> galaxy perm[s]; null means identity
  const int *perm;
  int s_begin, s_count;      // sorted range processed by this launch
  const int *n_live;         // device count of live galaxies, or null (live_in_range)
  // outputs (any may be null)
  float *w_user;             // [n_gal][n_met][n_age] natural order (by galaxy index)
  double *mstar;             // [n_gal]
  void *w_pad;               // [s_count][k_pad] float32 or bf16 (by sorted position - s_begin)
  int w_pad_bf16;
  int w_pad_age;             // w_pad is float32 age-major [s_count][AGE_K] instead
  GalaxyDustOld *dust_old;   // [n_gal] by sorted position (age-dependent attenuation)
  GalaxyIon *ion;            // [n_gal] by sorted position (ionization axis), or null
  GalaxyMeta *meta;          // [n_gal] by sorted position
  GalaxyRange *range;        // [n_gal] by sorted position
  double *mag_offset;        // [n_gal] D_mod(z) - 2.5 log10(1+z), by sorted position
  double obs_lo, obs_hi;     // filter support union for the window
  // [n_gal] cosmic time at z by sorted position, written by the per-galaxy
  // scalar pass and read by the weights kernel (required when it runs)
  double *t_obs;
};
int launch_weights(const WeightsLaunch &a, hipStream_t stream);

int launch_sfh_table(const double *t_table, int n_t, const double *params, int n_gal,
                     double *sfr, hipStream_t stream);
// Counting sort of galaxies by (metallicity-row range, redshift bucket).
struct SortLaunch {
  const float *z, *lgmet, *sigma_z;
  const float *lgmet_old;    // transition MDF, or null (linear model)
  int n_gal;
  double slope, pivot, mdf_width, lg_age_first, lg_age_last;
  const double *met_edges;   // [n_met + 1], device
  int n_met;
  const float *lgu, *sigma_u;  // ionization distribution (n_u > 1), or null
  const double *ion_edges;     // [n_u + 1], device
  int n_u;
  int *hist;                 // [SORT_BINS] scratch
  int *perm;                 // [n_gal] sorted position -> galaxy
  // device count of live galaxies, or null: galaxies at and past it are
  // not read and keep their own positions at the end of the order
  const int *n_live;
};
int launch_sort(const SortLaunch &a, hipStream_t stream);
int launch_quantize_bf16(const float *x, int rows, int cols, uint16_t *q, float *scale,
                         hipStream_t stream);
// Tables are written as rows of dst_stride elements (k_pad, or n_u * k_pad
// for one ionization point's block of a wider row).
int launch_pack_table(const float *lum_rows, const uint16_t *q_rows, int n_met, int n_age,
                      int n_wave, int n_wave_pad, int k_pad, int dst_stride, float *st32,
                      uint16_t *st16, hipStream_t stream);
int launch_pack_table_age(const float *lum_rows, int n_met, int n_age, int n_wave, int n_wave_pad,
                          float *sa32, hipStream_t stream);
int launch_pack_table_kmajor(const float *lum_rows, int n_age, int n_wave, int n_wave_pad,
                             int k_pad, int sk_rows, int differenced, float *sk32,
                             hipStream_t stream);

// Defined in k_mags.hip.
// Per 128-galaxy tile of the fused contraction, computed once before it: the
// union of the members' wavelength windows as chunks [c_first, c_last), the
// range of 1 + z, the K units that hold a non-zero weight for some member, in
// ascending order and padded with -1 (a unit of zeros) to whole stages of
// four, and the ionization points [u_lo, u_hi] some member's distribution
// reaches (0, 0 without the axis).
struct TilePlan {
  int c_first, c_last;
  int nk;                        // stages (four units each)
  float zp1_min, zp1_max;
  int u_lo, u_hi;
  int n_units;                   // units before the padding
  int koff[MAX_PLAN_K];           // K offset of each unit in elements, or -1
  // age-major: after stage s, fold the accumulated SED of the group whose
  // ages include tag[s] (-1: the group goes on)
  short tag[MAX_AGED_STAGES];
};

struct MagsLaunch {
  SspView ssp;
  FilterView flt;
  int precision;
  int s_begin, s_count;          // sorted range of this batch
  const int *n_live;             // device count of live galaxies, or null
  const void *w_pad;             // [s_count][k_pad]
  const GalaxyMeta *meta;        // full arrays, by sorted position
  const GalaxyRange *range;
  // age-dependent attenuation (float32 only): W and the table are age-major,
  // ages [0, age_young) use the young-star dust, ages [age_old, n_age) the
  // old-star dust, the ages between their own transition values
  int age_dust;
  const GalaxyDustOld *dust_old;
  int age_young, age_old;
  double dust_pivot, dust_width;
  const GalaxyIon *ion;          // ionization axis (float32 only), by sorted position, or null
  int ion_tangent;               // with ion: 0 weights, 1/2 their derivative in centre/width
  int n_groups;                  // workgroups per tile (upper bound on its chunk groups)
  int n_chunks;                  // n_wave_pad / TILE_L
  int moments;                   // also the three dust moments per band (float32 only)
  // [n_chunks / partial_chunks][part_rows][ncomp * n_band], slot-major: the
  // sums over the chunks of each slot (partial_chunks whole chunks from a
  // multiple of it) inside each tile's window; components num, den and, with
  // moments, the three dust moments
  float *partial;
  int part_rows;                 // galaxy rows per partial slot (>= s_count)
  TilePlan *plan;                // [n_tiles], written by the planning pass
};
// Components per band of the chunk partials.
__host__ __device__ inline int mags_components(int moments) { return moments ? 5 : 2; }
int launch_mags_gemm(const MagsLaunch &a, hipStream_t stream);
// The planning pass alone (reads ssp, precision, s_begin, s_count, meta,
// range, ion, age_dust; writes plan), for the unfused SED.
int launch_tile_plan(const MagsLaunch &a, hipStream_t stream);

struct FinalizeLaunch {
  int n_band, n_chunks;
  int s_begin, s_count;
  const int *n_live;  // device count of live galaxies, or null
  const float *partial;
  const TilePlan *plan;
  const double *mag_offset;
  const int *perm;
  int part_rows;  // galaxy rows per slot of the partials
  int pcg;        // chunks per partial slot (partial_chunks)
  int moments;    // partials carry the dust moments
  float *mags;    // [n_gal][n_band] by galaxy index
  float *bands;   // [n_gal][2][n_band] or null
  float *mom;     // [n_gal][3][n_band] or null (requires moments)
  // tangent pass: the partials hold the derivative's band sums num'; the
  // output is then dm = -2.5 / ln 10 num' / num with num from these forward
  // band sums ([n_gal][2][n_band] by galaxy index)
  const float *tangent_bands;
};
int launch_mags_finalize(const FinalizeLaunch &a, hipStream_t stream);

// Defined in k_eqw.hip.  Per line: centre, 1 / fit_half_width, the grid
// index ranges of the neighbourhood [f0, f1) and of the line window [m0, m1)
// (the continuum points are the first without the second), the inverse of
// the continuum fit's normal matrix, upper triangle row by row, and the
// offset of grid point n in an SED row (n + sed_off: 0 for full rows).
struct EqwLine {
  double centre, inv_fit;
  int f0, f1, m0, m1;
  int sed_off, pad;
  double ginv[6];
};
struct EqwLaunch {
  const double *wave;   // [n_wave] rest Angstrom, device
  const float *sed;     // [n_gal][sed_stride]
  const float *dsed;    // [n_gal][sed_stride] tangent of the SED, or null
  int sed_stride;
  int n_gal, n_wave, n_line;
  float *eqw;           // [n_gal][n_line]
  float *deqw;          // [n_gal][n_line] tangent of the widths (with dsed)
  // SED row r holds galaxy perm[row_begin + r] (rows in sorted order), or
  // galaxy r when perm is null; the widths go to that galaxy's row
  const int *perm;
  int row_begin;
  EqwLine line[DSPS_MAX_LINES];
};
int launch_eqw(const EqwLaunch &a, hipStream_t stream);

// Wavelength chunks one selective SED launch may compute.
constexpr int SED_MAX_CHUNKS = 64;

// Defined in k_sed.hip.
// Galaxies are in the ordering sort's order: g_begin, g_count is a range of
// sorted positions, perm maps a position to its galaxy, and plan holds each
// 128-galaxy tile's stage list (non-zero weight blocks) and ionization range.
struct SedLaunch {
  SspView ssp;
  int precision, apply_dust;
  int g_begin, g_count;
  const int *n_live;            // device count of live galaxies, or null
  const int *perm;
  const TilePlan *plan;         // [tiles of the range]
  const void *w_pad;            // [g_count][k_pad], by sorted position - g_begin
  const GalaxyMeta *meta;       // by sorted position
  const GalaxyIon *ion;         // by sorted position, or null (no ionization axis)
  // with ion: 0 the SED, 1 its derivative in the ionization centre, 2 in the
  // ionization width (the weights of the points replaced by their derivatives)
  int ion_tangent;
  // age-dependent attenuation (float32, apply_dust): W rows and the table
  // are age-major and the attenuation is folded per age group, as in the
  // fused kernel
  int age_dust;
  const GalaxyDustOld *dust_old;   // by sorted position
  int age_young, age_old;
  double dust_pivot, dust_width;
  // chunk selection (n_sel > 0): block x computes wavelength chunk
  // chunk_list[x] and writes it to columns x * TILE_L.. of row s - g_begin
  // (s the sorted position) of rows of out_stride floats (whole chunks,
  // padding included); n_sel == 0: every chunk, row perm[s] of n_wave floats
  int n_sel, out_stride;
  int chunk_list[SED_MAX_CHUNKS];
  float *sed;                   // [n_gal][n_wave]
};
int launch_sed_gemm(const SedLaunch &a, hipStream_t stream);

// Defined in k_vjp.hip.  Stages: 0 gamma, 1 recomputed forward tile with the
// adjoint epilogue, 2 transposed contraction, 3 per-galaxy pull-back.
struct VjpLaunch {
  SspView ssp;
  FilterView flt;
  int n_band, n_groups;         // n_groups: LBAR_CHUNKS-chunk groups per tile
  int s_begin, s_count;
  const int *n_live;            // device count of live galaxies, or null
  const int *perm;
  const float *mags_bar;      // [n_gal][n_band] by galaxy index
  // residual mode (target set, mags_bar unused): the cotangent is
  // (fwd_mags - target) * 2 resid_wt (resid_wt null: 1), all [n_gal][n_band]
  // by galaxy index
  const float *target, *resid_wt, *fwd_mags;
  const float *bands;         // [n_gal][2][n_band] by galaxy index
  const float *moments;       // [n_gal][3][n_band] by galaxy index
  float *gamma;               // [n_gal][n_band] by sorted position
  const GalaxyMeta *meta;
  const GalaxyRange *range;
  float *dust;                // [s_count][3] sum_b gamma_b x each moment
  float *lbar;                // [s_count][n_wave_pad], the tile windows
  float *wbar;                // [s_count][k_pad]
  // [s_count][AGE_PAD] plain Wbar of the lowest row of each galaxy's MDF
  // support (k_vjp_wbar_rows), or null: wbar row 0 is then plain as well
  float *wabs;
  const double *t_obs;        // [n_gal] cosmic time at z, by sorted position
  // population (for the per-galaxy pull-back)
  const double *t_table, *sfr, *sfh_params;
  const float *z, *lgmet, *sigma_z, *av;
  int n_gal, n_t;
  double slope, pivot;
  CosmoArgs cosmo;
  GaussLegendre gl;
  // outputs (by galaxy index; any may be null)
  double *sfr_bar, *sfh_params_bar;
  float *lgmet_bar, *sigma_bar, *av_bar, *delta_bar, *bump_bar;
  const float *lgmet_old;     // transition MDF, or null (linear model)
  double mdf_width;
  float *lgmet_old_bar;
  // ionization axis: the members' distributions by sorted position, or null;
  // then the adjoint table holds one K-major block per ionization point
  const GalaxyIon *ion;
  const float *w_rows;        // [s_count][k_pad] float32 W rows (with ion)
  float *wsuf;                // [s_count][k_pad] their suffix sums over metallicity
  float *ion_part;            // [sk_rows / TILE_L][s_count][2] partial lgu_bar, sigma_u_bar
  float *lgu_bar, *sigma_u_bar;   // by galaxy index, or null
  // age-dependent attenuation: Lbar is written without the attenuation and
  // the transposed contraction applies each age's own; w_rows then holds the
  // age-major float32 rows [s_count][AGE_K]
  int aged;
  const GalaxyDustOld *dust_old;   // by sorted position
  int age_young, age_old;          // ages below take the young, from age_old the old parameters
  double dust_pivot, dust_width;
  const float *av_old;             // by galaxy index
  float *aged_part;                // [n_age][s_count][3] per-age dust partials
  float *av_old_bar, *delta_old_bar;   // by galaxy index, or null
};
int launch_vjp(const VjpLaunch &a, int stage, hipStream_t stream);


// Defined in k_summary.hip.
constexpr int SUMMARY_CHUNK = 2048;   // galaxies per partial-histogram workgroup
struct SummaryLaunch {
  const float *mags;
  int n_gal, n_band, band_a, band_b, band_m;
  double cut, colour_width, mag_width;
  const double *edges;       // [n_bins + 1]
  int n_bins;
  double *partial;           // [ceil(n_gal / SUMMARY_CHUNK)][n_bins]
  double *hist;              // [n_bins]
  const double *hist_bar;    // [n_bins] (adjoint)
  float *mags_bar;           // [n_gal][n_band] (adjoint)
};
int launch_summary(const SummaryLaunch &a, hipStream_t stream);
int launch_summary_vjp(const SummaryLaunch &a, hipStream_t stream);

}  // namespace dsps
