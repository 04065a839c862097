// Host side of libdsps: argument checks, resident handles, workspace layout
// and the launch sequence of every C-ABI entry point.
#include "dsps_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

namespace dsps {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
  if (e == hipSuccess) return DSPS_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return DSPS_ERR_DEVICE;
}

// hipMalloc that reports the runtime's reason on failure.
static int hip_alloc(void **p, size_t bytes, const char *what) {
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) return DSPS_OK;
  *p = nullptr;
  set_error("hipMalloc of %zu bytes for %s failed: %s", bytes, what, hipGetErrorString(e));
  return DSPS_ERR_ALLOC;
}

#define DSPS_CHECK(cond, code, ...) \
  do {                              \
    if (!(cond)) {                  \
      set_error(__VA_ARGS__);       \
      return (code);                \
    }                               \
  } while (0)

#define DSPS_TRY(expr)           \
  do {                           \
    const int rc_ = (expr);      \
    if (rc_ != DSPS_OK) return rc_; \
  } while (0)

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_16.
static GaussLegendre build_gl16() {
  GaussLegendre gl{};
  const int n = GL_N;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    gl.x[i] = x;
    gl.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return gl;
}

const GaussLegendre &gauss_legendre16() {
  static const GaussLegendre gl = build_gl16();
  return gl;
}

CosmoArgs make_cosmo(const dsps_cosmo &c) {
  CosmoArgs a{};
  a.om0 = c.om0;
  a.ol = 1.0 - c.om0;
  a.w0 = c.w0;
  a.hubble_time_gyr = GYR_PER_MPC_S_KM / (100.0 * c.h);
  a.hubble_dist_mpc = LIGHT_KM_S / (100.0 * c.h);
  a.lcdm = c.w0 == -1.0 ? 1 : 0;
  return a;
}

static int check_cosmo(const dsps_cosmo *c) {
  DSPS_CHECK(c, DSPS_ERR_ARG, "cosmo is NULL");
  DSPS_CHECK(c->om0 > 0.0 && c->om0 <= 1.0, DSPS_ERR_ARG, "om0 must be in (0, 1], got %g", c->om0);
  DSPS_CHECK(c->h > 0.0 && std::isfinite(c->h), DSPS_ERR_ARG, "h must be positive, got %g", c->h);
  DSPS_CHECK(c->w0 < 0.0 && std::isfinite(c->w0), DSPS_ERR_ARG, "w0 must be negative, got %g", c->w0);
  return DSPS_OK;
}

static int check_device(int device) {
  int cur = -1;
  DSPS_TRY(hip_fail(hipGetDevice(&cur), "hipGetDevice"));
  DSPS_CHECK(cur == device, DSPS_ERR_ARG, "handle lives on device %d but device %d is current",
             device, cur);
  return DSPS_OK;
}

// ---------------------------------------------------------------- attenuation
// k0(lambda) of the Salim-type curve: Calzetti et al. (2000) starburst curve
// (R_V = 4.05; UV-optical branch below 0.63 micron) and Leitherer et al.
// (2002) far-UV curve, joined at 0.15 micron in the order chosen.
static double calzetti00(double um) {
  if (um < 0.63)
    return 2.659 * (-2.156 + 1.509 / um - 0.198 / (um * um) + 0.011 / (um * um * um)) + DUST_RV;
  return 2.659 * (-1.857 + 1.040 / um) + DUST_RV;
}
static double leitherer02(double um) {
  return 5.472 + 0.671 / um - 9.218e-3 / (um * um) + 2.620e-3 / (um * um * um);
}
static double k0_curve(double angstrom, int reading) {
  const double um = angstrom * 1e-4;
  const bool below = angstrom < DUST_SWITCH_ANGSTROM;
  if (reading == DSPS_K0_SALIM) return below ? leitherer02(um) : calzetti00(um);
  return below ? calzetti00(um) : leitherer02(um);
}
static double drude_shape(double l) {
  const double lw = l * BUMP_WIDTH;
  const double d = l * l - BUMP_CENTRE * BUMP_CENTRE;
  return lw * lw / (d * d + lw * lw);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace dsps

using namespace dsps;

struct dsps_ssp_s : SspHandle {};
struct dsps_filters_s : FiltersHandle {};

extern "C" {

int dsps_abi_version(void) { return DSPS_ABI_VERSION; }

const char *dsps_last_error(void) { return g_err; }

}  // extern "C"

// ------------------------------------------------------------------ SSP block
// Both create calls: lum is [n_met][n_age][n_u][n_wave] (n_u == 1: the plain
// block, lgu may then be NULL).
static int ssp_create(int n_met, int n_age, int n_u, int n_wave, const double *lgz,
                      const double *lg_age, const double *lgu, const double *wave, const float *lum,
                      int precisions, int k0_reading, dsps_ssp **out) {
  DSPS_CHECK(out && lgz && lg_age && wave && lum, DSPS_ERR_ARG, "NULL argument to dsps_ssp_create");
  DSPS_CHECK(n_met >= 1 && n_met <= DSPS_MAX_MET, DSPS_ERR_SHAPE, "n_met %d outside [1, %d]", n_met, DSPS_MAX_MET);
  DSPS_CHECK(n_age >= 1 && n_age <= DSPS_MAX_AGE, DSPS_ERR_SHAPE, "n_age %d outside [1, %d]", n_age, DSPS_MAX_AGE);
  DSPS_CHECK(n_u >= 1 && n_u <= DSPS_MAX_ION, DSPS_ERR_SHAPE, "n_u %d outside [1, %d]", n_u, DSPS_MAX_ION);
  DSPS_CHECK(n_wave >= 2, DSPS_ERR_SHAPE, "n_wave %d < 2", n_wave);
  DSPS_CHECK((precisions & 3) >= 1 && (precisions & ~(3 | DSPS_SSP_AGE_MAJOR)) == 0, DSPS_ERR_ARG,
             "precisions mask %d invalid", precisions);
  DSPS_CHECK(n_u == 1 || precisions == (1 << DSPS_FP32), DSPS_ERR_UNSUPPORTED,
             "an SSP block with an ionization axis is supported in float32 only");
  DSPS_CHECK(n_u == 1 || lgu, DSPS_ERR_ARG, "lgu is NULL");
  for (int k = 1; k < n_u; ++k) DSPS_CHECK(lgu[k] > lgu[k - 1], DSPS_ERR_ARG, "lgu not ascending");
  DSPS_CHECK(k0_reading == DSPS_K0_SALIM || k0_reading == DSPS_K0_PRINTED, DSPS_ERR_ARG,
             "k0_reading %d invalid", k0_reading);
  for (int j = 1; j < n_met; ++j) DSPS_CHECK(lgz[j] > lgz[j - 1], DSPS_ERR_ARG, "lgz not ascending");
  for (int i = 1; i < n_age; ++i) DSPS_CHECK(lg_age[i] > lg_age[i - 1], DSPS_ERR_ARG, "lg_age not ascending");
  for (int l = 0; l < n_wave; ++l) {
    DSPS_CHECK(wave[l] > 0.0 && std::isfinite(wave[l]), DSPS_ERR_ARG, "wave[%d] not positive", l);
    if (l) DSPS_CHECK(wave[l] > wave[l - 1], DSPS_ERR_ARG, "wave not ascending");
  }
  const size_t n_lum = (size_t)n_met * n_age * n_u * n_wave;
  for (size_t i = 0; i < n_lum; ++i)
    DSPS_CHECK(lum[i] >= 0.0f && std::isfinite(lum[i]), DSPS_ERR_ARG, "lum[%zu] negative or not finite", i);

  SspView v{};
  v.n_met = n_met;
  v.n_age = n_age;
  v.n_wave = n_wave;
  v.n_wave_pad = (n_wave + TILE_L - 1) / TILE_L * TILE_L;
  v.k_pad = n_met * AGE_PAD;
  v.n_u = n_u;
  v.k_row = n_u * v.k_pad;
  const int nwp = v.n_wave_pad, kp = v.k_pad;
  const bool want32 = precisions & (1 << DSPS_FP32), want16 = precisions & (1 << DSPS_BF16);
  const bool want_age = precisions & DSPS_SSP_AGE_MAJOR;

  // host-side derived tables
  std::vector<double> age_edges(n_age + 1), met_edges(n_met + 1);
  age_edges[0] = 0.0;
  for (int i = 1; i < n_age; ++i) age_edges[i] = std::pow(10.0, 0.5 * (lg_age[i - 1] + lg_age[i])) / YEARS_PER_GYR;
  age_edges[n_age] = std::numeric_limits<double>::infinity();
  met_edges[0] = -std::numeric_limits<double>::infinity();
  for (int j = 1; j < n_met; ++j) met_edges[j] = 0.5 * (lgz[j - 1] + lgz[j]);
  met_edges[n_met] = std::numeric_limits<double>::infinity();
  std::vector<double> ion_edges(n_u + 1);
  ion_edges[0] = -std::numeric_limits<double>::infinity();
  for (int k = 1; k < n_u; ++k) ion_edges[k] = 0.5 * (lgu[k - 1] + lgu[k]);
  ion_edges[n_u] = std::numeric_limits<double>::infinity();
  std::vector<float4> lconst(nwp);
  std::vector<float> qw(nwp, 0.0f);
  for (int l = 0; l < nwp; ++l) {
    const double lam = wave[std::min(l, n_wave - 1)];
    lconst[l] = make_float4((float)lam, (float)std::log2(lam / DUST_LAMBDA_V),
                            (float)k0_curve(lam, k0_reading), (float)drude_shape(lam));
    if (l < n_wave) {
      const double lo = wave[std::max(l - 1, 0)], hi = wave[std::min(l + 1, n_wave - 1)];
      qw[l] = (float)(0.5 * (hi - lo) / lam);
    }
  }

  // one device allocation for the resident block
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
  const size_t o_wave = take(sizeof(double) * n_wave);
  const size_t o_age = take(sizeof(double) * (n_age + 1));
  const size_t o_met = take(sizeof(double) * (n_met + 1));
  const size_t o_lg = take(sizeof(double) * n_age);
  const size_t o_ion = take(sizeof(double) * (n_u + 1));
  const size_t o_st32 = want32 ? take(sizeof(float) * (size_t)nwp * v.k_row) : 0;
  const size_t o_st16 = want16 ? take(sizeof(uint16_t) * (size_t)nwp * kp) : 0;
  const int sk_rows = (kp + TILE_L - 1) / TILE_L * TILE_L;
  const bool want_sk = want32;   // the adjoint's table, one block per ionization point
  // without the ionization axis the plain K-major rows follow the differenced ones
  const size_t o_sk = want_sk ? take(sizeof(float) * (size_t)(n_u == 1 ? 2 : n_u) * sk_rows * nwp) : 0;
  const size_t o_sa = want_age ? take(sizeof(float) * (size_t)nwp * AGE_K) : 0;
  const size_t o_ks = take(sizeof(float) * kp);
  const size_t o_lc = take(sizeof(float4) * nwp);
  const size_t o_q = take(sizeof(float) * nwp);
  void *base = nullptr;
  if (int e = hip_alloc(&base, off, "the SSP block")) return e;
  char *b = (char *)base;
  float *d_rows = nullptr;
  uint16_t *d_q = nullptr;
  float *d_scale = nullptr;
  int rc = DSPS_OK;
  auto cleanup = [&]() {
    if (d_rows) (void)hipFree(d_rows);
    if (d_q) (void)hipFree(d_q);
    if (d_scale) (void)hipFree(d_scale);
  };
  do {
    rc = hip_fail(hipMemcpy(b + o_wave, wave, sizeof(double) * n_wave, hipMemcpyHostToDevice), "upload wave");
    if (rc) break;
    rc = hip_fail(hipMemcpy(b + o_age, age_edges.data(), sizeof(double) * (n_age + 1), hipMemcpyHostToDevice), "upload ages");
    if (rc) break;
    rc = hip_fail(hipMemcpy(b + o_met, met_edges.data(), sizeof(double) * (n_met + 1), hipMemcpyHostToDevice), "upload mets");
    if (rc) break;
    rc = hip_fail(hipMemcpy(b + o_lg, lg_age, sizeof(double) * n_age, hipMemcpyHostToDevice), "upload lg_age");
    if (rc) break;
    rc = hip_fail(hipMemcpy(b + o_ion, ion_edges.data(), sizeof(double) * (n_u + 1), hipMemcpyHostToDevice), "upload ion edges");
    if (rc) break;
    rc = hip_fail(hipMemcpy(b + o_lc, lconst.data(), sizeof(float4) * nwp, hipMemcpyHostToDevice), "upload lconst");
    if (rc) break;
    rc = hip_fail(hipMemcpy(b + o_q, qw.data(), sizeof(float) * nwp, hipMemcpyHostToDevice), "upload qweight");
    if (rc) break;
    const int rows = n_met * n_age;
    rc = hip_alloc((void **)&d_rows, sizeof(float) * n_lum, "SSP staging");
    if (rc) break;
    if (n_u == 1) {
      rc = hip_fail(hipMemcpy(d_rows, lum, sizeof(float) * n_lum, hipMemcpyHostToDevice), "upload lum");
    } else {
      // one contiguous (met, age) block per ionization point: [u][met][age][l]
      std::vector<float> slabs(n_lum);
      const size_t slab = (size_t)rows * n_wave;
      for (size_t r = 0; r < (size_t)rows; ++r)
        for (int k = 0; k < n_u; ++k)
          std::copy(lum + (r * n_u + k) * n_wave, lum + (r * n_u + k + 1) * n_wave,
                    slabs.begin() + k * slab + r * n_wave);
      rc = hip_fail(hipMemcpy(d_rows, slabs.data(), sizeof(float) * n_lum, hipMemcpyHostToDevice), "upload lum");
    }
    if (rc) break;
    std::vector<float> kscale(kp, 1.0f);
    if (want16) {
      rc = hip_alloc((void **)&d_q, sizeof(uint16_t) * n_lum, "BF16 staging");
      if (!rc) rc = hip_alloc((void **)&d_scale, sizeof(float) * rows, "BF16 row scales");
      if (rc) break;
      rc = launch_quantize_bf16(d_rows, rows, n_wave, d_q, d_scale, nullptr);
      if (rc) break;
      std::vector<float> scale(rows);
      rc = hip_fail(hipMemcpy(scale.data(), d_scale, sizeof(float) * rows, hipMemcpyDeviceToHost), "download scales");
      if (rc) break;
      for (int j = 0; j < n_met; ++j)
        for (int i = 0; i < n_age; ++i) kscale[j * AGE_PAD + i] = scale[j * n_age + i];
    }
    rc = hip_fail(hipMemcpy(b + o_ks, kscale.data(), sizeof(float) * kp, hipMemcpyHostToDevice), "upload kscale");
    if (rc) break;
    for (int k = 0; k < n_u && !rc; ++k)
      rc = launch_pack_table(d_rows + (size_t)k * rows * n_wave, d_q, n_met, n_age, n_wave, nwp, kp,
                             v.k_row, want32 ? (float *)(b + o_st32) + (size_t)k * kp : nullptr,
                             want16 ? (uint16_t *)(b + o_st16) : nullptr, nullptr);
    if (rc) break;
    for (int k = 0; want_sk && k < n_u && !rc; ++k)
      rc = launch_pack_table_kmajor(d_rows + (size_t)k * rows * n_wave, n_age, n_wave, nwp, kp,
                                    sk_rows, 1, (float *)(b + o_sk) + (size_t)k * sk_rows * nwp,
                                    nullptr);
    if (rc) break;
    if (want_sk && n_u == 1)
      rc = launch_pack_table_kmajor(d_rows, n_age, n_wave, nwp, kp, sk_rows, 0,
                                    (float *)(b + o_sk) + (size_t)sk_rows * nwp, nullptr);
    if (rc) break;
    if (want_age) rc = launch_pack_table_age(d_rows, n_met, n_age, n_wave, nwp, (float *)(b + o_sa), nullptr);
    if (rc) break;
    rc = hip_fail(hipDeviceSynchronize(), "SSP block preparation");
  } while (false);
  cleanup();
  if (rc != DSPS_OK) {
    (void)hipFree(base);
    return rc;
  }
  v.wave = (const double *)(b + o_wave);
  v.age_edges = (const double *)(b + o_age);
  v.met_edges = (const double *)(b + o_met);
  v.lg_age = (const double *)(b + o_lg);
  v.ion_edges = (const double *)(b + o_ion);
  v.st32 = want32 ? (const float *)(b + o_st32) : nullptr;
  v.st16 = want16 ? (const uint16_t *)(b + o_st16) : nullptr;
  v.kscale = (const float *)(b + o_ks);
  v.lconst = (const float4 *)(b + o_lc);
  v.qweight = (const float *)(b + o_q);
  v.sk32 = want_sk ? (const float *)(b + o_sk) : nullptr;
  v.sk_rows = sk_rows;
  v.sa32 = want_age ? (const float *)(b + o_sa) : nullptr;
  dsps_ssp *h = new dsps_ssp();
  (void)hipGetDevice(&h->device);
  h->precisions = precisions;
  h->k0_reading = k0_reading;
  h->wave_host.assign(wave, wave + n_wave);
  h->lg_age_first = lg_age[0];
  h->lg_age_last = lg_age[n_age - 1];
  h->lg_age_host.assign(lg_age, lg_age + n_age);
  h->v = v;
  h->alloc = base;
  *out = h;
  return DSPS_OK;
}

extern "C" {

int dsps_ssp_create(int n_met, int n_age, int n_wave, const double *lgz, const double *lg_age,
                    const double *wave, const float *lum, int precisions, int k0_reading,
                    dsps_ssp **out) {
  return ssp_create(n_met, n_age, 1, n_wave, lgz, lg_age, nullptr, wave, lum, precisions,
                    k0_reading, out);
}

int dsps_ssp_create_neb(int n_met, int n_age, int n_u, int n_wave, const double *lgz,
                        const double *lg_age, const double *lgu, const double *wave,
                        const float *lum, int precisions, int k0_reading, dsps_ssp **out) {
  DSPS_CHECK(lgu, DSPS_ERR_ARG, "lgu is NULL");
  return ssp_create(n_met, n_age, n_u, n_wave, lgz, lg_age, lgu, wave, lum, precisions, k0_reading,
                    out);
}

int dsps_ssp_ion_info(const dsps_ssp *ssp, int *n_u) {
  DSPS_CHECK(ssp && n_u, DSPS_ERR_ARG, "NULL argument to dsps_ssp_ion_info");
  *n_u = ssp->v.n_u;
  return DSPS_OK;
}

void dsps_ssp_destroy(dsps_ssp *ssp) {
  if (!ssp) return;
  if (ssp->alloc) (void)hipFree(ssp->alloc);
  delete ssp;
}

int dsps_ssp_info(const dsps_ssp *ssp, int *n_met, int *n_age, int *n_wave, int *precisions,
                  int *k0_reading) {
  DSPS_CHECK(ssp, DSPS_ERR_ARG, "ssp is NULL");
  if (n_met) *n_met = ssp->v.n_met;
  if (n_age) *n_age = ssp->v.n_age;
  if (n_wave) *n_wave = ssp->v.n_wave;
  if (precisions) *precisions = ssp->precisions;
  if (k0_reading) *k0_reading = ssp->k0_reading;
  return DSPS_OK;
}

// ------------------------------------------------------------------ filters
int dsps_filters_create(int n_band, int n_pts, const double *wave, const double *trans,
                        dsps_filters **out) {
  DSPS_CHECK(out && wave && trans, DSPS_ERR_ARG, "NULL argument to dsps_filters_create");
  DSPS_CHECK(n_band >= 1 && n_band <= DSPS_MAX_BAND, DSPS_ERR_SHAPE, "n_band %d outside [1, %d]", n_band, DSPS_MAX_BAND);
  DSPS_CHECK(n_pts >= 2 && (long long)n_band * n_pts <= DSPS_MAX_FILTER_FLOATS, DSPS_ERR_SHAPE,
             "n_pts %d invalid (n_band * n_pts must be <= %d)", n_pts, DSPS_MAX_FILTER_FLOATS);
  std::vector<float> tr((size_t)n_band * n_pts);
  std::vector<float2> grid(n_band);
  double lo = std::numeric_limits<double>::infinity(), hi = -lo;
  for (int b = 0; b < n_band; ++b) {
    const double *w = wave + (size_t)b * n_pts;
    const double w0 = w[0], w1 = w[n_pts - 1];
    DSPS_CHECK(w1 > w0 && w0 > 0.0 && std::isfinite(w1), DSPS_ERR_ARG, "filter %d wavelengths invalid", b);
    const double dw = (w1 - w0) / (n_pts - 1);
    for (int i = 0; i < n_pts; ++i) {
      DSPS_CHECK(std::fabs(w[i] - (w0 + i * dw)) <= 1e-9 * w1, DSPS_ERR_UNSUPPORTED,
                 "filter %d is not uniformly gridded", b);
      const double t = trans[(size_t)b * n_pts + i];
      DSPS_CHECK(t >= 0.0 && std::isfinite(t), DSPS_ERR_ARG, "filter %d transmission invalid", b);
      tr[(size_t)b * n_pts + i] = (float)t;
    }
    grid[b] = make_float2((float)w0, (float)(1.0 / dw));
    lo = std::min(lo, w0);
    hi = std::max(hi, w1);
  }
  size_t off = 0;
  const size_t o_tr = off; off += align256(sizeof(float) * tr.size());
  const size_t o_gr = off; off += align256(sizeof(float2) * n_band);
  void *base = nullptr;
  if (int e = hip_alloc(&base, off, "the filter bank")) return e;
  char *b = (char *)base;
  int rc = hip_fail(hipMemcpy(b + o_tr, tr.data(), sizeof(float) * tr.size(), hipMemcpyHostToDevice), "upload filters");
  if (!rc) rc = hip_fail(hipMemcpy(b + o_gr, grid.data(), sizeof(float2) * n_band, hipMemcpyHostToDevice), "upload grids");
  if (rc) { (void)hipFree(base); return rc; }
  dsps_filters *h = new dsps_filters();
  (void)hipGetDevice(&h->device);
  h->v.n_band = n_band;
  h->v.n_pts = n_pts;
  h->v.trans = (const float *)(b + o_tr);
  h->v.grid = (const float2 *)(b + o_gr);
  h->obs_lo = lo;
  h->obs_hi = hi;
  h->alloc = base;
  *out = h;
  return DSPS_OK;
}

void dsps_filters_destroy(dsps_filters *f) {
  if (!f) return;
  if (f->alloc) (void)hipFree(f->alloc);
  delete f;
}

int dsps_filters_info(const dsps_filters *f, int *n_band, int *n_pts) {
  DSPS_CHECK(f, DSPS_ERR_ARG, "filters is NULL");
  if (n_band) *n_band = f->v.n_band;
  if (n_pts) *n_pts = f->v.n_pts;
  return DSPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ workspace
namespace dsps {

// Most galaxies per weights + GEMM round trip.  Populations of up to 256k
// galaxies run in one launch per kernel; the adjoint's per-galaxy scratch
// (Lbar, Wbar and the forward's partials, about 40 KB) then takes about
// 10 GB, which the device's HBM affords.
constexpr int BATCH_FWD = 262144;
constexpr int BATCH_VJP = 262144;

struct Layout {
  size_t hist = 0, perm = 0, meta = 0, range = 0, offset = 0, w = 0, partial = 0, total = 0;
  size_t gamma = 0, dust = 0, lbar = 0, wbar = 0, fbands = 0, tiles = 0, tobs = 0, dust_old = 0;
  size_t ion = 0, wsuf = 0, ipart = 0, apart = 0, ebuf = 0, dbuf = 0, wabs = 0;
  int batch = 0, n_groups = 0, n_chunks = 0;
};

// batch_cap > 0 lowers the galaxies per batch below the default.
static Layout make_layout(int op, const SspView &v, int n_band, int n_gal, int precision,
                          int batch_cap = 0) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
  // as few batches as the cap allows, of equal size in whole tiles (no small
  // last batch that would leave most of the device idle)
  const int cap = op == DSPS_OP_MAGS_VJP ? BATCH_VJP : BATCH_FWD;
  const int n_batches = std::max((n_gal + cap - 1) / cap, 1);
  L.batch = std::min(n_gal, ((n_gal + n_batches - 1) / n_batches + TILE_G - 1) / TILE_G * TILE_G);
  if (batch_cap > 0) L.batch = std::min(L.batch, batch_cap);
  L.n_chunks = v.n_wave_pad / TILE_L;
  const int cpg = chunks_per_group(precision);
  L.n_groups = (L.n_chunks + cpg - 1) / cpg;
  const size_t elem = precision == DSPS_BF16 ? 2 : 4;
  if (op == DSPS_OP_WEIGHTS) {
    L.tobs = take(sizeof(double) * (size_t)n_gal);
    L.total = off;
    return L;
  }
  if (op == DSPS_OP_SED) {
    L.hist = take(sizeof(int) * SORT_BINS);
    L.perm = take(sizeof(int) * (size_t)n_gal);
    L.meta = take(sizeof(GalaxyMeta) * (size_t)n_gal);
    L.range = take(sizeof(GalaxyRange) * (size_t)n_gal);
    L.tobs = take(sizeof(double) * (size_t)n_gal);
    if (v.n_u > 1) L.ion = take(sizeof(GalaxyIon) * (size_t)n_gal);
    // a handle with the age-major table may run the age-dependent attenuation
    L.w = take(elem * (size_t)L.batch * (v.sa32 ? std::max(v.k_pad, AGE_K) : v.k_pad));
    if (v.sa32) L.dust_old = take(sizeof(GalaxyDustOld) * (size_t)n_gal);
    L.tiles = take(sizeof(TilePlan) * (size_t)((L.batch + TILE_G - 1) / TILE_G));
    L.total = off;
    return L;
  }
  L.hist = take(sizeof(int) * SORT_BINS);
  L.perm = take(sizeof(int) * (size_t)n_gal);
  L.meta = take(sizeof(GalaxyMeta) * (size_t)n_gal);
  L.range = take(sizeof(GalaxyRange) * (size_t)n_gal);
  L.offset = take(sizeof(double) * (size_t)n_gal);
  L.tobs = take(sizeof(double) * (size_t)n_gal);
  // a handle with the age-major table may run the age-dependent attenuation,
  // whose weight rows are AGE_K wide
  const bool aged_ok = v.sa32 && (op == DSPS_OP_MAGS || op == DSPS_OP_MAGS_VJP);
  const int w_cols = aged_ok ? std::max(v.k_pad, AGE_K) : v.k_pad;
  L.w = take(elem * (size_t)L.batch * w_cols);
  if (aged_ok) L.dust_old = take(sizeof(GalaxyDustOld) * (size_t)n_gal);
  if (v.n_u > 1 && op == DSPS_OP_MAGS) {
    L.ion = take(sizeof(GalaxyIon) * (size_t)n_gal);
    // the forward magnitudes and band sums an ionization tangent may need
    L.fbands = take(sizeof(float) * (size_t)n_gal * 3 * n_band);
  }
  // float32 forward passes may carry the dust moments
  const int ncomp = mags_components(precision == DSPS_FP32);
  L.partial = take(sizeof(float) * (size_t)L.batch * L.n_chunks * ncomp * n_band);
  L.tiles = take(sizeof(TilePlan) * (size_t)((L.batch + TILE_G - 1) / TILE_G));
  if (op == DSPS_OP_MAGS_VJP) {
    L.gamma = take(sizeof(float) * (size_t)n_gal * n_band);
    L.dust = take(sizeof(float) * (size_t)L.batch * 3);
    L.lbar = take(sizeof(float) * (size_t)L.batch * v.n_wave_pad);
    L.wbar = take(sizeof(float) * (size_t)L.batch * v.k_pad);
    L.wabs = take(sizeof(float) * (size_t)L.batch * AGE_PAD);
    // bands, moments and magnitudes of the forward pass when not supplied
    L.fbands = take(sizeof(float) * (size_t)n_gal * 6 * n_band);
    if (v.n_u > 1) {
      // the members' ionization distributions, the W rows' suffix sums over
      // metallicity and the transposed contraction's per-block partials of
      // the ionization cotangents
      L.ion = take(sizeof(GalaxyIon) * (size_t)n_gal);
      L.wsuf = take(sizeof(float) * (size_t)L.batch * v.k_pad);
      L.ipart = take(sizeof(float) * (size_t)(v.sk_rows / TILE_L) * L.batch * 2);
    }
    // the age-dependent attenuation's per-age dust partials
    if (v.sa32) L.apart = take(sizeof(float) * (size_t)v.n_age * L.batch * 3);
  }
  L.total = off;
  return L;
}

static int check_pop(const dsps_pop *p, bool need_dust) {
  DSPS_CHECK(p, DSPS_ERR_ARG, "pop is NULL");
  DSPS_CHECK(p->n_gal >= 0, DSPS_ERR_SHAPE, "n_gal %d negative", p->n_gal);
  DSPS_CHECK(p->n_t >= 2 && p->n_t <= DSPS_MAX_NT, DSPS_ERR_SHAPE, "n_t %d outside [2, %d]", p->n_t, DSPS_MAX_NT);
  if (p->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(p->t_table, DSPS_ERR_ARG, "t_table is NULL");
  DSPS_CHECK((p->sfr != nullptr) != (p->sfh_params != nullptr), DSPS_ERR_ARG,
             "exactly one of sfr and sfh_params must be set");
  DSPS_CHECK(p->z && p->lgmet && p->sigma_z, DSPS_ERR_ARG, "z, lgmet and sigma_z are required");
  if (need_dust) DSPS_CHECK(p->av && p->delta && p->bump, DSPS_ERR_ARG, "av, delta and bump are required");
  DSPS_CHECK(std::isfinite(p->lgmet_slope) && std::isfinite(p->lg_age_pivot), DSPS_ERR_ARG,
             "lgmet_slope and lg_age_pivot must be finite");
  DSPS_CHECK(!p->lgmet_old || (std::isfinite(p->mdf_width) && p->mdf_width > 0.0), DSPS_ERR_ARG,
             "mdf_width must be finite and > 0 with lgmet_old, got %g", p->mdf_width);
  DSPS_CHECK((p->av_old == nullptr) == (p->delta_old == nullptr), DSPS_ERR_ARG,
             "av_old and delta_old must be given together or both be NULL");
  DSPS_CHECK(!p->av_old || (std::isfinite(p->dust_pivot) && std::isfinite(p->dust_width) &&
                            p->dust_width > 0.0),
             DSPS_ERR_ARG, "dust_pivot must be finite and dust_width finite and > 0 with av_old");
  return DSPS_OK;
}

// The ionization distribution is needed exactly when the block has the axis.
static int check_ion(const dsps_ssp *s, const dsps_pop *p) {
  DSPS_CHECK(s->v.n_u == 1 || p->n_gal == 0 || (p->lgu && p->sigma_u), DSPS_ERR_ARG,
             "the SSP block has an ionization axis: lgu and sigma_u are required");
  return DSPS_OK;
}

static int check_precision(const dsps_ssp *s, int precision) {
  DSPS_CHECK(precision == DSPS_FP32 || precision == DSPS_BF16, DSPS_ERR_ARG, "precision %d invalid", precision);
  DSPS_CHECK(s->precisions & (1 << precision), DSPS_ERR_UNSUPPORTED,
             "SSP handle was created without precision %d", precision);
  return DSPS_OK;
}

static int check_workspace(void *ws, size_t have, size_t need) {
  if (need == 0) return DSPS_OK;
  DSPS_CHECK(ws, DSPS_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
  DSPS_CHECK(((uintptr_t)ws & 255u) == 0, DSPS_ERR_WORKSPACE, "workspace not 256-byte aligned");
  DSPS_CHECK(have >= need, DSPS_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
  return DSPS_OK;
}

static int sort_population(const dsps_ssp *ssp, const dsps_pop *p, int *hist, int *perm,
                           hipStream_t stream) {
  SortLaunch s{};
  s.z = p->z;
  s.lgmet = p->lgmet;
  s.sigma_z = p->sigma_z;
  s.n_gal = p->n_gal;
  s.slope = p->lgmet_slope;
  s.pivot = p->lg_age_pivot;
  s.lgmet_old = p->lgmet_old;
  s.mdf_width = p->mdf_width;
  s.lg_age_first = ssp->lg_age_first;
  s.lg_age_last = ssp->lg_age_last;
  s.met_edges = ssp->v.met_edges;
  s.n_met = ssp->v.n_met;
  if (ssp->v.n_u > 1) {
    s.lgu = p->lgu;
    s.sigma_u = p->sigma_u;
    s.ion_edges = ssp->v.ion_edges;
    s.n_u = ssp->v.n_u;
  }
  s.hist = hist;
  s.perm = perm;
  s.n_live = p->n_live;
  return launch_sort(s, stream);
}

static WeightsLaunch base_weights(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *p) {
  WeightsLaunch a{};
  a.t_table = p->t_table;
  a.sfr = p->sfr;
  a.sfh_params = p->sfh_params;
  a.z = p->z; a.lgmet = p->lgmet; a.sigma_z = p->sigma_z;
  a.av = p->av; a.delta = p->delta; a.bump = p->bump;
  a.n_gal = p->n_gal;
  a.n_live = p->n_live;
  a.n_t = p->n_t;
  a.slope = p->lgmet_slope;
  a.pivot = p->lg_age_pivot;
  a.lgmet_old = p->lgmet_old;
  a.mdf_width = p->mdf_width;
  a.cosmo = make_cosmo(*cosmo);
  a.gl = gauss_legendre16();
  a.av_old = p->av_old;
  a.delta_old = p->delta_old;
  a.lgu = p->lgu;
  a.sigma_u = p->sigma_u;
  a.ssp = ssp->v;
  return a;
}

}  // namespace dsps

extern "C" {

int dsps_workspace_size(int op, const dsps_ssp *ssp, const dsps_filters *filters, int n_gal,
                        int n_t, int precision, size_t *bytes) {
  DSPS_CHECK(ssp && bytes, DSPS_ERR_ARG, "NULL argument to dsps_workspace_size");
  DSPS_CHECK(op >= DSPS_OP_WEIGHTS && op <= DSPS_OP_MAGS_VJP, DSPS_ERR_ARG, "op %d invalid", op);
  DSPS_CHECK(n_gal >= 0, DSPS_ERR_SHAPE, "n_gal negative");
  (void)n_t;
  int n_band = 0;
  if (op == DSPS_OP_MAGS || op == DSPS_OP_MAGS_VJP) {
    DSPS_CHECK(filters, DSPS_ERR_ARG, "filters required for this op");
    n_band = filters->v.n_band;
  }
  *bytes = make_layout(op, ssp->v, n_band, n_gal, precision).total;
  return DSPS_OK;
}

int dsps_sfh_table(const double *t_table, int n_t, const double *sfh_params, int n_gal,
                   double *sfr, hipStream_t stream) {
  DSPS_CHECK(n_gal >= 0 && n_t >= 1, DSPS_ERR_SHAPE, "bad sizes n_gal=%d n_t=%d", n_gal, n_t);
  if (n_gal == 0) return DSPS_OK;
  DSPS_CHECK(t_table && sfh_params && sfr, DSPS_ERR_ARG, "NULL argument to dsps_sfh_table");
  return launch_sfh_table(t_table, n_t, sfh_params, n_gal, sfr, stream);
}

int dsps_quantize_bf16(const float *x, int rows, int cols, uint16_t *q, float *scale,
                       hipStream_t stream) {
  DSPS_CHECK(rows >= 0 && cols >= 0, DSPS_ERR_SHAPE, "negative sizes");
  if (rows == 0 || cols == 0) return DSPS_OK;
  DSPS_CHECK(x && q && scale, DSPS_ERR_ARG, "NULL argument to dsps_quantize_bf16");
  return launch_quantize_bf16(x, rows, cols, q, scale, stream);
}

int dsps_weights(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop, float *w,
                 double *mstar, void *workspace, size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(ssp, DSPS_ERR_ARG, "ssp is NULL");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, false));
  if (pop->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(w, DSPS_ERR_ARG, "w is NULL");
  DSPS_TRY(check_device(ssp->device));
  const Layout L = make_layout(DSPS_OP_WEIGHTS, ssp->v, 0, pop->n_gal, DSPS_FP32);
  DSPS_TRY(check_workspace(workspace, workspace_bytes, L.total));
  WeightsLaunch a = base_weights(ssp, cosmo, pop);
  a.perm = nullptr;
  a.s_begin = 0;
  a.s_count = pop->n_gal;
  a.w_user = w;
  a.mstar = mstar;
  a.t_obs = (double *)((char *)workspace + L.tobs);
  return launch_weights(a, stream);
}

}  // extern "C"

// Unfused SED set-up for the sorted batch [s0, s0 + cnt): weights (W rows,
// per-galaxy scalars, non-zero block masks, ionization supports) and the
// tiles' stage lists.  The ordering sort has run.
// Ages whose dust transition weight is exactly 0 (young: [0, young)) or 1
// (old: [old, n_age)): the triweight's cumulative is 0 at or below -3 widths
// and 1 at or above +3.
static void age_groups(const dsps_ssp *ssp, const dsps_pop *pop, int &young, int &old) {
  const std::vector<double> &ag = ssp->lg_age_host;
  young = 0;
  old = (int)ag.size();
  for (int i = 0; i < (int)ag.size(); ++i) {
    const double zt = (ag[i] - pop->dust_pivot) / pop->dust_width;
    if (zt <= -3.0) young = i + 1;
    if (zt >= 3.0 && old == (int)ag.size()) old = i;
  }
  old = std::max(old, young);
}

static int sed_batch_prepare(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                             int precision, bool age_dust, const Layout &L, char *ws, int s0,
                             int cnt, hipStream_t stream) {
  GalaxyIon *ion = ssp->v.n_u > 1 ? (GalaxyIon *)(ws + L.ion) : nullptr;
  WeightsLaunch a = base_weights(ssp, cosmo, pop);
  a.perm = (const int *)(ws + L.perm);
  a.s_begin = s0;
  a.s_count = cnt;
  a.w_pad = ws + L.w;
  a.w_pad_bf16 = precision == DSPS_BF16;
  a.meta = (GalaxyMeta *)(ws + L.meta);
  a.range = (GalaxyRange *)(ws + L.range);
  a.obs_lo = 0.0;   // the whole grid (the window is not used here)
  a.obs_hi = std::numeric_limits<double>::infinity();
  a.ion = ion;
  a.t_obs = (double *)(ws + L.tobs);
  if (age_dust) {
    a.w_pad_age = 1;
    a.dust_old = (GalaxyDustOld *)(ws + L.dust_old);
  }
  DSPS_TRY(launch_weights(a, stream));
  MagsLaunch m{};
  m.age_dust = age_dust;
  if (age_dust) age_groups(ssp, pop, m.age_young, m.age_old);   // the plan groups ages by them
  m.ssp = ssp->v;
  m.precision = precision;
  m.s_begin = s0;
  m.s_count = cnt;
  m.n_live = pop->n_live;
  m.meta = (const GalaxyMeta *)(ws + L.meta);
  m.range = (const GalaxyRange *)(ws + L.range);
  m.ion = ion;
  m.plan = (TilePlan *)(ws + L.tiles);
  return launch_tile_plan(m, stream);
}

static SedLaunch sed_launch(const dsps_ssp *ssp, const dsps_pop *pop, const Layout &L, char *ws,
                            int precision, int apply_dust, bool age_dust, int s0, int cnt) {
  SedLaunch s{};
  if (age_dust) {
    s.age_dust = 1;
    s.dust_old = (const GalaxyDustOld *)(ws + L.dust_old);
    age_groups(ssp, pop, s.age_young, s.age_old);
    s.dust_pivot = pop->dust_pivot;
    s.dust_width = pop->dust_width;
  }
  s.ssp = ssp->v;
  s.precision = precision;
  s.apply_dust = apply_dust;
  s.g_begin = s0;
  s.g_count = cnt;
  s.n_live = pop->n_live;
  s.perm = (const int *)(ws + L.perm);
  s.plan = (const TilePlan *)(ws + L.tiles);
  s.w_pad = ws + L.w;
  s.meta = (const GalaxyMeta *)(ws + L.meta);
  s.ion = ssp->v.n_u > 1 ? (const GalaxyIon *)(ws + L.ion) : nullptr;
  return s;
}

// dsps_sed and, with ion_tangent 1 or 2, dsps_sed_ion_tangent.
static int sed_common(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                      int apply_dust, int precision, int ion_tangent, float *sed, void *workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(ssp, DSPS_ERR_ARG, "ssp is NULL");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, apply_dust != 0));
  DSPS_CHECK(apply_dust == 0 || apply_dust == 1, DSPS_ERR_ARG, "apply_dust must be 0 or 1");
  const bool age_dust = apply_dust && pop->av_old;
  DSPS_CHECK(!age_dust || (precision == DSPS_FP32 && ssp->v.sa32 && ssp->v.n_u == 1 && !ion_tangent),
             DSPS_ERR_UNSUPPORTED,
             "the age-dependent attenuation needs float32 and an SSP handle created with "
             "DSPS_SSP_AGE_MAJOR (and no ionization axis)");
  DSPS_TRY(check_precision(ssp, precision));
  DSPS_TRY(check_ion(ssp, pop));
  if (pop->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(sed, DSPS_ERR_ARG, "sed is NULL");
  DSPS_TRY(check_device(ssp->device));
  const Layout L = make_layout(DSPS_OP_SED, ssp->v, 0, pop->n_gal, precision);
  DSPS_TRY(check_workspace(workspace, workspace_bytes, L.total));
  char *ws = (char *)workspace;
  DSPS_TRY(sort_population(ssp, pop, (int *)(ws + L.hist), (int *)(ws + L.perm), stream));
  for (int s0 = 0; s0 < pop->n_gal; s0 += L.batch) {
    const int cnt = std::min(L.batch, pop->n_gal - s0);
    DSPS_TRY(sed_batch_prepare(ssp, cosmo, pop, precision, age_dust, L, ws, s0, cnt, stream));
    SedLaunch s = sed_launch(ssp, pop, L, ws, precision, apply_dust, age_dust, s0, cnt);
    s.ion_tangent = ion_tangent;
    s.sed = sed;
    DSPS_TRY(launch_sed_gemm(s, stream));
  }
  return DSPS_OK;
}

extern "C" {

int dsps_sed(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop, int apply_dust,
             int precision, float *sed, void *workspace, size_t workspace_bytes,
             hipStream_t stream) {
  return sed_common(ssp, cosmo, pop, apply_dust, precision, 0, sed, workspace, workspace_bytes,
                    stream);
}

int dsps_sed_ion_tangent(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                         int apply_dust, int wrt, float *dsed, void *workspace,
                         size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(ssp, DSPS_ERR_ARG, "ssp is NULL");
  DSPS_CHECK(wrt == 0 || wrt == 1, DSPS_ERR_ARG, "wrt must be 0 (lgu) or 1 (sigma_u)");
  DSPS_CHECK(ssp->v.n_u > 1, DSPS_ERR_UNSUPPORTED, "the SSP block has no ionization axis");
  return sed_common(ssp, cosmo, pop, apply_dust, DSPS_FP32, 1 + wrt, dsed, workspace,
                    workspace_bytes, stream);
}

// Most 128-wavelength chunks one galaxy's window can span: the window holds
// the rest wavelengths in [obs_lo, obs_hi] / (1+z) plus two points each side,
// i.e. a range of fixed ratio obs_hi/obs_lo; its widest count on the grid is
// reached with the lower end on a grid point.  Sizes the contraction's grid
// (workgroups past a tile's window leave at once, so this only trims them).
static int max_window_chunks(const SspHandle *ssp, const FiltersHandle *flt) {
  const std::vector<double> &w = ssp->wave_host;
  const int n = (int)w.size();
  const double ratio = flt->obs_hi / flt->obs_lo;
  int best = 0;
  for (int i = 0, j = 0; i < n; ++i) {
    j = std::max(j, i);
    while (j < n && w[j] <= w[i] * ratio) ++j;
    best = std::max(best, j - i);
  }
  const int span = std::min(best + 4, n);
  const int n_chunks = ssp->v.n_wave_pad / TILE_L;
  return std::min((span + TILE_L - 1) / TILE_L + 1, n_chunks);
}

// Forward pass over the sorted batch [s0, s0 + cnt): weights, fused
// contraction and finalize.  moments requires the float32 table.
// With ion_tangent (1: centre, 2: width) the weights of the ionization points
// are replaced by their derivatives and `mags` receives dm = -2.5/ln10 dnum/num
// with num from tangent_bands (the forward band sums).
static int mags_batch(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
                      const dsps_pop *pop, int precision, const Layout &L, char *ws, int s0,
                      int cnt, float *mags, float *bands, float *moments, hipStream_t stream,
                      int ion_tangent = 0, const float *tangent_bands = nullptr) {
  int *perm = (int *)(ws + L.perm);
  GalaxyMeta *meta = (GalaxyMeta *)(ws + L.meta);
  GalaxyRange *range = (GalaxyRange *)(ws + L.range);
  double *offset = (double *)(ws + L.offset);
  float *partial = (float *)(ws + L.partial);
  WeightsLaunch a = base_weights(ssp, cosmo, pop);
  a.perm = perm;
  a.s_begin = s0;
  a.s_count = cnt;
  a.w_pad = ws + L.w;
  a.w_pad_bf16 = precision == DSPS_BF16;
  a.meta = meta;
  a.range = range;
  a.mag_offset = offset;
  a.obs_lo = filters->obs_lo;
  a.obs_hi = filters->obs_hi;
  a.t_obs = (double *)(ws + L.tobs);
  const bool age_dust = pop->av_old != nullptr;
  if (age_dust) {
    a.w_pad_age = 1;
    a.dust_old = (GalaxyDustOld *)(ws + L.dust_old);
  }
  GalaxyIon *ion = ssp->v.n_u > 1 ? (GalaxyIon *)(ws + L.ion) : nullptr;
  a.ion = ion;
  DSPS_TRY(launch_weights(a, stream));
  MagsLaunch m{};
  m.ion = ion;
  m.ion_tangent = ion_tangent;
  if (age_dust) {
    m.age_dust = 1;
    m.dust_old = (const GalaxyDustOld *)(ws + L.dust_old);
    age_groups(ssp, pop, m.age_young, m.age_old);
    m.dust_pivot = pop->dust_pivot;
    m.dust_width = pop->dust_width;
  }
  m.ssp = ssp->v;
  m.flt = filters->v;
  m.precision = precision;
  m.s_begin = s0;
  m.s_count = cnt;
  m.n_live = pop->n_live;
  m.w_pad = ws + L.w;
  m.meta = meta;
  m.range = range;
  const int cpg = chunks_per_group(precision);
  // groups aligned to multiples of cpg (float32): a window may straddle one more
  const int pcg = partial_chunks(precision);
  m.n_groups = std::min(L.n_groups, (max_window_chunks(ssp, filters) + cpg - 1) / cpg + (pcg > 1));
  m.n_chunks = L.n_chunks;
  m.moments = moments != nullptr;
  m.partial = partial;
  m.part_rows = L.batch;
  m.plan = (TilePlan *)(ws + L.tiles);
  DSPS_TRY(launch_mags_gemm(m, stream));
  FinalizeLaunch f{};
  f.n_band = filters->v.n_band;
  f.n_chunks = L.n_chunks;
  f.plan = (const TilePlan *)(ws + L.tiles);
  f.s_begin = s0;
  f.s_count = cnt;
  f.n_live = pop->n_live;
  f.partial = partial;
  f.part_rows = L.batch;
  f.pcg = pcg;
  f.mag_offset = offset;
  f.perm = perm;
  f.moments = m.moments;
  f.mags = mags;
  f.bands = bands;
  f.mom = moments;
  f.tangent_bands = tangent_bands;
  return launch_mags_finalize(f, stream);
}

int dsps_mags(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
              const dsps_pop *pop, int precision, float *mags, float *bands, float *moments,
              void *workspace, size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(ssp && filters, DSPS_ERR_ARG, "ssp or filters is NULL");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, true));
  DSPS_TRY(check_precision(ssp, precision));
  DSPS_CHECK(!moments || precision == DSPS_FP32, DSPS_ERR_UNSUPPORTED,
             "dust moments are computed in float32 only");
  DSPS_CHECK(!pop->av_old || (precision == DSPS_FP32 && !moments && ssp->v.sa32), DSPS_ERR_UNSUPPORTED,
             "age-dependent attenuation needs float32, no moments and an SSP handle created with "
             "DSPS_SSP_AGE_MAJOR");
  DSPS_TRY(check_ion(ssp, pop));
  DSPS_CHECK(ssp->v.n_u == 1 || !pop->av_old, DSPS_ERR_UNSUPPORTED,
             "with an ionization axis dsps_mags does not apply the age-dependent attenuation");
  if (pop->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(mags, DSPS_ERR_ARG, "mags is NULL");
  DSPS_TRY(check_device(ssp->device));
  DSPS_CHECK(filters->device == ssp->device, DSPS_ERR_ARG, "ssp and filters on different devices");
  const int n_band = filters->v.n_band;
  const Layout L = make_layout(DSPS_OP_MAGS, ssp->v, n_band, pop->n_gal, precision);
  DSPS_TRY(check_workspace(workspace, workspace_bytes, L.total));
  char *ws = (char *)workspace;
  DSPS_TRY(sort_population(ssp, pop, (int *)(ws + L.hist), (int *)(ws + L.perm), stream));
  for (int s0 = 0; s0 < pop->n_gal; s0 += L.batch) {
    const int cnt = std::min(L.batch, pop->n_gal - s0);
    DSPS_TRY(mags_batch(ssp, filters, cosmo, pop, precision, L, ws, s0, cnt, mags, bands, moments,
                        stream));
  }
  return DSPS_OK;
}

}  // extern "C"

// ------------------------------------------------------- no-allocation scratch
namespace dsps {

// Scratch of dsps_mags_noalloc.  In host code this name is a host-side
// stand-in, not a device address: only the per-device pointer that
// hipGetSymbolAddress returns may reach a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[DSPS_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
static int noalloc_scratch(int device, void **ptr) {
  DSPS_CHECK(device >= 0 && device < MAX_DEVICES, DSPS_ERR_DEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    DSPS_TRY(hip_fail(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
    DSPS_CHECK(p && ((uintptr_t)p & 255u) == 0, DSPS_ERR_DEVICE, "scratch array misplaced");
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return DSPS_OK;
}

// The largest batch (a whole number of 128-galaxy tiles, at most the
// default) whose forward layout fits the scratch array; 0 when even one
// tile's batch does not.
static int noalloc_batch(const SspView &v, int n_band, int n_gal, int precision, Layout *out) {
  int lo = 0, hi = (std::min(n_gal, BATCH_FWD) + TILE_G - 1) / TILE_G;   // in tiles
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (make_layout(DSPS_OP_MAGS, v, n_band, n_gal, precision, mid * TILE_G).total <=
        DSPS_NOALLOC_SCRATCH_BYTES)
      lo = mid;
    else
      hi = mid - 1;
  }
  if (lo > 0) *out = make_layout(DSPS_OP_MAGS, v, n_band, n_gal, precision, lo * TILE_G);
  return lo * TILE_G;
}

}  // namespace dsps

extern "C" {

int dsps_mags_noalloc(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
                      const dsps_pop *pop, int precision, float *mags, float *bands,
                      float *moments, hipStream_t stream) {
  DSPS_CHECK(ssp && filters, DSPS_ERR_ARG, "ssp or filters is NULL");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, true));
  DSPS_TRY(check_precision(ssp, precision));
  DSPS_CHECK(!moments || precision == DSPS_FP32, DSPS_ERR_UNSUPPORTED,
             "dust moments are computed in float32 only");
  DSPS_CHECK(!pop->av_old || (precision == DSPS_FP32 && !moments && ssp->v.sa32), DSPS_ERR_UNSUPPORTED,
             "age-dependent attenuation needs float32, no moments and an SSP handle created with "
             "DSPS_SSP_AGE_MAJOR");
  DSPS_TRY(check_ion(ssp, pop));
  DSPS_CHECK(ssp->v.n_u == 1 || !pop->av_old, DSPS_ERR_UNSUPPORTED,
             "with an ionization axis dsps_mags does not apply the age-dependent attenuation");
  if (pop->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(mags, DSPS_ERR_ARG, "mags is NULL");
  const int n_band = filters->v.n_band;
  Layout L;
  const int batch = noalloc_batch(ssp->v, n_band, pop->n_gal, precision, &L);
  DSPS_CHECK(batch > 0, DSPS_ERR_SHAPE,
             "n_gal %d does not fit the %zu-byte scratch of dsps_mags_noalloc (it needs %zu bytes "
             "at one tile per batch); use dsps_mags with a workspace",
             pop->n_gal, (size_t)DSPS_NOALLOC_SCRATCH_BYTES,
             make_layout(DSPS_OP_MAGS, ssp->v, n_band, pop->n_gal, precision, TILE_G).total);
  DSPS_TRY(check_device(ssp->device));
  DSPS_CHECK(filters->device == ssp->device, DSPS_ERR_ARG, "ssp and filters on different devices");
  void *ptr = nullptr;
  DSPS_TRY(noalloc_scratch(ssp->device, &ptr));
  char *ws = (char *)ptr;
  ProfQuiet quiet;   // instrumentation would create events
  DSPS_TRY(sort_population(ssp, pop, (int *)(ws + L.hist), (int *)(ws + L.perm), stream));
  for (int s0 = 0; s0 < pop->n_gal; s0 += L.batch) {
    const int cnt = std::min(L.batch, pop->n_gal - s0);
    DSPS_TRY(mags_batch(ssp, filters, cosmo, pop, precision, L, ws, s0, cnt, mags, bands, moments,
                        stream));
  }
  return DSPS_OK;
}

int dsps_mags_ion_tangent(const dsps_ssp *ssp, const dsps_filters *filters,
                          const dsps_cosmo *cosmo, const dsps_pop *pop, int wrt,
                          const float *bands, float *dmags, void *workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(ssp && filters, DSPS_ERR_ARG, "ssp or filters is NULL");
  DSPS_CHECK(wrt == 0 || wrt == 1, DSPS_ERR_ARG, "wrt must be 0 (lgu) or 1 (sigma_u)");
  DSPS_CHECK(ssp->v.n_u > 1, DSPS_ERR_UNSUPPORTED, "the SSP block has no ionization axis");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, true));
  DSPS_TRY(check_ion(ssp, pop));
  DSPS_CHECK(!pop->av_old, DSPS_ERR_UNSUPPORTED,
             "with an ionization axis dsps_mags does not apply the age-dependent attenuation");
  if (pop->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(dmags, DSPS_ERR_ARG, "dmags is NULL");
  DSPS_TRY(check_device(ssp->device));
  DSPS_CHECK(filters->device == ssp->device, DSPS_ERR_ARG, "ssp and filters on different devices");
  const int n_band = filters->v.n_band;
  const Layout L = make_layout(DSPS_OP_MAGS, ssp->v, n_band, pop->n_gal, DSPS_FP32);
  DSPS_TRY(check_workspace(workspace, workspace_bytes, L.total));
  char *ws = (char *)workspace;
  float *fwd_mags = (float *)(ws + L.fbands);
  float *fwd_bands = fwd_mags + (size_t)pop->n_gal * n_band;
  const float *use_bands = bands ? bands : fwd_bands;
  DSPS_TRY(sort_population(ssp, pop, (int *)(ws + L.hist), (int *)(ws + L.perm), stream));
  for (int s0 = 0; s0 < pop->n_gal; s0 += L.batch) {
    const int cnt = std::min(L.batch, pop->n_gal - s0);
    if (!bands)
      DSPS_TRY(mags_batch(ssp, filters, cosmo, pop, DSPS_FP32, L, ws, s0, cnt, fwd_mags, fwd_bands,
                          nullptr, stream));
    DSPS_TRY(mags_batch(ssp, filters, cosmo, pop, DSPS_FP32, L, ws, s0, cnt, dmags, nullptr, nullptr,
                        stream, 1 + wrt, use_bands));
  }
  return DSPS_OK;
}

}  // extern "C"

namespace dsps {

// The cotangent of the magnitudes: given (mags_bar), or in residual mode
// (target set) the cotangent of sum wt (m - target)^2, formed on the device
// from the forward magnitudes, which go to mags_out.
struct MagsCotangent {
  const float *mags_bar;
  const float *target, *wt;
  float *mags_out;
};

static int mags_vjp_common(const dsps_ssp *ssp, const dsps_filters *filters,
                           const dsps_cosmo *cosmo, const dsps_pop *pop, int precision,
                           const MagsCotangent &ct, const float *bands, const float *moments,
                           double *sfr_bar, double *sfh_params_bar, float *lgmet_bar,
                           float *lgmet_old_bar, float *sigma_bar, float *av_bar, float *delta_bar,
                           float *bump_bar, float *av_old_bar, float *delta_old_bar,
                           float *lgu_bar, float *sigma_u_bar, void *workspace,
                           size_t workspace_bytes, hipStream_t stream) {
  const float *mags_bar = ct.mags_bar;
  const bool residual = ct.target != nullptr;
  DSPS_CHECK(ssp && filters, DSPS_ERR_ARG, "ssp or filters is NULL");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, true));
  DSPS_TRY(check_precision(ssp, precision));
  DSPS_CHECK(precision == DSPS_FP32, DSPS_ERR_UNSUPPORTED, "the adjoint runs in float32 only");
  const bool age_dust = pop->av_old != nullptr;
  DSPS_CHECK(!age_dust || (ssp->v.sa32 && ssp->v.n_u == 1), DSPS_ERR_UNSUPPORTED,
             "the age-dependent attenuation needs an SSP handle created with DSPS_SSP_AGE_MAJOR "
             "(and no ionization axis)");
  DSPS_CHECK(age_dust || (!av_old_bar && !delta_old_bar), DSPS_ERR_ARG,
             "av_old_bar and delta_old_bar require the population to carry av_old");
  DSPS_TRY(check_ion(ssp, pop));
  DSPS_CHECK(ssp->v.n_u > 1 || (!lgu_bar && !sigma_u_bar), DSPS_ERR_ARG,
             "lgu_bar and sigma_u_bar need an SSP block with an ionization axis");
  if (pop->n_gal == 0) return DSPS_OK;
  if (residual)
    DSPS_CHECK(ct.mags_out && !bands && !moments, DSPS_ERR_ARG, "mags is NULL");
  else
    DSPS_CHECK(mags_bar, DSPS_ERR_ARG, "mags_bar is NULL");
  if (age_dust)
    DSPS_CHECK(!moments, DSPS_ERR_ARG,
               "the age-dependent attenuation has no dust moments: pass moments = NULL");
  else
    DSPS_CHECK((bands == nullptr) == (moments == nullptr), DSPS_ERR_ARG,
               "bands and moments must be given together or both be NULL");
  DSPS_CHECK(!sfh_params_bar || pop->sfh_params, DSPS_ERR_ARG,
             "sfh_params_bar requires the population to carry sfh_params");
  DSPS_CHECK(!lgmet_old_bar || pop->lgmet_old, DSPS_ERR_ARG,
             "lgmet_old_bar requires the population to carry lgmet_old");
  DSPS_TRY(check_device(ssp->device));
  DSPS_CHECK(filters->device == ssp->device, DSPS_ERR_ARG, "ssp and filters on different devices");
  const int n_band = filters->v.n_band;
  const Layout L = make_layout(DSPS_OP_MAGS_VJP, ssp->v, n_band, pop->n_gal, precision);
  DSPS_TRY(check_workspace(workspace, workspace_bytes, L.total));
  char *ws = (char *)workspace;
  int *perm = (int *)(ws + L.perm);
  float *fwd = (float *)(ws + L.fbands);
  float *fwd_bands = fwd;
  float *fwd_mom = fwd + (size_t)pop->n_gal * 2 * n_band;
  float *fwd_mags = fwd + (size_t)pop->n_gal * 5 * n_band;
  const float *use_bands = bands ? bands : fwd_bands;
  const float *use_mom = moments ? moments : fwd_mom;
  DSPS_TRY(sort_population(ssp, pop, (int *)(ws + L.hist), perm, stream));
  for (int s0 = 0; s0 < pop->n_gal; s0 += L.batch) {
    const int cnt = std::min(L.batch, pop->n_gal - s0);
    if (bands) {
      // only the per-galaxy scalars and windows are needed (no weight rows)
      WeightsLaunch a = base_weights(ssp, cosmo, pop);
      a.perm = perm;
      a.s_begin = s0;
      a.s_count = cnt;
      a.meta = (GalaxyMeta *)(ws + L.meta);
      a.range = (GalaxyRange *)(ws + L.range);
      a.mag_offset = (double *)(ws + L.offset);
      a.obs_lo = filters->obs_lo;
      a.obs_hi = filters->obs_hi;
      a.ion = ssp->v.n_u > 1 ? (GalaxyIon *)(ws + L.ion) : nullptr;
      a.t_obs = (double *)(ws + L.tobs);
      if (ssp->v.n_u > 1 || age_dust)     // the W rows for the ionization or dust cotangents
        a.w_pad = ws + L.w;
      if (age_dust) {
        a.w_pad_age = 1;
        a.dust_old = (GalaxyDustOld *)(ws + L.dust_old);
      }
      DSPS_TRY(launch_weights(a, stream));
    } else {
      DSPS_TRY(mags_batch(ssp, filters, cosmo, pop, DSPS_FP32, L, ws, s0, cnt,
                          residual ? ct.mags_out : fwd_mags, fwd_bands,
                          age_dust ? nullptr : fwd_mom, stream));
    }
    VjpLaunch v{};
    v.ssp = ssp->v;
    v.flt = filters->v;
    v.n_band = n_band;
    v.n_groups = (L.n_chunks + LBAR_CHUNKS - 1) / LBAR_CHUNKS;
    v.s_begin = s0;
    v.s_count = cnt;
    v.n_live = pop->n_live;
    v.perm = perm;
    v.mags_bar = mags_bar;
    if (residual) {
      v.target = ct.target;
      v.resid_wt = ct.wt;
      v.fwd_mags = ct.mags_out;
    }
    v.bands = use_bands;
    v.moments = age_dust ? nullptr : use_mom;
    v.gamma = (float *)(ws + L.gamma);
    v.meta = (const GalaxyMeta *)(ws + L.meta);
    v.range = (const GalaxyRange *)(ws + L.range);
    v.dust = (float *)(ws + L.dust);
    v.lbar = (float *)(ws + L.lbar);
    v.wbar = (float *)(ws + L.wbar);
    // the plain transposed contraction starts each galaxy at its lowest
    // support row (k_vjp_wbar_rows)
    v.wabs = (ssp->v.n_u == 1 && !age_dust) ? (float *)(ws + L.wabs) : nullptr;
    v.t_obs = (const double *)(ws + L.tobs);
    v.t_table = pop->t_table;
    v.sfr = pop->sfr;
    v.sfh_params = pop->sfh_params;
    v.z = pop->z;
    v.lgmet = pop->lgmet;
    v.sigma_z = pop->sigma_z;
    v.av = pop->av;
    v.n_gal = pop->n_gal;
    v.n_t = pop->n_t;
    v.slope = pop->lgmet_slope;
    v.pivot = pop->lg_age_pivot;
    v.lgmet_old = pop->lgmet_old;
    v.mdf_width = pop->mdf_width;
    v.lgmet_old_bar = lgmet_old_bar;
    v.cosmo = make_cosmo(*cosmo);
    v.gl = gauss_legendre16();
    v.sfr_bar = sfr_bar;
    v.sfh_params_bar = sfh_params_bar;
    v.lgmet_bar = lgmet_bar;
    v.sigma_bar = sigma_bar;
    v.av_bar = av_bar;
    v.delta_bar = delta_bar;
    v.bump_bar = bump_bar;
    if (ssp->v.n_u > 1) {
      v.ion = (const GalaxyIon *)(ws + L.ion);
      v.w_rows = (const float *)(ws + L.w);
      v.wsuf = (float *)(ws + L.wsuf);
      v.ion_part = (float *)(ws + L.ipart);
      v.lgu_bar = lgu_bar;
      v.sigma_u_bar = sigma_u_bar;
    }
    if (age_dust) {
      v.aged = 1;
      v.dust_old = (const GalaxyDustOld *)(ws + L.dust_old);
      age_groups(ssp, pop, v.age_young, v.age_old);
      v.dust_pivot = pop->dust_pivot;
      v.dust_width = pop->dust_width;
      v.av_old = pop->av_old;
      v.w_rows = (const float *)(ws + L.w);
      v.aged_part = (float *)(ws + L.apart);
      v.av_old_bar = av_old_bar;
      v.delta_old_bar = delta_old_bar;
    }
    for (int stage = 0; stage < 4; ++stage) DSPS_TRY(launch_vjp(v, stage, stream));
  }
  return DSPS_OK;
}

}  // namespace dsps

extern "C" {

int dsps_mags_vjp(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
                  const dsps_pop *pop, int precision, const float *mags_bar, const float *bands,
                  const float *moments, double *sfr_bar, double *sfh_params_bar, float *lgmet_bar,
                  float *lgmet_old_bar, float *sigma_bar, float *av_bar, float *delta_bar,
                  float *bump_bar, float *av_old_bar, float *delta_old_bar, float *lgu_bar,
                  float *sigma_u_bar, void *workspace, size_t workspace_bytes,
                  hipStream_t stream) {
  return mags_vjp_common(ssp, filters, cosmo, pop, precision, {mags_bar, nullptr, nullptr, nullptr},
                         bands, moments, sfr_bar, sfh_params_bar, lgmet_bar, lgmet_old_bar,
                         sigma_bar, av_bar, delta_bar, bump_bar, av_old_bar, delta_old_bar,
                         lgu_bar, sigma_u_bar, workspace, workspace_bytes, stream);
}

int dsps_mags_residual_vjp(const dsps_ssp *ssp, const dsps_filters *filters,
                           const dsps_cosmo *cosmo, const dsps_pop *pop, const float *target,
                           const float *wt, float *mags, double *sfr_bar, double *sfh_params_bar,
                           float *lgmet_bar, float *lgmet_old_bar, float *sigma_bar,
                           float *av_bar, float *delta_bar, float *bump_bar, float *av_old_bar,
                           float *delta_old_bar, float *lgu_bar, float *sigma_u_bar,
                           void *workspace, size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(target || (pop && pop->n_gal == 0), DSPS_ERR_ARG, "target is NULL");
  return mags_vjp_common(ssp, filters, cosmo, pop, DSPS_FP32,
                         {nullptr, target, wt, mags}, nullptr,
                         nullptr, sfr_bar, sfh_params_bar, lgmet_bar, lgmet_old_bar, sigma_bar,
                         av_bar, delta_bar, bump_bar, av_old_bar, delta_old_bar, lgu_bar,
                         sigma_u_bar, workspace, workspace_bytes, stream);
}

}  // extern "C"

// Checks the lines and fills a.line (grid index ranges, inverted normal
// matrices; sed_off 0) and a.wave / a.n_wave / a.n_line.
static int prepare_lines(const dsps_ssp *ssp, const dsps_line *lines, int n_line, EqwLaunch &a) {
  DSPS_CHECK(ssp && lines, DSPS_ERR_ARG, "ssp or lines is NULL");
  DSPS_CHECK(n_line >= 1 && n_line <= DSPS_MAX_LINES, DSPS_ERR_SHAPE, "n_line %d outside [1, %d]",
             n_line, DSPS_MAX_LINES);
  const std::vector<double> &w = ssp->wave_host;
  const int n_wave = (int)w.size();
  a.wave = ssp->v.wave;
  a.n_wave = n_wave;
  a.n_line = n_line;
  for (int li = 0; li < n_line; ++li) {
    const dsps_line &L = lines[li];
    DSPS_CHECK(std::isfinite(L.centre) && std::isfinite(L.fit_half_width) && L.half_width > 0.0 &&
                   L.half_width < L.fit_half_width,
               DSPS_ERR_ARG, "line %d: need finite values with 0 < half_width < fit_half_width", li);
    // both windows are contiguous on the ascending grid
    int f0 = n_wave, f1 = 0, m0 = n_wave, m1 = 0;
    for (int n = 0; n < n_wave; ++n) {
      const double d = std::fabs(w[n] - L.centre);
      if (d <= L.fit_half_width) { f0 = std::min(f0, n); f1 = n + 1; }
      if (d <= L.half_width) { m0 = std::min(m0, n); m1 = n + 1; }
    }
    if (m1 <= m0) m0 = m1 = 0;
    DSPS_CHECK(m1 - m0 >= 2 && (f1 - f0) - (m1 - m0) >= 3, DSPS_ERR_SHAPE,
               "line %d: %d window and %d continuum points on the grid (need >= 2 and >= 3)", li,
               m1 - m0, std::max(0, (f1 - f0) - (m1 - m0)));
    EqwLine &e = a.line[li];
    e.centre = L.centre;
    e.inv_fit = 1.0 / L.fit_half_width;
    e.f0 = f0; e.f1 = f1; e.m0 = m0; e.m1 = m1;
    // normal matrix of the quadratic fit, inverted by cofactors
    long double S[5] = {0, 0, 0, 0, 0};
    for (int n = f0; n < f1; ++n) {
      if (n >= m0 && n < m1) continue;
      const long double x = (long double)((w[n] - L.centre) * e.inv_fit);
      long double p = 1.0L;
      for (int k = 0; k < 5; ++k) { S[k] += p; p *= x; }
    }
    const long double g00 = S[0], g01 = S[1], g02 = S[2], g11 = S[2], g12 = S[3], g22 = S[4];
    const long double a00 = g11 * g22 - g12 * g12, a01 = g02 * g12 - g01 * g22,
                      a02 = g01 * g12 - g02 * g11, a11 = g00 * g22 - g02 * g02,
                      a12 = g01 * g02 - g00 * g12, a22 = g00 * g11 - g01 * g01;
    const long double det = g00 * a00 + g01 * a01 + g02 * a02;
    DSPS_CHECK(det > 0.0L, DSPS_ERR_SHAPE, "line %d: continuum fit is singular", li);
    e.ginv[0] = (double)(a00 / det); e.ginv[1] = (double)(a01 / det); e.ginv[2] = (double)(a02 / det);
    e.ginv[3] = (double)(a11 / det); e.ginv[4] = (double)(a12 / det); e.ginv[5] = (double)(a22 / det);
    e.sed_off = 0;
  }
  return DSPS_OK;
}

static int eqw_common(const dsps_ssp *ssp, const float *sed, const float *dsed, int n_gal,
                      const dsps_line *lines, int n_line, float *eqw, float *deqw,
                      hipStream_t stream) {
  DSPS_CHECK(n_gal >= 0, DSPS_ERR_SHAPE, "n_gal %d negative", n_gal);
  EqwLaunch a{};
  DSPS_TRY(prepare_lines(ssp, lines, n_line, a));
  a.sed = sed;
  a.dsed = dsed;
  a.sed_stride = a.n_wave;
  a.n_gal = n_gal;
  a.eqw = eqw;
  a.deqw = deqw;
  if (n_gal == 0) return DSPS_OK;
  DSPS_CHECK(sed && eqw, DSPS_ERR_ARG, "sed or eqw is NULL");
  DSPS_TRY(check_device(ssp->device));
  return launch_eqw(a, stream);
}

// Wavelength chunks the lines' neighbourhoods touch, line by line (a chunk
// shared by two lines is listed twice), and each line's offset into the
// compact rows that hold them.
static int select_chunks(EqwLaunch &a, SedLaunch &s) {
  s.n_sel = 0;
  for (int li = 0; li < a.n_line; ++li) {
    EqwLine &e = a.line[li];
    const int c0 = e.f0 / TILE_L, c1 = (e.f1 - 1) / TILE_L + 1;
    DSPS_CHECK(s.n_sel + (c1 - c0) <= SED_MAX_CHUNKS, DSPS_ERR_SHAPE,
               "the lines' neighbourhoods span more than %d wavelength chunks of %d points",
               SED_MAX_CHUNKS, TILE_L);
    e.sed_off = (s.n_sel - c0) * TILE_L;
    for (int c = c0; c < c1; ++c) s.chunk_list[s.n_sel++] = c;
  }
  s.out_stride = s.n_sel * TILE_L;
  return DSPS_OK;
}

// Workspace of dsps_eqw_pop: the SED call's, then the compact SED rows (and
// their tangent) of one batch.
static size_t eqw_pop_bytes(const SspView &v, int n_gal, int n_sel, bool tangent, Layout *out) {
  Layout L = make_layout(DSPS_OP_SED, v, 0, n_gal, DSPS_FP32);
  const size_t rows = align256(sizeof(float) * (size_t)L.batch * n_sel * TILE_L);
  L.ebuf = L.total;
  L.dbuf = L.total + rows;
  L.total += rows * (tangent ? 2 : 1);
  if (out) *out = L;
  return L.total;
}

extern "C" {

int dsps_eqw(const dsps_ssp *ssp, const float *sed, int n_gal, const dsps_line *lines, int n_line,
             float *eqw, hipStream_t stream) {
  return eqw_common(ssp, sed, nullptr, n_gal, lines, n_line, eqw, nullptr, stream);
}

int dsps_eqw_jvp(const dsps_ssp *ssp, const float *sed, const float *dsed, int n_gal,
                 const dsps_line *lines, int n_line, float *eqw, float *deqw, hipStream_t stream) {
  DSPS_CHECK(n_gal == 0 || (dsed && deqw), DSPS_ERR_ARG, "dsed or deqw is NULL");
  return eqw_common(ssp, sed, dsed, n_gal, lines, n_line, eqw, deqw, stream);
}

int dsps_eqw_pop_workspace(const dsps_ssp *ssp, int n_gal, const dsps_line *lines, int n_line,
                           int wrt, size_t *bytes) {
  DSPS_CHECK(bytes, DSPS_ERR_ARG, "bytes is NULL");
  DSPS_CHECK(n_gal >= 0, DSPS_ERR_SHAPE, "n_gal %d negative", n_gal);
  EqwLaunch a{};
  SedLaunch s{};
  DSPS_TRY(prepare_lines(ssp, lines, n_line, a));
  DSPS_TRY(select_chunks(a, s));
  *bytes = eqw_pop_bytes(ssp->v, n_gal, s.n_sel, wrt >= 0, nullptr);
  return DSPS_OK;
}

int dsps_eqw_pop(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                 int apply_dust, const dsps_line *lines, int n_line, int wrt, float *eqw,
                 float *deqw, void *workspace, size_t workspace_bytes, hipStream_t stream) {
  DSPS_CHECK(ssp, DSPS_ERR_ARG, "ssp is NULL");
  DSPS_TRY(check_cosmo(cosmo));
  DSPS_TRY(check_pop(pop, apply_dust != 0));
  DSPS_CHECK(apply_dust == 0 || apply_dust == 1, DSPS_ERR_ARG, "apply_dust must be 0 or 1");
  DSPS_CHECK(wrt >= -1 && wrt <= 1, DSPS_ERR_ARG, "wrt must be -1 (none), 0 (lgu) or 1 (sigma_u)");
  DSPS_CHECK(wrt < 0 || ssp->v.n_u > 1, DSPS_ERR_UNSUPPORTED, "the SSP block has no ionization axis");
  const bool age_dust = apply_dust && pop->av_old;
  DSPS_CHECK(!age_dust || (ssp->v.sa32 && ssp->v.n_u == 1), DSPS_ERR_UNSUPPORTED,
             "the age-dependent attenuation needs an SSP handle created with DSPS_SSP_AGE_MAJOR "
             "(and no ionization axis)");
  DSPS_TRY(check_precision(ssp, DSPS_FP32));
  DSPS_TRY(check_ion(ssp, pop));
  DSPS_CHECK(!pop->n_live, DSPS_ERR_UNSUPPORTED, "dsps_eqw_pop does not take a live count");
  EqwLaunch e{};
  SedLaunch s{};
  DSPS_TRY(prepare_lines(ssp, lines, n_line, e));
  DSPS_TRY(select_chunks(e, s));
  if (pop->n_gal == 0) return DSPS_OK;
  DSPS_CHECK(eqw && (wrt < 0 || deqw), DSPS_ERR_ARG, "eqw or deqw is NULL");
  DSPS_TRY(check_device(ssp->device));
  Layout L;
  DSPS_TRY(check_workspace(workspace, workspace_bytes,
                           eqw_pop_bytes(ssp->v, pop->n_gal, s.n_sel, wrt >= 0, &L)));
  char *ws = (char *)workspace;
  float *rows = (float *)(ws + L.ebuf), *drows = (float *)(ws + L.dbuf);
  DSPS_TRY(sort_population(ssp, pop, (int *)(ws + L.hist), (int *)(ws + L.perm), stream));
  for (int s0 = 0; s0 < pop->n_gal; s0 += L.batch) {
    const int cnt = std::min(L.batch, pop->n_gal - s0);
    DSPS_TRY(sed_batch_prepare(ssp, cosmo, pop, DSPS_FP32, age_dust, L, ws, s0, cnt, stream));
    SedLaunch b = sed_launch(ssp, pop, L, ws, DSPS_FP32, apply_dust, age_dust, s0, cnt);
    b.n_sel = s.n_sel;
    b.out_stride = s.out_stride;
    for (int x = 0; x < s.n_sel; ++x) b.chunk_list[x] = s.chunk_list[x];
    b.ion_tangent = 0;
    b.sed = rows;
    DSPS_TRY(launch_sed_gemm(b, stream));
    if (wrt >= 0) {
      b.ion_tangent = 1 + wrt;
      b.sed = drows;
      DSPS_TRY(launch_sed_gemm(b, stream));
    }
    // compact rows are in sorted order: row r is galaxy perm[s0 + r]
    e.sed = rows;
    e.dsed = wrt >= 0 ? drows : nullptr;
    e.sed_stride = s.out_stride;
    e.n_gal = cnt;
    e.perm = (const int *)(ws + L.perm);
    e.row_begin = s0;
    e.eqw = eqw;
    e.deqw = wrt >= 0 ? deqw : nullptr;
    DSPS_TRY(launch_eqw(e, stream));
  }
  return DSPS_OK;
}

static int check_summary(const float *mags, int n_gal, int n_band, int band_a, int band_b,
                         double colour_width, int band_m, const double *edges, int n_bins,
                         double mag_width) {
  DSPS_CHECK(n_gal >= 0, DSPS_ERR_SHAPE, "n_gal %d negative", n_gal);
  DSPS_CHECK(n_band >= 1 && n_band <= DSPS_MAX_BAND, DSPS_ERR_SHAPE, "n_band %d outside [1, %d]",
             n_band, DSPS_MAX_BAND);
  DSPS_CHECK(band_a >= 0 && band_a < n_band && band_b >= 0 && band_b < n_band && band_m >= 0 &&
                 band_m < n_band,
             DSPS_ERR_ARG, "band index outside [0, %d)", n_band);
  DSPS_CHECK(n_bins >= 1 && n_bins <= DSPS_MAX_SUMMARY_BINS, DSPS_ERR_SHAPE,
             "n_bins %d outside [1, %d]", n_bins, DSPS_MAX_SUMMARY_BINS);
  DSPS_CHECK(std::isfinite(colour_width) && colour_width >= 0.0 && std::isfinite(mag_width) &&
                 mag_width >= 0.0,
             DSPS_ERR_ARG, "widths must be finite and >= 0");
  DSPS_CHECK(edges, DSPS_ERR_ARG, "edges is NULL");
  DSPS_CHECK(n_gal == 0 || mags, DSPS_ERR_ARG, "mags is NULL");
  return DSPS_OK;
}

int dsps_pop_summary_workspace(int n_gal, int n_bins, size_t *bytes) {
  DSPS_CHECK(bytes, DSPS_ERR_ARG, "bytes is NULL");
  DSPS_CHECK(n_gal >= 0 && n_bins >= 1 && n_bins <= DSPS_MAX_SUMMARY_BINS, DSPS_ERR_SHAPE,
             "n_gal %d or n_bins %d out of range", n_gal, n_bins);
  const size_t blocks = ((size_t)n_gal + SUMMARY_CHUNK - 1) / SUMMARY_CHUNK;
  *bytes = align256(sizeof(double) * std::max<size_t>(blocks, 1) * n_bins);
  return DSPS_OK;
}

int dsps_pop_summary(const float *mags, int n_gal, int n_band, int band_a, int band_b,
                     double colour_cut, double colour_width, int band_m, const double *edges,
                     int n_bins, double mag_width, double *hist, void *workspace,
                     size_t workspace_bytes, hipStream_t stream) {
  DSPS_TRY(check_summary(mags, n_gal, n_band, band_a, band_b, colour_width, band_m, edges,
                         n_bins, mag_width));
  DSPS_CHECK(std::isfinite(colour_cut), DSPS_ERR_ARG, "colour_cut must be finite");
  DSPS_CHECK(hist, DSPS_ERR_ARG, "hist is NULL");
  size_t need = 0;
  DSPS_TRY(dsps_pop_summary_workspace(n_gal, n_bins, &need));
  DSPS_TRY(check_workspace(workspace, workspace_bytes, need));
  SummaryLaunch a{};
  a.mags = mags;
  a.n_gal = n_gal;
  a.n_band = n_band;
  a.band_a = band_a;
  a.band_b = band_b;
  a.band_m = band_m;
  a.cut = colour_cut;
  a.colour_width = colour_width;
  a.mag_width = mag_width;
  a.edges = edges;
  a.n_bins = n_bins;
  a.partial = (double *)workspace;
  a.hist = hist;
  return launch_summary(a, stream);
}

int dsps_pop_summary_vjp(const float *mags, int n_gal, int n_band, int band_a, int band_b,
                         double colour_cut, double colour_width, int band_m,
                         const double *edges, int n_bins, double mag_width,
                         const double *hist_bar, float *mags_bar, hipStream_t stream) {
  DSPS_TRY(check_summary(mags, n_gal, n_band, band_a, band_b, colour_width, band_m, edges,
                         n_bins, mag_width));
  DSPS_CHECK(std::isfinite(colour_cut), DSPS_ERR_ARG, "colour_cut must be finite");
  if (n_gal == 0) return DSPS_OK;
  DSPS_CHECK(hist_bar && mags_bar, DSPS_ERR_ARG, "hist_bar or mags_bar is NULL");
  SummaryLaunch a{};
  a.mags = mags;
  a.n_gal = n_gal;
  a.n_band = n_band;
  a.band_a = band_a;
  a.band_b = band_b;
  a.band_m = band_m;
  a.cut = colour_cut;
  a.colour_width = colour_width;
  a.mag_width = mag_width;
  a.edges = edges;
  a.n_bins = n_bins;
  a.hist_bar = hist_bar;
  a.mags_bar = mags_bar;
  return launch_summary_vjp(a, stream);
}

}  // extern "C"
