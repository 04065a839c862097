// Host-side check of the C ABI, built with the address and undefined-behaviour
// sanitizers on the host code only (device code is compiled as usual): handle
// creation and destruction, workspace sizing, every compute entry point on a
// small synthetic population (with and without a device-side live count), the
// argument checks that must fail before any launch, and the error strings.
// The sanitizers abort the process on the first host-side memory or UB error;
// the program prints "host check passed" and exits 0 otherwise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>

#include "dsps.h"

#define CHECK(cond, ...)                                        \
  do {                                                          \
    if (!(cond)) {                                              \
      std::fprintf(stderr, "host check failed at line %d: ", __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                        \
      std::fprintf(stderr, " [%s]\n", dsps_last_error());       \
      std::exit(1);                                             \
    }                                                           \
  } while (0)
#define OK(call) CHECK((call) == DSPS_OK, "%s", #call)

template <typename T>
static T *dev_copy(const std::vector<T> &h) {
  T *d = nullptr;
  CHECK(hipMalloc(&d, h.size() * sizeof(T)) == hipSuccess, "hipMalloc");
  CHECK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess, "copy");
  return d;
}
template <typename T>
static T *dev_alloc(size_t n) {
  T *d = nullptr;
  CHECK(hipMalloc(&d, n * sizeof(T)) == hipSuccess, "hipMalloc");
  return d;
}
template <typename T>
static std::vector<T> host_copy(const T *d, size_t n) {
  std::vector<T> h(n);
  CHECK(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost) == hipSuccess, "copy back");
  return h;
}

int main() {
  CHECK(dsps_abi_version() == DSPS_ABI_VERSION, "ABI version");
  // ---- a small SSP block: smooth positive spectra on a 5 x 12 x 800 grid
  const int n_met = 5, n_age = 12, n_wave = 800, n_band = 3, n_pts = 64;
  std::vector<double> lgz(n_met), lg_age(n_age), wave(n_wave);
  for (int j = 0; j < n_met; ++j) lgz[j] = -3.5 + 0.4 * j;
  for (int i = 0; i < n_age; ++i) lg_age[i] = 6.0 + 0.35 * i;
  for (int l = 0; l < n_wave; ++l) wave[l] = 1000.0 * std::pow(20.0, l / (double)(n_wave - 1));
  std::vector<float> lum((size_t)n_met * n_age * n_wave);
  for (int j = 0; j < n_met; ++j)
    for (int i = 0; i < n_age; ++i)
      for (int l = 0; l < n_wave; ++l)
        lum[((size_t)j * n_age + i) * n_wave + l] =
            (float)(1e-6 * std::exp(-0.3 * i) * (1.0 + 0.1 * j) *
                    (1.0 + 0.5 * std::sin(3e-4 * wave[l] + i)));
  dsps_ssp *ssp = nullptr;
  OK(dsps_ssp_create(n_met, n_age, n_wave, lgz.data(), lg_age.data(), wave.data(), lum.data(),
                     (1 << DSPS_FP32) | (1 << DSPS_BF16) | DSPS_SSP_AGE_MAJOR, 0, &ssp));
  // ---- three triangular-ish filters between 3000 and 12000 Angstrom
  std::vector<double> fw((size_t)n_band * n_pts), ft((size_t)n_band * n_pts);
  for (int b = 0; b < n_band; ++b)
    for (int k = 0; k < n_pts; ++k) {
      const double x = k / (double)(n_pts - 1);
      fw[(size_t)b * n_pts + k] = 3000.0 + 2500.0 * b + 3000.0 * x;
      ft[(size_t)b * n_pts + k] = std::sin(M_PI * x);
    }
  dsps_filters *flt = nullptr;
  OK(dsps_filters_create(n_band, n_pts, fw.data(), ft.data(), &flt));

  // ---- a population of 300 galaxies with parametric histories
  const int n = 300, n_t = 50;
  std::vector<double> tt(n_t), par((size_t)5 * n);
  for (int k = 0; k < n_t; ++k) tt[k] = 0.05 + 13.7 * k / (n_t - 1.0);
  std::vector<float> z(n), lgmet(n), sig(n), av(n), delta(n), bump(n), tgt((size_t)n * n_band),
      av_old(n), delta_old(n);
  for (int g = 0; g < n; ++g) {
    par[g] = 1.0 + g % 7;
    par[n + g] = 2.0 + 0.01 * g;
    par[2 * n + g] = 1.5;
    par[3 * n + g] = 0.3;
    par[4 * n + g] = 9.0;
    z[g] = 0.1f + 1.5f * (float)g / n;
    lgmet[g] = -2.6f + 0.002f * (float)g;
    sig[g] = 0.3f;
    av[g] = 0.5f;
    delta[g] = -0.2f;
    bump[g] = 1.0f;
    av_old[g] = 0.2f;
    delta_old[g] = -0.1f;
    for (int b = 0; b < n_band; ++b) tgt[(size_t)g * n_band + b] = 22.0f;
  }
  dsps_pop pop{};
  pop.n_gal = n;
  pop.n_t = n_t;
  pop.t_table = dev_copy(tt);
  pop.sfh_params = dev_copy(par);
  pop.z = dev_copy(z);
  pop.lgmet = dev_copy(lgmet);
  pop.sigma_z = dev_copy(sig);
  pop.av = dev_copy(av);
  pop.delta = dev_copy(delta);
  pop.bump = dev_copy(bump);
  pop.lgmet_slope = 0.1;
  pop.lg_age_pivot = 9.0;
  pop.mdf_width = 0.5;
  pop.dust_pivot = 7.0;
  pop.dust_width = 0.25;
  const dsps_cosmo cosmo{0.3, -1.0, 0.7};

  size_t ws_bytes = 0;
  OK(dsps_workspace_size(DSPS_OP_MAGS_VJP, ssp, flt, n, n_t, DSPS_FP32, &ws_bytes));
  size_t ws2 = 0;
  OK(dsps_workspace_size(DSPS_OP_MAGS, ssp, flt, n, n_t, DSPS_BF16, &ws2));
  ws_bytes = std::max(ws_bytes, ws2);
  OK(dsps_workspace_size(DSPS_OP_SED, ssp, nullptr, n, n_t, DSPS_FP32, &ws2));
  ws_bytes = std::max(ws_bytes, ws2);
  void *ws = dev_alloc<char>(ws_bytes);

  float *mags = dev_alloc<float>((size_t)n * n_band);
  float *bands = dev_alloc<float>((size_t)n * 2 * n_band);
  float *mom = dev_alloc<float>((size_t)n * 3 * n_band);
  float *mags2 = dev_alloc<float>((size_t)n * n_band);
  float *w = dev_alloc<float>((size_t)n * n_met * n_age);
  double *mstar = dev_alloc<double>(n);
  float *sed = dev_alloc<float>((size_t)n * n_wave);
  double *par_bar = dev_alloc<double>((size_t)5 * n);
  float *g32 = dev_alloc<float>((size_t)5 * n);
  float *tgt_d = dev_copy(tgt);

  // ---- every compute entry point once
  OK(dsps_weights(ssp, &cosmo, &pop, w, mstar, ws, ws_bytes, nullptr));
  OK(dsps_sed(ssp, &cosmo, &pop, 1, DSPS_FP32, sed, ws, ws_bytes, nullptr));
  OK(dsps_mags(ssp, flt, &cosmo, &pop, DSPS_BF16, mags, nullptr, nullptr, ws, ws_bytes, nullptr));
  OK(dsps_mags(ssp, flt, &cosmo, &pop, DSPS_FP32, mags, bands, mom, ws, ws_bytes, nullptr));
  OK(dsps_mags_noalloc(ssp, flt, &cosmo, &pop, DSPS_FP32, mags2, nullptr, nullptr, nullptr));
  OK(dsps_mags_vjp(ssp, flt, &cosmo, &pop, DSPS_FP32, tgt_d, bands, mom, nullptr, par_bar, g32,
                   nullptr, g32 + n, g32 + 2 * n, g32 + 3 * n, g32 + 4 * n, nullptr, nullptr,
                   nullptr, nullptr, ws, ws_bytes, nullptr));
  OK(dsps_mags_residual_vjp(ssp, flt, &cosmo, &pop, tgt_d, nullptr, mags2, nullptr, par_bar, g32,
                            nullptr, g32 + n, g32 + 2 * n, g32 + 3 * n, g32 + 4 * n, nullptr,
                            nullptr, nullptr, nullptr, ws, ws_bytes, nullptr));
  CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
  {
    const std::vector<float> a = host_copy(mags, (size_t)n * n_band);
    const std::vector<float> b = host_copy(mags2, (size_t)n * n_band);
    for (size_t i = 0; i < a.size(); ++i) {
      CHECK(std::isfinite(a[i]), "finite magnitude %zu", i);
      CHECK(a[i] == b[i], "residual call magnitude %zu differs", i);
    }
    const std::vector<double> pb = host_copy(par_bar, (size_t)5 * n);
    for (double v : pb) CHECK(std::isfinite(v), "finite gradient");
  }
  // the age-dependent attenuation on the age-major table
  float *av_old_d = dev_copy(av_old), *delta_old_d = dev_copy(delta_old);
  pop.av_old = av_old_d;
  pop.delta_old = delta_old_d;
  OK(dsps_mags(ssp, flt, &cosmo, &pop, DSPS_FP32, mags, nullptr, nullptr, ws, ws_bytes, nullptr));
  pop.av_old = nullptr;
  pop.delta_old = nullptr;

  // ---- a device-side live count: rows past it are left as they were
  int *live = dev_copy(std::vector<int>{171});
  pop.n_live = live;
  CHECK(hipMemset(mags, 0, (size_t)n * n_band * sizeof(float)) == hipSuccess, "memset");
  OK(dsps_mags(ssp, flt, &cosmo, &pop, DSPS_FP32, mags, nullptr, nullptr, ws, ws_bytes, nullptr));
  CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
  {
    const std::vector<float> a = host_copy(mags, (size_t)n * n_band);
    for (int g = 171; g < n; ++g)
      for (int b = 0; b < n_band; ++b) CHECK(a[(size_t)g * n_band + b] == 0.0f, "padding row written");
  }
  pop.n_live = nullptr;

  // ---- checks that must fail before any launch, with a message
  CHECK(dsps_mags(nullptr, flt, &cosmo, &pop, DSPS_FP32, mags, nullptr, nullptr, ws, ws_bytes,
                  nullptr) == DSPS_ERR_ARG, "null ssp");
  CHECK(std::strlen(dsps_last_error()) > 0, "error string");
  CHECK(dsps_mags(ssp, flt, &cosmo, &pop, 7, mags, nullptr, nullptr, ws, ws_bytes, nullptr) != DSPS_OK,
        "bad precision");
  CHECK(dsps_mags(ssp, flt, &cosmo, &pop, DSPS_FP32, mags, nullptr, nullptr, ws, 16, nullptr) ==
            DSPS_ERR_WORKSPACE, "short workspace");
  dsps_pop bad = pop;
  bad.sigma_z = nullptr;
  CHECK(dsps_mags(ssp, flt, &cosmo, &bad, DSPS_FP32, mags, nullptr, nullptr, ws, ws_bytes,
                  nullptr) != DSPS_OK, "missing sigma_z");
  bad = pop;
  bad.n_t = 1;
  CHECK(dsps_weights(ssp, &cosmo, &bad, w, nullptr, ws, ws_bytes, nullptr) != DSPS_OK, "n_t = 1");
  const dsps_cosmo bad_cosmo{0.0, -1.0, 0.7};
  CHECK(dsps_mags(ssp, flt, &bad_cosmo, &pop, DSPS_FP32, mags, nullptr, nullptr, ws, ws_bytes,
                  nullptr) != DSPS_OK, "om0 = 0");
  CHECK(dsps_mags_residual_vjp(ssp, flt, &cosmo, &pop, nullptr, nullptr, mags, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, ws, ws_bytes, nullptr) == DSPS_ERR_ARG,
        "null target");
  dsps_ssp *bad_ssp = nullptr;
  std::vector<double> lgz_bad = lgz;
  lgz_bad[2] = lgz_bad[1];   // not strictly ascending
  CHECK(dsps_ssp_create(n_met, n_age, n_wave, lgz_bad.data(), lg_age.data(), wave.data(),
                        lum.data(), 1 << DSPS_FP32, 0, &bad_ssp) != DSPS_OK && bad_ssp == nullptr,
        "non-ascending metallicities");
  pop.n_gal = 0;
  OK(dsps_mags(ssp, flt, &cosmo, &pop, DSPS_FP32, mags, nullptr, nullptr, ws, ws_bytes, nullptr));

  // ---- teardown
  for (const void *p : {(const void *)pop.t_table, (const void *)pop.sfh_params, (const void *)pop.z,
                        (const void *)pop.lgmet, (const void *)pop.sigma_z, (const void *)pop.av,
                        (const void *)pop.delta, (const void *)pop.bump, (const void *)ws,
                        (const void *)mags, (const void *)bands, (const void *)mom,
                        (const void *)mags2, (const void *)w, (const void *)mstar,
                        (const void *)sed, (const void *)par_bar, (const void *)g32,
                        (const void *)tgt_d, (const void *)live, (const void *)av_old_d,
                        (const void *)delta_old_d})
    CHECK(hipFree(const_cast<void *>(p)) == hipSuccess, "hipFree");
  dsps_filters_destroy(flt);
  dsps_ssp_destroy(ssp);
  std::printf("host check passed\n");
  return 0;
}
