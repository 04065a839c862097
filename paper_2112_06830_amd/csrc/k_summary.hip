// Population summary of the Section 4.1 forward model: a red-colour cut and
// a histogram of one band's magnitude, smoothed with the triweight kernel of
// Appendix B (Eqs. triweight, terf) so that gradients reach every galaxy.
//
//   w_g    = T_erf((c_g - cut) / s_c),   c_g = m_a - m_b
//   B_k(m) = T_erf((e_{k+1} - m) / s_m) - T_erf((e_k - m) / s_m)
//   H_k    = sum_g w_g B_k(m_g)
//
// Zero widths select the hard cut and the plain histogram.  The forward pass
// is deterministic: each workgroup stages SUMMARY_CHUNK galaxies in LDS and
// one thread per bin sums them in order (float64); the partials are then
// added in workgroup order.  The adjoint runs one thread per galaxy over the
// bins within three widths of its magnitude.
#include "dsps_internal.hpp"

namespace dsps {

struct GalaxyInput {
  double c, m;
  bool ok;
};

__device__ __forceinline__ GalaxyInput summary_input(const SummaryLaunch &a, int g) {
  const float *row = a.mags + (size_t)g * a.n_band;
  GalaxyInput in;
  in.c = (double)row[a.band_a] - (double)row[a.band_b];
  in.m = (double)row[a.band_m];
  in.ok = isfinite(in.c) && isfinite(in.m);
  return in;
}

__device__ __forceinline__ double colour_weight(const SummaryLaunch &a, double c) {
  if (a.colour_width == 0.0) return c > a.cut ? 1.0 : 0.0;
  return triweight_cdf((c - a.cut) / a.colour_width);
}

__global__ __launch_bounds__(256) void k_summary_partial(SummaryLaunch a) {
  __shared__ double s_m[SUMMARY_CHUNK];
  __shared__ double s_w[SUMMARY_CHUNK];
  extern __shared__ double s_e[];                   // [n_bins + 1]
  const int g0 = blockIdx.x * SUMMARY_CHUNK;
  const int cnt = min(SUMMARY_CHUNK, a.n_gal - g0);
  for (int i = threadIdx.x; i <= a.n_bins; i += blockDim.x) s_e[i] = a.edges[i];
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const GalaxyInput in = summary_input(a, g0 + i);
    s_w[i] = in.ok ? colour_weight(a, in.c) : 0.0;
    s_m[i] = in.ok ? in.m : 0.0;
  }
  __syncthreads();
  const int last = a.n_bins - 1;
  for (int k = threadIdx.x; k < a.n_bins; k += blockDim.x) {
    const double lo = s_e[k], hi = s_e[k + 1];
    double acc = 0.0;
    if (a.mag_width == 0.0) {
      for (int i = 0; i < cnt; ++i) {
        const double m = s_m[i];
        if (m >= lo && (m < hi || (k == last && m == hi))) acc += s_w[i];
      }
    } else {
      const double inv = 1.0 / a.mag_width;
      for (int i = 0; i < cnt; ++i) {
        const double w = s_w[i];
        if (w == 0.0) continue;                     // adds an exact zero
        const double m = s_m[i];
        acc += w * (triweight_cdf((hi - m) * inv) - triweight_cdf((lo - m) * inv));
      }
    }
    a.partial[(size_t)blockIdx.x * a.n_bins + k] = acc;
  }
}

__global__ void k_summary_reduce(SummaryLaunch a, int n_blocks) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_bins) return;
  double acc = 0.0;
  for (int b = 0; b < n_blocks; ++b) acc += a.partial[(size_t)b * a.n_bins + k];
  a.hist[k] = acc;
}

int launch_summary(const SummaryLaunch &a, hipStream_t stream) {
  const int n_blocks = (a.n_gal + SUMMARY_CHUNK - 1) / SUMMARY_CHUNK;
  ProfScope prof(DSPS_KERNEL_SUMMARY, stream);
  if (n_blocks > 0) {
    const size_t lds = sizeof(double) * (a.n_bins + 1);
    hipLaunchKernelGGL(k_summary_partial, dim3(n_blocks), dim3(256), lds, stream, a);
  }
  hipLaunchKernelGGL(k_summary_reduce, dim3((a.n_bins + 255) / 256), dim3(256), 0, stream, a,
                     n_blocks);
  return hip_fail(hipGetLastError(), "population summary launch");
}

// d(sum_k hbar_k H_k)/d m: the weight's derivative goes to bands a (+) and b
// (-), the membership's to band_m; accumulated per band in that order.
__global__ __launch_bounds__(256) void k_summary_vjp(SummaryLaunch a) {
  extern __shared__ double s_e[];                   // [n_bins + 1] edges, then hist_bar
  double *s_hb = s_e + a.n_bins + 1;
  for (int i = threadIdx.x; i <= a.n_bins; i += blockDim.x) s_e[i] = a.edges[i];
  for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x) s_hb[i] = a.hist_bar[i];
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.n_gal) return;
  float *out = a.mags_bar + (size_t)g * a.n_band;
  const GalaxyInput in = summary_input(a, g);
  double g_a = 0.0, g_m = 0.0;                      // d/dc (times dw/dc) and d/dm
  if (in.ok && a.colour_width > 0.0 && a.mag_width > 0.0) {
    const double t = (in.c - a.cut) / a.colour_width;
    const double w = triweight_cdf(t);
    const double dw = triweight_pdf(t) / a.colour_width;
    const double inv = 1.0 / a.mag_width;
    const double reach = 3.0 * a.mag_width;
    // first bin whose upper edge lies above m - 3 s_m
    int lo = 0, hi = a.n_bins;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_e[mid + 1] > in.m - reach) hi = mid; else lo = mid + 1;
    }
    double gw = 0.0, gm = 0.0;
    for (int k = lo; k < a.n_bins && s_e[k] < in.m + reach; ++k) {
      const double u1 = (s_e[k + 1] - in.m) * inv, u0 = (s_e[k] - in.m) * inv;
      gw += s_hb[k] * (triweight_cdf(u1) - triweight_cdf(u0));
      gm += s_hb[k] * (triweight_pdf(u0) - triweight_pdf(u1)) * inv;
    }
    g_a = gw * dw;
    g_m = w * gm;
  }
  for (int b = 0; b < a.n_band; ++b) {
    double v = 0.0;
    if (b == a.band_a) v += g_a;
    if (b == a.band_b) v -= g_a;
    if (b == a.band_m) v += g_m;
    out[b] = (float)v;
  }
}

int launch_summary_vjp(const SummaryLaunch &a, hipStream_t stream) {
  if (a.n_gal <= 0) return DSPS_OK;
  const size_t lds = sizeof(double) * (2 * a.n_bins + 1);
  hipLaunchKernelGGL(k_summary_vjp, dim3((a.n_gal + 255) / 256), dim3(256), lds, stream, a);
  return hip_fail(hipGetLastError(), "population summary adjoint launch");
}

}  // namespace dsps
