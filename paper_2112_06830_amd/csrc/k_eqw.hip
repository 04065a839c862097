// Emission-line equivalent widths of rest-frame SEDs (Section 2.2.2, Eq. eqw).
//
// For each line the continuum is the least-squares quadratic in
// x = (lambda - centre) / fit_half_width over the neighbourhood's grid points
// outside the line window.  Its normal matrix depends on the grid only, so the
// host inverts it once per line; a galaxy needs the three moments
// sum L_n x_n^p of its own SED, then c = G^-1 b.  The width is the trapezoid
// rule of (L - L_0) / L_0 over the line window's grid points.  One wave64 per
// galaxy walks every line (the SED row stays in cache); sums run in float64
// and are reduced across the wave in a fixed order.
//
// With a tangent dL of the SED the kernel also returns the widths' tangent:
// the fit is linear, so dL_0 is the same fit of dL, and the ratio's
// derivative is (dL L_0 - L dL_0) / L_0^2.
#include "dsps_internal.hpp"

namespace dsps {

// Coefficients c = G^-1 b of the quadratic continuum from the lane-partial
// moments b (reduced across the wave here); G^-1 is stored as its upper
// triangle (00, 01, 02, 11, 12, 22).
__device__ __forceinline__ void fit_quadratic(const double *q, double (&b)[3], double (&c)[3]) {
#pragma unroll
  for (int p = 0; p < 3; ++p) b[p] = wave_sum(b[p]);
  c[0] = q[0] * b[0] + q[1] * b[1] + q[2] * b[2];
  c[1] = q[1] * b[0] + q[3] * b[1] + q[4] * b[2];
  c[2] = q[2] * b[0] + q[4] * b[1] + q[5] * b[2];
}

__global__ __launch_bounds__(256) void k_eqw(EqwLaunch a) {
  const int lane = threadIdx.x & 63;
  const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (g >= a.n_gal) return;   // whole waves leave together
  const bool tangent = a.dsed != nullptr;
  for (int li = 0; li < a.n_line; ++li) {
    const EqwLine &ln = a.line[li];
    // grid point n sits at row[n + off] (off is 0 for full rows)
    const float *row = a.sed + (size_t)g * a.sed_stride;
    const float *drow = tangent ? a.dsed + (size_t)g * a.sed_stride : row;
    const int off = ln.sed_off;
    // moments of the SED (and of its tangent) over the continuum points
    double b[3] = {0.0, 0.0, 0.0}, db[3] = {0.0, 0.0, 0.0};
    for (int n = ln.f0 + lane; n < ln.f1; n += 64) {
      if (n >= ln.m0 && n < ln.m1) continue;
      const double x = (a.wave[n] - ln.centre) * ln.inv_fit;
      const double v = (double)row[n + off], dv = (double)drow[n + off];
      b[0] += v;
      b[1] += v * x;
      b[2] += v * x * x;
      db[0] += dv;
      db[1] += dv * x;
      db[2] += dv * x * x;
    }
    double c[3], dc[3];
    fit_quadratic(ln.ginv, b, c);
    if (tangent) fit_quadratic(ln.ginv, db, dc);
    // trapezoid over the window's intervals [n, n + 1]
    double s = 0.0, ds = 0.0;
    for (int n = ln.m0 + lane; n + 1 < ln.m1; n += 64) {
      const double l0 = a.wave[n], l1 = a.wave[n + 1];
      const double x0 = (l0 - ln.centre) * ln.inv_fit, x1 = (l1 - ln.centre) * ln.inv_fit;
      const double k0 = c[0] + c[1] * x0 + c[2] * x0 * x0;
      const double k1 = c[0] + c[1] * x1 + c[2] * x1 * x1;
      const double v0 = (double)row[n + off], v1 = (double)row[n + 1 + off];
      s += 0.5 * ((v0 - k0) / k0 + (v1 - k1) / k1) * (l1 - l0);
      if (tangent) {
        const double dk0 = dc[0] + dc[1] * x0 + dc[2] * x0 * x0;
        const double dk1 = dc[0] + dc[1] * x1 + dc[2] * x1 * x1;
        const double r0 = ((double)drow[n + off] * k0 - v0 * dk0) / (k0 * k0);
        const double r1 = ((double)drow[n + 1 + off] * k1 - v1 * dk1) / (k1 * k1);
        ds += 0.5 * (r0 + r1) * (l1 - l0);
      }
    }
    s = wave_sum(s);
    const size_t go = a.perm ? (size_t)a.perm[a.row_begin + g] : (size_t)g;   // output galaxy
    if (lane == 0) a.eqw[go * a.n_line + li] = (float)s;
    if (tangent) {
      ds = wave_sum(ds);
      if (lane == 0) a.deqw[go * a.n_line + li] = (float)ds;
    }
  }
}

int launch_eqw(const EqwLaunch &a, hipStream_t stream) {
  if (a.n_gal <= 0) return DSPS_OK;
  ProfScope prof(DSPS_KERNEL_EQW, stream);
  hipLaunchKernelGGL(k_eqw, dim3((a.n_gal + 3) / 4), dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "k_eqw launch");
}

}  // namespace dsps
