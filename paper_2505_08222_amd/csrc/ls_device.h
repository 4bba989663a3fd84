// Range-only least-squares localisation of one target from one tracker's
// window, device side (arXiv 2505.08222, Sec. III-A: the squared-range
// equations linearised by least squares). Shared by the environment
// kernels and the batched estimator kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace mil {

// Linearised least squares over the present entries of one tracker's window,
// in FP64, followed by gn_iters Gauss-Newton steps on sum (|p-a_k| - r_k)^2
// (a step is kept only if it lowers the cost). NaN ranges are missing.
template <int WC, typename T = float>
__device__ __forceinline__ bool ls_masked(const T (&hx)[WC], const T (&hy)[WC],
                                          const T (&hr)[WC], int filled, int gn_iters,
                                          double tau, double &px, double &py) {
  int n = 0;
  double mx = 0.0, my = 0.0, mr = 0.0;
#pragma unroll
  for (int k = 0; k < WC; ++k) {
    if (k < filled && hr[k] == hr[k]) {
      ++n;
      mx += (double)hx[k];
      my += (double)hy[k];
      mr += (double)hr[k];
    }
  }
  if (n < 3) return false;
  const double invn = 1.0 / (double)n;
  mx *= invn;
  my *= invn;
  mr *= invn;
  double sxx = 0.0, sxy = 0.0, syy = 0.0, gx = 0.0, gy = 0.0;
#pragma unroll
  for (int k = 0; k < WC; ++k) {
    if (k < filled && hr[k] == hr[k]) {
      const double ux = (double)hx[k] - mx, uy = (double)hy[k] - my;
      const double d = (double)hr[k] - mr;
      const double c = fma(-d, fma(2.0, mr, d), fma(ux, ux, uy * uy));
      sxx = fma(ux, ux, sxx);
      sxy = fma(ux, uy, sxy);
      syy = fma(uy, uy, syy);
      gx = fma(ux, c, gx);
      gy = fma(uy, c, gy);
    }
  }
  const double det = sxx * syy - sxy * sxy, tr = sxx + syy;
  if (!(det > tau * tr * tr)) return false;
  const double h = 0.5 / det;
  double x = mx + h * (syy * gx - sxy * gy);
  double y = my + h * (sxx * gy - sxy * gx);
  for (int it = 0; it < gn_iters; ++it) {
    double hxx = 0.0, hxy = 0.0, hyy = 0.0, bx = 0.0, by = 0.0, j0 = 0.0;
#pragma unroll
    for (int k = 0; k < WC; ++k) {
      if (k < filled && hr[k] == hr[k]) {
        const double dx = x - (double)hx[k], dy = y - (double)hy[k];
        const double dist = sqrt(dx * dx + dy * dy);
        const double rho = dist - (double)hr[k];
        j0 += rho * rho;
        if (dist > 0.0) {
          const double jx = dx / dist, jy = dy / dist;
          hxx += jx * jx;
          hxy += jx * jy;
          hyy += jy * jy;
          bx += jx * rho;
          by += jy * rho;
        }
      }
    }
    const double dh = hxx * hyy - hxy * hxy, th = hxx + hyy;
    if (!(dh > tau * th * th)) break;
    const double sx = -(hyy * bx - hxy * by) / dh;
    const double sy = -(hxx * by - hxy * bx) / dh;
    double j1 = 0.0;
#pragma unroll
    for (int k = 0; k < WC; ++k) {
      if (k < filled && hr[k] == hr[k]) {
        const double dx = x + sx - (double)hx[k], dy = y + sy - (double)hy[k];
        const double rho = sqrt(dx * dx + dy * dy) - (double)hr[k];
        j1 += rho * rho;
      }
    }
    if (!(j1 < j0)) break;
    x += sx;
    y += sy;
  }
  px = x;
  py = y;
  return true;
}

}  // namespace mil
