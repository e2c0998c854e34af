// Second-order-cone arithmetic of one cone held by one lane (dim d <= SOC_DMAX):
// Nesterov-Todd scaling, spectral application of H and (H + delta I)^-1 and
// the combined-step d_s.  Shared by the per-family kernels (hc_cones.hip) and
// the wave-per-problem engine (hc_wave.hip).
#pragma once
#include "hc_common.h"

namespace hc {

struct SocSpec {
  double r, lp, lm, lo;   // |wbar_1|, eigenvalues eta^2 (w0 + r)^2, eta^2/(w0 + r)^2, eta^2
};

__device__ __forceinline__ SocSpec soc_spec(const double* wb, int d, double eta) {
  double r2 = 0;
  for (int j = 1; j < d; ++j) r2 += wb[j] * wb[j];
  SocSpec sp;
  sp.r = sqrt(r2);
  const double big = wb[0] + sp.r;
  const double e2 = eta * eta;
  sp.lp = e2 * big * big;
  sp.lm = e2 / (big * big);
  sp.lo = e2;
  return sp;
}

// y = V f(lam) V' x with V = [(1,u)/sqrt2, (1,-u)/sqrt2, perp]; f given as three values
__device__ __forceinline__ void soc_spec_apply(const double* wb, int d, const SocSpec& sp, double fp, double fm, double fo,
                                      const double* x, double* y) {
  const double is2 = 0.70710678118654752440;
  double u[SOC_DMAX];
  if (sp.r > 0.0) {
    for (int j = 1; j < d; ++j) u[j] = wb[j] / sp.r;
  } else {
    for (int j = 1; j < d; ++j) u[j] = (j == 1) ? 1.0 : 0.0;
  }
  double ux = 0;
  for (int j = 1; j < d; ++j) ux += u[j] * x[j];
  const double ap = (x[0] + ux) * is2, am = (x[0] - ux) * is2;
  y[0] = (fp * ap + fm * am) * is2;
  const double cu = (fp * ap - fm * am) * is2;
  for (int j = 1; j < d; ++j) y[j] = cu * u[j] + fo * (x[j] - u[j] * ux);
}


// Nesterov-Todd scaling point of s, z in int K (Appendix A, symmetric cones):
// wbar (normalised, wbar'J wbar = 1), lambda = W z = W^-T s; returns eta
__device__ __forceinline__ double soc_nt_scale(const double* sv, const double* zv, int d, double* wb, double* lam) {
  double sJs = sv[0] * sv[0], zJz = zv[0] * zv[0];
  for (int j = 1; j < d; ++j) {
    sJs -= sv[j] * sv[j];
    zJz -= zv[j] * zv[j];
  }
  const double ns = sqrt(sJs), nz = sqrt(zJz);
  double sz = 0;
  for (int j = 0; j < d; ++j) sz += (sv[j] / ns) * (zv[j] / nz);
  const double gamma = sqrt((1.0 + sz) / 2.0);
  for (int j = 0; j < d; ++j) wb[j] = (sv[j] / ns + (j == 0 ? 1.0 : -1.0) * (zv[j] / nz)) / (2.0 * gamma);
  const double eta = sqrt(ns / nz);
  // lambda = W z = eta Wbar z
  double w1z1 = 0;
  for (int j = 1; j < d; ++j) w1z1 += wb[j] * zv[j];
  lam[0] = eta * (wb[0] * zv[0] + w1z1);
  const double cf = zv[0] + w1z1 / (1.0 + wb[0]);
  for (int j = 1; j < d; ++j) lam[j] = eta * (zv[j] + cf * wb[j]);
  return eta;
}

// combined-step d_s of one cone (eq. ds-correction-step):
// x = W' (lam \ (lam o lam + (W^-T ds_a) o (W dz_a) - sm e))
__device__ __forceinline__ void soc_ds_one(const double* wb, double eta, const double* lam, const double* a,
                                       const double* b, int d, double sm, double* out) {
  // W^-T ds = W^-1 ds = eta^-1 J Wbar J ds ; W dz = eta Wbar dz
  double Ja[SOC_DMAX], p[SOC_DMAX], q[SOC_DMAX];
  for (int j = 0; j < d; ++j) Ja[j] = (j == 0) ? a[0] : -a[j];
  double w1a = 0, w1b = 0;
  for (int j = 1; j < d; ++j) {
    w1a += wb[j] * Ja[j];
    w1b += wb[j] * b[j];
  }
  p[0] = (wb[0] * Ja[0] + w1a) / eta;
  const double cfa = Ja[0] + w1a / (1.0 + wb[0]);
  for (int j = 1; j < d; ++j) p[j] = -(Ja[j] + cfa * wb[j]) / eta;   // J applied after Wbar
  q[0] = eta * (wb[0] * b[0] + w1b);
  const double cfb = b[0] + w1b / (1.0 + wb[0]);
  for (int j = 1; j < d; ++j) q[j] = eta * (b[j] + cfb * wb[j]);
  // v = lam o lam + p o q - sm e
  double v[SOC_DMAX];
  double ll = 0, pq = 0;
  for (int j = 0; j < d; ++j) {
    ll += lam[j] * lam[j];
    pq += p[j] * q[j];
  }
  v[0] = ll + pq - sm;
  for (int j = 1; j < d; ++j) v[j] = 2.0 * lam[0] * lam[j] + p[0] * q[j] + q[0] * p[j];
  // x = lam \ v
  double lJl = lam[0] * lam[0], l1v1 = 0;
  for (int j = 1; j < d; ++j) {
    lJl -= lam[j] * lam[j];
    l1v1 += lam[j] * v[j];
  }
  double x[SOC_DMAX];
  x[0] = (lam[0] * v[0] - l1v1) / lJl;
  for (int j = 1; j < d; ++j) x[j] = (v[j] - x[0] * lam[j]) / lam[0];
  // ds = W' x = eta Wbar x
  double w1x = 0;
  for (int j = 1; j < d; ++j) w1x += wb[j] * x[j];
  out[0] = eta * (wb[0] * x[0] + w1x);
  const double cfx = x[0] + w1x / (1.0 + wb[0]);
  for (int j = 1; j < d; ++j) out[j] = eta * (x[j] + cfx * wb[j]);
}

}  // namespace hc
