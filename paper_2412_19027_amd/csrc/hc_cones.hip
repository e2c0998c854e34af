// Cone layer of the IPM on gfx950 (Sec. 3.3 mixed parallel computing strategy,
// Algorithm 2; scalings of Appendix A; corrections of eq. ds-correction-step).
//
// Mapping: zero and nonnegative rows are plain vector ops (one lane per row);
// every other family runs one lane per cone with the cone's components stored
// component-major (row base + j*count + i), so each component load of a wave is
// one coalesced 512-byte access.  Second-order cones above 16 rows run one
// workgroup per cone (hc_soc.hip).  PSD cones (sides up to 32) run one wave
// per cone for the scaling, d_s correction, step, initial shift and spectral
// apply (parallel Jacobi, products split by output entry), and one lane per
// (cone, svec entry) for the explicit (H + delta I)^-1 block.
//
// Scalings are kept in spectral form H = V diag(lam) V': near the optimum
// cond(H) exceeds 1/eps, and applying H or (H + delta I)^-1 through the
// eigenpairs keeps each spectral component to relative accuracy.
//   nonneg: h = s/z.
//   SOC:    NT point wbar, eta; eigenpairs (1, +-u)/sqrt2 with eta^2 (w0 +- r)^2
//           (the small one as eta^2/(w0 + r)^2), eta^2 on the rest.
//   exp/pow: Hess f = G G' with G built from rank-one PSD pieces; a one-sided
//           Jacobi SVD of G gives Hess f^-1; the primal-dual (BFGS) scaling is
//           the Gram matrix of [s/sqrt<s,z>, ds/sqrt<ds,dz>, u sqrt(mu/u'Hf^-1 u)],
//           the dual scaling is mu G G'; both diagonalised by Jacobi.
//   PSD:    R, R^-1 from Cholesky factors and a Jacobi SVD; M = R R' = Q diag(m) Q';
//           H(X) = M X M has eigenvalues m_i m_j on svec(q_i q_j' + q_j q_i').
#include "hc_cones.h"
#include "hc_soc_math.h"

#include <cmath>

namespace hc {


__device__ inline double sq(double x) { return x * x; }

// ===========================================================================
// small dense helpers (per lane)
// ===========================================================================

// one-sided Jacobi on the 3 rows of G (3 x NC, row-major): on return rows
// are orthogonal, U (3x3, row-major) accumulates G = U G'.  NC is a
// compile-time size so that every index is static (registers, no scratch).
template <int NC>
__device__ void jacobi_rows3(double* G, double* U) {
  constexpr int nc = NC;
#pragma unroll
  for (int i = 0; i < 9; ++i) U[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rot = false;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = (pq == 2) ? 1 : 0, q = (pq == 0) ? 1 : 2;
      double a = 0, b = 0, g = 0;
#pragma unroll
      for (int c = 0; c < nc; ++c) {
        a += G[p * nc + c] * G[p * nc + c];
        b += G[q * nc + c] * G[q * nc + c];
        g += G[p * nc + c] * G[q * nc + c];
      }
      if (g == 0.0 || fabs(g) <= 1e-15 * sqrt(a * b)) continue;   // orthogonal to a few ulps
      rot = true;
      const double zeta = (b - a) / (2.0 * g);
      const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
      for (int c = 0; c < nc; ++c) {
        const double gp = G[p * nc + c], gq = G[q * nc + c];
        G[p * nc + c] = cs * gp - sn * gq;
        G[q * nc + c] = sn * gp + cs * gq;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double up = U[r * 3 + p], uq = U[r * 3 + q];
        U[r * 3 + p] = cs * up - sn * uq;
        U[r * 3 + q] = sn * up + cs * uq;
      }
    }
    if (!rot) break;
  }
}

// ===========================================================================
// exponential and power cones: barrier pieces on the dual cone
// ===========================================================================

// grad f(z)
__device__ void exp_grad(const double* z, double* g) {
  const double ell = log(z[2] / (-z[0]));
  const double psi = z[1] - z[0] - z[0] * ell;
  g[0] = ell / psi - 1.0 / z[0];
  g[1] = -1.0 / psi;
  g[2] = (z[0] / z[2]) / psi - 1.0 / z[2];
}

__device__ void pow_grad(const double* z, double a, double* g) {
  const double Pi = pow(z[0] / a, a) * pow(z[1] / (1.0 - a), 1.0 - a);
  const double gp0 = Pi * a / z[0], gp1 = Pi * (1.0 - a) / z[1];
  const double dm = Pi - z[2], dp = Pi + z[2];
  g[0] = -gp0 / dm - gp0 / dp - (1.0 - a) / z[0];
  g[1] = -gp1 / dm - gp1 / dp - a / z[1];
  g[2] = 1.0 / dm - 1.0 / dp;
}

// G (3 x nc, row-major) with G G' = Hess f(z); returns nc
__device__ int exp_hess_factor(const double* z, double* G) {
  const double z1 = z[0], z2 = z[1], z3 = z[2];
  const double ell = log(z3 / (-z1));
  const double psi = z2 - z1 - z1 * ell;
  const double rp = sqrt(psi);
  // columns: c/sqrt(psi), grad psi / psi, e1/|z1|, e3/z3
  const double c0 = 1.0 / sqrt(-z1), c2 = sqrt(-z1) / z3;
  G[0 * 4 + 0] = c0 / rp;    G[1 * 4 + 0] = 0.0;        G[2 * 4 + 0] = c2 / rp;
  G[0 * 4 + 1] = -ell / psi; G[1 * 4 + 1] = 1.0 / psi;  G[2 * 4 + 1] = (-z1 / z3) / psi;
  G[0 * 4 + 2] = 1.0 / (-z1); G[1 * 4 + 2] = 0.0;       G[2 * 4 + 2] = 0.0;
  G[0 * 4 + 3] = 0.0;        G[1 * 4 + 3] = 0.0;        G[2 * 4 + 3] = 1.0 / z3;
  return 4;
}

__device__ int pow_hess_factor(const double* z, double a, double* G) {
  const double Pi = pow(z[0] / a, a) * pow(z[1] / (1.0 - a), 1.0 - a);
  const double gp0 = Pi * a / z[0], gp1 = Pi * (1.0 - a) / z[1];
  const double d0 = 1.0 / z[0], d1 = -1.0 / z[1];
  int col = 0;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    const double den = Pi + sgn * z[2];
    const double w = sqrt(Pi * a * (1.0 - a) / den);
    G[0 * 6 + col] = w * d0; G[1 * 6 + col] = w * d1; G[2 * 6 + col] = 0.0;
    ++col;
    G[0 * 6 + col] = gp0 / den; G[1 * 6 + col] = gp1 / den; G[2 * 6 + col] = sgn / den;
    ++col;
  }
  G[0 * 6 + 4] = sqrt(1.0 - a) / z[0]; G[1 * 6 + 4] = 0.0; G[2 * 6 + 4] = 0.0;
  G[0 * 6 + 5] = 0.0; G[1 * 6 + 5] = sqrt(a) / z[1]; G[2 * 6 + 5] = 0.0;
  return 6;
}

// Third derivative contraction T_i = f'''(z)[u, v, e_i] of a term -log g(z):
//   -D3g[u,v]_i/g + (D2g[u,v] dg_i + (D2g u)_i dg[v] + (D2g v)_i dg[u])/g^2 - 2 dg[u] dg[v] dg_i / g^3
__device__ void neglog_third(double g, const double* dg, const double* D2g /*3x3*/, const double* D3uv,
                             const double* u, const double* v, double* T) {
  double du = 0, dv = 0, Duv = 0, D2u[3], D2v[3];
  for (int i = 0; i < 3; ++i) {
    du += dg[i] * u[i];
    dv += dg[i] * v[i];
    D2u[i] = D2g[i * 3 + 0] * u[0] + D2g[i * 3 + 1] * u[1] + D2g[i * 3 + 2] * u[2];
    D2v[i] = D2g[i * 3 + 0] * v[0] + D2g[i * 3 + 1] * v[1] + D2g[i * 3 + 2] * v[2];
  }
  for (int i = 0; i < 3; ++i) Duv += u[i] * D2v[i];
  const double g2 = g * g;
  for (int i = 0; i < 3; ++i)
    T[i] += -D3uv[i] / g + (Duv * dg[i] + D2u[i] * dv + D2v[i] * du) / g2 - 2.0 * du * dv * dg[i] / (g2 * g);
}

__device__ void exp_third(const double* z, const double* u, const double* v, double* T) {
  const double z1 = z[0], z2 = z[1], z3 = z[2];
  const double ell = log(z3 / (-z1));
  const double psi = z2 - z1 - z1 * ell;
  const double dg[3] = {-ell, 1.0, -z1 / z3};
  const double D2[9] = {1.0 / z1, 0.0, -1.0 / z3, 0.0, 0.0, 0.0, -1.0 / z3, 0.0, z1 / (z3 * z3)};
  double D3[3];
  D3[0] = -u[0] * v[0] / (z1 * z1) + u[2] * v[2] / (z3 * z3);
  D3[1] = 0.0;
  D3[2] = (u[0] * v[2] + u[2] * v[0]) / (z3 * z3) - 2.0 * z1 * u[2] * v[2] / (z3 * z3 * z3);
  T[0] = T[1] = T[2] = 0.0;
  neglog_third(psi, dg, D2, D3, u, v, T);
  T[0] += -2.0 * u[0] * v[0] / (z1 * z1 * z1);
  T[2] += -2.0 * u[2] * v[2] / (z3 * z3 * z3);
}

__device__ void pow_third(const double* z, double a, const double* u, const double* v, double* T) {
  const double Pi = pow(z[0] / a, a) * pow(z[1] / (1.0 - a), 1.0 - a);
  const double av[3] = {a / z[0], (1.0 - a) / z[1], 0.0};            // grad log Pi
  const double Bd[3] = {-a / (z[0] * z[0]), -(1.0 - a) / (z[1] * z[1]), 0.0};  // Hess log Pi (diag)
  const double au = av[0] * u[0] + av[1] * u[1], avv = av[0] * v[0] + av[1] * v[1];
  const double uBv = Bd[0] * u[0] * v[0] + Bd[1] * u[1] * v[1];
  double D2[9], D3[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D2[i * 3 + j] = Pi * (av[i] * av[j] + (i == j ? Bd[i] : 0.0));
  const double dL[3] = {2.0 * a * u[0] * v[0] / (z[0] * z[0] * z[0]),
                        2.0 * (1.0 - a) * u[1] * v[1] / (z[1] * z[1] * z[1]), 0.0};
  for (int i = 0; i < 3; ++i)
    D3[i] = Pi * (av[i] * au * avv + Bd[i] * u[i] * avv + Bd[i] * v[i] * au + av[i] * uBv + dL[i]);
  T[0] = T[1] = T[2] = 0.0;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    const double g = Pi + sgn * z[2];
    const double dg[3] = {Pi * av[0], Pi * av[1], (double)sgn};
    neglog_third(g, dg, D2, D3, u, v, T);
  }
  T[0] += -2.0 * (1.0 - a) * u[0] * v[0] / (z[0] * z[0] * z[0]);
  T[1] += -2.0 * a * u[1] * v[1] / (z[1] * z[1] * z[1]);
}

// membership of int K (primal) and int K* (dual)
__device__ bool exp_primal_in(const double* s) {
  if (!(s[1] > 0.0 && s[2] > 0.0)) return false;
  return s[1] * log(s[2] / s[1]) - s[0] > 0.0;
}
__device__ bool exp_dual_in(const double* z) {
  if (!(z[0] < 0.0 && z[2] > 0.0)) return false;
  return z[1] - z[0] - z[0] * log(z[2] / (-z[0])) > 0.0;
}
__device__ bool pow_primal_in(const double* s, double a) {
  if (!(s[0] > 0.0 && s[1] > 0.0)) return false;
  return 2.0 * a * log(s[0]) + 2.0 * (1.0 - a) * log(s[1]) - log(s[2] * s[2]) > 0.0;
}
__device__ bool pow_dual_in(const double* z, double a) {
  if (!(z[0] > 0.0 && z[1] > 0.0)) return false;
  return 2.0 * a * log(z[0] / a) + 2.0 * (1.0 - a) * log(z[1] / (1.0 - a)) - log(z[2] * z[2]) > 0.0;
}

// z~ = -grad f*(s): the z with -grad f(z) = s (s in int K), through a scalar
// equation solved by safeguarded Newton.
__device__ bool exp_conj(const double* s, double* z) {
  // y = 1/t > 0 solves log(1 + y) + y = r, r = log(s3/s2) - s1/s2; Newton from
  // the lower bound y0 = r/2 increases monotonically to the root (the left side
  // is concave increasing).
  const double r = log(s[2] / s[1]) - s[0] / s[1];
  if (!(r > 0.0)) return false;
  double y = 0.5 * r;
  for (int it = 0; it < 200; ++it) {
    const double h = log1p(y) + y - r;
    const double dy = -h / (1.0 / (1.0 + y) + 1.0);
    y += dy;
    // the exact steps increase y; once a step is down to a couple of ulps
    // (or rounding turns it negative) y is the root to working accuracy (a
    // bound of 1e-16 y, below half an ulp, let most cones run all 200 steps)
    if (!(dy > 4e-16 * y)) break;
  }
  const double t = 1.0 / y;
  const double u = -t / s[1];
  const double lw = log1p(y) + log(s[1] / s[2]);   // log(w / (-u))
  z[0] = u;
  z[2] = (1.0 + t) / s[2];
  z[1] = 1.0 / s[1] + u * (1.0 + lw);
  return isfinite(z[0]) && isfinite(z[1]) && isfinite(z[2]);
}

__device__ bool pow_conj(const double* s, double a, double* z) {
  if (s[2] == 0.0) {
    z[0] = (1.0 + a) / s[0];
    z[1] = (2.0 - a) / s[1];
    z[2] = 0.0;
    return true;
  }
  // y > 0 solves h(y) = 2a log(1+a+2ay) + 2(1-a) log(2-a+2(1-a)y) - log(1+y) - log y - log 4 + C = 0,
  // h strictly decreasing; Newton in t = log y inside a bisection bracket.
  const double C = 2.0 * log(fabs(s[2])) - 2.0 * a * log(a * s[0]) - 2.0 * (1.0 - a) * log((1.0 - a) * s[1]);
  auto h = [&](double t, double* dh) {
    const double y = exp(t);
    const double p1 = 1.0 + a + 2.0 * a * y, p2 = 2.0 - a + 2.0 * (1.0 - a) * y;
    const double val = 2.0 * a * log(p1) + 2.0 * (1.0 - a) * log(p2) - log1p(y) - t - 1.3862943611198906 + C;
    *dh = y * (4.0 * a * a / p1 + 4.0 * (1.0 - a) * (1.0 - a) / p2 - 1.0 / (1.0 + y)) - 1.0;
    return val;
  };
  double lo = -200.0, hi = 200.0;
  double t = 2.0 * a * log(1.0 + a) + 2.0 * (1.0 - a) * log(2.0 - a) - 1.3862943611198906 + C;  // small-y asymptote
  t = fmin(fmax(t, -150.0), 150.0);
  for (int it = 0; it < 300; ++it) {
    double dh;
    const double v = h(t, &dh);
    if (v > 0.0) lo = t; else hi = t;
    double tn = t - v / dh;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    const double step = fabs(tn - t);
    t = tn;
    if (step <= 1e-15 * fmax(1.0, fabs(t)) || hi - lo <= 1e-15 * fmax(1.0, fabs(t))) break;
  }
  const double y = exp(t);
  z[0] = (1.0 + a + 2.0 * a * y) / s[0];
  z[1] = (2.0 - a + 2.0 * (1.0 - a) * y) / s[1];
  z[2] = -2.0 * y / s[2];
  return isfinite(z[0]) && isfinite(z[1]) && isfinite(z[2]);
}

// ===========================================================================
// kernels: scaling
// ===========================================================================
// scaling of one zero/nonneg row or lane-per-cone SOC i of segment g
__device__ inline void sym_scale_one(const SegDev& g, int64_t i, const double* __restrict__ s,
                                     const double* __restrict__ z, double* __restrict__ hdiag) {
  if (g.kind == HC_CONE_ZERO) {
    hdiag[g.base + i] = 0.0;
    return;
  }
  if (g.kind == HC_CONE_NONNEG) {
    const double h = s[g.base + i] / z[g.base + i];
    g.state[i] = h;
    hdiag[g.base + i] = h;
    return;
  }
  const int d = g.dim;
  const int64_t N = g.count;
  double sv[SOC_DMAX], zv[SOC_DMAX];
  for (int j = 0; j < d; ++j) {
    sv[j] = s[g.base + j * N + i];
    zv[j] = z[g.base + j * N + i];
  }
  double wb[SOC_DMAX], lam[SOC_DMAX];
  const double eta = soc_nt_scale(sv, zv, d, wb, lam);
  for (int j = 0; j < d; ++j) {
    g.state[j * N + i] = wb[j];
    g.state[(d + 1 + j) * N + i] = lam[j];
  }
  g.state[d * N + i] = eta;
  const double e2 = eta * eta;
  for (int j = 0; j < d; ++j) hdiag[g.base + j * N + i] = e2 * (2.0 * wb[j] * wb[j] - (j == 0 ? 1.0 : -1.0));
}

__global__ __launch_bounds__(CONE_BLOCK) void k_sym_scale(SegDev g, const double* __restrict__ s, const double* __restrict__ z,
                            double* __restrict__ hdiag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.count) sym_scale_one(g, i, s, z, hdiag);
}

// exp/pow state fields (field-major): lam 0..2, V 3..11 (row-major), Uh 12..20,
// sig_h 21..23, grad 24..26, branch 27
constexpr int NS_LAM = 0, NS_V = 3, NS_UH = 12, NS_SH = 21, NS_GRAD = 24, NS_BR = 27;

__global__ __launch_bounds__(CONE_BLOCK) void k_nonsym_scale(SegDev g, const double* __restrict__ s, const double* __restrict__ z, double mu,
                               int force_dual, double* __restrict__ hdiag, int* __restrict__ pd_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.count) return;
  const int64_t N = g.count;
  const bool is_exp = (g.kind == HC_CONE_EXP);
  const double a = is_exp ? 0.0 : g.alpha[i];
  double sv[3], zv[3];
  for (int j = 0; j < 3; ++j) {
    sv[j] = s[g.base + j * N + i];
    zv[j] = z[g.base + j * N + i];
  }
  double gr[3];
  if (is_exp) exp_grad(zv, gr); else pow_grad(zv, a, gr);
  const double st[3] = {-gr[0], -gr[1], -gr[2]};
  double zt[3];
  const bool ok = is_exp ? exp_conj(sv, zt) : pow_conj(sv, a, zt);
  const double mu_i = (sv[0] * zv[0] + sv[1] * zv[1] + sv[2] * zv[2]) / 3.0;
  const double mut_i = (st[0] * zt[0] + st[1] * zt[1] + st[2] * zt[2]) / 3.0;
  bool dual = force_dual || !ok || !(mu_i * mut_i - 1.0 >= 1.4901161193847656e-08);
  // factor of Hess f and its SVD (Hess f^-1 = Uh diag(1/sig^2) Uh')
  double Uh[9], sig[3];
  if (is_exp) {
    double G[12];
    exp_hess_factor(zv, G);
    jacobi_rows3<4>(G, Uh);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc += G[r * 4 + c] * G[r * 4 + c];
      sig[r] = sqrt(acc);
    }
  } else {
    double G[18];
    pow_hess_factor(zv, a, G);
    jacobi_rows3<6>(G, Uh);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < 6; ++c) acc += G[r * 6 + c] * G[r * 6 + c];
      sig[r] = sqrt(acc);
    }
  }
  double lam[3], V[9];
  if (!dual) {
    const double szd = sv[0] * zv[0] + sv[1] * zv[1] + sv[2] * zv[2];
    double dsv[3], dzv[3], uu[3];
    for (int j = 0; j < 3; ++j) {
      dsv[j] = sv[j] - mu_i * st[j];
      dzv[j] = zv[j] - mu_i * zt[j];
    }
    uu[0] = zv[1] * zt[2] - zv[2] * zt[1];
    uu[1] = zv[2] * zt[0] - zv[0] * zt[2];
    uu[2] = zv[0] * zt[1] - zv[1] * zt[0];
    double uHu = 0;
    for (int r = 0; r < 3; ++r) {
      const double pr = (Uh[0 * 3 + r] * uu[0] + Uh[1 * 3 + r] * uu[1] + Uh[2 * 3 + r] * uu[2]) / sig[r];
      uHu += pr * pr;
    }
    const double dd = dsv[0] * dzv[0] + dsv[1] * dzv[1] + dsv[2] * dzv[2];
    const double c1 = 1.0 / sqrt(szd), c2 = 1.0 / sqrt(dd), c3 = sqrt(mu / uHu);
    double Gp[9];
    for (int r = 0; r < 3; ++r) {
      Gp[r * 3 + 0] = sv[r] * c1;
      Gp[r * 3 + 1] = dsv[r] * c2;
      Gp[r * 3 + 2] = uu[r] * c3;
    }
    bool fin = isfinite(c1) && isfinite(c2) && isfinite(c3) && dd > 0.0 && uHu > 0.0;
    if (fin) {
      jacobi_rows3<3>(Gp, V);
      for (int r = 0; r < 3; ++r) lam[r] = Gp[r * 3 + 0] * Gp[r * 3 + 0] + Gp[r * 3 + 1] * Gp[r * 3 + 1] +
                                           Gp[r * 3 + 2] * Gp[r * 3 + 2];
    } else {
      dual = true;
    }
  }
  if (dual) {
    for (int r = 0; r < 9; ++r) V[r] = Uh[r];
    for (int r = 0; r < 3; ++r) lam[r] = mu * sig[r] * sig[r];
  } else {
    atomicAdd(pd_count, 1);
  }
  for (int j = 0; j < 3; ++j) g.state[(NS_LAM + j) * N + i] = lam[j];
  for (int j = 0; j < 9; ++j) {
    g.state[(NS_V + j) * N + i] = V[j];
    g.state[(NS_UH + j) * N + i] = Uh[j];
  }
  for (int j = 0; j < 3; ++j) {
    g.state[(NS_SH + j) * N + i] = sig[j];
    g.state[(NS_GRAD + j) * N + i] = gr[j];
  }
  g.state[NS_BR * N + i] = dual ? 1.0 : 0.0;
  for (int j = 0; j < 3; ++j) {
    double hd = 0;
    for (int r = 0; r < 3; ++r) hd += lam[r] * V[j * 3 + r] * V[j * 3 + r];
    hdiag[g.base + j * N + i] = hd;
  }
}

// PSD kernels run one wave per cone for every side up to 32 (the paper's
// limit), with the cone's k x k matrices in LDS (the wave kernels below).  The
// spectral apply comes in two instantiations, KM = 12 and KM = 32, which size
// its LDS arrays.
constexpr int PSD_KSMALL = 12, PSD_KLARGE = 32;


// PSD scaling and d_s correction, one wave per cone (defined with the other
// wave kernels below)
__global__ __launch_bounds__(64) void k_psd_scale_wave(SegDev g, const double* __restrict__ s,
                                                       const double* __restrict__ z, double* __restrict__ hdiag);
__global__ __launch_bounds__(64) void k_psd_ds_wave(SegDev g, const double* __restrict__ dsa,
                                                    const double* __restrict__ dza, double sm,
                                                    double* __restrict__ ds);

void cone_scale(const SegDev& g, const double* s, const double* z, double mu, int force_dual, double* hdiag,
                int* pd_count, hipStream_t st) {
  if (g.count == 0) return;
  const int nb = cone_blocks(g);
  switch (g.kind) {
    case HC_CONE_ZERO:
    case HC_CONE_NONNEG:
      hipLaunchKernelGGL(k_sym_scale, dim3(nb), dim3(CONE_BLOCK), 0, st, g, s, z, hdiag);
      break;
    case HC_CONE_SOC:
      if (soc_large(g.kind, g.dim)) {
        lsoc_scale(g, s, z, hdiag, st);
        return;
      }
      hipLaunchKernelGGL(k_sym_scale, dim3(nb), dim3(CONE_BLOCK), 0, st, g, s, z, hdiag);
      break;
    case HC_CONE_EXP:
    case HC_CONE_POW:
      hipLaunchKernelGGL(k_nonsym_scale, dim3(nb), dim3(CONE_BLOCK), 0, st, g, s, z, mu, force_dual, hdiag,
                         pd_count);
      break;
    case HC_CONE_PSD:
      hipLaunchKernelGGL(k_psd_scale_wave, dim3((unsigned)std::min<int64_t>(g.count, 4096)), dim3(64), 0, st, g, s, z,
                         hdiag);
      break;
  }
  HC_LAUNCH_CHECK();
}

constexpr int FUSED_SEGS = 8;

// ===========================================================================
// spectral application of H or (H + delta I)^-1, and the explicit inverse block
// ===========================================================================
__device__ inline double fsel(int mode, double lam, double delta) { return mode == 0 ? lam : 1.0 / (lam + delta); }

// one cone (or zero/nonneg row) i of segment g: y = H x (mode 0) or
// (H + delta I)^-1 x (mode 1); with dsr (mode 0): y = -dsr - H x, the
// direction recovery of Delta s
__device__ inline void cone_apply_one(const SegDev& g, int64_t i, int mode, double delta, const double* __restrict__ x,
                                      const double* __restrict__ dsr, double* __restrict__ y) {
  const int64_t N = g.count;
  switch (g.kind) {
    case HC_CONE_ZERO:
      y[g.base + i] = dsr ? -dsr[g.base + i] : ((mode == 0) ? 0.0 : x[g.base + i] / delta);
      break;
    case HC_CONE_NONNEG: {
      const double h = g.state[i], xv = x[g.base + i];
      y[g.base + i] = dsr ? -dsr[g.base + i] - h * xv : ((mode == 0) ? h * xv : (1.0 / (h + delta)) * xv);
      break;
    }
    case HC_CONE_SOC: {
      const int d = g.dim;
      double wb[SOC_DMAX], xv[SOC_DMAX], yv[SOC_DMAX];
      for (int j = 0; j < d; ++j) {
        wb[j] = g.state[j * N + i];
        xv[j] = x[g.base + j * N + i];
      }
      const double eta = g.state[d * N + i];
      const SocSpec sp = soc_spec(wb, d, eta);
      soc_spec_apply(wb, d, sp, fsel(mode, sp.lp, delta), fsel(mode, sp.lm, delta), fsel(mode, sp.lo, delta), xv,
                     yv);
      for (int j = 0; j < d; ++j) y[g.base + j * N + i] = dsr ? -dsr[g.base + j * N + i] - yv[j] : yv[j];
      break;
    }
    case HC_CONE_EXP:
    case HC_CONE_POW: {
      double V[9], lam[3], xv[3];
      for (int j = 0; j < 9; ++j) V[j] = g.state[(NS_V + j) * N + i];
      for (int j = 0; j < 3; ++j) {
        lam[j] = fsel(mode, g.state[(NS_LAM + j) * N + i], delta);
        xv[j] = x[g.base + j * N + i];
      }
      double p[3];
      for (int r = 0; r < 3; ++r) p[r] = lam[r] * (V[0 * 3 + r] * xv[0] + V[1 * 3 + r] * xv[1] + V[2 * 3 + r] * xv[2]);
      for (int j = 0; j < 3; ++j) {
        const double hv = V[j * 3 + 0] * p[0] + V[j * 3 + 1] * p[1] + V[j * 3 + 2] * p[2];
        y[g.base + j * N + i] = dsr ? -dsr[g.base + j * N + i] - hv : hv;
      }
      break;
    }
    default:
      break;   // PSD and large SOC: their own kernels
  }
}

__global__ __launch_bounds__(CONE_BLOCK) void k_cone_apply(SegDev g, int mode, double delta, const double* __restrict__ x,
                             double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.count) cone_apply_one(g, i, mode, delta, x, nullptr, y);
}

// every lane-per-cone segment in one launch: block b belongs to the segment s
// with first[s] <= b < first[s + 1]
struct SegTable {
  SegDev g[FUSED_SEGS];
  int32_t first[FUSED_SEGS + 1];
  int32_t nseg;
};

__global__ __launch_bounds__(CONE_BLOCK) void k_cone_apply_fused(SegTable tb, int mode, double delta, const double* __restrict__ x,
                                   const double* __restrict__ dsr, double* __restrict__ y) {
  int s = 0;
  while (s + 1 < tb.nseg && (int)blockIdx.x >= tb.first[s + 1]) ++s;
  const int64_t i = (int64_t)(blockIdx.x - tb.first[s]) * blockDim.x + threadIdx.x;
  if (i < tb.g[s].count) cone_apply_one(tb.g[s], i, mode, delta, x, dsr, y);
}

// Spectral application, one workgroup per cone (one lane per cone would pay
// k^3 dependent LDS round trips for each of the four k x k products): one
// wave up to side 12, four above.  The threads split every product by output
// entry; Q, X and the two intermediate products live in LDS (row stride
// KM + 1).  With dsr the kernel returns the direction recovery -dsr - H dz
// instead (mode 0).
template <int KM>
__global__ __launch_bounds__(KM <= 12 ? 64 : 256) void k_psd_apply_wave(SegDev g, int mode, double delta, const double* __restrict__ x,
                                                       const double* __restrict__ dsr, double* __restrict__ y) {
  constexpr int LD = KM + 1;
  __shared__ double Q[KM * LD], X[KM * LD], T[KM * LD], U[KM * LD], m[KM];
  const int k = g.k, lane = threadIdx.x, sd = g.dim;
  const int64_t N = g.count, kk = (int64_t)k * k;
  constexpr int NT = KM <= 12 ? 64 : 256;   // four waves per cone above side 12
  for (int64_t c = blockIdx.x; c < N; c += gridDim.x) {
    const double* xc = x + g.base + c * sd;
    __syncthreads();   // the previous cone's readers are done
    for (int e = lane; e < k * k; e += NT) Q[(e / k) * LD + e % k] = g.state[(2 * kk + e) * N + c];
    for (int e = lane; e < k; e += NT) m[e] = g.state[(3 * kk + k + e) * N + c];
    for (int p = lane; p < sd; p += NT) {   // smat: svec entry p is (i, j), i <= j, column by column
      int j = (int)((sqrt(8.0 * p + 1.0) - 1.0) / 2.0);
      while (j * (j + 1) / 2 > p) --j;
      while ((j + 1) * (j + 2) / 2 <= p) ++j;
      const int i = p - j * (j + 1) / 2;
      const double v = xc[p] * (i == j ? 1.0 : 0.70710678118654752440);
      X[i * LD + j] = v;
      X[j * LD + i] = v;
    }
    __syncthreads();
    for (int e = lane; e < k * k; e += NT) {   // T = X Q
      const int i = e / k, j = e % k;
      double acc = 0;
      for (int p = 0; p < k; ++p) acc += X[i * LD + p] * Q[p * LD + j];
      T[i * LD + j] = acc;
    }
    __syncthreads();
    for (int e = lane; e < k * k; e += NT) {   // U = Q' T
      const int i = e / k, j = e % k;
      double acc = 0;
      for (int p = 0; p < k; ++p) acc += Q[p * LD + i] * T[p * LD + j];
      U[i * LD + j] = acc;
    }
    __syncthreads();
    // average the two roundings of each eigen-coefficient, then scale
    for (int e = lane; e < k * k; e += NT) {
      const int i = e / k, j = e % k;
      const double lam = m[i] * m[j];
      T[i * LD + j] = 0.5 * (U[i * LD + j] + U[j * LD + i]) * (mode == 0 ? lam : 1.0 / (lam + delta));
    }
    __syncthreads();
    for (int e = lane; e < k * k; e += NT) {   // U = T Q'
      const int i = e / k, j = e % k;
      double acc = 0;
      for (int p = 0; p < k; ++p) acc += T[i * LD + p] * Q[j * LD + p];
      U[i * LD + j] = acc;
    }
    __syncthreads();
    for (int e = lane; e < k * k; e += NT) {   // X = Q U
      const int i = e / k, j = e % k;
      double acc = 0;
      for (int p = 0; p < k; ++p) acc += Q[i * LD + p] * U[p * LD + j];
      X[i * LD + j] = acc;
    }
    __syncthreads();
    for (int p = lane; p < sd; p += NT) {   // svec of the upper triangle
      int j = (int)((sqrt(8.0 * p + 1.0) - 1.0) / 2.0);
      while (j * (j + 1) / 2 > p) --j;
      while ((j + 1) * (j + 2) / 2 <= p) ++j;
      const int i = p - j * (j + 1) / 2;
      const double v = X[i * LD + j] * (i == j ? 1.0 : 1.41421356237309504880);
      const int64_t r = g.base + c * sd + p;
      y[r] = dsr ? -dsr[r] - v : v;
    }
  }
}

void cone_apply(const SegDev& g, int mode, double delta, const double* x, double* y, hipStream_t st) {
  if (g.count == 0) return;
  if (soc_large(g.kind, g.dim))
    lsoc_apply(g, mode, delta, x, nullptr, y, st);
  else if (g.kind == HC_CONE_PSD)
    if (g.k <= PSD_KSMALL)
      hipLaunchKernelGGL(k_psd_apply_wave<PSD_KSMALL>, dim3((unsigned)std::min<int64_t>(g.count, 4096)), dim3(64), 0,
                         st, g, mode, delta, x, (const double*)nullptr, y);
    else
      hipLaunchKernelGGL(k_psd_apply_wave<PSD_KLARGE>, dim3((unsigned)std::min<int64_t>(g.count, 4096)), dim3(256), 0,
                         st, g, mode, delta, x, (const double*)nullptr, y);
  else
    hipLaunchKernelGGL(k_cone_apply, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, mode, delta, x, y);
  HC_LAUNCH_CHECK();
}

__global__ __launch_bounds__(CONE_BLOCK) void k_cone_recover(SegDev g, const double* __restrict__ dsr, const double* __restrict__ dz,
                               double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.count) cone_apply_one(g, i, 0, 0.0, dz, dsr, out);
}

void cone_recover_ds(const SegDev& g, const double* dsrhs, const double* dz, double* out, hipStream_t st) {
  if (g.count == 0) return;
  if (soc_large(g.kind, g.dim))
    lsoc_apply(g, 0, 0.0, dz, dsrhs, out, st);
  else if (g.kind == HC_CONE_PSD)
    if (g.k <= PSD_KSMALL)
      hipLaunchKernelGGL(k_psd_apply_wave<PSD_KSMALL>, dim3((unsigned)std::min<int64_t>(g.count, 4096)), dim3(64), 0,
                         st, g, 0, 0.0, dz, dsrhs, out);
    else
      hipLaunchKernelGGL(k_psd_apply_wave<PSD_KLARGE>, dim3((unsigned)std::min<int64_t>(g.count, 4096)), dim3(256), 0,
                         st, g, 0, 0.0, dz, dsrhs, out);
  else
    hipLaunchKernelGGL(k_cone_recover, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, dsrhs, dz, out);
  HC_LAUNCH_CHECK();
}

bool lane_per_cone(const SegDev& g) {
  return g.count > 0 && g.kind != HC_CONE_PSD && !soc_large(g.kind, g.dim);
}

void cone_apply_all(const std::vector<SegDev>& segs, int mode, double delta, const double* x, const double* dsr,
                    double* y, hipStream_t st) {
  SegTable tb{};
  int nb = 0;
  auto flush = [&]() {
    if (tb.nseg == 0) return;
    tb.first[tb.nseg] = nb;
    hipLaunchKernelGGL(k_cone_apply_fused, dim3((unsigned)nb), dim3(CONE_BLOCK), 0, st, tb, mode, delta, x, dsr, y);
    HC_LAUNCH_CHECK();
    tb.nseg = 0;
    nb = 0;
  };
  for (const SegDev& g : segs) {
    if (g.count == 0) continue;
    if (!lane_per_cone(g)) {   // PSD and large SOC keep their own kernels
      if (dsr) cone_recover_ds(g, dsr, x, y, st);
      else cone_apply(g, mode, delta, x, y, st);
      continue;
    }
    if (tb.nseg == FUSED_SEGS) flush();
    tb.g[tb.nseg] = g;
    tb.first[tb.nseg] = nb;
    tb.nseg++;
    nb += (int)ceil_div(g.count, CONE_BLOCK);
  }
  flush();
}

__global__ __launch_bounds__(CONE_BLOCK) void k_sym_scale_fused(SegTable tb, const double* __restrict__ s, const double* __restrict__ z,
                                  double* __restrict__ hdiag) {
  int q = 0;
  while (q + 1 < tb.nseg && (int)blockIdx.x >= tb.first[q + 1]) ++q;
  const int64_t i = (int64_t)(blockIdx.x - tb.first[q]) * blockDim.x + threadIdx.x;
  if (i < tb.g[q].count) sym_scale_one(tb.g[q], i, s, z, hdiag);
}

void cone_scale_all(const std::vector<SegDev>& segs, const double* s, const double* z, double mu, int force_dual,
                    double* hdiag, int* pd_count, hipStream_t st) {
  SegTable tb{};
  int nb = 0;
  auto flush = [&]() {
    if (tb.nseg == 0) return;
    tb.first[tb.nseg] = nb;
    hipLaunchKernelGGL(k_sym_scale_fused, dim3((unsigned)nb), dim3(CONE_BLOCK), 0, st, tb, s, z, hdiag);
    HC_LAUNCH_CHECK();
    tb.nseg = 0;
    nb = 0;
  };
  for (const SegDev& g : segs) {
    if (g.count == 0) continue;
    const bool sym = g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG || (g.kind == HC_CONE_SOC && !soc_large(g.kind, g.dim));
    if (!sym) {   // exp/pow (primal-dual or dual scaling), PSD, large SOC: their own kernels
      cone_scale(g, s, z, mu, force_dual, hdiag, pd_count, st);
      continue;
    }
    if (tb.nseg == FUSED_SEGS) flush();
    tb.g[tb.nseg] = g;
    tb.first[tb.nseg] = nb;
    tb.nseg++;
    nb += (int)ceil_div(g.count, CONE_BLOCK);
  }
  flush();
}

// explicit lower-triangle entries of M = (H + delta I)^-1, packed index
// p = a (a + 1) / 2 + b for a >= b, stored mblk[p * count + cone]
//
// PSD: with f(i,j) = 1/(m_i m_j + delta) and svec index a = (ia, ja),
//   M_ab = (c_a c_b / 2) sum_i Q[ia][i] (Q[ib][i] G_i[ja][jb] + Q[jb][i] G_i[ja][ib]),
//   G_i[q][s] = sum_j f(i,j) Q[q][j] Q[s][j],
// (c = 1 on the diagonal, sqrt2 off it), which is sum_e svec(E_e)_a svec(E_e)_b f_e
// over the eigenvectors E_e = (q_i q_j' + q_j q_i')/sqrt2 of H, expanded by the
// Kronecker structure: k^4 flops for the G_i and 2k per entry instead of k(k+1)/2
// per entry.  G (k^3 per cone) lives in the caller's work buffer.
__global__ __launch_bounds__(256) void k_psd_mblock_g(SegDev g, double delta, double* __restrict__ G) {
  __shared__ double Q[PSD_KLARGE * (PSD_KLARGE + 1)], m[PSD_KLARGE];
  const int k = g.k, LQ = PSD_KLARGE + 1;
  const int64_t N = g.count, kk = (int64_t)k * k, c = blockIdx.x;
  const int i = blockIdx.y;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) Q[(e / k) * LQ + e % k] = g.state[(2 * kk + e) * N + c];
  for (int e = threadIdx.x; e < k; e += blockDim.x) m[e] = g.state[(3 * kk + k + e) * N + c];
  __syncthreads();
  double* Gi = G + (c * k + i) * kk;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int q = e / k, sx = e % k;
    double acc = 0;
    for (int j = 0; j < k; ++j) acc += Q[q * LQ + j] * Q[sx * LQ + j] / (m[i] * m[j] + delta);
    Gi[e] = acc;
  }
}

__device__ inline void tri_index(int e, int& i, int& j);

// one thread per (cone, packed entry p = a (a + 1) / 2 + b): the grid's y
// dimension covers a cone's entries, so even a few large cones fill the chip
__global__ __launch_bounds__(256) void k_psd_mblock(SegDev g, const double* __restrict__ G) {
  __shared__ double Q[PSD_KLARGE * (PSD_KLARGE + 1)];
  const int k = g.k, LQ = PSD_KLARGE + 1, sd = g.dim;
  const int64_t N = g.count, kk = (int64_t)k * k, c = blockIdx.x;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) Q[(e / k) * LQ + e % k] = g.state[(2 * kk + e) * N + c];
  __syncthreads();
  const int np = sd * (sd + 1) / 2;
  const int p = (int)blockIdx.y * (int)blockDim.x + (int)threadIdx.x;
  if (p >= np) return;
  int a, b, ja, ia, jb, ib;
  tri_index(p, a, b);
  tri_index(a, ja, ia);
  tri_index(b, jb, ib);
  const double ca = (ia == ja) ? 1.0 : 1.41421356237309504880, cb = (ib == jb) ? 1.0 : 1.41421356237309504880;
  const double* Gc = G + c * k * kk + (int64_t)ja * k;
  double acc = 0;
  for (int i = 0; i < k; ++i) {
    const double* Gi = Gc + (int64_t)i * kk;
    acc += Q[ia * LQ + i] * (Q[ib * LQ + i] * Gi[jb] + Q[jb * LQ + i] * Gi[ib]);
  }
  g.mblk[(int64_t)p * N + c] = 0.5 * ca * cb * acc;
}

__device__ inline void cone_mblock_one(const SegDev& g, int64_t i, double delta) {
  const int64_t N = g.count;
  switch (g.kind) {
    case HC_CONE_ZERO:
      g.mblk[i] = 1.0 / delta;
      break;
    case HC_CONE_NONNEG:
      g.mblk[i] = 1.0 / (g.state[i] + delta);
      break;
    case HC_CONE_SOC: {
      const int d = g.dim;
      if (d > SOC_DMAX) {   // diagonal plus rank-2 coefficients (hc_soc.hip)
        const double w0 = g.state[i], eta = g.state[(int64_t)d * N + i], r = g.state[(2 * (int64_t)d + 1) * N + i];
        const double big = w0 + r, e2 = eta * eta;
        const double fp = 1.0 / (e2 * big * big + delta), fm = 1.0 / (e2 / (big * big) + delta);
        const double fo = 1.0 / (e2 + delta);
        g.mblk[i] = fo;
        g.mblk[N + i] = fp - fo;
        g.mblk[2 * N + i] = fm - fo;
        break;
      }
      double wb[SOC_DMAX], u[SOC_DMAX];
      for (int j = 0; j < d; ++j) wb[j] = g.state[j * N + i];
      const SocSpec sp = soc_spec(wb, d, g.state[d * N + i]);
      for (int j = 1; j < d; ++j) u[j] = (sp.r > 0.0) ? wb[j] / sp.r : (j == 1 ? 1.0 : 0.0);
      const double fp = 1.0 / (sp.lp + delta), fm = 1.0 / (sp.lm + delta), fo = 1.0 / (sp.lo + delta);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b <= a; ++b) {
          double v;
          if (a == 0) v = 0.5 * (fp + fm);
          else if (b == 0) v = 0.5 * (fp - fm) * u[a];
          else v = 0.5 * (fp + fm) * u[a] * u[b] + fo * ((a == b ? 1.0 : 0.0) - u[a] * u[b]);
          g.mblk[((int64_t)a * (a + 1) / 2 + b) * N + i] = v;
        }
      break;
    }
    case HC_CONE_EXP:
    case HC_CONE_POW: {
      double V[9], f[3];
      for (int j = 0; j < 9; ++j) V[j] = g.state[(NS_V + j) * N + i];
      for (int j = 0; j < 3; ++j) f[j] = 1.0 / (g.state[(NS_LAM + j) * N + i] + delta);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b <= a; ++b) {
          double v = 0;
          for (int r = 0; r < 3; ++r) v += V[a * 3 + r] * f[r] * V[b * 3 + r];
          g.mblk[((int64_t)a * (a + 1) / 2 + b) * N + i] = v;
        }
      break;
    }
  }
}

__global__ void k_cone_mblock(SegDev g, double delta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.count) cone_mblock_one(g, i, delta);
}

__global__ __launch_bounds__(CONE_BLOCK) void k_cone_mblock_fused(SegTable tb, double delta) {
  int q = 0;
  while (q + 1 < tb.nseg && (int)blockIdx.x >= tb.first[q + 1]) ++q;
  const int64_t i = (int64_t)(blockIdx.x - tb.first[q]) * blockDim.x + threadIdx.x;
  if (i < tb.g[q].count) cone_mblock_one(tb.g[q], i, delta);
}

int64_t cone_mblock_work(const SegDev& g) {
  return g.kind == HC_CONE_PSD ? g.count * (int64_t)g.k * g.k * g.k : 0;
}

void cone_mblock(const SegDev& g, double delta, double* work, hipStream_t st) {
  if (g.count == 0) return;
  if (g.kind == HC_CONE_PSD) {
    hipLaunchKernelGGL(k_psd_mblock_g, dim3((unsigned)g.count, (unsigned)g.k), dim3(256), 0, st, g, delta, work);
    HC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_psd_mblock, dim3((unsigned)g.count, (unsigned)ceil_div((int64_t)g.dim * (g.dim + 1) / 2, 256)),
                       dim3(256), 0, st, g, (const double*)work);
  } else
    hipLaunchKernelGGL(k_cone_mblock, dim3((unsigned)std::max<int64_t>(1, ceil_div(g.count, CONE_BLOCK))),
                       dim3(CONE_BLOCK), 0, st, g, delta);
  HC_LAUNCH_CHECK();
}

void cone_mblock_all(const std::vector<SegDev>& segs, double delta, double* work, hipStream_t st) {
  SegTable tb{};
  int nb = 0;
  auto flush = [&]() {
    if (tb.nseg == 0) return;
    tb.first[tb.nseg] = nb;
    hipLaunchKernelGGL(k_cone_mblock_fused, dim3((unsigned)nb), dim3(CONE_BLOCK), 0, st, tb, delta);
    HC_LAUNCH_CHECK();
    tb.nseg = 0;
    nb = 0;
  };
  for (const SegDev& g : segs) {
    if (g.count == 0) continue;
    if (g.kind == HC_CONE_PSD) {   // PSD: its own kernels (and the work buffer)
      cone_mblock(g, delta, work, st);
      continue;
    }
    if (tb.nseg == FUSED_SEGS) flush();
    tb.g[tb.nseg] = g;
    tb.first[tb.nseg] = nb;
    tb.nseg++;
    nb += (int)ceil_div(g.count, CONE_BLOCK);
  }
  flush();
}

// ===========================================================================
// combined-step d_s (eq. ds-correction-step)
// ===========================================================================
__device__ inline void cone_ds_one(const SegDev& g, int64_t i, const double* __restrict__ s,
                                   const double* __restrict__ z, const double* __restrict__ dsa,
                                   const double* __restrict__ dza, double sm, double* __restrict__ ds) {
  const int64_t N = g.count;
  switch (g.kind) {
    case HC_CONE_ZERO:
      ds[g.base + i] = 0.0;
      break;
    case HC_CONE_NONNEG: {
      const int64_t r = g.base + i;
      ds[r] = (s[r] * z[r] + dsa[r] * dza[r] - sm) / z[r];
      break;
    }
    case HC_CONE_SOC: {
      const int d = g.dim;
      double wb[SOC_DMAX], lam[SOC_DMAX], a[SOC_DMAX], b[SOC_DMAX];
      for (int j = 0; j < d; ++j) {
        wb[j] = g.state[j * N + i];
        lam[j] = g.state[(d + 1 + j) * N + i];
        a[j] = dsa[g.base + j * N + i];
        b[j] = dza[g.base + j * N + i];
      }
      double x[SOC_DMAX];
      soc_ds_one(wb, g.state[d * N + i], lam, a, b, d, sm, x);
      for (int j = 0; j < d; ++j) ds[g.base + j * N + i] = x[j];
      break;
    }
    case HC_CONE_EXP:
    case HC_CONE_POW: {
      const bool is_exp = (g.kind == HC_CONE_EXP);
      const double al = is_exp ? 0.0 : g.alpha[i];
      double zv[3], sv[3], a[3], b[3], Uh[9], sig[3], gr[3];
      for (int j = 0; j < 3; ++j) {
        zv[j] = z[g.base + j * N + i];
        sv[j] = s[g.base + j * N + i];
        a[j] = dsa[g.base + j * N + i];
        b[j] = dza[g.base + j * N + i];
        sig[j] = g.state[(NS_SH + j) * N + i];
        gr[j] = g.state[(NS_GRAD + j) * N + i];
      }
      for (int j = 0; j < 9; ++j) Uh[j] = g.state[(NS_UH + j) * N + i];
      // u = Hess f^-1 ds_a
      double pr[3], u[3];
      for (int r = 0; r < 3; ++r) pr[r] = (Uh[0 * 3 + r] * a[0] + Uh[1 * 3 + r] * a[1] + Uh[2 * 3 + r] * a[2]) / (sig[r] * sig[r]);
      for (int j = 0; j < 3; ++j) u[j] = Uh[j * 3 + 0] * pr[0] + Uh[j * 3 + 1] * pr[1] + Uh[j * 3 + 2] * pr[2];
      double T[3];
      if (is_exp) exp_third(zv, b, u, T); else pow_third(zv, al, b, u, T);
      for (int j = 0; j < 3; ++j) ds[g.base + j * N + i] = sv[j] + sm * gr[j] - 0.5 * T[j];
      break;
    }
    default:
      break;   // PSD: k_psd_ds_wave; large SOC: lsoc_ds
  }
}

__global__ __launch_bounds__(CONE_BLOCK) void k_cone_ds(SegDev g, const double* __restrict__ s, const double* __restrict__ z,
                          const double* __restrict__ dsa, const double* __restrict__ dza, double sm,
                          double* __restrict__ ds) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.count) cone_ds_one(g, i, s, z, dsa, dza, sm, ds);
}

__global__ __launch_bounds__(CONE_BLOCK) void k_cone_ds_fused(SegTable tb, const double* __restrict__ s, const double* __restrict__ z,
                                const double* __restrict__ dsa, const double* __restrict__ dza, double sm,
                                double* __restrict__ ds) {
  int q = 0;
  while (q + 1 < tb.nseg && (int)blockIdx.x >= tb.first[q + 1]) ++q;
  const int64_t i = (int64_t)(blockIdx.x - tb.first[q]) * blockDim.x + threadIdx.x;
  if (i < tb.g[q].count) cone_ds_one(tb.g[q], i, s, z, dsa, dza, sm, ds);
}

void cone_ds_all(const std::vector<SegDev>& segs, const double* s, const double* z, const double* dsa,
                 const double* dza, double sm, double* ds, hipStream_t st) {
  SegTable tb{};
  int nb = 0;
  auto flush = [&]() {
    if (tb.nseg == 0) return;
    tb.first[tb.nseg] = nb;
    hipLaunchKernelGGL(k_cone_ds_fused, dim3((unsigned)nb), dim3(CONE_BLOCK), 0, st, tb, s, z, dsa, dza, sm, ds);
    HC_LAUNCH_CHECK();
    tb.nseg = 0;
    nb = 0;
  };
  for (const SegDev& g : segs) {
    if (g.count == 0) continue;
    if (!lane_per_cone(g)) {
      cone_ds_combined(g, s, z, dsa, dza, sm, ds, st);
      continue;
    }
    if (tb.nseg == FUSED_SEGS) flush();
    tb.g[tb.nseg] = g;
    tb.first[tb.nseg] = nb;
    tb.nseg++;
    nb += (int)ceil_div(g.count, CONE_BLOCK);
  }
  flush();
}

void cone_ds_combined(const SegDev& g, const double* s, const double* z, const double* dsa, const double* dza,
                      double sm, double* ds, hipStream_t st) {
  if (g.count == 0) return;
  if (soc_large(g.kind, g.dim))
    lsoc_ds(g, dsa, dza, sm, ds, st);
  else if (g.kind == HC_CONE_PSD)
    hipLaunchKernelGGL(k_psd_ds_wave, dim3((unsigned)std::min<int64_t>(g.count, 4096)), dim3(64), 0, st, g, dsa, dza,
                       sm, ds);
  else
    hipLaunchKernelGGL(k_cone_ds, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, s, z, dsa, dza, sm, ds);
  HC_LAUNCH_CHECK();
}

// ===========================================================================
// step lengths
// ===========================================================================
__device__ inline double soc_step_one(const double* x, const double* dx, int d) {
  double a = dx[0] * dx[0], b = x[0] * dx[0], c = x[0] * x[0];
  for (int j = 1; j < d; ++j) {
    a -= dx[j] * dx[j];
    b -= x[j] * dx[j];
    c -= x[j] * x[j];
  }
  return soc_boundary_step(a, b, c);
}

// exact boundary step of one nonneg row or lane-per-cone SOC
__device__ inline double step_sym_one(const SegDev& g, int64_t i, const double* __restrict__ s,
                                      const double* __restrict__ z, const double* __restrict__ ds,
                                      const double* __restrict__ dz) {
  const int64_t N = g.count;
  double a = INFINITY;
  {
    if (g.kind == HC_CONE_NONNEG) {
      const int64_t r = g.base + i;
      if (ds[r] < 0.0) a = fmin(a, -s[r] / ds[r]);
      if (dz[r] < 0.0) a = fmin(a, -z[r] / dz[r]);
    } else if (g.kind == HC_CONE_SOC) {
      const int d = g.dim;
      double xs[SOC_DMAX], xds[SOC_DMAX], xz[SOC_DMAX], xdz[SOC_DMAX];
      for (int j = 0; j < d; ++j) {
        xs[j] = s[g.base + j * N + i];
        xds[j] = ds[g.base + j * N + i];
        xz[j] = z[g.base + j * N + i];
        xdz[j] = dz[g.base + j * N + i];
      }
      a = fmin(soc_step_one(xs, xds, d), soc_step_one(xz, xdz, d));
    }
  }
  return a;
}

__device__ inline void block_min_to(double a, double* __restrict__ partial) {
  __shared__ double red[CONE_BLOCK];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = CONE_BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(CONE_BLOCK) void k_step_sym(SegDev g, const double* __restrict__ s, const double* __restrict__ z,
                           const double* __restrict__ ds, const double* __restrict__ dz, double* __restrict__ partial) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  block_min_to(i < g.count ? step_sym_one(g, i, s, z, ds, dz) : INFINITY, partial);
}

__global__ __launch_bounds__(CONE_BLOCK) void k_step_sym_fused(SegTable tb, const double* __restrict__ s, const double* __restrict__ z,
                                 const double* __restrict__ ds, const double* __restrict__ dz,
                                 double* __restrict__ partial) {
  int q = 0;
  while (q + 1 < tb.nseg && (int)blockIdx.x >= tb.first[q + 1]) ++q;
  const int64_t i = (int64_t)(blockIdx.x - tb.first[q]) * blockDim.x + threadIdx.x;
  block_min_to(i < tb.g[q].count ? step_sym_one(tb.g[q], i, s, z, ds, dz) : INFINITY, partial);
}

// PSD: grid-stride over the cones with at most PSD_STEP_GRID blocks, one
// partial minimum per block
constexpr int PSD_STEP_GRID = 2048;

// ---------------------------------------------------------------------------
// One wave per cone for the Jacobi-based PSD kernels (every side).  The k
// indices (padded to an even count kk with one that never rotates) are paired
// round-robin (circle method: index kk - 1 fixed, the others turning), so the
// kk/2 pairs of a round are disjoint and their rotations are applied at once;
// a sweep is kk - 1 rounds.  Matrices sit in LDS, row stride PW_LD.
// ---------------------------------------------------------------------------
constexpr int PW_LD = PSD_KLARGE + 1;
constexpr int PW_MAT = PSD_KLARGE * PW_LD;

__device__ inline void rr_pair(int kk, int r, int i, int& p, int& q) {
  if (i == 0) {
    p = kk - 1;
    q = r;
  } else {
    p = (r + i) % (kk - 1);
    q = (r - i + (kk - 1)) % (kk - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// (i, j) of entry e of the packed triangle i >= j (row by row)
__device__ inline void tri_index(int e, int& i, int& j) {
  i = (int)((sqrt(8.0 * e + 1.0) - 1.0) / 2.0);
  while (i * (i + 1) / 2 > e) --i;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  j = e - i * (i + 1) / 2;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// X = smat(v) (k x k, symmetric)
__device__ inline void wave_smat(const double* v, int k, double* X, int lane) {
  const int sd = k * (k + 1) / 2;
  for (int p = lane; p < sd; p += 64) {
    int j, i;
    tri_index(p, j, i);   // svec: column j, rows i <= j
    const double x = v[p] * (i == j ? 1.0 : 0.70710678118654752440);
    X[i * PW_LD + j] = x;
    X[j * PW_LD + i] = x;
  }
}

// lower Cholesky in place (upper part zeroed); false (on every lane) when a
// pivot is not positive
__device__ bool wave_chol(double* A, int k, int lane) {
  for (int j = 0; j < k; ++j) {
    __syncthreads();
    const double d = A[j * PW_LD + j];
    if (!(d > 0.0)) return false;
    const double r = sqrt(d);
    __syncthreads();
    if (lane == 0) A[j * PW_LD + j] = r;
    for (int i = j + 1 + lane; i < k; i += 64) A[i * PW_LD + j] /= r;
    __syncthreads();
    const int t = k - j - 1;
    for (int e = lane; e < t * (t + 1) / 2; e += 64) {
      int i, l;
      tri_index(e, i, l);
      i += j + 1;
      l += j + 1;
      A[i * PW_LD + l] -= A[i * PW_LD + j] * A[l * PW_LD + j];
    }
  }
  __syncthreads();
  for (int e = lane; e < k * k; e += 64)
    if (e / k < e % k) A[(e / k) * PW_LD + e % k] = 0.0;
  __syncthreads();
  return true;
}

// smallest eigenvalue of the symmetric A (destroyed): parallel cyclic Jacobi.
// An off-diagonal entry at most 1e-18 |A|_F moves no eigenvalue by more than
// rounding does, so it is not rotated; the sweeps end on a sweep without
// rotations (quadratic convergence: a handful), or after 60.
__device__ double wave_min_eig(double* A, int k, int lane, double* rc, double* rs, int* rp, int* rq, int* flag) {
  double tot = 0;
  for (int e = lane; e < k * k; e += 64) tot += sq(A[(e / k) * PW_LD + e % k]);
  const double small = 1e-18 * sqrt(wave_sum(tot));
  const int kk = (k + 1) & ~1, np = kk / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    __syncthreads();
    if (lane == 0) *flag = 0;
    for (int r = 0; r < kk - 1; ++r) {
      __syncthreads();
      if (lane < np) {
        int p, q;
        rr_pair(kk, r, lane, p, q);
        double c = 1.0, sn = 0.0;
        if (q < k) {
          const double apq = A[p * PW_LD + q];
          if (fabs(apq) > small) {
            const double theta = (A[q * PW_LD + q] - A[p * PW_LD + p]) / (2.0 * apq);
            const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = c * t;
            *flag = 1;
          }
        }
        rp[lane] = p;
        rq[lane] = q;
        rc[lane] = c;
        rs[lane] = sn;
      }
      __syncthreads();
      for (int e = lane; e < k * np; e += 64) {   // A <- A J: columns p, q of every pair
        const int row = e / np, pi = e % np, p = rp[pi], q = rq[pi];
        if (q >= k || rs[pi] == 0.0) continue;
        const double arp = A[row * PW_LD + p], arq = A[row * PW_LD + q];
        A[row * PW_LD + p] = rc[pi] * arp - rs[pi] * arq;
        A[row * PW_LD + q] = rs[pi] * arp + rc[pi] * arq;
      }
      __syncthreads();
      for (int e = lane; e < k * np; e += 64) {   // A <- J' A: rows p, q
        const int col = e / np, pi = e % np, p = rp[pi], q = rq[pi];
        if (q >= k || rs[pi] == 0.0) continue;
        const double apc = A[p * PW_LD + col], aqc = A[q * PW_LD + col];
        A[p * PW_LD + col] = rc[pi] * apc - rs[pi] * aqc;
        A[q * PW_LD + col] = rs[pi] * apc + rc[pi] * aqc;
      }
    }
    __syncthreads();
    if (!*flag) break;
  }
  double m = INFINITY;
  for (int i = lane; i < k; i += 64) m = fmin(m, A[i * PW_LD + i]);
  return wave_min(m);
}

// one-sided Jacobi (Hestenes) on the columns of B (k x k): on return the
// columns are orthogonal and W accumulates B_in W = B_out.  Four lanes per
// pair, each summing and rotating rows sub, sub + 4, ...; a pair is skipped
// when |b_p'b_q| <= 1e-16 |b_p||b_q| (as the exp/pow Jacobi does).
__device__ void wave_jacobi_cols(double* B, int k, double* W, int lane, int* flag) {
  for (int e = lane; e < k * k; e += 64) W[(e / k) * PW_LD + e % k] = (e / k == e % k) ? 1.0 : 0.0;
  const int kk = (k + 1) & ~1, np = kk / 2, grp = lane >> 2, sub = lane & 3;
  for (int sweep = 0; sweep < 60; ++sweep) {
    __syncthreads();
    if (lane == 0) *flag = 0;
    for (int r = 0; r < kk - 1; ++r) {
      __syncthreads();
      if (grp >= np) continue;
      int p, q;
      rr_pair(kk, r, grp, p, q);
      if (q >= k) continue;
      double a = 0, b = 0, gg = 0;
      for (int row = sub; row < k; row += 4) {
        const double bp = B[row * PW_LD + p], bq = B[row * PW_LD + q];
        a += bp * bp;
        b += bq * bq;
        gg += bp * bq;
      }
      for (int off = 1; off < 4; off <<= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
        gg += __shfl_xor(gg, off, 64);
      }
      if (gg == 0.0 || fabs(gg) <= 1e-15 * sqrt(a * b)) continue;   // orthogonal to a few ulps
      const double zeta = (b - a) / (2.0 * gg);
      const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
      for (int row = sub; row < k; row += 4) {
        const double bp = B[row * PW_LD + p], bq = B[row * PW_LD + q];
        B[row * PW_LD + p] = cs * bp - sn * bq;
        B[row * PW_LD + q] = sn * bp + cs * bq;
        const double wp = W[row * PW_LD + p], wq = W[row * PW_LD + q];
        W[row * PW_LD + p] = cs * wp - sn * wq;
        W[row * PW_LD + q] = sn * wp + cs * wq;
      }
      if (sub == 0) *flag = 1;
    }
    __syncthreads();
    if (!*flag) break;
  }
  __syncthreads();
}

// C = op(X) op(Y) over the wave (entry per lane); tx / ty transpose X / Y
__device__ inline void wave_mm(const double* X, bool tx, const double* Y, bool ty, int k, double* C, int lane) {
  for (int e = lane; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    double acc = 0;
    for (int p = 0; p < k; ++p)
      acc += (tx ? X[p * PW_LD + i] : X[i * PW_LD + p]) * (ty ? Y[j * PW_LD + p] : Y[p * PW_LD + j]);
    C[i * PW_LD + j] = acc;
  }
  __syncthreads();
}

// PSD scaling, one wave per cone: Cholesky factors L_s, L_z; the SVD of
// L_z' L_s = U diag(lam) V' gives R = L_s V lam^-1/2 and R^-1 = lam^-1/2 U' L_z';
// a second one-sided Jacobi on R' gives M = R R' = Q diag(m) Q'.  State
// fields: R (k*k row-major) | R^-1 | Q | lambda (k) | m (k)
__global__ __launch_bounds__(64) void k_psd_scale_wave(SegDev g, const double* __restrict__ s,
                                                       const double* __restrict__ z, double* __restrict__ hdiag) {
  __shared__ double Ls[PW_MAT], Lz[PW_MAT], B[PW_MAT], W[PW_MAT], R[PW_MAT], Ri[PW_MAT], lam[PSD_KLARGE],
      m[PSD_KLARGE];
  __shared__ int flag;
  const int lane = threadIdx.x, k = g.k, sd = g.dim;
  const int64_t N = g.count, kk = (int64_t)k * k;
  for (int64_t c = blockIdx.x; c < N; c += gridDim.x) {
    __syncthreads();
    wave_smat(s + g.base + c * sd, k, Ls, lane);
    wave_smat(z + g.base + c * sd, k, Lz, lane);
    wave_chol(Ls, k, lane);
    wave_chol(Lz, k, lane);
    wave_mm(Lz, true, Ls, false, k, B, lane);   // B = Lz' Ls
    wave_jacobi_cols(B, k, W, lane, &flag);     // B W = U diag(lam), V = W
    if (lane < k) {
      double acc = 0;
      for (int r = 0; r < k; ++r) acc += B[r * PW_LD + lane] * B[r * PW_LD + lane];
      lam[lane] = sqrt(acc);
    }
    __syncthreads();
    // R = Ls V lam^-1/2 ; Rinv = lam^-1/2 U' Lz' with U = B diag(1/lam)
    for (int e = lane; e < k * k; e += 64) {
      const int i = e / k, j = e % k;
      double acc = 0, acc2 = 0;
      for (int p = 0; p < k; ++p) {
        acc += Ls[i * PW_LD + p] * W[p * PW_LD + j];
        acc2 += (B[p * PW_LD + i] / lam[i]) * Lz[j * PW_LD + p];
      }
      R[i * PW_LD + j] = acc / sqrt(lam[j]);
      Ri[i * PW_LD + j] = acc2 / sqrt(lam[i]);
    }
    __syncthreads();
    // M = R R' = Q diag(m) Q': one-sided Jacobi on the columns of R' (in Ls) gives Q (in W)
    for (int e = lane; e < k * k; e += 64) Ls[(e / k) * PW_LD + e % k] = R[(e % k) * PW_LD + e / k];
    __syncthreads();
    wave_jacobi_cols(Ls, k, W, lane, &flag);
    if (lane < k) {
      double acc = 0;
      for (int r = 0; r < k; ++r) acc += Ls[r * PW_LD + lane] * Ls[r * PW_LD + lane];
      m[lane] = acc;
    }
    for (int e = lane; e < k * k; e += 64) {
      const int i = e / k, j = e % k;
      g.state[(int64_t)e * N + c] = R[i * PW_LD + j];
      g.state[(kk + e) * N + c] = Ri[i * PW_LD + j];
      g.state[(2 * kk + e) * N + c] = W[i * PW_LD + j];
    }
    __syncthreads();
    if (lane < k) {
      g.state[(3 * kk + lane) * N + c] = lam[lane];
      g.state[(3 * kk + k + lane) * N + c] = m[lane];
    }
    wave_mm(R, false, R, true, k, B, lane);     // Mm = R R'
    for (int p = lane; p < sd; p += 64) {       // diag of H in svec coordinates
      int b, a;
      tri_index(p, b, a);
      const double v = (a == b) ? sq(B[a * PW_LD + a])
                                : (B[a * PW_LD + a] * B[b * PW_LD + b] + sq(B[a * PW_LD + b]));
      hdiag[g.base + c * sd + p] = v;
    }
  }
}

// combined-step d_s of a PSD cone (as k_psd_ds), one wave per cone:
//   A = R^-1 dS R^-T, B = R' dZ R, V = (A B + B A)/2 + diag(lam^2) - sm I,
//   X_ij = 2 V_ij / (lam_i + lam_j), ds = svec(R X R')
__global__ __launch_bounds__(64) void k_psd_ds_wave(SegDev g, const double* __restrict__ dsa,
                                                    const double* __restrict__ dza, double sm,
                                                    double* __restrict__ ds) {
  __shared__ double R[PW_MAT], Ri[PW_MAT], dS[PW_MAT], dZ[PW_MAT], T1[PW_MAT], Aa[PW_MAT], Bb[PW_MAT],
      lam[PSD_KLARGE];
  const int lane = threadIdx.x, k = g.k, sd = g.dim;
  const int64_t N = g.count, kk = (int64_t)k * k;
  for (int64_t c = blockIdx.x; c < N; c += gridDim.x) {
    __syncthreads();
    for (int e = lane; e < k * k; e += 64) {
      R[(e / k) * PW_LD + e % k] = g.state[(int64_t)e * N + c];
      Ri[(e / k) * PW_LD + e % k] = g.state[(kk + e) * N + c];
    }
    if (lane < k) lam[lane] = g.state[(3 * kk + lane) * N + c];
    wave_smat(dsa + g.base + c * sd, k, dS, lane);
    wave_smat(dza + g.base + c * sd, k, dZ, lane);
    __syncthreads();
    wave_mm(Ri, false, dS, false, k, T1, lane);   // Ri dS
    wave_mm(T1, false, Ri, true, k, Aa, lane);    // (Ri dS) Ri'
    wave_mm(R, true, dZ, false, k, T1, lane);     // R' dZ
    wave_mm(T1, false, R, false, k, Bb, lane);    // (R' dZ) R
    // V on the upper triangle, mirrored, so X is exactly symmetric before the
    // large 1/(lam_i + lam_j) factors
    for (int e = lane; e < k * k; e += 64) {
      const int r = e / k, j = e % k;
      if (j < r) continue;
      double acc = 0;
      for (int p = 0; p < k; ++p)
        acc += Aa[r * PW_LD + p] * Bb[p * PW_LD + j] + Bb[r * PW_LD + p] * Aa[p * PW_LD + j];
      double v = 0.5 * acc;
      if (r == j) v += lam[r] * lam[r] - sm;
      const double x = 2.0 * v / (lam[r] + lam[j]);
      dS[r * PW_LD + j] = x;   // dS and dZ are free now
      dS[j * PW_LD + r] = x;
    }
    __syncthreads();
    wave_mm(R, false, dS, false, k, T1, lane);    // R X
    wave_mm(T1, false, R, true, k, dZ, lane);     // (R X) R'
    for (int p = lane; p < sd; p += 64) {
      int j, i;
      tri_index(p, j, i);
      ds[g.base + c * sd + p] = dZ[i * PW_LD + j] * (i == j ? 1.0 : 1.41421356237309504880);
    }
  }
}

// largest alpha with x + alpha dx PSD (INFINITY if unbounded): Cholesky
// L L' = x, then the smallest eigenvalue of L^-1 dx L^-T
__device__ double wave_step_one(const double* x, const double* dx, int k, int lane, double* L, double* D, double* T,
                                double* rc, double* rs, int* rp, int* rq, int* flag) {
  __syncthreads();
  wave_smat(x, k, L, lane);
  wave_smat(dx, k, D, lane);
  if (!wave_chol(L, k, lane)) return 0.0;
  // Y = L^-1 D (lane j owns column j), then Z = L^-1 Y', T = (Z + Z')/2
  if (lane < k)
    for (int i = 0; i < k; ++i) {
      double v = D[i * PW_LD + lane];
      for (int p = 0; p < i; ++p) v -= L[i * PW_LD + p] * D[p * PW_LD + lane];
      D[i * PW_LD + lane] = v / L[i * PW_LD + i];
    }
  __syncthreads();
  if (lane < k)
    for (int i = 0; i < k; ++i) {
      double v = D[lane * PW_LD + i];
      for (int p = 0; p < i; ++p) v -= L[i * PW_LD + p] * T[p * PW_LD + lane];
      T[i * PW_LD + lane] = v / L[i * PW_LD + i];
    }
  __syncthreads();
  for (int e = lane; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    L[i * PW_LD + j] = 0.5 * (T[i * PW_LD + j] + T[j * PW_LD + i]);
  }
  const double lmin = wave_min_eig(L, k, lane, rc, rs, rp, rq, flag);
  return (lmin < 0.0) ? -1.0 / lmin : INFINITY;
}

// one wave per cone: per-workgroup minimum over its cones, or per cone
// (capped at amax) when per_cone
__global__ __launch_bounds__(64) void k_step_psd_wave(SegDev g, const double* __restrict__ s,
                                                      const double* __restrict__ z, const double* __restrict__ ds,
                                                      const double* __restrict__ dz, double amax, int per_cone,
                                                      double* __restrict__ out) {
  __shared__ double L[PW_MAT], D[PW_MAT], T[PW_MAT], rc[PSD_KLARGE / 2], rs[PSD_KLARGE / 2];
  __shared__ int rp[PSD_KLARGE / 2], rq[PSD_KLARGE / 2], flag;
  const int lane = threadIdx.x, sd = g.dim;
  double best = INFINITY;
  if (per_cone) {
    for (int64_t c = blockIdx.x; c < g.count; c += gridDim.x) {
      const int64_t o = g.base + c * sd;
      const double a1 = wave_step_one(s + o, ds + o, g.k, lane, L, D, T, rc, rs, rp, rq, &flag);
      const double a2 = wave_step_one(z + o, dz + o, g.k, lane, L, D, T, rc, rs, rp, rq, &flag);
      if (lane == 0) out[c] = fmin(amax, fmin(a1, a2));
    }
    return;
  }
  // the minimum over all cones: the s and z halves of a cone are separate
  // tasks, so twice as many waves share the chip
  for (int64_t t = blockIdx.x; t < 2 * g.count; t += gridDim.x) {
    const int64_t o = g.base + (t >> 1) * sd;
    const bool zh = (t & 1) != 0;
    best = fmin(best, wave_step_one((zh ? z : s) + o, (zh ? dz : ds) + o, g.k, lane, L, D, T, rc, rs, rp, rq, &flag));
  }
  if (lane == 0) out[blockIdx.x] = best;
}

int cone_step_sym(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz,
                  double* partial, hipStream_t st) {
  if (g.count == 0 || g.kind == HC_CONE_ZERO || g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW) return 0;
  if (soc_large(g.kind, g.dim)) return lsoc_step(g, s, z, ds, dz, INFINITY, false, partial, st);
  if (g.kind == HC_CONE_PSD) {
    const int nbp = (int)std::min<int64_t>(2 * g.count, PSD_STEP_GRID);
    hipLaunchKernelGGL(k_step_psd_wave, dim3(nbp), dim3(64), 0, st, g, s, z, ds, dz, INFINITY, 0, partial);
    HC_LAUNCH_CHECK();
    return nbp;
  }
  const int nb = cone_blocks(g);
  hipLaunchKernelGGL(k_step_sym, dim3(nb), dim3(CONE_BLOCK), 0, st, g, s, z, ds, dz, partial);
  HC_LAUNCH_CHECK();
  return nb;
}

int64_t cone_step_sym_all(const std::vector<SegDev>& segs, const double* s, const double* z, const double* ds,
                          const double* dz, double* partial, hipStream_t st) {
  int64_t off = 0;
  SegTable tb{};
  int nb = 0;
  auto flush = [&]() {
    if (tb.nseg == 0) return;
    tb.first[tb.nseg] = nb;
    hipLaunchKernelGGL(k_step_sym_fused, dim3((unsigned)nb), dim3(CONE_BLOCK), 0, st, tb, s, z, ds, dz,
                       partial + off);
    HC_LAUNCH_CHECK();
    off += nb;
    tb.nseg = 0;
    nb = 0;
  };
  for (const SegDev& g : segs) {
    if (g.count == 0 || g.kind == HC_CONE_ZERO || g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW) continue;
    if (!lane_per_cone(g)) {
      off += cone_step_sym(g, s, z, ds, dz, partial + off, st);
      continue;
    }
    if (tb.nseg == FUSED_SEGS) flush();
    tb.g[tb.nseg] = g;
    tb.first[tb.nseg] = nb;
    tb.nseg++;
    nb += (int)ceil_div(g.count, CONE_BLOCK);
  }
  flush();
  return off;
}

// trial t is a0 r^t, the products formed in sequence (as the host forms them)
__global__ __launch_bounds__(CONE_BLOCK) void k_trial_nonsym(SegDev g, const double* __restrict__ s, const double* __restrict__ z,
                               const double* __restrict__ ds, const double* __restrict__ dz, double a0,
                               double ratio, int ntrial,
                               int check_nbhd, double beta, double c0, double c1, double c2, double nu1,
                               unsigned long long* __restrict__ partial) {
  __shared__ unsigned long long red[CONE_BLOCK];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  unsigned long long mask = (ntrial >= 64) ? ~0ull : ((1ull << ntrial) - 1ull);
  if (i < N) {
    const bool is_exp = (g.kind == HC_CONE_EXP);
    const double al = is_exp ? 0.0 : g.alpha[i];
    double sv[3], zv[3], dsv[3], dzv[3];
    for (int j = 0; j < 3; ++j) {
      sv[j] = s[g.base + j * N + i];
      zv[j] = z[g.base + j * N + i];
      dsv[j] = ds[g.base + j * N + i];
      dzv[j] = dz[g.base + j * N + i];
    }
    mask = 0;
    double a = a0;
    for (int t = 0; t < ntrial; ++t, a *= ratio) {
      double sa[3], za[3];
      for (int j = 0; j < 3; ++j) {
        sa[j] = sv[j] + a * dsv[j];
        za[j] = zv[j] + a * dzv[j];
      }
      bool ok = is_exp ? (exp_primal_in(sa) && exp_dual_in(za)) : (pow_primal_in(sa, al) && pow_dual_in(za, al));
      if (ok && check_nbhd) {
        double gz[3], zt[3];
        if (is_exp) exp_grad(za, gz); else pow_grad(za, al, gz);
        const bool cok = is_exp ? exp_conj(sa, zt) : pow_conj(sa, al, zt);
        const double inner = -(gz[0] * zt[0] + gz[1] * zt[1] + gz[2] * zt[2]);
        const double mua = (c0 + a * (c1 + a * c2)) / nu1;
        ok = cok && (3.0 / inner >= beta * mua);
      }
      if (ok) mask |= (1ull << t);
    }
  }
  red[threadIdx.x] = mask;
  __syncthreads();
  for (int off = CONE_BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] &= red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

int cone_trial_nonsym(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz,
                      double a0, double ratio, int ntrial, int check_nbhd, double beta, double c0, double c1,
                      double c2, double nu1, unsigned long long* partial, hipStream_t st) {
  if (g.count == 0) return 0;
  const int nb = cone_blocks(g);
  hipLaunchKernelGGL(k_trial_nonsym, dim3(nb), dim3(CONE_BLOCK), 0, st, g, s, z, ds, dz, a0, ratio, std::min(ntrial, 8),
                     check_nbhd, beta, c0, c1, c2, nu1, partial);
  HC_LAUNCH_CHECK();
  return nb;
}

// ===========================================================================
// initial point helpers
// ===========================================================================
__global__ void k_cone_unit(SegDev g, double* __restrict__ v, double e0, double e1, double e2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  if (i >= N) return;
  switch (g.kind) {
    case HC_CONE_ZERO: v[g.base + i] = 0.0; break;
    case HC_CONE_NONNEG: v[g.base + i] = 1.0; break;
    case HC_CONE_SOC:
      for (int j = 0; j < g.dim; ++j) v[g.base + j * N + i] = (j == 0) ? 1.0 : 0.0;
      break;
    case HC_CONE_EXP:
      v[g.base + i] = e0; v[g.base + N + i] = e1; v[g.base + 2 * N + i] = e2;
      break;
    case HC_CONE_POW: {
      const double a = g.alpha[i];
      v[g.base + i] = sqrt(1.0 + a); v[g.base + N + i] = sqrt(2.0 - a); v[g.base + 2 * N + i] = 0.0;
      break;
    }
    case HC_CONE_PSD: {
      int p = 0;
      for (int j = 0; j < g.k; ++j)
        for (int r = 0; r <= j; ++r, ++p) v[g.base + i * g.dim + p] = (r == j) ? 1.0 : 0.0;
      break;
    }
  }
}

// the unit point of the exp cone: u = -grad f(u), by Newton on the host
static void exp_unit_point(double* u) {
  double z[3] = {-1.0513839, 0.5564096, 1.2589679};
  for (int it = 0; it < 60; ++it) {
    // F(z) = z + grad f(z); J = I + Hess f(z) (closed forms, host copy)
    const double z1 = z[0], z2 = z[1], z3 = z[2];
    const double ell = std::log(z3 / (-z1));
    const double psi = z2 - z1 - z1 * ell;
    const double g[3] = {ell / psi - 1.0 / z1, -1.0 / psi, (z1 / z3) / psi - 1.0 / z3};
    const double dps[3] = {-ell, 1.0, -z1 / z3};
    const double D2[9] = {1.0 / z1, 0.0, -1.0 / z3, 0.0, 0.0, 0.0, -1.0 / z3, 0.0, z1 / (z3 * z3)};
    double J[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        J[a * 3 + b] = (a == b ? 1.0 : 0.0) - D2[a * 3 + b] / psi + dps[a] * dps[b] / (psi * psi) +
                       (a == b && a == 0 ? 1.0 / (z1 * z1) : 0.0) + (a == b && a == 2 ? 1.0 / (z3 * z3) : 0.0);
    double F[3] = {z[0] + g[0], z[1] + g[1], z[2] + g[2]};
    // solve J d = F (Cramer)
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    double d[3];
    for (int c = 0; c < 3; ++c) {
      double M[9];
      for (int a = 0; a < 9; ++a) M[a] = J[a];
      for (int a = 0; a < 3; ++a) M[a * 3 + c] = F[a];
      d[c] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
              M[2] * (M[3] * M[7] - M[4] * M[6])) / det;
    }
    for (int c = 0; c < 3; ++c) z[c] -= d[c];
  }
  for (int c = 0; c < 3; ++c) u[c] = z[c];
}

void cone_unit(const SegDev& g, double* v, hipStream_t st) {
  if (g.count == 0) return;
  struct UnitPoint {
    double u[3];
    UnitPoint() { exp_unit_point(u); }
  };
  static const UnitPoint eu;   // computed once, thread-safe (solvers on several threads)
  hipLaunchKernelGGL(k_cone_unit, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, v, eu.u[0], eu.u[1], eu.u[2]);
  HC_LAUNCH_CHECK();
}

__global__ void k_max_neg_eig(SegDev g, const double* __restrict__ v, double* __restrict__ partial) {
  __shared__ double red[CONE_BLOCK];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  double a = -INFINITY;
  if (i < N) {
    if (g.kind == HC_CONE_NONNEG) {
      a = -v[g.base + i];
    } else if (g.kind == HC_CONE_SOC) {
      double nx = 0;
      for (int j = 1; j < g.dim; ++j) nx += sq(v[g.base + j * N + i]);
      a = sqrt(nx) - v[g.base + i];
    }
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = CONE_BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// PSD: one wave per cone (Jacobi eigenvalues as in the step kernel),
// grid-stride over the cones, one partial maximum per workgroup
__global__ __launch_bounds__(64) void k_psd_max_neg_eig_wave(SegDev g, const double* __restrict__ v,
                                                             double* __restrict__ partial) {
  __shared__ double X[PW_MAT], rc[PSD_KLARGE / 2], rs[PSD_KLARGE / 2];
  __shared__ int rp[PSD_KLARGE / 2], rq[PSD_KLARGE / 2], flag;
  const int lane = threadIdx.x;
  double a = -INFINITY;
  for (int64_t c = blockIdx.x; c < g.count; c += gridDim.x) {
    __syncthreads();
    wave_smat(v + g.base + c * g.dim, g.k, X, lane);
    __syncthreads();
    a = fmax(a, -wave_min_eig(X, g.k, lane, rc, rs, rp, rq, &flag));
  }
  if (lane == 0) partial[blockIdx.x] = a;
}

int cone_max_neg_eig(const SegDev& g, const double* v, double* partial, hipStream_t st) {
  if (g.count == 0 || !(g.kind == HC_CONE_NONNEG || g.kind == HC_CONE_SOC || g.kind == HC_CONE_PSD)) return 0;
  if (soc_large(g.kind, g.dim)) return lsoc_max_neg_eig(g, v, partial, st);
  if (g.kind == HC_CONE_PSD) {
    const int nbp = (int)std::min<int64_t>(g.count, PSD_STEP_GRID);
    hipLaunchKernelGGL(k_psd_max_neg_eig_wave, dim3(nbp), dim3(64), 0, st, g, v, partial);
    HC_LAUNCH_CHECK();
    return nbp;
  }
  const int nb = cone_blocks(g);
  hipLaunchKernelGGL(k_max_neg_eig, dim3(nb), dim3(CONE_BLOCK), 0, st, g, v, partial);
  HC_LAUNCH_CHECK();
  return nb;
}

__global__ void k_add_e(SegDev g, double a, double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  if (i >= N) return;
  if (g.kind == HC_CONE_NONNEG) v[g.base + i] += a;
  else if (g.kind == HC_CONE_SOC) v[g.base + i] += a;
  else if (g.kind == HC_CONE_PSD) {
    int p = 0;
    for (int j = 0; j < g.k; ++j)
      for (int r = 0; r <= j; ++r, ++p)
        if (r == j) v[g.base + i * g.dim + p] += a;
  }
}

void cone_add_e(const SegDev& g, double a, double* v, hipStream_t st) {
  if (g.count == 0) return;
  hipLaunchKernelGGL(k_add_e, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, a, v);
  HC_LAUNCH_CHECK();
}

}  // namespace hc

namespace hc {

// ===========================================================================
// kernel test support: per-cone views of the state and per-cone steps
// ===========================================================================
__global__ void k_test_extract(SegDev g, const double* __restrict__ s, int what, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  if (i >= N) return;
  if (what == 2) {   // exp/pow branch
    out[i] = (g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW) ? g.state[NS_BR * N + i] : 0.0;
    return;
  }
  switch (g.kind) {
    case HC_CONE_ZERO: out[i] = 0.0; break;
    case HC_CONE_NONNEG: out[i] = g.state[i]; break;
    case HC_CONE_SOC:
      for (int j = 0; j < g.dim; ++j) out[j * N + i] = g.state[(g.dim + 1 + j) * N + i];
      break;
    case HC_CONE_EXP:
    case HC_CONE_POW: {
      double sv[3], zt[3] = {NAN, NAN, NAN};
      for (int j = 0; j < 3; ++j) sv[j] = s[g.base + j * N + i];
      if (g.kind == HC_CONE_EXP) exp_conj(sv, zt); else pow_conj(sv, g.alpha[i], zt);
      for (int j = 0; j < 3; ++j) out[j * N + i] = zt[j];
      break;
    }
    case HC_CONE_PSD: {
      const int64_t kk = (int64_t)g.k * g.k;
      for (int j = 0; j < g.dim; ++j) out[i * g.dim + j] = (j < g.k) ? g.state[(3 * kk + j) * N + i] : 0.0;
      break;
    }
  }
}

void cone_test_extract(const SegDev& g, const double* s, int what, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_test_extract, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, s, what, out);
  HC_LAUNCH_CHECK();
}

__global__ void k_test_step(SegDev g, const double* __restrict__ s, const double* __restrict__ z,
                            const double* __restrict__ ds, const double* __restrict__ dz, double amax,
                            double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  if (i >= N) return;
  double a = amax;
  if (g.kind == HC_CONE_NONNEG) {
    const int64_t r = g.base + i;
    if (ds[r] < 0.0) a = fmin(a, -s[r] / ds[r]);
    if (dz[r] < 0.0) a = fmin(a, -z[r] / dz[r]);
  } else if (g.kind == HC_CONE_SOC) {
    double xs[SOC_DMAX], xds[SOC_DMAX], xz[SOC_DMAX], xdz[SOC_DMAX];
    for (int j = 0; j < g.dim; ++j) {
      xs[j] = s[g.base + j * N + i];
      xds[j] = ds[g.base + j * N + i];
      xz[j] = z[g.base + j * N + i];
      xdz[j] = dz[g.base + j * N + i];
    }
    a = fmin(a, fmin(soc_step_one(xs, xds, g.dim), soc_step_one(xz, xdz, g.dim)));
  } else if (g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW) {
    const double al = (g.kind == HC_CONE_POW) ? g.alpha[i] : 0.0;
    double t = amax;
    a = 0.0;
    for (int j = 0; j < 64; ++j) {
      double sa[3], za[3];
      for (int c = 0; c < 3; ++c) {
        sa[c] = s[g.base + c * N + i] + t * ds[g.base + c * N + i];
        za[c] = z[g.base + c * N + i] + t * dz[g.base + c * N + i];
      }
      const bool ok = (g.kind == HC_CONE_EXP) ? (exp_primal_in(sa) && exp_dual_in(za))
                                              : (pow_primal_in(sa, al) && pow_dual_in(za, al));
      if (ok) {
        a = t;
        break;
      }
      t *= 0.8;
    }
  }
  out[i] = a;
}

void cone_test_step(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz,
                    double amax, double* out, hipStream_t st) {
  if (soc_large(g.kind, g.dim)) {
    lsoc_step(g, s, z, ds, dz, amax, true, out, st);
    return;
  }
  if (g.kind == HC_CONE_PSD) {
    hipLaunchKernelGGL(k_step_psd_wave, dim3((unsigned)std::min<int64_t>(g.count, PSD_STEP_GRID)), dim3(64), 0, st, g,
                       s, z, ds, dz, amax, 1, out);
    HC_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL(k_test_step, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, s, z, ds, dz, amax, out);
  HC_LAUNCH_CHECK();
}

}  // namespace hc
