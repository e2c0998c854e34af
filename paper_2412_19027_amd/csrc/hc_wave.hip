// Wave-per-problem engine (see hc_wave.h): device code and slot layout.
//
// One workgroup of 64 lanes (a single wavefront) per problem.  Vectors are
// walked lane-strided; a __syncthreads() closes every phase that later lanes
// read through global memory (for a one-wave workgroup it is a wait for the
// wave's own memory operations, not a cross-wave barrier).  The band Cholesky
// and the triangular solves keep their active rows in LDS (a circular window
// of WAVE_WB rows) and fetch the rows of the next WAVE_PB steps while the
// current ones are computed.
#include "hc_cones.h"
#include "hc_soc_math.h"
#include "hc_wave.h"

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>

namespace hc {

namespace {

constexpr int WL = 64;   // lanes per slot

// work vectors of max(n, m) doubles
enum WaveVec {
  WV_X = 0, WV_S, WV_Z, WV_PX, WV_AX, WV_ATZ, WV_RDV, WV_RPV, WV_X2, WV_Z2, WV_X1, WV_Z1, WV_DX, WV_DZ, WV_DSV,
  WV_DSRHS, WV_DXA, WV_DZA, WV_DSA, WV_R1, WV_R2, WV_IRX, WV_IRZ, WV_IRXN, WV_IRZN, WV_IRBX, WV_IRBZ, WV_IRRX,
  WV_IRRZ, WV_KX, WV_KZ, WV_T1, WV_T2, WV_U1, WV_W1, WV_COUNT
};

__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }

// Values the whole wave shares, made visibly uniform (scalar registers, scalar
// branches), and pointers into the slot's blob as global-memory pointers
// (global loads count only against the vector-memory counter, so LDS waits do
// not wait for them and loads issued ahead stay in flight).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
using lptr = __attribute__((address_space(3))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) {
  const unsigned long long u = (unsigned long long)p;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return (gptr<T>)(((unsigned long long)hi << 32) | lo);
}

// the wave's own global-memory writes are visible to all its lanes after this
__device__ __forceinline__ void gsync() { __syncthreads(); }
// orders the wave's LDS accesses (the LDS executes one wave's instructions in order)
__device__ __forceinline__ void lsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wsum(double v) {
  for (int o = WL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WL);
  return v;
}
__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || b != b) ? NAN : fmax(a, b); }
__device__ __forceinline__ double wmax(double v) {
  for (int o = WL / 2; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o, WL));
  return v;
}
__device__ __forceinline__ double wmin(double v) {
  for (int o = WL / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WL));
  return v;
}

// ---------------------------------------------------------------- vectors
// Each lane walks its elements four at a time, the loads of a group issued
// together, so a wave keeps several memory accesses in flight per lane (one
// wave per problem has no other source of memory parallelism).
constexpr int UN = 4;

__device__ void v_fill(int n_, double a, double* y_) {
  const int n = uni(n_);
  const auto y = gp(y_);
  for (int i = lane_id(); i < n; i += WL) y[i] = a;
  gsync();
}
// o = a x + b y + c z (y, z optional)
__device__ void v_lin(int n_, double a, const double* x_, double b, const double* y_, double c, const double* z_,
                      double* o_) {
  const int n = uni(n_);
  const auto x = gp(x_), y = gp(y_), z = gp(z_);
  const auto o = gp(o_);
  for (int i0 = lane_id(); i0 < n; i0 += UN * WL) {
    double xv[UN], yv[UN], zv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + u * WL;
      xv[u] = i < n ? x[i] : 0.0;
      yv[u] = (y && i < n) ? y[i] : 0.0;
      zv[u] = (z && i < n) ? z[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + u * WL;
      double v = a * xv[u];
      if (y) v += b * yv[u];
      if (z) v += c * zv[u];
      if (i < n) o[i] = v;
    }
  }
  gsync();
}
__device__ void v_copy(int n, const double* x, double* y) { v_lin(n, 1.0, x, 0.0, nullptr, 0.0, nullptr, y); }
// y = a x + b y
__device__ void v_axpby(int n_, double a, const double* x_, double b, double* y_) {
  const int n = uni(n_);
  const auto x = gp(x_);
  const auto y = gp(y_);
  for (int i0 = lane_id(); i0 < n; i0 += UN * WL) {
    double xv[UN], yv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + u * WL;
      xv[u] = i < n ? x[i] : 0.0;
      yv[u] = i < n ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + u * WL;
      if (i < n) y[i] = a * xv[u] + b * yv[u];
    }
  }
  gsync();
}
__device__ double v_dot(int n_, const double* x_, const double* y_) {
  const int n = uni(n_);
  const auto x = gp(x_), y = gp(y_);
  double acc = 0.0;
  for (int i0 = lane_id(); i0 < n; i0 += UN * WL) {
    double xv[UN], yv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + u * WL;
      xv[u] = i < n ? x[i] : 0.0;
      yv[u] = i < n ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) acc += xv[u] * yv[u];
  }
  return wsum(acc);
}
// max |(x + yc y) w| (divide: / w); w and y optional
__device__ double v_maxabs(int n_, const double* x_, const double* w_ = nullptr, bool divide = false,
                           const double* y_ = nullptr, double yc = 0.0) {
  const int n = uni(n_);
  const auto x = gp(x_), w = gp(w_), y = gp(y_);
  double acc = 0.0;
  for (int i0 = lane_id(); i0 < n; i0 += UN * WL) {
    double xv[UN], yv[UN], wv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + u * WL;
      xv[u] = i < n ? x[i] : 0.0;
      yv[u] = (y && i < n) ? y[i] : 0.0;
      wv[u] = (w && i < n) ? w[i] : 1.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      double v = xv[u];
      if (y) v += yc * yv[u];
      if (w) v = divide ? v / wv[u] : v * wv[u];
      acc = nanmax(acc, fabs(v));
    }
  }
  return wmax(acc);
}
// y = alpha A x + beta y (CSR, lane per row; beta = 0 does not read y); a
// row's entries are taken four at a time (their column indices and values
// loaded together, then the four gathers of x), summed in order
__device__ void spmv(int rows_, const int32_t* rp_, const int32_t* ci_, const double* va_, const double* x_,
                     double* y_, double alpha, double beta) {
  const int rows = uni(rows_);
  const auto rp = gp(rp_), ci = gp(ci_);
  const auto va = gp(va_), x = gp(x_);
  const auto y = gp(y_);
  for (int r = lane_id(); r < rows; r += WL) {
    const int k0 = rp[r], k1 = rp[r + 1];
    double acc = 0.0;
    int k = k0;
    for (; k + UN <= k1; k += UN) {
      int cc[UN];
      double aa[UN], xx[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        cc[u] = ci[k + u];
        aa[u] = va[k + u];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) xx[u] = x[cc[u]];
#pragma unroll
      for (int u = 0; u < UN; ++u) acc += aa[u] * xx[u];
    }
    for (; k < k1; ++k) acc += va[k] * x[ci[k]];
    y[r] = (beta == 0.0) ? alpha * acc : alpha * acc + beta * y[r];
  }
  gsync();
}

// ---------------------------------------------------------------- cones
struct Cone {
  int o, d;        // first row, rows
  double* st;      // wbar (d), eta, lambda (d)
};
__device__ __forceinline__ Cone soc_cone(const WaveDesc& D, int c) {
  Cone k;
  k.o = D.nz + D.nn + D.soc_off[c];
  k.d = D.soc_off[c + 1] - D.soc_off[c];
  k.st = D.hst + D.nn + 2 * D.soc_off[c] + c;
  return k;
}

// scaling at (s, z): nonneg h = s / z; SOC the Nesterov-Todd point; diag(H)
__device__ void c_scale(const WaveDesc& D, const double* s, const double* z) {
  for (int r = lane_id(); r < D.nz; r += WL) D.hdiag[r] = 0.0;
  for (int i = lane_id(); i < D.nn; i += WL) {
    const int r = D.nz + i;
    const double h = s[r] / z[r];
    D.hst[i] = h;
    D.hdiag[r] = h;
  }
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    double sv[SOC_DMAX], zv[SOC_DMAX], wb[SOC_DMAX], lam[SOC_DMAX];
    for (int j = 0; j < k.d; ++j) {
      sv[j] = s[k.o + j];
      zv[j] = z[k.o + j];
    }
    const double eta = soc_nt_scale(sv, zv, k.d, wb, lam);
    for (int j = 0; j < k.d; ++j) {
      k.st[j] = wb[j];
      k.st[k.d + 1 + j] = lam[j];
    }
    k.st[k.d] = eta;
    const double e2 = eta * eta;
    for (int j = 0; j < k.d; ++j) D.hdiag[k.o + j] = e2 * (2.0 * wb[j] * wb[j] - (j == 0 ? 1.0 : -1.0));
  }
  gsync();
}

// H = I on the cone rows (0 on zero rows): the initial point's scaling
__device__ void c_identity(const WaveDesc& D) {
  for (int r = lane_id(); r < D.nz; r += WL) D.hdiag[r] = 0.0;
  for (int i = lane_id(); i < D.nn; i += WL) {
    D.hst[i] = 1.0;
    D.hdiag[D.nz + i] = 1.0;
  }
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    for (int j = 0; j < k.d; ++j) {
      k.st[j] = (j == 0) ? 1.0 : 0.0;
      k.st[k.d + 1 + j] = (j == 0) ? 1.0 : 0.0;
      D.hdiag[k.o + j] = 1.0;
    }
    k.st[k.d] = 1.0;
  }
  gsync();
}

// M = (H + delta I)^-1: one entry per zero/nonneg row, a full d x d block per SOC
__device__ void c_mblock(const WaveDesc& D, double delta) {
  for (int r = lane_id(); r < D.nz; r += WL) D.Mv[r] = 1.0 / delta;
  for (int i = lane_id(); i < D.nn; i += WL) D.Mv[D.nz + i] = 1.0 / (D.hst[i] + delta);
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    double wb[SOC_DMAX], u[SOC_DMAX];
    for (int j = 0; j < k.d; ++j) wb[j] = k.st[j];
    const SocSpec sp = soc_spec(wb, k.d, k.st[k.d]);
    for (int j = 1; j < k.d; ++j) u[j] = (sp.r > 0.0) ? wb[j] / sp.r : (j == 1 ? 1.0 : 0.0);
    const double fp = 1.0 / (sp.lp + delta), fm = 1.0 / (sp.lm + delta), fo = 1.0 / (sp.lo + delta);
    double* M = D.Mv + D.soc_moff[c];
    for (int a = 0; a < k.d; ++a)
      for (int b = 0; b <= a; ++b) {
        double v;
        if (a == 0) v = 0.5 * (fp + fm);
        else if (b == 0) v = 0.5 * (fp - fm) * u[a];
        else v = 0.5 * (fp + fm) * u[a] * u[b] + fo * ((a == b ? 1.0 : 0.0) - u[a] * u[b]);
        M[a * k.d + b] = v;
        M[b * k.d + a] = v;
      }
  }
  gsync();
}

// y = H x (mode 0) or (H + delta I)^-1 x (mode 1); with dsr: y = -dsr - H x
__device__ void c_apply(const WaveDesc& D, int mode, double delta, const double* x, const double* dsr, double* y) {
  for (int r = lane_id(); r < D.nz; r += WL) y[r] = dsr ? -dsr[r] : ((mode == 0) ? 0.0 : x[r] / delta);
  for (int i = lane_id(); i < D.nn; i += WL) {
    const int r = D.nz + i;
    const double h = D.hst[i];
    if (dsr) y[r] = -dsr[r] - h * x[r];
    else y[r] = (mode == 0) ? h * x[r] : x[r] / (h + delta);
  }
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    double wb[SOC_DMAX], xv[SOC_DMAX], yv[SOC_DMAX];
    for (int j = 0; j < k.d; ++j) {
      wb[j] = k.st[j];
      xv[j] = x[k.o + j];
    }
    const SocSpec sp = soc_spec(wb, k.d, k.st[k.d]);
    if (mode == 0)
      soc_spec_apply(wb, k.d, sp, sp.lp, sp.lm, sp.lo, xv, yv);
    else
      soc_spec_apply(wb, k.d, sp, 1.0 / (sp.lp + delta), 1.0 / (sp.lm + delta), 1.0 / (sp.lo + delta), xv, yv);
    for (int j = 0; j < k.d; ++j) y[k.o + j] = dsr ? -dsr[k.o + j] - yv[j] : yv[j];
  }
  gsync();
}

// combined-step d_s (eq. ds-correction-step)
__device__ void c_ds(const WaveDesc& D, const double* s, const double* z, const double* dsa, const double* dza,
                     double sm, double* ds) {
  for (int r = lane_id(); r < D.nz; r += WL) ds[r] = 0.0;
  for (int i = lane_id(); i < D.nn; i += WL) {
    const int r = D.nz + i;
    ds[r] = (s[r] * z[r] + dsa[r] * dza[r] - sm) / z[r];
  }
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    double wb[SOC_DMAX], lam[SOC_DMAX], a[SOC_DMAX], b[SOC_DMAX], x[SOC_DMAX];
    for (int j = 0; j < k.d; ++j) {
      wb[j] = k.st[j];
      lam[j] = k.st[k.d + 1 + j];
      a[j] = dsa[k.o + j];
      b[j] = dza[k.o + j];
    }
    soc_ds_one(wb, k.st[k.d], lam, a, b, k.d, sm, x);
    for (int j = 0; j < k.d; ++j) ds[k.o + j] = x[j];
  }
  gsync();
}

__device__ __forceinline__ double soc_step_x(const double* x, const double* dx, int d) {
  double a = dx[0] * dx[0], b = x[0] * dx[0], c = x[0] * x[0];
  for (int j = 1; j < d; ++j) {
    a -= dx[j] * dx[j];
    b -= x[j] * dx[j];
    c -= x[j] * x[j];
  }
  return soc_boundary_step(a, b, c);
}

// largest alpha keeping s + alpha ds and z + alpha dz in the closed cones
__device__ double c_step(const WaveDesc& D, const double* s, const double* z, const double* ds, const double* dz) {
  double a = INFINITY;
  for (int i = lane_id(); i < D.nn; i += WL) {
    const int r = D.nz + i;
    if (ds[r] < 0.0) a = fmin(a, -s[r] / ds[r]);
    if (dz[r] < 0.0) a = fmin(a, -z[r] / dz[r]);
  }
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    double xs[SOC_DMAX], xds[SOC_DMAX], xz[SOC_DMAX], xdz[SOC_DMAX];
    for (int j = 0; j < k.d; ++j) {
      xs[j] = s[k.o + j];
      xds[j] = ds[k.o + j];
      xz[j] = z[k.o + j];
      xdz[j] = dz[k.o + j];
    }
    a = fmin(a, fmin(soc_step_x(xs, xds, k.d), soc_step_x(xz, xdz, k.d)));
  }
  return wmin(a);
}

// max over cones of -lambda_min(v)
__device__ double c_max_neg_eig(const WaveDesc& D, const double* v) {
  double a = -INFINITY;
  for (int i = lane_id(); i < D.nn; i += WL) a = fmax(a, -v[D.nz + i]);
  for (int c = lane_id(); c < D.nsoc; c += WL) {
    const Cone k = soc_cone(D, c);
    double r2 = 0.0;
    for (int j = 1; j < k.d; ++j) r2 += v[k.o + j] * v[k.o + j];
    a = fmax(a, sqrt(r2) - v[k.o]);
  }
  for (int o = WL / 2; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, WL));
  return a;
}

// v += a e on the cone rows
__device__ void c_add_e(const WaveDesc& D, double a, double* v) {
  for (int i = lane_id(); i < D.nn; i += WL) v[D.nz + i] += a;
  for (int c = lane_id(); c < D.nsoc; c += WL) v[soc_cone(D, c).o] += a;
  gsync();
}

// ---------------------------------------------------------------- band Cholesky and solves
// lane k's value in every lane (k uniform)
__device__ __forceinline__ float wget(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double wget(double v, int k) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// lane t receives lane t + 1's value, lane 63 receives 0 (DPP wavefront shift)
__device__ __forceinline__ int wshl1_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float wshl1(float v) { return __int_as_float(wshl1_i(__float_as_int(v))); }
__device__ __forceinline__ double wshl1(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)wshl1_i((int)(unsigned)u);
  const unsigned hi = (unsigned)wshl1_i((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// S in band storage: column j holds S(j + t, j), t = 0..w, at Sb[j W + t].
// In place: L (the diagonal L_jj at t = 0) and dinv[j] = 1 / L_jj.  A pivot
// that is not positive is replaced by `fix` and counted.  Blocked by PB
// columns: the rows a block's columns reach (j0 .. j0 + PB - 1 + w) sit in a
// circular LDS window (row i at i mod WB, entry (i, c) at column slot
// c mod WB).  Lane r takes row j0 + r of the block's columns into registers,
// the PB columns are factored there (pivots and multipliers exchanged by
// readlane), the block's L goes out to Sb and to an LDS panel, and each lane
// then applies the block's rank-PB update to the rest of its row in the
// window.  Every entry receives its updates in column order, as in the
// column-by-column algorithm.
template <typename T>
__device__ int band_cholesky(T* Sb_, T* dinv_, int n_, int w_, T fix, T* win_) {
  constexpr int WB = WAVE_WB, PB = WAVE_PB, LD = WAVE_WB + 1, PLD = sizeof(T) == 8 ? 10 : 12;
  const lptr<T> win = (lptr<T>)win_;   // the kernel's LDS array: window, then panel
  const lptr<T> pl = win + WB * LD;    // row r of the block's columns of L (PB entries, stride PLD)
  const auto Sb = gp(Sb_);
  const auto dinv = gp(dinv_);
  const int n = uni(n_), w = uni(w_);
  const int lane = lane_id();
  const int W = w + 1;
  int hits = 0;
  // rows [0, w + PB) of the band
  for (int i = 0; i < min(n, w + PB); ++i)
    if (lane <= w && i - lane >= 0) win[(i & (WB - 1)) * LD + ((i - lane) & (WB - 1))] = Sb[(size_t)(i - lane) * W + lane];
  lsync();
  for (int j0 = 0; j0 < n; j0 += PB) {
    // rows entering the window after this block, fetched now
    T pf[PB];
#pragma unroll
    for (int s = 0; s < PB; ++s) {
      const int i = j0 + w + PB + s;
      pf[s] = (lane <= w && i < n && i - lane >= 0) ? Sb[(size_t)(i - lane) * W + lane] : T(0);
    }
    const int nb = min(PB, n - j0);
    const int r = lane, i = j0 + lane;
    const bool live = r < nb + w && i < n;   // a row the block's columns reach
    const lptr<T> row = win + (i & (WB - 1)) * LD;
    T P[PB];
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      const T v = row[(j0 + k) & (WB - 1)];
      P[k] = (live && k < nb && k <= r && r - k <= w) ? v : T(0);
    }
    // the block's columns, one after another
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      if (k < nb) {
        T d = wget(P[k], k);
        if (!(d > T(0))) {
          d = fix;
          ++hits;
        }
        const T ljj = sqrt(d);
        const T inv = T(1) / ljj;
        if (lane == 0) dinv[j0 + k] = inv;
        P[k] = (r == k) ? ljj : (r > k ? P[k] * inv : T(0));
#pragma unroll
        for (int c = k + 1; c < PB; ++c) {
          const T lc = wget(P[k], c);
          if (c < nb && r >= c) P[c] -= P[k] * lc;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      if (live && k < nb && r >= k && r - k <= w) Sb[(size_t)(j0 + k) * W + (r - k)] = P[k];
      pl[r * PLD + k] = P[k];
    }
    lsync();
    // rank-PB update of rows j0 + nb .. j0 + nb + w - 1 at columns from j0 + nb
    // on: entry (i, j0 + c) for c = r - dd, two at a time (reads first)
    const bool upd = live && r >= nb;
    for (int dd = 0; dd <= w; dd += 2) {
      const int c0 = r - dd, c1 = r - dd - 1;
      const bool u0 = upd && c0 >= nb, u1 = upd && c1 >= nb && dd + 1 <= w;
      const lptr<T> p0 = pl + (u0 ? c0 : 0) * PLD;
      const lptr<T> p1 = pl + (u1 ? c1 : 0) * PLD;
      T a0 = row[(j0 + c0) & (WB - 1)], a1 = row[(j0 + c1) & (WB - 1)];
      T q0[PB], q1[PB];
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        q0[k] = p0[k];
        q1[k] = p1[k];
      }
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        a0 -= P[k] * q0[k];
        a1 -= P[k] * q1[k];
      }
      if (u0) row[(j0 + c0) & (WB - 1)] = a0;
      if (u1) row[(j0 + c1) & (WB - 1)] = a1;
    }
#pragma unroll
    for (int s = 0; s < PB; ++s) {
      const int i2 = j0 + w + PB + s;
      if (lane <= w && i2 < n && i2 - lane >= 0) win[(i2 & (WB - 1)) * LD + ((i2 - lane) & (WB - 1))] = pf[s];
    }
    lsync();
  }
  gsync();
  return hits;
}

// L y = b then L' x = y, in place on b (global, n entries).  Both sweeps keep
// the w + 1 pending entries in registers (lane t: the entry t places ahead of
// the current column), take the current one from lane 0, subtract its
// multiples and shift the window down one lane; the next SB columns of L, the
// reciprocal pivots and the entries entering the window are loaded one block
// ahead, and each block's results are stored together at its end.
constexpr int SB = 32;
template <typename T>
struct SweepBlock {
  T l[SB];   // lane t: the multiplier of column (row) s for the entry t places away
  T dv;      // lane s: 1 / L_jj of the block's step s
  T nb;      // lane s: the entry entering the window after step s
};

template <typename T, bool FWD>
__device__ __forceinline__ void sweep_load(SweepBlock<T>& B, gptr<const T> L, gptr<const T> dinv, gptr<T> b, int n,
                                           int w, int j0) {
  const int lane = lane_id();
  const int W = w + 1;
  // every load is issued (masked lanes read entry 0), so the wait for one
  // block never waits for the block loaded after it
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const int j = FWD ? j0 + s : j0 - s;
    const bool ok = lane >= 1 && lane <= w && (FWD ? j + lane < n : j - lane >= 0);
    const T v = L[ok ? (FWD ? (size_t)j * W + lane : (size_t)(j - lane) * W + lane) : 0];
    B.l[s] = ok ? v : T(0);
  }
  const int j = FWD ? j0 + lane : j0 - lane;
  const bool okj = lane < SB && j >= 0 && j < n;
  const T dv = dinv[okj ? j : 0];
  B.dv = okj ? dv : T(0);
  const int i = FWD ? j0 + lane + 1 + w : j0 - lane - 1 - w;
  const bool oki = lane < SB && i >= 0 && i < n;
  const T nb = b[oki ? i : 0];
  B.nb = oki ? nb : T(0);
}

template <typename T, bool FWD>
__device__ __forceinline__ void sweep_run(const SweepBlock<T>& B, T& r, gptr<T> b, int n, int w, int j0) {
  const int lane = lane_id();
  T out = T(0);
  const int steps = FWD ? min(SB, n - j0) : min(SB, j0 + 1);
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    if (s < steps) {
      const T y = wget(r, 0) * wget(B.dv, s);
      if (lane == s) out = y;
      r = wshl1(r - B.l[s] * y);
      if (lane == w) r = wget(B.nb, s);
    }
  }
  const int j = FWD ? j0 + lane : j0 - lane;
  if (lane < steps) b[j] = out;
}

template <typename T, bool FWD>
__device__ void band_sweep(const T* L_, const T* dinv_, int n_, int w_, T* b_) {
  const auto L = gp(L_), dinv = gp(dinv_);
  const auto b = gp(b_);
  const int n = uni(n_), w = uni(w_);
  if (n <= 0) return;
  const int lane = lane_id();
  const int nblk = (n + SB - 1) / SB;
  T r = T(0);
  {
    const int i = FWD ? lane : n - 1 - lane;
    if (lane <= w && i >= 0 && i < n) r = b[i];
  }
  // block k starts at column k SB (forward) or n - 1 - k SB (backward)
  auto start = [&](int k) { return FWD ? k * SB : n - 1 - k * SB; };
  SweepBlock<T> A, C;
  sweep_load<T, FWD>(A, L, dinv, b, n, w, start(0));
  for (int k = 0; k < nblk; k += 2) {
    sweep_load<T, FWD>(C, L, dinv, b, n, w, start(k + 1));
    sweep_run<T, FWD>(A, r, b, n, w, start(k));
    if (k + 1 >= nblk) break;
    sweep_load<T, FWD>(A, L, dinv, b, n, w, start(k + 2));
    sweep_run<T, FWD>(C, r, b, n, w, start(k + 1));
  }
  gsync();
}

template <typename T>
__device__ void band_solve(const T* L, const T* dinv, int n, int w, T* b) {
  band_sweep<T, true>(L, dinv, n, w, b);
  band_sweep<T, false>(L, dinv, n, w, b);
}

// ---------------------------------------------------------------- one problem
struct Wave {
  const WaveDesc& D;
  double* lds;        // WAVE_WB * (WAVE_WB + 1) + 640 doubles: the factorisation's window and panel
  int L;              // max(n, m)
  double tau, kappa, delta, sdmax, xPx;
  double mu_it = 0.0; // the iteration's mu (the refinement's relative stop; 0 at the initial point)
  bool use64;
  int64_t hits, fallbacks, irs, facts;

  __device__ double* V(int k) const { return D.v + (size_t)k * L; }

  // S = P + delta I + A'MA into band storage (FP64; FP32 copy when low);
  // returns max |S_jj|.  The zero rows' part is Zband / delta (their M), the
  // rest a short list of entries with their nonneg-row and cone terms.
  __device__ double assemble(bool low) {
    const int W = D.W, ne = D.n * W;
    const double inv_delta = 1.0 / delta;
    for (int e0 = lane_id(); e0 < ne; e0 += UN * WL) {
      double pv[UN], zv[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int e = e0 + u * WL;
        pv[u] = e < ne ? D.Pband[e] : 0.0;
        zv[u] = e < ne ? D.Zband[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int e = e0 + u * WL;
        if (e < ne) D.Sb[e] = pv[u] + ((e % W) == 0 ? delta : 0.0) + zv[u] * inv_delta;
      }
    }
    gsync();
    for (int k = lane_id(); k < D.nte; k += WL) {
      const int e = D.te[k];
      double v = D.Sb[e];
      for (int t2 = D.trp[k]; t2 < D.trp[k + 1]; ++t2) v += D.tc[t2] * D.Mv[D.tm[t2]];
      D.Sb[e] = v;
    }
    gsync();
    double dmax = 0.0;
    for (int j = lane_id(); j < D.n; j += WL) dmax = nanmax(dmax, fabs(D.Sb[(size_t)j * W]));
    if (low) {
      for (int e = lane_id(); e < ne; e += WL) D.Sb32[e] = (float)D.Sb[e];
      gsync();
    }
    return wmax(dmax);
  }

  // factor the regularised system at the current scaling (hdiag and state filled)
  __device__ void factor(bool fp64) {
    const bool low = D.mixed && !fp64;
    if (low) {
      delta = D.static_reg + D.dyn_reg * fmax(D.maxPdiag, sdmax);
    } else {
      const double hmax = v_maxabs(D.m, D.hdiag);
      const double ds = D.mixed ? 1e-8 : D.static_reg;
      const double dd = D.mixed ? ldexp(1.0, -104) : D.dyn_reg;
      delta = ds + dd * fmax(D.maxPdiag, hmax);
    }
    c_mblock(D, delta);
    const double dmax = assemble(low);
    if (low) {
      sdmax = dmax;
      hits += band_cholesky<float>(D.Sb32, D.dinv32, D.n, D.w, (float)delta, (float*)lds);
    } else {
      hits += band_cholesky<double>(D.Sb, D.dinv, D.n, D.w, delta, lds);
    }
    facts++;
  }

  // x = S^-1 u in the factor precision (FP32 right-hand sides scaled by 1/|u|_inf)
  __device__ void schur_solve(const double* u, double* x) {
    if (D.mixed && !use64) {
      double sc = v_maxabs(D.n, u);
      sc = (sc > 0.0) ? sc : 1.0;
      for (int i = lane_id(); i < D.n; i += WL) D.f32[i] = (float)(u[i] / sc);
      gsync();
      band_solve<float>(D.Sb32, D.dinv32, D.n, D.w, D.f32);
      for (int i = lane_id(); i < D.n; i += WL) x[i] = (double)D.f32[i] * sc;
      gsync();
    } else {
      v_copy(D.n, u, x);
      band_solve<double>(D.Sb, D.dinv, D.n, D.w, x);
    }
  }

  // K_reg [x; z] = [r1; r2]: z = M (A x - r2), S x = r1 + A'M r2
  __device__ void solve_reg(const double* r1, const double* r2, double* x, double* z) {
    double* t1 = V(WV_T1);
    double* u1 = V(WV_U1);
    double* w1 = V(WV_W1);
    c_apply(D, 1, delta, r2, nullptr, t1);
    v_copy(D.n, r1, u1);
    spmv(D.n, D.Atrp, D.Atci, D.Atv, t1, u1, 1.0, 1.0);
    schur_solve(u1, x);
    spmv(D.m, D.Arp, D.Aci, D.Av, x, w1, 1.0, 0.0);
    v_axpby(D.m, -1.0, r2, 1.0, w1);
    c_apply(D, 1, delta, w1, nullptr, z);
  }

  // the residual at which the refinement stops (as the per-slot solver)
  __device__ double ir_target(double nb) const {
    return fmax(D.ir_abstol + D.ir_reltol * nb, D.ir_mu_frac * fmin(mu_it, 1.0) * (1.0 + nb));
  }

  // iterative refinement against the unregularised K; result in (xo, zo)
  __device__ void kkt_solve_once(const double* r1, const double* r2, double* xo, double* zo, double* best_out,
                                 double* nb_out) {
    const int n = D.n, m = D.m;
    const double nb = fmax(v_maxabs(n, r1), v_maxabs(m, r2));
    double *x = V(WV_IRX), *z = V(WV_IRZ), *xn = V(WV_IRXN), *zn = V(WV_IRZN);
    double *rx = V(WV_IRRX), *rz = V(WV_IRRZ), *kx = V(WV_KX), *kz = V(WV_KZ), *t2 = V(WV_T2);
    v_fill(n, 0.0, x);
    v_fill(m, 0.0, z);
    v_copy(n, r1, rx);
    v_copy(m, r2, rz);
    double best = nb, rnorm = nb;
    const double target = ir_target(nb);
    bool have_best = false;
    for (int it = 0; it <= D.ir_max; ++it) {
      solve_reg(rx, rz, kx, kz);
      v_lin(n, 1.0, x, 1.0, kx, 0.0, nullptr, xn);
      v_lin(m, 1.0, z, 1.0, kz, 0.0, nullptr, zn);
      ++irs;
      // r - K [xn; zn]
      spmv(n, D.Prp, D.Pci, D.Pv, xn, kx, 1.0, 0.0);
      spmv(n, D.Atrp, D.Atci, D.Atv, zn, kx, 1.0, 1.0);
      spmv(m, D.Arp, D.Aci, D.Av, xn, kz, 1.0, 0.0);
      c_apply(D, 0, 0.0, zn, nullptr, t2);
      v_axpby(m, -1.0, t2, 1.0, kz);
      v_lin(n, 1.0, r1, -1.0, kx, 0.0, nullptr, kx);
      v_lin(m, 1.0, r2, -1.0, kz, 0.0, nullptr, kz);
      const double rn = fmax(v_maxabs(n, kx), v_maxabs(m, kz));
      if (rn < best || !have_best) {
        if (rn < best) {
          v_copy(n, xn, V(WV_IRBX));
          v_copy(m, zn, V(WV_IRBZ));
          best = rn;
          have_best = true;
        }
      }
      if (rn <= target) break;
      if (it > 0 && rn > 0.5 * rnorm) break;
      double* tp;
      tp = x; x = xn; xn = tp;
      tp = z; z = zn; zn = tp;
      tp = rx; rx = kx; kx = tp;
      tp = rz; rz = kz; kz = tp;
      rnorm = rn;
    }
    if (have_best) {
      v_copy(n, V(WV_IRBX), xo);
      v_copy(m, V(WV_IRBZ), zo);
    } else {
      v_fill(n, 0.0, xo);
      v_fill(m, 0.0, zo);
    }
    *best_out = have_best ? best : NAN;
    *nb_out = nb;
  }

  __device__ void kkt_solve(const double* r1, const double* r2, double* xo, double* zo) {
    double best = 0.0, nb = 0.0;
    kkt_solve_once(r1, r2, xo, zo, &best, &nb);
    if (D.mixed && !use64 && !(best <= fmax(1e-6 * (1.0 + nb), ir_target(nb)))) {
      use64 = true;            // FP64 factorisation for the rest of the iteration
      factor(true);
      fallbacks++;
      kkt_solve_once(r1, r2, xo, zo, &best, &nb);
    }
  }

  struct Resid {
    double xPx, qx, bz, sz, rd_n, rp_n, x_n, s_n, z_n, atz_n, px_n, axs_n;
  };

  __device__ Resid residuals() {
    const int n = D.n, m = D.m;
    double *x = V(WV_X), *s = V(WV_S), *z = V(WV_Z), *Px = V(WV_PX), *Ax = V(WV_AX), *Atz = V(WV_ATZ);
    double *rdv = V(WV_RDV), *rpv = V(WV_RPV);
    spmv(n, D.Prp, D.Pci, D.Pv, x, Px, 1.0, 0.0);
    spmv(m, D.Arp, D.Aci, D.Av, x, Ax, 1.0, 0.0);
    spmv(n, D.Atrp, D.Atci, D.Atv, z, Atz, 1.0, 0.0);
    v_lin(n, 1.0, Px, 1.0, Atz, tau, D.q, rdv);
    v_lin(m, -1.0, Ax, -1.0, s, tau, D.b, rpv);
    Resid R;
    R.xPx = v_dot(n, x, Px);
    R.qx = v_dot(n, D.q, x);
    R.rd_n = v_maxabs(n, rdv, D.D, true);
    R.x_n = v_maxabs(n, x, D.D, false);
    R.atz_n = v_maxabs(n, Atz, D.D, true);
    R.px_n = v_maxabs(n, Px, D.D, true);
    R.bz = v_dot(m, D.b, z);
    R.sz = v_dot(m, s, z);
    R.rp_n = v_maxabs(m, rpv, D.E, true);
    R.s_n = v_maxabs(m, s, D.E, true);
    R.z_n = v_maxabs(m, z, D.E, false);
    R.axs_n = v_maxabs(m, Ax, D.E, true, s, 1.0);
    return R;
  }

  // termination tests (eq. termination-check, infeasibility-check); fills the report
  __device__ int check(const Resid& R) {
    const double t = tau, c = D.cscale, eps = D.eps_feas, ei = D.eps_inf;
    const double rp = R.rp_n / t, rd = R.rd_n / (c * t);
    const double gp = (0.5 * R.xPx / t + R.qx) / (c * t), gd = (-0.5 * R.xPx / t - R.bz) / (c * t);
    const double xn = R.x_n / t, sn = R.s_n / t, zn = R.z_n / (c * t);
    if (lane_id() == 0) {
      D.sc[SC_RESP] = rp;
      D.sc[SC_RESD] = rd;
      D.sc[SC_OBJP] = gp;
      D.sc[SC_OBJD] = gd;
      D.sc[SC_GAP] = fabs(gp - gd);
    }
    if (rp < eps * fmax(1.0, D.bnorm + xn + sn) && rd < eps * fmax(1.0, D.qnorm + xn + zn) &&
        fabs(gp - gd) < eps * fmax(1.0, fmin(fabs(gp), fabs(gd))))
      return HC_STATUS_SOLVED;
    const double bz = R.bz / c, xu = R.x_n, zu = R.z_n / c, su = R.s_n;
    if (bz < -ei && R.atz_n / c < -ei * fmax(1.0, xu + zu) * bz) return HC_STATUS_PRIMAL_INFEASIBLE;
    const double qx = R.qx / c;
    if (qx < -ei && R.px_n / c < -ei * fmax(1.0, xu) * qx && R.axs_n < -ei * fmax(1.0, xu + su) * qx)
      return HC_STATUS_DUAL_INFEASIBLE;
    if (!isfinite(rp) || !isfinite(rd) || !isfinite(gp)) return HC_STATUS_NUMERICAL_ERROR;
    return 0;
  }

  __device__ double step_length(const double* ds, const double* dz, double dtau, double dkappa) {
    double a = 1.0;
    if (dtau < 0) a = fmin(a, -tau / dtau);
    if (dkappa < 0) a = fmin(a, -kappa / dkappa);
    return fmin(a, c_step(D, V(WV_S), V(WV_Z), ds, dz));
  }

  struct Dir {
    double dtau, dkappa;
  };

  // solve for the right-hand side (d_x = r1, -(d_z - d_s) = r2, d_tau, d_kappa)
  // and recover Delta (eq. step-direction)
  __device__ Dir direction(const double* r1, const double* r2, double dtau_rhs, double dkap_rhs,
                           const double* ds_rhs, double* dxo, double* dzo, double* dso) {
    const int n = D.n, m = D.m;
    double *x1 = V(WV_X1), *z1 = V(WV_Z1), *x2 = V(WV_X2), *z2 = V(WV_Z2), *t2 = V(WV_T2);
    kkt_solve(r1, r2, x1, z1);
    v_lin(n, 2.0 / tau, V(WV_PX), 1.0, D.q, 0.0, nullptr, t2);
    const double a1 = v_dot(n, t2, x1), a2 = v_dot(n, t2, x2);
    const double b1 = v_dot(m, D.b, z1), b2 = v_dot(m, D.b, z2);
    Dir d;
    const double num = dtau_rhs - dkap_rhs / tau + a1 + b1;
    const double den = kappa / tau + xPx / (tau * tau) - a2 - b2;
    d.dtau = num / den;
    v_lin(n, 1.0, x1, d.dtau, x2, 0.0, nullptr, dxo);
    v_lin(m, 1.0, z1, d.dtau, z2, 0.0, nullptr, dzo);
    c_apply(D, 0, 0.0, dzo, ds_rhs, dso);
    d.dkappa = -(dkap_rhs + kappa * d.dtau) / tau;
    return d;
  }

  // one pass of the loop body after the termination tests; status or 0
  __device__ int iterate(const Resid& R) {
    const int n = D.n, m = D.m;
    const double mu = (R.sz + kappa * tau) / D.nu1;
    const double gt = kappa + R.qx + R.bz + R.xPx / tau;
    mu_it = mu;
    use64 = false;
    c_scale(D, V(WV_S), V(WV_Z));
    factor(false);
    // constant system K [x2; z2] = [-q; b]
    double* r1 = V(WV_R1);
    double* r2 = V(WV_R2);
    v_lin(n, -1.0, D.q, 0.0, nullptr, 0.0, nullptr, r1);
    kkt_solve(r1, D.b, V(WV_X2), V(WV_Z2));
    // affine: r1 = -rdv, r2 = rpv + s
    v_lin(n, -1.0, V(WV_RDV), 0.0, nullptr, 0.0, nullptr, r1);
    v_lin(m, 1.0, V(WV_RPV), 1.0, V(WV_S), 0.0, nullptr, r2);
    const Dir da = direction(r1, r2, gt, kappa * tau, V(WV_S), V(WV_DXA), V(WV_DZA), V(WV_DSA));
    const double alpha_a = step_length(V(WV_DSA), V(WV_DZA), da.dtau, da.dkappa);
    const double sigma = (1.0 - alpha_a) * (1.0 - alpha_a) * (1.0 - alpha_a);
    // combined
    const double dk = kappa * tau + da.dkappa * da.dtau - sigma * mu;
    c_ds(D, V(WV_S), V(WV_Z), V(WV_DSA), V(WV_DZA), sigma * mu, V(WV_DSRHS));
    const double f = 1.0 - sigma;
    v_lin(n, -f, V(WV_RDV), 0.0, nullptr, 0.0, nullptr, r1);
    v_lin(m, f, V(WV_RPV), 1.0, V(WV_DSRHS), 0.0, nullptr, r2);
    const Dir dc = direction(r1, r2, f * gt, dk, V(WV_DSRHS), V(WV_DX), V(WV_DZ), V(WV_DSV));
    const double alpha_c = step_length(V(WV_DSV), V(WV_DZ), dc.dtau, dc.dkappa);
    if (alpha_c < 1e-4) return HC_STATUS_INSUFFICIENT_PROGRESS;
    const double a = D.step_fraction * alpha_c;
    v_axpby(n, a, V(WV_DX), 1.0, V(WV_X));
    v_axpby(m, a, V(WV_DSV), 1.0, V(WV_S));
    v_axpby(m, a, V(WV_DZ), 1.0, V(WV_Z));
    tau += a * dc.dtau;
    kappa += a * dc.dkappa;
    return 0;
  }

  // initial point: K with H = I for [-q; b], s = -z (0 on zero rows), then s
  // and z moved along e by 1 + max(-lambda_min) when that is not negative
  __device__ void init_point() {
    const int n = D.n, m = D.m;
    tau = kappa = 1.0;
    use64 = false;
    c_identity(D);
    factor(false);
    double* r1 = V(WV_R1);
    v_lin(n, -1.0, D.q, 0.0, nullptr, 0.0, nullptr, r1);
    kkt_solve(r1, D.b, V(WV_X), V(WV_Z));
    double* s = V(WV_S);
    double* z = V(WV_Z);
    v_lin(m, -1.0, z, 0.0, nullptr, 0.0, nullptr, s);
    v_fill(D.nz, 0.0, s);
    for (int which = 0; which < 2; ++which) {
      double* v = which == 0 ? s : z;
      const double amax = c_max_neg_eig(D, v);
      if (amax >= 0.0) c_add_e(D, 1.0 + amax, v);
    }
  }

  // the result in the user's coordinates (the certificate for infeasible statuses)
  __device__ void write_result(int status) {
    const bool cert = status == HC_STATUS_PRIMAL_INFEASIBLE || status == HC_STATUS_DUAL_INFEASIBLE;
    const double t = cert ? 1.0 : tau;
    const double *x = V(WV_X), *s = V(WV_S), *z = V(WV_Z);
    for (int i = lane_id(); i < D.n; i += WL) D.xo[D.colperm[i]] = D.D[i] * x[i] / t;
    for (int r = lane_id(); r < D.m; r += WL) {
      const int u = D.rowperm[r];
      D.so[u] = s[r] / D.E[r] / t;
      D.zo[u] = D.E[r] * z[r] / (D.cscale * t);
    }
    gsync();
  }
};

// Passes of the Algorithm 1 loop for one slot until its solve ends or the
// next pass would overrun `budget` (wall-clock ticks of 10 ns from the start
// of the launch, judged by the length of the pass just done); at least one
// pass.  The state between passes is the same as between launches, so the
// result does not depend on how the passes fall into launches.
__global__ __launch_bounds__(WL) void k_wave_tick(const WaveDesc* __restrict__ descs,
                                                 const int32_t* __restrict__ active, int nslots,
                                                 int32_t* __restrict__ status, const int64_t* __restrict__ budget) {
  __shared__ __align__(16) double lds[WAVE_WB * (WAVE_WB + 1) + 64 * 10];
  const int slot = blockIdx.x;
  if (slot >= nslots || !active[slot]) return;
  const uint64_t t_start = wall_clock64();
  const int64_t limit = *budget;
  const WaveDesc D = descs[slot];
  double* sc = D.sc;
  int phase = (int)sc[SC_PHASE];
  if (phase == PH_DONE) {
    if (threadIdx.x == 0) status[slot] = PH_DONE;
    return;
  }
  Wave w{D, lds, max(D.n, D.m)};
  w.sdmax = sc[SC_SDMAX];
  w.hits = (int64_t)sc[SC_HITS];
  w.fallbacks = (int64_t)sc[SC_FALLBACKS];
  w.irs = (int64_t)sc[SC_IRS];
  w.facts = (int64_t)sc[SC_FACTS];
  int k = (int)sc[SC_K], iters = (int)sc[SC_ITERS];
  if (phase == PH_NEW) {
    w.delta = 0.0;
    w.use64 = false;
    w.sdmax = 0.0;
    w.init_point();
    k = 0;
    iters = 0;
  } else {
    w.tau = sc[SC_TAU];
    w.kappa = sc[SC_KAPPA];
  }
  int st = 0;
  double mu = 0.0;
  bool done = false;
  for (;;) {
    const uint64_t t_pass = wall_clock64();
    w.delta = 0.0;
    w.use64 = false;
    // one pass of the Algorithm 1 loop
    const Wave::Resid R = w.residuals();
    w.xPx = R.xPx;
    st = w.check(R);
    mu = (R.sz + w.kappa * w.tau) / D.nu1;
    if (st) {
      done = true;
    } else if (k == D.max_iter) {
      st = HC_STATUS_MAX_ITER;
      done = true;
    } else {
      st = w.iterate(R);
      iters++;
      if (st) {
        const Wave::Resid R2 = w.residuals();
        w.check(R2);
        done = true;
      }
    }
    k++;
    if (done) break;
    const uint64_t t_now = wall_clock64();
    const int64_t elapsed = (int64_t)(t_now - t_start), pass = (int64_t)(t_now - t_pass);
    if (__builtin_amdgcn_readfirstlane((int)(elapsed + pass >= limit))) break;
  }
  if (done) w.write_result(st);
  if (threadIdx.x == 0) {
    sc[SC_TAU] = w.tau;
    sc[SC_KAPPA] = w.kappa;
    sc[SC_K] = k;
    sc[SC_ITERS] = iters;
    sc[SC_STATUS] = st;
    sc[SC_SDMAX] = w.sdmax;
    sc[SC_HITS] = (double)w.hits;
    sc[SC_FALLBACKS] = (double)w.fallbacks;
    sc[SC_IRS] = (double)w.irs;
    sc[SC_FACTS] = (double)w.facts;
    sc[SC_MU] = mu;
    sc[SC_PHASE] = done ? PH_DONE : PH_RUN;
    status[slot] = done ? PH_DONE : PH_RUN;
  }
}

// bump layout of one slot's blob
struct Carve {
  char* base;
  size_t used = 0;
  template <typename T> T* take(size_t count) {
    used = (used + 255) / 256 * 256;
    T* p = base ? (T*)(base + used) : nullptr;
    used += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

template <typename T>
T* put(Carve& c, const std::vector<T>& v, hipStream_t st) {
  T* p = c.take<T>(v.size());
  if (p && !v.empty()) HC_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return p;
}

void layout(const WavePlan& P, Carve& c, WaveDesc* d, hipStream_t st) {
  const size_t L = (size_t)std::max(P.n, P.m);
  const size_t ne = (size_t)P.n * (P.w + 1);
  std::memset(d, 0, sizeof(*d));
  d->n = P.n;
  d->m = P.m;
  d->w = P.w;
  d->W = P.w + 1;
  d->nz = P.nz;
  d->nn = P.nn;
  d->nsoc = P.nsoc;
  d->mtot = P.mtot;
  d->ir_max = P.st.ir_max;
  d->max_iter = P.st.max_iter;
  d->mixed = P.mixed ? 1 : 0;
  d->nte = (int32_t)P.te.size();
  d->cscale = P.cscale;
  d->bnorm = P.bnorm;
  d->qnorm = P.qnorm;
  d->maxPdiag = P.maxPdiag;
  d->nu1 = (double)(P.nu + 1);
  d->eps_feas = P.st.eps_feas;
  d->eps_inf = P.st.eps_inf;
  d->static_reg = P.st.static_reg;
  d->dyn_reg = P.st.dyn_reg;
  d->ir_abstol = P.st.ir_abstol;
  d->ir_reltol = P.st.ir_reltol;
  d->ir_mu_frac = P.st.ir_mu_frac;
  d->step_fraction = P.st.step_fraction;
  d->Arp = put(c, P.Arp, st);
  d->Aci = put(c, P.Aci, st);
  d->Av = put(c, P.Av, st);
  d->Atrp = put(c, P.Atrp, st);
  d->Atci = put(c, P.Atci, st);
  d->Atv = put(c, P.Atv, st);
  d->Prp = put(c, P.Prp, st);
  d->Pci = put(c, P.Pci, st);
  d->Pv = put(c, P.Pv, st);
  d->q = put(c, P.q, st);
  d->b = put(c, P.b, st);
  d->D = put(c, P.D, st);
  d->E = put(c, P.E, st);
  d->Pband = put(c, P.Pband, st);
  d->Zband = put(c, P.Zband, st);
  d->te = put(c, P.te, st);
  d->trp = put(c, P.trp, st);
  d->tm = put(c, P.tm, st);
  d->tc = put(c, P.tc, st);
  d->soc_off = put(c, P.soc_off, st);
  d->soc_moff = put(c, P.soc_moff, st);
  d->colperm = put(c, P.colperm, st);
  d->rowperm = put(c, P.rowperm, st);
  d->v = c.take<double>(WV_COUNT * L);
  d->Sb = c.take<double>(ne);
  d->dinv = c.take<double>(P.n);
  d->hst = c.take<double>((size_t)P.nn + 2 * (size_t)(P.m - P.nz - P.nn) + P.nsoc);
  d->hdiag = c.take<double>(P.m);
  d->Mv = c.take<double>(P.mtot);
  d->sc = c.take<double>(SC_COUNT);
  if (P.mixed) {
    d->Sb32 = c.take<float>(ne);
    d->dinv32 = c.take<float>(P.n);
    d->f32 = c.take<float>(P.n);
  }
  d->xo = c.take<double>(P.n);
  d->so = c.take<double>(P.m);
  d->zo = c.take<double>(P.m);
}

}  // namespace

size_t WavePlan::blob_bytes() const {
  Carve c{nullptr};
  WaveDesc d;
  layout(*this, c, &d, nullptr);
  return c.used + 256;
}

void wave_upload(const WavePlan& plan, void* blob, WaveDesc* desc, hipStream_t st) {
  Carve c{(char*)(((uintptr_t)blob + 255) / 256 * 256)};
  layout(plan, c, desc, st);
  // fresh scalars: phase NEW
  std::vector<double> sc(SC_COUNT, 0.0);
  HC_HIP(hipMemcpyAsync(desc->sc, sc.data(), SC_COUNT * sizeof(double), hipMemcpyHostToDevice, st));
}

void wave_tick(const WaveDesc* descs, const int32_t* active, int nslots, int32_t* status, const int64_t* budget,
               hipStream_t st) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_wave_tick, dim3((unsigned)nslots), dim3(WL), 0, st, descs, active, nslots, status, budget);
  HC_LAUNCH_CHECK();
}

void wave_result(const WaveDesc& d, const WavePlan& plan, hc_info* info, double* x, double* s, double* z,
                 hipStream_t st) {
  double sc[SC_COUNT];
  HC_HIP(hipMemcpyAsync(sc, d.sc, sizeof(sc), hipMemcpyDeviceToHost, st));
  if (x) HC_HIP(hipMemcpyAsync(x, d.xo, (size_t)plan.n * sizeof(double), hipMemcpyDeviceToHost, st));
  if (s) HC_HIP(hipMemcpyAsync(s, d.so, (size_t)plan.m * sizeof(double), hipMemcpyDeviceToHost, st));
  if (z) HC_HIP(hipMemcpyAsync(z, d.zo, (size_t)plan.m * sizeof(double), hipMemcpyDeviceToHost, st));
  HC_HIP(hipStreamSynchronize(st));
  if (info) {
    info->status = (int32_t)sc[SC_STATUS];
    info->iterations = (int32_t)sc[SC_ITERS];
    info->obj_primal = sc[SC_OBJP];
    info->obj_dual = sc[SC_OBJD];
    info->res_primal = sc[SC_RESP];
    info->res_dual = sc[SC_RESD];
    info->gap = sc[SC_GAP];
    info->mu = sc[SC_MU];
    info->pivot_guard_hits = (int64_t)sc[SC_HITS];
    info->fp64_fallbacks = (int64_t)sc[SC_FALLBACKS];
    info->ir_solves = (int64_t)sc[SC_IRS];
    info->factorizations = (int64_t)sc[SC_FACTS];
  }
}

}  // namespace hc

// ===========================================================================
// C-ABI: batched solve of many small problems, one wavefront each
// ===========================================================================
using namespace hc;

extern "C" {

int32_t hc_batch_check(const hc_solver* s, int32_t* band) {
  if (!s) return HC_ERR_INVALID_ARG;
  WavePlan plan;
  std::string why;
  if (!wave_plan(s, &plan, &why)) {
    set_last_error("not eligible for the batched engine: " + why);
    return HC_ERR_UNSUPPORTED;
  }
  if (band) *band = plan.w;
  return HC_OK;
}

int32_t hc_solve_batch(hc_solver* const* handles, int32_t count, void* stream, int32_t device, hc_result* results) {
  if (!handles || !results || count < 1) return HC_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  std::vector<WavePlan> plans(count);
  for (int32_t i = 0; i < count; ++i) {
    std::string why;
    if (!handles[i]) return HC_ERR_INVALID_ARG;
    if (!wave_plan(handles[i], &plans[i], &why)) {
      set_last_error("problem " + std::to_string(i) + " is not eligible for the batched engine: " + why);
      return HC_ERR_UNSUPPORTED;
    }
  }
  char* mem = nullptr;
  void* aux = nullptr;
  int32_t rc = HC_OK;
  try {
    HC_HIP(hipSetDevice(device));
    std::vector<size_t> off(count + 1, 0);
    for (int32_t i = 0; i < count; ++i) off[i + 1] = off[i] + (plans[i].blob_bytes() + 255) / 256 * 256;
    const size_t tab = (size_t)count * (sizeof(WaveDesc) + 2 * sizeof(int32_t)) + 1024;
    if (hipMalloc((void**)&mem, off[count] + 256) != hipSuccess) throw Error{HC_ERR_OOM, "hipMalloc of the batch"};
    if (hipMalloc(&aux, tab) != hipSuccess) throw Error{HC_ERR_OOM, "hipMalloc of the slot table"};
    WaveDesc* ddesc = (WaveDesc*)aux;
    int32_t* dactive = (int32_t*)((char*)aux + (size_t)count * sizeof(WaveDesc));
    int32_t* dstatus = dactive + count;
    // no time limit: every slot runs to the end of its solve in one launch
    int64_t* dbudget = (int64_t*)(((uintptr_t)(dstatus + count) + 15) / 16 * 16);
    const int64_t unlimited = INT64_MAX / 4;
    HC_HIP(hipMemcpyAsync(dbudget, &unlimited, sizeof(int64_t), hipMemcpyHostToDevice, st));
    std::vector<WaveDesc> desc(count);
    const double t0 = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
    for (int32_t i = 0; i < count; ++i) wave_upload(plans[i], mem + off[i], &desc[i], st);
    std::vector<int32_t> act(count, 1), stat(count, PH_RUN);
    HC_HIP(hipMemcpyAsync(ddesc, desc.data(), count * sizeof(WaveDesc), hipMemcpyHostToDevice, st));
    HC_HIP(hipMemcpyAsync(dactive, act.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st));
    int max_ticks = 0;
    for (const WavePlan& p : plans) max_ticks = std::max(max_ticks, p.st.max_iter + 2);
    for (int tick = 0; tick < max_ticks; ++tick) {
      wave_tick(ddesc, dactive, count, dstatus, dbudget, st);
      HC_HIP(hipMemcpyAsync(stat.data(), dstatus, count * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      bool all = true;
      for (int32_t i = 0; i < count; ++i) all = all && stat[i] == PH_DONE;
      if (all) break;
    }
    const double t1 = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
    for (int32_t i = 0; i < count; ++i) {
      hc_result& r = results[i];
      hc_info inf{};
      wave_result(desc[i], plans[i], &inf, r.x, r.s, r.z, st);
      r.tag = (uint64_t)i;
      r.status = stat[i] == PH_DONE ? inf.status : HC_STATUS_MAX_ITER;
      r.error = HC_OK;
      r.iterations = inf.iterations;
      r.obj_primal = inf.obj_primal;
      r.obj_dual = inf.obj_dual;
      r.res_primal = inf.res_primal;
      r.res_dual = inf.res_dual;
      r.queue_ms = 0.0;
      r.solve_ms = t1 - t0;
      r.latency_ms = t1 - t0;
      r.n = plans[i].n;
      r.m = plans[i].m;
    }
  } catch (const Error& e) {
    set_last_error(e.msg);
    rc = e.code;
  }
  if (st) (void)hipStreamSynchronize(st);
  if (mem) (void)hipFree(mem);
  if (aux) (void)hipFree(aux);
  return rc;
}

}  // extern "C"
