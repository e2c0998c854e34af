// Second-order cones of high dimension (Sec. 3.4): one workgroup per cone.
//
// The paper computes the per-cone quantities t^2 - |u|^2 of large cones with
// child kernels launched from a parent kernel (dynamic parallelism) and a
// shared-memory tree reduction per child.  HIP has no device-side launch, so
// here one workgroup of LS_TB lanes owns a cone: each lane accumulates a
// strided slice of the cone's components, partial sums meet through wave
// shuffles and one LDS exchange, and every lane then holds the cone's sums.
// A grid of at most LS_GRID workgroups strides over the cones of a segment, so
// many large cones run concurrently (the cone-level parallelism the paper
// recovers with its parent kernel).
//
// Layout and state are those of the small-SOC kernels: component j of cone c
// at row base + j*count + c; state wbar (dim), eta, lambda (dim), then
// r = |wbar_1| (kept because the spectral form needs it and recomputing it
// would cost another reduction per use).
//
// In the Schur complement a large cone is not written as an explicit d x d
// block.  With v_+- = (1, +-u)/sqrt2 the eigenvectors of H_c for eta^2 (w0 +- r)^2,
//   M_c = (H_c + delta I)^-1 = f_o I + (f_+ - f_o) v_+ v_+' + (f_- - f_o) v_- v_-',
// so A_c' M_c A_c = f_o A_c' A_c + (f_+ - f_o) p_+ p_+' + (f_- - f_o) p_- p_-'
// with p_+- = A_c' v_+-: a diagonal term assembled like nonnegative rows and two
// dense rows that join the dense-row product of the Schur complement.
#include "hc_cones.h"

namespace hc {

constexpr int LS_TB = 256;    // lanes per cone (four wave64)

// sums of K per-lane values over the workgroup; every lane receives the sums
template <int K> __device__ inline void block_sum(double (&v)[K], double* red) {
#pragma unroll
  for (int k = 0; k < K; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();   // the previous call's readers are done with red
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * 4 + w] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = (red[k * 4 + 0] + red[k * 4 + 1]) + (red[k * 4 + 2] + red[k * 4 + 3]);
}

struct LsView {
  const SegDev& g;
  int64_t c;
  __device__ int64_t row(int64_t j) const { return g.base + j * g.count + c; }
  __device__ double wb(int64_t j) const { return g.state[j * g.count + c]; }
  __device__ double eta() const { return g.state[(int64_t)g.dim * g.count + c]; }
  __device__ double lam(int64_t j) const { return g.state[(g.dim + 1 + j) * g.count + c]; }
  __device__ double r() const { return g.state[(2 * (int64_t)g.dim + 1) * g.count + c]; }
  // component j >= 1 of u = wbar_1 / |wbar_1| (e_1 when wbar_1 = 0)
  __device__ double u(int64_t j, double r) const { return r > 0.0 ? wb(j) / r : (j == 1 ? 1.0 : 0.0); }
};

// ---------------------------------------------------------------------------
// scaling (Appendix A, NT point of the SOC): wbar, eta, lambda = W z, diag(H)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LS_TB) void k_lsoc_scale(SegDev g, const double* __restrict__ s,
                                                      const double* __restrict__ z, double* __restrict__ hdiag) {
  __shared__ double red[4 * 3];
  const int d = g.dim;
  const int64_t N = g.count;
  for (int64_t c = blockIdx.x; c < N; c += gridDim.x) {
    const LsView v{g, c};
    const double s0 = s[v.row(0)], z0 = z[v.row(0)];
    double a[3] = {0.0, 0.0, 0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double sj = s[v.row(j)], zj = z[v.row(j)];
      a[0] += sj * sj;
      a[1] += zj * zj;
      a[2] += sj * zj;
    }
    block_sum<3>(a, red);
    const double ns = sqrt(s0 * s0 - a[0]), nz = sqrt(z0 * z0 - a[1]);
    const double sz = (s0 * z0 + a[2]) / (ns * nz);
    const double gamma = sqrt((1.0 + sz) / 2.0);
    const double w0 = (s0 / ns + z0 / nz) / (2.0 * gamma);
    const double eta = sqrt(ns / nz);
    double b[2] = {0.0, 0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double zj = z[v.row(j)];
      const double wj = (s[v.row(j)] / ns - zj / nz) / (2.0 * gamma);
      b[0] += wj * zj;
      b[1] += wj * wj;
    }
    block_sum<2>(b, red);
    const double w1z1 = b[0], e2 = eta * eta;
    const double cf = z0 + w1z1 / (1.0 + w0);
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double zj = z[v.row(j)];
      const double wj = (s[v.row(j)] / ns - zj / nz) / (2.0 * gamma);
      g.state[(int64_t)j * N + c] = wj;
      g.state[(int64_t)(d + 1 + j) * N + c] = eta * (zj + cf * wj);
      hdiag[v.row(j)] = e2 * (2.0 * wj * wj + 1.0);
    }
    if (threadIdx.x == 0) {
      g.state[c] = w0;
      g.state[(int64_t)d * N + c] = eta;
      g.state[(int64_t)(d + 1) * N + c] = eta * (w0 * z0 + w1z1);
      g.state[(2 * (int64_t)d + 1) * N + c] = sqrt(b[1]);
      hdiag[v.row(0)] = e2 * (2.0 * w0 * w0 - 1.0);
    }
  }
}

// ---------------------------------------------------------------------------
// y = V f(lam) V' x (mode 0: H, mode 1: (H + delta I)^-1); with dsr, the
// direction recovery out = -dsr - H x instead
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LS_TB) void k_lsoc_apply(SegDev g, int mode, double delta, const double* __restrict__ x,
                                                      const double* __restrict__ dsr, double* __restrict__ y) {
  __shared__ double red[4];
  const int d = g.dim;
  const double is2 = 0.70710678118654752440;
  for (int64_t c = blockIdx.x; c < g.count; c += gridDim.x) {
    const LsView v{g, c};
    const double w0 = v.wb(0), eta = v.eta(), r = v.r();
    const double x0 = x[v.row(0)];
    double a[1] = {0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) a[0] += v.u(j, r) * x[v.row(j)];
    block_sum<1>(a, red);
    const double ux = a[0];
    const double big = w0 + r, e2 = eta * eta;
    const double lp = e2 * big * big, lm = e2 / (big * big), lo = e2;
    const double fp = mode == 0 ? lp : 1.0 / (lp + delta);
    const double fm = mode == 0 ? lm : 1.0 / (lm + delta);
    const double fo = mode == 0 ? lo : 1.0 / (lo + delta);
    const double ap = (x0 + ux) * is2, am = (x0 - ux) * is2;
    const double cu = (fp * ap - fm * am) * is2;
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double uj = v.u(j, r);
      const double yj = cu * uj + fo * (x[v.row(j)] - uj * ux);
      y[v.row(j)] = dsr ? -dsr[v.row(j)] - yj : yj;
    }
    if (threadIdx.x == 0) {
      const double y0 = (fp * ap + fm * am) * is2;
      y[v.row(0)] = dsr ? -dsr[v.row(0)] - y0 : y0;
    }
  }
}

// ---------------------------------------------------------------------------
// combined-step d_s (eq. ds-correction-step): ds = W' (lam \ (lam o lam +
// (W^-T dsa) o (W dza) - sm e)); each phase recomputes its per-component
// values from the inputs and carries only the cone's sums forward
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LS_TB) void k_lsoc_ds(SegDev g, const double* __restrict__ dsa,
                                                   const double* __restrict__ dza, double sm,
                                                   double* __restrict__ ds) {
  __shared__ double red[4 * 2];
  const int d = g.dim;
  for (int64_t c = blockIdx.x; c < g.count; c += gridDim.x) {
    const LsView v{g, c};
    const double w0 = v.wb(0), eta = v.eta(), l0 = v.lam(0);
    const double a0 = dsa[v.row(0)], b0 = dza[v.row(0)];
    // W^-T dsa (= W^-1 dsa, W symmetric) needs wbar_1'(J dsa)_1 = -wbar_1'dsa_1,
    // W dza needs wbar_1'dza_1
    double t[2] = {0.0, 0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double wj = v.wb(j);
      t[0] -= wj * dsa[v.row(j)];
      t[1] += wj * dza[v.row(j)];
    }
    block_sum<2>(t, red);
    const double w1a = t[0], w1b = t[1];
    const double p0 = (w0 * a0 + w1a) / eta, cfa = a0 + w1a / (1.0 + w0);
    const double q0 = eta * (w0 * b0 + w1b), cfb = b0 + w1b / (1.0 + w0);
    auto pj = [&](int j, double wj) { return -(-dsa[v.row(j)] + cfa * wj) / eta; };
    auto qj = [&](int j, double wj) { return eta * (dza[v.row(j)] + cfb * wj); };
    double u[2] = {0.0, 0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double wj = v.wb(j), lj = v.lam(j);
      u[0] += lj * lj;
      u[1] += pj(j, wj) * qj(j, wj);
    }
    block_sum<2>(u, red);
    const double v0 = (l0 * l0 + u[0]) + (p0 * q0 + u[1]) - sm;
    const double lJl = l0 * l0 - u[0];
    auto vj = [&](int j) {
      const double wj = v.wb(j);
      return 2.0 * l0 * v.lam(j) + p0 * qj(j, wj) + q0 * pj(j, wj);
    };
    double h[1] = {0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) h[0] += v.lam(j) * vj(j);
    block_sum<1>(h, red);
    const double x0 = (l0 * v0 - h[0]) / lJl;
    auto xj = [&](int j) { return (vj(j) - x0 * v.lam(j)) / l0; };
    double k[1] = {0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) k[0] += v.wb(j) * xj(j);
    block_sum<1>(k, red);
    const double w1x = k[0];
    const double cfx = x0 + w1x / (1.0 + w0);
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) ds[v.row(j)] = eta * (xj(j) + cfx * v.wb(j));
    if (threadIdx.x == 0) ds[v.row(0)] = eta * (w0 * x0 + w1x);
  }
}

// ---------------------------------------------------------------------------
// step length: largest alpha keeping s + alpha ds and z + alpha dz in the
// cone (roots of the quadratic (x + a dx)'J(x + a dx)); per workgroup the
// minimum over its cones, or per cone (capped at amax) when per_cone
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LS_TB) void k_lsoc_step(SegDev g, const double* __restrict__ s,
                                                     const double* __restrict__ z, const double* __restrict__ ds,
                                                     const double* __restrict__ dz, double amax, int per_cone,
                                                     double* __restrict__ out) {
  __shared__ double red[4 * 6];
  const int d = g.dim;
  double best = INFINITY;
  for (int64_t c = blockIdx.x; c < g.count; c += gridDim.x) {
    const LsView v{g, c};
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) {
      const double xs = s[v.row(j)], dxs = ds[v.row(j)], xz = z[v.row(j)], dxz = dz[v.row(j)];
      a[0] += dxs * dxs;
      a[1] += xs * dxs;
      a[2] += xs * xs;
      a[3] += dxz * dxz;
      a[4] += xz * dxz;
      a[5] += xz * xz;
    }
    block_sum<6>(a, red);
    const double s0 = s[v.row(0)], ds0 = ds[v.row(0)], z0 = z[v.row(0)], dz0 = dz[v.row(0)];
    const double as = soc_boundary_step(ds0 * ds0 - a[0], s0 * ds0 - a[1], s0 * s0 - a[2]);
    const double az = soc_boundary_step(dz0 * dz0 - a[3], z0 * dz0 - a[4], z0 * z0 - a[5]);
    const double st = fmin(as, az);
    if (per_cone) {
      if (threadIdx.x == 0) out[c] = fmin(amax, st);
    } else {
      best = fmin(best, st);
    }
  }
  if (!per_cone && threadIdx.x == 0) out[blockIdx.x] = best;
}

// max over the workgroup's cones of -lambda_min(v_c) = |v_1| - v_0
__global__ __launch_bounds__(LS_TB) void k_lsoc_max_neg_eig(SegDev g, const double* __restrict__ x,
                                                            double* __restrict__ partial) {
  __shared__ double red[4];
  const int d = g.dim;
  double best = -INFINITY;
  for (int64_t c = blockIdx.x; c < g.count; c += gridDim.x) {
    const LsView v{g, c};
    double a[1] = {0.0};
    for (int j = 1 + threadIdx.x; j < d; j += LS_TB) a[0] += x[v.row(j)] * x[v.row(j)];
    block_sum<1>(a, red);
    best = fmax(best, sqrt(a[0]) - x[v.row(0)]);
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = best;
}

// ---------------------------------------------------------------------------
// rank-2 part of the cone's Schur block: for each (cone, touched column j)
// entry, p_+-[j] = sum over the cone's rows r of A[r, j] v_+-[r], written into
// the two dense rows reserved for the cone (p_- at dst, p_+ at dst + plus_off)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lsoc_lowrank(SegDev g, int64_t nent, const int32_t* __restrict__ ent_cone,
                                                      const int32_t* __restrict__ ent_col,
                                                      const int64_t* __restrict__ ent_dst, Csr At, int64_t plus_off,
                                                      double* __restrict__ Ad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  const int64_t c = ent_cone[e], N = g.count, rows = (int64_t)g.dim * N;
  const int32_t j = ent_col[e];
  const LsView v{g, c};
  const double r = v.r();
  double pp = 0.0, pm = 0.0;
  for (int32_t k = At.rowptr[j]; k < At.rowptr[j + 1]; ++k) {
    const int64_t off = (int64_t)At.col[k] - g.base;
    if (off < 0 || off >= rows || off % N != c) continue;
    const int64_t comp = off / N;
    const double a = At.val[k];
    if (comp == 0) {
      pp += a;
      pm += a;
    } else {
      const double au = a * v.u(comp, r);
      pp += au;
      pm -= au;
    }
  }
  const double is2 = 0.70710678118654752440;
  Ad[ent_dst[e]] = is2 * pm;
  Ad[ent_dst[e] + plus_off] = is2 * pp;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void lsoc_scale(const SegDev& g, const double* s, const double* z, double* hdiag, hipStream_t st) {
  hipLaunchKernelGGL(k_lsoc_scale, dim3(lsoc_grid(g.count)), dim3(LS_TB), 0, st, g, s, z, hdiag);
  HC_LAUNCH_CHECK();
}

void lsoc_apply(const SegDev& g, int mode, double delta, const double* x, const double* dsr, double* y,
                hipStream_t st) {
  hipLaunchKernelGGL(k_lsoc_apply, dim3(lsoc_grid(g.count)), dim3(LS_TB), 0, st, g, mode, delta, x, dsr, y);
  HC_LAUNCH_CHECK();
}

void lsoc_ds(const SegDev& g, const double* dsa, const double* dza, double sm, double* ds, hipStream_t st) {
  hipLaunchKernelGGL(k_lsoc_ds, dim3(lsoc_grid(g.count)), dim3(LS_TB), 0, st, g, dsa, dza, sm, ds);
  HC_LAUNCH_CHECK();
}

int lsoc_step(const SegDev& g, const double* s, const double* z, const double* ds, const double* dz, double amax,
              bool per_cone, double* out, hipStream_t st) {
  const int nb = lsoc_grid(g.count);
  hipLaunchKernelGGL(k_lsoc_step, dim3(nb), dim3(LS_TB), 0, st, g, s, z, ds, dz, amax, per_cone ? 1 : 0, out);
  HC_LAUNCH_CHECK();
  return nb;
}

int lsoc_max_neg_eig(const SegDev& g, const double* v, double* partial, hipStream_t st) {
  const int nb = lsoc_grid(g.count);
  hipLaunchKernelGGL(k_lsoc_max_neg_eig, dim3(nb), dim3(LS_TB), 0, st, g, v, partial);
  HC_LAUNCH_CHECK();
  return nb;
}

void lsoc_lowrank(const SegDev& g, int64_t nent, const int32_t* ent_cone, const int32_t* ent_col,
                  const int64_t* ent_dst, const Csr& At, int64_t plus_off, double* Ad, hipStream_t st) {
  if (nent == 0) return;
  hipLaunchKernelGGL(k_lsoc_lowrank, dim3((unsigned)ceil_div(nent, 256)), dim3(256), 0, st, g, nent, ent_cone,
                     ent_col, ent_dst, At, plus_off, Ad);
  HC_LAUNCH_CHECK();
}

}  // namespace hc
