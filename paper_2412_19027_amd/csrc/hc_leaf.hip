// Leaf blocks of the two-level Schur factorisation (gfx950): assembly through
// the column map, batched per-leaf Cholesky and coupling, leaf solves.
#include "hc_leaf.h"

#include <algorithm>
#include <cmath>

namespace hc {

// address of S[j, k] (either order) inside the two-level storage
__device__ inline double* dest(const ColMap& cm, int32_t j, int32_t k) {
  const int32_t bj = cm.leaf[j], bk = cm.leaf[k];
  const int32_t lj = cm.loc[j], lk = cm.loc[k];
  if (bj < 0 && bk < 0) {
    const int32_t hi = lj > lk ? lj : lk, lo = lj > lk ? lk : lj;
    return cm.ST + hi + (int64_t)lo * cm.ldt;
  }
  if (bj >= 0 && bk >= 0) {
    if (bj != bk) return cm.sink;   // cannot happen: leaves are connected components
    const int32_t l = cm.lsize[bj];
    const int32_t hi = lj > lk ? lj : lk, lo = lj > lk ? lk : lj;
    return cm.lval + cm.lval_off[bj] + hi + (int64_t)lo * l;
  }
  const int32_t b = bj >= 0 ? bj : bk;
  const int32_t l = bj >= 0 ? lj : lk;
  const int32_t t = bj >= 0 ? lk : lj;
  const int32_t* cl = cm.clist + cm.clist_off[b];
  int lo = 0, hi = cm.ccnt[b] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t v = cl[mid];
    if (v == t) return cm.cval + cm.cval_off[b] + mid + (int64_t)l * cm.ccnt[b];
    if (v < t) lo = mid + 1;
    else hi = mid - 1;
  }
  return cm.sink;   // cannot happen: the coupling list holds every neighbour
}

// pair tasks through the column map (lane per task, or wave per long task:
// see k_assemble_pairs)
template <bool WIDE>
__global__ __launch_bounds__(256) void k_assemble_pairs_map(int64_t ntask, const int32_t* __restrict__ tra,
                                                            const int32_t* __restrict__ trb,
                                                            const int64_t* __restrict__ tm,
                                                            const double* __restrict__ mval,
                                                            const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const double* __restrict__ av, ColMap cm) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = WIDE ? gid / 64 : gid;
  const int lane = WIDE ? (int)(threadIdx.x & 63) : 0, nl = WIDE ? 64 : 1;
  if (t >= ntask) return;
  const int32_t ra = tra[t], rb = trb[t];
  const double m = mval[tm[t]];
  if (m == 0.0) return;
  const int32_t ba = rp[ra], ea = rp[ra + 1], bb = rp[rb], eb = rp[rb + 1];
  if (ra == rb) {
    for (int32_t p = ba + lane; p < ea; p += nl) {
      const double mj = m * av[p];
      for (int32_t q = ba; q <= p; ++q) atomicAdd(dest(cm, ci[p], ci[q]), mj * av[q]);
    }
  } else {
    for (int32_t p = ba + lane; p < ea; p += nl) {
      const int32_t j = ci[p];
      const double mj = m * av[p];
      for (int32_t q = bb; q < eb; ++q) {
        const int32_t k = ci[q];
        double v = mj * av[q];
        if (j == k) v *= 2.0;
        atomicAdd(dest(cm, j, k), v);
      }
    }
  }
}

void assemble_pairs_map(int64_t ntask, const int32_t* tra, const int32_t* trb, const int64_t* tm, const double* mval,
                        const Csr& A, const ColMap& cm, bool wide, hipStream_t st) {
  if (ntask == 0) return;
  if (wide)
    hipLaunchKernelGGL(k_assemble_pairs_map<true>, dim3((unsigned)ceil_div(ntask * 64, 256)), dim3(256), 0, st,
                       ntask, tra, trb, tm, mval, A.rowptr, A.col, A.val, cm);
  else
    hipLaunchKernelGGL(k_assemble_pairs_map<false>, dim3((unsigned)ceil_div(ntask, 256)), dim3(256), 0, st, ntask,
                       tra, trb, tm, mval, A.rowptr, A.col, A.val, cm);
  HC_LAUNCH_CHECK();
}

__global__ void k_add_P_map(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ v, double delta, ColMap cm) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  *dest(cm, i, i) += delta;   // each diagonal entry has exactly one writer here
  if (!rp) return;
  for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
    const int32_t j = ci[p];
    if (j <= i) atomicAdd(dest(cm, i, j), v[p]);
  }
}

void add_P_delta_map(const Csr& P, int64_t n, double delta, const ColMap& cm, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_add_P_map, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, (int32_t)n, P.rowptr, P.col,
                     P.val, delta, cm);
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// one wave per leaf
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_leaf_factor(ColMap cm, double tol, double fix,
                                                    unsigned long long* __restrict__ hits) {
  __shared__ double Lb[LEAF_MAX][LEAF_MAX + 1];
  __shared__ double W[LEAF_CPL_MAX][LEAF_MAX + 1];
  const int b = blockIdx.x, lane = threadIdx.x;
  const int l = cm.lsize[b], cnt = cm.ccnt[b];
  double* lv = cm.lval + cm.lval_off[b];
  double* cv = cm.cval + cm.cval_off[b];
  const int32_t* cl = cm.clist + cm.clist_off[b];
  for (int e = lane; e < l * l; e += 64) {
    const int i = e % l, j = e / l;
    Lb[i][j] = (i >= j) ? lv[e] : 0.0;
  }
  for (int e = lane; e < cnt * l; e += 64) W[e % cnt][e / cnt] = cv[e];
  __syncthreads();
  int nh = 0;
  for (int j = 0; j < l; ++j) {
    double d = Lb[j][j];
    if (!(d > tol)) {
      d = fix;
      ++nh;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (lane == j) Lb[j][j] = ljj;
    if (lane > j && lane < l) Lb[lane][j] /= ljj;
    __syncthreads();
    for (int k = j + 1; k < l; ++k)
      if (lane >= k && lane < l) Lb[lane][k] -= Lb[lane][j] * Lb[k][j];
    __syncthreads();
  }
  if (lane == 0 && nh) atomicAdd(hits, (unsigned long long)nh);
  // row a of W solves L_b w = s_a:  w_j = (s_aj - sum_{k<j} L_jk w_k) / L_jj
  if (lane < cnt)
    for (int j = 0; j < l; ++j) {
      double v = W[lane][j];
      for (int k = 0; k < j; ++k) v -= Lb[j][k] * W[lane][k];
      W[lane][j] = v / Lb[j][j];
    }
  __syncthreads();
  for (int e = lane; e < l * l; e += 64) {
    const int i = e % l, j = e / l;
    lv[e] = (i >= j) ? Lb[i][j] : 0.0;
  }
  for (int e = lane; e < cnt * l; e += 64) cv[e] = W[e % cnt][e / cnt];
  // S_TT[cl[a], cl[c]] -= sum_j W[a][j] W[c][j] for a >= c (cl ascending, so
  // the target is in the lower triangle)
  const int npair = cnt * (cnt + 1) / 2;
  for (int p = lane; p < npair; p += 64) {
    int a = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > p) --a;
    while ((a + 1) * (a + 2) / 2 <= p) ++a;
    const int c = p - a * (a + 1) / 2;
    double v = 0.0;
    for (int j = 0; j < l; ++j) v += W[a][j] * W[c][j];
    if (cm.lslot) cm.lslot[cm.lp_off[b] + p] = -v;
    else atomicAdd(&cm.ST[cl[a] + (int64_t)cl[c] * cm.ldt], -v);
  }
}

void leaf_factor(const ColMap& cm, double tol, double fix, unsigned long long* hits, hipStream_t st) {
  if (cm.nleaf == 0) return;
  hipLaunchKernelGGL(k_leaf_factor, dim3((unsigned)cm.nleaf), dim3(64), 0, st, cm, tol, fix, hits);
  HC_LAUNCH_CHECK();
}

__device__ inline void load_leaf_L(const ColMap& cm, int b, int l, int lane, double (*Lb)[LEAF_MAX + 1]) {
  const double* lv = cm.lval + cm.lval_off[b];
  for (int e = lane; e < l * l; e += 64) Lb[e % l][e / l] = lv[e];
}

// Leaf solves.  Leaves of at most LEAF_SMALL columns run one lane each
// (their L and coupling rows read straight from memory), larger ones one wave
// each through LDS; the tail's share of the forward solve is a gather per tail
// index over the leaves coupled to it (no atomics, a fixed order).
__global__ __launch_bounds__(256) void k_leaf_fwd_small(ColMap cm, const double* __restrict__ u,
                                                        double* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= cm.nsmall) return;
  const int b = cm.small[k];
  const int l = cm.lsize[b];
  const double* lv = cm.lval + cm.lval_off[b];   // L_b column-major: L[i][j] = lv[i + j l]
  const int32_t* cols = cm.lcols + cm.lcol_off[b];
  double yb[LEAF_SMALL];
#pragma unroll
  for (int j = 0; j < LEAF_SMALL; ++j) {
    if (j < l) {
      double v = u[cols[j]];
#pragma unroll
      for (int q = 0; q < j; ++q) v -= lv[j + q * l] * yb[q];
      yb[j] = v / lv[j + j * l];
      y[cols[j]] = yb[j];
    }
  }
}

__global__ __launch_bounds__(64) void k_leaf_fwd(ColMap cm, const double* __restrict__ u, double* __restrict__ y) {
  __shared__ double Lb[LEAF_MAX][LEAF_MAX + 1];
  __shared__ double yb[LEAF_MAX];
  const int b = cm.large[blockIdx.x], lane = threadIdx.x;
  const int l = cm.lsize[b];
  const int32_t* cols = cm.lcols + cm.lcol_off[b];
  load_leaf_L(cm, b, l, lane, Lb);
  if (lane < l) yb[lane] = u[cols[lane]];
  __syncthreads();
  if (lane == 0)
    for (int j = 0; j < l; ++j) {
      double v = yb[j];
      for (int k = 0; k < j; ++k) v -= Lb[j][k] * yb[k];
      yb[j] = v / Lb[j][j];
    }
  __syncthreads();
  if (lane < l) y[cols[lane]] = yb[lane];
}

// uT[t] -= sum over the couplings (b, a) of t of sum_j W_b[a][j] y_b[j]; one
// wave per tail index, lanes over its couplings, then a shuffle tree
// one workgroup per tail index, of cm.tail_threads threads: its W entries
// (flattened at set-up into (cval index, leaf column) pairs, so each costs
// two independent gathers) split over the threads; per-wave shuffle sums meet
// in LDS in a fixed order
constexpr int TAIL_THREADS_MAX = 1024;
__global__ __launch_bounds__(TAIL_THREADS_MAX) void k_leaf_tail(ColMap cm, const double* __restrict__ y,
                                                                double* __restrict__ uT) {
  __shared__ double part[TAIL_THREADS_MAX / 64];
  const int64_t t = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
  const int64_t e0 = cm.tc_ptr[t], e1 = cm.tc_ptr[t + 1];
  double acc = 0.0;
  for (int64_t e = e0 + tid; e < e1; e += nthr) acc += cm.cval[cm.te_cv[e]] * y[cm.te_y[e]];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) part[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0 && e1 > e0) {
    double s = 0.0;
    for (int w = 0; w < nthr / 64; ++w) s += part[w];
    uT[t] -= s;
  }
}

__global__ __launch_bounds__(256) void k_leaf_bwd_small(ColMap cm, const double* __restrict__ xT,
                                                        double* __restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= cm.nsmall) return;
  const int b = cm.small[k];
  const int l = cm.lsize[b], cnt = cm.ccnt[b];
  const double* lv = cm.lval + cm.lval_off[b];
  const int32_t* cols = cm.lcols + cm.lcol_off[b];
  const int32_t* cl = cm.clist + cm.clist_off[b];
  const double* cv = cm.cval + cm.cval_off[b];
  double vb[LEAF_SMALL];
#pragma unroll
  for (int j = 0; j < LEAF_SMALL; ++j) {
    if (j < l) {
      double v = x[cols[j]];
      for (int a = 0; a < cnt; ++a) v -= cv[a + (int64_t)j * cnt] * xT[cl[a]];
      vb[j] = v;
    }
  }
#pragma unroll
  for (int j = LEAF_SMALL - 1; j >= 0; --j) {
    if (j < l) {
      double v = vb[j];
#pragma unroll
      for (int q = j + 1; q < LEAF_SMALL; ++q)
        if (q < l) v -= lv[q + j * l] * vb[q];
      vb[j] = v / lv[j + j * l];
      x[cols[j]] = vb[j];
    }
  }
}

__global__ __launch_bounds__(64) void k_leaf_bwd(ColMap cm, const double* __restrict__ xT, double* __restrict__ x) {
  __shared__ double Lb[LEAF_MAX][LEAF_MAX + 1];
  __shared__ double vb[LEAF_MAX];
  const int b = cm.large[blockIdx.x], lane = threadIdx.x;
  const int l = cm.lsize[b], cnt = cm.ccnt[b];
  const int32_t* cols = cm.lcols + cm.lcol_off[b];
  const int32_t* cl = cm.clist + cm.clist_off[b];
  const double* cv = cm.cval + cm.cval_off[b];
  load_leaf_L(cm, b, l, lane, Lb);
  if (lane < l) {
    double v = x[cols[lane]];
    for (int a = 0; a < cnt; ++a) v -= cv[a + (int64_t)lane * cnt] * xT[cl[a]];
    vb[lane] = v;
  }
  __syncthreads();
  if (lane == 0)
    for (int j = l - 1; j >= 0; --j) {
      double v = vb[j];
      for (int k = j + 1; k < l; ++k) v -= Lb[k][j] * vb[k];
      vb[j] = v / Lb[j][j];
    }
  __syncthreads();
  if (lane < l) x[cols[lane]] = vb[lane];
}

void leaf_forward(const ColMap& cm, const double* u, double* y, double* uT, hipStream_t st) {
  if (cm.nleaf == 0) return;
  if (cm.nsmall) {
    hipLaunchKernelGGL(k_leaf_fwd_small, dim3((unsigned)ceil_div(cm.nsmall, 256)), dim3(256), 0, st, cm, u, y);
    HC_LAUNCH_CHECK();
  }
  if (cm.nlarge) {
    hipLaunchKernelGGL(k_leaf_fwd, dim3((unsigned)cm.nlarge), dim3(64), 0, st, cm, u, y);
    HC_LAUNCH_CHECK();
  }
  if (cm.nt) {
    const int thr = cm.tail_threads == 1024 || cm.tail_threads == 256 ? cm.tail_threads : 64;
    hipLaunchKernelGGL(k_leaf_tail, dim3((unsigned)cm.nt), dim3(thr), 0, st, cm, (const double*)y, uT);
    HC_LAUNCH_CHECK();
  }
}

void leaf_backward(const ColMap& cm, const double* xT, double* x, hipStream_t st) {
  if (cm.nleaf == 0) return;
  if (cm.nsmall) {
    hipLaunchKernelGGL(k_leaf_bwd_small, dim3((unsigned)ceil_div(cm.nsmall, 256)), dim3(256), 0, st, cm, xT, x);
    HC_LAUNCH_CHECK();
  }
  if (cm.nlarge) {
    hipLaunchKernelGGL(k_leaf_bwd, dim3((unsigned)cm.nlarge), dim3(64), 0, st, cm, xT, x);
    HC_LAUNCH_CHECK();
  }
}

__global__ void k_gather_tail(int64_t nt, const int32_t* __restrict__ tcols, const double* __restrict__ u,
                              double* __restrict__ uT) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nt) uT[t] = u[tcols[t]];
}
__global__ void k_scatter_tail(int64_t nt, const int32_t* __restrict__ tcols, const double* __restrict__ xT,
                               double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nt) x[tcols[t]] = xT[t];
}

void gather_tail(const ColMap& cm, const double* u, double* uT, hipStream_t st) {
  if (cm.nt == 0) return;
  hipLaunchKernelGGL(k_gather_tail, dim3((unsigned)ceil_div(cm.nt, 256)), dim3(256), 0, st, cm.nt, cm.tcols, u, uT);
  HC_LAUNCH_CHECK();
}
void scatter_tail(const ColMap& cm, const double* xT, double* x, hipStream_t st) {
  if (cm.nt == 0) return;
  hipLaunchKernelGGL(k_scatter_tail, dim3((unsigned)ceil_div(cm.nt, 256)), dim3(256), 0, st, cm.nt, cm.tcols, xT, x);
  HC_LAUNCH_CHECK();
}

}  // namespace hc
