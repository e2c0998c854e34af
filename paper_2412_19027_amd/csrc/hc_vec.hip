// Vector, sparse and reduction kernels of the IPM (gfx950): SpMV for A, A'
// and P (residuals, eq. residuals-objectives; KKT products), fused axpys,
// ordered block reductions, and the assembly of the KKT Schur complement.
#include "hc_vec.h"

#include <cmath>

namespace hc {

// max that propagates NaN (a NaN residual must never pass a test)
__device__ inline double nmax(double a, double b) { return (a != a || b != b) ? NAN : (a > b ? a : b); }

// ---------------------------------------------------------------------------
// CSR SpMV: LPR lanes per row (1, 4, 16 or 64), chosen from the mean row length
// ---------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(256) void k_spmv(int32_t nrows, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                                              const double* __restrict__ x, double* __restrict__ y, double alpha,
                                              double beta, int32_t long_nnz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = t / LPR;
  const int sub = (int)(t % LPR);
  double acc = 0.0;
  bool mine = false;   // rows above long_nnz entries belong to k_spmv_long
  if (row < nrows) {
    const int32_t b = rp[row], e = rp[row + 1];
    mine = (e - b) <= long_nnz;
    if (mine)
      for (int32_t p = b + sub; p < e; p += LPR) acc += v[p] * x[ci[p]];
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (mine && sub == 0) y[row] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[row]);
}

// the long rows, one wave each
// one workgroup of 1024 threads per long row (many independent loads in
// flight for a row of tens of thousands of entries); per-wave shuffle sums
// meet in LDS in a fixed order
constexpr int LONG_THREADS = 1024;
__global__ __launch_bounds__(LONG_THREADS) void k_spmv_long(int32_t nlong, const int32_t* __restrict__ rows,
                                                            const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const double* __restrict__ v,
                                                            const double* __restrict__ x, double* __restrict__ y,
                                                            double alpha, double beta) {
  __shared__ double part[LONG_THREADS / 64];
  if ((int32_t)blockIdx.x >= nlong) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int32_t row = rows[blockIdx.x], b = rp[row], e = rp[row + 1];
  double acc = 0.0;
  for (int32_t p = b + tid; p < e; p += LONG_THREADS) acc += v[p] * x[ci[p]];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) part[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < LONG_THREADS / 64; ++w) s += part[w];
    y[row] = alpha * s + (beta == 0.0 ? 0.0 : beta * y[row]);
  }
}

void spmv(const Csr& A, const double* x, double* y, double alpha, double beta, hipStream_t st) {
  if (A.nrows == 0) return;
  const int64_t threads = (int64_t)A.nrows * A.lanes;
  const unsigned grid = (unsigned)ceil_div(threads, 256);
  const int32_t ln = A.long_nnz;
  switch (A.lanes) {
    case 1: hipLaunchKernelGGL(k_spmv<1>, dim3(grid), dim3(256), 0, st, A.nrows, A.rowptr, A.col, A.val, x, y, alpha, beta, ln); break;
    case 4: hipLaunchKernelGGL(k_spmv<4>, dim3(grid), dim3(256), 0, st, A.nrows, A.rowptr, A.col, A.val, x, y, alpha, beta, ln); break;
    case 16: hipLaunchKernelGGL(k_spmv<16>, dim3(grid), dim3(256), 0, st, A.nrows, A.rowptr, A.col, A.val, x, y, alpha, beta, ln); break;
    default: hipLaunchKernelGGL(k_spmv<64>, dim3(grid), dim3(256), 0, st, A.nrows, A.rowptr, A.col, A.val, x, y, alpha, beta, ln); break;
  }
  HC_LAUNCH_CHECK();
  if (A.nlong > 0) {
    hipLaunchKernelGGL(k_spmv_long, dim3((unsigned)A.nlong), dim3(LONG_THREADS), 0, st, A.nlong, A.longrows,
                       A.rowptr, A.col, A.val, x, y, alpha, beta);
    HC_LAUNCH_CHECK();
  }
}

int choose_lanes(double mean_nnz) {
  if (mean_nnz <= 6.0) return 1;
  if (mean_nnz <= 24.0) return 4;
  if (mean_nnz <= 96.0) return 16;
  return 64;
}

// dense rows (row-major nd x n; column t is variable cols[t], or t when cols
// is null): y[rows[r]] += alpha * Ad[r, :] x   (one workgroup per row)
__global__ __launch_bounds__(256) void k_dense_rows(int64_t n, const double* __restrict__ Ad,
                                                    const int32_t* __restrict__ rows,
                                                    const int32_t* __restrict__ cols, const double* __restrict__ x,
                                                    double* __restrict__ y, double alpha) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double acc = 0;
  for (int64_t j = threadIdx.x; j < n; j += 256) acc += Ad[(int64_t)r * n + j] * x[cols ? cols[j] : j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) y[rows[r]] += alpha * red[0];
}

void dense_rows_gemv(int nd, int64_t n, const double* Ad, const int32_t* rows, const int32_t* cols, const double* x,
                     double* y, double alpha, hipStream_t st) {
  if (nd == 0) return;
  hipLaunchKernelGGL(k_dense_rows, dim3(nd), dim3(256), 0, st, n, Ad, rows, cols, x, y, alpha);
  HC_LAUNCH_CHECK();
}

// y[cols[j]] += alpha * sum_r Ad[r, j] v[rows[r]]  (cols null: y[j]; cols is
// one-to-one).  The rows are split into chunks of DRT_ROWS: workgroup (x, c)
// sums chunk c for 256 columns (coalesced row reads) into part[c][j], and a
// second kernel adds the chunks in order, so the result does not depend on
// scheduling.  part holds dense_rows_t_parts(nd) * n doubles.
constexpr int DRT_ROWS = 64;
int64_t dense_rows_t_parts(int nd) { return ceil_div(nd, DRT_ROWS); }

__global__ __launch_bounds__(256) void k_dense_rows_t(int nd, int64_t n, const double* __restrict__ Ad,
                                                      const int32_t* __restrict__ rows, const double* __restrict__ v,
                                                      double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * DRT_ROWS, r1 = min(nd, r0 + DRT_ROWS);
  if (j >= n) return;
  double acc = 0;
  for (int r = r0; r < r1; ++r) acc += Ad[(int64_t)r * n + j] * v[rows[r]];
  part[(int64_t)blockIdx.y * n + j] = acc;
}

__global__ __launch_bounds__(256) void k_dense_rows_t_sum(int64_t n, int nparts, const double* __restrict__ part,
                                                          const int32_t* __restrict__ cols, double* __restrict__ y,
                                                          double alpha) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0;
  for (int c = 0; c < nparts; ++c) acc += part[(int64_t)c * n + j];
  y[cols ? cols[j] : j] += alpha * acc;
}

void dense_rows_gemv_t(int nd, int64_t n, const double* Ad, const int32_t* rows, const int32_t* cols,
                       const double* v, double* y, double alpha, double* part, hipStream_t st) {
  if (nd == 0) return;
  const int np = (int)dense_rows_t_parts(nd);
  hipLaunchKernelGGL(k_dense_rows_t, dim3((unsigned)ceil_div(n, 256), (unsigned)np), dim3(256), 0, st, nd, n, Ad, rows,
                     v, part);
  HC_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_dense_rows_t_sum, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, np, part, cols, y,
                     alpha);
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}
void vaxpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, a, x, b, y);
  HC_LAUNCH_CHECK();
}
// z = a x + b y + c w  (any of y, w may be null)
__global__ void k_lin3(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                       double c, const double* __restrict__ w, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = a * x[i];
  if (y) v += b * y[i];
  if (w) v += c * w[i];
  z[i] = v;
}
void vlin3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* w, double* z,
           hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_lin3, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, a, x, b, y, c, w, z);
  HC_LAUNCH_CHECK();
}
void vcopy(int64_t n, const double* x, double* y, hipStream_t st) {
  if (n == 0 || x == y) return;
  HC_HIP(hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
}
__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
void vfill(int64_t n, double v, double* y, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, v, y);
  HC_LAUNCH_CHECK();
}
// y[i] = x[i] * w[i]  or  x[i] / w[i]
__global__ void k_scale_by(int64_t n, const double* __restrict__ x, const double* __restrict__ w, int divide,
                           double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = divide ? x[i] / w[i] : x[i] * w[i];
}
void vscale_by(int64_t n, const double* x, const double* w, bool divide, double* y, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_scale_by, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, x, w, divide ? 1 : 0, y);
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// reductions: per-block partials, combined on the host in block order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(int64_t n, RedOps ops, double* __restrict__ partial) {
  __shared__ double red[256];
  for (int o = 0; o < ops.nops; ++o) {
    const RedOp op = ops.op[o];
    const bool is_sum = (op.kind == RED_DOT);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
      if (op.kind == RED_DOT) {
        acc += op.x[i] * op.y[i];
      } else {
        double v = op.x[i];
        if (op.y) v += op.yc * op.y[i];
        if (op.w) v = (op.kind == RED_MAX_MUL) ? v * op.w[i] : v / op.w[i];
        acc = nmax(acc, fabs(v));
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off)
        red[threadIdx.x] = is_sum ? red[threadIdx.x] + red[threadIdx.x + off] : nmax(red[threadIdx.x], red[threadIdx.x + off]);
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * ops.nops + o] = red[0];
    __syncthreads();
  }
}

int reduce_launch(int64_t n, const RedOps& ops, double* partial, hipStream_t st) {
  const int nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, ceil_div(n, 256)));
  hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(256), 0, st, n, ops, partial);
  HC_LAUNCH_CHECK();
  return nb;
}

// device-side max of partials into out[0] (no host round trip); used to scale
// FP32 right-hand sides
__global__ void k_combine_max(int nb, const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += 256) acc = fmax(acc, partial[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (red[0] > 0.0) ? red[0] : 1.0;
}
void combine_max(int nb, const double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_combine_max, dim3(1), dim3(256), 0, st, nb, partial, out);
  HC_LAUNCH_CHECK();
}

// FP64 <-> FP32 with a device-side scale
__global__ void k_to_f32(int64_t n, const double* __restrict__ x, const double* __restrict__ scale,
                         float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)(x[i] / scale[0]);
}
__global__ void k_from_f32(int64_t n, const float* __restrict__ x, const double* __restrict__ scale,
                           double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i] * scale[0];
}
void to_f32(int64_t n, const double* x, const double* scale, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, x, scale, y);
  HC_LAUNCH_CHECK();
}
void from_f32(int64_t n, const float* x, const double* scale, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_from_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, x, scale, y);
  HC_LAUNCH_CHECK();
}
// lower triangle (including diagonal) of a column-major n x n FP64 matrix -> FP32
__global__ void k_lower_to_f32(int64_t n, int64_t ld, const double* __restrict__ S, float* __restrict__ S32) {
  const int64_t j = blockIdx.y;
  for (int64_t i = j + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    S32[i + j * ld] = (float)S[i + j * ld];
}
void lower_to_f32(int64_t n, int64_t ld, const double* S, float* S32, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_lower_to_f32, dim3((unsigned)std::min<int64_t>(64, ceil_div(n, 256)), (unsigned)n), dim3(256),
                     0, st, n, ld, S, S32);
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Schur complement assembly  S = P + delta I + A' M A  (lower triangle)
// ---------------------------------------------------------------------------
__global__ void k_fill_lower_zero(int64_t n, int64_t ld, double* __restrict__ S) {
  const int64_t j = blockIdx.y;
  for (int64_t i = j + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    S[i + j * ld] = 0.0;
}
void fill_lower_zero(int64_t n, int64_t ld, double* S, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_lower_zero, dim3((unsigned)std::min<int64_t>(64, ceil_div(n, 256)), (unsigned)n),
                     dim3(256), 0, st, n, ld, S);
  HC_LAUNCH_CHECK();
}

// P (full CSR) lower part + delta on the diagonal
__global__ void k_add_P(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                        const double* __restrict__ v, double delta, int64_t ld, double* __restrict__ S) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  S[i + (int64_t)i * ld] += delta;
  if (!rp) return;
  for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
    const int32_t j = ci[p];
    if (j <= i) S[i + (int64_t)j * ld] += v[p];
  }
}
void add_P_delta(const Csr& P, int64_t n, double delta, int64_t ld, double* S, hipStream_t st) {
  hipLaunchKernelGGL(k_add_P, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, (int32_t)n, P.rowptr, P.col, P.val,
                     delta, ld, S);
  HC_LAUNCH_CHECK();
}

// one task = an unordered pair of rows (ra >= rb, same cone) with the index of
// M_c[ra, rb]; adds M * (a_ra a_rb' + a_rb a_ra') (or M a a' when ra == rb)
// into the lower triangle with hardware FP64 atomics.
// One task adds m (a_ra a_rb' + a_rb a_ra') (m a_ra a_ra' when ra = rb) to the
// lower triangle of S.  Short tasks run one lane each; long ones (rows with
// hundreds of entries) one wave each, the lanes striding over the entries of
// row ra, so no single lane issues the whole row's quadratic update.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_assemble_pairs(int64_t ntask, const int32_t* __restrict__ tra,
                                                        const int32_t* __restrict__ trb,
                                                        const int64_t* __restrict__ tm,
                                                        const double* __restrict__ mval, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci, const double* __restrict__ av,
                                                        int64_t ld, double* __restrict__ S) {
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
      const int32_t j = ci[p];
      const double mj = m * av[p];
      for (int32_t q = ba; q <= p; ++q) atomicAdd(&S[j + (int64_t)ci[q] * ld], mj * av[q]);
    }
  } else {
    for (int32_t p = ba + lane; p < ea; p += nl) {
      const int32_t j = ci[p];
      const double mj = m * av[p];
      for (int32_t q = bb; q < eb; ++q) {
        const int32_t k = ci[q];
        double v = mj * av[q];
        if (j == k) v *= 2.0;
        const int32_t hi = j > k ? j : k, lo = j > k ? k : j;
        atomicAdd(&S[hi + (int64_t)lo * ld], v);
      }
    }
  }
}
void assemble_pairs(int64_t ntask, const int32_t* tra, const int32_t* trb, const int64_t* tm, const double* mval,
                    const Csr& A, int64_t ld, double* S, bool wide, hipStream_t st) {
  if (ntask == 0) return;
  if (wide)
    hipLaunchKernelGGL(k_assemble_pairs<true>, dim3((unsigned)ceil_div(ntask * 64, 256)), dim3(256), 0, st, ntask,
                       tra, trb, tm, mval, A.rowptr, A.col, A.val, ld, S);
  else
    hipLaunchKernelGGL(k_assemble_pairs<false>, dim3((unsigned)ceil_div(ntask, 256)), dim3(256), 0, st, ntask, tra,
                       trb, tm, mval, A.rowptr, A.col, A.val, ld, S);
  HC_LAUNCH_CHECK();
}

// T[e, j] = sum_b M_c[a, b] A[row b of cone c, j] for segment row e = c dim + a
// (M_c symmetric, stored as its lower triangle: entry (a, b), a >= b, at
// moff + (a (a + 1) / 2 + b) count + c).  One workgroup per row, a thread per
// column the cone touches summing that column's entries in row order.
__global__ __launch_bounds__(256) void k_psd_dense_T(int32_t dim, int64_t count, int64_t coff, int64_t moff,
                                                     const double* __restrict__ mval, PsdCols pc,
                                                     const double* __restrict__ av, int64_t n,
                                                     double* __restrict__ T) {
  const int64_t rows = count * dim;
  for (int64_t e = blockIdx.x; e < rows; e += gridDim.x) {
    const int64_t c = e / dim;
    const int a = (int)(e % dim);
    for (int64_t u = pc.cu_off[coff + c] + threadIdx.x; u < pc.cu_off[coff + c + 1]; u += blockDim.x) {
      double acc = 0.0;
      for (int64_t k = pc.cu_ptr[u]; k < pc.cu_ptr[u + 1]; ++k) {
        const int b = pc.cu_b[k];
        const int hi = a > b ? a : b, lo = a > b ? b : a;
        acc += mval[moff + ((int64_t)hi * (hi + 1) / 2 + lo) * count + c] * av[pc.cu_p[k]];
      }
      T[e * n + pc.cu_col[u]] = acc;
    }
  }
}
void psd_dense_T(int32_t dim, int64_t count, int64_t coff, int64_t moff, const double* mval, const PsdCols& pc,
                 const double* av, int64_t n, double* T, hipStream_t st) {
  const int64_t rows = count * dim;
  if (rows == 0) return;
  hipLaunchKernelGGL(k_psd_dense_T, dim3((unsigned)std::min<int64_t>(rows, 16384)), dim3(256), 0, st, dim, count,
                     coff, moff, mval, pc, av, n, T);
  HC_LAUNCH_CHECK();
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_ordered_sum(OrderedSum os, int64_t first, int64_t cnt,
                                                     const double* __restrict__ mval, const double* __restrict__ av,
                                                     const double* __restrict__ slot, double* b0, double* b1,
                                                     double* b2) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = WIDE ? gid / 64 : gid;
  const int lane = WIDE ? (int)(threadIdx.x & 63) : 0, nl = WIDE ? 64 : 1;
  if (i >= cnt) return;   // wide: one destination per wave, so whole waves leave together
  const int64_t d = first + i;
  const int64_t k0 = os.ptr[d], k1 = os.ptr[d + 1];
  double acc = 0.0;
  if (os.pm) {
    for (int64_t k = k0 + lane; k < k1; k += nl) {
      int32_t q = os.pq[k];
      const bool two = q < 0;
      if (two) q = ~q;
      double v = mval[os.pm[k]] * av[os.pp[k]] * av[q];
      if (two) v *= 2.0;
      acc += v;
    }
  } else {
    for (int64_t k = k0 + lane; k < k1; k += nl) acc += slot[os.pp[k]];
  }
  if (WIDE)
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    const int64_t e = os.dst[d];
    const int sel = (int)((uint64_t)e >> 62);
    double* base = sel == 0 ? b0 : sel == 1 ? b1 : b2;
    base[e & ((int64_t(1) << 62) - 1)] += acc;
  }
}
void ordered_sum(const OrderedSum& os, const double* mval, const double* av, const double* slot, double* b0,
                 double* b1, double* b2, hipStream_t st) {
  const int64_t ns = os.nshort, nl = os.nd - os.nshort;
  if (ns > 0) {
    hipLaunchKernelGGL(k_ordered_sum<false>, dim3((unsigned)ceil_div(ns, 256)), dim3(256), 0, st, os, (int64_t)0,
                       ns, mval, av, slot, b0, b1, b2);
    HC_LAUNCH_CHECK();
  }
  if (nl > 0) {
    hipLaunchKernelGGL(k_ordered_sum<true>, dim3((unsigned)ceil_div(nl * 64, 256)), dim3(256), 0, st, os, ns, nl,
                       mval, av, slot, b0, b1, b2);
    HC_LAUNCH_CHECK();
  }
}

// S[j, k] += sum_e A[row(e), j] T[e, k] for k <= j: one workgroup per column
// j of A (row j of S), lanes over k, so each entry has one writer and the T
// rows are read contiguously
__global__ __launch_bounds__(256) void k_dense_T_gather(int64_t n, const int32_t* __restrict__ erp,
                                                        const int32_t* __restrict__ ee, const int32_t* __restrict__ ep,
                                                        const double* __restrict__ atval,
                                                        const double* __restrict__ T, int64_t ld,
                                                        double* __restrict__ S) {
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    const int32_t b = erp[j], e = erp[j + 1];
    if (b == e) continue;
    for (int64_t k = threadIdx.x; k <= j; k += blockDim.x) {
      double s = 0.0;
      for (int32_t p = b; p < e; ++p) s += atval[ep[p]] * T[(int64_t)ee[p] * n + k];
      S[j + k * ld] += s;
    }
  }
}
void dense_T_gather(int64_t n, const int32_t* erp, const int32_t* ee, const int32_t* ep, const double* atval,
                    const double* T, int64_t ld, double* S, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_dense_T_gather, dim3((unsigned)std::min<int64_t>(n, 8192)), dim3(256), 0, st, n, erp, ee, ep,
                     atval, T, ld, S);
  HC_LAUNCH_CHECK();
}

__global__ __launch_bounds__(64) void k_group_T(GroupPlan gp, const double* __restrict__ mval,
                                                const double* __restrict__ av) {
  const int lane = threadIdx.x;
  for (int64_t g = blockIdx.x; g < gp.ng; g += gridDim.x) {
    const int64_t nr = gp.rows_off[g + 1] - gp.rows_off[g];
    const int64_t uo = gp.u_off[g], s = gp.u_off[g + 1] - uo;
    const int64_t* gm = gp.gm + gp.m_off[g];
    double* T = gp.T + gp.t_off[g];
    for (int64_t a = 0; a < nr; ++a)
      for (int64_t t = lane; t < s; t += 64) {
        double v = 0.0;
        for (int64_t e = gp.c_ptr[uo + t]; e < gp.c_ptr[uo + t + 1]; ++e) {
          const int64_t mi = gm[a * nr + gp.c_b[e]];
          if (mi >= 0) v += mval[mi] * av[gp.c_k[e]];
        }
        T[a * s + t] = v;
      }
  }
}
void group_T(const GroupPlan& gp, const double* mval, const Csr& A, hipStream_t st) {
  if (gp.ng == 0) return;
  hipLaunchKernelGGL(k_group_T, dim3((unsigned)std::min<int64_t>(gp.ng, 65536)), dim3(64), 0, st, gp, mval, A.val);
  HC_LAUNCH_CHECK();
}

__global__ __launch_bounds__(64) void k_group_gather(GroupPlan gp, int64_t n, const int32_t* __restrict__ atrp,
                                                     const int32_t* __restrict__ atci,
                                                     const double* __restrict__ atv, int64_t ld,
                                                     double* __restrict__ S) {
  __shared__ double acc[GATHER_CHUNK];
  const int lane = threadIdx.x;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    const int32_t p0 = atrp[j], p1 = atrp[j + 1];
    for (int64_t c0 = j; c0 < n; c0 += GATHER_CHUNK) {
      const int64_t c1 = std::min<int64_t>(n, c0 + GATHER_CHUNK);
      for (int64_t i = c0 + lane; i < c1; i += 64) acc[i - c0] = 0.0;
      // each row's T row and column list come from per-entry tables (one
      // load level), and the next row's are loaded before this row's sum
      int32_t s_nx = p0 < p1 ? gp.e_s[p0] : 0;
      int64_t u_nx = p0 < p1 ? gp.e_u[p0] : 0, t_nx = p0 < p1 ? gp.e_t[p0] : 0;
      double c_nx = p0 < p1 ? atv[p0] : 0.0;
      for (int32_t p = p0; p < p1; ++p) {
        const int64_t s = s_nx, uo = u_nx, to = t_nx;
        const double coef = c_nx;
        if (p + 1 < p1) {
          s_nx = gp.e_s[p + 1];
          u_nx = gp.e_u[p + 1];
          t_nx = gp.e_t[p + 1];
          c_nx = atv[p + 1];
        }
        if (s == 0) continue;
        const double* vals = gp.T + to;
        for (int64_t t = lane; t < s; t += 64) {
          const int64_t i = gp.u[uo + t];
          if (i >= c0 && i < c1) acc[i - c0] += coef * vals[t];
        }
      }
      for (int64_t i = c0 + lane; i < c1; i += 64) {
        const double v = acc[i - c0];
        if (v != 0.0) S[i + j * ld] += v;
      }
    }
  }
}
void group_gather(const GroupPlan& gp, int64_t n, const Csr& At, int64_t ld, double* S, hipStream_t st) {
  if (gp.ng == 0 || n == 0) return;
  hipLaunchKernelGGL(k_group_gather, dim3((unsigned)std::min<int64_t>(n, 16384)), dim3(64), 0, st, gp, n, At.rowptr,
                     At.col, At.val, ld, S);
  HC_LAUNCH_CHECK();
}

// B (nd x n row-major, i.e. n x nd column-major with ld n) = sqrt|m_r| Ad[r, :];
// rows with midx < 0 are padding and stay zero
__global__ void k_scale_dense_rows(int nd, int64_t n, const double* __restrict__ Ad, const int64_t* __restrict__ midx,
                                   const double* __restrict__ mval, double* __restrict__ B) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int64_t mi = midx[r];
  if (j < n) B[(int64_t)r * n + j] = mi < 0 ? 0.0 : sqrt(fabs(mval[mi])) * Ad[(int64_t)r * n + j];
}
void scale_dense_rows(int nd, int64_t n, const double* Ad, const int64_t* midx, const double* mval, double* B,
                      hipStream_t st) {
  if (nd == 0) return;
  hipLaunchKernelGGL(k_scale_dense_rows, dim3((unsigned)ceil_div(n, 256), (unsigned)nd), dim3(256), 0, st, nd, n, Ad,
                     midx, mval, B);
  HC_LAUNCH_CHECK();
}

// transpose between cone-by-cone (AoS) and component-major layouts (test entry points)
__global__ void k_aos_to_cm(int64_t count, int dim, const double* __restrict__ a, double* __restrict__ c, int inverse) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * dim) return;
  const int64_t i = t / dim;
  const int j = (int)(t % dim);
  if (!inverse) c[j * count + i] = a[t];
  else c[t] = a[j * count + i];
}
void aos_to_cm(int64_t count, int dim, const double* a, double* c, bool inverse, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_aos_to_cm, dim3((unsigned)ceil_div(count * dim, 256)), dim3(256), 0, st, count, dim, a, c,
                     inverse ? 1 : 0);
  HC_LAUNCH_CHECK();
}

}  // namespace hc
