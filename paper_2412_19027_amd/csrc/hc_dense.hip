// Dense factorisation of the KKT Schur complement on gfx950.
//
// After the cone rows are eliminated (their pivots are the -(H_c + delta I)
// blocks), the quasi-definite LDL' of the regularised KKT matrix
// (eq. linsys_2x2, Sec. 3.5) continues on the positive definite Schur
// complement S = P + delta I + A' M A.  This file factors S = L L' (the
// positive pivots of the LDL', D = diag(L)^2 absorbed into L) and solves with
// L, in FP64 or -- for the mixed-precision mode of Sec. 3.5 -- FP32 with FP32
// accumulation.
//
// Layout: S is column-major with leading dimension ld, lower triangle used.
// Algorithm: blocked right-looking Cholesky with 64-wide diagonal blocks.
//   diag:   the 64x64 block is factored in LDS by one workgroup, which also
//           writes the inverse of the factor block (Linv, 64x64 per block)
//   trsm:   L21 = A21 * Linv' in place, one workgroup per 64 rows
//   update: trailing C -= L21 L21' on MFMA (v_mfma_f64_16x16x4f64 or
//           v_mfma_f32_16x16x4f32), 128x128 tiles, lower tiles only.  The
//           update of the trailing matrix is delayed to every NB = 256
//           columns (the panel's own columns are updated eagerly), so the
//           trailing matrix is read and written once per 256 columns.
// Triangular solves use the stored Linv blocks: one launch per 256 rows.
#include "hc_dense.h"

#include <algorithm>
#include <cmath>

namespace hc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Both instructions take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  Output element r of lane l is D[row(l, r)][l % 16]; the FP64
// form interleaves rows (l/16 + 4 r), the FP32 form blocks them (4 (l/16) + r).
template <> struct Mfma<double> {
  typedef v4d acc_t;
  __device__ static inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  __device__ static inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int BS = 64;    // diagonal block
constexpr int NB = 256;   // delayed-update panel width (multiple of BS)

// ---------------------------------------------------------------------------
// diagonal block: Cholesky in LDS + inverse of the factor
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_chol_diag(T* __restrict__ A, int64_t ld, int64_t c, int64_t n,
                                                   T* __restrict__ Linv, double tol, double fix,
                                                   unsigned long long* __restrict__ hits) {
  __shared__ T L[BS][BS + 1];   // L[row][col]
  __shared__ T X[BS][BS + 1];   // inverse
  const int tid = threadIdx.x;
  const int bs = (int)std::min<int64_t>(BS, n - c);
  for (int e = tid; e < BS * BS; e += 256) {
    int i = e % BS, j = e / BS;
    T v = 0;
    if (i < bs && j < bs && i >= j) v = A[(c + i) + (c + j) * ld];
    if (i >= bs || j >= bs) v = (i == j) ? T(1) : T(0);
    L[i][j] = v;
  }
  __syncthreads();
  for (int j = 0; j < bs; ++j) {
    if (tid == 0) {
      double d = (double)L[j][j];
      if (!(d > tol)) {
        d = fix;
        atomicAdd(hits, 1ull);
      }
      L[j][j] = (T)sqrt(d);
    }
    __syncthreads();
    const T ljj = L[j][j];
    for (int i = j + 1 + tid; i < bs; i += 256) L[i][j] = L[i][j] / ljj;
    __syncthreads();
    // rank-1 update of the trailing triangle
    const int m = bs - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      int i = j + 1 + e % m, k = j + 1 + e / m;
      if (i >= k) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular factor, one column per thread
  if (tid < BS) {
    const int j = tid;
    for (int i = 0; i < BS; ++i) X[i][j] = 0;
    if (j < bs) {
      X[j][j] = T(1) / L[j][j];
      for (int i = j + 1; i < bs; ++i) {
        T acc = 0;
        for (int k = j; k < i; ++k) acc += L[i][k] * X[k][j];
        X[i][j] = -acc / L[i][i];
      }
    } else {
      X[j][j] = 1;
    }
  }
  __syncthreads();
  for (int e = tid; e < BS * BS; e += 256) {
    int i = e % BS, j = e / BS;
    if (i < bs && j < bs && i >= j) A[(c + i) + (c + j) * ld] = L[i][j];
    Linv[i + j * BS] = X[i][j];
  }
}

// ---------------------------------------------------------------------------
// TRSM: rows [r0, r1) of the 64 columns starting at c: A21 <- A21 * Linv'
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(T* __restrict__ A, int64_t ld, int64_t c, int64_t r0, int64_t r1,
                                              const T* __restrict__ Linv) {
  __shared__ T Xs[BS][BS + 1];   // A rows (local row, k)
  __shared__ T Ls[BS][BS + 1];   // Linv (j, k)
  const int tid = threadIdx.x;
  const int64_t rb = r0 + (int64_t)blockIdx.x * BS;
  for (int e = tid; e < BS * BS; e += 256) {
    int i = e % BS, k = e / BS;
    int64_t r = rb + i;
    Xs[i][k] = (r < r1) ? A[r + (c + k) * ld] : T(0);
    Ls[i][k] = Linv[i + k * BS];
  }
  __syncthreads();
  // each thread computes a 4 x 4 sub-block: rows 4*(tid%16)+a, cols 4*(tid/16)+b
  const int i0 = 4 * (tid % 16), j0 = 4 * (tid / 16);
  T acc[4][4] = {};
  for (int k = 0; k < BS; ++k) {
    T xa[4], lb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xa[a] = Xs[i0 + a][k];
#pragma unroll
    for (int b = 0; b < 4; ++b) lb[b] = Ls[j0 + b][k];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * lb[b];
  }
  // X[i][j] = sum_k A[i][k] Linv[j][k]; only k <= j contributes (Linv lower)
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int64_t r = rb + i0 + a;
    if (r < r1)
#pragma unroll
      for (int b = 0; b < 4; ++b) A[r + (c + j0 + b) * ld] = acc[a][b];
  }
}

// ---------------------------------------------------------------------------
// C[i, j] += alpha * sum_k A[i, k] * B[j, k]  (i < M, j < N, k < K), all
// column-major; 128 x 128 tiles of 4 waves, each wave 64 x 64 on 16 MFMA
// accumulators.  `lower` skips tiles strictly above the global diagonal, whose
// position is given by the global indices (gr, gc) of C[0, 0].
// ---------------------------------------------------------------------------
constexpr int TM = 128, TN = 128, TK = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nt(T* __restrict__ C, int64_t ldc, const T* __restrict__ A, int64_t lda,
                                                 const T* __restrict__ B, int64_t ldb, int64_t M, int64_t N, int64_t K,
                                                 T alpha, int lower, int64_t gr, int64_t gc, int tiles_n) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[TK][TM + 4];
  __shared__ T Bs[TK][TN + 4];
  const int tile_m = blockIdx.x / tiles_n, tile_n = blockIdx.x % tiles_n;
  const int64_t i_base = (int64_t)tile_m * TM, j_base = (int64_t)tile_n * TN;
  if (lower && gr + i_base + TM - 1 < gc + j_base) return;   // tile strictly above the diagonal
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    for (int e = tid; e < TK * TM; e += 256) {
      const int i = e % TM, k = e / TM;
      const int64_t gk = k0 + k;
      const int64_t gi = i_base + i, gj = j_base + i;
      As[k][i] = (gi < M && gk < K) ? A[gi + gk * lda] : T(0);
      Bs[k][i] = (gj < N && gk < K) ? B[gj + gk * ldb] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      T a_op[4], b_op[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a_op[t] = As[kk + (lane >> 4)][wm + t * 16 + (lane & 15)];
        b_op[t] = Bs[kk + (lane >> 4)][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::op(a_op[a], b_op[b], acc[a][b]);
    }
    __syncthreads();
  }
  // lane holds D[row(lane, r)][lane % 16] of each 16 x 16 tile
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t j = j_base + wn + b * 16 + (lane & 15);
      if (j >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i_base + wm + a * 16 + Mfma<T>::row(lane, r);
        if (i < M) {
          T* p = &C[i + j * ldc];
          *p = *p + alpha * acc[a][b][r];
        }
      }
    }
}

template <typename T>
void gemm_nt(T* C, int64_t ldc, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t M, int64_t N, int64_t K,
             T alpha, bool lower, int64_t gr, int64_t gc, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  const int tm = (int)ceil_div(M, TM), tn = (int)ceil_div(N, TN);
  hipLaunchKernelGGL(k_gemm_nt<T>, dim3(tm * tn), dim3(256), 0, st, C, ldc, A, lda, B, ldb, M, N, K, alpha,
                     lower ? 1 : 0, gr, gc, tn);
  HC_LAUNCH_CHECK();
}

hipEvent_t Prof::next() {
  if (used == ev.size()) {
    hipEvent_t e;
    HC_HIP(hipEventCreate(&e));
    ev.push_back(e);
  }
  return ev[used++];
}

double Prof::collect_ms() {
  double ms = 0;
  for (size_t i = 0; i + 1 < used; i += 2) {
    HC_HIP(hipEventSynchronize(ev[i + 1]));
    float t = 0;
    HC_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
    ms += t;
  }
  used = 0;
  return ms;
}

Prof::~Prof() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

// lower-triangle entries (global row >= global col) of the C block
static double lower_entries(int64_t rc, int64_t cc, int64_t M, int64_t N) {
  double cnt = 0;
  for (int64_t j = cc; j < cc + N; ++j) cnt += (double)std::max<int64_t>(0, rc + M - std::max(rc, j));
  return cnt;
}

// C -= A B' with every operand inside the one column-major matrix S
template <typename T>
static void gemm_nt_sub(T* S, int64_t ld, int64_t rc, int64_t cc, int64_t ra, int64_t rb, int64_t ka, int64_t M,
                        int64_t N, int64_t K, bool lower, hipStream_t st, Prof* prof) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  if (prof) HC_HIP(hipEventRecord(prof->next(), st));
  gemm_nt<T>(S + rc + cc * ld, ld, S + ra + ka * ld, ld, S + rb + ka * ld, ld, M, N, K, T(-1), lower, rc, cc, st);
  if (prof) {
    HC_HIP(hipEventRecord(prof->next(), st));
    prof->flops += 2.0 * (double)K * lower_entries(rc, cc, M, N);
    prof->launches++;
  }
}

template <typename T>
void dense_cholesky(T* S, int64_t n, int64_t ld, T* Linv, double tol, double fix, unsigned long long* hits,
                    hipStream_t st, Prof* prof) {
  for (int64_t K0 = 0; K0 < n; K0 += NB) {
    const int64_t Kend = std::min<int64_t>(n, K0 + NB);
    for (int64_t c = K0; c < Kend; c += BS) {
      const int64_t cb = std::min<int64_t>(BS, n - c);
      hipLaunchKernelGGL(k_chol_diag<T>, dim3(1), dim3(256), 0, st, S, ld, c, n, Linv + (c / BS) * BS * BS, tol,
                         fix, hits);
      HC_LAUNCH_CHECK();
      const int64_t r0 = c + cb;
      if (r0 < n) {
        hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)ceil_div(n - r0, BS)), dim3(256), 0, st, S, ld, c, r0, n,
                           (const T*)(Linv + (c / BS) * BS * BS));
        HC_LAUNCH_CHECK();
      }
      // eager update of the rest of this panel: columns [r0, Kend), rows [r0, n)
      if (r0 < Kend)
        gemm_nt_sub<T>(S, ld, r0, r0, r0, r0, c, n - r0, Kend - r0, cb, true, st, prof);
    }
    // delayed update of the trailing matrix with the whole panel
    if (Kend < n) gemm_nt_sub<T>(S, ld, Kend, Kend, Kend, Kend, K0, n - Kend, n - Kend, Kend - K0, true, st, prof);
  }
}

// ---------------------------------------------------------------------------
// triangular solves with L (lower, column-major) and the Linv blocks,
// nrhs right-hand sides stored column-major with leading dimension n.
// forward:  Y = L^-1 B     (B is overwritten with partial updates)
// backward: X = L^-T Y     (Y is overwritten with partial updates)
// ---------------------------------------------------------------------------
constexpr int SB = 256;   // rows per launch
constexpr int MAXRHS = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd(const T* __restrict__ L, int64_t ld, const T* __restrict__ Linv,
                                                  int64_t c, int64_t n, T* __restrict__ B, T* __restrict__ Y,
                                                  int nrhs) {
  __shared__ T yb[SB][MAXRHS];
  const int tid = threadIdx.x;
  const int64_t cb = std::min<int64_t>(SB, n - c);
  // every workgroup solves the diagonal 256-block redundantly
  for (int e = tid; e < SB * nrhs; e += 256) {
    int i = e % SB, r = e / SB;
    yb[i][r] = (i < cb) ? B[(c + i) + r * n] : T(0);
  }
  __syncthreads();
  for (int s = 0; s < SB / BS && s * BS < cb; ++s) {
    const T* Li = Linv + ((c + s * BS) / BS) * BS * BS;
    // y_s = Linv_s * b_s  (64 x 64 matvec, thread per (row, rhs))
    T v = 0;
    int i = tid % BS, r = tid / BS;
    if (r < nrhs) {
      for (int k = 0; k <= i; ++k) v += Li[i + k * BS] * yb[s * BS + k][r];
    }
    __syncthreads();
    if (r < nrhs) yb[s * BS + i][r] = v;
    __syncthreads();
    // b_t -= L[t, s] y_s for the later sub-blocks of this 256 block
    for (int e = tid; e < (SB - (s + 1) * BS) * nrhs; e += 256) {
      int ii = (s + 1) * BS + e % (SB - (s + 1) * BS), rr = e / (SB - (s + 1) * BS);
      if (ii < cb) {
        T acc = 0;
        for (int k = 0; k < BS; ++k) acc += L[(c + ii) + (c + s * BS + k) * ld] * yb[s * BS + k][rr];
        yb[ii][rr] -= acc;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0)
    for (int e = tid; e < cb * nrhs; e += 256) {
      int i = e % cb, r = e / cb;
      Y[(c + i) + r * n] = yb[i][r];
    }
  // rows below: B[row] -= L[row, c:c+cb] * y
  const int64_t row = c + cb + (int64_t)blockIdx.x * 256 + tid;
  if (row < n) {
    T acc[MAXRHS] = {};
    for (int k = 0; k < cb; ++k) {
      T l = L[row + (c + k) * ld];
#pragma unroll
      for (int r = 0; r < MAXRHS; ++r)
        if (r < nrhs) acc[r] += l * yb[k][r];
    }
    for (int r = 0; r < nrhs; ++r) B[row + r * n] -= acc[r];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd(const T* __restrict__ L, int64_t ld, const T* __restrict__ Linv,
                                                  int64_t c, int64_t n, T* __restrict__ Yv, T* __restrict__ X,
                                                  int nrhs) {
  __shared__ T xb[SB][MAXRHS];
  const int tid = threadIdx.x;
  const int64_t cb = std::min<int64_t>(SB, n - c);
  const int nsub = (int)ceil_div(cb, BS);
  for (int e = tid; e < SB * nrhs; e += 256) {
    int i = e % SB, r = e / SB;
    xb[i][r] = (i < cb) ? Yv[(c + i) + r * n] : T(0);
  }
  __syncthreads();
  for (int s = nsub - 1; s >= 0; --s) {
    const T* Li = Linv + ((c + s * BS) / BS) * BS * BS;
    // x_s = Linv_s' * y_s
    T v = 0;
    int i = tid % BS, r = tid / BS;
    if (r < nrhs)
      for (int k = i; k < BS; ++k) v += Li[k + i * BS] * xb[s * BS + k][r];
    __syncthreads();
    if (r < nrhs) xb[s * BS + i][r] = v;
    __syncthreads();
    // y_t -= L[s rows, t cols]' x_s for earlier sub-blocks t < s
    for (int e = tid; e < s * BS * nrhs; e += 256) {
      int jj = e % (s * BS), rr = e / (s * BS);
      T acc = 0;
      for (int k = 0; k < BS; ++k)
        if (s * BS + k < cb) acc += L[(c + s * BS + k) + (c + jj) * ld] * xb[s * BS + k][rr];
      xb[jj][rr] -= acc;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0)
    for (int e = tid; e < cb * nrhs; e += 256) {
      int i = e % cb, r = e / cb;
      X[(c + i) + r * n] = xb[i][r];
    }
  // columns j < c: Y[j] -= sum_i L[c + i, j] x[i]; one wave per column
  const int lane = tid & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (tid >> 6);
  if (j < c) {
    T acc[MAXRHS] = {};
    for (int i = lane; i < cb; i += 64) {
      T l = L[(c + i) + j * ld];
#pragma unroll
      for (int r = 0; r < MAXRHS; ++r)
        if (r < nrhs) acc[r] += l * xb[i][r];
    }
#pragma unroll
    for (int r = 0; r < MAXRHS; ++r) {
      T v = acc[r];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[r] = v;
    }
    if (lane == 0)
      for (int r = 0; r < nrhs; ++r) Yv[j + r * n] -= acc[r];
  }
}

template <typename T>
void dense_solve(const T* L, int64_t n, int64_t ld, const T* Linv, T* B, T* Y, T* X, int nrhs, hipStream_t st) {
  // B -> Y (forward), Y -> X (backward); B and Y are overwritten
  for (int64_t c = 0; c < n; c += SB) {
    const int64_t below = n - std::min<int64_t>(n, c + SB);
    unsigned grid = (unsigned)std::max<int64_t>(1, ceil_div(below, 256));
    hipLaunchKernelGGL(k_trsv_fwd<T>, dim3(grid), dim3(256), 0, st, L, ld, Linv, c, n, B, Y, nrhs);
    HC_LAUNCH_CHECK();
  }
  const int64_t last = ((n - 1) / SB) * SB;
  for (int64_t c = last; c >= 0; c -= SB) {
    unsigned grid = (unsigned)std::max<int64_t>(1, ceil_div(c, 4));
    hipLaunchKernelGGL(k_trsv_bwd<T>, dim3(grid), dim3(256), 0, st, L, ld, Linv, c, n, Y, X, nrhs);
    HC_LAUNCH_CHECK();
  }
}

template void dense_cholesky<double>(double*, int64_t, int64_t, double*, double, double, unsigned long long*,
                                     hipStream_t, Prof*);
template void dense_cholesky<float>(float*, int64_t, int64_t, float*, double, double, unsigned long long*,
                                    hipStream_t, Prof*);
template void gemm_nt<double>(double*, int64_t, const double*, int64_t, const double*, int64_t, int64_t, int64_t,
                              int64_t, double, bool, int64_t, int64_t, hipStream_t);
template void gemm_nt<float>(float*, int64_t, const float*, int64_t, const float*, int64_t, int64_t, int64_t,
                             int64_t, float, bool, int64_t, int64_t, hipStream_t);
template void dense_solve<double>(const double*, int64_t, int64_t, const double*, double*, double*, double*, int,
                                  hipStream_t);
template void dense_solve<float>(const float*, int64_t, int64_t, const float*, float*, float*, float*, int,
                                 hipStream_t);

int64_t linv_elems(int64_t n) { return ceil_div(n, BS) * BS * BS; }

// factor flops of a dense n x n Cholesky
double cholesky_flops(int64_t n) { return (double)n * n * n / 3.0; }

}  // namespace hc
