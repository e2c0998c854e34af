// Internal declarations shared by the hipcone HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "hipcone.h"

namespace hc {

// ---------------------------------------------------------------------------
// error handling inside the library (never crosses the C-ABI)
// ---------------------------------------------------------------------------
struct Error {
  int32_t code;
  std::string msg;
};

#define HC_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::hc::Error{HC_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HC_LAUNCH_CHECK() HC_HIP(hipGetLastError())

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// cone families in the internal row order
//   zero rows | nonneg rows | SOC (one segment per dim, component-major) |
//   EXP (component-major) | POW (component-major) | PSD (cone by cone, svec)
// Component-major: row base + j*count + i holds component j of cone i, so the
// lane that owns cone i reads each component with coalesced loads.
// ---------------------------------------------------------------------------
struct Segment {
  int32_t kind;    // HC_CONE_*
  int64_t base;    // first internal row
  int64_t count;   // cones (zero/nonneg: rows)
  int32_t dim;     // rows per cone (PSD: svec dim)
  int32_t k;       // PSD side
  int64_t state;   // offset of this segment's per-cone state (doubles)
  int64_t moff;    // offset of its (H + delta I)^-1 lower-triangle entries
};

// Second-order cones of dimension up to SOC_DMAX run one lane per cone; larger
// ones one workgroup per cone (the intra-cone reductions of Sec. 3.4) and enter
// the Schur complement through a diagonal plus rank-2 form of their block
// (M_c = f_o I + (f_+ - f_o) v_+ v_+' + (f_- - f_o) v_- v_-').
constexpr int SOC_DMAX = 16;
__host__ __device__ inline bool soc_large(int kind, int dim) { return kind == HC_CONE_SOC && dim > SOC_DMAX; }

// per-cone scaling state, doubles per cone
inline int64_t state_doubles(int kind, int dim, int k) {
  switch (kind) {
    case HC_CONE_ZERO: return 0;
    case HC_CONE_NONNEG: return 1;                 // h = s / z
    case HC_CONE_SOC:                              // wbar (dim), eta, lambda (dim) [, |wbar_1|]
      return dim + 1 + dim + (dim > SOC_DMAX ? 1 : 0);
    case HC_CONE_EXP:
    case HC_CONE_POW: return 3 + 9 + 9 + 3 + 3 + 1;  // lam, V, Uhinv, sig_hinv, grad, branch
    case HC_CONE_PSD: return 3 * (int64_t)k * k + 2 * k;    // R, Rinv, Q, lambda, m
  }
  return 0;
}
inline int64_t mblock_doubles(int kind, int dim) {
  if (kind == HC_CONE_ZERO || kind == HC_CONE_NONNEG) return 1;
  if (soc_large(kind, dim)) return 3;   // f_o, f_+ - f_o, f_- - f_o
  return (int64_t)dim * (dim + 1) / 2;
}

// ---------------------------------------------------------------------------
// kernels (hc_vec.hip, hc_cones.hip, hc_dense.hip); all launch on `st`
// ---------------------------------------------------------------------------
struct Csr {          // device CSR, int32 indices
  int32_t nrows = 0, ncols = 0;
  int64_t nnz = 0;
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  int32_t lanes = 1;  // lanes per row used by spmv
  // rows longer than long_nnz entries (a few long rows among short ones) are
  // left to a second kernel with one wave per row
  int32_t long_nnz = 0x7fffffff;
  int32_t nlong = 0;
  int32_t* longrows = nullptr;
};

// y = alpha * A x + beta * y
void spmv(const Csr& A, const double* x, double* y, double alpha, double beta, hipStream_t st);
// y[rows_i] += alpha * (Ad x)_i for the dense rows Ad (nd x n row-major;
// column j is variable cols[j], or j when cols is null)
void dense_rows_gemv(int nd, int64_t n, const double* Ad, const int32_t* rows, const int32_t* cols, const double* x,
                     double* y, double alpha, hipStream_t st);
// y[cols[j]] += alpha * sum_r Ad[r, j] v[rows[r]]  (cols null: y[j]); part is
// scratch of dense_rows_t_parts(nd) * n doubles (per-chunk partial sums)
void dense_rows_gemv_t(int nd, int64_t n, const double* Ad, const int32_t* rows, const int32_t* cols,
                       const double* v, double* y, double alpha, double* part, hipStream_t st);
int64_t dense_rows_t_parts(int nd);

// generic fused vector kernels
void vaxpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);   // y = a x + b y
void vcopy(int64_t n, const double* x, double* y, hipStream_t st);
void vfill(int64_t n, double v, double* y, hipStream_t st);

// reductions: each returns per-block partials that the host combines in order
struct Reducer {
  double* dev = nullptr;    // partials, device
  double* host = nullptr;   // pinned host copy
  int nblocks = 0;
  int nvals = 0;
};

}  // namespace hc
