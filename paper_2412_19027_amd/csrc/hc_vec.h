// Vector / sparse / reduction / assembly kernels (gfx950).
#pragma once
#include "hc_common.h"

namespace hc {

int choose_lanes(double mean_nnz);
void vlin3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* w, double* z,
           hipStream_t st);
void vscale_by(int64_t n, const double* x, const double* w, bool divide, double* y, hipStream_t st);

enum { RED_DOT = 0, RED_MAX_MUL = 1, RED_MAX_DIV = 2 };
// DOT: sum x*y.  MAX_MUL / MAX_DIV: max |(x + yc*y) * w| or |(x + yc*y) / w|
// (y and w optional).
struct RedOp {
  int kind;
  const double* x;
  const double* y;
  double yc;
  const double* w;
};
constexpr int MAX_RED_OPS = 8;
struct RedOps {
  int nops;
  RedOp op[MAX_RED_OPS];
};
int reduce_launch(int64_t n, const RedOps& ops, double* partial, hipStream_t st);   // returns blocks
void combine_max(int nb, const double* partial, double* out, hipStream_t st);
void to_f32(int64_t n, const double* x, const double* scale, float* y, hipStream_t st);
void from_f32(int64_t n, const float* x, const double* scale, double* y, hipStream_t st);
void lower_to_f32(int64_t n, int64_t ld, const double* S, float* S32, hipStream_t st);
void fill_lower_zero(int64_t n, int64_t ld, double* S, hipStream_t st);
void add_P_delta(const Csr& P, int64_t n, double delta, int64_t ld, double* S, hipStream_t st);
// wide: one wave per task (long rows) instead of one lane
void assemble_pairs(int64_t ntask, const int32_t* tra, const int32_t* trb, const int64_t* tm, const double* mval,
                    const Csr& A, int64_t ld, double* S, bool wide, hipStream_t st);
// Schur contribution of PSD cones whose blocks touch most columns, as a
// gather instead of row-pair atomics: T = M_c A_c for every row of the
// segment (psd_dense_T, row-major rows of n doubles starting at T), then the
// lower triangle of S gains A_e' T over the rows of all such segments
// (dense_T_gather, erp/ee/ep: per column j of A the T rows e and the
// positions in atval of the values A[row(e), j]).  n <= PSD_DENSE_NMAX (one
// LDS row of n doubles per workgroup).
constexpr int64_t PSD_DENSE_NMAX = 8192;
void psd_dense_T(int64_t base, int32_t dim, int64_t count, int64_t moff, const double* mval, const Csr& A, int64_t n,
                 double* T, hipStream_t st);
void dense_T_gather(int64_t n, const int32_t* erp, const int32_t* ee, const int32_t* ep, const double* atval,
                    const double* T, int64_t ld, double* S, hipStream_t st);
void scale_dense_rows(int nd, int64_t n, const double* Ad, const int64_t* midx, const double* mval, double* B,
                      hipStream_t st);
void aos_to_cm(int64_t count, int dim, const double* a, double* c, bool inverse, hipStream_t st);

}  // namespace hc
