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
// psd_dense_T writes T[e, j] for the columns j the cone touches (per cone
// coff + c its columns cu_col[cu_off[.] ..] and per column u its entries
// cu_ptr[u] .. cu_ptr[u + 1] as (row b of the cone, index of A[row b, j] in A),
// rows ascending): a thread per column, no atomics, a fixed order.  T's other
// columns stay zero (cleared once when T is allocated).
constexpr int64_t PSD_DENSE_NMAX = 8192;
struct PsdCols {
  const int64_t *cu_off = nullptr, *cu_ptr = nullptr;
  const int32_t *cu_col = nullptr, *cu_b = nullptr, *cu_p = nullptr;
};
void psd_dense_T(int32_t dim, int64_t count, int64_t coff, int64_t moff, const double* mval, const PsdCols& pc,
                 const double* av, int64_t n, double* T, hipStream_t st);
void dense_T_gather(int64_t n, const int32_t* erp, const int32_t* ee, const int32_t* ep, const double* atval,
                    const double* T, int64_t ld, double* S, hipStream_t st);
// Schur contribution A' M A of the cone rows as a gather (no atomics, a fixed
// order).  The rows the cones couple form groups g (one per cone; one per row
// of a zero or nonneg segment) with the sorted union U_g of their columns.
// group_T: T_g = M_g A_g (|R_g| x |U_g|, row-major at T + t_off[g]), one wave
// per group, a lane per column of U_g summing over that column's entries of
// the group's rows (c_ptr / c_b / c_k: per entry of the concatenated U lists,
// the group-local row b and the index k of the entry in A), in row order; gm
// (|R_g|^2 per group at m_off[g]) holds the index of M_g[a][b] in mval or -1.
// group_gather: column j of S (rows i >= j) gains sum over the rows r of
// column j of A, in order, of A[r][j] T_r[i]; one wave per column, the column
// in LDS chunks of GATHER_CHUNK rows.
constexpr int GATHER_CHUNK = 4096;
struct GroupPlan {
  int64_t ng = 0;
  const int64_t *rows_off = nullptr, *u_off = nullptr, *m_off = nullptr, *t_off = nullptr, *gm = nullptr,
                *c_ptr = nullptr;
  const int32_t *rows = nullptr, *u = nullptr, *c_b = nullptr, *c_k = nullptr, *rgrp = nullptr, *rloc = nullptr;
  // per entry of A' (the column gather's rows): offset of the row's T row,
  // its group's column list, that list's length (0: the row is in no group)
  const int64_t *e_t = nullptr, *e_u = nullptr;
  const int32_t* e_s = nullptr;
  double* T = nullptr;
};
void group_T(const GroupPlan& gp, const double* mval, const Csr& A, hipStream_t st);
void group_gather(const GroupPlan& gp, int64_t n, const Csr& At, int64_t ld, double* S, hipStream_t st);
// Ordered Schur sums (no atomics, a fixed order): destination d gains the sum,
// in list order, of its terms k in [ptr[d], ptr[d + 1]).  Pair terms are
// mval[pm[k]] A[pp[k]] A[q] with q = pq[k], or q = ~pq[k] and the term doubled
// when pq[k] < 0 (the two products of a row pair that meet on the diagonal);
// slot terms (pm == nullptr) are slot[pp[k]].  dst[d] names the entry: bits
// 62-63 select base[0], base[1] or base[2], the rest is the offset in it; no
// two destinations name one entry.  Destinations [0, nshort) run one lane
// each, the rest (more than ORDERED_WIDE terms) one wave each with a fixed
// shuffle-tree sum.
constexpr int ORDERED_WIDE = 32;
struct OrderedSum {
  int64_t nd = 0, nshort = 0;
  const int64_t *ptr = nullptr, *dst = nullptr;
  const int32_t *pm = nullptr, *pp = nullptr, *pq = nullptr;
};
void ordered_sum(const OrderedSum& os, const double* mval, const double* av, const double* slot, double* b0,
                 double* b1, double* b2, hipStream_t st);
void scale_dense_rows(int nd, int64_t n, const double* Ad, const int64_t* midx, const double* mval, double* B,
                      hipStream_t st);
void aos_to_cm(int64_t count, int dim, const double* a, double* c, bool inverse, hipStream_t st);

}  // namespace hc
