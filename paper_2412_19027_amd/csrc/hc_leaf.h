// Two-level factorisation of the Schur complement S = P + delta I + A' M A.
//
// The columns of S are split at setup into a dense tail and small leaf blocks:
// after the tail columns are removed from the graph of S, every connected
// component (at most LEAF_MAX columns) is one leaf.  Ordered leaves first,
//
//   S = [ S_LL  S_TL' ]      S_LL block diagonal (one dense block per leaf),
//       [ S_TL  S_TT  ]      S_TL: each leaf couples to a few tail columns,
//
// so the LDL' of Sec. 3.7 becomes: per leaf L_b L_b' = S_bb and
// W_b = S_Tb L_b^-T (batched, one wave per leaf), then the tail
// S_TT - sum_b W_b W_b' is factored densely on MFMA.  The leaves are the
// "many tiny supernodes" of a supernodal factorisation and the tail its dense
// root supernode.
#pragma once
#include "hc_common.h"

namespace hc {

constexpr int LEAF_MAX = 32;       // columns per leaf block
constexpr int LEAF_CPL_MAX = 64;   // tail columns coupled to one leaf
constexpr int LEAF_SMALL = 4;      // leaves up to this size are solved one lane per leaf

// Where column j of S lives: leaf[j] < 0 -> tail index loc[j]; otherwise
// leaf block leaf[j], local index loc[j].  All arrays are device arrays.
struct ColMap {
  int64_t nleaf = 0, nt = 0, ldt = 0;
  const int32_t* leaf = nullptr;       // per column
  const int32_t* loc = nullptr;        // per column
  const int32_t* tcols = nullptr;      // per tail index: column
  const int32_t* lsize = nullptr;      // per leaf: l
  const int64_t* lval_off = nullptr;   // per leaf: l x l block, column-major, lower part used
  const int64_t* lcol_off = nullptr;   // per leaf: offset of its columns in lcols
  const int32_t* lcols = nullptr;      // leaf columns, ascending within a leaf
  const int32_t* ccnt = nullptr;       // per leaf: coupled tail columns
  const int64_t* clist_off = nullptr;  // per leaf: offset in clist (and in cval / l)
  const int32_t* clist = nullptr;      // coupled tail indices, ascending within a leaf
  const int64_t* cval_off = nullptr;   // per leaf: ccnt x l block, column-major
  double* lval = nullptr;              // leaf blocks (S_bb, then L_b)
  double* cval = nullptr;              // coupling blocks (S_Tb, then W_b)
  double* ST = nullptr;                // tail matrix, column-major, leading dim ldt
  double* sink = nullptr;              // one double: target of impossible pairs
  // the leaf solves: leaves of at most LEAF_SMALL columns (one lane each) and
  // the rest (one wave each), and per tail index its couplings (the leaf and
  // the row of that leaf's coupling block), for a gather instead of atomics
  int64_t nsmall = 0, nlarge = 0;
  const int32_t* small = nullptr;
  const int32_t* large = nullptr;
  const int64_t* tc_ptr = nullptr;     // nt + 1: per tail index its range of W entries
  int32_t tail_threads = 64;           // threads per tail index in the tail gather (64, 256 or 1024)
  const int64_t* te_cv = nullptr;      // per entry: index into cval
  const int32_t* te_y = nullptr;       // per entry: the leaf column it multiplies
  // per leaf the first of its cnt (cnt + 1) / 2 slots: with lslot set the leaf
  // factor stores -(W_b W_b')[a][c] there (pair p = a (a + 1) / 2 + c) and an
  // ordered sum adds the slots to S_TT, instead of FP64 atomics
  double* lslot = nullptr;
  const int64_t* lp_off = nullptr;
};

// Schur assembly over row pairs of one cone (as assemble_pairs), routed
// through the column map; wide: one wave per task.
void assemble_pairs_map(int64_t ntask, const int32_t* tra, const int32_t* trb, const int64_t* tm, const double* mval,
                        const Csr& A, const ColMap& cm, bool wide, hipStream_t st);
// P (full CSR, lower part used) and delta on the diagonal, through the map.
void add_P_delta_map(const Csr& P, int64_t n, double delta, const ColMap& cm, hipStream_t st);
// Per leaf: Cholesky of S_bb (pivots <= tol replaced by fix and counted),
// W_b = S_Tb L_b^-T, and S_TT -= W_b W_b' (lower part: into cm.lslot for an
// ordered sum when set, else with FP64 atomics).
void leaf_factor(const ColMap& cm, double tol, double fix, unsigned long long* hits, hipStream_t st);
// Forward half of the leaf solve: y_b = L_b^-1 u_b written to y at the leaf
// columns, then uT[t] -= sum over the leaves coupled to t of (W_b y_b)[t]
// (uT: compact tail vector, already gathered), one writer per t in a fixed
// order.
void leaf_forward(const ColMap& cm, const double* u, double* y, double* uT, hipStream_t st);
// Backward half: x_b = L_b^-T (y_b - W_b' xT), reading y_b from x at the
// leaf columns and overwriting it.
void leaf_backward(const ColMap& cm, const double* xT, double* x, hipStream_t st);
// uT[t] = u[tcols[t]] and x[tcols[t]] = xT[t]
void gather_tail(const ColMap& cm, const double* u, double* uT, hipStream_t st);
void scatter_tail(const ColMap& cm, const double* xT, double* x, hipStream_t st);

}  // namespace hc
