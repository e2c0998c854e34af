// hipcone solver: setup on the host, every per-iteration step on the GPU.
//
// Algorithm 1 (Sec. 3.2) step by step; the host holds only scalars (tau,
// kappa, step lengths, reduction results) and launches the kernels of the
// cone layer (hc_cones.hip), the vector/sparse layer (hc_vec.hip) and the
// dense factorisation of the KKT Schur complement (hc_dense.hip).
//
// Readings where the paper is silent or inconsistent (same as the design
// notes):
//   * Delta tau uses the first printed form of eq. step-direction;
//   * affine d: d_kappa = kappa tau, d_s = s;
//   * regularisation: +delta on the P block, -delta on the -H block;
//     delta = delta_s + delta_d max_i |K_ii|;
//   * refinement: first solve + at most ir_max corrections, stop on the
//     tolerance or when a correction fails to halve the residual; FP32
//     right-hand sides are scaled by 1/||r||_inf;
//   * step rule: alpha_0 = min(1, tau/kappa ratio tests, symmetric-cone
//     boundary steps), then x0.8 backtracking while an exp/pow cone leaves its
//     interior or (combined step) violates N(beta); zero below 1e-10;
//   * alpha_c < 0.1 with a primal-dual exp/pow scaling -> the iteration is
//     redone with the dual scaling; alpha_c < 1e-4 -> insufficient progress;
//   * equilibration: 10 modified Ruiz passes (factors clamped to
//     [1e-4, 1e4], row factors averaged over each SOC/exp/pow/PSD cone), cost
//     scale 1/max(1, mean column max of P, |Dq|_inf);
//   * dual-infeasibility test multiplies by q'x.
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "hc_cones.h"
#include "hc_dense.h"
#include "hc_leaf.h"
#include "hc_symbolic.h"
#include "hc_vec.h"
#include "hc_wave.h"

using namespace hc;

namespace {

thread_local std::string g_last_error;

struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};

struct Buf {   // bump allocator over one device block; `dry` only counts bytes
  char* base = nullptr;
  size_t size = 0, used = 0;
  bool dry = false;
  template <typename T> T* take(size_t count) {
    size_t bytes = ((std::max<size_t>(count, 1) * sizeof(T) + 255) / 256) * 256;
    if (!dry && used + bytes > size) throw Error{HC_ERR_OOM, "device arena exhausted"};
    T* p = dry ? nullptr : reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

}  // namespace

struct hc_solver {
  hc_settings st{};
  int64_t n = 0, m = 0;
  // ---- host setup products
  std::vector<int64_t> perm;       // internal row -> user row
  std::vector<Segment> segs;
  std::vector<double> alpha_pow;   // POW exponents in segment order
  HostCsr A, At, P;                // scaled, internal order (A without dense rows)
  std::vector<double> Ad;          // dense rows, row-major nd x n
  std::vector<int32_t> drows;      // their internal rows
  std::vector<int64_t> dmidx;      // their M index
  // second-order cones above SOC_DMAX enter S as f_o A_c'A_c (diagonal tasks)
  // plus two dense rows each, p_- = A_c'v_- (weight f_- - f_o >= 0) and
  // p_+ = A_c'v_+ (weight f_+ - f_o <= 0).  Dense-row operand rows:
  // [0, nd) real dense rows, [nd, nd + nls) p_-, zero padding to K1 (a multiple
  // of 16, product with +1), [K1, K1 + nls) p_+, padding to K1 + K2 (with -1).
  int64_t nls = 0, K1 = 0, K2 = 0;
  std::vector<int64_t> dmidx_all;  // M index per operand row (-1: padding)
  std::vector<int32_t> ls_cone, ls_col;   // (cone, column) entries of the p rows
  std::vector<int64_t> ls_dst;            // offset of p_- for the entry in the operand
  struct LsRange {
    int seg;
    int64_t first, count;
  };
  std::vector<LsRange> ls_ranges;  // entries of each large-SOC segment
  std::vector<double> q, b, D, E;  // scaled q, b; equilibration factors
  double cscale = 1.0;
  double bnorm_user = 0, qnorm_user = 0, maxPdiag = 0;
  int64_t nu = 0;                  // cone degree
  bool has_nonsym = false;
  // Schur assembly by groups (the cones' row sets) and a column gather; the
  // pair tasks below keep only what the groups do not take
  std::vector<int64_t> ga_rows_off, ga_u_off, ga_m_off, ga_t_off, ga_gm, ga_c_ptr;
  std::vector<int32_t> ga_rows, ga_u, ga_c_b, ga_c_k, ga_rgrp, ga_rloc;
  std::vector<int64_t> ga_e_t, ga_e_u;   // per entry of A': its T row and column list
  std::vector<int32_t> ga_e_s;           // and the list's length (0: row in no group)
  int64_t ga_ng = 0, ga_t_total = 0;
  GroupPlan gplan;
  std::vector<int32_t> tra, trb;   // Schur assembly tasks: short ones first, then
  std::vector<int64_t> tm;         // those of more than PAIR_WIDE products (one wave each)
  int64_t ntask_short = 0;
  // PSD segments assembled by the T = M_c A_c gather (build_psd_dense): their
  // segment index and first T row; per column j of A the T rows and the
  // positions of their values in A' (so new values need no rebuild)
  std::vector<std::pair<int, int64_t>> pdense;
  std::vector<int32_t> pe_rp, pe_e, pe_p;
  int64_t pe_rows = 0;
  // and per cone of those segments (pdense_coff: each segment's first cone)
  // its columns with their entries, for the column-ordered T rows
  std::vector<int64_t> pdense_coff, pc_cu_off, pc_cu_ptr;
  std::vector<int32_t> pc_cu_col, pc_cu_b, pc_cu_p;
  PsdCols pcols;
  // ordered Schur sums (build_ordered): the products of the pair tasks grouped
  // by the entry of S they land on, and the leaves' updates of S_TT grouped by
  // tail entry (leaf_lp_off: each leaf's first slot); `ordered` is false when
  // the lists would exceed ORDERED_MAX_TERMS (the FP64-atomic kernels run)
  bool ordered = false;
  std::vector<int64_t> op_ptr, op_dst, ol_ptr, ol_dst, leaf_lp_off;
  std::vector<int32_t> op_pm, op_pp, op_pq, ol_pp;
  int64_t op_nshort = 0, ol_nshort = 0, lpair_total = 0;
  OrderedSum opair, oleaf;
  // two-level split of the Schur complement (leaf blocks + dense tail)
  int64_t nt = 0;                  // tail columns
  std::vector<int64_t> tail_last;  // envelope of the tail (see dense_cholesky), padded to ld
  bool leaves = false;             // any leaf block
  std::vector<int32_t> col_leaf, col_loc, tail_cols, leaf_size, leaf_cols, leaf_ccnt, leaf_clist;
  std::vector<int64_t> leaf_lval_off, leaf_lcol_off, leaf_clist_off, leaf_cval_off;
  std::vector<int32_t> leaf_small, leaf_large;   // solve lists
  std::vector<int64_t> tc_ptr, te_cv;             // per tail index its W entries: index into cval,
  std::vector<int32_t> te_y;                      // and the leaf column they multiply
  int64_t lval_total = 0, cval_total = 0;
  double leaf_flops = 0;
  int64_t mtotal = 0, stotal = 0;  // M entries, state entries
  int64_t ld = 0;
  bool mixed = false;
  // ---- device
  bool bound = false;
  bool noalloc = false;             // bound to the static workspace for one hc_solve_noalloc call
  // symbolic analysis of the components split along their elimination tree
  int64_t sym_split_columns = 0, sym_supernodes = 0, sym_levels = 0, sym_nnz_l = 0;
  bool own_mem = false;
  void* mem = nullptr;
  size_t mem_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  Csr dA, dAt, dP;
  double *dAd = nullptr, *dBd = nullptr;
  int32_t* ddrows = nullptr;
  int64_t* ddmidx = nullptr;
  double* dDrT = nullptr;           // per-chunk partial sums of A'z over the dense rows
  double* dmwork = nullptr;         // scratch of the PSD M blocks (largest segment's need)
  int32_t *dpe_rp = nullptr, *dpe_e = nullptr, *dpe_p = nullptr;
  double* dT = nullptr;   // the T rows of the gathered PSD segments (pe_rows x n)
  int32_t *dls_cone = nullptr, *dls_col = nullptr;
  int64_t* dls_dst = nullptr;
  double *dq = nullptr, *db = nullptr, *dD = nullptr, *dE = nullptr, *dalpha = nullptr;
  int64_t* dperm = nullptr;         // internal row -> user row (device copy of perm)
  double *wx = nullptr, *ws = nullptr, *wz = nullptr;   // last solved iterate, unscaled, internal rows
  bool have_warm = false;
  int32_t *dtra = nullptr, *dtrb = nullptr;
  int64_t* dtm = nullptr;
  double *dstate = nullptr, *dmval = nullptr, *dhdiag = nullptr;
  double* dS = nullptr;             // dense tail (nt x nt, leading dim ld)
  double* dLinv = nullptr;
  ColMap cm;                        // column map of the two-level split
  double *uT = nullptr, *xT = nullptr;   // compact tail vectors
  double *uTb = nullptr, *xTb = nullptr; // and those of a second right-hand side
  float *dS32 = nullptr, *dLinv32 = nullptr;
  double *dX256 = nullptr, *dXT256 = nullptr;
  float *dX256f = nullptr, *dXT256f = nullptr;
  unsigned long long* dhits = nullptr;
  int* dpd = nullptr;
  double* dscal = nullptr;          // device scalars (FP32 rhs scale)
  int64_t npart = 0;                // capacity of the partial buffers (two reductions, or every segment's step partials)
  double* dpart = nullptr;          // reduction partials
  double* hpart = nullptr;          // pinned host copy
  bool own_stage = false;           // hpart/hmask allocated here (no caller staging)
  unsigned long long *dmask = nullptr, *hmask = nullptr;
  // iterate and work vectors
  double *x, *s, *z;
  double tau = 1, kappa = 1;
  double *Px, *Ax, *Atz, *rdv, *rpv;   // rdv = Px + A'z + q tau ; rpv = -Ax - s + b tau
  double *x2, *z2, *x1, *z1, *dx, *dz, *dsv, *dsrhs, *dxa, *dza, *dsa;
  double *r1, *r2, *irx, *irz, *irxn, *irzn, *irbx, *irbz, *irrx, *irrz, *kx, *kz, *t1, *t2, *u1, *w1;
  double *sb, *sy, *sx;             // dense solve buffers (two right-hand sides of n_T)
  // the second system's refinement vectors (kkt_solve_pair) and the constant
  // system's first block
  double *jrx, *jrz, *jrxn, *jrzn, *jrbx, *jrbz, *jrrx, *jrrz, *jkx, *jkz, *u1b, *r1c;
  float *sb32, *sy32, *sx32;
  std::vector<SegDev> sdev;
  // ---- results
  hc_info info{};
  int status = 0;
  double delta = 0;
  double xPx_cache = 0;             // x'Px of the current iterate (from residuals)
  std::unique_ptr<Prof> prof;
  std::unique_ptr<Prof> cprof;      // events around the cone-layer launches (settings.profile)
  Aux aux;   // side stream + events of the look-ahead factorisation
  bool use64 = false;               // mixed mode: this iteration fell back to the FP64 factor
  int kiter = 0;                    // loop counter of the current solve
  double sdiag_max = 0;             // mixed mode: max |S_ii| of the last FP32 factorisation
  double t_begin = 0;               // host clock at the start of the solve
  double* snap_S = nullptr;         // test hook: host copy of the dense tail before its Cholesky
  // the user's data as last given (structure fixed at setup), for hc_update_data
  std::vector<int64_t> uPrp, uArp;
  std::vector<int32_t> uPci, uAci;
  std::vector<double> uPv, uq, uAv, ub;
  std::vector<hc_cone> ucones;
  std::string last_error;
};

namespace {

// ===========================================================================
// setup
// ===========================================================================
void fail(int32_t code, const std::string& msg) { throw Error{code, msg}; }

void validate(const hc_problem* p) {
  if (!p) fail(HC_ERR_INVALID_ARG, "problem is NULL");
  if (p->n <= 0 || p->m <= 0) fail(HC_ERR_DIM, "n and m must be positive");
  if (p->n >= (int64_t)1 << 31 || p->m >= (int64_t)1 << 31) fail(HC_ERR_UNSUPPORTED, "n or m exceeds 2^31");
  if (!p->q || !p->b || !p->A_rowptr || !p->cones || p->ncones <= 0) fail(HC_ERR_INVALID_ARG, "NULL array");
  const int64_t nnzA = p->A_rowptr[p->m];
  if (nnzA > 0 && (!p->A_col || !p->A_val)) fail(HC_ERR_INVALID_ARG, "A arrays NULL");
  if (nnzA >= (int64_t)1 << 31) fail(HC_ERR_UNSUPPORTED, "nnz(A) exceeds 2^31");
  if (p->A_rowptr[0] != 0) fail(HC_ERR_CSR, "A rowptr[0] != 0");
  for (int64_t i = 0; i < p->m; ++i) {
    if (p->A_rowptr[i + 1] < p->A_rowptr[i]) fail(HC_ERR_CSR, "A rowptr decreasing");
    for (int64_t k = p->A_rowptr[i]; k < p->A_rowptr[i + 1]; ++k) {
      if (p->A_col[k] < 0 || p->A_col[k] >= p->n) fail(HC_ERR_CSR, "A column out of range");
      if (k > p->A_rowptr[i] && p->A_col[k] <= p->A_col[k - 1]) fail(HC_ERR_CSR, "A columns unsorted or duplicate");
      if (!std::isfinite(p->A_val[k])) fail(HC_ERR_NONFINITE, "A has a non-finite value");
    }
  }
  if (p->P_rowptr) {
    if (p->P_rowptr[0] != 0) fail(HC_ERR_CSR, "P rowptr[0] != 0");
    const int64_t nnzP = p->P_rowptr[p->n];
    if (nnzP > 0 && (!p->P_col || !p->P_val)) fail(HC_ERR_INVALID_ARG, "P arrays NULL");
    for (int64_t i = 0; i < p->n; ++i) {
      if (p->P_rowptr[i + 1] < p->P_rowptr[i]) fail(HC_ERR_CSR, "P rowptr decreasing");
      for (int64_t k = p->P_rowptr[i]; k < p->P_rowptr[i + 1]; ++k) {
        if (p->P_col[k] < i || p->P_col[k] >= p->n) fail(HC_ERR_CSR, "P entry below the diagonal or out of range");
        if (k > p->P_rowptr[i] && p->P_col[k] <= p->P_col[k - 1]) fail(HC_ERR_CSR, "P columns unsorted or duplicate");
        if (!std::isfinite(p->P_val[k])) fail(HC_ERR_NONFINITE, "P has a non-finite value");
      }
    }
  }
  for (int64_t j = 0; j < p->n; ++j)
    if (!std::isfinite(p->q[j])) fail(HC_ERR_NONFINITE, "q has a non-finite value");
  for (int64_t i = 0; i < p->m; ++i)
    if (!std::isfinite(p->b[i])) fail(HC_ERR_NONFINITE, "b has a non-finite value");
  int64_t rows = 0;
  for (int c = 0; c < p->ncones; ++c) {
    const hc_cone& k = p->cones[c];
    switch (k.type) {
      case HC_CONE_ZERO:
      case HC_CONE_NONNEG:
        if (k.dim < 1) fail(HC_ERR_CONE, "zero/nonneg dim < 1");
        rows += k.dim;
        break;
      case HC_CONE_SOC:
        if (k.dim < 2) fail(HC_ERR_CONE, "SOC dim < 2");
        if (k.dim > (1 << 24)) fail(HC_ERR_UNSUPPORTED, "SOC dim > 2^24 is not handled by this build");
        rows += k.dim;
        break;
      case HC_CONE_EXP:
        if (k.dim != 3) fail(HC_ERR_CONE, "EXP dim != 3");
        rows += 3;
        break;
      case HC_CONE_POW:
        if (k.dim != 3) fail(HC_ERR_CONE, "POW dim != 3");
        if (!(k.alpha > 0.0 && k.alpha < 1.0)) fail(HC_ERR_CONE, "POW alpha outside (0,1)");
        rows += 3;
        break;
      case HC_CONE_PSD:
        if (k.dim < 1 || k.dim > 32) fail(HC_ERR_CONE, "PSD side outside [1, 32]");
        rows += (int64_t)k.dim * (k.dim + 1) / 2;
        break;
      default:
        fail(HC_ERR_CONE, "unknown cone type");
    }
  }
  if (rows != p->m) fail(HC_ERR_DIM, "cone rows do not add up to m");
}

void build_segments(hc_solver* S, const hc_problem* p) {
  std::vector<int64_t> zero_rows, nn_rows, exp_st, pow_st;
  std::vector<double> pow_a;
  std::map<int, std::vector<int64_t>> soc_st, psd_st;   // by SOC dim / PSD side
  int64_t r = 0;
  for (int c = 0; c < p->ncones; ++c) {
    const hc_cone& k = p->cones[c];
    switch (k.type) {
      case HC_CONE_ZERO: for (int j = 0; j < k.dim; ++j) zero_rows.push_back(r + j); r += k.dim; break;
      case HC_CONE_NONNEG: for (int j = 0; j < k.dim; ++j) nn_rows.push_back(r + j); r += k.dim; break;
      case HC_CONE_SOC: soc_st[k.dim].push_back(r); r += k.dim; break;
      case HC_CONE_EXP: exp_st.push_back(r); r += 3; break;
      case HC_CONE_POW: pow_st.push_back(r); pow_a.push_back(k.alpha); r += 3; break;
      case HC_CONE_PSD: psd_st[k.dim].push_back(r); r += (int64_t)k.dim * (k.dim + 1) / 2; break;
    }
  }
  S->perm.assign(S->m, -1);
  int64_t base = 0, state = 0, moff = 0;
  auto add = [&](int kind, int64_t count, int dim, int k) {
    Segment g{kind, base, count, dim, k, state, moff};
    S->segs.push_back(g);
    const int64_t units = (kind == HC_CONE_ZERO || kind == HC_CONE_NONNEG) ? count : count;
    state += state_doubles(kind, dim, k) * units;
    moff += mblock_doubles(kind, dim) * units;
    base += (kind == HC_CONE_ZERO || kind == HC_CONE_NONNEG) ? count : count * dim;
  };
  if (!zero_rows.empty()) {
    for (size_t i = 0; i < zero_rows.size(); ++i) S->perm[base + i] = zero_rows[i];
    add(HC_CONE_ZERO, zero_rows.size(), 1, 0);
  }
  if (!nn_rows.empty()) {
    for (size_t i = 0; i < nn_rows.size(); ++i) S->perm[base + i] = nn_rows[i];
    add(HC_CONE_NONNEG, nn_rows.size(), 1, 0);
  }
  for (auto& kv : soc_st) {
    const int d = kv.first;
    const int64_t N = kv.second.size();
    for (int64_t i = 0; i < N; ++i)
      for (int j = 0; j < d; ++j) S->perm[base + j * N + i] = kv.second[i] + j;
    add(HC_CONE_SOC, N, d, 0);
  }
  if (!exp_st.empty()) {
    const int64_t N = exp_st.size();
    for (int64_t i = 0; i < N; ++i)
      for (int j = 0; j < 3; ++j) S->perm[base + j * N + i] = exp_st[i] + j;
    add(HC_CONE_EXP, N, 3, 0);
  }
  if (!pow_st.empty()) {
    const int64_t N = pow_st.size();
    for (int64_t i = 0; i < N; ++i)
      for (int j = 0; j < 3; ++j) S->perm[base + j * N + i] = pow_st[i] + j;
    S->alpha_pow = pow_a;
    add(HC_CONE_POW, N, 3, 0);
  }
  // PSD cones of several sides: one segment per side (ascending), each with
  // its own k, state and M-block layout
  for (auto& kv : psd_st) {
    const int pk = kv.first;
    const int64_t N = kv.second.size();
    const int sd = pk * (pk + 1) / 2;
    for (int64_t i = 0; i < N; ++i)
      for (int j = 0; j < sd; ++j) S->perm[base + i * sd + j] = kv.second[i] + j;
    add(HC_CONE_PSD, N, sd, pk);
  }
  S->stotal = state;
  S->mtotal = moff;
  S->nu = 0;
  for (auto& g : S->segs) {
    if (g.kind == HC_CONE_NONNEG) S->nu += g.count;
    else if (g.kind == HC_CONE_SOC) S->nu += g.count;
    else if (g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW) S->nu += 3 * g.count;
    else if (g.kind == HC_CONE_PSD) S->nu += (int64_t)g.k * g.count;
    if (g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW) S->has_nonsym = true;
  }
}

// internal row -> (segment index, cone index, local component)
struct RowLoc {
  int seg;
  int64_t cone;
  int comp;
};
RowLoc locate(const hc_solver* S, int64_t r) {
  for (int gi = 0; gi < (int)S->segs.size(); ++gi) {
    const Segment& g = S->segs[gi];
    const int64_t rows = (g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG) ? g.count : g.count * g.dim;
    if (r >= g.base && r < g.base + rows) {
      const int64_t o = r - g.base;
      if (g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG) return {gi, o, 0};
      if (g.kind == HC_CONE_PSD) return {gi, o / g.dim, (int)(o % g.dim)};
      return {gi, o % g.count, (int)(o / g.count)};
    }
  }
  return {-1, 0, 0};
}

void equilibrate(hc_solver* S, const HostCsr& A, const HostCsr& Pf, const std::vector<double>& q) {
  const int64_t n = S->n, m = S->m;
  S->D.assign(n, 1.0);
  S->E.assign(m, 1.0);
  S->cscale = 1.0;
  if (!S->st.equilibrate) return;
  const double lo = 1e-4, hi = 1e4;
  auto clampv = [&](double v) { return std::min(std::max(v, lo), hi); };
  std::vector<double> colP(n), colA(n), rowA(m), d(n), e(m);
  for (int it = 0; it < S->st.equil_iters; ++it) {
    std::fill(colP.begin(), colP.end(), 0.0);
    std::fill(colA.begin(), colA.end(), 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t k = Pf.rp[i]; k < Pf.rp[i + 1]; ++k) {
        const int32_t j = Pf.ci[k];
        colP[j] = std::max(colP[j], std::fabs(S->D[i] * Pf.v[k] * S->D[j]));
      }
    for (int64_t i = 0; i < m; ++i) {
      double rmax = 0;
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int32_t j = A.ci[k];
        const double v = std::fabs(S->E[i] * A.v[k] * S->D[j]);
        colA[j] = std::max(colA[j], v);
        rmax = std::max(rmax, v);
      }
      rowA[i] = rmax;
    }
    for (int64_t j = 0; j < n; ++j) {
      const double cn = std::max(colP[j], colA[j]);
      d[j] = cn > 0 ? 1.0 / std::sqrt(cn) : 1.0;
    }
    for (int64_t i = 0; i < m; ++i) e[i] = rowA[i] > 0 ? 1.0 / std::sqrt(rowA[i]) : 1.0;
    // cone-uniform row factors for the non-separable cones
    for (const Segment& g : S->segs) {
      if (g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG) continue;
      for (int64_t c = 0; c < g.count; ++c) {
        double sum = 0;
        for (int j = 0; j < g.dim; ++j) {
          const int64_t r = (g.kind == HC_CONE_PSD) ? g.base + c * g.dim + j : g.base + j * g.count + c;
          sum += e[r];
        }
        const double mean = sum / g.dim;
        for (int j = 0; j < g.dim; ++j) {
          const int64_t r = (g.kind == HC_CONE_PSD) ? g.base + c * g.dim + j : g.base + j * g.count + c;
          e[r] = mean;
        }
      }
    }
    for (int64_t j = 0; j < n; ++j) S->D[j] = clampv(S->D[j] * clampv(d[j]));
    for (int64_t i = 0; i < m; ++i) S->E[i] = clampv(S->E[i] * clampv(e[i]));
  }
  std::fill(colP.begin(), colP.end(), 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = Pf.rp[i]; k < Pf.rp[i + 1]; ++k) {
      const int32_t j = Pf.ci[k];
      colP[j] = std::max(colP[j], std::fabs(S->D[i] * Pf.v[k] * S->D[j]));
    }
  double mean = 0;
  for (int64_t j = 0; j < n; ++j) mean += colP[j];
  mean /= (double)n;
  double dq = 0;
  for (int64_t j = 0; j < n; ++j) dq = std::max(dq, std::fabs(S->D[j] * q[j]));
  S->cscale = clampv(1.0 / std::max(1.0, std::max(mean, dq)));
}

// ---------------------------------------------------------------------------
// Two-level split of the Schur complement.  The graph of S is the union of one
// clique per cone (the columns its rows touch; every nonneg/zero row is a cone
// of its own) and the off-diagonal entries of P.  Columns touched by a dense
// row or of estimated degree above LEAF_DEGREE go to the dense tail; the
// connected components of the remaining columns become leaf blocks when they
// have at most LEAF_MAX columns and touch at most LEAF_CPL_MAX tail columns,
// otherwise they join the tail.  Removing a component from the leaves never
// changes another leaf's coupling (distinct components are not adjacent).
// ---------------------------------------------------------------------------
constexpr int LEAF_DEGREE = 64;
constexpr int64_t PAIR_WIDE = 1024;   // products per pair task above which one wave takes the task

void build_psd_dense(hc_solver* S);
void build_groups(hc_solver* S);
void build_ordered(hc_solver* S);
void build_lowrank(hc_solver* S, int nd);

// Leaf blocks from the symbolic analysis of the columns outside the tail:
// their graph (cliques and P restricted to them) is ordered by approximate
// minimum degree and its elimination tree postordered, so that every subtree
// is a run of consecutive columns.  A subtree couples, outside itself, only
// to its ancestors (the factor column of its root, without the root) and to
// tail columns; the maximal subtrees of at most LEAF_MAX columns with at most
// LEAF_CPL_MAX such couplings become leaf blocks (a connected component that
// fits is one subtree), and the other columns join the tail.  The symbolic
// figures (supernodes, level sets, factor nonzeros of this graph) are
// recorded in the handle.  Should a subtree touch a column of another leaf
// (which the tree rules out), or the ordering exceed its work limit, every
// component of more than LEAF_MAX columns goes to the tail whole and the
// others stay leaf candidates as they are.
void etree_leaves(hc_solver* S, std::vector<std::vector<int32_t>>& comp, std::vector<char>& tail,
                  const std::vector<int64_t>& cp, const std::vector<int32_t>& cc, const std::vector<int64_t>& ip,
                  const std::vector<int32_t>& inc) {
  const HostCsr& P = S->P;
  const int64_t n = S->n;
  std::vector<int32_t> big;
  for (auto& c : comp) big.insert(big.end(), c.begin(), c.end());
  if (big.empty()) return;
  std::vector<std::vector<int32_t>> saved;
  saved.swap(comp);
  auto to_tail = [&]() {   // the rule without the tree: components that fit stay candidates
    comp.clear();
    for (auto& c : saved) {
      if ((int)c.size() > LEAF_MAX) {
        for (int32_t j : c) tail[j] = 1;
      } else {
        comp.push_back(c);
      }
    }
  };
  std::sort(big.begin(), big.end());
  const int32_t nb = (int32_t)big.size();
  std::vector<int32_t> loc(n, -1);
  for (int32_t a = 0; a < nb; ++a) loc[big[a]] = a;
  // graph of the components' columns and, per column, its tail neighbours
  SymGraph g;
  g.n = nb;
  g.ptr.assign(nb + 1, 0);
  std::vector<std::vector<int32_t>> nbr(nb), tnb(nb);
  for (int32_t a = 0; a < nb; ++a) {
    const int32_t j = big[a];
    for (int64_t e = ip[j]; e < ip[j + 1]; ++e) {
      const int32_t c = inc[e];
      for (int64_t f = cp[c]; f < cp[c + 1]; ++f) {
        const int32_t u = cc[f];
        if (u == j) continue;
        if (loc[u] >= 0) nbr[a].push_back(loc[u]);
        else if (tail[u]) tnb[a].push_back(u);
      }
    }
    for (int32_t k = P.rp[j]; k < P.rp[j + 1]; ++k) {
      const int32_t u = P.ci[k];
      if (u == j) continue;
      if (loc[u] >= 0) {
        nbr[a].push_back(loc[u]);
        nbr[loc[u]].push_back(a);
      } else if (tail[u]) {
        tnb[a].push_back(u);
      }
    }
  }
  for (int32_t a = 0; a < nb; ++a) {
    for (int32_t k = P.rp[big[a]]; k < P.rp[big[a] + 1]; ++k) {   // P's other triangle
      const int32_t u = P.ci[k];
      if (u != big[a] && loc[u] < 0 && tail[u]) tnb[a].push_back(u);
    }
    std::sort(nbr[a].begin(), nbr[a].end());
    nbr[a].erase(std::unique(nbr[a].begin(), nbr[a].end()), nbr[a].end());
    std::sort(tnb[a].begin(), tnb[a].end());
    tnb[a].erase(std::unique(tnb[a].begin(), tnb[a].end()), tnb[a].end());
    g.ptr[a + 1] = g.ptr[a] + (int64_t)nbr[a].size();
  }
  g.adj.reserve(g.ptr[nb]);
  for (int32_t a = 0; a < nb; ++a) g.adj.insert(g.adj.end(), nbr[a].begin(), nbr[a].end());
  // symmetric closure (P may be stored as one triangle)
  {
    std::vector<std::vector<int32_t>> sym(nb);
    for (int32_t a = 0; a < nb; ++a)
      for (int32_t b : nbr[a]) {
        sym[a].push_back(b);
        sym[b].push_back(a);
      }
    g.adj.clear();
    for (int32_t a = 0; a < nb; ++a) {
      std::sort(sym[a].begin(), sym[a].end());
      sym[a].erase(std::unique(sym[a].begin(), sym[a].end()), sym[a].end());
      g.ptr[a + 1] = g.ptr[a] + (int64_t)sym[a].size();
      g.adj.insert(g.adj.end(), sym[a].begin(), sym[a].end());
    }
  }
  const std::vector<int32_t> o = amd_order(g, 64 * (g.ptr[nb] + nb) + (1 << 20));
  if ((int32_t)o.size() != nb) {
    to_tail();
    return;
  }
  const std::vector<int32_t> par0 = elimination_tree(g, o);
  const std::vector<int32_t> post = tree_postorder(par0);
  std::vector<int32_t> order(nb);
  for (int32_t k = 0; k < nb; ++k) order[k] = o[post[k]];
  const std::vector<int32_t> parent = elimination_tree(g, order);
  std::vector<int32_t> pos(nb);
  for (int32_t k = 0; k < nb; ++k) pos[order[k]] = k;
  // per position: subtree size, its couplings to ancestors (the factor column's
  // rows below the root, exact: the column counts) and to tail columns (kept
  // only up to CAP entries: a set above that stays above it in every ancestor)
  constexpr size_t CAP = LEAF_CPL_MAX + 2;
  std::vector<int32_t> size(nb, 1);
  std::vector<std::vector<int32_t>> up(nb), tl(nb);
  std::vector<char> over(nb, 0);
  std::vector<std::vector<int32_t>> kids(nb);
  for (int32_t k = 0; k < nb; ++k)
    if (parent[k] >= 0) kids[parent[k]].push_back(k);
  std::vector<int32_t> mark(nb, -1);
  std::vector<int64_t> count(nb, 1);
  std::vector<char> eligible(nb, 0);
  for (int32_t k = 0; k < nb; ++k) {
    const int32_t a = order[k];
    auto& u = up[k];
    auto& tt = tl[k];
    mark[k] = k;
    bool ov = false;
    for (int64_t e = g.ptr[a]; e < g.ptr[a + 1]; ++e) {
      const int32_t i = pos[g.adj[e]];
      if (i > k && mark[i] != k) {
        mark[i] = k;
        u.push_back(i);
      }
    }
    tt = tnb[a];
    for (int32_t c : kids[k]) {
      size[k] += size[c];
      ov = ov || over[c];
      for (int32_t i : up[c])
        if (i > k && mark[i] != k) {
          mark[i] = k;
          u.push_back(i);
        }
      tt.insert(tt.end(), tl[c].begin(), tl[c].end());
      std::vector<int32_t>().swap(up[c]);
      std::vector<int32_t>().swap(tl[c]);
    }
    std::sort(tt.begin(), tt.end());
    tt.erase(std::unique(tt.begin(), tt.end()), tt.end());
    count[k] = 1 + (int64_t)u.size();
    if (u.size() + tt.size() > CAP) {   // the ancestor rows stay exact (column counts)
      ov = true;
      tt.resize(std::min(tt.size(), CAP));
    }
    over[k] = ov;
    eligible[k] = !ov && size[k] <= LEAF_MAX && u.size() + tt.size() <= (size_t)LEAF_CPL_MAX;
  }
  // leaves: eligible subtrees whose parent's subtree is not
  std::vector<int32_t> leaf_of(nb, -1);
  std::vector<std::vector<int32_t>> leaves;
  for (int32_t k = 0; k < nb; ++k) {
    if (!eligible[k] || (parent[k] >= 0 && eligible[parent[k]])) continue;
    std::vector<int32_t> cols;
    for (int32_t q = k - size[k] + 1; q <= k; ++q) {
      leaf_of[q] = (int32_t)leaves.size();
      cols.push_back(big[order[q]]);
    }
    leaves.push_back(std::move(cols));
  }
  // every neighbour of a leaf's column lies in the leaf or outside all leaves
  for (int32_t k = 0; k < nb; ++k) {
    if (leaf_of[k] < 0) continue;
    const int32_t a = order[k];
    for (int64_t e = g.ptr[a]; e < g.ptr[a + 1]; ++e) {
      const int32_t other = leaf_of[pos[g.adj[e]]];
      if (other >= 0 && other != leaf_of[k]) {
        to_tail();
        return;
      }
    }
  }
  for (int32_t k = 0; k < nb; ++k)
    if (leaf_of[k] < 0) tail[big[order[k]]] = 1;
  for (auto& c : leaves) comp.push_back(std::move(c));
  std::sort(comp.begin(), comp.end(), [](const std::vector<int32_t>& x, const std::vector<int32_t>& y) {
    return *std::min_element(x.begin(), x.end()) < *std::min_element(y.begin(), y.end());
  });
  // symbolic figures of the split components (their graph, before the split)
  const Supernodes sn = find_supernodes(parent, count);
  S->sym_supernodes += (int64_t)sn.parent.size();
  S->sym_levels = std::max<int64_t>(S->sym_levels, sn.nlevels);
  for (int64_t c : count) S->sym_nnz_l += c;
  S->sym_split_columns += nb;
}

void build_leaves(hc_solver* S) {
  S->sym_split_columns = S->sym_supernodes = S->sym_levels = S->sym_nnz_l = 0;
  const int64_t n = S->n;
  const HostCsr& A = S->A;
  const HostCsr& P = S->P;
  std::vector<char> tail(n, 0);
  const int nd = (int)S->drows.size();
  for (int d = 0; d < nd; ++d)
    for (int64_t j = 0; j < n; ++j)
      if (S->Ad[(size_t)d * n + j] != 0.0) tail[j] = 1;
  // the rank-2 rows of large second-order cones are dense rows on the tail
  for (const Segment& g : S->segs)
    if (soc_large(g.kind, g.dim))
      for (int64_t r = g.base; r < g.base + (int64_t)g.dim * g.count; ++r)
        for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) tail[A.ci[k]] = 1;
  // cliques (CSR over columns)
  std::vector<int64_t> cp{0};
  std::vector<int32_t> cc;
  std::vector<int32_t> buf;
  auto close_clique = [&]() {
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    if (buf.size() > 0) {
      cc.insert(cc.end(), buf.begin(), buf.end());
      cp.push_back((int64_t)cc.size());
    }
    buf.clear();
  };
  auto add_row = [&](int64_t r) {
    for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) buf.push_back(A.ci[k]);
  };
  for (const Segment& g : S->segs) {
    if (g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG) {
      for (int64_t i = 0; i < g.count; ++i) {
        add_row(g.base + i);
        close_clique();
      }
      continue;
    }
    for (int64_t c = 0; c < g.count; ++c) {
      for (int a = 0; a < g.dim; ++a)
        add_row(g.kind == HC_CONE_PSD ? g.base + c * g.dim + a : g.base + (int64_t)a * g.count + c);
      close_clique();
    }
  }
  const int64_t ncl = (int64_t)cp.size() - 1;
  std::vector<int64_t> deg(n, 0);
  for (int64_t c = 0; c < ncl; ++c)
    for (int64_t e = cp[c]; e < cp[c + 1]; ++e) deg[cc[e]] += cp[c + 1] - cp[c] - 1;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k)
      if (P.ci[k] != i) deg[i]++;
  for (int64_t j = 0; j < n; ++j)
    if (!S->st.leaf_blocks || deg[j] > LEAF_DEGREE) tail[j] = 1;
  // connected components of the non-tail columns (union-find)
  std::vector<int32_t> parent(n);
  for (int64_t j = 0; j < n; ++j) parent[j] = (int32_t)j;
  auto find = [&](int32_t x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  };
  auto unite = [&](int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) parent[std::max(a, b)] = std::min(a, b);
  };
  for (int64_t c = 0; c < ncl; ++c) {
    int32_t first = -1;
    for (int64_t e = cp[c]; e < cp[c + 1]; ++e) {
      const int32_t j = cc[e];
      if (tail[j]) continue;
      if (first < 0) first = j;
      else unite(first, j);
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k)
      if (!tail[i] && !tail[P.ci[k]]) unite((int32_t)i, P.ci[k]);
  std::vector<std::vector<int32_t>> comp;   // members, indexed by root order
  std::vector<int32_t> comp_of(n, -1);
  for (int64_t j = 0; j < n; ++j) {
    if (tail[j]) continue;
    const int32_t r = find((int32_t)j);
    if (comp_of[r] < 0) {
      comp_of[r] = (int32_t)comp.size();
      comp.emplace_back();
    }
    comp[comp_of[r]].push_back((int32_t)j);
  }
  // incidence column -> cliques
  std::vector<int64_t> ip(n + 1, 0);
  for (int64_t e = 0; e < (int64_t)cc.size(); ++e) ip[cc[e] + 1]++;
  for (int64_t j = 0; j < n; ++j) ip[j + 1] += ip[j];
  std::vector<int32_t> inc(cc.size());
  {
    std::vector<int64_t> fillp(ip.begin(), ip.end() - 1);
    for (int64_t c = 0; c < ncl; ++c)
      for (int64_t e = cp[c]; e < cp[c + 1]; ++e) inc[fillp[cc[e]]++] = (int32_t)c;
  }
  // leaf blocks: subtrees of the elimination tree of the non-tail columns
  etree_leaves(S, comp, tail, cp, cc, ip, inc);
  std::vector<std::vector<int32_t>> cpl(comp.size());
  for (size_t b = 0; b < comp.size(); ++b) {
    if (tail[comp[b][0]]) continue;
    std::vector<int32_t>& t = cpl[b];
    for (int32_t j : comp[b]) {
      for (int64_t e = ip[j]; e < ip[j + 1]; ++e) {
        const int32_t c = inc[e];
        for (int64_t f = cp[c]; f < cp[c + 1]; ++f)
          if (tail[cc[f]]) t.push_back(cc[f]);
      }
      for (int32_t k = P.rp[j]; k < P.rp[j + 1]; ++k)
        if (tail[P.ci[k]]) t.push_back(P.ci[k]);
    }
    std::sort(t.begin(), t.end());
    t.erase(std::unique(t.begin(), t.end()), t.end());
  }
  for (size_t b = 0; b < comp.size(); ++b)
    if (!tail[comp[b][0]] && (int)cpl[b].size() > LEAF_CPL_MAX)
      for (int32_t j : comp[b]) tail[j] = 1;
  // final numbering: tail ascending by column, leaves in order of first column
  S->col_leaf.assign(n, -1);
  S->col_loc.assign(n, 0);
  S->tail_cols.clear();
  for (int64_t j = 0; j < n; ++j)
    if (tail[j]) {
      S->col_loc[j] = (int32_t)S->tail_cols.size();
      S->tail_cols.push_back((int32_t)j);
    }
  S->nt = (int64_t)S->tail_cols.size();
  S->leaf_size.clear();
  S->leaf_cols.clear();
  S->leaf_ccnt.clear();
  S->leaf_clist.clear();
  S->leaf_lval_off.clear();
  S->leaf_lcol_off.clear();
  S->leaf_clist_off.clear();
  S->leaf_cval_off.clear();
  S->lval_total = S->cval_total = 0;
  S->leaf_flops = 0;
  for (size_t b = 0; b < comp.size(); ++b) {
    if (tail[comp[b][0]]) continue;
    const int32_t id = (int32_t)S->leaf_size.size();
    const int l = (int)comp[b].size(), cnt = (int)cpl[b].size();
    S->leaf_size.push_back(l);
    S->leaf_lval_off.push_back(S->lval_total);
    S->leaf_lcol_off.push_back((int64_t)S->leaf_cols.size());
    S->leaf_clist_off.push_back((int64_t)S->leaf_clist.size());
    S->leaf_cval_off.push_back(S->cval_total);
    S->leaf_ccnt.push_back(cnt);
    for (int i = 0; i < l; ++i) {
      S->col_leaf[comp[b][i]] = id;
      S->col_loc[comp[b][i]] = i;
      S->leaf_cols.push_back(comp[b][i]);
    }
    for (int32_t k : cpl[b]) S->leaf_clist.push_back(S->col_loc[k]);
    S->lval_total += (int64_t)l * l;
    S->cval_total += (int64_t)cnt * l;
    S->leaf_flops += (double)l * l * l / 3.0 + (double)cnt * l * l + (double)cnt * cnt * l;
  }
  S->leaves = !S->leaf_size.empty();
  // leaf solve lists (one lane per small leaf, one wave per larger one) and,
  // per tail index, the (leaf, coupling row) pairs in leaf order
  S->leaf_small.clear();
  S->leaf_large.clear();
  for (int32_t b = 0; b < (int32_t)S->leaf_size.size(); ++b)
    (S->leaf_size[b] <= LEAF_SMALL ? S->leaf_small : S->leaf_large).push_back(b);
  // per tail index t the entries of its rows of the W_b, flattened: W_b[a][j]
  // (at cval index cval_off[b] + a + j cnt_b) times y at leaf column j, for
  // every leaf b coupled to t (a: t's coupling row in b), in leaf order
  S->tc_ptr.assign(S->nt + 1, 0);
  for (size_t b = 0; b < S->leaf_size.size(); ++b)
    for (int a = 0; a < S->leaf_ccnt[b]; ++a)
      S->tc_ptr[S->leaf_clist[S->leaf_clist_off[b] + a] + 1] += S->leaf_size[b];
  for (int64_t t2 = 0; t2 < S->nt; ++t2) S->tc_ptr[t2 + 1] += S->tc_ptr[t2];
  S->te_cv.assign(S->tc_ptr[S->nt], 0);
  S->te_y.assign(S->tc_ptr[S->nt], 0);
  {
    std::vector<int64_t> fill(S->tc_ptr.begin(), S->tc_ptr.end() - 1);
    for (size_t b = 0; b < S->leaf_size.size(); ++b) {
      const int l = S->leaf_size[b], cnt = S->leaf_ccnt[b];
      for (int a = 0; a < cnt; ++a) {
        const int32_t tt = S->leaf_clist[S->leaf_clist_off[b] + a];
        for (int j = 0; j < l; ++j) {
          const int64_t o = fill[tt]++;
          S->te_cv[o] = S->leaf_cval_off[b] + a + (int64_t)j * cnt;
          S->te_y[o] = S->leaf_cols[S->leaf_lcol_off[b] + j];
        }
      }
    }
  }
  // Envelope of the tail in its order: the first tail column each tail row is
  // coupled to, through a cone's clique (dense rows and large SOC rank-2 rows
  // included), an entry of P, or a leaf block's update W_b W_b' (a clique on
  // the leaf's coupled columns).  Then tail_last[j] = 1 + the last row whose
  // first coupled column is <= j.
  const int64_t nt = S->nt;
  std::vector<int64_t> first(nt);
  for (int64_t t = 0; t < nt; ++t) first[t] = t;
  std::vector<int64_t> mem;
  auto clique = [&](const std::vector<int64_t>& ts) {
    if (ts.empty()) return;
    const int64_t mn = *std::min_element(ts.begin(), ts.end());
    for (int64_t t : ts) first[t] = std::min(first[t], mn);
  };
  for (int64_t c = 0; c < ncl; ++c) {
    mem.clear();
    for (int64_t e = cp[c]; e < cp[c + 1]; ++e)
      if (tail[cc[e]]) mem.push_back(S->col_loc[cc[e]]);
    clique(mem);
  }
  for (int d = 0; d < nd; ++d) {
    mem.clear();
    for (int64_t j = 0; j < n; ++j)
      if (S->Ad[(size_t)d * n + j] != 0.0) mem.push_back(S->col_loc[j]);
    clique(mem);
  }
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k)
      if (tail[i] && tail[P.ci[k]]) clique({(int64_t)S->col_loc[i], (int64_t)S->col_loc[P.ci[k]]});
  for (size_t b = 0; b < S->leaf_size.size(); ++b) {
    mem.assign(S->leaf_clist.begin() + S->leaf_clist_off[b],
               S->leaf_clist.begin() + S->leaf_clist_off[b] + S->leaf_ccnt[b]);
    clique(mem);
  }
  S->tail_last.assign(nt, 0);
  for (int64_t t = 0; t < nt; ++t) S->tail_last[first[t]] = std::max(S->tail_last[first[t]], t + 1);
  for (int64_t t = 0; t < nt; ++t)
    S->tail_last[t] = std::max({S->tail_last[t], t + 1, t > 0 ? S->tail_last[t - 1] : 0});
}

void setup_host(hc_solver* S, const hc_problem* p) {
  const int64_t n = p->n, m = p->m;
  S->n = n;
  S->m = m;
  S->mixed = (S->st.precision == HC_PRECISION_MIXED);
  build_segments(S, p);
  // full P (user order of variables is kept)
  HostCsr Pf;
  Pf.nrows = Pf.ncols = n;
  {
    std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
    if (p->P_rowptr)
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = p->P_rowptr[i]; k < p->P_rowptr[i + 1]; ++k) {
          const int32_t j = p->P_col[k];
          const double v = p->P_val[k];
          rows[i].push_back({j, v});
          if (j != i) rows[j].push_back({(int32_t)i, v});
        }
    Pf.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      std::sort(rows[i].begin(), rows[i].end());
      Pf.rp[i + 1] = Pf.rp[i] + (int32_t)rows[i].size();
      for (auto& e : rows[i]) {
        Pf.ci.push_back(e.first);
        Pf.v.push_back(e.second);
      }
    }
  }
  // A in internal row order
  HostCsr Ai;
  Ai.nrows = m;
  Ai.ncols = n;
  Ai.rp.assign(m + 1, 0);
  for (int64_t r = 0; r < m; ++r) {
    const int64_t u = S->perm[r];
    Ai.rp[r + 1] = Ai.rp[r] + (int32_t)(p->A_rowptr[u + 1] - p->A_rowptr[u]);
  }
  Ai.ci.resize(Ai.rp[m]);
  Ai.v.resize(Ai.rp[m]);
  for (int64_t r = 0; r < m; ++r) {
    const int64_t u = S->perm[r];
    int32_t o = Ai.rp[r];
    for (int64_t k = p->A_rowptr[u]; k < p->A_rowptr[u + 1]; ++k, ++o) {
      Ai.ci[o] = p->A_col[k];
      Ai.v[o] = p->A_val[k];
    }
  }
  std::vector<double> qv(p->q, p->q + n), bi(m);
  for (int64_t r = 0; r < m; ++r) bi[r] = p->b[S->perm[r]];
  S->bnorm_user = 0;
  for (int64_t i = 0; i < m; ++i) S->bnorm_user = std::max(S->bnorm_user, std::fabs(p->b[i]));
  S->qnorm_user = 0;
  for (int64_t j = 0; j < n; ++j) S->qnorm_user = std::max(S->qnorm_user, std::fabs(p->q[j]));
  equilibrate(S, Ai, Pf, qv);
  // scaled data
  const double c = S->cscale;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = Pf.rp[i]; k < Pf.rp[i + 1]; ++k) Pf.v[k] *= c * S->D[i] * S->D[Pf.ci[k]];
  for (int64_t r = 0; r < m; ++r)
    for (int32_t k = Ai.rp[r]; k < Ai.rp[r + 1]; ++k) Ai.v[k] *= S->E[r] * S->D[Ai.ci[k]];
  S->q.resize(n);
  for (int64_t j = 0; j < n; ++j) S->q[j] = c * S->D[j] * qv[j];
  S->b.resize(m);
  for (int64_t r = 0; r < m; ++r) S->b[r] = S->E[r] * bi[r];
  S->maxPdiag = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = Pf.rp[i]; k < Pf.rp[i + 1]; ++k)
      if (Pf.ci[k] == i) S->maxPdiag = std::max(S->maxPdiag, std::fabs(Pf.v[k]));
  S->P = std::move(Pf);
  // dense rows: zero/nonneg rows with more than 512 nonzeros go through a dense SYRK
  std::vector<char> is_dense(m, 0);
  for (const Segment& g : S->segs) {
    if (g.kind != HC_CONE_ZERO && g.kind != HC_CONE_NONNEG) continue;
    for (int64_t i = 0; i < g.count; ++i) {
      const int64_t r = g.base + i;
      if (Ai.rp[r + 1] - Ai.rp[r] > 512) {
        is_dense[r] = 1;
        S->drows.push_back((int32_t)r);
        S->dmidx.push_back(g.moff + i);
      }
    }
  }
  const int nd = (int)S->drows.size();
  S->Ad.assign((size_t)nd * n, 0.0);
  for (int d = 0; d < nd; ++d) {
    const int64_t r = S->drows[d];
    for (int32_t k = Ai.rp[r]; k < Ai.rp[r + 1]; ++k) S->Ad[(size_t)d * n + Ai.ci[k]] = Ai.v[k];
  }
  HostCsr As;   // A without the dense rows
  As.nrows = m;
  As.ncols = n;
  As.rp.assign(m + 1, 0);
  for (int64_t r = 0; r < m; ++r) As.rp[r + 1] = As.rp[r] + (is_dense[r] ? 0 : (Ai.rp[r + 1] - Ai.rp[r]));
  As.ci.reserve(As.rp[m]);
  As.v.reserve(As.rp[m]);
  for (int64_t r = 0; r < m; ++r)
    if (!is_dense[r])
      for (int32_t k = Ai.rp[r]; k < Ai.rp[r + 1]; ++k) {
        As.ci.push_back(Ai.ci[k]);
        As.v.push_back(Ai.v[k]);
      }
  // transpose of As
  HostCsr At;
  At.nrows = n;
  At.ncols = m;
  At.rp.assign(n + 1, 0);
  for (int32_t k = 0; k < As.rp[m]; ++k) At.rp[As.ci[k] + 1]++;
  for (int64_t j = 0; j < n; ++j) At.rp[j + 1] += At.rp[j];
  At.ci.resize(As.rp[m]);
  At.v.resize(As.rp[m]);
  {
    std::vector<int32_t> fillp(At.rp.begin(), At.rp.end() - 1);
    for (int64_t r = 0; r < m; ++r)
      for (int32_t k = As.rp[r]; k < As.rp[r + 1]; ++k) {
        const int32_t j = As.ci[k];
        At.ci[fillp[j]] = (int32_t)r;
        At.v[fillp[j]] = As.v[k];
        fillp[j]++;
      }
  }
  // Schur assembly tasks: unordered row pairs within each cone
  for (const Segment& g : S->segs) {
    if (g.kind == HC_CONE_ZERO || g.kind == HC_CONE_NONNEG) {
      for (int64_t i = 0; i < g.count; ++i) {
        const int64_t r = g.base + i;
        if (is_dense[r] || As.rp[r + 1] == As.rp[r]) continue;
        S->tra.push_back((int32_t)r);
        S->trb.push_back((int32_t)r);
        S->tm.push_back(g.moff + i);
      }
      continue;
    }
    if (soc_large(g.kind, g.dim)) {   // f_o A_c'A_c: one diagonal task per row, weight f_o of its cone
      for (int a = 0; a < g.dim; ++a)
        for (int64_t c2 = 0; c2 < g.count; ++c2) {
          const int64_t ra = g.base + a * g.count + c2;
          if (As.rp[ra + 1] == As.rp[ra]) continue;
          S->tra.push_back((int32_t)ra);
          S->trb.push_back((int32_t)ra);
          S->tm.push_back(g.moff + c2);
        }
      continue;
    }
    for (int64_t c2 = 0; c2 < g.count; ++c2)
      for (int a = 0; a < g.dim; ++a)
        for (int bb = 0; bb <= a; ++bb) {
          const int64_t ra = (g.kind == HC_CONE_PSD) ? g.base + c2 * g.dim + a : g.base + a * g.count + c2;
          const int64_t rb = (g.kind == HC_CONE_PSD) ? g.base + c2 * g.dim + bb : g.base + bb * g.count + c2;
          if (As.rp[ra + 1] == As.rp[ra] || As.rp[rb + 1] == As.rp[rb]) continue;
          S->tra.push_back((int32_t)ra);
          S->trb.push_back((int32_t)rb);
          S->tm.push_back(g.moff + ((int64_t)a * (a + 1) / 2 + bb) * g.count + c2);
        }
  }
  {   // long tasks last, for the one-wave-per-task kernel
    const int64_t nt = (int64_t)S->tra.size();
    std::vector<int64_t> ord(nt);
    for (int64_t t = 0; t < nt; ++t) ord[t] = t;
    auto cost = [&](int64_t t) {
      const int64_t a = As.rp[S->tra[t] + 1] - As.rp[S->tra[t]], b = As.rp[S->trb[t] + 1] - As.rp[S->trb[t]];
      return a * b;
    };
    auto mid = std::stable_partition(ord.begin(), ord.end(), [&](int64_t t) { return cost(t) <= PAIR_WIDE; });
    S->ntask_short = mid - ord.begin();
    std::vector<int32_t> a2(nt), b2(nt);
    std::vector<int64_t> m2(nt);
    for (int64_t t = 0; t < nt; ++t) {
      a2[t] = S->tra[ord[t]];
      b2[t] = S->trb[ord[t]];
      m2[t] = S->tm[ord[t]];
    }
    S->tra.swap(a2);
    S->trb.swap(b2);
    S->tm.swap(m2);
  }
  S->A = std::move(As);
  S->At = std::move(At);
  build_leaves(S);
  build_psd_dense(S);
  build_groups(S);
  if (S->leaves && nd) {   // dense rows live on tail columns only: re-index them
    std::vector<double> Adt((size_t)nd * S->nt);
    for (int d = 0; d < nd; ++d)
      for (int64_t t = 0; t < S->nt; ++t) Adt[(size_t)d * S->nt + t] = S->Ad[(size_t)d * n + S->tail_cols[t]];
    S->Ad.swap(Adt);
  }
  build_lowrank(S, nd);
  S->ld = ((S->nt + 63) / 64) * 64;
  for (int64_t t = S->nt; t < S->ld; ++t) S->tail_last.push_back(t + 1);   // identity padding
  if (S->st.static_reg <= 0) S->st.static_reg = S->mixed ? 3.4526698300124393e-04 : 1e-8;
  if (S->st.dyn_reg < 0) S->st.dyn_reg = S->mixed ? std::ldexp(1.0, -46) : std::ldexp(1.0, -104);
  if (S->st.ir_mu_frac < 0) S->st.ir_mu_frac = S->mixed ? 1e-3 : 0.0;
  build_ordered(S);
}

// Groups of the Schur assembly (only without leaf blocks): the rows the pair
// tasks link (a cone's rows; a single row of a zero or nonneg segment or of a
// large SOC) form a group g, with U_g the sorted union of their columns.  Per
// iteration T_g = M_g A_g and each column of S gathers A[r][j] T_r over the
// rows of that column of A (group_T, group_gather: one writer per entry, a
// fixed order).  When a column of S fits two LDS chunks (n <= 2 GATHER_CHUNK)
// every group is taken, so the whole assembly has one writer per entry and a
// fixed order; on larger problems only groups of at least GROUP_MIN_ROWS rows
// (PSD cones: many row pairs, each S entry hit by many of them) are taken, and
// the rest keep their pair tasks, which are cheaper there (a gather over a
// 20,000-row column in five chunks costs more than the few atomics a 3-row
// cone adds).  A group whose T_g would exceed GROUP_T_MAX entries keeps its
// pair tasks.
constexpr int64_t GROUP_MIN_ROWS = 6;
constexpr int64_t GROUP_T_MAX = int64_t(1) << 22;
void build_groups(hc_solver* S) {
  S->ga_ng = S->ga_t_total = 0;
  S->ga_rows_off.assign(1, 0);
  S->ga_u_off.assign(1, 0);
  S->ga_c_ptr.assign(1, 0);
  S->ga_m_off.clear();
  S->ga_t_off.clear();
  S->ga_gm.clear();
  S->ga_rows.clear();
  S->ga_u.clear();
  S->ga_c_b.clear();
  S->ga_c_k.clear();
  S->ga_rgrp.clear();
  S->ga_rloc.clear();
  if (S->leaves || S->tra.empty()) return;
  const HostCsr& A = S->A;
  const int64_t m = A.nrows, nt = (int64_t)S->tra.size();
  std::vector<int32_t> par(m);
  for (int64_t r = 0; r < m; ++r) par[r] = (int32_t)r;
  auto find = [&](int32_t x) {
    while (par[x] != x) x = par[x] = par[par[x]];
    return x;
  };
  std::vector<char> used(m, 0);
  for (int64_t k = 0; k < nt; ++k) {
    used[S->tra[k]] = used[S->trb[k]] = 1;
    const int32_t a = find(S->tra[k]), b = find(S->trb[k]);
    if (a != b) par[std::max(a, b)] = std::min(a, b);
  }
  // groups in order of their first row, rows ascending within a group
  std::vector<int32_t> gid(m, -1), loc(m, 0);
  std::vector<std::vector<int32_t>> rows;
  for (int64_t r = 0; r < m; ++r) {
    if (!used[r]) continue;
    const int32_t root = find((int32_t)r);
    if (gid[root] < 0) {
      gid[root] = (int32_t)rows.size();
      rows.emplace_back();
    }
    const int32_t g = gid[root];
    gid[r] = g;
    loc[r] = (int32_t)rows[g].size();
    rows[g].push_back((int32_t)r);
  }
  S->ga_rgrp.assign(m, -1);
  S->ga_rloc.assign(m, 0);
  std::vector<int32_t> u, cnt;
  struct Ent {
    int32_t col, k, b;   // column, index in A, group-local row
  };
  std::vector<Ent> ent;   // the group's entries in row order
  for (size_t g = 0; g < rows.size(); ++g) {
    ent.clear();
    for (int32_t r : rows[g])
      for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) ent.push_back({A.ci[k], k, loc[r]});
    u.clear();
    for (const Ent& en : ent) u.push_back(en.col);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    const int64_t nr = (int64_t)rows[g].size(), s = (int64_t)u.size();
    if ((A.ncols > 2 * GATHER_CHUNK && nr < GROUP_MIN_ROWS) || nr * s > GROUP_T_MAX) continue;
    const int32_t id = (int32_t)S->ga_ng++;
    S->ga_m_off.push_back((int64_t)S->ga_gm.size());
    S->ga_t_off.push_back(S->ga_t_total);
    S->ga_gm.resize(S->ga_gm.size() + nr * nr, -1);
    S->ga_t_total += nr * s;
    for (int32_t r : rows[g]) {
      S->ga_rows.push_back(r);
      S->ga_rgrp[r] = id;
      S->ga_rloc[r] = loc[r];
    }
    // per column of U_g its entries, in row order (a stable counting sort)
    cnt.assign(s + 1, 0);
    std::vector<int32_t> pos(ent.size());
    for (size_t e = 0; e < ent.size(); ++e) {
      pos[e] = (int32_t)(std::lower_bound(u.begin(), u.end(), ent[e].col) - u.begin());
      cnt[pos[e] + 1]++;
    }
    for (int64_t q = 0; q < s; ++q) cnt[q + 1] += cnt[q];
    const int64_t base = (int64_t)S->ga_c_b.size();
    S->ga_c_b.resize(base + ent.size());
    S->ga_c_k.resize(base + ent.size());
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (size_t e = 0; e < ent.size(); ++e) {
      const int64_t o = base + fill[pos[e]]++;
      S->ga_c_b[o] = ent[e].b;
      S->ga_c_k[o] = ent[e].k;
    }
    for (int64_t q = 0; q < s; ++q) S->ga_c_ptr.push_back(base + cnt[q + 1]);
    S->ga_u.insert(S->ga_u.end(), u.begin(), u.end());
    S->ga_rows_off.push_back((int64_t)S->ga_rows.size());
    S->ga_u_off.push_back((int64_t)S->ga_u.size());
  }
  // M entries of the taken groups; their tasks leave the pair list
  int64_t keep = 0, keep_short = 0;
  for (int64_t k = 0; k < nt; ++k) {
    const int32_t ra = S->tra[k], rb = S->trb[k], g = S->ga_rgrp[ra];
    if (g >= 0) {
      const int64_t nr = S->ga_rows_off[g + 1] - S->ga_rows_off[g];
      int64_t* gm = S->ga_gm.data() + S->ga_m_off[g];
      gm[(int64_t)S->ga_rloc[ra] * nr + S->ga_rloc[rb]] = S->tm[k];
      gm[(int64_t)S->ga_rloc[rb] * nr + S->ga_rloc[ra]] = S->tm[k];
      continue;
    }
    if (k < S->ntask_short) keep_short++;
    S->tra[keep] = ra;
    S->trb[keep] = rb;
    S->tm[keep] = S->tm[k];
    keep++;
  }
  S->tra.resize(keep);
  S->trb.resize(keep);
  S->tm.resize(keep);
  S->ntask_short = keep_short;
  // per entry p of A' (row r of column j): the T row of r's group (offset in
  // T), that group's column list and length, 0 length when r is in no group
  const HostCsr& At = S->At;
  S->ga_e_t.assign(At.ci.size(), 0);
  S->ga_e_u.assign(At.ci.size(), 0);
  S->ga_e_s.assign(At.ci.size(), 0);
  for (size_t p = 0; p < At.ci.size(); ++p) {
    const int32_t r = At.ci[p], g = S->ga_rgrp[r];
    if (g < 0) continue;
    const int64_t uo = S->ga_u_off[g], sz = S->ga_u_off[g + 1] - uo;
    S->ga_e_t[p] = S->ga_t_off[g] + (int64_t)S->ga_rloc[r] * sz;
    S->ga_e_u[p] = uo;
    S->ga_e_s[p] = (int32_t)sz;
  }
}

// PSD segments whose row pairs would cost more than forming T = M_c A_c for
// each of their rows (n entries per row) leave the pair tasks: their block
// A_c' M_c A_c is added as A_e' T, a gather over the columns of A (one writer
// per entry of S, no atomics).  Only without leaf blocks (every column is a
// Schur column), for n up to PSD_DENSE_NMAX, and with T within 4 GiB.
void build_psd_dense(hc_solver* S) {
  S->pdense.clear();
  S->pdense_coff.clear(), S->pc_cu_off.clear(), S->pc_cu_ptr.clear();
  S->pc_cu_col.clear(), S->pc_cu_b.clear(), S->pc_cu_p.clear();
  S->pe_rp.assign(1, 0);
  S->pe_e.clear();
  S->pe_p.clear();
  S->pe_rows = 0;
  const int64_t n = S->n, m = S->m;
  if (S->leaves || n > PSD_DENSE_NMAX || n == 0) return;
  const HostCsr& A = S->A;
  std::vector<int64_t> trow(m, -1);   // T row of an internal row, -1 if none
  for (size_t si = 0; si < S->segs.size(); ++si) {
    const Segment& g = S->segs[si];
    if (g.kind != HC_CONE_PSD || g.count == 0) continue;
    double pairs = 0;
    for (int64_t c = 0; c < g.count; ++c) {
      double sum = 0, sq = 0;
      for (int a = 0; a < g.dim; ++a) {
        const int64_t r = g.base + c * g.dim + a;
        const double k = A.rp[r + 1] - A.rp[r];
        sum += k;
        sq += k * k;
      }
      pairs += 0.5 * (sum * sum + sq);
    }
    const int64_t rows = g.count * g.dim;
    if (!(pairs > (double)rows * (double)n)) continue;
    if ((double)(S->pe_rows + rows) * (double)n * 8.0 > 4294967296.0) continue;
    S->pdense.push_back({(int)si, S->pe_rows});
    for (int64_t e = 0; e < rows; ++e) trow[g.base + e] = S->pe_rows + e;
    S->pe_rows += rows;
  }
  if (S->pdense.empty()) return;
  // drop the pair tasks of those segments (both rows of a task lie in one cone)
  const int64_t nt = (int64_t)S->tra.size();
  int64_t keep = 0, keep_short = 0;
  for (int64_t t = 0; t < nt; ++t) {
    if (trow[S->tra[t]] >= 0) continue;
    if (t < S->ntask_short) keep_short++;
    S->tra[keep] = S->tra[t];
    S->trb[keep] = S->trb[t];
    S->tm[keep] = S->tm[t];
    keep++;
  }
  S->tra.resize(keep);
  S->trb.resize(keep);
  S->tm.resize(keep);
  S->ntask_short = keep_short;
  // per column j: the T rows of its entries in those segments
  const HostCsr& At = S->At;
  S->pe_rp.assign(n + 1, 0);
  for (int64_t j = 0; j < n; ++j) {
    for (int32_t p = At.rp[j]; p < At.rp[j + 1]; ++p) {
      const int64_t e = trow[At.ci[p]];
      if (e < 0) continue;
      S->pe_e.push_back((int32_t)e);
      S->pe_p.push_back(p);
    }
    S->pe_rp[j + 1] = (int32_t)S->pe_e.size();
  }
  // per cone its columns, each with its entries (row of the cone, index in A)
  // in row order
  std::vector<std::array<int64_t, 3>> ent;
  for (const auto& pd : S->pdense) {
    const Segment& g = S->segs[pd.first];
    S->pdense_coff.push_back((int64_t)S->pc_cu_off.size());
    for (int64_t c = 0; c < g.count; ++c) {
      S->pc_cu_off.push_back((int64_t)S->pc_cu_col.size());
      ent.clear();
      for (int b = 0; b < g.dim; ++b) {
        const int64_t r = g.base + c * g.dim + b;
        for (int32_t p = A.rp[r]; p < A.rp[r + 1]; ++p) ent.push_back({(int64_t)A.ci[p], (int64_t)b, (int64_t)p});
      }
      std::stable_sort(ent.begin(), ent.end(),
                       [](const std::array<int64_t, 3>& x, const std::array<int64_t, 3>& y) { return x[0] < y[0]; });
      for (size_t k = 0; k < ent.size(); ++k) {
        if (k == 0 || ent[k][0] != ent[k - 1][0]) {
          S->pc_cu_col.push_back((int32_t)ent[k][0]);
          S->pc_cu_ptr.push_back((int64_t)S->pc_cu_b.size());
        }
        S->pc_cu_b.push_back((int32_t)ent[k][1]);
        S->pc_cu_p.push_back((int32_t)ent[k][2]);
      }
    }
  }
  S->pc_cu_off.push_back((int64_t)S->pc_cu_col.size());
  S->pc_cu_ptr.push_back((int64_t)S->pc_cu_b.size());
}

// Stable sort of 0 .. key.size() - 1 by key (LSD radix, 16-bit digits; digits
// that every key shares are skipped).
std::vector<int64_t> radix_order(const std::vector<uint64_t>& key) {
  const int64_t np = (int64_t)key.size();
  std::vector<int64_t> idx(np), tmp(np);
  for (int64_t i = 0; i < np; ++i) idx[i] = i;
  std::vector<int64_t> cnt(65537);
  for (int sh = 0; sh < 64; sh += 16) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t i = 0; i < np; ++i) cnt[((key[i] >> sh) & 0xffff) + 1]++;
    if (np == 0 || *std::max_element(cnt.begin(), cnt.end()) == np) continue;
    for (int d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
    for (int64_t i = 0; i < np; ++i) tmp[cnt[(key[idx[i]] >> sh) & 0xffff]++] = idx[i];
    idx.swap(tmp);
  }
  return idx;
}

// Group terms (sorted by destination, enumeration order kept within one) into
// destinations: ptr / dst, short destinations first (order kept), then those
// of more than ORDERED_WIDE terms; `perm` receives the term order to use.
void group_terms(const std::vector<uint64_t>& key, std::vector<int64_t>& ptr, std::vector<int64_t>& dst,
                 int64_t& nshort, std::vector<int64_t>& perm) {
  const std::vector<int64_t> ord = radix_order(key);
  const int64_t np = (int64_t)key.size();
  std::vector<int64_t> b;   // start of each destination's run in ord
  for (int64_t i = 0; i < np; ++i)
    if (i == 0 || key[ord[i]] != key[ord[i - 1]]) b.push_back(i);
  const int64_t nd = (int64_t)b.size();
  b.push_back(np);
  std::vector<int64_t> dorder;
  for (int pass = 0; pass < 2; ++pass)
    for (int64_t d = 0; d < nd; ++d)
      if ((b[d + 1] - b[d] > ORDERED_WIDE) == (pass == 1)) dorder.push_back(d);
  nshort = 0;
  for (int64_t d = 0; d < nd; ++d) nshort += (b[d + 1] - b[d] <= ORDERED_WIDE);
  ptr.assign(1, 0);
  dst.clear();
  perm.clear();
  perm.reserve(np);
  for (int64_t d : dorder) {
    for (int64_t i = b[d]; i < b[d + 1]; ++i) perm.push_back(ord[i]);
    ptr.push_back((int64_t)perm.size());
    dst.push_back((int64_t)key[ord[b[d]]]);
  }
}

// The ordered Schur sums.  Every product a pair task adds, m_t A[ra][j]
// A[rb][k] (doubled where two products of a row pair meet on the diagonal),
// becomes a term of the entry of S it lands on, and each leaf's update of
// S_TT[t_a][t_c] a slot; terms keep the order of the tasks, so each entry of
// S is one sum in a fixed order (bitwise the same from run to run).  Entries
// are encoded as in OrderedSum: the dense S (or S_TT) at hi + lo ld, a leaf
// block at lval_off + hi + lo l, a coupling block at cval_off + row + col cnt.
constexpr int64_t ORDERED_MAX_TERMS = int64_t(1) << 30;
void build_ordered(hc_solver* S) {
  S->ordered = false;
  S->op_ptr.clear(), S->op_dst.clear(), S->op_pm.clear(), S->op_pp.clear(), S->op_pq.clear();
  S->ol_ptr.clear(), S->ol_dst.clear(), S->ol_pp.clear(), S->leaf_lp_off.clear();
  S->op_nshort = S->ol_nshort = S->lpair_total = 0;
  const HostCsr& A = S->A;
  const int64_t nt = (int64_t)S->tra.size();
  int64_t np = 0;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t ka = A.rp[S->tra[t] + 1] - A.rp[S->tra[t]], kb = A.rp[S->trb[t] + 1] - A.rp[S->trb[t]];
    np += S->tra[t] == S->trb[t] ? ka * (ka + 1) / 2 : ka * kb;
  }
  int64_t nl = 0;
  for (size_t b = 0; b < S->leaf_size.size(); ++b) nl += (int64_t)S->leaf_ccnt[b] * (S->leaf_ccnt[b] + 1) / 2;
  if (np > ORDERED_MAX_TERMS || nl > ORDERED_MAX_TERMS || S->mtotal >= (int64_t(1) << 31)) return;
  const int64_t ld = S->ld;
  const uint64_t SEL1 = uint64_t(1) << 62, SEL2 = uint64_t(2) << 62;
  const uint64_t NONE = ~uint64_t(0);   // two distinct leaves (never coupled); selector 3 is unused
  auto enc = [&](int32_t j, int32_t k) -> uint64_t {
    if (!S->leaves) return (uint64_t)std::max(j, k) + (uint64_t)std::min(j, k) * ld;
    const int32_t bj = S->col_leaf[j], bk = S->col_leaf[k], lj = S->col_loc[j], lk = S->col_loc[k];
    if (bj < 0 && bk < 0) return (uint64_t)std::max(lj, lk) + (uint64_t)std::min(lj, lk) * ld;
    if (bj >= 0 && bk >= 0) {
      if (bj != bk) return NONE;
      return SEL1 | (uint64_t)(S->leaf_lval_off[bj] + std::max(lj, lk) + (int64_t)std::min(lj, lk) * S->leaf_size[bj]);
    }
    const int32_t b = bj >= 0 ? bj : bk, l = bj >= 0 ? lj : lk, t = bj >= 0 ? lk : lj;
    const int32_t* cl = S->leaf_clist.data() + S->leaf_clist_off[b];
    const int32_t* f = std::lower_bound(cl, cl + S->leaf_ccnt[b], t);
    if (f == cl + S->leaf_ccnt[b] || *f != t) return NONE;
    return SEL2 | (uint64_t)(S->leaf_cval_off[b] + (f - cl) + (int64_t)l * S->leaf_ccnt[b]);
  };
  {
    std::vector<uint64_t> key;
    std::vector<int32_t> pm, pp, pq;
    key.reserve(np), pm.reserve(np), pp.reserve(np), pq.reserve(np);
    auto term = [&](int64_t t, int32_t p, int32_t q, bool two) {
      const uint64_t e = enc(A.ci[p], A.ci[q]);
      if (e == NONE) return;
      key.push_back(e);
      pm.push_back((int32_t)S->tm[t]);
      pp.push_back(p);
      pq.push_back(two ? ~q : q);
    };
    for (int64_t t = 0; t < nt; ++t) {
      const int32_t ra = S->tra[t], rb = S->trb[t];
      if (ra == rb) {
        for (int32_t p = A.rp[ra]; p < A.rp[ra + 1]; ++p)
          for (int32_t q = A.rp[ra]; q <= p; ++q) term(t, p, q, false);
      } else {
        for (int32_t p = A.rp[ra]; p < A.rp[ra + 1]; ++p)
          for (int32_t q = A.rp[rb]; q < A.rp[rb + 1]; ++q) term(t, p, q, A.ci[p] == A.ci[q]);
      }
    }
    std::vector<int64_t> perm;
    group_terms(key, S->op_ptr, S->op_dst, S->op_nshort, perm);
    const int64_t nk = (int64_t)perm.size();
    S->op_pm.resize(nk), S->op_pp.resize(nk), S->op_pq.resize(nk);
    for (int64_t i = 0; i < nk; ++i) {
      S->op_pm[i] = pm[perm[i]];
      S->op_pp[i] = pp[perm[i]];
      S->op_pq[i] = pq[perm[i]];
    }
  }
  {   // leaf b's pair p = a (a + 1) / 2 + c (a >= c) lands on S_TT[cl[a]][cl[c]]
    std::vector<uint64_t> key;
    key.reserve(nl);
    for (size_t b = 0; b < S->leaf_size.size(); ++b) {
      S->leaf_lp_off.push_back(S->lpair_total);
      const int cnt = S->leaf_ccnt[b];
      const int32_t* cl = S->leaf_clist.data() + S->leaf_clist_off[b];
      for (int a = 0; a < cnt; ++a)
        for (int c = 0; c <= a; ++c) key.push_back((uint64_t)(cl[a] + (int64_t)cl[c] * ld));
      S->lpair_total += (int64_t)cnt * (cnt + 1) / 2;
    }
    std::vector<int64_t> perm;
    group_terms(key, S->ol_ptr, S->ol_dst, S->ol_nshort, perm);
    S->ol_pp.resize(perm.size());
    for (size_t i = 0; i < perm.size(); ++i) S->ol_pp[i] = (int32_t)perm[i];
  }
  S->ordered = true;
}

// (cone, column) entries of the rank-2 rows of the large second-order cones
// and the M index of every row of the dense-row operand
void build_lowrank(hc_solver* S, int nd) {
  const int64_t nt = S->nt;
  S->nls = 0;
  S->ls_cone.clear();
  S->ls_col.clear();
  S->ls_dst.clear();
  S->ls_ranges.clear();
  std::vector<int32_t> cols;
  for (size_t si = 0; si < S->segs.size(); ++si) {
    const Segment& g = S->segs[si];
    if (!soc_large(g.kind, g.dim)) continue;
    const int64_t first = (int64_t)S->ls_cone.size();
    for (int64_t c = 0; c < g.count; ++c) {
      cols.clear();
      for (int a = 0; a < g.dim; ++a) {
        const int64_t r = g.base + a * g.count + c;
        for (int32_t k = S->A.rp[r]; k < S->A.rp[r + 1]; ++k) cols.push_back(S->A.ci[k]);
      }
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      for (int32_t j : cols) {
        if (S->col_leaf[j] >= 0) fail(HC_ERR_UNSUPPORTED, "large SOC column outside the dense tail");
        S->ls_cone.push_back((int32_t)c);
        S->ls_col.push_back(j);
        S->ls_dst.push_back((nd + S->nls + c) * nt + S->col_loc[j]);
      }
    }
    S->ls_ranges.push_back({(int)si, first, (int64_t)S->ls_cone.size() - first});
    S->nls += g.count;
  }
  S->K1 = (nd + S->nls + 15) / 16 * 16;
  S->K2 = (S->nls + 15) / 16 * 16;
  S->dmidx_all.assign(S->K1 + S->K2, -1);
  for (int d = 0; d < nd; ++d) S->dmidx_all[d] = S->dmidx[d];
  int64_t lc = 0;
  for (const auto& rg : S->ls_ranges) {
    const Segment& g = S->segs[rg.seg];
    for (int64_t c = 0; c < g.count; ++c, ++lc) {
      S->dmidx_all[nd + lc] = g.moff + 2 * g.count + c;   // f_- - f_o
      S->dmidx_all[S->K1 + lc] = g.moff + g.count + c;    // f_+ - f_o
    }
  }
}

// keep a copy of the user's problem (hc_update_data rebuilds from it)
void keep_user_data(hc_solver* S, const hc_problem* p) {
  const int64_t n = p->n, m = p->m;
  if (p->P_rowptr) {
    S->uPrp.assign(p->P_rowptr, p->P_rowptr + n + 1);
    S->uPci.assign(p->P_col, p->P_col + p->P_rowptr[n]);
    S->uPv.assign(p->P_val, p->P_val + p->P_rowptr[n]);
  }
  S->uArp.assign(p->A_rowptr, p->A_rowptr + m + 1);
  S->uAci.assign(p->A_col, p->A_col + p->A_rowptr[m]);
  S->uAv.assign(p->A_val, p->A_val + p->A_rowptr[m]);
  S->uq.assign(p->q, p->q + n);
  S->ub.assign(p->b, p->b + m);
  S->ucones.assign(p->cones, p->cones + p->ncones);
}

hc_problem user_problem(hc_solver* S) {
  hc_problem p{};
  p.n = S->n;
  p.m = S->m;
  if (!S->uPrp.empty()) {
    p.P_rowptr = S->uPrp.data();
    p.P_col = S->uPci.data();
    p.P_val = S->uPv.data();
  }
  p.q = S->uq.data();
  p.A_rowptr = S->uArp.data();
  p.A_col = S->uAci.data();
  p.A_val = S->uAv.data();
  p.b = S->ub.data();
  p.cones = S->ucones.data();
  p.ncones = (int32_t)S->ucones.size();
  return p;
}

// Parametric update (same sparsity, new values): redo every value-dependent
// step of the set-up -- full P, A in the internal row order, equilibration,
// scaling, the dense rows, A without them and its transpose -- on the
// structures kept from the set-up (row order, dense-row choice, assembly
// tasks, leaf blocks and tail ordering are reused as they are).
void refresh_values(hc_solver* S) {
  const hc_problem up = user_problem(S);
  const hc_problem* p = &up;
  const int64_t n = S->n, m = S->m;
  HostCsr Pf;
  Pf.nrows = Pf.ncols = n;
  {
    std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
    if (p->P_rowptr)
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = p->P_rowptr[i]; k < p->P_rowptr[i + 1]; ++k) {
          const int32_t j = p->P_col[k];
          rows[i].push_back({j, p->P_val[k]});
          if (j != i) rows[j].push_back({(int32_t)i, p->P_val[k]});
        }
    Pf.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      std::sort(rows[i].begin(), rows[i].end());
      Pf.rp[i + 1] = Pf.rp[i] + (int32_t)rows[i].size();
      for (auto& e : rows[i]) {
        Pf.ci.push_back(e.first);
        Pf.v.push_back(e.second);
      }
    }
  }
  if (Pf.ci != S->P.ci || Pf.rp != S->P.rp) fail(HC_ERR_CSR, "hc_update_data: P structure differs from set-up");
  HostCsr Ai;
  Ai.nrows = m;
  Ai.ncols = n;
  Ai.rp.assign(m + 1, 0);
  for (int64_t r = 0; r < m; ++r) {
    const int64_t u = S->perm[r];
    Ai.rp[r + 1] = Ai.rp[r] + (int32_t)(p->A_rowptr[u + 1] - p->A_rowptr[u]);
  }
  Ai.ci.resize(Ai.rp[m]);
  Ai.v.resize(Ai.rp[m]);
  for (int64_t r = 0; r < m; ++r) {
    const int64_t u = S->perm[r];
    int32_t o = Ai.rp[r];
    for (int64_t k = p->A_rowptr[u]; k < p->A_rowptr[u + 1]; ++k, ++o) {
      Ai.ci[o] = p->A_col[k];
      Ai.v[o] = p->A_val[k];
    }
  }
  std::vector<double> qv(p->q, p->q + n), bi(m);
  for (int64_t r = 0; r < m; ++r) bi[r] = p->b[S->perm[r]];
  S->bnorm_user = 0;
  for (int64_t i = 0; i < m; ++i) S->bnorm_user = std::max(S->bnorm_user, std::fabs(p->b[i]));
  S->qnorm_user = 0;
  for (int64_t j = 0; j < n; ++j) S->qnorm_user = std::max(S->qnorm_user, std::fabs(p->q[j]));
  equilibrate(S, Ai, Pf, qv);
  const double c = S->cscale;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = Pf.rp[i]; k < Pf.rp[i + 1]; ++k) Pf.v[k] *= c * S->D[i] * S->D[Pf.ci[k]];
  for (int64_t r = 0; r < m; ++r)
    for (int32_t k = Ai.rp[r]; k < Ai.rp[r + 1]; ++k) Ai.v[k] *= S->E[r] * S->D[Ai.ci[k]];
  for (int64_t j = 0; j < n; ++j) S->q[j] = c * S->D[j] * qv[j];
  for (int64_t r = 0; r < m; ++r) S->b[r] = S->E[r] * bi[r];
  S->maxPdiag = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = Pf.rp[i]; k < Pf.rp[i + 1]; ++k)
      if (Pf.ci[k] == i) S->maxPdiag = std::max(S->maxPdiag, std::fabs(Pf.v[k]));
  S->P.v = Pf.v;
  // dense rows (full n columns first, then re-indexed to the tail as at set-up)
  const int nd = (int)S->drows.size();
  std::vector<char> is_dense(m, 0);
  for (int d = 0; d < nd; ++d) is_dense[S->drows[d]] = 1;
  std::vector<double> Ad((size_t)nd * n, 0.0);
  for (int d = 0; d < nd; ++d) {
    const int64_t r = S->drows[d];
    for (int32_t k = Ai.rp[r]; k < Ai.rp[r + 1]; ++k) Ad[(size_t)d * n + Ai.ci[k]] = Ai.v[k];
  }
  if (S->leaves && nd) {
    std::vector<double> Adt((size_t)nd * S->nt);
    for (int d = 0; d < nd; ++d)
      for (int64_t t = 0; t < S->nt; ++t) Adt[(size_t)d * S->nt + t] = Ad[(size_t)d * n + S->tail_cols[t]];
    Ad.swap(Adt);
  }
  S->Ad.swap(Ad);
  // A without the dense rows, and its transpose, in the set-up's positions
  {
    int64_t o = 0;
    for (int64_t r = 0; r < m; ++r)
      if (!is_dense[r])
        for (int32_t k = Ai.rp[r]; k < Ai.rp[r + 1]; ++k) S->A.v[o++] = Ai.v[k];
    std::vector<int32_t> fillp(S->At.rp.begin(), S->At.rp.end() - 1);
    for (int64_t r = 0; r < m; ++r)
      for (int32_t k = S->A.rp[r]; k < S->A.rp[r + 1]; ++k) S->At.v[fillp[S->A.ci[k]]++] = S->A.v[k];
  }
}

template <typename T> T* upload(Buf& buf, const std::vector<T>& h, hipStream_t st) {
  T* d = buf.take<T>(std::max<size_t>(1, h.size()));
  if (!buf.dry && !h.empty()) HC_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}

Csr upload_csr(Buf& buf, const HostCsr& h, hipStream_t st) {
  Csr c;
  c.nrows = (int32_t)h.nrows;
  c.ncols = (int32_t)h.ncols;
  c.nnz = h.ci.size();
  c.rowptr = upload(buf, h.rp, st);
  c.col = upload(buf, h.ci, st);
  c.val = upload(buf, h.v, st);
  c.lanes = choose_lanes(h.nrows ? (double)c.nnz / (double)h.nrows : 0.0);
  // rows of more than 32 x lanes entries go to one wave each
  c.long_nnz = 32 * c.lanes;
  std::vector<int32_t> lr;
  for (int64_t r = 0; r < h.nrows; ++r)
    if (h.rp[r + 1] - h.rp[r] > c.long_nnz) lr.push_back((int32_t)r);
  c.nlong = (int32_t)lr.size();
  c.longrows = upload(buf, lr, st);
  return c;
}

// ===========================================================================
// device-side building blocks of one iteration
// ===========================================================================
struct Red {
  hc_solver* S;
  RedOps ops{};
  int64_t n;
  explicit Red(hc_solver* s, int64_t len) : S(s), n(len) { ops.nops = 0; }
  int dot(const double* x, const double* y) {
    ops.op[ops.nops] = RedOp{RED_DOT, x, y, 0.0, nullptr};
    return ops.nops++;
  }
  int maxabs(const double* x, const double* w = nullptr, bool divide = false, const double* y = nullptr,
             double yc = 0.0) {
    ops.op[ops.nops] = RedOp{divide ? RED_MAX_DIV : RED_MAX_MUL, x, y, yc, w};
    return ops.nops++;
  }
  // launch into dpart + off; returns the partials it will write
  int64_t launch(int64_t off) {
    if (n == 0 || ops.nops == 0) return 0;
    nblk = reduce_launch(n, ops, S->dpart + off, S->stream);
    base = off;
    return (int64_t)nblk * ops.nops;
  }
  // combine this reduction's partials (already copied to hpart)
  std::vector<double> collect() const {
    std::vector<double> out(ops.nops, 0.0);
    if (n == 0 || ops.nops == 0) return out;
    for (int o = 0; o < ops.nops; ++o) {
      double acc = 0.0;
      for (int bk = 0; bk < nblk; ++bk) {
        const double v = S->hpart[base + (size_t)bk * ops.nops + o];
        if (ops.op[o].kind == RED_DOT) acc += v;
        else acc = (std::isnan(v) || std::isnan(acc)) ? NAN : std::max(acc, v);
      }
      out[o] = acc;
    }
    return out;
  }
  std::vector<double> run() {
    const int64_t cnt = launch(0);
    if (cnt) {
      HC_HIP(hipMemcpyAsync(S->hpart, S->dpart, cnt * sizeof(double), hipMemcpyDeviceToHost, S->stream));
      HC_HIP(hipStreamSynchronize(S->stream));
    }
    return collect();
  }
  int nblk = 0;
  int64_t base = 0;
};

// two reductions (over lengths n and m) with one host round trip
void run_pair(Red& a, Red& b, std::vector<double>& va, std::vector<double>& vb) {
  const int64_t ca = a.launch(0);
  const int64_t cb = b.launch(ca);
  if (ca + cb) {
    HC_HIP(hipMemcpyAsync(a.S->hpart, a.S->dpart, (ca + cb) * sizeof(double), hipMemcpyDeviceToHost, a.S->stream));
    HC_HIP(hipStreamSynchronize(a.S->stream));
  }
  va = a.collect();
  vb = b.collect();
}

// max(|x|_inf, |y|_inf) for vectors of lengths n and m, one host round trip
double maxabs2(hc_solver* S, const double* x, int64_t n, const double* y, int64_t m) {
  RedOps ox{}, oy{};
  ox.nops = oy.nops = 1;
  ox.op[0] = RedOp{RED_MAX_MUL, x, nullptr, 0.0, nullptr};
  oy.op[0] = RedOp{RED_MAX_MUL, y, nullptr, 0.0, nullptr};
  const int na = n > 0 ? reduce_launch(n, ox, S->dpart, S->stream) : 0;
  const int nb = m > 0 ? reduce_launch(m, oy, S->dpart + na, S->stream) : 0;
  if (na + nb == 0) return 0.0;
  HC_HIP(hipMemcpyAsync(S->hpart, S->dpart, (size_t)(na + nb) * sizeof(double), hipMemcpyDeviceToHost, S->stream));
  HC_HIP(hipStreamSynchronize(S->stream));
  double acc = 0.0;
  for (int i = 0; i < na + nb; ++i) {
    const double v = S->hpart[i];
    acc = (std::isnan(v) || std::isnan(acc)) ? NAN : std::max(acc, v);
  }
  return acc;
}

void A_mul(hc_solver* S, const double* x, double* y, double alpha, double beta) {
  spmv(S->dA, x, y, alpha, beta, S->stream);
  // with leaf blocks the dense rows are stored on the tail columns only
  dense_rows_gemv((int)S->drows.size(), S->leaves ? S->nt : S->n, S->dAd, S->ddrows,
                  S->leaves ? S->cm.tcols : nullptr, x, y, alpha, S->stream);
}
void At_mul(hc_solver* S, const double* z, double* y, double alpha, double beta) {
  spmv(S->dAt, z, y, alpha, beta, S->stream);
  dense_rows_gemv_t((int)S->drows.size(), S->leaves ? S->nt : S->n, S->dAd, S->ddrows,
                    S->leaves ? S->cm.tcols : nullptr, z, y, alpha, S->dDrT, S->stream);
}
// Cone-layer probes (settings.profile): an event pair on the handle's stream
// around each group of cone launches, and the algorithmic HBM bytes of every
// launch from its segment's size: what the step must read and write at least
// once (iterate and direction rows, the scaling state, H diagonal, M blocks).
enum ConeOp { CO_SCALE, CO_MBLOCK, CO_APPLY, CO_RECOVER, CO_DS, CO_STEP };
double cone_op_bytes(const SegDev& g, ConeOp op) {
  if (g.count == 0 || g.kind == HC_CONE_ZERO) return 0.0;
  const double R = (double)g.count * (double)g.dim;
  const double SD = (double)state_doubles(g.kind, g.dim, g.k) * (double)g.count;
  const double MB = (double)mblock_doubles(g.kind, g.dim) * (double)g.count;
  switch (op) {
    case CO_SCALE: return 8.0 * (3.0 * R + SD);     // s, z in; state, diag(H) out
    case CO_MBLOCK: return 8.0 * (SD + MB);         // state in; M blocks out
    case CO_APPLY: return 8.0 * (2.0 * R + SD);     // x, state in; y out
    case CO_RECOVER: return 8.0 * (3.0 * R + SD);   // d_s, dz, state in; ds out
    case CO_DS: return 8.0 * (5.0 * R + SD);        // s, z, ds_a, dz_a, state in; d_s out
    case CO_STEP: return 8.0 * 4.0 * R;             // s, z, ds, dz in
  }
  return 0.0;
}
struct ConeProbe {
  hc_solver* S;
  // which: 0 every segment, 1 the symmetric ones, 2 exp/pow
  // (only: that segment alone)
  explicit ConeProbe(hc_solver* S_, ConeOp op, int which = 0, const SegDev* only = nullptr) : S(S_) {
    if (!S->st.profile || !S->cprof) return;
    HC_HIP(hipEventRecord(S->cprof->next(), S->stream));
    for (const SegDev& g : S->sdev) {
      const bool ns = g.kind == HC_CONE_EXP || g.kind == HC_CONE_POW;
      if ((which == 1 && ns) || (which == 2 && !ns) || (only && only != &g)) continue;
      const double b = cone_op_bytes(g, op);
      if (b > 0.0) {
        S->info.cone_bytes += b;
        S->info.cone_launches++;
      }
    }
  }
  ~ConeProbe() {
    if (S->st.profile && S->cprof) (void)hipEventRecord(S->cprof->next(), S->stream);
  }
};

void P_mul(hc_solver* S, const double* x, double* y, double alpha, double beta) {
  if (S->dP.nnz == 0) {
    if (beta == 0.0) vfill(S->n, 0.0, y, S->stream);
    else if (beta != 1.0) vaxpby(S->n, 0.0, x, beta, y, S->stream);
    return;
  }
  spmv(S->dP, x, y, alpha, beta, S->stream);
}
void H_apply(hc_solver* S, int mode, const double* x, double* y) {
  ConeProbe probe(S, CO_APPLY);
  cone_apply_all(S->sdev, mode, S->delta, x, nullptr, y, S->stream);
}

// unit diagonal on the padding rows [nt, ntp) of the dense tail
__global__ void k_pad_identity(int64_t nt, int64_t ntp, int64_t ld, double* __restrict__ S) {
  for (int64_t i = nt + threadIdx.x; i < ntp; i += blockDim.x) S[i + i * ld] = 1.0;
}

__global__ void k_get_diag(int64_t n, int64_t ld, const double* __restrict__ A, double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[i + i * ld];
}

// the look-ahead's schedule; with settings.profile = 2 its launches run one at
// a time on the handle's stream, so that the MFMA update durations do not
// overlap other kernels
Aux* lookahead(hc_solver* S) {
  S->aux.serial = S->st.profile == 2 || S->noalloc;   // the allocation-free call creates no stream or events
  return &S->aux;
}

// factor the regularised KKT system at the current scaling (state + hdiag
// filled).  FP64: delta = delta_s + delta_d max|K_ii| (the oracle's reading).
// Mixed mode factors only the Schur complement in FP32 (the cone pivots
// -(H_c + delta I) are inverted exactly in FP64), so the proportional term
// takes max|S_ii| of the last FP32-factored S; `fp64` redoes the whole
// factorisation with the FP64 regularisation (the refinement fallback).
void factor(hc_solver* S, bool fp64 = false) {
  hipStream_t st = S->stream;
  const bool low = S->mixed && !fp64;
  if (low) {
    S->delta = S->st.static_reg + S->st.dyn_reg * std::max(S->maxPdiag, S->sdiag_max);
  } else {
    Red r(S, S->m);
    r.maxabs(S->dhdiag);
    const double hmax = r.run()[0];
    const double ds = S->mixed ? 1e-8 : S->st.static_reg;
    const double dd = S->mixed ? std::ldexp(1.0, -104) : S->st.dyn_reg;
    S->delta = ds + dd * std::max(S->maxPdiag, hmax);
  }
  {
    ConeProbe probe(S, CO_MBLOCK);
    cone_mblock_all(S->sdev, S->delta, S->dmwork, st);   // segments run in order: one work buffer
  }
  // The tail is factored padded to ld (a multiple of 64) with an identity
  // block on the padding: [[S, 0], [0, I]] = [[L, 0], [0, I]] [[L, 0], [0, I]]',
  // so every panel, TRSM and trailing update is a whole number of 64-blocks
  // (no edge tiles), and the solves use the leading nt x nt part.
  const int64_t nt = S->nt, ntp = S->ld;
  fill_lower_zero(ntp, S->ld, S->dS, st);
  if (ntp > nt) {
    hipLaunchKernelGGL(k_pad_identity, dim3(1), dim3(64), 0, st, nt, ntp, S->ld, S->dS);
    HC_LAUNCH_CHECK();
  }
  if (S->leaves) {
    vfill(S->lval_total, 0.0, S->cm.lval, st);
    vfill(S->cval_total, 0.0, S->cm.cval, st);
    add_P_delta_map(S->dP, S->n, S->delta, S->cm, st);
    if (S->ordered) {
      ordered_sum(S->opair, S->dmval, S->dA.val, nullptr, S->cm.ST, S->cm.lval, S->cm.cval, st);
    } else {
      const int64_t ns = S->ntask_short, nl = (int64_t)S->tra.size() - ns;
      assemble_pairs_map(ns, S->dtra, S->dtrb, S->dtm, S->dmval, S->dA, S->cm, false, st);
      assemble_pairs_map(nl, S->dtra + ns, S->dtrb + ns, S->dtm + ns, S->dmval, S->dA, S->cm, true, st);
    }
  } else {
    add_P_delta(S->dP, S->n, S->delta, S->ld, S->dS, st);
    group_T(S->gplan, S->dmval, S->dA, st);
    group_gather(S->gplan, S->n, S->dAt, S->ld, S->dS, st);
    if (S->ordered) {
      ordered_sum(S->opair, S->dmval, S->dA.val, nullptr, S->dS, nullptr, nullptr, st);
    } else {
      const int64_t ns = S->ntask_short, nl = (int64_t)S->tra.size() - ns;
      assemble_pairs(ns, S->dtra, S->dtrb, S->dtm, S->dmval, S->dA, S->ld, S->dS, false, st);
      assemble_pairs(nl, S->dtra + ns, S->dtrb + ns, S->dtm + ns, S->dmval, S->dA, S->ld, S->dS, true, st);
    }
    if (!S->pdense.empty()) {
      for (size_t i = 0; i < S->pdense.size(); ++i) {
        const auto& pd = S->pdense[i];
        const Segment& g = S->segs[pd.first];
        psd_dense_T(g.dim, g.count, S->pdense_coff[i], g.moff, S->dmval, S->pcols, S->dA.val, S->n,
                    S->dT + pd.second * S->n, st);
      }
      dense_T_gather(S->n, S->dpe_rp, S->dpe_e, S->dpe_p, S->dAt.val, S->dT, S->ld, S->dS, st);
    }
  }
  const int nd = (int)S->drows.size();
  if (S->K1 > 0) {
    for (const auto& rg : S->ls_ranges)
      lsoc_lowrank(S->sdev[rg.seg], rg.count, S->dls_cone + rg.first, S->dls_col + rg.first, S->dls_dst + rg.first,
                   S->dAt, (S->K1 - nd) * nt, S->dAd, st);
    // the operand carries zero rows up to multiples of 16 (set at bind), which
    // lets the update run on the MFMA DMA kernel; rows of negative weight
    // (the p_+ rows) form the second block, subtracted
    scale_dense_rows((int)(S->K1 + S->K2), nt, S->dAd, S->ddmidx, S->dmval, S->dBd, st);
    gemm_nt<double>(S->dS, S->ld, S->dBd, nt, S->dBd, nt, nt, nt, S->K1, 1.0, true, 0, 0, st);
    if (S->K2 > 0)
      gemm_nt<double>(S->dS, S->ld, S->dBd + S->K1 * nt, nt, S->dBd + S->K1 * nt, nt, nt, nt, S->K2, -1.0, true, 0,
                      0, st);
  }
  const double tol = 0.0;
  // leaves are factored in FP64 in both modes; their updates land in the tail
  leaf_factor(S->cm, tol, S->delta, S->dhits, st);
  if (S->cm.lslot) ordered_sum(S->oleaf, nullptr, nullptr, S->cm.lslot, S->cm.ST, nullptr, nullptr, st);
  S->use64 = !low;
  Prof* pf = S->st.profile ? S->prof.get() : nullptr;
  if (low && nt > 0) {   // max |S_ii| for the next FP32 factorisation's delta
    hipLaunchKernelGGL(k_get_diag, dim3((unsigned)ceil_div(nt, 256)), dim3(256), 0, st, nt, S->ld, S->dS, S->sb);
    HC_LAUNCH_CHECK();
    Red r(S, nt);
    r.maxabs(S->sb);
    S->sdiag_max = r.run()[0];
  }
  if (S->snap_S && nt > 0) {
    HC_HIP(hipMemcpy2DAsync(S->snap_S, nt * 8, S->dS, S->ld * 8, nt * 8, nt, hipMemcpyDeviceToHost, st));
    HC_HIP(hipStreamSynchronize(st));
  }
  if (nt == 0) {
    // every column sits in a leaf block: nothing dense to factor
  } else if (low) {
    lower_to_f32(ntp, S->ld, S->dS, S->dS32, st);
    dense_cholesky<float>(S->dS32, ntp, S->ld, S->dLinv32, tol, S->delta, S->dhits, st, pf, lookahead(S),
                          S->tail_last.data());
    dense_block_inverses<float>(S->dS32, ntp, S->ld, S->dLinv32, S->dX256f, S->dXT256f, st);
  } else {
    dense_cholesky<double>(S->dS, ntp, S->ld, S->dLinv, tol, S->delta, S->dhits, st, pf, lookahead(S),
                           S->tail_last.data());
    dense_block_inverses<double>(S->dS, ntp, S->ld, S->dLinv, S->dX256, S->dXT256, st);
  }
  S->info.factorizations++;
  if (pf) {
    S->info.gemm_ms += pf->collect_ms();
    S->info.gemm_flops += pf->flops;
    S->info.gemm_launches += pf->launches;
    pf->flops = 0;
    pf->launches = 0;
  }
}

// mixed mode: factor the (still FP64) Schur complement in FP64 for the rest of
// this iteration
void fallback_fp64(hc_solver* S) {
  factor(S, true);
  S->info.fp64_fallbacks++;
}

// x_r = S^-1 u_r for k = 1 or 2 right-hand sides: leaves in FP64 (one pass
// per right-hand side), the tail in the factor precision with both
// right-hand sides in one pass of the dense triangular solves
void schur_solve_n(hc_solver* S, int k, const double* const* u, double* const* x) {
  hipStream_t st = S->stream;
  const int64_t nt = S->nt;
  const double* ut[2] = {u[0], k > 1 ? u[1] : nullptr};
  double* xt[2] = {x[0], k > 1 ? x[1] : nullptr};
  double* uTs[2] = {S->uT, S->uTb};
  double* xTs[2] = {S->xT, S->xTb};
  if (S->leaves)
    for (int r = 0; r < k; ++r) {
      gather_tail(S->cm, u[r], uTs[r], st);
      leaf_forward(S->cm, u[r], x[r], uTs[r], st);   // y_b into x at the leaf columns
      ut[r] = uTs[r];
      xt[r] = xTs[r];
    }
  if (nt == 0) {
    // all columns in leaf blocks
  } else if (S->mixed && !S->use64) {
    for (int r = 0; r < k; ++r) {   // per right-hand side: scale by its max |entry| for FP32
      RedOps ops{};
      ops.nops = 1;
      ops.op[0] = RedOp{RED_MAX_MUL, ut[r], nullptr, 0.0, nullptr};
      const int nb = reduce_launch(nt, ops, S->dpart, st);
      combine_max(nb, S->dpart, S->dscal + r, st);
      to_f32(nt, ut[r], S->dscal + r, S->sb32 + r * nt, st);
    }
    dense_solve<float>(S->dS32, nt, S->ld, S->dX256f, S->dXT256f, S->sb32, S->sy32, S->sx32, k, st,
                       S->tail_last.data());
    for (int r = 0; r < k; ++r) from_f32(nt, S->sx32 + r * nt, S->dscal + r, xt[r], st);
  } else if (k == 1) {
    vcopy(nt, ut[0], S->sb, st);
    dense_solve<double>(S->dS, nt, S->ld, S->dX256, S->dXT256, S->sb, S->sy, xt[0], 1, st, S->tail_last.data());
  } else {
    for (int r = 0; r < k; ++r) vcopy(nt, ut[r], S->sb + r * nt, st);
    dense_solve<double>(S->dS, nt, S->ld, S->dX256, S->dXT256, S->sb, S->sy, S->sx, k, st, S->tail_last.data());
    for (int r = 0; r < k; ++r) vcopy(nt, S->sx + r * nt, xt[r], st);
  }
  if (S->leaves)
    for (int r = 0; r < k; ++r) {
      leaf_backward(S->cm, xTs[r], x[r], st);
      scatter_tail(S->cm, xTs[r], x[r], st);
    }
}
void schur_solve(hc_solver* S, const double* u, double* x) { schur_solve_n(S, 1, &u, &x); }

// K_reg [x; z] = [r1; r2]:  z = M (A x - r2),  S x = r1 + A' M r2
void solve_reg(hc_solver* S, const double* r1, const double* r2, double* x, double* z) {
  hipStream_t st = S->stream;
  H_apply(S, 1, r2, S->t1);                    // t1 = M r2
  vcopy(S->n, r1, S->u1, st);
  At_mul(S, S->t1, S->u1, 1.0, 1.0);           // u1 = r1 + A' t1
  schur_solve(S, S->u1, x);
  A_mul(S, x, S->w1, 1.0, 0.0);                // w1 = A x
  vaxpby(S->m, -1.0, r2, 1.0, S->w1, st);      // w1 -= r2
  H_apply(S, 1, S->w1, z);
}

// iterative refinement against the unregularised K; result in (xo, zo)
int64_t kkt_solve_once(hc_solver* S, const double* r1, const double* r2, double* xo, double* zo, double* best_out,
                       double* nb_out);
// the residual at which the refinement stops: the fixed tolerances, or (with
// ir_mu_frac) a fraction of the iteration's mu relative to the right-hand side
double ir_target(const hc_solver* S, double nb) {
  return std::max(S->st.ir_abstol + S->st.ir_reltol * nb,
                  S->st.ir_mu_frac * std::min(S->info.mu, 1.0) * (1.0 + nb));
}

int64_t kkt_solve(hc_solver* S, const double* r1, const double* r2, double* xo, double* zo) {
  double best = 0, nb = 0;
  int64_t k = kkt_solve_once(S, r1, r2, xo, zo, &best, &nb);
  if (S->mixed && !S->use64 && !(best <= std::max(1e-6 * (1.0 + nb), ir_target(S, nb)))) {
    fallback_fp64(S);
    k += kkt_solve_once(S, r1, r2, xo, zo, &best, &nb);
  }
  return k;
}

int64_t kkt_solve_once(hc_solver* S, const double* r1, const double* r2, double* xo, double* zo, double* best_out,
                       double* nb_out) {
  hipStream_t st = S->stream;
  const int64_t n = S->n, m = S->m;
  double nb;
  nb = maxabs2(S, r1, n, r2, m);
  double* x = S->irx;
  double* z = S->irz;
  double* xn = S->irxn;
  double* zn = S->irzn;
  vfill(n, 0.0, x, st);
  vfill(m, 0.0, z, st);
  vcopy(n, r1, S->irrx, st);
  vcopy(m, r2, S->irrz, st);
  double best = nb, rnorm = nb;
  const double target = ir_target(S, nb);
  bool have_best = false;
  int64_t solves = 0;
  for (int it = 0; it <= S->st.ir_max; ++it) {
    solve_reg(S, S->irrx, S->irrz, S->kx, S->kz);   // correction in kx, kz
    vlin3(n, 1.0, x, 1.0, S->kx, 0.0, nullptr, xn, st);
    vlin3(m, 1.0, z, 1.0, S->kz, 0.0, nullptr, zn, st);
    ++solves;
    // residual r - K [xn; zn] with the unregularised K
    P_mul(S, xn, S->kx, 1.0, 0.0);
    At_mul(S, zn, S->kx, 1.0, 1.0);
    A_mul(S, xn, S->kz, 1.0, 0.0);
    H_apply(S, 0, zn, S->t2);
    vaxpby(m, -1.0, S->t2, 1.0, S->kz, st);         // kz = A xn - H zn
    vlin3(n, 1.0, r1, -1.0, S->kx, 0.0, nullptr, S->kx, st);
    vlin3(m, 1.0, r2, -1.0, S->kz, 0.0, nullptr, S->kz, st);
    const double rn = maxabs2(S, S->kx, n, S->kz, m);
    if (rn < best || !have_best) {
      if (rn < best) {
        vcopy(n, xn, S->irbx, st);
        vcopy(m, zn, S->irbz, st);
        best = rn;
        have_best = true;
      }
    }
    if (rn <= target) break;
    if (it > 0 && rn > 0.5 * rnorm) break;
    std::swap(x, xn);
    std::swap(z, zn);
    std::swap(S->irrx, S->kx);
    std::swap(S->irrz, S->kz);
    rnorm = rn;
  }
  if (have_best) {
    vcopy(n, S->irbx, xo, st);
    vcopy(m, S->irbz, zo, st);
  } else {
    vfill(n, 0.0, xo, st);
    vfill(m, 0.0, zo, st);
  }
  S->irx = x;
  S->irz = z;
  S->irxn = xn;
  S->irzn = zn;
  S->info.ir_solves += solves;
  *best_out = have_best ? best : NAN;
  *nb_out = nb;
  if (S->st.verbose >= 2) {
    std::printf("      kkt solve: |rhs| %.3e best residual %.3e (%s) solves %lld\n", nb, have_best ? best : NAN,
                S->mixed && !S->use64 ? "fp32 factor" : "fp64 factor", (long long)solves);
    std::fflush(stdout);
  }
  return solves;
}

// Two systems K [x; z] = [r1; r2] refined in lockstep (kkt_solve_once's
// rule for each): every step's two Schur solves share one pass of the dense
// triangular solves; a system leaves the loop under its own stopping test.
// Results in (xa, za) and (xb, zb); the mixed mode's FP64 fallback as in
// kkt_solve, per system.
struct IRSys {
  const double *r1, *r2;
  double *xo, *zo, *x, *z, *xn, *zn, *bx, *bz, *rx, *rz, *kx, *kz, *u;
  double nb = 0, best = 0, rnorm = 0, target = 0;
  bool have_best = false, done = false;
};
int64_t kkt_solve_pair(hc_solver* S, const double* r1a, const double* r2a, double* xa, double* za, const double* r1b,
                       const double* r2b, double* xb, double* zb) {
  hipStream_t st = S->stream;
  const int64_t n = S->n, m = S->m;
  const bool low = S->mixed && !S->use64;
  IRSys sy[2];
  sy[0] = IRSys{r1a, r2a, xa, za, S->irx, S->irz, S->irxn, S->irzn, S->irbx, S->irbz, S->irrx, S->irrz, S->kx,
                S->kz, S->u1};
  sy[1] = IRSys{r1b, r2b, xb, zb, S->jrx, S->jrz, S->jrxn, S->jrzn, S->jrbx, S->jrbz, S->jrrx, S->jrrz, S->jkx,
                S->jkz, S->u1b};
  for (IRSys& y : sy) {
    y.nb = maxabs2(S, y.r1, n, y.r2, m);
    vfill(n, 0.0, y.x, st);
    vfill(m, 0.0, y.z, st);
    vcopy(n, y.r1, y.rx, st);
    vcopy(m, y.r2, y.rz, st);
    y.best = y.rnorm = y.nb;
    y.target = ir_target(S, y.nb);
  }
  int64_t solves = 0;
  for (int it = 0; it <= S->st.ir_max; ++it) {
    IRSys* act[2];
    int k = 0;
    for (IRSys& y : sy)
      if (!y.done) act[k++] = &y;
    if (k == 0) break;
    const double* us[2];
    double* xs[2];
    for (int r = 0; r < k; ++r) {   // Schur right-hand side r1 + A' M r2 of the residual
      IRSys& y = *act[r];
      H_apply(S, 1, y.rz, S->t1);
      vcopy(n, y.rx, y.u, st);
      At_mul(S, S->t1, y.u, 1.0, 1.0);
      us[r] = y.u;
      xs[r] = y.kx;
    }
    schur_solve_n(S, k, us, xs);
    for (int r = 0; r < k; ++r) {
      IRSys& y = *act[r];
      A_mul(S, y.kx, S->w1, 1.0, 0.0);           // correction z = M (A x - r2)
      vaxpby(m, -1.0, y.rz, 1.0, S->w1, st);
      H_apply(S, 1, S->w1, y.kz);
      vlin3(n, 1.0, y.x, 1.0, y.kx, 0.0, nullptr, y.xn, st);
      vlin3(m, 1.0, y.z, 1.0, y.kz, 0.0, nullptr, y.zn, st);
      ++solves;
      P_mul(S, y.xn, y.kx, 1.0, 0.0);            // residual with the unregularised K
      At_mul(S, y.zn, y.kx, 1.0, 1.0);
      A_mul(S, y.xn, y.kz, 1.0, 0.0);
      H_apply(S, 0, y.zn, S->t2);
      vaxpby(m, -1.0, S->t2, 1.0, y.kz, st);
      vlin3(n, 1.0, y.r1, -1.0, y.kx, 0.0, nullptr, y.kx, st);
      vlin3(m, 1.0, y.r2, -1.0, y.kz, 0.0, nullptr, y.kz, st);
      const double rn = maxabs2(S, y.kx, n, y.kz, m);
      if (rn < y.best) {
        vcopy(n, y.xn, y.bx, st);
        vcopy(m, y.zn, y.bz, st);
        y.best = rn;
        y.have_best = true;
      }
      if (rn <= y.target || (it > 0 && rn > 0.5 * y.rnorm)) {
        y.done = true;
        continue;
      }
      std::swap(y.x, y.xn);
      std::swap(y.z, y.zn);
      std::swap(y.rx, y.kx);
      std::swap(y.rz, y.kz);
      y.rnorm = rn;
    }
  }
  for (IRSys& y : sy) {
    if (y.have_best) {
      vcopy(n, y.bx, y.xo, st);
      vcopy(m, y.bz, y.zo, st);
    } else {
      vfill(n, 0.0, y.xo, st);
      vfill(m, 0.0, y.zo, st);
    }
  }
  S->irx = sy[0].x, S->irz = sy[0].z, S->irxn = sy[0].xn, S->irzn = sy[0].zn;
  S->irrx = sy[0].rx, S->irrz = sy[0].rz, S->kx = sy[0].kx, S->kz = sy[0].kz;
  S->jrx = sy[1].x, S->jrz = sy[1].z, S->jrxn = sy[1].xn, S->jrzn = sy[1].zn;
  S->jrrx = sy[1].rx, S->jrrz = sy[1].rz, S->jkx = sy[1].kx, S->jkz = sy[1].kz;
  S->info.ir_solves += solves;
  if (S->st.verbose >= 2) {
    std::printf("      kkt solve pair: |rhs| %.3e / %.3e best residual %.3e / %.3e solves %lld\n", sy[0].nb, sy[1].nb,
                sy[0].have_best ? sy[0].best : NAN, sy[1].have_best ? sy[1].best : NAN, (long long)solves);
    std::fflush(stdout);
  }
  if (low)
    for (IRSys& y : sy) {   // the mixed mode's fallback, per system
      if (y.have_best && y.best <= std::max(1e-6 * (1.0 + y.nb), ir_target(S, y.nb))) continue;
      if (!S->use64) fallback_fp64(S);
      double best = 0, nb = 0;
      solves += kkt_solve_once(S, y.r1, y.r2, y.xo, y.zo, &best, &nb);
    }
  return solves;
}

struct Resid {
  double xPx, qx, bz, sz, rd_n, rp_n, x_n, s_n, z_n, atz_n, px_n, axs_n;
};

// Px, Ax, A'z, r_d and r_p vectors and all norms of the termination tests
Resid residuals(hc_solver* S) {
  hipStream_t st = S->stream;
  const int64_t n = S->n, m = S->m;
  P_mul(S, S->x, S->Px, 1.0, 0.0);
  A_mul(S, S->x, S->Ax, 1.0, 0.0);
  At_mul(S, S->z, S->Atz, 1.0, 0.0);
  vlin3(n, 1.0, S->Px, 1.0, S->Atz, S->tau, S->dq, S->rdv, st);        // P x + A'z + q tau
  vlin3(m, -1.0, S->Ax, -1.0, S->s, S->tau, S->db, S->rpv, st);        // -A x - s + b tau
  Red rn(S, n), rm(S, m);
  const int i_xPx = rn.dot(S->x, S->Px), i_qx = rn.dot(S->dq, S->x), i_rd = rn.maxabs(S->rdv, S->dD, true),
            i_x = rn.maxabs(S->x, S->dD, false), i_atz = rn.maxabs(S->Atz, S->dD, true),
            i_px = rn.maxabs(S->Px, S->dD, true);
  const int i_bz = rm.dot(S->db, S->z), i_sz = rm.dot(S->s, S->z), i_rp = rm.maxabs(S->rpv, S->dE, true),
            i_s = rm.maxabs(S->s, S->dE, true), i_z = rm.maxabs(S->z, S->dE, false),
            i_axs = rm.maxabs(S->Ax, S->dE, true, S->s, 1.0);
  std::vector<double> a, b;
  run_pair(rn, rm, a, b);
  Resid R;
  R.xPx = a[i_xPx]; R.qx = a[i_qx]; R.rd_n = a[i_rd]; R.x_n = a[i_x]; R.atz_n = a[i_atz]; R.px_n = a[i_px];
  R.bz = b[i_bz]; R.sz = b[i_sz]; R.rp_n = b[i_rp]; R.s_n = b[i_s]; R.z_n = b[i_z]; R.axs_n = b[i_axs];
  return R;
}

int check(hc_solver* S, const Resid& R) {
  const double t = S->tau, c = S->cscale, eps = S->st.eps_feas, ei = S->st.eps_inf;
  const double rp = R.rp_n / t, rd = R.rd_n / (c * t);
  const double gp = (0.5 * R.xPx / t + R.qx) / (c * t), gd = (-0.5 * R.xPx / t - R.bz) / (c * t);
  const double xn = R.x_n / t, sn = R.s_n / t, zn = R.z_n / (c * t);
  S->info.res_primal = rp;
  S->info.res_dual = rd;
  S->info.obj_primal = gp;
  S->info.obj_dual = gd;
  S->info.gap = std::fabs(gp - gd);
  if (rp < eps * std::max(1.0, S->bnorm_user + xn + sn) && rd < eps * std::max(1.0, S->qnorm_user + xn + zn) &&
      std::fabs(gp - gd) < eps * std::max(1.0, std::min(std::fabs(gp), std::fabs(gd))))
    return HC_STATUS_SOLVED;
  const double bz = R.bz / c, xu = R.x_n, zu = R.z_n / c, su = R.s_n;
  if (bz < -ei && R.atz_n / c < -ei * std::max(1.0, xu + zu) * bz) return HC_STATUS_PRIMAL_INFEASIBLE;
  const double qx = R.qx / c;
  if (qx < -ei && R.px_n / c < -ei * std::max(1.0, xu) * qx && R.axs_n < -ei * std::max(1.0, xu + su) * qx)
    return HC_STATUS_DUAL_INFEASIBLE;
  if (!std::isfinite(rp) || !std::isfinite(rd) || !std::isfinite(gp)) return HC_STATUS_NUMERICAL_ERROR;
  return 0;
}

void scale_all(hc_solver* S, double mu, bool force_dual, int* pd_count) {
  vfill(1, 0.0, (double*)S->dpd, S->stream);   // both counters (fill kernels, not memsets, throughout)
  {
    ConeProbe probe(S, CO_SCALE);
    cone_scale_all(S->sdev, S->s, S->z, mu, force_dual ? 1 : 0, S->dhdiag, S->dpd, S->stream);
  }
  int h = 0;
  HC_HIP(hipMemcpyAsync(&h, S->dpd, sizeof(int), hipMemcpyDeviceToHost, S->stream));
  HC_HIP(hipStreamSynchronize(S->stream));
  *pd_count = h;
}

struct Dir {
  double dtau, dkappa;
};

// solve for the RHS (d_x = r1, -(d_z - d_s) = r2, d_tau, d_kappa) and recover
// Delta (r1 == nullptr: (x1, z1) already solved for it)
Dir direction(hc_solver* S, const double* r1, const double* r2, double dtau_rhs, double dkap_rhs,
              const double* ds_rhs, double* dxo, double* dzo, double* dso) {
  hipStream_t st = S->stream;
  const int64_t n = S->n, m = S->m;
  if (r1) kkt_solve(S, r1, r2, S->x1, S->z1);
  // w = 2 P xi + q with xi = x / tau:  w'x1, w'x2 ; b'z1, b'z2
  Red rn(S, n), rm(S, m);
  const double ti = 1.0 / S->tau;
  vlin3(n, 2.0 * ti, S->Px, 1.0, S->dq, 0.0, nullptr, S->t2, st);
  const int a1 = rn.dot(S->t2, S->x1), a2 = rn.dot(S->t2, S->x2);
  const int b1 = rm.dot(S->db, S->z1), b2 = rm.dot(S->db, S->z2);
  std::vector<double> va, vb;
  run_pair(rn, rm, va, vb);
  Dir d;
  const double xPx = S->xPx_cache;
  const double num = dtau_rhs - dkap_rhs / S->tau + va[a1] + vb[b1];
  const double den = S->kappa / S->tau + xPx / (S->tau * S->tau) - va[a2] - vb[b2];
  d.dtau = num / den;
  vlin3(n, 1.0, S->x1, d.dtau, S->x2, 0.0, nullptr, dxo, st);
  vlin3(m, 1.0, S->z1, d.dtau, S->z2, 0.0, nullptr, dzo, st);
  {
    ConeProbe probe(S, CO_RECOVER);
    cone_apply_all(S->sdev, 0, 0.0, dzo, ds_rhs, dso, st);
  }
  d.dkappa = -(dkap_rhs + S->kappa * d.dtau) / S->tau;
  return d;
}

}  // namespace

namespace {

// ===========================================================================
// step rule
// ===========================================================================
struct Step {
  const double *ds, *dz;
  double dtau, dkappa;
};

double step_length(hc_solver* S, const Step& d, bool combined) {
  hipStream_t st = S->stream;
  double a = 1.0;
  if (d.dtau < 0) a = std::min(a, -S->tau / d.dtau);
  if (d.dkappa < 0) a = std::min(a, -S->kappa / d.dkappa);
  {   // every symmetric segment's partial minima, then one host round trip
    int64_t off = 0;
    {
      ConeProbe probe(S, CO_STEP, 1);
      off = cone_step_sym_all(S->sdev, S->s, S->z, d.ds, d.dz, S->dpart, st);
    }
    if (off) {
      HC_HIP(hipMemcpyAsync(S->hpart, S->dpart, off * sizeof(double), hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      for (int64_t i = 0; i < off; ++i) a = std::min(a, S->hpart[i]);
    }
  }
  if (!S->has_nonsym) return a;
  // mu(alpha) = (c0 + c1 a + c2 a^2) / (nu + 1)
  double c0 = 0, c1 = 0, c2 = 0;
  if (combined) {
    Red r(S, S->m);
    const int i0 = r.dot(S->s, S->z), i1 = r.dot(S->s, d.dz), i2 = r.dot(d.ds, S->z), i3 = r.dot(d.ds, d.dz);
    const auto v = r.run();
    c0 = v[i0] + S->kappa * S->tau;
    c1 = v[i1] + v[i2] + S->kappa * d.dtau + d.dkappa * S->tau;
    c2 = v[i3] + d.dkappa * d.dtau;
  }
  const double ratio = S->st.backtrack;
  // the first batch is the first trial alone (the usual outcome is that it
  // passes, and each trial of a batch costs every cone a conjugate-point
  // solve); later batches take up to 8
  int batch = 1;
  while (true) {
    if (a < 1e-10) return 0.0;
    // the next trials a, a r, a r^2, ... (products formed in sequence)
    double trial[8];
    double t = a;
    int nt = 0;
    for (; nt < batch; ++nt) {
      if (t < 1e-10) break;
      trial[nt] = t;
      t *= ratio;
    }
    unsigned long long all = (nt >= 64) ? ~0ull : ((1ull << nt) - 1ull);
    for (auto& g : S->sdev) {
      if (g.kind != HC_CONE_EXP && g.kind != HC_CONE_POW) continue;
      int nb = 0;
      {
        ConeProbe probe(S, CO_STEP, 2, &g);
        nb = cone_trial_nonsym(g, S->s, S->z, d.ds, d.dz, a, ratio, nt, combined ? 1 : 0, S->st.beta, c0, c1, c2,
                               (double)(S->nu + 1), S->dmask, st);
      }
      HC_HIP(hipMemcpyAsync(S->hmask, S->dmask, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < nb; ++i) all &= S->hmask[i];
    }
    for (int j = 0; j < nt; ++j)
      if (all & (1ull << j)) return trial[j];
    if (nt < batch) return 0.0;
    a = t;
    batch = 8;
  }
}

// ===========================================================================
// initial point
// ===========================================================================
__global__ void k_identity_state(SegDev g, double* hdiag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = g.count;
  if (i >= N) return;
  if (g.kind == HC_CONE_ZERO) {
    hdiag[g.base + i] = 0.0;
  } else if (g.kind == HC_CONE_NONNEG) {
    g.state[i] = 1.0;
    hdiag[g.base + i] = 1.0;
  } else if (g.kind == HC_CONE_SOC) {
    for (int j = 0; j < g.dim; ++j) {
      g.state[j * N + i] = (j == 0) ? 1.0 : 0.0;
      hdiag[g.base + j * N + i] = 1.0;
    }
    g.state[g.dim * N + i] = 1.0;
    if (g.dim > SOC_DMAX) g.state[(2 * (int64_t)g.dim + 1) * N + i] = 0.0;   // |wbar_1|
  } else if (g.kind == HC_CONE_PSD) {
    const int k = g.k;
    const int64_t kk = (int64_t)k * k;
    for (int r = 0; r < k; ++r)
      for (int j = 0; j < k; ++j) {
        const double v = (r == j) ? 1.0 : 0.0;
        g.state[(r * k + j) * N + i] = v;
        g.state[(kk + r * k + j) * N + i] = v;
        g.state[(2 * kk + r * k + j) * N + i] = v;
      }
    for (int j = 0; j < k; ++j) {
      g.state[(3 * kk + j) * N + i] = 1.0;
      g.state[(3 * kk + k + j) * N + i] = 1.0;
    }
    for (int p = 0; p < g.dim; ++p) hdiag[g.base + i * g.dim + p] = 1.0;
  }
}

// the last solved iterate without the equilibration: x D / tau, s / (E tau),
// E z / (c tau), internal rows
__global__ void k_warm_store(int64_t n, int64_t m, const double* __restrict__ x, const double* __restrict__ s,
                             const double* __restrict__ z, const double* __restrict__ D, const double* __restrict__ E,
                             double inv_ct, double inv_t, double* __restrict__ wx, double* __restrict__ ws,
                             double* __restrict__ wz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n > m ? n : m);
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n) wx[i] = D[i] * x[i] * inv_t;
    if (i < m) {
      ws[i] = s[i] / E[i] * inv_t;
      wz[i] = E[i] * z[i] * inv_ct;
    }
  }
}
// v = (1 - th) v_prev + th v, with v_prev carried to the current equilibration
__global__ void k_warm_blend(int64_t n, int64_t m, double th, const double* __restrict__ wx,
                             const double* __restrict__ ws, const double* __restrict__ wz,
                             const double* __restrict__ D, const double* __restrict__ E, double c,
                             double* __restrict__ x, double* __restrict__ s, double* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n > m ? n : m);
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n) x[i] = (1.0 - th) * (wx[i] / D[i]) + th * x[i];
    if (i < m) {
      s[i] = (1.0 - th) * (ws[i] * E[i]) + th * s[i];
      z[i] = (1.0 - th) * (wz[i] * c / E[i]) + th * z[i];
    }
  }
}

void init_point(hc_solver* S) {
  hipStream_t st = S->stream;
  const int64_t n = S->n, m = S->m;
  S->tau = S->kappa = 1.0;
  if (S->has_nonsym) {
    vfill(n, 0.0, S->x, st);
    for (auto& g : S->sdev) {
      cone_unit(g, S->s, st);
      cone_unit(g, S->z, st);
    }
    return;
  }
  for (auto& g : S->sdev) {
    hipLaunchKernelGGL(k_identity_state, dim3(cone_blocks(g)), dim3(CONE_BLOCK), 0, st, g, S->dhdiag);
    HC_LAUNCH_CHECK();
  }
  factor(S);
  vlin3(n, -1.0, S->dq, 0.0, nullptr, 0.0, nullptr, S->r1, st);
  kkt_solve(S, S->r1, S->db, S->x, S->z);
  vaxpby(m, -1.0, S->z, 0.0, S->s, st);                      // s = -z
  for (auto& g : S->sdev)
    if (g.kind == HC_CONE_ZERO) vfill(g.count, 0.0, S->s + g.base, st);
  for (int which = 0; which < 2; ++which) {
    double* v = which == 0 ? S->s : S->z;
    double amax = -INFINITY;
    for (auto& g : S->sdev) {
      const int nb = cone_max_neg_eig(g, v, S->dpart, st);
      if (!nb) continue;
      HC_HIP(hipMemcpyAsync(S->hpart, S->dpart, nb * sizeof(double), hipMemcpyDeviceToHost, st));
      HC_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < nb; ++i) amax = std::max(amax, S->hpart[i]);
    }
    if (amax >= 0)
      for (auto& g : S->sdev) cone_add_e(g, 1.0 + amax, v, st);
  }
}

// ===========================================================================
// one iteration (loop body of Algorithm 1); returns a status (0 = continue)
// ===========================================================================
double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int iterate(hc_solver* S, const Resid& R) {
  hipStream_t st = S->stream;
  const int64_t n = S->n, m = S->m;
  const double mu = (R.sz + S->kappa * S->tau) / (double)(S->nu + 1);
  S->info.mu = mu;
  // G(v): gx = -(P x + A'z + q tau) = -rdv ; gz = s + A x - b tau = -rpv
  const double gt = S->kappa + R.qx + R.bz + R.xPx / S->tau;
  bool force_dual = S->st.force_dual_scaling != 0;
  double alpha_c = 0, sigma = 0, alpha_a = 0;
  Dir dc{};
  for (int attempt = 0; attempt < 2; ++attempt) {
    double t0 = now_ms();
    int pd = 0;
    scale_all(S, mu, force_dual, &pd);
    double t1 = now_ms();
    factor(S);
    HC_HIP(hipStreamSynchronize(st));
    double t2 = now_ms();
    S->info.cone_ms += t1 - t0;
    S->info.factor_ms += t2 - t1;
    // constant system K [x2; z2] = [-q; b] and the affine one, r1 = gx,
    // r2 = -(gz - s) = rpv + s, refined together
    vlin3(n, -1.0, S->dq, 0.0, nullptr, 0.0, nullptr, S->r1c, st);
    vlin3(n, -1.0, S->rdv, 0.0, nullptr, 0.0, nullptr, S->r1, st);
    vlin3(m, 1.0, S->rpv, 1.0, S->s, 0.0, nullptr, S->r2, st);
    kkt_solve_pair(S, S->r1c, S->db, S->x2, S->z2, S->r1, S->r2, S->x1, S->z1);
    const Dir da = direction(S, nullptr, nullptr, gt, S->kappa * S->tau, S->s, S->dxa, S->dza, S->dsa);
    alpha_a = step_length(S, Step{S->dsa, S->dza, da.dtau, da.dkappa}, false);
    sigma = (1.0 - alpha_a) * (1.0 - alpha_a) * (1.0 - alpha_a);
    // combined
    const double dk = S->kappa * S->tau + da.dkappa * da.dtau - sigma * mu;
    {
      ConeProbe probe(S, CO_DS);
      cone_ds_all(S->sdev, S->s, S->z, S->dsa, S->dza, sigma * mu, S->dsrhs, st);
    }
    const double f = 1.0 - sigma;
    vlin3(n, -f, S->rdv, 0.0, nullptr, 0.0, nullptr, S->r1, st);
    // r2 = -(f gz - ds) = f rpv + ds
    vlin3(m, f, S->rpv, 1.0, S->dsrhs, 0.0, nullptr, S->r2, st);
    dc = direction(S, S->r1, S->r2, f * gt, dk, S->dsrhs, S->dx, S->dz, S->dsv);
    alpha_c = step_length(S, Step{S->dsv, S->dz, dc.dtau, dc.dkappa}, true);
    S->info.solve_kkt_ms += now_ms() - t2;
    if (alpha_c < 0.1 && pd > 0 && !force_dual) {
      force_dual = true;
      S->info.dual_switches++;
      continue;
    }
    break;
  }
  if (S->st.profile && S->cprof) S->info.cone_kernel_ms += S->cprof->collect_ms();
  if (S->st.verbose) {
    std::printf("    sigma %.3e alpha_a %.4f alpha_c %.4f delta %.2e ir %lld fp64-fallbacks %lld\n", sigma, alpha_a,
                alpha_c, S->delta, (long long)S->info.ir_solves, (long long)S->info.fp64_fallbacks);
    std::fflush(stdout);
  }
  if (alpha_c < 1e-4) return HC_STATUS_INSUFFICIENT_PROGRESS;
  const double a = S->st.step_fraction * alpha_c;
  vaxpby(n, a, S->dx, 1.0, S->x, st);
  vaxpby(m, a, S->dsv, 1.0, S->s, st);
  vaxpby(m, a, S->dz, 1.0, S->z, st);
  S->tau += a * dc.dtau;
  S->kappa += a * dc.dkappa;
  return 0;
}

void begin_solve(hc_solver* S) {
  const hc_info keep = S->info;
  S->info = hc_info{};
  S->info.setup_ms = keep.setup_ms;
  S->info.n_ordered = keep.n_ordered;
  S->info.n_leaves = keep.n_leaves;
  S->info.leaf_columns = keep.leaf_columns;
  S->info.sym_split_columns = keep.sym_split_columns;
  S->info.sym_supernodes = keep.sym_supernodes;
  S->info.sym_levels = keep.sym_levels;
  S->info.sym_nnz_l = keep.sym_nnz_l;
  S->info.psd_gathered_rows = keep.psd_gathered_rows;
  S->info.factor_flops = keep.factor_flops;
  vfill(1, 0.0, (double*)S->dhits, S->stream);
  S->sdiag_max = 0;
  init_point(S);
  if (S->st.warm_start && S->have_warm) {   // parametric re-solve from the last solution (Sec. 4.6)
    const int64_t L = std::max(S->n, S->m);
    const int nb = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div(L, 256)), 65535);
    hipLaunchKernelGGL(k_warm_blend, dim3(nb), dim3(256), 0, S->stream, S->n, S->m, S->st.warm_blend, S->wx, S->ws,
                       S->wz, S->dD, S->dE, S->cscale, S->x, S->s, S->z);
    HC_LAUNCH_CHECK();
    S->tau = S->kappa = 1.0;
  }
  S->status = 0;
  S->kiter = 0;
}

// keeps a solved iterate for the next warm start
void end_solve(hc_solver* S) {
  if (!S->st.warm_start || S->status != HC_STATUS_SOLVED) return;
  const int64_t L = std::max(S->n, S->m);
  const int nb = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div(L, 256)), 65535);
  hipLaunchKernelGGL(k_warm_store, dim3(nb), dim3(256), 0, S->stream, S->n, S->m, S->x, S->s, S->z, S->dD, S->dE,
                     1.0 / (S->cscale * S->tau), 1.0 / S->tau, S->wx, S->ws, S->wz);
  HC_LAUNCH_CHECK();
  S->have_warm = true;
}

// one pass of the loop body of Algorithm 1 (residuals, termination tests,
// one iteration); true when the solve has ended
bool step_solve(hc_solver* S) {
  const int k = S->kiter;
  const Resid R = residuals(S);
  S->xPx_cache = R.xPx;
  int status = check(S, R);
  S->info.mu = (R.sz + S->kappa * S->tau) / (double)(S->nu + 1);
  if (S->st.verbose)
    std::printf("%3d gp=%+.8e gd=%+.8e rp=%.2e rd=%.2e mu=%.2e tau=%.3e\n", k, S->info.obj_primal, S->info.obj_dual,
                S->info.res_primal, S->info.res_dual, S->info.mu, S->tau);
  bool done = false;
  if (status) {
    S->status = status;
    done = true;
  } else if (k == S->st.max_iter) {
    S->status = HC_STATUS_MAX_ITER;
    done = true;
  } else {
    status = iterate(S, R);
    S->info.iterations++;
    if (status) {
      S->status = status;
      const Resid R2 = residuals(S);
      check(S, R2);
      done = true;
    }
  }
  S->kiter++;
  S->info.status = S->status;
  return done;
}

void run_solve(hc_solver* S) {
  begin_solve(S);
  while (!step_solve(S)) {
  }
  end_solve(S);
}

// every device allocation of a solver, in order (dry run: byte count only)
void alloc_all(hc_solver* S, Buf& buf, hipStream_t st) {
  const int64_t n = S->n, m = S->m;
  S->dA = upload_csr(buf, S->A, st);
  S->dAt = upload_csr(buf, S->At, st);
  S->dP = upload_csr(buf, S->P, st);
  {   // real dense rows, then the rows the large second-order cones fill
    const size_t rows = std::max<size_t>(S->drows.size(), (size_t)(S->K1 + S->K2));
    S->dAd = buf.take<double>(std::max<size_t>(1, rows * (size_t)S->nt));
    if (!buf.dry && !S->Ad.empty())
      HC_HIP(hipMemcpyAsync(S->dAd, S->Ad.data(), S->Ad.size() * sizeof(double), hipMemcpyHostToDevice, st));
  }
  S->dBd = buf.take<double>(std::max<size_t>(1, (size_t)(S->K1 + S->K2) * (size_t)S->nt));
  S->dDrT = buf.take<double>(std::max<size_t>(
      1, (size_t)dense_rows_t_parts((int)S->drows.size()) * (size_t)(S->leaves ? S->nt : S->n)));
  S->ddrows = upload(buf, S->drows, st);
  S->ddmidx = upload(buf, S->dmidx_all, st);
  S->dls_cone = upload(buf, S->ls_cone, st);
  S->dls_col = upload(buf, S->ls_col, st);
  S->dls_dst = upload(buf, S->ls_dst, st);
  S->dq = upload(buf, S->q, st);
  S->db = upload(buf, S->b, st);
  S->dD = upload(buf, S->D, st);
  S->dE = upload(buf, S->E, st);
  S->dperm = upload(buf, S->perm, st);
  S->dalpha = upload(buf, S->alpha_pow, st);
  {
    GroupPlan& gp = S->gplan;
    gp.ng = S->ga_ng;
    gp.rows_off = upload(buf, S->ga_rows_off, st);
    gp.u_off = upload(buf, S->ga_u_off, st);
    gp.m_off = upload(buf, S->ga_m_off, st);
    gp.t_off = upload(buf, S->ga_t_off, st);
    gp.gm = upload(buf, S->ga_gm, st);
    gp.rows = upload(buf, S->ga_rows, st);
    gp.u = upload(buf, S->ga_u, st);
    gp.c_ptr = upload(buf, S->ga_c_ptr, st);
    gp.c_b = upload(buf, S->ga_c_b, st);
    gp.c_k = upload(buf, S->ga_c_k, st);
    gp.rgrp = upload(buf, S->ga_rgrp, st);
    gp.rloc = upload(buf, S->ga_rloc, st);
    gp.e_t = upload(buf, S->ga_e_t, st);
    gp.e_u = upload(buf, S->ga_e_u, st);
    gp.e_s = upload(buf, S->ga_e_s, st);
    gp.T = buf.take<double>(S->ga_t_total + 1);
  }
  S->dtra = upload(buf, S->tra, st);
  S->dtrb = upload(buf, S->trb, st);
  S->dtm = upload(buf, S->tm, st);
  S->dstate = buf.take<double>(S->stotal + 1);
  S->dmval = buf.take<double>(S->mtotal + 1);
  S->dhdiag = buf.take<double>(m);
  const int64_t nt = S->nt, ntp = S->ld;   // the tail is factored padded to ld
  S->dS = buf.take<double>((size_t)S->ld * ntp);
  S->dLinv = buf.take<double>(linv_elems(ntp));
  S->dX256 = buf.take<double>(inv256_elems(ntp));
  S->dXT256 = buf.take<double>(inv256_elems(ntp));
  if (S->mixed) {
    S->dS32 = buf.take<float>((size_t)S->ld * ntp);
    S->dLinv32 = buf.take<float>(linv_elems(ntp));
    S->dX256f = buf.take<float>(inv256_elems(ntp));
    S->dXT256f = buf.take<float>(inv256_elems(ntp));
    S->sb32 = buf.take<float>(2 * nt);   // two right-hand sides (kkt_solve_pair)
    S->sy32 = buf.take<float>(2 * nt);
    S->sx32 = buf.take<float>(2 * nt);
  }
  // column map of the two-level split
  ColMap& cm = S->cm;
  cm.nleaf = (int64_t)S->leaf_size.size();
  cm.nt = nt;
  cm.ldt = S->ld;
  cm.ST = S->dS;
  cm.leaf = upload(buf, S->col_leaf, st);
  cm.loc = upload(buf, S->col_loc, st);
  cm.tcols = upload(buf, S->tail_cols, st);
  cm.lsize = upload(buf, S->leaf_size, st);
  cm.lval_off = upload(buf, S->leaf_lval_off, st);
  cm.lcol_off = upload(buf, S->leaf_lcol_off, st);
  cm.lcols = upload(buf, S->leaf_cols, st);
  cm.ccnt = upload(buf, S->leaf_ccnt, st);
  cm.clist_off = upload(buf, S->leaf_clist_off, st);
  cm.clist = upload(buf, S->leaf_clist, st);
  cm.cval_off = upload(buf, S->leaf_cval_off, st);
  cm.nsmall = (int64_t)S->leaf_small.size();
  cm.nlarge = (int64_t)S->leaf_large.size();
  cm.small = upload(buf, S->leaf_small, st);
  cm.large = upload(buf, S->leaf_large, st);
  cm.tc_ptr = upload(buf, S->tc_ptr, st);
  {   // threads per tail index: enough for the mean number of W entries
    const double mean = nt > 0 && !S->tc_ptr.empty() ? (double)S->tc_ptr[nt] / (double)nt : 0.0;
    cm.tail_threads = mean >= 1024 ? 1024 : mean >= 128 ? 256 : 64;
  }
  cm.te_cv = upload(buf, S->te_cv, st);
  cm.te_y = upload(buf, S->te_y, st);
  if (S->ordered) {
    auto dev = [&](OrderedSum& o, const std::vector<int64_t>& ptr, const std::vector<int64_t>& dst, int64_t nshort,
                   const std::vector<int32_t>* pm, const std::vector<int32_t>& pp, const std::vector<int32_t>* pq) {
      o.nd = (int64_t)dst.size();
      o.nshort = nshort;
      o.ptr = upload(buf, ptr, st);
      o.dst = upload(buf, dst, st);
      o.pm = pm ? upload(buf, *pm, st) : nullptr;
      o.pp = upload(buf, pp, st);
      o.pq = pq ? upload(buf, *pq, st) : nullptr;
    };
    dev(S->opair, S->op_ptr, S->op_dst, S->op_nshort, &S->op_pm, S->op_pp, &S->op_pq);
    dev(S->oleaf, S->ol_ptr, S->ol_dst, S->ol_nshort, nullptr, S->ol_pp, nullptr);
    cm.lp_off = upload(buf, S->leaf_lp_off, st);
    cm.lslot = S->lpair_total > 0 ? buf.take<double>(S->lpair_total) : nullptr;
  } else {
    S->opair = OrderedSum{};
    S->oleaf = OrderedSum{};
    cm.lp_off = nullptr;
    cm.lslot = nullptr;
  }
  cm.lval = buf.take<double>(S->lval_total + 1);
  cm.cval = buf.take<double>(S->cval_total + 1);
  cm.sink = buf.take<double>(1);
  S->uT = buf.take<double>(nt);
  S->xT = buf.take<double>(nt);
  S->uTb = buf.take<double>(nt);
  S->xTb = buf.take<double>(nt);
  S->dhits = buf.take<unsigned long long>(1);
  S->dpd = buf.take<int>(2);
  S->dscal = buf.take<double>(8);
  S->npart = 2 * 512 * MAX_RED_OPS;   // two reductions read back together
  for (const Segment& sg : S->segs) {
    SegDev d{};
    d.kind = sg.kind;
    d.dim = sg.dim;
    d.k = sg.k;
    d.count = sg.count;
    S->npart += cone_blocks(d) + 2048;   // a step or max kernel writes at most this many
  }
  {
    int64_t mw = 1;
    for (const Segment& sg : S->segs) {
      SegDev d{};
      d.kind = sg.kind;
      d.dim = sg.dim;
      d.k = sg.k;
      d.count = sg.count;
      mw = std::max(mw, cone_mblock_work(d));
    }
    S->dmwork = buf.take<double>(mw);
  }
  S->dpe_rp = upload(buf, S->pe_rp, st);
  S->dpe_e = upload(buf, S->pe_e, st);
  S->dpe_p = upload(buf, S->pe_p, st);
  S->dT = buf.take<double>(std::max<size_t>(1, (size_t)S->pe_rows * (size_t)S->n));
  S->pcols.cu_off = upload(buf, S->pc_cu_off, st);
  S->pcols.cu_ptr = upload(buf, S->pc_cu_ptr, st);
  S->pcols.cu_col = upload(buf, S->pc_cu_col, st);
  S->pcols.cu_b = upload(buf, S->pc_cu_b, st);
  S->pcols.cu_p = upload(buf, S->pc_cu_p, st);
  // T's columns outside a cone's own stay zero from here on
  if (!buf.dry && S->pe_rows > 0) vfill(S->pe_rows * S->n, 0.0, S->dT, st);
  S->dpart = buf.take<double>(S->npart);
  S->dmask = buf.take<unsigned long long>(S->npart);
  const int64_t L = std::max(n, m);
  double** vecs[] = {&S->x, &S->s, &S->z, &S->Px, &S->Ax, &S->Atz, &S->rdv, &S->rpv, &S->x2, &S->z2, &S->x1,
                     &S->z1, &S->dx, &S->dz, &S->dsv, &S->dsrhs, &S->dxa, &S->dza, &S->dsa, &S->r1, &S->r2,
                     &S->irx, &S->irz, &S->irxn, &S->irzn, &S->irbx, &S->irbz, &S->irrx, &S->irrz, &S->kx};
  for (double** v : vecs) *v = buf.take<double>(L);
  S->kz = buf.take<double>(L);
  S->t1 = buf.take<double>(L);
  S->t2 = buf.take<double>(L);
  S->u1 = buf.take<double>(L);
  S->w1 = buf.take<double>(L);
  S->sb = buf.take<double>(2 * nt);
  S->sy = buf.take<double>(2 * nt);
  S->sx = buf.take<double>(2 * nt);
  // the second system of kkt_solve_pair
  double** vecs2[] = {&S->jrx, &S->jrz, &S->jrxn, &S->jrzn, &S->jrbx, &S->jrbz, &S->jrrx, &S->jrrz,
                      &S->jkx, &S->jkz, &S->u1b, &S->r1c};
  for (double** v : vecs2) *v = buf.take<double>(L);
  S->wx = buf.take<double>(n);
  S->ws = buf.take<double>(m);
  S->wz = buf.take<double>(m);
}

size_t workspace_bytes(const hc_solver* S) {
  if (S->bound) return S->mem_bytes;   // the dry run below would overwrite the device pointers
  Buf b;
  b.dry = true;
  alloc_all(const_cast<hc_solver*>(S), b, nullptr);
  return b.used + 4096;
}

// pinned read-back staging: the partials, then the step masks (npart is set
// by alloc_all, real or dry)
size_t stage_bytes_of(const hc_solver* S) {
  return (size_t)S->npart * (sizeof(double) + sizeof(unsigned long long));
}

// before bind only: the dry run that sets npart also sets every device
// pointer of the handle (to null)
size_t host_stage_bytes(const hc_solver* S) {
  if (!S->bound) workspace_bytes(S);
  return stage_bytes_of(S);
}

void bind(hc_solver* S, const hc_device* dev) {
  S->device = dev ? dev->device : 0;
  HC_HIP(hipSetDevice(S->device));
  S->stream = dev ? (hipStream_t)dev->stream : nullptr;
  const size_t need = workspace_bytes(S);
  Buf buf;
  if (dev && dev->arena) {
    if (dev->arena_bytes < need)
      fail(HC_ERR_OOM, "arena too small: need " + std::to_string(need) + " bytes");
    buf.base = (char*)dev->arena;
    buf.size = dev->arena_bytes;
  } else {
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) fail(HC_ERR_OOM, "hipMalloc of " + std::to_string(need) + " bytes failed");
    S->own_mem = true;
    S->mem = p;
    buf.base = (char*)p;
    buf.size = need;
  }
  S->mem_bytes = need;
  hipStream_t st = S->stream;
  alloc_all(S, buf, st);
  if (dev && dev->host_stage && dev->host_stage_bytes >= stage_bytes_of(S)) {   // npart from the allocation above
    S->hpart = (double*)dev->host_stage;
    S->hmask = (unsigned long long*)(S->hpart + S->npart);
  } else {
    HC_HIP(hipHostMalloc((void**)&S->hpart, S->npart * sizeof(double), hipHostMallocDefault));
    HC_HIP(hipHostMalloc((void**)&S->hmask, S->npart * sizeof(unsigned long long), hipHostMallocDefault));
    S->own_stage = true;
  }
  vfill(1, 0.0, (double*)S->dhits, st);
  if (S->K1 + S->K2 > 0) {   // zero padding rows of the dense-row operand, zero rank-2 rows
    vfill((S->K1 + S->K2) * S->nt, 0.0, S->dBd, st);
    const size_t real = S->drows.size() * (size_t)S->nt;
    const size_t rows = std::max<size_t>(S->drows.size(), (size_t)(S->K1 + S->K2));
    if (rows * S->nt > real)
      vfill((int64_t)(rows * S->nt - real), 0.0, S->dAd + real, st);
  }
  // segment views
  int pow_off = 0;
  S->sdev.clear();
  for (const Segment& g : S->segs) {
    SegDev d;
    d.kind = g.kind;
    d.dim = g.dim;
    d.k = g.k;
    d.base = g.base;
    d.count = g.count;
    d.state = S->dstate + g.state;
    d.mblk = S->dmval + g.moff;
    d.alpha = (g.kind == HC_CONE_POW) ? S->dalpha + pow_off : nullptr;
    if (g.kind == HC_CONE_POW) pow_off += (int)g.count;
    S->sdev.push_back(d);
  }
  S->prof.reset(new Prof());
  S->cprof.reset(new Prof());
  S->bound = true;
  HC_HIP(hipStreamSynchronize(st));
}

void record(hc_solver* S, const Error& e) { S->last_error = e.msg; }

}  // namespace

// ===========================================================================
// plan of a problem for the wave-per-problem engine (hc_wave.hip)
// ===========================================================================
namespace hc {

namespace {

// reverse Cuthill-McKee order of a symmetric graph (adjacency lists without
// self loops): breadth-first from a pseudo-peripheral vertex of each
// component, neighbours by increasing degree, the whole order reversed
std::vector<int32_t> rcm_order(const std::vector<std::vector<int32_t>>& adj) {
  const int32_t n = (int32_t)adj.size();
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int32_t> level(n, -1);
  auto bfs_last = [&](int32_t s, int32_t* depth) {   // farthest vertex of s's component (least degree at that level)
    std::vector<int32_t> q{s};
    for (int32_t v : q) level[v] = -1;
    level[s] = 0;
    size_t h = 0;
    int32_t best = s;
    while (h < q.size()) {
      const int32_t v = q[h++];
      for (int32_t u : adj[v])
        if (level[u] < 0) {
          level[u] = level[v] + 1;
          q.push_back(u);
        }
    }
    int32_t maxl = 0;
    for (int32_t v : q) maxl = std::max(maxl, level[v]);
    for (int32_t v : q)
      if (level[v] == maxl && (best == s || adj[v].size() < adj[best].size())) best = v;
    for (int32_t v : q) level[v] = -1;
    *depth = maxl;
    return best;
  };
  for (int32_t start = 0; start < n; ++start) {
    if (seen[start]) continue;
    // pseudo-peripheral start: repeat the farthest-vertex search while the depth grows
    int32_t r = start, depth = 0;
    for (int it = 0; it < 3; ++it) {
      int32_t d2 = 0;
      const int32_t far = bfs_last(r, &d2);
      if (it > 0 && d2 <= depth) break;
      depth = d2;
      r = far;
    }
    std::vector<int32_t> q{r};
    seen[r] = 1;
    size_t h = 0;
    std::vector<int32_t> nb;
    while (h < q.size()) {
      const int32_t v = q[h++];
      nb.clear();
      for (int32_t u : adj[v])
        if (!seen[u]) {
          seen[u] = 1;
          nb.push_back(u);
        }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return adj[a].size() != adj[b].size() ? adj[a].size() < adj[b].size() : a < b;
      });
      for (int32_t u : nb) q.push_back(u);
    }
    for (int32_t v : q) order.push_back(v);
  }
  std::reverse(order.begin(), order.end());
  return order;
}

}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

bool wave_plan(const hc_solver* S, WavePlan* out, std::string* why) {
  auto no = [&](const std::string& m) {
    if (why) *why = m;
    return false;
  };
  if (S->has_nonsym) return no("exponential or power cones");
  if (!S->drows.empty() || S->K1 + S->K2 > 0) return no("dense rows or second-order cones above 16 rows");
  if (S->n < 1 || S->m < 1 || S->n > (1 << 24) || S->m > (1 << 24)) return no("size outside the engine's range");
  WavePlan& P = *out;
  P = WavePlan{};
  const int32_t n = (int32_t)S->n, m = (int32_t)S->m;
  P.n = n;
  P.m = m;
  // engine rows: zero rows, nonneg rows, then second-order cones one after another
  std::vector<int32_t> wrow_of(m, -1), srow_of;   // S-internal row -> engine row, and back
  srow_of.reserve(m);
  std::vector<int32_t> soc_dims;
  for (const Segment& g : S->segs) {
    if (g.kind == HC_CONE_PSD) return no("PSD cones");
    if (g.kind == HC_CONE_SOC && g.dim > SOC_DMAX) return no("second-order cones above 16 rows");
  }
  for (int pass = 0; pass < 3; ++pass)
    for (const Segment& g : S->segs) {
      const int kind = pass == 0 ? HC_CONE_ZERO : pass == 1 ? HC_CONE_NONNEG : HC_CONE_SOC;
      if (g.kind != kind) continue;
      if (kind != HC_CONE_SOC) {
        for (int64_t i = 0; i < g.count; ++i) srow_of.push_back((int32_t)(g.base + i));
        if (kind == HC_CONE_ZERO) P.nz += (int32_t)g.count;
        else P.nn += (int32_t)g.count;
      } else {
        for (int64_t i = 0; i < g.count; ++i) {
          for (int j = 0; j < g.dim; ++j) srow_of.push_back((int32_t)(g.base + (int64_t)j * g.count + i));
          soc_dims.push_back(g.dim);
        }
      }
    }
  if ((int32_t)srow_of.size() != m) return no("row bookkeeping");
  for (int32_t r = 0; r < m; ++r) wrow_of[srow_of[r]] = r;
  P.nsoc = (int32_t)soc_dims.size();
  P.soc_off.assign(P.nsoc + 1, 0);
  P.soc_moff.assign(P.nsoc, 0);
  P.mtot = P.nz + P.nn;
  for (int32_t c = 0; c < P.nsoc; ++c) {
    P.soc_off[c + 1] = P.soc_off[c] + soc_dims[c];
    P.soc_moff[c] = P.mtot;
    P.mtot += soc_dims[c] * soc_dims[c];
  }
  // blocks of S: each zero/nonneg row, each cone; their column sets are cliques of S
  const int32_t nblk = P.nz + P.nn + P.nsoc;
  auto block_rows = [&](int32_t bk, int32_t* r0, int32_t* r1) {
    if (bk < P.nz + P.nn) {
      *r0 = bk;
      *r1 = bk + 1;
    } else {
      const int32_t c = bk - P.nz - P.nn;
      *r0 = P.nz + P.nn + P.soc_off[c];
      *r1 = P.nz + P.nn + P.soc_off[c + 1];
    }
  };
  const HostCsr& A = S->A;   // S-internal rows
  // graph of S as adjacency lists: the cliques of the blocks and P's pattern,
  // through the column -> block incidence (duplicates removed by a stamp)
  std::vector<std::vector<int32_t>> adj(n);
  {
    std::vector<int32_t> brp(nblk + 1, 0), bci;   // block -> columns
    bci.reserve(A.ci.size());
    for (int32_t bk = 0; bk < nblk; ++bk) {
      int32_t r0, r1;
      block_rows(bk, &r0, &r1);
      const size_t first = bci.size();
      for (int32_t r = r0; r < r1; ++r) {
        const int32_t sr = srow_of[r];
        for (int32_t k = A.rp[sr]; k < A.rp[sr + 1]; ++k) bci.push_back(A.ci[k]);
      }
      if (r1 - r0 > 1) {
        std::sort(bci.begin() + first, bci.end());
        bci.erase(std::unique(bci.begin() + first, bci.end()), bci.end());
      }
      if (bci.size() - first > (size_t)2 * WAVE_WMAX + 2)
        return no("a cone or row couples more columns than the band allows");
      brp[bk + 1] = (int32_t)bci.size();
    }
    std::vector<int32_t> crp(n + 1, 0), cbk(bci.size());   // column -> blocks
    for (int32_t c : bci) crp[c + 1]++;
    for (int32_t i = 0; i < n; ++i) crp[i + 1] += crp[i];
    {
      std::vector<int32_t> f(crp.begin(), crp.end() - 1);
      for (int32_t bk = 0; bk < nblk; ++bk)
        for (int32_t k = brp[bk]; k < brp[bk + 1]; ++k) cbk[f[bci[k]]++] = bk;
    }
    std::vector<int32_t> stamp(n, -1);
    for (int32_t a = 0; a < n; ++a) {
      stamp[a] = a;
      std::vector<int32_t>& nb = adj[a];
      for (int32_t k = crp[a]; k < crp[a + 1]; ++k) {
        const int32_t bk = cbk[k];
        for (int32_t l = brp[bk]; l < brp[bk + 1]; ++l)
          if (stamp[bci[l]] != a) {
            stamp[bci[l]] = a;
            nb.push_back(bci[l]);
          }
      }
      for (int32_t k = S->P.rp[a]; k < S->P.rp[a + 1]; ++k)
        if (stamp[S->P.ci[k]] != a) {
          stamp[S->P.ci[k]] = a;
          nb.push_back(S->P.ci[k]);
        }
    }
  }
  const std::vector<int32_t> order = rcm_order(adj);   // band position -> column
  std::vector<int32_t> pos(n);
  for (int32_t i = 0; i < n; ++i) pos[order[i]] = i;
  int32_t w = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t u : adj[i]) w = std::max(w, std::abs(pos[i] - pos[u]));
  if (w > WAVE_WMAX) return no("band half-width " + std::to_string(w) + " above " + std::to_string(WAVE_WMAX));
  P.w = w;
  const int32_t W = w + 1;
  P.colperm = order;
  P.rowperm.resize(m);
  for (int32_t r = 0; r < m; ++r) P.rowperm[r] = (int32_t)S->perm[srow_of[r]];
  // A in engine rows and band columns, and its transpose
  P.Arp.assign(m + 1, 0);
  for (int32_t r = 0; r < m; ++r) {
    const int32_t sr = srow_of[r];
    P.Arp[r + 1] = P.Arp[r] + (A.rp[sr + 1] - A.rp[sr]);
  }
  P.Aci.resize(P.Arp[m]);
  P.Av.resize(P.Arp[m]);
  {
    std::vector<std::pair<int32_t, double>> ent;
    for (int32_t r = 0; r < m; ++r) {
      const int32_t sr = srow_of[r];
      ent.clear();
      for (int32_t k = A.rp[sr]; k < A.rp[sr + 1]; ++k) ent.emplace_back(pos[A.ci[k]], A.v[k]);
      std::sort(ent.begin(), ent.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      int32_t o = P.Arp[r];
      for (const auto& e : ent) {
        P.Aci[o] = e.first;
        P.Av[o++] = e.second;
      }
    }
  }
  P.Atrp.assign(n + 1, 0);
  for (int32_t k = 0; k < P.Arp[m]; ++k) P.Atrp[P.Aci[k] + 1]++;
  for (int32_t j = 0; j < n; ++j) P.Atrp[j + 1] += P.Atrp[j];
  P.Atci.resize(P.Arp[m]);
  P.Atv.resize(P.Arp[m]);
  {
    std::vector<int32_t> fill(P.Atrp.begin(), P.Atrp.end() - 1);
    for (int32_t r = 0; r < m; ++r)
      for (int32_t k = P.Arp[r]; k < P.Arp[r + 1]; ++k) {
        const int32_t o = fill[P.Aci[k]]++;
        P.Atci[o] = r;
        P.Atv[o] = P.Av[k];
      }
  }
  // P (full, both triangles) in band columns, and its lower band
  P.Prp.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) P.Prp[i + 1] = P.Prp[i] + (S->P.rp[order[i] + 1] - S->P.rp[order[i]]);
  P.Pci.resize(P.Prp[n]);
  P.Pv.resize(P.Prp[n]);
  P.Pband.assign((size_t)n * W, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    int32_t o = P.Prp[i];
    for (int32_t k = S->P.rp[order[i]]; k < S->P.rp[order[i] + 1]; ++k, ++o) {
      const int32_t j = pos[S->P.ci[k]];
      P.Pci[o] = j;
      P.Pv[o] = S->P.v[k];
      if (i >= j) P.Pband[(size_t)j * W + (i - j)] += S->P.v[k];
    }
  }
  P.q.resize(n);
  P.D.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    P.q[i] = S->q[order[i]];
    P.D[i] = S->D[order[i]];
  }
  P.b.resize(m);
  P.E.resize(m);
  for (int32_t r = 0; r < m; ++r) {
    P.b[r] = S->b[srow_of[r]];
    P.E[r] = S->E[srow_of[r]];
  }
  // A'MA: every zero row has the same M = 1/delta, so their products are
  // summed per band entry here (in row order) into Zband; the nonneg rows' and
  // cones' products A_pi A_qj M_pq (p = q for a nonneg row) are listed per
  // band entry, only for the entries that have any (te), in block order
  // within an entry (a stable counting sort)
  {
    struct Term {
      int32_t e, mi;
      double c;
    };
    const size_t ne = (size_t)n * W;
    P.Zband.assign(ne, 0.0);
    std::vector<Term> terms;
    std::vector<int32_t> cnt(ne, 0);
    for (int32_t bk = 0; bk < nblk; ++bk) {
      int32_t r0, r1;
      block_rows(bk, &r0, &r1);
      if (bk < P.nz + P.nn) {   // one row; its columns ascend, so kb <= ka gives i >= j
        const bool zero = bk < P.nz;
        for (int32_t ka = P.Arp[r0]; ka < P.Arp[r0 + 1]; ++ka) {
          const int32_t i = P.Aci[ka];
          const double va = P.Av[ka];
          for (int32_t kb = P.Arp[r0]; kb <= ka; ++kb) {
            const int32_t e = P.Aci[kb] * W + (i - P.Aci[kb]);
            if (zero) {
              P.Zband[e] += va * P.Av[kb];
            } else {
              terms.push_back(Term{e, bk, va * P.Av[kb]});
              cnt[e]++;
            }
          }
        }
        continue;
      }
      const int32_t d = r1 - r0;
      const int32_t mo = P.soc_moff[bk - P.nz - P.nn];
      for (int32_t p = r0; p < r1; ++p)
        for (int32_t q2 = r0; q2 < r1; ++q2)
          for (int32_t ka = P.Arp[p]; ka < P.Arp[p + 1]; ++ka)
            for (int32_t kb = P.Arp[q2]; kb < P.Arp[q2 + 1]; ++kb) {
              const int32_t i = P.Aci[ka], j = P.Aci[kb];
              if (i < j) continue;
              const int32_t e = j * W + (i - j);
              terms.push_back(Term{e, mo + (p - r0) * d + (q2 - r0), P.Av[ka] * P.Av[kb]});
              cnt[e]++;
            }
    }
    std::vector<int32_t> slot(ne, -1);
    P.te.clear();
    P.trp.assign(1, 0);
    for (size_t e = 0; e < ne; ++e)
      if (cnt[e]) {
        slot[e] = (int32_t)P.te.size();
        P.te.push_back((int32_t)e);
        P.trp.push_back(P.trp.back() + cnt[e]);
      }
    P.tm.resize(terms.size());
    P.tc.resize(terms.size());
    std::vector<int32_t> fill(P.trp.begin(), P.trp.end() - 1);
    for (const Term& tt : terms) {
      const int32_t o = fill[slot[tt.e]]++;
      P.tm[o] = tt.mi;
      P.tc[o] = tt.c;
    }
  }
  P.cscale = S->cscale;
  P.bnorm = S->bnorm_user;
  P.qnorm = S->qnorm_user;
  P.maxPdiag = S->maxPdiag;
  P.nu = S->nu;
  P.st = S->st;
  P.mixed = S->mixed;
  return true;
}

}  // namespace hc

// ===========================================================================
// step-wise driving (continuous-batching server)
// ===========================================================================
namespace hc {

int32_t solver_begin(hc_solver* S) {
  if (!S || !S->bound) return HC_ERR_STATE;
  try {
    HC_HIP(hipSetDevice(S->device));
    S->t_begin = now_ms();
    begin_solve(S);
  } catch (const Error& e) {
    record(S, e);
    return e.code;
  }
  return HC_OK;
}

int32_t solver_step(hc_solver* S, int* done) {
  if (!S || !S->bound || !done) return HC_ERR_STATE;
  try {
    HC_HIP(hipSetDevice(S->device));
    *done = step_solve(S) ? 1 : 0;
  } catch (const Error& e) {
    record(S, e);
    *done = 1;
    return e.code;
  }
  return HC_OK;
}

int32_t solver_finish(hc_solver* S) {
  if (!S || !S->bound) return HC_ERR_STATE;
  try {
    HC_HIP(hipSetDevice(S->device));
    HC_HIP(hipStreamSynchronize(S->stream));
    S->info.solve_ms = now_ms() - S->t_begin;
    unsigned long long h = 0;
    HC_HIP(hipMemcpy(&h, S->dhits, sizeof(h), hipMemcpyDeviceToHost));
    S->info.pivot_guard_hits = (int64_t)h;
  } catch (const Error& e) {
    record(S, e);
    return e.code;
  }
  return HC_OK;
}

}  // namespace hc

// ===========================================================================
// allocation-free solve (hc_solve_noalloc): the workspace is a static device
// array (one copy per device, its address taken once per device), the
// read-back staging a static host block, and the dense factorisation issues
// the look-ahead schedule's launches on the caller's stream alone
// ===========================================================================
static __device__ __align__(256) unsigned char scratch[HC_NOALLOC_BYTES];

namespace {

constexpr size_t NOALLOC_STAGE_BYTES = (size_t)4 << 20;
alignas(256) unsigned char g_noalloc_stage[NOALLOC_STAGE_BYTES];
std::mutex g_noalloc_mu;                 // one call at a time in the process
constexpr int NOALLOC_MAX_DEVICES = 64;
void* g_scratch[NOALLOC_MAX_DEVICES];    // device -> address of its copy of `scratch`

// the handle leaves the static workspace: unbound, nothing of it kept
void noalloc_release(hc_solver* S) {
  S->bound = false;
  S->noalloc = false;
  S->hpart = nullptr;
  S->hmask = nullptr;
  S->own_stage = false;
  S->have_warm = false;
  S->mem_bytes = 0;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
// the iterate in the user's coordinates: x = D x~ / t, s[perm] = s~ / E / t,
// z[perm] = E z~ / (c t) (the host form's operations, so both agree bit for bit)
__global__ void k_user_solution(int64_t n, int64_t m, const double* __restrict__ xi, const double* __restrict__ si,
                                const double* __restrict__ zi, const double* __restrict__ D,
                                const double* __restrict__ E, const int64_t* __restrict__ perm, double c,
                                double t, double* __restrict__ x, double* __restrict__ s, double* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n > m ? n : m);
       i += (int64_t)gridDim.x * blockDim.x) {
    if (x && i < n) x[i] = D[i] * xi[i] / t;
    if (i < m) {
      const int64_t u = perm[i];
      if (s) s[u] = si[i] / E[i] / t;
      if (z) z[u] = E[i] * zi[i] / (c * t);
    }
  }
}

extern "C" {

int32_t hc_settings_default(hc_settings* o) {
  if (!o) return HC_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->eps_feas = 1e-8;
  o->eps_inf = 1e-8;
  o->max_iter = 200;
  o->precision = HC_PRECISION_FP64;
  o->static_reg = 0.0;
  o->dyn_reg = -1.0;
  o->ir_abstol = 1e-12;
  o->ir_reltol = 1e-12;
  o->ir_max = 10;
  o->beta = 1e-6;
  o->backtrack = 0.8;
  o->step_fraction = 0.99;
  o->equilibrate = 1;
  o->equil_iters = 10;
  o->force_dual_scaling = 0;
  o->verbose = 0;
  o->profile = 0;
  o->leaf_blocks = 1;
  o->warm_start = 0;
  o->warm_blend = 0.02;
  o->ir_mu_frac = -1.0;
  return HC_OK;
}

int32_t hc_setup(hc_solver** out, const hc_problem* prob, const hc_settings* settings) {
  if (!out) return HC_ERR_INVALID_ARG;
  *out = nullptr;
  hc_solver* S = new (std::nothrow) hc_solver();
  if (!S) return HC_ERR_OOM;
  try {
    if (settings) S->st = *settings;
    else hc_settings_default(&S->st);
    const double t0 = now_ms();
    validate(prob);
    setup_host(S, prob);
    keep_user_data(S, prob);
    S->info.setup_ms = now_ms() - t0;
    S->info.n_ordered = S->nt;
    S->info.n_leaves = (int64_t)S->leaf_size.size();
    S->info.leaf_columns = S->n - S->nt;
    S->info.sym_split_columns = S->sym_split_columns;
    S->info.sym_supernodes = S->sym_supernodes;
    S->info.sym_levels = S->sym_levels;
    S->info.sym_nnz_l = S->sym_nnz_l;
    S->info.psd_gathered_rows = S->pe_rows;
    S->info.factor_flops = envelope_cholesky_flops(S->nt, S->tail_last.data()) + S->leaf_flops;
  } catch (const Error& e) {
    g_last_error = e.msg;
    delete S;
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    delete S;
    return HC_ERR_INVALID_ARG;
  }
  *out = S;
  return HC_OK;
}

int32_t hc_workspace_bytes(const hc_solver* S, size_t* bytes) {
  if (!S || !bytes) return HC_ERR_INVALID_ARG;
  *bytes = workspace_bytes(S);
  return HC_OK;
}

int32_t hc_host_stage_bytes(const hc_solver* S, size_t* bytes) {
  if (!S || !bytes) return HC_ERR_INVALID_ARG;
  *bytes = host_stage_bytes(S);
  return HC_OK;
}

int32_t hc_bind(hc_solver* S, const hc_device* dev) {
  if (!S) return HC_ERR_INVALID_ARG;
  if (S->bound) return HC_ERR_STATE;
  try {
    const double t0 = now_ms();
    bind(S, dev);
    S->info.setup_ms += now_ms() - t0;
  } catch (const Error& e) {
    record(S, e);
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

int32_t hc_solve(hc_solver* S) {
  if (!S) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  try {
    HC_HIP(hipSetDevice(S->device));
    const double t0 = now_ms();
    run_solve(S);
    HC_HIP(hipStreamSynchronize(S->stream));
    S->info.solve_ms = now_ms() - t0;
    unsigned long long h = 0;
    HC_HIP(hipMemcpy(&h, S->dhits, sizeof(h), hipMemcpyDeviceToHost));
    S->info.pivot_guard_hits = (int64_t)h;
  } catch (const Error& e) {
    record(S, e);
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

int32_t hc_solve_noalloc(hc_solver* S, void* stream, int32_t device, double* x, double* sv, double* z,
                         hc_info* info) {
  if (!S || device < 0 || device >= NOALLOC_MAX_DEVICES) return HC_ERR_INVALID_ARG;
  if (S->bound) return HC_ERR_STATE;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  const int32_t profile = S->st.profile;
  try {
    const size_t need = workspace_bytes(S), stage = host_stage_bytes(S);
    if (need > HC_NOALLOC_BYTES || stage > NOALLOC_STAGE_BYTES)
      fail(HC_ERR_TOO_LARGE, "hc_solve_noalloc: the problem needs " + std::to_string(need) +
                                 " bytes of device workspace (at most " + std::to_string((size_t)HC_NOALLOC_BYTES) +
                                 ") and " + std::to_string(stage) + " bytes of read-back staging (at most " +
                                 std::to_string(NOALLOC_STAGE_BYTES) + ")");
    HC_HIP(hipSetDevice(device));
    if (!g_scratch[device]) {
      void* p = nullptr;
      const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (rc != hipSuccess || !p)
        fail(HC_ERR_DEVICE, std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(rc));
      g_scratch[device] = p;
    }
    hc_device dev{g_scratch[device], (size_t)HC_NOALLOC_BYTES, stream, device, g_noalloc_stage, NOALLOC_STAGE_BYTES};
    S->st.profile = 0;   // no timing events
    S->noalloc = true;
    const double t0 = now_ms();
    bind(S, &dev);
    run_solve(S);
    HC_HIP(hipStreamSynchronize(S->stream));
    S->info.solve_ms = now_ms() - t0;
    unsigned long long h = 0;
    HC_HIP(hipMemcpy(&h, S->dhits, sizeof(h), hipMemcpyDeviceToHost));
    S->info.pivot_guard_hits = (int64_t)h;
    const int32_t rc = hc_get_solution(S, x, sv, z, 0);
    if (rc != HC_OK) fail(rc, g_last_error);
    if (info) *info = S->info;
  } catch (const Error& e) {
    if (S->bound) (void)hipStreamSynchronize(S->stream);
    noalloc_release(S);
    S->st.profile = profile;
    record(S, e);
    g_last_error = e.msg;
    return e.code;
  }
  noalloc_release(S);
  S->st.profile = profile;
  return HC_OK;
}

int32_t hc_get_info(const hc_solver* S, hc_info* out) {
  if (!S || !out) return HC_ERR_INVALID_ARG;
  *out = S->info;
  return HC_OK;
}

int32_t hc_get_solution(const hc_solver* S, double* x, double* sv, double* z, int32_t on_device) {
  if (!S) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  try {
    const int64_t n = S->n, m = S->m;
    const bool cert0 = S->status == HC_STATUS_PRIMAL_INFEASIBLE || S->status == HC_STATUS_DUAL_INFEASIBLE;
    if (on_device) {
      const int64_t L = std::max(n, m);
      const int nb = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div(L, 256)), 65535);
      hipLaunchKernelGGL(k_user_solution, dim3(nb), dim3(256), 0, S->stream, n, m, S->x, S->s, S->z, S->dD, S->dE,
                         S->dperm, S->cscale, cert0 ? 1.0 : S->tau, x, sv, z);
      HC_LAUNCH_CHECK();
      HC_HIP(hipStreamSynchronize(S->stream));
      return HC_OK;
    }
    std::vector<double> hx(n), hs(m), hz(m);
    HC_HIP(hipMemcpy(hx.data(), S->x, n * 8, hipMemcpyDeviceToHost));
    HC_HIP(hipMemcpy(hs.data(), S->s, m * 8, hipMemcpyDeviceToHost));
    HC_HIP(hipMemcpy(hz.data(), S->z, m * 8, hipMemcpyDeviceToHost));
    const bool cert = S->status == HC_STATUS_PRIMAL_INFEASIBLE || S->status == HC_STATUS_DUAL_INFEASIBLE;
    const double t = cert ? 1.0 : S->tau;
    if (x)
      for (int64_t j = 0; j < n; ++j) x[j] = S->D[j] * hx[j] / t;
    for (int64_t r = 0; r < m; ++r) {
      const int64_t u = S->perm[r];
      if (sv) sv[u] = hs[r] / S->E[r] / t;
      if (z) z[u] = S->E[r] * hz[r] / (S->cscale * t);
    }
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

int32_t hc_get_iterate(const hc_solver* S, double* x, double* sv, double* z, double* tau, double* kappa,
                       int64_t* row_of_internal) {
  if (!S) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  try {
    if (x) HC_HIP(hipMemcpy(x, S->x, S->n * 8, hipMemcpyDeviceToHost));
    if (sv) HC_HIP(hipMemcpy(sv, S->s, S->m * 8, hipMemcpyDeviceToHost));
    if (z) HC_HIP(hipMemcpy(z, S->z, S->m * 8, hipMemcpyDeviceToHost));
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  if (tau) *tau = S->tau;
  if (kappa) *kappa = S->kappa;
  if (row_of_internal) std::memcpy(row_of_internal, S->perm.data(), S->m * sizeof(int64_t));
  return HC_OK;
}

int32_t hc_set_iterate(hc_solver* S, const double* x, const double* sv, const double* z, double tau, double kappa) {
  if (!S || !x || !sv || !z) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  if (!(tau > 0) || !(kappa > 0)) return HC_ERR_INVALID_ARG;
  try {
    HC_HIP(hipSetDevice(S->device));
    HC_HIP(hipMemcpy(S->x, x, S->n * 8, hipMemcpyHostToDevice));
    HC_HIP(hipMemcpy(S->s, sv, S->m * 8, hipMemcpyHostToDevice));
    HC_HIP(hipMemcpy(S->z, z, S->m * 8, hipMemcpyHostToDevice));
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  S->tau = tau;
  S->kappa = kappa;
  return HC_OK;
}

int32_t hc_update_data(hc_solver* S, const double* P_val, const double* q, const double* A_val, const double* b) {
  if (!S) return HC_ERR_INVALID_ARG;
  try {
    auto finite = [](const double* v, size_t cnt) {
      for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(v[i])) return false;
      return true;
    };
    const size_t pn = S->uPv.size(), an = S->uAv.size();
    if ((P_val && !finite(P_val, pn)) || (q && !finite(q, S->n)) || (A_val && !finite(A_val, an)) ||
        (b && !finite(b, S->m)))
      fail(HC_ERR_NONFINITE, "hc_update_data: non-finite value");
    if (P_val) std::copy(P_val, P_val + pn, S->uPv.begin());
    if (q) std::copy(q, q + S->n, S->uq.begin());
    if (A_val) std::copy(A_val, A_val + an, S->uAv.begin());
    if (b) std::copy(b, b + S->m, S->ub.begin());
    refresh_values(S);
    if (S->bound) {
      HC_HIP(hipSetDevice(S->device));
      hipStream_t st = S->stream;
      auto put = [&](double* d, const std::vector<double>& h) {
        if (!h.empty()) HC_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
      };
      put(S->dA.val, S->A.v);
      put(S->dAt.val, S->At.v);
      put(S->dP.val, S->P.v);
      put(S->dAd, S->Ad);
      put(S->dq, S->q);
      put(S->db, S->b);
      put(S->dD, S->D);
      put(S->dE, S->E);
      HC_HIP(hipStreamSynchronize(st));
    }
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HC_ERR_INVALID_ARG;
  }
  return HC_OK;
}

int32_t hc_test_ordered_sums(hc_solver* S, int32_t* ordered, double* out) {
  if (!S || !ordered || !out) return HC_ERR_INVALID_ARG;
  try {
    *ordered = S->ordered ? 1 : 0;
    out[0] = out[1] = out[2] = 0.0;
    if (!S->ordered) return HC_OK;
    const HostCsr& A = S->A;
    const int64_t ld = S->ld;
    auto weight = [](int64_t i) { return 1.0 + 0.001 * (double)(i % 97); };
    std::vector<double> ST0((size_t)ld * ld), L0(S->lval_total + 1), C0(S->cval_total + 1);
    std::vector<double> ST1(ST0.size()), L1(L0.size()), C1(C0.size());
    double lost = 0.0;
    // (1) each product added where it lands: the tail (or the whole dense S)
    // at (hi, lo); one leaf's block at (hi, lo) of its l x l block; a leaf
    // column l against tail index t at row i of the coupling block, where
    // the leaf's coupling list holds t at position i (linear search)
    auto at = [&](int32_t j, int32_t k) -> double* {
      if (!S->leaves) return &ST0[std::max(j, k) + (int64_t)std::min(j, k) * ld];
      const int32_t bj = S->col_leaf[j], bk = S->col_leaf[k], lj = S->col_loc[j], lk = S->col_loc[k];
      if (bj < 0 && bk < 0) return &ST0[std::max(lj, lk) + (int64_t)std::min(lj, lk) * ld];
      if (bj >= 0 && bk >= 0)
        return bj == bk ? &L0[S->leaf_lval_off[bj] + std::max(lj, lk) + (int64_t)std::min(lj, lk) * S->leaf_size[bj]]
                        : &lost;
      const int32_t b = bj >= 0 ? bj : bk, l = bj >= 0 ? lj : lk, t = bj >= 0 ? lk : lj;
      for (int i = 0; i < S->leaf_ccnt[b]; ++i)
        if (S->leaf_clist[S->leaf_clist_off[b] + i] == t)
          return &C0[S->leaf_cval_off[b] + i + (int64_t)l * S->leaf_ccnt[b]];
      return &lost;
    };
    for (size_t t = 0; t < S->tra.size(); ++t) {
      const int32_t ra = S->tra[t], rb = S->trb[t];
      const double m = weight(S->tm[t]);
      for (int32_t p = A.rp[ra]; p < A.rp[ra + 1]; ++p)
        for (int32_t q = A.rp[rb]; q < (ra == rb ? p + 1 : A.rp[rb + 1]); ++q) {
          double v = m * A.v[p] * A.v[q];
          if (ra != rb && A.ci[p] == A.ci[q]) v *= 2.0;
          *at(A.ci[p], A.ci[q]) += v;
        }
    }
    // (2) the ordered lists
    for (size_t d = 0; d + 1 < S->op_ptr.size(); ++d) {
      double acc = 0.0;
      for (int64_t k = S->op_ptr[d]; k < S->op_ptr[d + 1]; ++k) {
        int32_t q = S->op_pq[k];
        const bool two = q < 0;
        if (two) q = ~q;
        double v = weight(S->op_pm[k]) * A.v[S->op_pp[k]] * A.v[q];
        if (two) v *= 2.0;
        acc += v;
      }
      const uint64_t e = (uint64_t)S->op_dst[d];
      const uint64_t off = e & ((uint64_t(1) << 62) - 1);
      std::vector<double>& tgt = (e >> 62) == 0 ? ST1 : (e >> 62) == 1 ? L1 : C1;
      if ((e >> 62) == 3 || off >= tgt.size()) fail(HC_ERR_STATE, "ordered sum: destination out of range");
      tgt[off] += acc;
    }
    double big = 0.0, diff = std::fabs(lost);
    const std::vector<double>* pairs[3][2] = {{&ST0, &ST1}, {&L0, &L1}, {&C0, &C1}};
    for (auto& pr : pairs)
      for (size_t i = 0; i < pr[0]->size(); ++i) {
        big = std::max(big, std::fabs((*pr[0])[i]));
        diff = std::max(diff, std::fabs((*pr[0])[i] - (*pr[1])[i]));
      }
    out[0] = big > 0.0 ? diff / big : diff;
    // leaf slots: every slot in exactly one list, the list's entry being the
    // (coupling row a, coupling row c) entry of S_TT the slot's pair names
    std::vector<int> seen(S->lpair_total, 0);
    double bad = 0.0;
    std::vector<std::pair<int64_t, int64_t>> who(S->lpair_total);   // slot -> (leaf, pair)
    for (size_t b = 0; b < S->leaf_size.size(); ++b)
      for (int64_t p = 0; p < (int64_t)S->leaf_ccnt[b] * (S->leaf_ccnt[b] + 1) / 2; ++p)
        who[S->leaf_lp_off[b] + p] = {(int64_t)b, p};
    for (size_t d = 0; d + 1 < S->ol_ptr.size(); ++d)
      for (int64_t k = S->ol_ptr[d]; k < S->ol_ptr[d + 1]; ++k) {
        const int32_t sl = S->ol_pp[k];
        if (sl < 0 || sl >= S->lpair_total) { bad += 1; continue; }
        seen[sl]++;
        const int64_t b = who[sl].first, p = who[sl].second;
        int64_t a = 0;
        while ((a + 1) * (a + 2) / 2 <= p) ++a;
        const int64_t c = p - a * (a + 1) / 2;
        const int32_t* cl = S->leaf_clist.data() + S->leaf_clist_off[b];
        if (S->ol_dst[d] != cl[a] + (int64_t)cl[c] * ld) bad += 1;
      }
    for (int64_t i = 0; i < S->lpair_total; ++i) bad += (seen[i] != 1);
    out[1] = bad;
    out[2] = (double)S->op_ptr.size() - 1.0 + (double)S->ol_ptr.size() - 1.0;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

int32_t hc_test_schur(hc_solver* S, double mu, int32_t force_dual, double* S_out, double* L_out, double* stats) {
  if (!S || !S_out) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  if (!(mu > 0)) return HC_ERR_INVALID_ARG;
  if (S->leaves || S->nt != S->n) {
    g_last_error = "hc_test_schur: leaf blocks in use (set leaf_blocks = 0)";
    return HC_ERR_STATE;
  }
  try {
    HC_HIP(hipSetDevice(S->device));
    hipStream_t st = S->stream;
    const int64_t n = S->n;
    int pd = 0;
    scale_all(S, mu, force_dual != 0, &pd);
    S->snap_S = S_out;
    try {
      factor(S);
    } catch (...) {
      S->snap_S = nullptr;
      throw;
    }
    S->snap_S = nullptr;
    if (L_out && n > 0) {
      if (S->use64) {
        HC_HIP(hipMemcpy2DAsync(L_out, n * 8, S->dS, S->ld * 8, n * 8, n, hipMemcpyDeviceToHost, st));
        HC_HIP(hipStreamSynchronize(st));
      } else {
        std::vector<float> tmp((size_t)n * n);
        HC_HIP(hipMemcpy2DAsync(tmp.data(), n * 4, S->dS32, S->ld * 4, n * 4, n, hipMemcpyDeviceToHost, st));
        HC_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < tmp.size(); ++i) L_out[i] = tmp[i];
      }
    }
    HC_HIP(hipStreamSynchronize(st));
    if (stats) {
      stats[0] = S->delta;
      stats[1] = (double)pd;
      stats[2] = S->use64 ? 64.0 : 32.0;
    }
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

int32_t hc_test_kkt_ops(hc_solver* S, double mu, int32_t force_dual, const double* r1, const double* r2, double* xr,
                        double* zr, double* kx, double* kz) {
  if (!S || !r1 || !r2 || !xr || !zr || !kx || !kz) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  if (!(mu > 0)) return HC_ERR_INVALID_ARG;
  try {
    HC_HIP(hipSetDevice(S->device));
    hipStream_t st = S->stream;
    const int64_t n = S->n, m = S->m;
    int pd = 0;
    scale_all(S, mu, force_dual != 0, &pd);
    factor(S);
    HC_HIP(hipMemcpyAsync(S->r1, r1, n * 8, hipMemcpyHostToDevice, st));
    HC_HIP(hipMemcpyAsync(S->r2, r2, m * 8, hipMemcpyHostToDevice, st));
    solve_reg(S, S->r1, S->r2, S->x1, S->z1);
    // K [x1; z1] with the unregularised K, as the refinement forms it
    P_mul(S, S->x1, S->kx, 1.0, 0.0);
    At_mul(S, S->z1, S->kx, 1.0, 1.0);
    A_mul(S, S->x1, S->kz, 1.0, 0.0);
    H_apply(S, 0, S->z1, S->t2);
    vaxpby(m, -1.0, S->t2, 1.0, S->kz, st);
    HC_HIP(hipMemcpyAsync(xr, S->x1, n * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipMemcpyAsync(zr, S->z1, m * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipMemcpyAsync(kx, S->kx, n * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipMemcpyAsync(kz, S->kz, m * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipStreamSynchronize(st));
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

int32_t hc_test_kkt_solve(hc_solver* S, double mu, int32_t force_dual, const double* r1, const double* r2,
                          double* xo, double* zo, double* stats) {
  if (!S || !r1 || !r2 || !xo || !zo) return HC_ERR_INVALID_ARG;
  if (!S->bound) return HC_ERR_STATE;
  if (!(mu > 0)) return HC_ERR_INVALID_ARG;
  try {
    HC_HIP(hipSetDevice(S->device));
    hipStream_t st = S->stream;
    const int64_t n = S->n, m = S->m;
    int pd = 0;
    scale_all(S, mu, force_dual != 0, &pd);
    factor(S);
    HC_HIP(hipMemcpyAsync(S->r1, r1, n * 8, hipMemcpyHostToDevice, st));
    HC_HIP(hipMemcpyAsync(S->r2, r2, m * 8, hipMemcpyHostToDevice, st));
    const int64_t before = S->info.ir_solves, fb = S->info.fp64_fallbacks;
    kkt_solve(S, S->r1, S->r2, S->x1, S->z1);
    HC_HIP(hipMemcpyAsync(xo, S->x1, n * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipMemcpyAsync(zo, S->z1, m * 8, hipMemcpyDeviceToHost, st));
    HC_HIP(hipStreamSynchronize(st));
    if (stats) {
      stats[0] = (double)(S->info.ir_solves - before);
      stats[1] = S->delta;
      stats[2] = (double)pd;
      stats[3] = (double)(S->info.fp64_fallbacks - fb);
    }
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
  return HC_OK;
}

void hc_destroy(hc_solver* S) {
  if (!S) return;
  if (S->own_mem && S->mem) (void)hipFree(S->mem);
  if (S->own_stage) {
    if (S->hpart) (void)hipHostFree(S->hpart);
    if (S->hmask) (void)hipHostFree(S->hmask);
  }
  delete S;
}

const char* hc_last_error(const hc_solver* S) {
  if (S && !S->last_error.empty()) return S->last_error.c_str();
  return g_last_error.c_str();
}

const char* hc_status_str(int32_t status) {
  switch (status) {
    case HC_STATUS_UNSOLVED: return "unsolved";
    case HC_STATUS_SOLVED: return "solved";
    case HC_STATUS_PRIMAL_INFEASIBLE: return "primal_infeasible";
    case HC_STATUS_DUAL_INFEASIBLE: return "dual_infeasible";
    case HC_STATUS_MAX_ITER: return "max_iter";
    case HC_STATUS_INSUFFICIENT_PROGRESS: return "insufficient_progress";
    case HC_STATUS_NUMERICAL_ERROR: return "numerical_error";
    case HC_STATUS_CANCELLED: return "cancelled";
  }
  return "unknown";
}

}  // extern "C"
