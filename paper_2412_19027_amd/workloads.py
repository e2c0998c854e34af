"""Seeded synthetic conic problems shaped like the paper's workloads.

This module only *builds inputs*: sparse matrices, vectors and cone lists of
problems in the form (P) of the paper (minimize 1/2 x'Px + q'x subject to
Ax + s = b, s in K).  It holds none of the interior-point method's arithmetic
and is the one module shared by the CPU oracle's tests and by the GPU path's
tests and benchmark.

Cone kinds and the `dim` convention (rows a cone occupies):
  ZERO, NONNEG : dim = number of rows
  SOC          : dim = number of rows (t, x_1 .. x_{dim-1})
  EXP, POW     : dim = 3 (POW carries its exponent alpha in (0, 1))
  PSD          : dim = matrix side k; rows = k (k + 1) / 2 in the svec
                 encoding (upper triangle, column by column, off-diagonal
                 entries scaled by sqrt(2)).

Workload families (sizes of the full configurations in parentheses):
  tiny_lp       dense LP with a planted primal/dual interior point (n=50, m=100)
  sparse_socp   factor-model SOCP with zero, nonneg and SOC-3 rows (n=20,020)
  logreg_exp    l1-regularised logistic regression via exp cones (n=301,000)
  psd_pow       equal-size PSD cones plus 3-d power cones (n=5,000)
  mpc_socp      one request of the served MPC stream (n <= 1,812)
  entropy_max   the paper's entropy maximisation with m = n/2 dense
                inequalities (n = 2,000 .. 10,000)
  portfolio_qp  the paper's factor-model portfolio QP, rank p = n/10
                (n = 5,000 .. 25,000)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

ZERO, NONNEG, SOC, EXP, POW, PSD = 0, 1, 2, 3, 4, 5
KIND_NAMES = {ZERO: "zero", NONNEG: "nonneg", SOC: "soc", EXP: "exp", POW: "pow", PSD: "psd"}


def cone_rows(kind: int, dim: int) -> int:
    """Rows occupied by one cone of the given kind and dim."""
    if kind == PSD:
        return dim * (dim + 1) // 2
    return dim


@dataclasses.dataclass
class Problem:
    """A conic problem in the paper's form (P).

    P is stored as the upper triangle (col >= row) in CSR; A is CSR with
    m rows; cones is a list of (kind, dim, alpha) in row order.
    """

    n: int
    m: int
    P: sp.csr_matrix
    q: np.ndarray
    A: sp.csr_matrix
    b: np.ndarray
    cones: list
    name: str = ""

    def __post_init__(self):
        self.P = sp.csr_matrix(self.P, dtype=np.float64)
        self.A = sp.csr_matrix(self.A, dtype=np.float64)
        self.P.sort_indices()
        self.A.sort_indices()
        self.P.sum_duplicates()
        self.A.sum_duplicates()
        self.q = np.ascontiguousarray(self.q, dtype=np.float64)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)
        assert self.P.shape == (self.n, self.n)
        assert self.A.shape == (self.m, self.n)
        assert self.q.shape == (self.n,) and self.b.shape == (self.m,)
        assert sum(cone_rows(k, d) for k, d, _ in self.cones) == self.m

    def cone_array(self) -> np.ndarray:
        """Cones as a structured array matching the C struct {int32 type; int32 dim; double alpha;}."""
        dt = np.dtype([("type", np.int32), ("dim", np.int32), ("alpha", np.float64)])
        out = np.zeros(len(self.cones), dtype=dt)
        for i, (k, d, a) in enumerate(self.cones):
            out[i] = (k, d, a)
        return out


def merge_cones(cones):
    """Merge consecutive ZERO / NONNEG cones (pure bookkeeping of the cone list)."""
    out = []
    for k, d, a in cones:
        if out and k in (ZERO, NONNEG) and out[-1][0] == k:
            out[-1] = (k, out[-1][1] + d, 0.0)
        else:
            out.append((k, d, a))
    return out


# --------------------------------------------------------------------------
# interior samples used to plant feasible primal / dual points
# --------------------------------------------------------------------------

def _soc_interior(rng, count, dim):
    u = rng.standard_normal((count, dim - 1))
    t = np.linalg.norm(u, axis=1) + rng.uniform(0.1, 1.0, count)
    return np.concatenate([t[:, None], u], axis=1)


def _pow_interior(rng, alpha, dual):
    a = rng.uniform(0.5, 1.5, alpha.shape)
    bb = rng.uniform(0.5, 1.5, alpha.shape)
    if dual:
        g = (a / alpha) ** alpha * (bb / (1 - alpha)) ** (1 - alpha)
    else:
        g = a ** alpha * bb ** (1 - alpha)
    c = rng.uniform(-0.9, 0.9, alpha.shape) * g
    return np.stack([a, bb, c], axis=1)


def svec_encode(X: np.ndarray) -> np.ndarray:
    """Encode symmetric k x k matrices (..., k, k) in the svec convention."""
    k = X.shape[-1]
    out = []
    for j in range(k):
        for i in range(j + 1):
            f = 1.0 if i == j else math.sqrt(2.0)
            out.append(X[..., i, j] * f)
    return np.stack(out, axis=-1)


def _spd_sample(rng, count, k):
    G = rng.standard_normal((count, k, k))
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diagonal(R, axis1=1, axis2=2))
    sgn[sgn == 0] = 1.0
    Q = Q * sgn[:, None, :]
    lam = rng.uniform(0.5, 2.0, (count, k))
    return np.einsum("cij,cj,ckj->cik", Q, lam, Q)


def _random_rows(rng, nrows, ncols, nnz_per_row, col_offset=0):
    """CSR pieces for rows with `nnz_per_row` distinct uniform columns, N(0,1) values."""
    cols = np.empty((nrows, nnz_per_row), dtype=np.int64)
    for i in range(nrows):
        cols[i] = rng.choice(ncols, nnz_per_row, replace=False)
    cols.sort(axis=1)
    vals = rng.standard_normal((nrows, nnz_per_row))
    indptr = np.arange(nrows + 1, dtype=np.int64) * nnz_per_row
    return indptr, cols.ravel() + col_offset, vals.ravel()


def _random_rows_fast(rng, nrows, ncols, nnz_per_row):
    """Same distribution as `_random_rows`, vectorised (rejection of duplicate columns)."""
    cols = rng.integers(0, ncols, size=(nrows, nnz_per_row))
    cols.sort(axis=1)
    while True:
        dup = np.any(cols[:, 1:] == cols[:, :-1], axis=1)
        nd = int(dup.sum())
        if nd == 0:
            break
        cols[dup] = rng.integers(0, ncols, size=(nd, nnz_per_row))
        cols[dup] = np.sort(cols[dup], axis=1)
    vals = rng.standard_normal((nrows, nnz_per_row))
    return cols, vals


# --------------------------------------------------------------------------
# tiny LP (n = 50, m = 100 nonnegative rows)
# --------------------------------------------------------------------------

def tiny_lp(seed: int = 0, n: int = 50, m: int = 100) -> Problem:
    """Dense LP, P = 0; A ~ N(0,1); x0 ~ N(0,1); s0, z0 ~ U(0.1, 1); b = A x0 + s0, q = -A' z0."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    x0 = rng.standard_normal(n)
    s0 = rng.uniform(0.1, 1.0, m)
    z0 = rng.uniform(0.1, 1.0, m)
    b = A @ x0 + s0
    q = -A.T @ z0
    return Problem(n, m, sp.csr_matrix((n, n)), q, sp.csr_matrix(A), b,
                   [(NONNEG, m, 0.0)], name=f"tiny_lp(seed={seed})")


# --------------------------------------------------------------------------
# sparse factor-model SOCP
# --------------------------------------------------------------------------

def sparse_socp(seed: int = 0, nx: int = 20000, rank: int = 20, n_zero: int = 10000,
                n_nonneg: int = 30000, n_soc: int = 40000, nnz_row: int = 6) -> Problem:
    """Factor-model SOCP: P = diag(D) + F F' lifted as y = F'x (rank extra zero rows).

    Variables (x, y), n = nx + rank; P = blkdiag(diag(D), I).  Rows in order:
    n_zero zero rows, rank lift rows y_i - F[:, i]'x = 0 (zero cone), n_nonneg
    nonneg rows, n_soc SOC-3 cones; every non-lift row has nnz_row distinct
    uniform columns over x with N(0,1) values.  Primal and dual interior
    points are planted so the problem is feasible and bounded.
    """
    rng = np.random.default_rng(seed)
    n = nx + rank
    D = rng.uniform(0.01, 1.0, nx)
    F = rng.standard_normal((nx, rank)) / math.sqrt(rank)
    n_plain = n_zero + n_nonneg + 3 * n_soc
    cols, vals = _random_rows_fast(rng, n_plain, nx, nnz_row)
    # assemble rows: zero block, lift rows, nonneg block, soc block
    rows_zero = (cols[:n_zero], vals[:n_zero])
    rows_rest = (cols[n_zero:], vals[n_zero:])
    indptr = [np.zeros(1, dtype=np.int64)]
    ind_list, val_list, lens = [], [], []
    ind_list.append(rows_zero[0].ravel()); val_list.append(rows_zero[1].ravel())
    lens += [nnz_row] * n_zero
    for i in range(rank):
        ind_list.append(np.concatenate([np.arange(nx), [nx + i]]))
        val_list.append(np.concatenate([-F[:, i], [1.0]]))
        lens.append(nx + 1)
    ind_list.append(rows_rest[0].ravel()); val_list.append(rows_rest[1].ravel())
    lens += [nnz_row] * (n_nonneg + 3 * n_soc)
    indptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    m = n_zero + rank + n_nonneg + 3 * n_soc
    A = sp.csr_matrix((np.concatenate(val_list), np.concatenate(ind_list), indptr), shape=(m, n))
    P = sp.diags(np.concatenate([D, np.ones(rank)])).tocsr()
    x0 = rng.standard_normal(nx)
    xy0 = np.concatenate([x0, F.T @ x0])
    s0 = np.zeros(m)
    z0 = np.zeros(m)
    z0[:n_zero] = rng.standard_normal(n_zero)
    z0[n_zero:n_zero + rank] = rng.standard_normal(rank)
    o = n_zero + rank
    s0[o:o + n_nonneg] = rng.uniform(0.1, 1.0, n_nonneg)
    z0[o:o + n_nonneg] = rng.uniform(0.1, 1.0, n_nonneg)
    o += n_nonneg
    s0[o:] = _soc_interior(rng, n_soc, 3).ravel()
    z0[o:] = _soc_interior(rng, n_soc, 3).ravel()
    b = A @ xy0 + s0
    q = -(A.T @ z0)
    cones = [(ZERO, n_zero + rank, 0.0), (NONNEG, n_nonneg, 0.0)] + [(SOC, 3, 0.0)] * n_soc
    return Problem(n, m, P, q, A, b, cones, name=f"sparse_socp(seed={seed},nx={nx})")


# --------------------------------------------------------------------------
# l1-regularised logistic regression with exponential cones
# --------------------------------------------------------------------------

def logreg_exp(seed: int = 0, samples: int = 100000, features: int = 500, nnz_row: int = 10,
               lam_frac: float = 0.1) -> Problem:
    """min sum_i t_i + lam ||theta||_1 with log(1 + exp(-y_i x_i'theta)) <= t_i.

    Variables [theta (F), r (F), t, w1, w2 (N each)].  Per sample two exp cones
    (-y_i x_i'theta - t_i, 1, w1_i) and (-t_i, 1, w2_i) plus w1_i + w2_i <= 1;
    |theta| <= r via 2F nonneg rows.  X is N x F with nnz_row distinct uniform
    columns per row (N(0,1)); y = +-1 with probability 1/2.
    """
    rng = np.random.default_rng(seed)
    N, Fe = samples, features
    cols, vals = _random_rows_fast(rng, N, Fe, nnz_row)
    X = sp.csr_matrix((vals.ravel(), cols.ravel(), np.arange(N + 1) * nnz_row), shape=(N, Fe))
    y = np.where(rng.random(N) < 0.5, -1.0, 1.0)
    lam = lam_frac * 0.5 * np.abs(X.T @ y).max()
    o_th, o_r, o_t, o_w1, o_w2 = 0, Fe, 2 * Fe, 2 * Fe + N, 2 * Fe + 2 * N
    n = 2 * Fe + 3 * N
    q = np.zeros(n)
    q[o_r:o_r + Fe] = lam
    q[o_t:o_t + N] = 1.0
    r_i, c_i, v_i = [], [], []
    b = []
    row = 0
    idx = np.arange(N)
    # nonneg: w1 + w2 <= 1
    r_i += [row + idx, row + idx]; c_i += [o_w1 + idx, o_w2 + idx]; v_i += [np.ones(N), np.ones(N)]
    b.append(np.ones(N)); row += N
    jf = np.arange(Fe)
    # theta_j - r_j <= 0  ->  s = r_j - theta_j
    r_i += [row + jf, row + jf]; c_i += [o_th + jf, o_r + jf]; v_i += [np.ones(Fe), -np.ones(Fe)]
    b.append(np.zeros(Fe)); row += Fe
    # -theta_j - r_j <= 0 ->  s = theta_j + r_j
    r_i += [row + jf, row + jf]; c_i += [o_th + jf, o_r + jf]; v_i += [-np.ones(Fe), -np.ones(Fe)]
    b.append(np.zeros(Fe)); row += Fe
    # exp cones, two per sample, interleaved per sample in row order
    base = row
    r1 = base + 6 * idx          # first exp cone rows r1, r1+1, r1+2
    r2 = r1 + 3                  # second exp cone rows
    # row r1: s = -y x'theta - t  -> A = y x' at theta, +1 at t
    Xc = X.tocoo()
    r_i += [r1[Xc.row], r1]; c_i += [o_th + Xc.col, o_t + idx]; v_i += [y[Xc.row] * Xc.data, np.ones(N)]
    # row r1+2: s = w1 -> A = -1 at w1
    r_i += [r1 + 2]; c_i += [o_w1 + idx]; v_i += [-np.ones(N)]
    # row r2: s = -t -> A = +1 at t
    r_i += [r2]; c_i += [o_t + idx]; v_i += [np.ones(N)]
    r_i += [r2 + 2]; c_i += [o_w2 + idx]; v_i += [-np.ones(N)]
    bexp = np.zeros(6 * N)
    bexp[6 * idx + 1] = 1.0
    bexp[6 * idx + 4] = 1.0
    b.append(bexp)
    m = row + 6 * N
    A = sp.csr_matrix((np.concatenate(v_i), (np.concatenate(r_i), np.concatenate(c_i))), shape=(m, n))
    cones = [(NONNEG, N + 2 * Fe, 0.0)] + [(EXP, 3, 0.0)] * (2 * N)
    return Problem(n, m, sp.csr_matrix((n, n)), q, A, np.concatenate(b), cones,
                   name=f"logreg_exp(seed={seed},N={N},F={Fe})")


# --------------------------------------------------------------------------
# equal-size PSD cones plus power cones
# --------------------------------------------------------------------------

def psd_pow(seed: int = 0, n: int = 5000, n_pow: int = 20000, n_psd: int = 2000, k: int = 10,
            nnz_row: int = 8) -> Problem:
    """P = 0; rows: n_pow POW-3 cones (alpha ~ U(0.2, 0.8)) then n_psd PSD cones of side k.

    A has nnz_row distinct uniform columns per row, N(0,1).  Planted interior
    points: power cones by the interior recipe; PSD blocks S0, Z0 = Q diag(U(0.5,2)) Q'.
    """
    rng = np.random.default_rng(seed)
    sd = k * (k + 1) // 2
    m = 3 * n_pow + sd * n_psd
    cols, vals = _random_rows_fast(rng, m, n, nnz_row)
    A = sp.csr_matrix((vals.ravel(), cols.ravel(), np.arange(m + 1) * nnz_row), shape=(m, n))
    x0 = rng.standard_normal(n)
    alpha = rng.uniform(0.2, 0.8, n_pow)
    s_pow = _pow_interior(rng, alpha, dual=False)
    z_pow = _pow_interior(rng, alpha, dual=True)
    S0 = svec_encode(_spd_sample(rng, n_psd, k))
    Z0 = svec_encode(_spd_sample(rng, n_psd, k))
    s0 = np.concatenate([s_pow.ravel(), S0.ravel()])
    z0 = np.concatenate([z_pow.ravel(), Z0.ravel()])
    b = A @ x0 + s0
    q = -(A.T @ z0)
    cones = [(POW, 3, float(a)) for a in alpha] + [(PSD, k, 0.0)] * n_psd
    return Problem(n, m, sp.csr_matrix((n, n)), q, A, b, cones,
                   name=f"psd_pow(seed={seed},n={n},pow={n_pow},psd={n_psd}x{k})")


def psd_mixed(seed: int = 0, n: int = 300, sides=(3, 5, 8), per_side: int = 20, nnz_row: int = 8) -> Problem:
    """P = 0; PSD cones of several sides (per_side cones of each side, the
    sides interleaved in row order) with planted interior points as in
    psd_pow; A has nnz_row distinct uniform columns per row, N(0,1)."""
    rng = np.random.default_rng(seed)
    order = [k for _ in range(per_side) for k in sides]
    m = sum(k * (k + 1) // 2 for k in order)
    cols, vals = _random_rows_fast(rng, m, n, nnz_row)
    A = sp.csr_matrix((vals.ravel(), cols.ravel(), np.arange(m + 1) * nnz_row), shape=(m, n))
    x0 = rng.standard_normal(n)
    s0 = np.concatenate([svec_encode(_spd_sample(rng, 1, k)).ravel() for k in order])
    z0 = np.concatenate([svec_encode(_spd_sample(rng, 1, k)).ravel() for k in order])
    b = A @ x0 + s0
    q = -(A.T @ z0)
    cones = [(PSD, k, 0.0) for k in order]
    return Problem(n, m, sp.csr_matrix((n, n)), q, A, b, cones,
                   name=f"psd_mixed(seed={seed},n={n},sides={tuple(sides)}x{per_side})")


# --------------------------------------------------------------------------
# served MPC stream
# --------------------------------------------------------------------------

def mpc_socp(seed: int, index: int, T: int | None = None, nx: int | None = None,
             nu: int | None = None, x_scale: float = 3.0) -> Problem:
    """One MPC request: min 1/2 sum |x_t|^2 + 0.05 sum |u_t|^2 subject to dynamics,

    |u_t|_inf <= 1 (nonneg rows) and |(u_t0, u_t1)|_2 <= 1 (SOC-3 per step).
    A_d = 0.95 M / rho(M); B_d ~ N(0,1); x_init ~ N(0, x_scale^2 I).
    """
    rng = np.random.default_rng(seed * 10**6 + index)
    T = int(rng.integers(10, 101)) if T is None else T
    nx = int(rng.integers(4, 13)) if nx is None else nx
    nu = int(rng.integers(2, 7)) if nu is None else nu
    M = rng.standard_normal((nx, nx))
    Ad = 0.95 * M / np.abs(np.linalg.eigvals(M)).max()
    Bd = rng.standard_normal((nx, nu))
    x_init = x_scale * rng.standard_normal(nx)
    n = (T + 1) * nx + T * nu
    xo = lambda t: t * nx
    uo = lambda t: (T + 1) * nx + t * nu
    rows, cols, vals, b = [], [], [], []
    r = 0
    for i in range(nx):
        rows.append(r + i); cols.append(xo(0) + i); vals.append(1.0)
    b += list(x_init); r += nx
    for t in range(T):
        for i in range(nx):
            rows.append(r + i); cols.append(xo(t + 1) + i); vals.append(1.0)
            for j in range(nx):
                if Ad[i, j] != 0.0:
                    rows.append(r + i); cols.append(xo(t) + j); vals.append(-Ad[i, j])
            for j in range(nu):
                rows.append(r + i); cols.append(uo(t) + j); vals.append(-Bd[i, j])
        b += [0.0] * nx; r += nx
    n_zero = r
    for t in range(T):
        for j in range(nu):
            rows.append(r); cols.append(uo(t) + j); vals.append(1.0); b.append(1.0); r += 1
            rows.append(r); cols.append(uo(t) + j); vals.append(-1.0); b.append(1.0); r += 1
    n_nn = r - n_zero
    for t in range(T):
        b.append(1.0); r += 1
        rows.append(r); cols.append(uo(t) + 0); vals.append(-1.0); b.append(0.0); r += 1
        rows.append(r); cols.append(uo(t) + 1); vals.append(-1.0); b.append(0.0); r += 1
    m = r
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    pd = np.concatenate([np.ones((T + 1) * nx), 0.1 * np.ones(T * nu)])
    cones = [(ZERO, n_zero, 0.0), (NONNEG, n_nn, 0.0)] + [(SOC, 3, 0.0)] * T
    return Problem(n, m, sp.diags(pd).tocsr(), np.zeros(n), A, np.array(b), cones,
                   name=f"mpc_socp(seed={seed},i={index},T={T},nx={nx},nu={nu})")


def mpc_arrivals(seed: int, count: int, rate: float = 2000.0) -> np.ndarray:
    """Poisson arrival times (seconds) of the served stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


# --------------------------------------------------------------------------
# named full-size configurations
# --------------------------------------------------------------------------

# --------------------------------------------------------------------------
# the paper's exponential-cone and QP benchmark problems (Sec. 4.4, 4.2)
# --------------------------------------------------------------------------

def entropy_max(seed: int = 0, n: int = 10000) -> Problem:
    """maximize -sum x_i log x_i s.t. 1'x = 1, A x <= b, with m = round(n/2)
    dense rows A_ij ~ N(0, n) (variance n) and b = A v / 1'v, v_i ~ U(0, 1)
    (so v / 1'v is feasible).  Variables [x (n), t (n)], minimize -sum t with
    (t_i, x_i, 1) in K_exp, i.e. x_i exp(t_i / x_i) <= 1."""
    rng = np.random.default_rng(seed)
    m_in = int(round(0.5 * n))
    Ad = rng.standard_normal((m_in, n)) * math.sqrt(n)
    v = rng.uniform(0.0, 1.0, n)
    bin_ = Ad @ v / v.sum()
    nv = 2 * n
    q = np.concatenate([np.zeros(n), -np.ones(n)])
    idx = np.arange(n)
    # row 0: 1'x = 1 (zero cone); rows 1..m_in: A x + s = b (nonneg); then exp cones
    top = sp.hstack([sp.csr_matrix(np.vstack([np.ones((1, n)), Ad])), sp.csr_matrix((1 + m_in, n))]).tocsr()
    r0 = np.repeat(3 * idx, 1)
    ex = sp.csr_matrix((-np.ones(2 * n), (np.concatenate([r0, r0 + 1]), np.concatenate([n + idx, idx]))),
                       shape=(3 * n, nv))
    A = sp.vstack([top, ex]).tocsr()
    bexp = np.zeros(3 * n)
    bexp[3 * idx + 2] = 1.0
    b = np.concatenate([[1.0], bin_, bexp])
    cones = [(ZERO, 1, 0.0), (NONNEG, m_in, 0.0)] + [(EXP, 3, 0.0)] * n
    return Problem(nv, A.shape[0], sp.csr_matrix((nv, nv)), q, A, b, cones, name=f"entropy_max(seed={seed},n={n})")


def portfolio_qp(seed: int = 0, n: int = 25000, density: float = 0.1, gamma: float = 1.0) -> Problem:
    """maximize mu'x - gamma x'(F F' + D)x s.t. 1'x = 1, x >= 0, rank
    p = round(n/10), lifted as y = F'x: minimize gamma (x'Dx + y'y) - mu'x
    with the p rows y - F'x = 0 and 1'x = 1 in the zero cone and x >= 0.
    Distributions (the paper gives none): F_ij ~ N(0, 1) present with
    probability `density`, D_ii ~ U(0, sqrt(p)), mu_i ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    p = max(1, int(round(0.1 * n)))
    F = sp.random(n, p, density=density, random_state=rng, data_rvs=rng.standard_normal, format="csc")
    D = rng.uniform(0.0, math.sqrt(p), n)
    mu = rng.standard_normal(n)
    nv = n + p
    P = sp.diags(np.concatenate([2.0 * gamma * D, 2.0 * gamma * np.ones(p)])).tocsr()
    q = np.concatenate([-mu, np.zeros(p)])
    lift = sp.hstack([-F.T, sp.identity(p)]).tocsr()                 # y - F'x = 0
    budget = sp.csr_matrix(np.concatenate([np.ones(n), np.zeros(p)])[None, :])
    nonneg = sp.hstack([-sp.identity(n), sp.csr_matrix((n, p))]).tocsr()   # s = x >= 0
    A = sp.vstack([lift, budget, nonneg]).tocsr()
    b = np.concatenate([np.zeros(p), [1.0], np.zeros(n)])
    cones = [(ZERO, p + 1, 0.0), (NONNEG, n, 0.0)]
    return Problem(nv, A.shape[0], sp.triu(P).tocsr(), q, A, b, cones, name=f"portfolio_qp(seed={seed},n={n},p={p})")


def multistage_portfolio(seed: int = 0, n: int = 5000, k: int = 50, T: int = 5, density: float = 0.1,
                         gamma: float = 1.0, cost: float = 0.01, inflow: float = 0.1) -> Problem:
    """Multistage portfolio SOCP (eq. multistage_socp): over T periods,
    minimize sum_t -mu_t'x_t + cost 1'z_t + gamma r_t subject to
    z_t >= +-(x_t - x_{t-1}), 1'x_1 = inflow + 1'x_0, 1'x_t = 1'x_{t-1},
    y_t = F_t x_t, (r_t, U y_t, D_sqrt o x_t) in the SOC of dimension n + k + 1,
    x_t in [0, 0.1]^n, y_t in [0, 0.1]^k, r_t >= 0 (z_t free).
    Variables stage by stage: [x_t (n), y_t (k), z_t (n), r_t].
    Distributions (the paper gives none): x_0 = 1/n, mu_t ~ N(0, 1),
    F_t (k x n) with N(0, 1) entries present with probability `density`,
    U the upper Cholesky factor of G G'/k + I (G ~ N(0, 1), k x k),
    D_sqrt = sqrt(D) with D_ii ~ U(0, sqrt(k))."""
    rng = np.random.default_rng(seed)
    V = 2 * n + k + 1
    nv = T * V
    G = rng.standard_normal((k, k))
    U = np.linalg.cholesky(G @ G.T / k + np.eye(k)).T
    Dsq = np.sqrt(rng.uniform(0.0, math.sqrt(k), n))
    x0 = np.full(n, 1.0 / n)
    xo = lambda t: t * V
    yo = lambda t: t * V + n
    zo = lambda t: t * V + n + k
    ro = lambda t: t * V + 2 * n + k
    q = np.zeros(nv)
    zr, zc, zv, zb = [], [], [], []       # zero rows
    nr, nc_, nvv, nb = [], [], [], []     # nonneg rows
    sr, sc, svv = [], [], []              # SOC rows
    row = [0, 0]

    def add(cols, vals, tgt, r):
        tgt[0].extend([r] * len(cols))
        tgt[1].extend(cols)
        tgt[2].extend(vals)

    ar = np.arange(n)
    for t in range(T):
        q[xo(t):xo(t) + n] = -rng.standard_normal(n)
        q[zo(t):zo(t) + n] = cost
        q[ro(t)] = gamma
        F = sp.random(k, n, density=density, random_state=rng, data_rvs=rng.standard_normal, format="csr")
        # budget
        cols = list(xo(t) + ar)
        vals = [1.0] * n
        if t > 0:
            cols += list(xo(t - 1) + ar)
            vals += [-1.0] * n
        add(cols, vals, (zr, zc, zv), row[0])
        zb.append(inflow + x0.sum() if t == 0 else 0.0)
        row[0] += 1
        # y_t - F_t x_t = 0
        for i in range(k):
            lo, hi = F.indptr[i], F.indptr[i + 1]
            add([yo(t) + i] + list(xo(t) + F.indices[lo:hi]), [1.0] + list(-F.data[lo:hi]),
                (zr, zc, zv), row[0])
            zb.append(0.0)
            row[0] += 1
        # transactions: +-(x_t - x_{t-1}) - z_t <= 0 (x_0 moves to the right-hand side)
        for sgn in (1.0, -1.0):
            for i in range(n):
                cols, vals = [xo(t) + i, zo(t) + i], [sgn, -1.0]
                if t > 0:
                    cols.append(xo(t - 1) + i)
                    vals.append(-sgn)
                add(cols, vals, (nr, nc_, nvv), row[1])
                nb.append(sgn * x0[i] if t == 0 else 0.0)
                row[1] += 1
        # bounds: -x <= 0, x <= 0.1, -y <= 0, y <= 0.1, -r <= 0
        for off, cnt in ((xo(t), n), (yo(t), k)):
            for sgn, bound in ((-1.0, 0.0), (1.0, 0.1)):
                for i in range(cnt):
                    add([off + i], [sgn], (nr, nc_, nvv), row[1])
                    nb.append(bound)
                    row[1] += 1
        add([ro(t)], [-1.0], (nr, nc_, nvv), row[1])
        nb.append(0.0)
        row[1] += 1
    # SOC blocks: s = -A v = (r_t, U y_t, D_sqrt o x_t)
    d = n + k + 1
    for t in range(T):
        base = t * d
        add([ro(t)], [-1.0], (sr, sc, svv), base)
        for i in range(k):
            cols = [yo(t) + j for j in range(i, k)]
            add(cols, list(-U[i, i:]), (sr, sc, svv), base + 1 + i)
        sr.extend(base + 1 + k + ar)
        sc.extend(xo(t) + ar)
        svv.extend(-Dsq)
    mz, mn, ms = row[0], row[1], T * d
    Az = sp.csr_matrix((zv, (zr, zc)), shape=(mz, nv))
    An = sp.csr_matrix((nvv, (nr, nc_)), shape=(mn, nv))
    As = sp.csr_matrix((svv, (sr, sc)), shape=(ms, nv))
    A = sp.vstack([Az, An, As]).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    b = np.concatenate([zb, nb, np.zeros(ms)])
    cones = [(ZERO, mz, 0.0), (NONNEG, mn, 0.0)] + [(SOC, d, 0.0)] * T
    return Problem(nv, A.shape[0], sp.csr_matrix((nv, nv)), q, A, b, cones,
                   name=f"multistage_portfolio(seed={seed},n={n},k={k},T={T})")


def config(name: str, seed: int = 0) -> Problem:
    if name == "tiny_lp":
        return tiny_lp(seed)
    if name == "sparse_socp":
        return sparse_socp(seed)
    if name == "logreg_exp":
        return logreg_exp(seed)
    if name == "psd_pow":
        return psd_pow(seed)
    if name == "entropy_max":
        return entropy_max(seed)
    if name == "portfolio_qp":
        return portfolio_qp(seed)
    if name == "multistage_portfolio":
        return multistage_portfolio(seed)
    raise KeyError(name)
