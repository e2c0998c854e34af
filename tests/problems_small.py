"""Tiny problems with optima known in closed form (or by an independent
routine), each exercising one cone family.  Pure problem construction."""
import math

import numpy as np
import scipy.sparse as sp

from paper_2412_19027_amd.workloads import EXP, NONNEG, POW, PSD, SOC, ZERO, Problem, svec_encode


def box_lp(seed=0, n=6):
    """min c'x, l <= x <= u  ->  x_i = l_i if c_i > 0 else u_i."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n)
    l = -rng.uniform(0.5, 2, n)
    u = rng.uniform(0.5, 2, n)
    A = sp.vstack([sp.identity(n), -sp.identity(n)]).tocsr()
    b = np.concatenate([u, -l])
    xstar = np.where(c > 0, l, u)
    return Problem(n, 2 * n, sp.csr_matrix((n, n)), c, A, b, [(NONNEG, 2 * n, 0.0)], "box_lp"), c @ xstar


def soc_ball(seed=0, n=4, r=1.7):
    """min c'x, |x|_2 <= r  ->  -r |c|."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n)
    A = sp.vstack([sp.csr_matrix((1, n)), -sp.identity(n)]).tocsr()
    b = np.concatenate([[r], np.zeros(n)])
    return Problem(n, n + 1, sp.csr_matrix((n, n)), c, A, b, [(SOC, n + 1, 0.0)], "soc_ball"), -r * np.linalg.norm(c)


def soc_balls(seed=0, dims=(20, 150, 700), radii=(0.5, 1.0, 2.0)):
    """min sum_i c_i'x_i, |x_i|_2 <= r_i over separate balls  ->  -sum_i r_i |c_i|."""
    rng = np.random.default_rng(seed)
    n = sum(dims)
    c = rng.standard_normal(n)
    blocks, b, fstar, off = [], [], 0.0, 0
    for d, r in zip(dims, radii):
        blk = sp.lil_matrix((d + 1, n))
        for i in range(d):
            blk[1 + i, off + i] = -1.0
        blocks.append(blk.tocsr())
        b += [r] + [0.0] * d
        fstar -= r * np.linalg.norm(c[off:off + d])
        off += d
    A = sp.vstack(blocks).tocsr()
    cones = [(SOC, d + 1, 0.0) for d in dims]
    return Problem(n, A.shape[0], sp.csr_matrix((n, n)), c, A, np.array(b), cones, "soc_balls"), fstar


def soc_ball_budget(seed=0, n=600, r=1.3):
    """min c'x, |x|_2 <= r, 1'x = 0  ->  -r |c - mean(c) 1|  (the minimiser is
    -r times the unit projection of c onto the hyperplane 1'x = 0)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n)
    A = sp.vstack([sp.csr_matrix(np.ones((1, n))), sp.csr_matrix((1, n)), -sp.identity(n)]).tocsr()
    b = np.concatenate([[0.0, r], np.zeros(n)])
    cones = [(ZERO, 1, 0.0), (SOC, n + 1, 0.0)]
    return Problem(n, n + 2, sp.csr_matrix((n, n)), c, A, b, cones, "soc_ball_budget"), -r * np.linalg.norm(c - c.mean())


def exp_max():
    """max x s.t. (x, 1, e) in K_exp  ->  x = 1 (objective -1)."""
    A = sp.csr_matrix(np.array([[-1.0], [0.0], [0.0]]))
    b = np.array([0.0, 1.0, math.e])
    return Problem(1, 3, sp.csr_matrix((1, 1)), np.array([-1.0]), A, b, [(EXP, 3, 0.0)], "exp_max"), -1.0


def softplus(u=0.7):
    """min t s.t. t >= log(1 + e^u) via two exp cones and w1 + w2 <= 1."""
    # variables t, w1, w2; rows: (u - t, 1, w1), (-t, 1, w2), w1 + w2 <= 1
    A = np.zeros((7, 3))
    b = np.zeros(7)
    A[0, 0] = 1.0; b[0] = u          # s = u - t
    b[1] = 1.0
    A[2, 1] = -1.0                   # s = w1
    A[3, 0] = 1.0                    # s = -t
    b[4] = 1.0
    A[5, 2] = -1.0                   # s = w2
    A[6, 1] = 1.0; A[6, 2] = 1.0; b[6] = 1.0
    cones = [(EXP, 3, 0.0), (EXP, 3, 0.0), (NONNEG, 1, 0.0)]
    return Problem(3, 7, sp.csr_matrix((3, 3)), np.array([1.0, 0, 0]), sp.csr_matrix(A), b, cones, "softplus"), \
        math.log1p(math.exp(u))


def entropy(n=5):
    """min sum x_i log x_i s.t. sum x = 1  ->  -log n  (epigraph (-t_i, x_i, 1) in K_exp)."""
    N = 2 * n  # variables x (n), t (n)
    rows, b = [], []
    A = np.zeros((1 + 3 * n, N))
    A[0, :n] = 1.0
    b = np.zeros(1 + 3 * n)
    b[0] = 1.0
    for i in range(n):
        r = 1 + 3 * i
        A[r, n + i] = 1.0            # s = -t_i
        A[r + 1, i] = -1.0           # s = x_i
        b[r + 2] = 1.0               # s = 1
    q = np.concatenate([np.zeros(n), np.ones(n)])
    cones = [(ZERO, 1, 0.0)] + [(EXP, 3, 0.0)] * n
    return Problem(N, 1 + 3 * n, sp.csr_matrix((N, N)), q, sp.csr_matrix(A), b, cones, "entropy"), -math.log(n)


def pow_max(alpha=1.0 / 3.0, x=2.0, y=8.0):
    """max z s.t. (x, y, z) in K_pow,alpha  ->  x^a y^(1-a)."""
    A = sp.csr_matrix(np.array([[0.0], [0.0], [-1.0]]))
    b = np.array([x, y, 0.0])
    return Problem(1, 3, sp.csr_matrix((1, 1)), np.array([-1.0]), A, b, [(POW, 3, alpha)], "pow_max"), \
        -(x ** alpha) * (y ** (1 - alpha))


def trace_min(seed=0, k=4):
    """min tr(CX) s.t. tr X = 1, X PSD  ->  lambda_min(C)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((k, k))
    Cm = G + G.T
    sd = k * (k + 1) // 2
    cvec = svec_encode(Cm[None])[0]
    ivec = svec_encode(np.eye(k)[None])[0]
    A = sp.vstack([sp.csr_matrix(ivec[None]), -sp.identity(sd)]).tocsr()
    b = np.concatenate([[1.0], np.zeros(sd)])
    return Problem(sd, sd + 1, sp.csr_matrix((sd, sd)), cvec, A, b, [(ZERO, 1, 0.0), (PSD, k, 0.0)], "trace_min"), \
        np.linalg.eigvalsh(Cm)[0]


def lqr(seed=0, T=12, nx=4, nu=2, x_scale=0.05):
    """MPC request with inactive limits -> finite-horizon LQR cost by the Riccati recursion."""
    from paper_2412_19027_amd.workloads import mpc_socp
    prob = mpc_socp(seed, 7, T=T, nx=nx, nu=nu, x_scale=x_scale)
    rng = np.random.default_rng(seed * 10**6 + 7)
    M = rng.standard_normal((nx, nx))
    Ad = 0.95 * M / np.abs(np.linalg.eigvals(M)).max()
    Bd = rng.standard_normal((nx, nu))
    x0 = x_scale * rng.standard_normal(nx)
    Q, R = np.eye(nx), 0.1 * np.eye(nu)
    V = Q.copy()
    for _ in range(T):
        K = np.linalg.solve(R + Bd.T @ V @ Bd, Bd.T @ V @ Ad)
        V = Q + Ad.T @ V @ (Ad - Bd @ K)
    return prob, 0.5 * x0 @ V @ x0


def infeasible_lp():
    """x >= 1 and x <= 0: primal infeasible."""
    A = sp.csr_matrix(np.array([[-1.0], [1.0]]))
    b = np.array([-1.0, 0.0])
    return Problem(1, 2, sp.csr_matrix((1, 1)), np.array([1.0]), A, b, [(NONNEG, 2, 0.0)], "infeasible_lp")


def unbounded_lp():
    """min -x s.t. x >= 0: dual infeasible."""
    A = sp.csr_matrix(np.array([[-1.0]]))
    b = np.array([0.0])
    return Problem(1, 1, sp.csr_matrix((1, 1)), np.array([-1.0]), A, b, [(NONNEG, 1, 0.0)], "unbounded_lp")


def infeasible_socp():
    """|(x1, x2)|_2 <= 1 and x1 >= 2: primal infeasible."""
    A = sp.csr_matrix(np.array([[0.0, 0.0], [-1.0, 0.0], [0.0, -1.0], [-1.0, 0.0]]))
    b = np.array([1.0, 0.0, 0.0, -2.0])
    return Problem(2, 4, sp.csr_matrix((2, 2)), np.array([1.0, 1.0]), A, b,
                   [(SOC, 3, 0.0), (NONNEG, 1, 0.0)], "infeasible_socp")


def unbounded_socp():
    """min -x1 s.t. (x1, x2, x3) in the second-order cone, x2 <= 1: dual infeasible."""
    A = sp.csr_matrix(np.array([[-1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]]))
    b = np.array([0.0, 0.0, 0.0, 1.0])
    return Problem(3, 4, sp.csr_matrix((3, 3)), np.array([-1.0, 0.0, 0.0]), A, b,
                   [(SOC, 3, 0.0), (NONNEG, 1, 0.0)], "unbounded_socp")


def random_small_lp(seed):
    """n <= 3, m <= 8 LP with box rows (bounded); optimum by vertex enumeration."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 4))
    mr = int(rng.integers(1, 3))
    G = rng.standard_normal((mr, n))
    h = G @ rng.uniform(-0.5, 0.5, n) + rng.uniform(0.1, 1, mr)
    A = np.vstack([G, np.eye(n), -np.eye(n)])
    b = np.concatenate([h, np.ones(n), np.ones(n)])
    c = rng.standard_normal(n)
    return Problem(n, A.shape[0], sp.csr_matrix((n, n)), c, sp.csr_matrix(A), b, [(NONNEG, A.shape[0], 0.0)],
                   f"random_small_lp({seed})")


def vertex_enumeration(prob):
    import itertools
    A = prob.A.toarray()
    b = prob.b
    best = np.inf
    for rows in itertools.combinations(range(A.shape[0]), prob.n):
        M = A[list(rows)]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, b[list(rows)])
        if np.all(A @ x <= b + 1e-9):
            best = min(best, prob.q @ x)
    return best
