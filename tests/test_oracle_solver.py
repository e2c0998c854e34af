"""Whole-oracle pins: known optima, independent library solvers (HiGHS),
vertex enumeration, the Riccati recursion, infeasibility certificates, the
4x4 Newton system and the KKT solve against numpy.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

from oracle import ipm
from oracle.linsys import KKT, SpectralBlocks
from paper_2412_19027_amd import workloads as W
from tests import problems_small as PS


def solved(prob, **kw):
    s = ipm.solve(prob, **kw)
    assert s.status == ipm.SOLVED, (prob.name, ipm.STATUS_NAMES[s.status])
    return s


def certify(s, prob, eps=1e-8):
    """Re-check the optimality inequalities on the user's data."""
    x, sv, z = s.solution()
    P = prob.P + prob.P.T - sp.diags(prob.P.diagonal())
    rp = -(prob.A @ x) - sv + prob.b
    rd = P @ x + prob.A.T @ z + prob.q
    gp = 0.5 * x @ (P @ x) + prob.q @ x
    gd = -0.5 * x @ (P @ x) - prob.b @ z
    inf = lambda v: np.abs(v).max() if v.size else 0.0
    assert inf(rp) < eps * max(1, inf(prob.b) + inf(x) + inf(sv))
    assert inf(rd) < eps * max(1, inf(prob.q) + inf(x) + inf(z))
    assert abs(gp - gd) < eps * max(1, min(abs(gp), abs(gd)))


@pytest.mark.parametrize("make", [PS.box_lp, PS.soc_ball, PS.exp_max, PS.softplus, PS.entropy,
                                  PS.pow_max, PS.trace_min, PS.lqr, PS.soc_balls, PS.soc_ball_budget,
                                  lambda: PS.trace_min(1, k=32)])
def test_known_optimum(make):
    prob, fstar = make()
    s = solved(prob)
    certify(s, prob)
    assert abs(s.objective - fstar) <= 1e-6 * max(1.0, abs(fstar)), (s.objective, fstar)


@pytest.mark.parametrize("seed", range(6))
def test_random_lp_vertex_enumeration(seed):
    prob = PS.random_small_lp(seed)
    s = solved(prob)
    assert abs(s.objective - PS.vertex_enumeration(prob)) < 1e-6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_lp_against_highs(seed):
    prob = W.tiny_lp(seed)
    s = solved(prob)
    certify(s, prob)
    r = linprog(prob.q, A_ub=prob.A.toarray(), b_ub=prob.b, bounds=[(None, None)] * prob.n, method="highs")
    assert abs(s.objective - r.fun) <= 1e-7 * abs(r.fun)


def test_primal_infeasible_certificate():
    prob = PS.infeasible_lp()
    s = ipm.solve(prob)
    assert s.status == ipm.PRIMAL_INFEASIBLE
    z = s.E * s.z / s.c
    assert prob.b @ z < 0 and np.all(z >= -1e-12)
    assert np.abs(prob.A.T @ z).max() <= 1e-6 * abs(prob.b @ z)


def test_dual_infeasible_certificate():
    prob = PS.unbounded_lp()
    s = ipm.solve(prob)
    assert s.status == ipm.DUAL_INFEASIBLE
    x = s.D * s.x
    assert prob.q @ x < 0 and np.all(-(prob.A @ x) >= -1e-12)


def test_socp_infeasibility_certificates():
    """Second-order-cone cases of eq. infeasibility-check: the certificate
    lies in the dual (resp. primal) cone and meets the inequalities."""
    prob = PS.infeasible_socp()
    s = ipm.solve(prob)
    assert s.status == ipm.PRIMAL_INFEASIBLE
    z = s.E * s.z / s.c
    assert prob.b @ z < 0 and np.abs(prob.A.T @ z).max() <= 1e-6 * abs(prob.b @ z)
    assert z[0] >= np.linalg.norm(z[1:3]) - 1e-12 and z[3] >= -1e-12
    prob = PS.unbounded_socp()
    s = ipm.solve(prob)
    assert s.status == ipm.DUAL_INFEASIBLE
    x = s.D * s.x
    w = -(prob.A @ x)
    assert prob.q @ x < 0 and w[0] >= np.linalg.norm(w[1:3]) - 1e-9 * abs(prob.q @ x) and w[3] >= -1e-12


@pytest.mark.parametrize("make", [lambda: W.sparse_socp(1, nx=300, rank=4, n_zero=60, n_nonneg=200, n_soc=200),
                                  lambda: W.logreg_exp(1, samples=200, features=15),
                                  lambda: W.psd_pow(1, n=150, n_pow=60, n_psd=12, k=3)])
def test_newton_system_residual(make):
    """The recovered direction satisfies the 4x4 linearised system (eq. linsys_4x4)."""
    prob = make()
    s = ipm.Solver(prob)
    for _ in range(3):
        s.iterate()
    mu = s.mu()
    scal = s.scale(mu)
    kkt = s._kkt([(g.rows, sc["Hb"]) for g, sc in zip(s.groups, scal)])
    c2 = s._solve(kkt, -s.qs, s.bs)
    gx, gz, gt = s.G()
    d = s.direction(kkt, scal, gx, gz, gt, s.s.copy(), s.kappa * s.tau, c2)
    xi = s.x / s.tau
    scale = max(np.abs(gx).max(), np.abs(gz).max(), abs(gt))
    ra = -(s.Ps @ d["x"] + s.As.T @ d["z"] + s.qs * d["tau"]) + gx
    rb = d["s"] + s.As @ d["x"] - s.bs * d["tau"] + gz
    rc = d["kappa"] + (s.qs + 2 * s.Ps @ xi) @ d["x"] + s.bs @ d["z"] - xi @ (s.Ps @ xi) * d["tau"] + gt
    rd = s.H_apply(scal, d["z"]) + d["s"] + s.s
    re = s.kappa * d["tau"] + s.tau * d["kappa"] + s.kappa * s.tau
    for r in (ra, rb, np.atleast_1d(rc), rd, np.atleast_1d(re)):
        assert np.abs(r).max() < 1e-9 * scale


def test_kkt_solve_against_numpy():
    rng = np.random.default_rng(3)
    n, m = 30, 45
    A = sp.random(m, n, density=0.2, random_state=4, format="csr") + sp.vstack([sp.identity(n), sp.csr_matrix((m - n, n))])
    P = sp.diags(rng.uniform(0.1, 1, n)).tocsr()
    rows = np.arange(m).reshape(15, 3)
    G = rng.standard_normal((15, 3, 3))
    H = np.einsum("cij,ckj->cik", G, G) + 0.1 * np.eye(3)
    lam, V = np.linalg.eigh(H)
    kkt = KKT(P, A, [(rows, SpectralBlocks(lam, V))], 1e-8, 0.0)
    r1, r2 = rng.standard_normal(n), rng.standard_normal(m)
    x, z, info = kkt.solve(r1, r2)
    K = np.zeros((n + m, n + m))
    K[:n, :n] = P.toarray(); K[n:, :n] = A.toarray(); K[:n, n:] = A.toarray().T
    for c in range(15):
        K[np.ix_(n + rows[c], n + rows[c])] = -H[c]
    ref = np.linalg.solve(K, np.concatenate([r1, r2]))
    assert np.abs(np.concatenate([x, z]) - ref).max() < 1e-10 * np.abs(ref).max()
    assert info["resid"] <= 1e-12 + 1e-12 * max(np.abs(r1).max(), np.abs(r2).max())
    # inertia of the regularised KKT: n positive and m negative eigenvalues
    Kr = K.copy(); Kr[:n, :n] += kkt.delta * np.eye(n); Kr[n:, n:] -= kkt.delta * np.eye(m)
    ev = np.linalg.eigvalsh(Kr)
    assert (ev > 0).sum() == n and (ev < 0).sum() == m


@pytest.mark.parametrize("make", [lambda: W.sparse_socp(2, nx=300, rank=4, n_zero=60, n_nonneg=200, n_soc=200),
                                  lambda: W.mpc_socp(0, 3),
                                  lambda: W.logreg_exp(2, samples=200, features=15),
                                  lambda: W.psd_pow(2, n=150, n_pow=60, n_psd=12, k=3)])
def test_family_instances_certify(make):
    prob = make()
    s = solved(prob)
    certify(s, prob)
