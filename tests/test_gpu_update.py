"""Parametric re-solve (hc_update_data): a solver set up for one problem
and given the values of another problem of the same structure solves that
problem as a fresh set-up does, against the oracle's objective."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import ipm  # noqa: E402
from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402
from tests.test_gpu_solver import certify  # noqa: E402


def same_structure(a, b):
    for M1, M2 in ((a.P.tocsr(), b.P.tocsr()), (a.A.tocsr(), b.A.tocsr())):
        if M1.shape != M2.shape or not (np.array_equal(M1.indptr, M2.indptr)
                                        and np.array_equal(M1.indices, M2.indices)):
            return False
    return a.cones == b.cones


PAIRS = [
    ("tiny_lp", lambda s: W.tiny_lp(s)),
    ("mpc", lambda s: W.mpc_socp(s, 7, T=40, nx=8, nu=3)),
    # SOCs of dimension 45 (rank-2 Schur rows) with new risk aversion,
    # transaction cost and inflow: new q and b on the same structure
    ("multistage", lambda s: W.multistage_portfolio(0, n=40, k=4, T=3, gamma=1.0 + s, cost=0.01 * (1 + s),
                                                    inflow=0.1 - 0.05 * s)),
    # PSD sides 14 and 32 assembled through T = M_c A_c and the column gather
    # (its value positions follow new A values): A scaled by 1.1, which keeps
    # the problem feasible (x / 1.1 and z / 1.1 are feasible)
    ("psd_gathered", lambda s: dataclasses.replace(
        W.psd_mixed(0, n=300, sides=(3, 14, 32), per_side=6),
        A=W.psd_mixed(0, n=300, sides=(3, 14, 32), per_side=6).A * (1.0 + 0.1 * s))),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make", PAIRS)
def test_update_solves_the_new_problem(name, make, precision):
    a, b = make(0), make(1)
    assert same_structure(a, b)
    ref = ipm.solve(b)
    assert ref.status == ipm.SOLVED
    s = HC.Solver(a, precision=precision)
    try:
        assert s.solve()["status_name"] == "solved"
        s.update_data(P_val=b.P.tocsr().data, q=b.q, A_val=b.A.tocsr().data, b=b.b)
        info = s.solve()
        x, sv, z = s.solution()
    finally:
        s.close()
    fresh = HC.Solver(b, precision=precision)
    try:
        finfo = fresh.solve()
        fx, _, _ = fresh.solution()
    finally:
        fresh.close()
    assert info["status_name"] == "solved" and finfo["status_name"] == "solved", (info, finfo)
    gp = certify(b, x, sv, z)
    assert abs(gp - ref.objective) <= 1e-7 * max(1.0, abs(ref.objective)), (gp, ref.objective)
    # same data, same algorithm: the same iterates up to the order of FP64 atomics
    assert info["iterations"] == finfo["iterations"]
    assert np.abs(x - fx).max() <= 1e-6 * max(1.0, np.abs(fx).max())


def test_update_only_b_is_a_new_initial_state():
    """The MPC re-solve of the paper's parametric setting: same dynamics,
    a new initial state (only b changes)."""
    a = W.mpc_socp(0, 3, T=30, nx=6, nu=2)
    other = W.mpc_socp(5, 3, T=30, nx=6, nu=2)
    b = W.Problem(a.n, a.m, a.P, a.q, a.A, a.b.copy(), a.cones, name="mpc new initial state")
    b.b[:6] = other.b[:6]          # the first nx rows fix x_0
    ref = ipm.solve(b)
    assert ref.status == ipm.SOLVED
    s = HC.Solver(a)
    try:
        s.solve()
        s.update_data(b=b.b)
        info = s.solve()
        x, sv, z = s.solution()
    finally:
        s.close()
    assert info["status_name"] == "solved", info
    gp = certify(b, x, sv, z)
    assert abs(gp - ref.objective) <= 1e-7 * max(1.0, abs(ref.objective)), (gp, ref.objective)


def test_rejected_update_changes_nothing():
    a = W.tiny_lp(2)
    s = HC.Solver(a)
    try:
        first = s.solve()
        bad = a.q.copy()
        bad[0] = np.nan
        with pytest.raises(HC.HipconeError) as e:
            s.update_data(q=bad)
        assert e.value.code == -5
        again = s.solve()
    finally:
        s.close()
    assert again["status_name"] == "solved"
    assert abs(again["obj_primal"] - first["obj_primal"]) <= 1e-9 * max(1.0, abs(first["obj_primal"]))


def mpc_sequence(T, nx, nu, steps, eps, seed=3):
    """Receding-horizon re-solves: one MPC problem whose initial state moves by
    a relative eps per step (new b on the same structure)."""
    base = W.mpc_socp(seed, 0, T=T, nx=nx, nu=nu)
    rng = np.random.default_rng(seed)
    seq = [base]
    for _ in range(steps):
        b = seq[-1].b.copy()
        b[:nx] = b[:nx] * (1.0 + eps * rng.standard_normal(nx))
        seq.append(dataclasses.replace(base, b=b))
    return seq


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_start_resolves(precision):
    """Parametric re-solves from the last solution (Sec. 4.6): every re-solve
    matches the oracle on its own data, with at least 30 % fewer iterations
    in total than solving each from the cold initial point."""
    seq = mpc_sequence(80, 10, 4, 6, 0.02)
    warm = HC.Solver(seq[0], precision=precision, warm_start=1)
    warm_it = cold_it = 0
    try:
        assert warm.solve()["status_name"] == "solved"
        for p in seq[1:]:
            warm.update_data(b=p.b)
            info = warm.solve()
            assert info["status_name"] == "solved"
            x, sv, z = warm.solution()
            gp = certify(p, x, sv, z)
            fo = ipm.solve(p).objective
            assert abs(gp - fo) <= 1e-7 * max(1.0, abs(fo)), (gp, fo)
            warm_it += info["iterations"]
            c = HC.Solver(p, precision=precision)
            cold_it += c.solve()["iterations"]
            c.close()
    finally:
        warm.close()
    print(f"{precision}: warm {warm_it} iterations, cold {cold_it}")
    assert warm_it <= 0.7 * cold_it, (warm_it, cold_it)
