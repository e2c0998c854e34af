"""GPU whole-solver parity: hc_solve through the C-ABI against the FP64 CPU
oracle on the same seeded problems (objective 1e-7 relative, residuals 1e-8),
plus known optima."""
import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import ipm  # noqa: E402
from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402
from tests import problems_small as PS  # noqa: E402


def gpu_solve(prob, **kw):
    s = HC.Solver(prob, **kw)
    info = s.solve()
    x, sv, z = s.solution()
    s.close()
    return info, x, sv, z


def certify(prob, x, sv, z, eps=1e-8):
    P = prob.P + prob.P.T - sp.diags(prob.P.diagonal())
    rp = -(prob.A @ x) - sv + prob.b
    rd = P @ x + prob.A.T @ z + prob.q
    gp = 0.5 * x @ (P @ x) + prob.q @ x
    gd = -0.5 * x @ (P @ x) - prob.b @ z
    inf = lambda v: np.abs(v).max() if v.size else 0.0
    assert inf(rp) < eps * max(1, inf(prob.b) + inf(x) + inf(sv))
    assert inf(rd) < eps * max(1, inf(prob.q) + inf(x) + inf(z))
    assert abs(gp - gd) < eps * max(1, min(abs(gp), abs(gd)))
    return gp


@pytest.mark.parametrize("make", [PS.box_lp, PS.soc_ball, PS.exp_max, PS.softplus, PS.entropy, PS.pow_max,
                                  PS.trace_min, PS.lqr, PS.soc_balls, PS.soc_ball_budget,
                                  lambda: PS.trace_min(0, k=24), lambda: PS.trace_min(1, k=32)])
def test_known_optimum(make):
    prob, fstar = make()
    info, x, sv, z = gpu_solve(prob)
    assert info["status_name"] == "solved", info
    certify(prob, x, sv, z)
    assert abs(info["obj_primal"] - fstar) <= 1e-6 * max(1.0, abs(fstar))


CASES = [
    ("tiny_lp_0", lambda: W.tiny_lp(0)),
    ("tiny_lp_1", lambda: W.tiny_lp(1)),
    ("socp_small", lambda: W.sparse_socp(0, nx=600, rank=5, n_zero=150, n_nonneg=400, n_soc=500)),
    ("mpc_0", lambda: W.mpc_socp(0, 0)),
    ("exp_small", lambda: W.logreg_exp(0, samples=400, features=30)),
    ("psdpow_small", lambda: W.psd_pow(0, n=250, n_pow=120, n_psd=25, k=4)),
    ("entropy_small", lambda: W.entropy_max(0, n=200)),
    # rows of more than 512 entries go through the dense-row path, here together
    # with leaf blocks (the t variables)
    ("entropy_dense_rows", lambda: W.entropy_max(0, n=600)),
    ("portfolio_small", lambda: W.portfolio_qp(0, n=300)),
    ("psd_mixed_sides", lambda: W.psd_mixed(0)),
    # sides above 12 (two cones per workgroup, up to the paper's 32) beside a small one
    ("psd_sides_to_32", lambda: W.psd_mixed(0, n=300, sides=(3, 14, 32), per_side=6)),
    # second-order cones above 16 rows (one workgroup per cone, diagonal plus
    # rank-2 Schur form): several dims, with leaf blocks (the z variables),
    # and with dense budget rows on the same columns
    ("multistage_small", lambda: W.multistage_portfolio(0, n=40, k=4, T=3)),
    ("multistage_dense_rows", lambda: W.multistage_portfolio(1, n=600, k=6, T=2)),
    # SOC dimension 16, the largest on the lane-per-cone path (a withdrawal
    # instead of an inflow: with 12 assets capped at 0.1 a budget of 1.1
    # leaves y_t = F_t x_t >= 0 infeasible)
    ("multistage_dim16", lambda: W.multistage_portfolio(2, n=12, k=3, T=2, inflow=-0.5)),
    # a tail of 2,040 columns in ten stages (three panels) whose envelope ends
    # one stage below each column: envelope-limited TRSM and updates
    ("multistage_panels", lambda: W.multistage_portfolio(3, n=200, k=3, T=10)),
]

@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_against_oracle(name, make, precision):
    prob = make()
    ref = ipm.solve(prob)
    assert ref.status == ipm.SOLVED
    info, x, sv, z = gpu_solve(prob, precision=precision)
    assert info["status_name"] == "solved", (name, info)
    gp = certify(prob, x, sv, z)
    assert abs(gp - ref.objective) <= 1e-7 * max(1.0, abs(ref.objective)), (gp, ref.objective)


@pytest.mark.parametrize("name,make", [
    ("psd_sides_to_32", lambda: W.psd_mixed(0, n=300, sides=(3, 14, 32), per_side=6)),
    ("trace_min_32", lambda: PS.trace_min(1, k=32)[0]),
    ("soc_balls", lambda: PS.soc_balls()[0]),
    ("multistage_small", lambda: W.multistage_portfolio(0, n=40, k=4, T=3)),
])
def test_initial_point_against_oracle(name, make):
    """The starting iterate before any iteration (Section 2.2: a KKT solve with
    identity scaling, then s and z each moved along e by one plus the largest
    negative cone eigenvalue when it is not positive) against the oracle's,
    in the scaled internal coordinates and row order."""
    prob = make()
    o = ipm.Solver(prob)
    g = HC.Solver(prob, max_iter=0)
    try:
        g.solve()
        x, s, z, tau, kappa, perm = g.iterate()
    finally:
        g.close()
    for a, b, what in ((x, o.x, "x"), (s, o.s[perm], "s"), (z, o.z[perm], "z")):
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        assert err <= 1e-9, (name, what, err)
    assert tau == 1.0 and kappa == 1.0


@pytest.mark.parametrize("name,make,status", [
    ("infeasible_lp", PS.infeasible_lp, ipm.PRIMAL_INFEASIBLE),
    ("unbounded_lp", PS.unbounded_lp, ipm.DUAL_INFEASIBLE),
    ("infeasible_socp", PS.infeasible_socp, ipm.PRIMAL_INFEASIBLE),
    ("unbounded_socp", PS.unbounded_socp, ipm.DUAL_INFEASIBLE),
])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_infeasibility_certificates(name, make, status, precision):
    """eq. infeasibility-check on the GPU: the same status as the oracle, and
    the certificate hc_get_solution returns meets the inequalities on the
    user's data and lies in the dual (resp. primal) cone."""
    prob = make()
    ref = ipm.solve(prob)
    assert ref.status == status
    info, x, sv, z = gpu_solve(prob, precision=precision)
    assert info["status"] == status, (name, info)
    if status == ipm.PRIMAL_INFEASIBLE:
        bz = prob.b @ z
        assert bz < 0 and np.abs(prob.A.T @ z).max() <= 1e-6 * abs(bz), (bz, prob.A.T @ z)
        soc = z[: 3] if name == "infeasible_socp" else None
        if soc is not None:
            assert soc[0] >= np.linalg.norm(soc[1:]) - 1e-9 * abs(bz) and z[3] >= -1e-9 * abs(bz)
        else:
            assert np.all(z >= -1e-9 * abs(bz))
    else:
        qx = prob.q @ x
        w = -(prob.A @ x)
        assert qx < 0
        if name == "unbounded_socp":
            assert w[0] >= np.linalg.norm(w[1:3]) - 1e-9 * abs(qx) and w[3] >= -1e-9 * abs(qx)
        else:
            assert np.all(w >= -1e-9 * abs(qx))


def test_solution_on_device_matches_host():
    """hc_get_solution with on_device: the same values as the host form."""
    for prob in (W.mpc_socp(0, 3), PS.infeasible_lp()):
        s = HC.Solver(prob)
        s.solve()
        xh, sh, zh = s.solution()
        xd, sd, zd = s.solution(on_device=True)
        s.close()
        assert np.array_equal(xh, xd.cpu().numpy())
        assert np.array_equal(sh, sd.cpu().numpy())
        assert np.array_equal(zh, zd.cpu().numpy())


# 24 requests of the served MPC stream's generator (horizons 10..100, 4..12
# states, 2..6 inputs), each against the oracle
MPC_STREAM = [(7, i) for i in range(24)]
_MPC_REF = {}


def mpc_reference(seed, i):
    if (seed, i) not in _MPC_REF:
        prob = W.mpc_socp(seed, i)
        ref = ipm.solve(prob)
        assert ref.status == ipm.SOLVED
        _MPC_REF[(seed, i)] = (prob, ref.objective)
    return _MPC_REF[(seed, i)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mpc_stream_against_oracle(precision):
    sizes = set()
    for seed, i in MPC_STREAM:
        prob, fo = mpc_reference(seed, i)
        sizes.add(prob.n)
        info, x, sv, z = gpu_solve(prob, precision=precision)
        assert info["status_name"] == "solved", (prob.name, info)
        gp = certify(prob, x, sv, z)
        assert abs(gp - fo) <= 1e-7 * max(1.0, abs(fo)), (prob.name, gp, fo)
    assert max(sizes) > 4 * min(sizes)


@pytest.mark.parametrize("make", [lambda: W.psd_pow(0, n=250, n_pow=120, n_psd=25, k=4),
                                  lambda: W.psd_mixed(0, n=300, sides=(3, 5, 8), per_side=20)],
                         ids=["psd_pow_small", "psd_mixed_small"])
def test_schur_assembly_deterministic(make):
    """Problems whose Schur columns fit two gather chunks assemble S with one
    writer per entry in a fixed order (no atomics): two solves agree bit for
    bit, iterations and solution."""
    prob = make()
    runs = []
    for _ in range(2):
        s = HC.Solver(prob)
        info = s.solve()
        x, sv, z = s.solution()
        s.close()
        assert info["status_name"] == "solved", info
        runs.append((info["iterations"], x, z))
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profile_mode_serial_schedule(precision):
    """settings.profile = 2 issues the look-ahead factorisation's launches one
    at a time on the handle's stream (for per-launch timing).  A dense tail of
    four 768-column panels, so both trailing updates of the look-ahead run:
    the timed schedule reaches the same solution as the overlapped one (each
    entry of S receives its updates in the same order; the pair assembly's
    atomics may reorder sums, hence a tolerance rather than bitwise)."""
    prob = W.sparse_socp(0, nx=2500, rank=5, n_zero=1250, n_nonneg=3750, n_soc=5000)
    runs = []
    for profile in (0, 2):
        s = HC.Solver(prob, precision=precision, profile=profile)
        info = s.solve()
        x, sv, z = s.solution()
        s.close()
        assert info["status_name"] == "solved", info
        runs.append((info, x, sv, z))
    (ia, xa, _, _), (ib, xb, sb, zb) = runs
    assert ib["n_ordered"] > 2 * 768, ib["n_ordered"]
    assert ib["gemm_launches"] > 0 and ib["gemm_ms"] > 0
    assert ia["iterations"] == ib["iterations"]
    assert abs(ia["obj_primal"] - ib["obj_primal"]) <= 1e-9 * max(1.0, abs(ia["obj_primal"]))
    assert np.abs(xa - xb).max() <= 1e-6 * max(1.0, np.abs(xa).max())
    certify(prob, xb, sb, zb)


@pytest.mark.parametrize("make", [lambda: W.mpc_socp(0, 3),
                                  lambda: W.sparse_socp(0, nx=600, rank=5, n_zero=150, n_nonneg=400, n_soc=500)],
                         ids=["mpc", "socp_small"])
def test_bind_with_caller_pinned_stage(make):
    """hc_bind with a caller-owned arena and caller-owned pinned read-back
    staging (the form the served form's per-slot workers use) solves as with
    the library's own staging.  Binding once checked the staging size by a
    dry run of the allocation that reset the handle's device pointers."""
    prob = make()
    a, xa, _, _ = gpu_solve(prob)
    b, xb, sb, zb = gpu_solve(prob, pinned_stage=True)
    assert a["status_name"] == b["status_name"] == "solved", (a, b)
    assert a["iterations"] == b["iterations"]
    assert abs(a["obj_primal"] - b["obj_primal"]) <= 1e-9 * max(1.0, abs(a["obj_primal"]))
    assert np.abs(xa - xb).max() <= 1e-6 * max(1.0, np.abs(xa).max())
    certify(prob, xb, sb, zb)
