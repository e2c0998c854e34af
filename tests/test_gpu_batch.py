"""The batched engine (one wavefront per problem, hc_solve_batch) against the
FP64 oracle: every problem of a batch of uneven MPC requests, small LPs and
second-order-cone problems, in FP64 and in mixed precision (objective 1e-7
relative, the optimality inequalities on the user's data at 1e-8), the
infeasibility certificates, and the same result alone and in a batch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import ipm  # noqa: E402
from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402
from tests import problems_small as PS  # noqa: E402
from tests.test_gpu_solver import MPC_STREAM, certify, mpc_reference  # noqa: E402


def batch_cases():
    probs = [mpc_reference(seed, i)[0] for seed, i in MPC_STREAM]
    probs += [W.tiny_lp(0), W.tiny_lp(1), PS.lqr()[0], PS.box_lp()[0], PS.soc_ball()[0]]
    return probs


_REF = {}


def oracle_objective(p):
    if p.name not in _REF:
        r = ipm.solve(p)
        assert r.status == ipm.SOLVED, p.name
        _REF[p.name] = r.objective
    return _REF[p.name]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_against_oracle(precision):
    probs = batch_cases()
    for p in probs:
        assert HC.batch_band(p, precision=precision) is not None, p.name
    print(f"batch {precision}: {len(probs)} problems", flush=True)
    res = HC.solve_batch(probs, precision=precision)
    for p, r in zip(probs, res):
        assert r["status_name"] == "solved", (p.name, r["status_name"], r["iterations"])
        gp = certify(p, r["x"], r["s"], r["z"])
        fo = oracle_objective(p)
        assert abs(gp - fo) <= 1e-7 * max(1.0, abs(fo)), (p.name, gp, fo)


def test_batch_infeasibility_certificates():
    probs = [PS.infeasible_lp(), PS.unbounded_lp(), PS.infeasible_socp(), PS.unbounded_socp()]
    want = [ipm.PRIMAL_INFEASIBLE, ipm.DUAL_INFEASIBLE, ipm.PRIMAL_INFEASIBLE, ipm.DUAL_INFEASIBLE]
    res = HC.solve_batch(probs)
    for p, r, st in zip(probs, res, want):
        assert ipm.solve(p).status == st
        assert r["status"] == st, (p.name, r["status_name"])
        if st == ipm.PRIMAL_INFEASIBLE:
            bz = p.b @ r["z"]
            assert bz < 0 and np.abs(p.A.T @ r["z"]).max() <= 1e-6 * abs(bz)
        else:
            assert p.q @ r["x"] < 0


def test_batch_alone_equals_in_the_mix():
    """A problem's result does not depend on what else is in the batch: each
    wave works on its own problem only, in a fixed order (bitwise equal)."""
    probs = batch_cases()
    mix = HC.solve_batch(probs)
    for k in (0, 5, len(probs) - 1):
        alone = HC.solve_batch([probs[k]])[0]
        assert alone["iterations"] == mix[k]["iterations"]
        assert np.array_equal(alone["x"], mix[k]["x"]) and np.array_equal(alone["z"], mix[k]["z"])


def test_batch_rejects_ineligible():
    with pytest.raises(HC.HipconeError) as e:
        HC.solve_batch([W.tiny_lp(0), PS.exp_max()[0]])
    assert e.value.code == HC.ERR_UNSUPPORTED
