"""hc_solve_noalloc (the allocation-free solve in the library's static
device workspace) against the existing path hc_bind + hc_solve +
hc_get_solution, through the C-ABI: two calls in a row on one device, the
second with a smaller problem, each to the parity bar of the whole-solve
tests (objective 1e-7 relative, the optimality inequalities on the user's
data, and the iterate itself)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402
from tests.test_gpu_solver import certify, gpu_solve  # noqa: E402


def close(a, b, rtol):
    return np.abs(a - b).max() <= rtol * max(1.0, np.abs(b).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_bound_solve_two_calls(precision):
    big = W.mpc_socp(0, 0, T=100, nx=12, nu=6)      # the largest request shape of the served stream
    small = W.mpc_socp(0, 1, T=12, nx=4, nu=2)
    assert HC.analyze(big, precision=precision)["workspace_bytes"] <= HC.NOALLOC_BYTES
    for prob in (big, small):
        print(f"noalloc {precision}: {prob.name}", flush=True)
        info_r, xr, sr, zr = gpu_solve(prob, precision=precision)
        info, x, s, z = HC.solve_noalloc(prob, precision=precision)
        assert info_r["status_name"] == "solved" and info["status_name"] == "solved", (info_r, info)
        gp = certify(prob, x, s, z)
        assert abs(gp - info_r["obj_primal"]) <= 1e-7 * max(1.0, abs(info_r["obj_primal"]))
        assert close(x, xr, 1e-6) and close(s, sr, 1e-6) and close(z, zr, 1e-6)
        assert info["iterations"] == info_r["iterations"]


def test_noalloc_dense_tail_and_rejects_oversize():
    """A problem with a dense tail of several look-ahead panels (its launches
    then run on the caller's stream alone), then one whose workspace exceeds
    the static array: rejected with HC_ERR_TOO_LARGE before any device work."""
    prob = W.sparse_socp(0, nx=1600, rank=5, n_zero=400, n_nonneg=1200, n_soc=1600)
    assert HC.analyze(prob)["workspace_bytes"] <= HC.NOALLOC_BYTES
    info_r, xr, _, _ = gpu_solve(prob)
    info, x, s, z = HC.solve_noalloc(prob)
    assert info["status_name"] == "solved" and info["n_ordered"] > 768
    assert info["iterations"] == info_r["iterations"] and close(x, xr, 1e-6)
    certify(prob, x, s, z)
    big = W.sparse_socp(0, nx=3000, rank=5, n_zero=500, n_nonneg=2000, n_soc=2000)
    assert HC.analyze(big)["workspace_bytes"] > HC.NOALLOC_BYTES
    with pytest.raises(HC.HipconeError) as e:
        HC.solve_noalloc(big)
    assert e.value.code == HC.ERR_TOO_LARGE
