"""Run-to-run reproducibility: the Schur complement is assembled by ordered
sums (every entry one sum in a fixed order, no floating-point atomics), so two
solves of one problem, on two handles or twice on one, give bitwise equal
iterates, iteration counts and solutions.  The cases cover the ordered pair
sums on a dense tail (n above the all-groups limit, three-row cones left to
the pair terms), through the leaf/tail column map with the leaves' slot sums
(logistic regression, MPC), and the column-ordered T rows of large PSD cones."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402

CASES = {
    "dense_pairs": lambda: W.sparse_socp(0, nx=9000, rank=10, n_zero=4000, n_nonneg=12000, n_soc=16000),
    "leaves_logreg": lambda: W.logreg_exp(0, samples=2000, features=50),
    "leaves_mpc": lambda: W.mpc_socp(0, 3),
    "psd_dense_T": lambda: W.psd_mixed(0, sides=(3, 14, 32), per_side=10),
}


def run(prob, solver=None, **kw):
    s = solver or HC.Solver(prob, **kw)
    info = s.solve()
    x, sv, z = s.solution()
    return s, info, x, sv, z


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_two_solves_bitwise_equal(case, precision):
    prob = CASES[case]()
    print(case, precision, prob.n, prob.m, flush=True)
    s1, i1, x1, s1v, z1 = run(prob, precision=precision)
    s2, i2, x2, s2v, z2 = run(prob, precision=precision)
    _, i3, x3, s3v, z3 = run(prob, solver=s1)
    s1.close()
    s2.close()
    assert i1["status_name"] == "solved", i1
    for info, x, sv, z in ((i2, x2, s2v, z2), (i3, x3, s3v, z3)):
        assert info["iterations"] == i1["iterations"]
        assert info["obj_primal"] == i1["obj_primal"]
        assert np.array_equal(x, x1) and np.array_equal(sv, s1v) and np.array_equal(z, z1)
