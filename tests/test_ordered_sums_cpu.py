"""The Schur complement's ordered sums (hc_test_ordered_sums, host only): the
products of A' M A grouped by the entry of S they land on reproduce, with
synthetic weights, every product added where it lands one by one (dense S,
the tail, a leaf's block, a leaf's coupling block); the leaf blocks' tail
updates are listed once each, under the tail entry their pair names.  The
cases cover the dense tail with three-row cones left to the pair terms
(n above the all-groups limit), the leaf/tail map with exponential cones
(logistic regression) and second-order cones (MPC), and small leaves."""
import pytest

from paper_2412_19027_amd import hipcone as HC
from paper_2412_19027_amd import workloads as W

CASES = {
    "dense_pairs": lambda: W.sparse_socp(0, nx=9000, rank=10, n_zero=4000, n_nonneg=12000, n_soc=16000),
    "leaves_logreg": lambda: W.logreg_exp(0, samples=2000, features=50),
    "leaves_mpc": lambda: W.mpc_socp(0, 3),
    "leaves_mpc_big": lambda: W.mpc_socp(0, 0, T=100, nx=12, nu=6),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ordered_sums_match_products(case):
    out = HC.ordered_sums_check(CASES[case]())
    assert out["ordered"] and out["destinations"] > 0, out
    assert out["rel_diff"] <= 1e-14, out
    assert out["bad_slots"] == 0, out


def test_ordered_sums_dense_tail_without_leaves():
    """leaf_blocks = 0: every column in the dense S, no leaf slots."""
    out = HC.ordered_sums_check(W.logreg_exp(0, samples=300, features=20), leaf_blocks=0)
    assert out["ordered"] and out["rel_diff"] <= 1e-14 and out["bad_slots"] == 0, out
