"""The paper's entropy-maximisation and portfolio-QP problems (Sec. 4.4, 4.2) as
generated here, and the oracle's solutions of small instances pinned by
bounds that hold for any correct optimum."""
import numpy as np
import pytest

from oracle import ipm
from paper_2412_19027_amd import workloads as W


def test_entropy_max_shape_and_planted_point():
    n = 60
    p = W.entropy_max(3, n=n)
    m_in = round(0.5 * n)
    assert (p.n, p.m) == (2 * n, 1 + m_in + 3 * n)
    rng = np.random.default_rng(3)
    Ad = rng.standard_normal((m_in, n)) * np.sqrt(n)
    v = rng.uniform(0.0, 1.0, n)
    x = v / v.sum()
    # the planted point satisfies 1'x = 1 and A x <= b (with equality: b = A v / 1'v)
    A = p.A.toarray()
    assert np.allclose(A[0, :n], 1.0) and abs(p.b[0] - 1.0) == 0.0
    assert np.allclose(A[1:1 + m_in, :n], Ad) and np.allclose(A[1:1 + m_in, :n] @ x, p.b[1:1 + m_in])


@pytest.mark.parametrize("seed", [0, 1])
def test_entropy_max_oracle_bounds(seed):
    """max entropy over {x: 1'x = 1, Ax <= b} lies between the entropy of
    the planted feasible point v/1'v and log n (the unconstrained maximum)."""
    n = 80
    p = W.entropy_max(seed, n=n)
    r = ipm.solve(p)
    assert r.status == ipm.SOLVED
    rng = np.random.default_rng(seed)
    rng.standard_normal((round(0.5 * n), n))
    v = rng.uniform(0.0, 1.0, n)
    xh = v / v.sum()
    h_planted = -np.sum(xh * np.log(xh))
    h_opt = -r.objective
    assert h_planted - 1e-7 <= h_opt <= np.log(n) + 1e-9
    x, s, z = r.solution()
    xs = x[:n]
    assert abs(xs.sum() - 1.0) < 1e-7 and xs.min() > -1e-9
    # t_i <= -x_i log x_i, with equality at the optimum up to the tolerance
    assert abs(-np.sum(xs * np.log(np.maximum(xs, 1e-300))) - h_opt) < 1e-5


@pytest.mark.parametrize("seed", [0, 1])
def test_portfolio_qp_oracle_bounds(seed):
    """The optimum is no worse than the uniform portfolio or any single asset,
    and the oracle's x is a portfolio (1'x = 1, x >= 0) whose objective,
    recomputed from Sigma = F F' + D directly, matches."""
    n = 120
    p = W.portfolio_qp(seed, n=n)
    r = ipm.solve(p)
    assert r.status == ipm.SOLVED
    pr = max(1, round(0.1 * n))
    F = -p.A[:pr, :n].toarray().T                    # lift rows are y - F'x
    Dv = p.P.diagonal()[:n] / 2.0
    mu = -p.q[:n]
    Sigma = F @ F.T + np.diag(Dv)
    f = lambda x: x @ Sigma @ x - mu @ x           # gamma = 1
    assert r.objective <= f(np.full(n, 1.0 / n)) + 1e-8
    for j in np.argsort(-mu)[:3]:
        e = np.zeros(n)
        e[j] = 1.0
        assert r.objective <= f(e) + 1e-8
    x, s, z = r.solution()
    xs = x[:n]
    assert abs(xs.sum() - 1.0) < 1e-7 and xs.min() > -1e-8
    assert abs(f(xs) - r.objective) <= 1e-6 * max(1.0, abs(r.objective))


def test_psd_cones_of_several_sides_oracle():
    """PSD cones of sides 3, 5 and 8 interleaved in row order: the oracle
    groups them by side and solves; the solution satisfies the termination
    inequalities on the user's data and s, z are PSD cone by cone."""
    p = W.psd_mixed(0, n=120, sides=(2, 4, 6), per_side=6)
    r = ipm.solve(p)
    assert r.status == ipm.SOLVED
    x, s, z = r.solution()
    row = 0
    for kind, k, _ in p.cones:
        sd = k * (k + 1) // 2
        for v in (s, z):
            X = np.zeros((k, k))
            # svec: upper triangle column by column, off-diagonals scaled by sqrt 2
            vals = v[row:row + sd]
            idx = 0
            for j in range(k):
                for i in range(j + 1):
                    X[i, j] = X[j, i] = vals[idx] / (1.0 if i == j else np.sqrt(2.0))
                    idx += 1
            assert np.linalg.eigvalsh(X).min() > -1e-7
        row += sd
    assert abs(s @ z) <= 1e-6 * max(1.0, abs(r.objective))
