"""The KKT layer at every interior-point iterate, GPU against the oracle.

The oracle runs the homogeneous-embedding iteration (Algorithm 1) on the CPU;
at each of its iterates the same (x, s, z, tau, kappa) is loaded into the GPU
solver (hc_set_iterate) and the GPU forms, at the scaling of that iterate
(Sec. 3.3, Appendix A), the three things one iteration needs:

* the Schur complement S = P + delta I + A'MA and its Cholesky factor
  (Sec. 3.7; hc_test_schur), against the oracle's S;
* one regularised solve and the unregularised product K [x; z]
  (hc_test_kkt_ops): the residual left by one regularised solve must be as
  small as the oracle's, which catches operators H and M = (H + delta I)^-1
  that are each right but not inverse to each other in floating point;
* the refined solve (hc_test_kkt_solve), against the oracle's.

Tolerances.  Early iterates agree to rounding.  Near the end the scalings of
the exponential and power cones depend on the conjugate point z~ of s, found
by Newton's method on a system whose condition grows like 1/mu; the oracle
and the GPU find it independently, so S and the solutions differ by up to
~1e-13/mu relative (measured 1.2e-4 at mu = 5e-9 on the exponential-cone case,
2.2e-4 at mu = 6e-10 on the PSD/power case).  The bound 1e-10 + 5e-12/mu
holds that with a margin of about 8x.  Problems with symmetric cones only
are held to 1e-10 + 5e-13/mu (largest measured 5.4e-14/mu).
"""
import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import ipm  # noqa: E402
from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402

CASES = [
    ("socp_small", lambda: W.sparse_socp(0, nx=600, rank=5, n_zero=150, n_nonneg=400, n_soc=500)),
    ("mpc_0", lambda: W.mpc_socp(0, 0)),
    ("exp_small", lambda: W.logreg_exp(0, samples=400, features=30)),
    ("psdpow_small", lambda: W.psd_pow(0, n=250, n_pow=120, n_psd=25, k=4)),
    ("multistage_small", lambda: W.multistage_portfolio(0, n=40, k=4, T=3)),
    ("multistage_dense_rows", lambda: W.multistage_portfolio(1, n=600, k=6, T=2)),
    # PSD sides 14 and 32 touch most of the 300 columns: their blocks enter S
    # through T = M_c A_c and a column gather, side 3 through row pairs
    ("psd_gathered", lambda: W.psd_mixed(0, n=300, sides=(3, 14, 32), per_side=6)),
]


def tol(mu, nonsym=True):
    """nonsym: the problem has exponential or power cones (conjugate points
    found independently on the two sides); symmetric cones only: 10x tighter
    (largest measured 5.4e-14/mu, the multistage case with rank-2 SOC rows)."""
    return 1e-10 + (5e-12 if nonsym else 5e-13) / mu


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name,make", CASES)
def test_kkt_layer_along_the_oracle_path(name, make):
    prob = make()
    nonsym = any(c[0] in (W.EXP, W.POW) for c in prob.cones)
    o = ipm.Solver(prob)
    g = HC.Solver(prob, leaf_blocks=0)
    if name == "psd_gathered":
        assert g.info()["psd_gathered_rows"] > 0, "the T = M_c A_c gather path was not taken"
    worst = 0.0
    perm = g.iterate()[5]                       # internal row -> user row

    def to_user(v):
        out = np.empty_like(v)
        out[perm] = v
        return out

    def load():
        g.set_iterate(o.x, o.s[perm], o.z[perm], o.tau, o.kappa)

    it = 0
    try:
        while o.check(o.residuals()) == 0:
            mu = o.mu()
            scal = o.scale(mu, False)
            kkt = o._kkt([(grp.rows, sc["Hb"]) for grp, sc in zip(o.groups, scal)])
            rng = np.random.default_rng(it)
            r1, r2 = rng.standard_normal(prob.n), rng.standard_normal(prob.m)
            nb = max(np.abs(r1).max(), np.abs(r2).max())
            case = f"{name} iterate {it} mu {mu:.2e}"

            load()
            Sg, Lg, st = g.test_schur(mu)
            So = (kkt.P + kkt.delta * sp.identity(prob.n) + kkt.A.T @ kkt.Mbd @ kkt.A).toarray()
            assert st["bits"] == 64 and abs(st["delta"] - kkt.delta) <= 1e-12 * kkt.delta, (case, st)
            assert rel(Sg, So) <= tol(mu, nonsym), (case, "S", rel(Sg, So))
            worst = max(worst, rel(Sg, So) * mu)
            assert np.abs(Lg @ Lg.T - Sg).max() <= 1e-14 * np.abs(Sg).max(), (case, "factor")

            load()
            xr, zr, kx, kz = g.test_kkt_ops(mu, r1, r2[perm])
            zr, kz = to_user(zr), to_user(kz)
            xo, zo = kkt.solve_reg(r1, r2)
            kxo, kzo = kkt.matvec(xo, zo)
            res_g = max(np.abs(r1 - kx).max(), np.abs(r2 - kz).max())
            res_o = max(np.abs(r1 - kxo).max(), np.abs(r2 - kzo).max())
            assert res_g <= 50 * res_o + 1e-10 * nb, (case, "one solve", res_g, res_o)
            # before refinement x carries cond(S) eps (the two sides solve S
            # differently: block inverses against LAPACK substitution)
            assert rel(xr, xo) <= max(tol(mu, nonsym), 1e-4), (case, "x of one solve", rel(xr, xo))

            load()
            xs, zs, info = g.test_kkt_solve(mu, r1, r2[perm])
            zs = to_user(zs)
            xo, zo, oinfo = kkt.solve(r1, r2, 1e-12, 1e-12, 10)
            assert rel(xs, xo) <= tol(mu, nonsym) and rel(zs, zo) <= tol(mu, nonsym), (case, rel(xs, xo), rel(zs, zo))
            worst = max(worst, rel(xs, xo) * mu, rel(zs, zo) * mu)
            assert info["solves"] <= oinfo["solves"] + 2, (case, info, oinfo)

            assert o.iterate() == 0, case
            it += 1
    finally:
        g.close()
    print(f"{name}: largest relative difference x mu = {worst:.2e}")
    assert it >= 5, (name, it)
