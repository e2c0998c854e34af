"""Pins of the oracle's combined-step right-hand side (eq. ds-correction-step),
of its Hessian-inverse application for exp/pow cones and of its step rule with
the neighbourhood check N(beta) (Sec. 2.2, "Update iterates").

Each expected value here is computed by a route the oracle does not take:
Jordan-algebra inverses from numpy.linalg.inv, arrow products written out,
third derivatives by central differences of the (separately pinned) jet
Hessian, the conjugate point by a damped Newton method instead of the
oracle's bisection, and the step by walking alpha_0 * 0.8^k by hand.  A
swapped W / W^-T, a sign error in the Mehrotra or third-order term, a wrong
factor in front of it, or a neighbourhood test on the wrong quantity fails one
of them.  CPU only."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cones as C
from oracle import ipm
from oracle import jets
from paper_2412_19027_amd.workloads import Problem
from tests.test_oracle_cones import exp_dual, exp_primal, pow_dual, pow_primal, soc_interior, spd

RNG = np.random.default_rng(4242)
SQ2 = math.sqrt(2.0)


# ------------------------------------------------------------------ helpers of the test's own
def svec_t(X):
    """Upper triangle column by column, off-diagonal entries times sqrt(2)."""
    k = X.shape[-1]
    out = []
    for j in range(k):
        for i in range(j + 1):
            out.append(X[..., i, j] * (1.0 if i == j else SQ2))
    return np.stack(out, axis=-1)


def smat_t(v, k):
    X = np.zeros(v.shape[:-1] + (k, k))
    c = 0
    for j in range(k):
        for i in range(j + 1):
            if i == j:
                X[..., i, i] = v[..., c]
            else:
                X[..., i, j] = X[..., j, i] = v[..., c] / SQ2
            c += 1
    return X


def arrow(x, y):
    """SOC Jordan product x o y = (x'y, x0 y1 + y0 x1)."""
    return np.concatenate([np.sum(x * y, axis=1, keepdims=True),
                           x[:, :1] * y[:, 1:] + y[:, :1] * x[:, 1:]], axis=1)


def scaling_state(kind, s, z, k=0):
    if kind == ipm.NONNEG:
        return C.nn_scale(s, z)
    if kind == ipm.SOC:
        return C.soc_scale(s, z)
    return C.psd_scale(s, z, k)


# ------------------------------------------------------------------ symmetric cones
@pytest.mark.parametrize("case", [("nonneg", 1), ("soc", 3), ("soc", 7), ("soc", 60),
                                  ("psd", 3), ("psd", 10), ("psd", 32)])
def test_ds_zero_affine_step_is_s_minus_sigma_mu_zinv(case):
    """With ds_a = dz_a = 0 the corrected RHS is d_s = s - sigma mu z^-1, z^-1
    the Jordan-algebra inverse: nonneg 1/z, SOC Jz/(z'Jz), PSD svec(Z^-1)."""
    name, d = case
    N = 40 if d < 32 else 6
    sm = 0.37
    if name == "nonneg":
        kind = ipm.NONNEG
        s, z = RNG.uniform(0.1, 3, (N, 1)), RNG.uniform(0.1, 3, (N, 1))
        zinv = 1.0 / z
    elif name == "soc":
        kind = ipm.SOC
        s, z = soc_interior(N, d, RNG), soc_interior(N, d, RNG)
        Jz = z.copy()
        Jz[:, 1:] *= -1.0
        zinv = Jz / np.sum(z * Jz, axis=1, keepdims=True)
    else:
        kind = ipm.PSD
        S, Z = spd(N, d, RNG), spd(N, d, RNG)
        s, z = svec_t(S), svec_t(Z)
        zinv = svec_t(np.linalg.inv(Z))
    sc = scaling_state(kind, s, z, d)
    zero = np.zeros_like(s)
    ds = ipm.ds_family(kind, s, z, sc, zero, zero, sm, k=d)
    ref = s - sm * zinv
    assert np.abs(ds - ref).max() <= 1e-11 * np.abs(ref).max()


def test_ds_nonneg_closed_form():
    """Nonneg: d_s = (s z + ds_a dz_a - sigma mu) / z."""
    s, z = RNG.uniform(0.05, 3, (500, 1)), RNG.uniform(0.05, 3, (500, 1))
    a, b = RNG.standard_normal((500, 1)), RNG.standard_normal((500, 1))
    sm = 0.2
    ds = ipm.ds_family(ipm.NONNEG, s, z, C.nn_scale(s, z), a, b, sm)
    ref = (s * z + a * b - sm) / z
    assert np.abs(ds - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("d", [3, 5, 40])
def test_ds_soc_linearised_complementarity(d):
    """SOC: lambda o (W^-T d_s) = lambda o lambda + (W^-T ds_a) o (W dz_a) - sigma mu e,
    with W^-T from numpy.linalg.inv and the arrow product written out."""
    N = 50
    s, z = soc_interior(N, d, RNG), soc_interior(N, d, RNG)
    a, b = 0.4 * RNG.standard_normal((N, d)), 0.4 * RNG.standard_normal((N, d))
    sm = 0.11
    sc = C.soc_scale(s, z)
    ds = ipm.ds_family(ipm.SOC, s, z, sc, a, b, sm)
    W = sc["W"]
    WinvT = np.linalg.inv(W).transpose(0, 2, 1)
    lam = np.einsum("cij,cj->ci", W, z)                # lambda = W z
    e = np.zeros((N, d))
    e[:, 0] = 1.0
    lhs = arrow(lam, np.einsum("cij,cj->ci", WinvT, ds))
    rhs = arrow(lam, lam) + arrow(np.einsum("cij,cj->ci", WinvT, a), np.einsum("cij,cj->ci", W, b)) - sm * e
    assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(rhs).max()


@pytest.mark.parametrize("k", [2, 3, 10, 32])
def test_ds_psd_linearised_complementarity(k):
    """PSD with W(X) = R'XR, W^-T(X) = R^-1 X R^-T and Lambda = R'ZR:
    Lambda o Y = Lambda^2 + A o B - sigma mu I for Y = W^-T(D_s), A = W^-T(dS_a),
    B = W(dZ_a), where X o Y = (XY + YX)/2 and R^-1 comes from numpy.linalg.inv."""
    N = 12 if k < 32 else 3
    S, Z = spd(N, k, RNG), spd(N, k, RNG)
    s, z = svec_t(S), svec_t(Z)
    a, b = 0.3 * RNG.standard_normal(s.shape), 0.3 * RNG.standard_normal(s.shape)
    sm = 0.23
    sc = C.psd_scale(s, z, k)
    ds = ipm.ds_family(ipm.PSD, s, z, sc, a, b, sm, k=k)
    R = sc["R"]
    Ri = np.linalg.inv(R)
    RiT = Ri.transpose(0, 2, 1)
    RT = R.transpose(0, 2, 1)
    Lam = RT @ Z @ R
    off = np.abs(Lam - np.einsum("cii->ci", Lam)[:, :, None] * np.eye(k)[None]).max()
    assert off <= 1e-10 * np.abs(Lam).max()          # the scaling point diagonalises
    Y = Ri @ smat_t(ds, k) @ RiT
    Aa = Ri @ smat_t(a, k) @ RiT
    Bb = RT @ smat_t(b, k) @ R
    jordan = lambda X, Y_: 0.5 * (X @ Y_ + Y_ @ X)    # noqa: E731
    lhs = jordan(Lam, Y)
    rhs = Lam @ Lam + jordan(Aa, Bb) - sm * np.eye(k)[None]
    assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max()


# ------------------------------------------------------------------ exp / pow cones
def _nonsym_points(kind, N):
    if kind == "exp":
        return exp_primal(N, RNG), exp_dual(N, RNG), None, C.f_exp
    alpha = RNG.uniform(0.2, 0.8, N)
    return pow_primal(N, alpha, RNG), pow_dual(N, alpha, RNG), alpha, C.f_pow


@pytest.mark.parametrize("kind", ["exp", "pow"])
def test_hinv_apply_against_linear_solve(kind):
    """Hess f(z)^-1 v from the factor's SVD equals numpy.linalg.solve on the jet Hessian."""
    N = 60
    s, z, alpha, f = _nonsym_points(kind, N)
    fam = C.NonsymFamily(kind, alpha)
    sc = fam.scale(s, z, 0.7)
    v = RNG.standard_normal((N, 3))
    _, Hf = jets.derivatives(f, z, alpha)
    ref = np.linalg.solve(Hf, v[..., None])[..., 0]
    got = fam.hinv_apply(sc["hinv"], v)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("kind", ["exp", "pow"])
def test_ds_nonsym_third_order_term_by_finite_differences(kind):
    """d_s - s - sigma mu grad f(z) = -1/2 grad^3 f(z)[dz_a, Hf^-1 ds_a]; the
    directional third derivative is taken as a central difference of the jet
    Hessian along dz_a, and Hf^-1 ds_a by numpy.linalg.solve."""
    N = 40
    s, z, alpha, f = _nonsym_points(kind, N)
    fam = C.NonsymFamily(kind, alpha)
    mu, sm = 0.9, 0.3
    sc = fam.scale(s, z, mu)
    a = 0.3 * RNG.standard_normal((N, 3))
    b = 0.3 * RNG.standard_normal((N, 3))
    ds = ipm.ds_family(ipm.EXP if kind == "exp" else ipm.POW, s, z, sc, a, b, sm, fam=fam)
    g, Hf = jets.derivatives(f, z, alpha)
    u = np.linalg.solve(Hf, a[..., None])[..., 0]
    h = 1e-5 * np.linalg.norm(z, axis=1, keepdims=True) / np.linalg.norm(b, axis=1, keepdims=True)
    _, Hp = jets.derivatives(f, z + h * b, alpha)
    _, Hm = jets.derivatives(f, z - h * b, alpha)
    third = np.einsum("cij,cj->ci", (Hp - Hm) / (2.0 * h[:, :, None]), u)
    eta_ref = -0.5 * third
    eta = ds - s - sm * g
    err = np.abs(eta - eta_ref).max(axis=1) / np.maximum(np.abs(eta_ref).max(axis=1), 1e-300)
    assert err.max() <= 1e-6, err.max()
    # the term is not negligible against d_s in these cases
    assert np.median(np.abs(eta_ref).max(axis=1) / np.abs(ds).max(axis=1)) > 1e-3


# ------------------------------------------------------------------ step rule with N(beta)
def _exp_primal_in(s):
    return (s[:, 1] > 0) & (s[:, 2] > s[:, 1] * np.exp(s[:, 0] / np.where(s[:, 1] > 0, s[:, 1], 1.0)))


def _exp_dual_in(z):
    with np.errstate(all="ignore"):
        psi = z[:, 1] - z[:, 0] - z[:, 0] * np.log(z[:, 2] / (-z[:, 0]))
    return (z[:, 0] < 0) & (z[:, 2] > 0) & (psi > 0)


def _pow_primal_in(s, a):
    return (s[:, 0] > 0) & (s[:, 1] > 0) & (np.abs(s[:, 2]) < np.abs(s[:, 0]) ** a * np.abs(s[:, 1]) ** (1 - a))


def _pow_dual_in(z, a):
    return (z[:, 0] > 0) & (z[:, 1] > 0) & (np.abs(z[:, 2]) < np.abs(z[:, 0] / a) ** a * np.abs(z[:, 1] / (1 - a)) ** (1 - a))


def conj_point_newton(f, s, start, params=None, iters=200):
    """z with -grad f(z) = s: the minimiser of f(z) + <s, z>, by the damped
    Newton method for self-concordant functions (step 1/(1 + decrement)),
    which stays inside the domain, then full Newton steps."""
    z = np.array(start, dtype=float)
    for it in range(iters):
        g, H = jets.derivatives(f, z, params)
        r = g + s
        dz = np.linalg.solve(H, r[..., None])[..., 0]
        lam = np.sqrt(np.maximum(np.einsum("ci,ci->c", r, dz), 0.0))
        damp = np.where(lam > 0.25, 1.0 / (1.0 + lam), 1.0)
        z = z - damp[:, None] * dz
        if lam.max() < 1e-14:
            break
    return z


def _neighbourhood_ok(f, s, z, start, params, beta, mu):
    """nu_i / <grad f*(s), grad f(z)> >= beta mu with nu_i = 3, s~ = -grad f(z), z~ = -grad f*(s).
    Returns the test per cone and z~ (the next trial's Newton start)."""
    g, _ = jets.derivatives(f, z, params)
    zt = conj_point_newton(f, s, start, params)
    return 3.0 / np.sum(-g * zt, axis=1) >= beta * mu, zt


def _brute_force_step(sv, d, tau, kappa, nn, ex, pw, alpha, nu, beta, with_nbhd):
    """alpha_0 from the ratio tests of tau, kappa and the nonneg rows, then
    alpha_0, 0.8 alpha_0, 0.8^2 alpha_0, ... until every exp/pow cone is
    interior (and, if asked, inside N(beta))."""
    s, z = sv
    a = 1.0
    if d["tau"] < 0:
        a = min(a, -tau / d["tau"])
    if d["kappa"] < 0:
        a = min(a, -kappa / d["kappa"])
    for v, dv in ((s[nn], d["s"][nn]), (z[nn], d["z"][nn])):
        neg = dv < 0
        if neg.any():
            a = min(a, float(np.min(-v[neg] / dv[neg])))
    start_e = np.tile([-1.0, 1.0, 1.0], (ex.shape[0], 1))
    start_p = np.tile([1.0, 1.0, 0.0], (pw.shape[0], 1))
    while a >= 1e-10:
        sa, za = s + a * d["s"], z + a * d["z"]
        ok = (_exp_primal_in(sa[ex]).all() and _exp_dual_in(za[ex]).all()
              and _pow_primal_in(sa[pw], alpha).all() and _pow_dual_in(za[pw], alpha).all())
        if ok and with_nbhd:
            mu_a = (sa @ za + (tau + a * d["tau"]) * (kappa + a * d["kappa"])) / (nu + 1)
            ok_e, start_e = _neighbourhood_ok(C.f_exp, sa[ex], za[ex], start_e, None, beta, mu_a)
            ok_p, start_p = _neighbourhood_ok(C.f_pow, sa[pw], za[pw], start_p, alpha, beta, mu_a)
            ok = ok_e.all() and ok_p.all()
        if ok:
            return a
        a *= 0.8
    return 0.0


def test_conj_point_newton_agrees_with_oracle_bisection():
    """The two routes to z~ = -grad f*(s) meet (the test's Newton is used below)."""
    s = exp_primal(30, RNG)
    zt = conj_point_newton(C.f_exp, s, np.tile([-1.0, 1.0, 1.0], (30, 1)))
    g, _ = jets.derivatives(C.f_exp, zt)
    assert np.abs(-g - s).max() <= 1e-10 * np.abs(s).max()
    zo = C.NonsymFamily("exp").conj_grad_point(s)
    assert np.abs(zt - zo).max() <= 1e-8 * np.abs(zo).max()


def _min_ratio(sa, za, ex, pw, alpha):
    """min over exp/pow cones of nu_i / <s~, z~> at one trial point."""
    g, _ = jets.derivatives(C.f_exp, za[ex])
    zt = conj_point_newton(C.f_exp, sa[ex], np.tile([-1.0, 1.0, 1.0], (ex.shape[0], 1)))
    re_ = 3.0 / np.sum(-g * zt, axis=1)
    g, _ = jets.derivatives(C.f_pow, za[pw], alpha)
    zt = conj_point_newton(C.f_pow, sa[pw], np.tile([1.0, 1.0, 0.0], (pw.shape[0], 1)), alpha)
    rp = 3.0 / np.sum(-g * zt, axis=1)
    return min(re_.min(), rp.min())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_step_length_neighbourhood_brute_force(seed):
    """The oracle's combined step (backtracking x0.8 from the symmetric-cone
    alpha_0 until interior and inside N(beta)) equals the brute-force walk.
    beta is placed so that N(beta) rejects the first two interior trials and
    accepts the third, and so that a test against mu of the current iterate
    instead of the trial point's would reject the third as well."""
    rng = np.random.default_rng(100 + seed)
    ne, npw, nn_rows = 6, 5, 4
    alpha = rng.uniform(0.25, 0.75, npw)
    cones = [(ipm.NONNEG, nn_rows, 0.0)] + [(ipm.EXP, 3, 0.0)] * ne + [(ipm.POW, 3, float(a)) for a in alpha]
    m = nn_rows + 3 * (ne + npw)
    prob = Problem(1, m, sp.csr_matrix((1, 1)), np.array([1.0]), sp.csr_matrix(np.ones((m, 1))),
                   np.ones(m), cones, "step_pin")
    nn = np.arange(nn_rows)
    ex = nn_rows + np.arange(3 * ne).reshape(ne, 3)
    pw = nn_rows + 3 * ne + np.arange(3 * npw).reshape(npw, 3)
    s = np.zeros(m)
    z = np.zeros(m)
    s[nn], z[nn] = rng.uniform(0.5, 2, nn_rows), rng.uniform(0.5, 2, nn_rows)
    s[ex], z[ex] = exp_primal(ne, rng), exp_dual(ne, rng)
    s[pw], z[pw] = pow_primal(npw, alpha, rng), pow_dual(npw, alpha, rng)
    # a direction that shrinks s (lowering mu along the step) while the
    # nonneg rows allow a long step
    d = {"s": np.zeros(m), "z": np.zeros(m), "x": np.zeros(1), "tau": -0.1, "kappa": 0.05}
    d["s"][nn], d["z"][nn] = -0.1 * s[nn], -0.05 * z[nn]
    d["s"][ex] = -0.9 * s[ex] + 0.5 * rng.standard_normal((ne, 3)) * np.abs(s[ex])
    d["z"][ex] = 0.3 * rng.standard_normal((ne, 3)) * np.abs(z[ex])
    d["s"][pw] = -0.9 * s[pw] + 0.4 * rng.standard_normal((npw, 3)) * np.abs(s[pw])
    d["z"][pw] = 0.3 * rng.standard_normal((npw, 3)) * np.abs(z[pw])
    nu = nn_rows + 3 * (ne + npw)
    feas_only = _brute_force_step((s, z), d, 1.0, 1.0, nn, ex, pw, alpha, nu, 0.0, False)
    assert feas_only > 0

    def mu_at(a):
        return ((s + a * d["s"]) @ (z + a * d["z"]) + (1.0 - 0.1 * a) * (1.0 + 0.05 * a)) / (nu + 1)
    trials = [feas_only, feas_only * 0.8, feas_only * 0.8 * 0.8]   # the walk multiplies step by step
    q = [_min_ratio(s + a * d["s"], z + a * d["z"], ex, pw, alpha) / mu_at(a) for a in trials]
    assert q[0] < q[1] < q[2], q
    beta = q[1] + 0.9 * (q[2] - q[1])
    ratio_third = q[2] * mu_at(trials[2])
    assert ratio_third < beta * mu_at(0.0), "case does not separate the trial mu from the current mu"

    sol = ipm.Solver(prob, ipm.Settings(beta=beta))
    sol.s, sol.z, sol.tau, sol.kappa = s, z, 1.0, 1.0
    got = sol.step_length(d, combined=True)
    want = _brute_force_step((s, z), d, 1.0, 1.0, nn, ex, pw, alpha, nu, beta, True)
    assert want == trials[2]
    assert got == want, (got, want)
    # the affine step applies only the interior test
    assert sol.step_length(d, combined=False) == feas_only
