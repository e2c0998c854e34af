"""Pins of the oracle's per-cone operations against facts outside the oracle:
algebraic identities, finite differences, textbook routines (LAPACK eigh) and
brute force.  A dropped term, wrong sign or transposed operand in the oracle
fails at least one of these.  CPU only."""
import math

import numpy as np
import pytest

from oracle import cones as C
from oracle import jets

RNG = np.random.default_rng(12345)


def soc_interior(N, d, rng=RNG):
    u = rng.standard_normal((N, d - 1))
    t = np.linalg.norm(u, axis=1) + rng.uniform(0.05, 1.0, N)
    return np.concatenate([t[:, None], u], axis=1)


def spd(N, k, rng=RNG):
    G = rng.standard_normal((N, k, k))
    return np.einsum("cij,ckj->cik", G, G) + 0.3 * np.eye(k)[None]


def exp_primal(N, rng=RNG):
    s = np.stack([rng.uniform(-2, 1, N), rng.uniform(0.2, 2, N), np.zeros(N)], 1)
    s[:, 2] = s[:, 1] * np.exp(s[:, 0] / s[:, 1]) * rng.uniform(1.05, 4, N)
    return s


def exp_dual(N, rng=RNG):
    z = np.stack([-rng.uniform(0.2, 2, N), np.zeros(N), rng.uniform(0.2, 2, N)], 1)
    z[:, 1] = z[:, 0] + z[:, 0] * np.log(z[:, 2] / (-z[:, 0])) + rng.uniform(0.1, 2, N)
    return z


def pow_primal(N, a, rng=RNG):
    s = np.stack([rng.uniform(0.5, 1.5, N), rng.uniform(0.5, 1.5, N), np.zeros(N)], 1)
    s[:, 2] = rng.uniform(-0.9, 0.9, N) * s[:, 0] ** a * s[:, 1] ** (1 - a)
    return s


def pow_dual(N, a, rng=RNG):
    z = np.stack([rng.uniform(0.5, 1.5, N), rng.uniform(0.5, 1.5, N), np.zeros(N)], 1)
    z[:, 2] = rng.uniform(-0.9, 0.9, N) * (z[:, 0] / a) ** a * (z[:, 1] / (1 - a)) ** (1 - a)
    return z


# ------------------------------------------------------------------ nonneg
def test_nonneg_scaling_identities():
    s, z = RNG.uniform(0.01, 3, 200), RNG.uniform(0.01, 3, 200)
    sc = C.nn_scale(s, z)
    assert np.allclose(sc["H"][:, 0] * z, s, rtol=1e-15)
    assert np.allclose(sc["lam"] ** 2, s * z, rtol=1e-14)
    assert np.allclose(sc["w"] * z, sc["lam"], rtol=1e-14)       # W z = lambda
    assert np.allclose(s / sc["w"], sc["lam"], rtol=1e-14)       # W^-T s = lambda


def test_nonneg_step_bisection():
    x = RNG.uniform(0.1, 2, 300)
    dx = RNG.standard_normal(300)
    a = C.nn_step(x, dx)
    for i in range(0, 300, 7):
        ai = _bisect(lambda t: x[i] + t * dx[i] >= 0)
        if np.isinf(a[i]):
            assert ai > 1e5
        else:
            assert abs(ai - a[i]) <= 1e-12 * max(1, a[i])


def _bisect(member, hi=1e6, halvings=200):
    if member(hi):
        return hi
    lo = 0.0
    for _ in range(halvings):
        mid = 0.5 * (lo + hi)
        if member(mid):
            lo = mid
        else:
            hi = mid
    return lo


# ------------------------------------------------------------------ SOC
@pytest.mark.parametrize("d", [2, 3, 5, 64, 400])
def test_soc_nt_identities(d):
    s, z = soc_interior(100, d), soc_interior(100, d)
    sc = C.soc_scale(s, z)
    W, H, lam, Winv = sc["W"], sc["H"], sc["lam"], sc["Winv"]
    assert np.abs(np.einsum("cij,cj->ci", H, z) - s).max() < 1e-12 * np.abs(s).max()
    assert np.abs(np.einsum("cij,cjk->cik", W, W) - H).max() < 1e-12 * np.abs(H).max()
    assert np.abs(np.einsum("cij,cj->ci", Winv, s) - lam).max() < 1e-12 * np.abs(lam).max()
    assert np.allclose(np.sum(lam * lam, 1), np.sum(s * z, 1), rtol=1e-12)
    assert np.allclose(C.jdot(lam, lam), np.sqrt(C.jdot(s, s) * C.jdot(z, z)), rtol=1e-12)
    # the scaling point is NT: the same W maps z and W^-1 maps s to one point
    wb = sc["wbar"]
    assert np.allclose(C.jdot(wb, wb), 1.0, rtol=1e-12)


@pytest.mark.parametrize("d", [2, 3, 5, 64, 200])
def test_soc_spectral_equals_explicit(d):
    s, z = soc_interior(60, d), soc_interior(60, d)
    sc = C.soc_scale(s, z)
    lam, V = C.soc_spectral(sc["wbar"], sc["eta"])
    Hs = np.einsum("cij,cj,ckj->cik", V, lam, V)
    assert np.abs(Hs - sc["H"]).max() < 1e-12 * np.abs(sc["H"]).max()
    assert np.abs(np.einsum("cji,cjk->cik", V, V) - np.eye(d)).max() < 1e-13
    ev = np.linalg.eigvalsh(sc["H"])
    assert np.allclose(np.sort(lam, 1), ev, rtol=1e-9, atol=1e-13)


def test_soc_jordan_inverse():
    lam, v = soc_interior(50, 4), RNG.standard_normal((50, 4))
    x = C.soc_inv_circ(lam, v)
    assert np.abs(C.soc_circ(lam, x) - v).max() < 1e-12


@pytest.mark.parametrize("d", [3, 300])
def test_soc_step_bisection(d):
    x = soc_interior(60, d)
    dx = 2 * RNG.standard_normal((60, d))
    a = C.soc_step(x, dx)
    for i in range(60):
        member = lambda t: (x[i, 0] + t * dx[i, 0]) >= np.linalg.norm(x[i, 1:] + t * dx[i, 1:])
        ai = _bisect(member)
        if np.isinf(a[i]):
            assert ai > 1e5
        else:
            assert abs(ai - a[i]) <= 1e-9 * max(1.0, a[i])


# ------------------------------------------------------------------ PSD
def test_svec_isometry():
    k = 5
    X, Y = spd(10, k), spd(10, k)
    assert np.allclose(np.sum(C.svec(X) * C.svec(Y), 1), np.einsum("cij,cji->c", X, Y), rtol=1e-13)
    assert np.allclose(C.smat(C.svec(X), k), X)


@pytest.mark.parametrize("k", [2, 4])
def test_psd_nt_against_geometric_mean(k):
    S, Z = spd(20, k), spd(20, k)
    sc = C.psd_scale(C.svec(S), C.svec(Z), k)
    # textbook NT point: W_nt = Z^-1/2 (Z^1/2 S Z^1/2)^1/2 Z^-1/2, via LAPACK eigh
    ez, Qz = np.linalg.eigh(Z)
    Zh = np.einsum("cij,cj,ckj->cik", Qz, np.sqrt(ez), Qz)
    Zmh = np.einsum("cij,cj,ckj->cik", Qz, 1 / np.sqrt(ez), Qz)
    Mid = np.einsum("cij,cjk,ckl->cil", Zh, S, Zh)
    em, Qm = np.linalg.eigh(Mid)
    Midh = np.einsum("cij,cj,ckj->cik", Qm, np.sqrt(em), Qm)
    Wnt = np.einsum("cij,cjk,ckl->cil", Zmh, Midh, Zmh)
    assert np.abs(sc["M"] - Wnt).max() < 1e-11 * np.abs(Wnt).max()
    # lambda^2 are the eigenvalues of S Z
    ev = np.sort(np.real(np.linalg.eigvals(np.einsum("cij,cjk->cik", S, Z))), 1)
    assert np.allclose(np.sort(sc["lam"] ** 2, 1), ev, rtol=1e-10)
    # H svec(Z) = svec(S)
    Hz = np.einsum("cij,cj->ci", sc["H"], C.svec(Z))
    assert np.abs(Hz - C.svec(S)).max() < 1e-11 * np.abs(C.svec(S)).max()
    lam, V = C.psd_spectral(sc["R"])
    assert np.abs(np.einsum("cij,cj,ckj->cik", V, lam, V) - sc["H"]).max() < 1e-11 * np.abs(sc["H"]).max()


def test_psd_step_bisection():
    k = 3
    X = C.svec(spd(15, k))
    dX = C.svec(2 * np.stack([a + a.T for a in RNG.standard_normal((15, k, k))]))
    a = C.psd_step(X, dX, k)
    for i in range(15):
        member = lambda t: np.linalg.eigvalsh(C.smat((X[i] + t * dX[i])[None], k)[0])[0] >= 0
        ai = _bisect(member)
        if np.isinf(a[i]):
            assert ai > 1e5
        else:
            assert abs(ai - a[i]) <= 1e-9 * max(1.0, a[i])


# ------------------------------------------------------------------ exp / pow barriers
def _families(N):
    a = RNG.uniform(0.2, 0.8, N)
    return [(C.NonsymFamily("exp"), exp_dual(N), exp_primal(N)),
            (C.NonsymFamily("pow", a), pow_dual(N, a), pow_primal(N, a))]


@pytest.mark.parametrize("which", [0, 1])
def test_barrier_derivatives_finite_differences(which):
    fam, z, _ = _families(8)[which]
    g, H = fam.grad_hess(z)
    h = 1e-5
    for k in range(3):
        e = np.zeros(3); e[k] = h
        f2 = jets.value(fam.f, z + 2 * e, fam.alpha); f1 = jets.value(fam.f, z + e, fam.alpha)
        fm1 = jets.value(fam.f, z - e, fam.alpha); fm2 = jets.value(fam.f, z - 2 * e, fam.alpha)
        fd = (-f2 + 8 * f1 - 8 * fm1 + fm2) / (12 * h)
        assert np.allclose(g[:, k], fd, rtol=1e-7, atol=1e-8)
        g1, _ = fam.grad_hess(z + e); gm1, _ = fam.grad_hess(z - e)
        assert np.allclose(H[:, :, k], (g1 - gm1) / (2 * h), rtol=1e-6, atol=1e-6)
    u, v = RNG.standard_normal((8, 3)), RNG.standard_normal((8, 3))
    T = fam.third(z, u, v)
    _, Hp = fam.grad_hess(z + h * u)
    _, Hm = fam.grad_hess(z - h * u)
    fdT = np.einsum("cij,cj->ci", (Hp - Hm) / (2 * h), v)
    assert np.allclose(T, fdT, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("which", [0, 1])
def test_barrier_homogeneity_identities(which):
    fam, z, _ = _families(30)[which]
    g, H = fam.grad_hess(z)
    assert np.allclose(np.sum(g * z, 1), -3.0, rtol=1e-13)                       # <grad f(z), z> = -nu
    assert np.abs(np.einsum("cij,cj->ci", H, z) + g).max() < 1e-12 * np.abs(g).max()  # Hf z = -grad f
    u = RNG.standard_normal((30, 3))
    T = fam.third(z, z, u)                                                       # f'''[z] = -2 Hf
    assert np.abs(T + 2 * np.einsum("cij,cj->ci", H, u)).max() < 1e-10 * np.abs(H).max()
    G = fam.hess_factor(z)
    assert np.abs(np.einsum("cik,cjk->cij", G, G) - H).max() < 1e-13 * np.abs(H).max()


def test_unit_points():
    e = C.NonsymFamily("exp").unit_point(1)
    g, _ = C.NonsymFamily("exp").grad_hess(e)
    assert np.abs(e + g).max() < 1e-15
    assert np.allclose(e[0], [-1.051383945, 0.556409619, 1.258967884], atol=1e-9)
    a = np.array([0.3, 0.5, 0.7])
    fam = C.NonsymFamily("pow", a)
    u = fam.unit_point(3)
    g, _ = fam.grad_hess(u)
    assert np.abs(u + g).max() < 1e-14


@pytest.mark.parametrize("which", [0, 1])
def test_conjugate_point(which):
    fam, _, s = _families(40)[which]
    zt = fam.conj_grad_point(s)
    g, _ = fam.grad_hess(zt)
    assert np.abs(-g - s).max() < 1e-11 * np.abs(s).max()
    assert np.allclose(np.sum(s * zt, 1), 3.0, rtol=1e-12)
    assert fam.dual_interior(zt).all()


@pytest.mark.parametrize("which", [0, 1])
def test_bfgs_scaling(which):
    fam, z, s = _families(40)[which]
    mu = 0.7
    sc = fam.scale(s, z, mu)
    H = sc["H"]
    assert (sc["branch"] == 0).all()
    assert np.abs(np.einsum("cij,cj->ci", H, z) - s).max() < 1e-10 * np.abs(s).max()            # H z = s
    assert np.abs(np.einsum("cij,cj->ci", H, sc["zt"]) - sc["st"]).max() < 1e-9 * np.abs(sc["st"]).max()
    assert np.abs(H - H.transpose(0, 2, 1)).max() < 1e-13 * np.abs(H).max()
    assert (np.linalg.eigvalsh(H)[:, 0] > 0).all()
    _, Hf = fam.grad_hess(z)
    raw = fam.bfgs_raw(s, z, sc["st"], sc["zt"], Hf, mu)
    assert np.abs(raw - H).max() < 1e-9 * np.abs(H).max()
    # dual branch when forced: H = mu Hess f(z)
    scd = fam.scale(s, z, mu, force_dual=True)
    assert np.abs(scd["H"] - mu * Hf).max() < 1e-11 * np.abs(mu * Hf).max()


@pytest.mark.parametrize("which", [0, 1])
def test_membership_brute_force(which):
    fam, z, s = _families(20)[which]
    d = 3 * RNG.standard_normal((20, 3))
    for i in range(20):
        sub = C.NonsymFamily(fam.kind, None if fam.alpha is None else fam.alpha[i:i + 1])
        t = _bisect(lambda a: bool(sub.primal_interior(s[i:i + 1] + a * d[i:i + 1])[0]), hi=1e3)
        # every 0.8^k below the boundary is interior, every one above is not
        for kk in range(40):
            a = 0.8 ** kk * 10.0
            inside = bool(sub.primal_interior(s[i:i + 1] + a * d[i:i + 1])[0])
            if a < t * (1 - 1e-9):
                assert inside
            elif a > t * (1 + 1e-9):
                assert not inside
