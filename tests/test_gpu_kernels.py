"""GPU parity of single steps: the C-ABI's kernel entry points against the
CPU oracle on the same seeded inputs (FP64: 1e-12 relative), and the dense
Schur-complement factorisation against numpy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cones as C  # noqa: E402
from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from tests.test_oracle_cones import exp_dual, exp_primal, pow_dual, pow_primal, soc_interior, spd  # noqa: E402

DEV = "cuda"
RNG = np.random.default_rng(2024)


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ----------------------------------------------------------------- dense factor
@pytest.mark.parametrize("n", [1, 37, 64, 200, 333, 700, 1100, 2049])
@pytest.mark.parametrize("nrhs", [1, 2, 3])
def test_dense_cholesky_fp64(n, nrhs):
    G = RNG.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    B = RNG.standard_normal((n, nrhs))
    X, L, hits = HC.test_dense_chol_solve(T(A), T(B), HC.PRECISION_FP64)
    ref = np.linalg.solve(A, B)
    assert hits == 0
    assert relerr(N(X), ref) < 1e-11
    Lh = np.tril(N(L))
    assert relerr(Lh @ Lh.T, A) < 1e-13


@pytest.mark.parametrize("n", [333, 681, 1101, 1537])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dense_cholesky_odd_sizes_padded_ld(n, precision):
    """The solver's layout: n odd (or not a multiple of 4), leading dimension
    rounded up to 64, so the MFMA DMA updates run and leave edge rows/columns
    to the edge kernel."""
    ld = (n + 63) // 64 * 64
    G = RNG.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    B = RNG.standard_normal((n, 2))
    code = HC.PRECISION_FP64 if precision == "fp64" else HC.PRECISION_MIXED
    X, L, hits = HC.test_dense_chol_solve(T(A), T(B), code, ld=ld)
    assert hits == 0
    assert relerr(N(X), np.linalg.solve(A, B)) < (1e-11 if precision == "fp64" else 1e-4)
    if precision == "fp64":
        Lh = np.tril(N(L))
        assert relerr(Lh @ Lh.T, A) < 1e-13


def _envelope_spd(first, rng):
    """SPD matrix whose row i has its first nonzero at column first[i]
    (non-decreasing): L0 L0' with L0 lower triangular of that profile."""
    n = len(first)
    L0 = np.tril(rng.standard_normal((n, n)))
    cols = np.arange(n)[None, :]
    L0[cols < np.asarray(first)[:, None]] = 0.0
    L0[np.arange(n), np.arange(n)] = np.sqrt(n) + np.abs(L0[np.arange(n), np.arange(n)])
    return L0 @ L0.T


def _envelope_last(first):
    n = len(first)
    last = np.arange(1, n + 1)
    for i, f in enumerate(first):
        last[f] = max(last[f], i + 1)
    return np.maximum.accumulate(last)


@pytest.mark.parametrize("shape", ["stages", "random"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dense_cholesky_envelope(shape, precision):
    """Envelope-limited factorisation (the solver's dense tail): rows of a
    stage couple back to the start of the previous stage (stages wider than a
    768-column panel, so some panels update later columns and some do not),
    or a random non-decreasing profile; n not a multiple of 64."""
    n = 3300
    if shape == "stages":
        w = 900
        first = np.array([max(0, w * (i // w - 1)) for i in range(n)])
    else:
        first = np.maximum.accumulate(np.maximum(0, np.arange(n) - RNG.integers(1, 700, n)))
    A = _envelope_spd(first, RNG)
    last = _envelope_last(first)
    B = RNG.standard_normal((n, 2))
    ld = (n + 63) // 64 * 64
    code = HC.PRECISION_FP64 if precision == "fp64" else HC.PRECISION_MIXED
    X, L, hits = HC.test_dense_chol_solve(T(A), T(B), code, ld=ld, last=last)
    assert hits == 0
    assert relerr(N(X), np.linalg.solve(A, B)) < (1e-11 if precision == "fp64" else 1e-4)
    if precision == "fp64":
        Lh = np.tril(N(L))
        assert relerr(Lh @ Lh.T, A) < 1e-13
        outside = np.arange(n)[None, :] < first[:, None]
        assert np.all(Lh[outside] == 0.0)


@pytest.mark.parametrize("n", [64, 300, 513, 1600])
def test_dense_cholesky_fp32(n):
    G = RNG.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    B = RNG.standard_normal((n, 2))
    X, _, hits = HC.test_dense_chol_solve(T(A), T(B), HC.PRECISION_MIXED)
    assert hits == 0
    assert relerr(N(X), np.linalg.solve(A, B)) < 1e-4


# ----------------------------------------------------------------- cone scaling
def test_nonneg_scale():
    s, z = RNG.uniform(0.01, 3, (40, 5)), RNG.uniform(0.01, 3, (40, 5))
    H, lam, _ = HC.test_cone_scale(HC.NONNEG, 5, T(s), T(z), 1.0)
    assert relerr(N(lam), s / z) < 1e-15
    assert relerr(np.diagonal(N(H), axis1=1, axis2=2), s / z) < 1e-15


@pytest.mark.parametrize("d", [2, 3, 5, 17, 64, 700])
def test_soc_scale(d):
    Nc = 300 if d <= 64 else 5
    s, z = soc_interior(Nc, d, RNG), soc_interior(Nc, d, RNG)
    H, lam, _ = HC.test_cone_scale(HC.SOC, d, T(s), T(z), 1.0)
    ref = C.soc_scale(s, z)
    assert relerr(N(H), ref["H"]) < 1e-12
    assert relerr(N(lam), ref["lam"]) < 1e-12


@pytest.mark.parametrize("kind", ["exp", "pow"])
def test_nonsym_scale(kind):
    Nc = 400
    if kind == "exp":
        fam, s, z, alpha = C.NonsymFamily("exp"), exp_primal(Nc, RNG), exp_dual(Nc, RNG), None
    else:
        a = RNG.uniform(0.2, 0.8, Nc)
        fam, s, z, alpha = C.NonsymFamily("pow", a), pow_primal(Nc, a, RNG), pow_dual(Nc, a, RNG), T(a)
    mu = 0.37
    H, zt, br = HC.test_cone_scale(HC.EXP if kind == "exp" else HC.POW, 3, T(s), T(z), mu, alpha)
    ref = fam.scale(s, z, mu)
    assert (N(br) == ref["branch"]).all()
    assert relerr(N(zt), ref["zt"]) < 1e-12
    assert relerr(N(H), ref["H"]) < 1e-12


@pytest.mark.parametrize("k", [2, 3, 4, 10, 13, 20, 32])
def test_psd_scale(k):
    """Sides up to 12 run eight cones per workgroup, sides 13..32 two
    (measured relative errors at k = 32: 3e-14 for H, 5e-15 for lambda)."""
    Nc = 60 if k <= 13 else 12
    S, Z = spd(Nc, k, RNG), spd(Nc, k, RNG)
    s, z = C.svec(S), C.svec(Z)
    H, lam, _ = HC.test_cone_scale(HC.PSD, k, T(s), T(z), 1.0)
    ref = C.psd_scale(s, z, k)
    eh, el = relerr(N(H), ref["H"]), relerr(np.sort(N(lam)[:, :k], 1), np.sort(ref["lam"], 1))
    print(k, eh, el)
    assert eh < 1e-12 and el < 1e-12


# ----------------------------------------------------------------- combined-step d_s
def _oracle_ds(kind, s, z, dsa, dza, mu, sm, k=None, alpha=None, force_dual=False):
    """The oracle's d_s of one family (oracle.ipm.ds_family) on the oracle's scaling state."""
    from oracle import ipm
    if kind == "nonneg":
        return ipm.ds_family(ipm.NONNEG, s, z, C.nn_scale(s, z), dsa, dza, sm)
    if kind == "soc":
        return ipm.ds_family(ipm.SOC, s, z, C.soc_scale(s, z), dsa, dza, sm)
    if kind == "psd":
        return ipm.ds_family(ipm.PSD, s, z, C.psd_scale(s, z, k), dsa, dza, sm, k=k)
    fam = C.NonsymFamily(kind, alpha)
    sc = fam.scale(s, z, mu, force_dual=force_dual)
    return ipm.ds_family(ipm.EXP if kind == "exp" else ipm.POW, s, z, sc, dsa, dza, sm, fam=fam)


@pytest.mark.parametrize("kind", ["nonneg", "soc", "soc_large", "exp", "pow", "psd", "psd10", "psd32"])
def test_combined_ds(kind):
    Nc = 200
    mu, sm = 0.8, 0.05
    alpha = None
    if kind == "nonneg":
        s, z, dim, code = RNG.uniform(0.1, 2, (Nc, 1)), RNG.uniform(0.1, 2, (Nc, 1)), 1, HC.NONNEG
    elif kind == "soc":
        s, z, dim, code = soc_interior(Nc, 4, RNG), soc_interior(Nc, 4, RNG), 4, HC.SOC
    elif kind == "soc_large":
        s, z, dim, code = soc_interior(30, 300, RNG), soc_interior(30, 300, RNG), 300, HC.SOC
        kind = "soc"
    elif kind == "exp":
        s, z, dim, code = exp_primal(Nc, RNG), exp_dual(Nc, RNG), 3, HC.EXP
    elif kind == "pow":
        alpha = RNG.uniform(0.2, 0.8, Nc)
        s, z, dim, code = pow_primal(Nc, alpha, RNG), pow_dual(Nc, alpha, RNG), 3, HC.POW
    else:
        k = {"psd": 3, "psd10": 10, "psd32": 32}[kind]
        nc = Nc if k == 3 else (60 if k == 10 else 10)
        s, z, dim, code = C.svec(spd(nc, k, RNG)), C.svec(spd(nc, k, RNG)), k, HC.PSD
        kind = "psd"
    dsa, dza = 0.3 * RNG.standard_normal(s.shape), 0.3 * RNG.standard_normal(s.shape)
    out = HC.test_cone_ds(code, dim, T(s), T(z), T(dsa), T(dza), mu, sm, None if alpha is None else T(alpha))
    ref = _oracle_ds(kind, s, z, dsa, dza, mu, sm, k=dim if kind == "psd" else 3, alpha=alpha)
    err = relerr(N(out), ref)
    print(kind, dim, err)
    assert err < 1e-12


# ----------------------------------------------------------------- step lengths
@pytest.mark.parametrize("kind", ["nonneg", "soc", "soc_large", "psd", "psd10", "psd32", "exp", "pow"])
def test_step(kind):
    Nc = 150
    alpha = None
    if kind == "nonneg":
        s, z, dim, code = RNG.uniform(0.1, 2, (Nc, 1)), RNG.uniform(0.1, 2, (Nc, 1)), 1, HC.NONNEG
    elif kind == "soc":
        s, z, dim, code = soc_interior(Nc, 3, RNG), soc_interior(Nc, 3, RNG), 3, HC.SOC
    elif kind == "soc_large":   # more cones than the grid of one launch (2048)
        Nc = 2100
        s, z, dim, code = soc_interior(Nc, 257, RNG), soc_interior(Nc, 257, RNG), 257, HC.SOC
        kind = "soc"
    elif kind == "psd":
        s, z, dim, code = C.svec(spd(Nc, 3, RNG)), C.svec(spd(Nc, 3, RNG)), 3, HC.PSD
    elif kind in ("psd10", "psd32"):
        k = int(kind[3:])
        Nc = 20 if k == 32 else Nc
        s, z, dim, code = C.svec(spd(Nc, k, RNG)), C.svec(spd(Nc, k, RNG)), k, HC.PSD
        kind = "psd"
    elif kind == "exp":
        s, z, dim, code = exp_primal(Nc, RNG), exp_dual(Nc, RNG), 3, HC.EXP
    else:
        alpha = RNG.uniform(0.2, 0.8, Nc)
        s, z, dim, code = pow_primal(Nc, alpha, RNG), pow_dual(Nc, alpha, RNG), 3, HC.POW
    ds, dz = 2 * RNG.standard_normal(s.shape), 2 * RNG.standard_normal(s.shape)
    out = N(HC.test_cone_step(code, dim, T(s), T(z), T(ds), T(dz), 1.0, None if alpha is None else T(alpha)))
    if kind == "nonneg":
        ref = np.minimum(1.0, np.minimum(C.nn_step(s, ds), C.nn_step(z, dz))[:, 0])
    elif kind == "soc":
        ref = np.minimum(1.0, np.minimum(C.soc_step(s, ds), C.soc_step(z, dz)))
    elif kind == "psd":
        ref = np.minimum(1.0, np.minimum(C.psd_step(s, ds, dim), C.psd_step(z, dz, dim)))
    else:
        fam = C.NonsymFamily(kind, alpha)
        ref = np.zeros(Nc)
        for i in range(Nc):
            sub = C.NonsymFamily(kind, None if alpha is None else alpha[i:i + 1])
            a = 1.0
            for _ in range(64):
                if sub.primal_interior(s[i:i + 1] + a * ds[i:i + 1])[0] and sub.dual_interior(z[i:i + 1] + a * dz[i:i + 1])[0]:
                    ref[i] = a
                    break
                a *= 0.8
        assert (out == ref).all()
        return
    assert relerr(out, ref) < 1e-12


# ----------------------------------------------------------------- explicit M blocks
@pytest.mark.parametrize("kind", ["nonneg", "soc", "soc_large", "exp", "pow", "psd3", "psd5", "psd16"])
@pytest.mark.parametrize("delta", [1e-8, 1e-3])
def test_mblock_inverts_the_applied_scaling(kind, delta):
    """The explicit blocks M_c that the Schur complement is assembled from are
    (H_c + delta I)^-1 for the H_c that the refinement residual applies, and
    match the oracle's scaling; both near the centre and close to the
    boundary (mu small)."""
    Nc = 120
    alpha = None
    if kind == "nonneg":
        s, z, dim, code = RNG.uniform(0.1, 2, (Nc, 1)), RNG.uniform(0.1, 2, (Nc, 1)), 1, HC.NONNEG
    elif kind == "soc":
        s, z, dim, code = soc_interior(Nc, 4, RNG), soc_interior(Nc, 4, RNG), 4, HC.SOC
    elif kind == "soc_large":   # the diagonal plus rank-2 form of M_c
        s, z, dim, code = soc_interior(12, 90, RNG), soc_interior(12, 90, RNG), 90, HC.SOC
    elif kind == "exp":
        s, z, dim, code = exp_primal(Nc, RNG), exp_dual(Nc, RNG), 3, HC.EXP
    elif kind == "pow":
        alpha = RNG.uniform(0.2, 0.8, Nc)
        s, z, dim, code = pow_primal(Nc, alpha, RNG), pow_dual(Nc, alpha, RNG), 3, HC.POW
    else:
        k = int(kind[3:])
        s, z, dim, code = C.svec(spd(Nc, k, RNG)), C.svec(spd(Nc, k, RNG)), k, HC.PSD
    mu = 0.7
    a_t = None if alpha is None else T(alpha)
    H, _, _ = HC.test_cone_scale(code, dim, T(s), T(z), mu, a_t)
    M = HC.test_cone_mblock(code, dim, T(s), T(z), mu, delta, a_t)
    H, M = N(H), N(M)
    rows = H.shape[1]
    eye = np.eye(rows)
    prod = np.einsum("cij,cjk->cik", M, H + delta * eye[None])
    err = np.abs(prod - eye[None]).max(axis=(1, 2))
    cond = np.array([np.linalg.cond(h + delta * eye) for h in H])
    assert np.all(err <= 1e-13 * np.maximum(cond, 1.0) + 1e-12), (err.max(), cond[np.argmax(err)])
    assert np.allclose(M, np.transpose(M, (0, 2, 1)), rtol=0, atol=1e-12 * np.abs(M).max())


# ----------------------------------------------------------------- the solver's step-length launch
@pytest.mark.parametrize("kind", ["nonneg", "soc3", "soc_large", "psd3", "psd10", "psd32"])
def test_step_min_solver_launch(kind):
    """The launch hc_solve takes for the symmetric step (PSD: the s and z
    halves as separate wave tasks; more tasks than the grid, so the
    grid-stride loop wraps) against the oracle's minimum over all cones."""
    if kind == "nonneg":
        Nc = 300000
        s, z, dim, code = RNG.uniform(0.1, 2, (Nc, 1)), RNG.uniform(0.1, 2, (Nc, 1)), 1, HC.NONNEG
        ds, dz = RNG.standard_normal(s.shape), RNG.standard_normal(s.shape)
        ref = min(C.nn_step(s, ds).min(), C.nn_step(z, dz).min())
    elif kind.startswith("soc"):
        Nc, d = (120000, 3) if kind == "soc3" else (2100, 257)
        s, z, dim, code = soc_interior(Nc, d, RNG), soc_interior(Nc, d, RNG), d, HC.SOC
        ds, dz = 0.5 * RNG.standard_normal(s.shape), 0.5 * RNG.standard_normal(s.shape)
        ref = min(C.soc_step(s, ds).min(), C.soc_step(z, dz).min())
    else:
        k = int(kind[3:])
        Nc = 1100 if k < 32 else 1030
        s, z, dim, code = C.svec(spd(Nc, k, RNG)), C.svec(spd(Nc, k, RNG)), k, HC.PSD
        ds, dz = 0.5 * RNG.standard_normal(s.shape), 0.5 * RNG.standard_normal(s.shape)
        ref = min(C.psd_step(s, ds, k).min(), C.psd_step(z, dz, k).min())
    got = HC.test_cone_step_min(code, dim, T(s), T(z), T(ds), T(dz))
    print(kind, got, ref)
    assert abs(got - ref) <= 1e-12 * ref


# ----------------------------------------------------------------- exp/pow dual scaling
@pytest.mark.parametrize("kind", ["exp", "pow"])
def test_nonsym_dual_scaling(kind):
    """The dual scaling H = mu grad^2 f(z) (Appendix A; taken by hc_solve
    after a short primal-dual step): H, branch, M blocks and d_s against the
    oracle's scale(force_dual=True)."""
    Nc = 300
    if kind == "exp":
        fam, s, z, alpha = C.NonsymFamily("exp"), exp_primal(Nc, RNG), exp_dual(Nc, RNG), None
    else:
        a = RNG.uniform(0.2, 0.8, Nc)
        fam, s, z, alpha = C.NonsymFamily("pow", a), pow_primal(Nc, a, RNG), pow_dual(Nc, a, RNG), a
    code = HC.EXP if kind == "exp" else HC.POW
    a_t = None if alpha is None else T(alpha)
    mu, delta = 0.37, 1e-8
    H, zt, br = HC.test_cone_scale(code, 3, T(s), T(z), mu, a_t, force_dual=True)
    ref = fam.scale(s, z, mu, force_dual=True)
    assert (N(br) == 1).all() and (ref["branch"] == 1).all()
    assert relerr(N(H), ref["H"]) < 1e-12
    assert relerr(N(zt), ref["zt"]) < 1e-12
    M = N(HC.test_cone_mblock(code, 3, T(s), T(z), mu, delta, a_t, force_dual=True))
    Mref = np.linalg.inv(ref["H"] + delta * np.eye(3)[None])
    assert relerr(M, Mref) < 1e-10
    dsa, dza = 0.3 * RNG.standard_normal(s.shape), 0.3 * RNG.standard_normal(s.shape)
    out = HC.test_cone_ds(code, 3, T(s), T(z), T(dsa), T(dza), mu, 0.05, a_t, force_dual=True)
    want = _oracle_ds(kind, s, z, dsa, dza, mu, 0.05, alpha=alpha, force_dual=True)
    assert relerr(N(out), want) < 1e-12
    # and the primal-dual scaling really differs here
    Hpd = fam.scale(s, z, mu)["H"]
    assert relerr(Hpd, ref["H"]) > 1e-3
