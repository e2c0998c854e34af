"""Per-cone operations of the interior-point method, written from the paper.

TEST INFRASTRUCTURE ONLY: part of the CPU oracle (plain FP64 numpy).  Nothing
in the product path may import this package.

Each function acts on one *family* of equal-size cones at once: the cone
vectors are arrays of shape (N, d) (N cones of d rows).  There is no
blocking or fusion; vectorisation over cones does not change any cone's
arithmetic.

Sources (sections / equations of arXiv 2412.19027):
  cones and dual cones ............ Sec. 2.1 "Supported cones"
  barriers f on K* and degrees .... Sec. 2.2, barrier list after the smoothed
                                    complementarity s = -mu grad f(z)
  scaling H, W, lambda ............ Appendix A (NT scaling for symmetric cones
                                    following CVXOPT; rank-4 BFGS primal-dual
                                    scaling with shadow iterates for exp/pow)
  combined-step d_s and the
  higher-order corrections ........ eq. (ds-correction-step) and the
                                    Mehrotra / 3rd-order correction equations
  step length / backtracking 0.8 /
  neighbourhood N(beta) ........... Sec. 2.2, "Update iterates"

Readings taken where the paper is silent or garbled:
  * svec = upper triangle column by column, off-diagonals times sqrt(2).
  * shadow iterates: s~ = -grad f(z) and z~ = -grad f*(s) (the printed
    definitions swap f and f*; the types require this reading).
  * BFGS scaling maps z to s: H = S (S'Z)^-1 S' + Ha - Ha Z (Z'Ha Z)^-1 Z'Ha
    with S = [s, s~], Z = [z, z~], Ha = mu Hess f(z), mu the global mu.
  * the Mehrotra term uses W^-T ds (equal to the paper's W^-1 ds on the
    self-adjoint nonneg/SOC scalings).
  * dual scaling H = mu Hess f(z) when mu_i mu~_i - 1 < sqrt(eps).
"""
from __future__ import annotations

import math

import numpy as np

from . import jets

EPS = np.finfo(np.float64).eps
THETA_PD = math.sqrt(EPS)
SQRT2 = math.sqrt(2.0)


# ===========================================================================
# nonnegative cone (rows are independent 1-d cones), barrier -sum log z_i
# ===========================================================================

def nn_scale(s, z):
    """NT scaling of R+: W = diag(sqrt(s/z)), lambda = sqrt(s z), H = W'W = s/z."""
    w = np.sqrt(s / z)
    lam = np.sqrt(s * z)
    return {"w": w, "lam": lam, "H": (s / z)[..., None]}


def nn_H(s, z):
    return s / z


def nn_step(x, dx):
    """Largest alpha with x + alpha dx >= 0 (inf if none), per row."""
    a = np.full(x.shape, np.inf)
    neg = dx < 0
    a[neg] = -x[neg] / dx[neg]
    return a


# ===========================================================================
# second-order cone {(t, x): |x| <= t}, barrier -1/2 log(z0^2 - |z1|^2)
# ===========================================================================

def soc_J(d):
    J = -np.eye(d)
    J[0, 0] = 1.0
    return J


def jdot(u, v):
    """u' J v for each cone."""
    return u[:, 0] * v[:, 0] - np.sum(u[:, 1:] * v[:, 1:], axis=1)


def soc_scale(s, z):
    """NT scaling point of the SOC (CVXOPT construction).

    s_bar = s / sqrt(s'Js), z_bar = z / sqrt(z'Jz), gamma = sqrt((1 + s_bar'z_bar)/2),
    w_bar = (s_bar + J z_bar) / (2 gamma), eta = (s'Js / z'Jz)^(1/4);
    W = eta [[w0, w1'], [w1, I + w1 w1'/(1 + w0)]]; H = W'W = eta^2 (2 w w' - J);
    lambda = W z.
    """
    N, d = s.shape
    ns = np.sqrt(jdot(s, s))
    nz = np.sqrt(jdot(z, z))
    sb = s / ns[:, None]
    zb = z / nz[:, None]
    gamma = np.sqrt((1.0 + np.sum(sb * zb, axis=1)) / 2.0)
    Jzb = zb.copy()
    Jzb[:, 1:] *= -1.0
    wb = (sb + Jzb) / (2.0 * gamma[:, None])
    eta = np.sqrt(ns / nz)
    Wb = np.zeros((N, d, d))
    Wb[:, 0, 0] = wb[:, 0]
    Wb[:, 0, 1:] = wb[:, 1:]
    Wb[:, 1:, 0] = wb[:, 1:]
    Wb[:, 1:, 1:] = np.eye(d - 1)[None] + np.einsum("ci,cj->cij", wb[:, 1:], wb[:, 1:]) / (1.0 + wb[:, 0])[:, None, None]
    W = eta[:, None, None] * Wb
    H = np.einsum("cij,cjk->cik", W.transpose(0, 2, 1), W)
    lam = np.einsum("cij,cj->ci", W, z)
    Winv = np.linalg.inv(W)
    return {"wbar": wb, "eta": eta, "W": W, "Winv": Winv, "lam": lam, "H": H}


def soc_circ(u, v):
    """Jordan product of the SOC: (u'v, u0 v1 + v0 u1)."""
    out = np.empty_like(u)
    out[:, 0] = np.sum(u * v, axis=1)
    out[:, 1:] = u[:, :1] * v[:, 1:] + v[:, :1] * u[:, 1:]
    return out


def soc_inv_circ(lam, v):
    """x solving lam o x = v (the operator lam \\ v)."""
    det = jdot(lam, lam)
    x0 = (lam[:, 0] * v[:, 0] - np.sum(lam[:, 1:] * v[:, 1:], axis=1)) / det
    out = np.empty_like(v)
    out[:, 0] = x0
    out[:, 1:] = (v[:, 1:] - x0[:, None] * lam[:, 1:]) / lam[:, :1]
    return out


def soc_step(x, dx):
    """Largest alpha with x + alpha dx in the SOC, from the quadratic in alpha."""
    a = jdot(dx, dx)
    b = jdot(x, dx)
    c = jdot(x, x)
    out = np.full(x.shape[0], np.inf)
    for i in range(x.shape[0]):
        roots = _pos_roots(a[i], 2.0 * b[i], c[i])
        if roots:
            out[i] = min(roots)
    return out


def _pos_roots(a, b, c):
    """Positive roots of a t^2 + b t + c = 0 (cancellation-free formula)."""
    if a == 0.0:
        if b == 0.0:
            return []
        t = -c / b
        return [t] if t > 0 else []
    disc = b * b - 4.0 * a * c
    if disc < 0:
        return []
    sq = math.sqrt(disc)
    qq = -0.5 * (b + math.copysign(sq, b))
    roots = []
    if qq != 0.0:
        roots += [qq / a, c / qq]
    else:
        roots += [0.0]
    return [r for r in roots if r > 0]


# ===========================================================================
# PSD cone, svec encoding, barrier -log det X
# ===========================================================================

def svec_dim(k):
    return k * (k + 1) // 2


def svec_index(k):
    """List of (i, j, factor) for each svec slot: upper triangle column by column."""
    out = []
    for j in range(k):
        for i in range(j + 1):
            out.append((i, j, 1.0 if i == j else SQRT2))
    return out


def smat(v, k):
    """svec (N, k(k+1)/2) -> symmetric matrices (N, k, k)."""
    N = v.shape[0]
    X = np.zeros((N, k, k))
    for p, (i, j, f) in enumerate(svec_index(k)):
        X[:, i, j] = v[:, p] / f
        X[:, j, i] = v[:, p] / f
    return X


def svec(X):
    k = X.shape[-1]
    return np.stack([X[:, i, j] * f for (i, j, f) in svec_index(k)], axis=1)


def psd_scale(s, z, k):
    """NT scaling of the PSD cone via Cholesky factors and an SVD.

    Ls = chol(S), Lz = chol(Z), Lz' Ls = U diag(lam) V';  R = Ls V lam^-1/2,
    R^-1 = lam^-1/2 U' Lz'.  W(X) = R'XR, W^-T(X) = R^-1 X R^-T,
    W'(Y) = R Y R', lambda = diag(lam).  H(X) = M X M with M = R R'.
    """
    S = smat(s, k)
    Z = smat(z, k)
    Ls = np.linalg.cholesky(S)
    Lz = np.linalg.cholesky(Z)
    U, lam, Vt = np.linalg.svd(np.einsum("cji,cjk->cik", Lz, Ls))
    R = np.einsum("cij,ckj->cik", Ls, Vt) / np.sqrt(lam)[:, None, :]
    Rinv = np.einsum("ci,cji,ckj->cik", 1.0 / np.sqrt(lam), U, Lz)
    M = np.einsum("cij,ckj->cik", R, R)
    H = psd_H_from_M(M)
    return {"R": R, "Rinv": Rinv, "lam": lam, "M": M, "H": H}


def psd_H_from_M(M):
    """Matrix of X -> M X M in svec coordinates:
    H[(i,j),(k,l)] = c_ij c_kl / 2 (M_ik M_jl + M_il M_jk)."""
    k = M.shape[-1]
    idx = svec_index(k)
    sd = len(idx)
    H = np.zeros((M.shape[0], sd, sd))
    for p, (i, j, cij) in enumerate(idx):
        for r, (kk, ll, ckl) in enumerate(idx):
            H[:, p, r] = cij * ckl / 2.0 * (M[:, i, kk] * M[:, j, ll] + M[:, i, ll] * M[:, j, kk])
    return H


def psd_step(x, dx, k):
    """Largest alpha with X + alpha dX PSD: 1 / max(0, -lambda_min(L^-1 dX L^-T))."""
    X = smat(x, k)
    dX = smat(dx, k)
    L = np.linalg.cholesky(X)
    Li = np.linalg.inv(L)
    Mm = np.einsum("cij,cjk,clk->cil", Li, dX, Li)
    lmin = np.linalg.eigvalsh(Mm)[:, 0]
    out = np.full(x.shape[0], np.inf)
    neg = lmin < 0
    out[neg] = -1.0 / lmin[neg]
    return out


def psd_circ(U, V):
    return 0.5 * (np.einsum("cij,cjk->cik", U, V) + np.einsum("cij,cjk->cik", V, U))


# ===========================================================================
# exponential and power cones: barriers of the dual cones (degree 3)
# ===========================================================================

def f_exp(zj, params=None):
    """f(z) = -log(z2 - z1 - z1 log(z3/(-z1))) - log(-z1) - log(z3) (z in K_exp*)."""
    z1, z2, z3 = zj
    psi = z2 - z1 - z1 * (z3 / (-z1)).log()
    return -(psi.log()) - ((-z1).log()) - z3.log()


def f_pow(zj, alpha):
    """f(z) = -log((z1/a)^(2a) (z2/(1-a))^(2(1-a)) - z3^2) - (1-a) log z1 - a log z2."""
    z1, z2, z3 = zj
    a = alpha
    phi = (z1 / a).powc(2 * a) * (z2 / (1 - a)).powc(2 * (1 - a)) - z3 * z3
    return -(phi.log()) - (z1.log()) * (1 - a) - (z2.log()) * a


def exp_primal_interior(s):
    """s in int K_exp: s2 > 0, s3 > 0 and s2 log(s3/s2) - s1 > 0."""
    out = (s[:, 1] > 0) & (s[:, 2] > 0)
    with np.errstate(all="ignore"):
        out &= s[:, 1] * np.log(s[:, 2] / s[:, 1]) - s[:, 0] > 0
    return out


def exp_dual_interior(z):
    """z in int K_exp*: z1 < 0, z3 > 0 and z2 - z1 - z1 log(z3/(-z1)) > 0."""
    out = (z[:, 0] < 0) & (z[:, 2] > 0)
    with np.errstate(all="ignore"):
        out &= z[:, 1] - z[:, 0] - z[:, 0] * np.log(z[:, 2] / (-z[:, 0])) > 0
    return out


def pow_primal_interior(s, alpha):
    """s in int K_pow: s1, s2 > 0 and s1^a s2^(1-a) > |s3| (log form)."""
    out = (s[:, 0] > 0) & (s[:, 1] > 0)
    with np.errstate(all="ignore"):
        out &= 2 * alpha * np.log(s[:, 0]) + 2 * (1 - alpha) * np.log(s[:, 1]) - np.log(s[:, 2] ** 2) > 0
    return out


def pow_dual_interior(z, alpha):
    """z in int K_pow*: z1, z2 > 0 and (z1/a)^a (z2/(1-a))^(1-a) > |z3| (log form)."""
    out = (z[:, 0] > 0) & (z[:, 1] > 0)
    with np.errstate(all="ignore"):
        out &= (2 * alpha * np.log(z[:, 0] / alpha) + 2 * (1 - alpha) * np.log(z[:, 1] / (1 - alpha))
                - np.log(z[:, 2] ** 2) > 0)
    return out


class NonsymFamily:
    """Shared operations of the exp and pow families, driven by the barrier f."""

    def __init__(self, kind, alpha=None):
        self.kind = kind
        self.alpha = alpha  # (N,) for pow

    def f(self, zj, params):
        return f_exp(zj) if self.kind == "exp" else f_pow(zj, params)

    def unit_point(self, N):
        """The point u with u = -grad f(u), in both K and K*."""
        if self.kind == "pow":
            a = self.alpha
            return np.stack([np.sqrt(1 + a), np.sqrt(2 - a), np.zeros_like(a)], axis=1)
        return np.tile(_exp_unit_point(), (N, 1))

    def grad_hess(self, z):
        return jets.derivatives(self.f, z, self.alpha)

    def third(self, z, u, v):
        return jets.third(self.f, z, u, v, self.alpha)

    def primal_interior(self, s):
        if self.kind == "exp":
            return exp_primal_interior(s)
        return pow_primal_interior(s, self.alpha)

    def dual_interior(self, z):
        if self.kind == "exp":
            return exp_dual_interior(z)
        return pow_dual_interior(z, self.alpha)

    def conj_grad_point(self, s, with_status=False, steps=200):
        """z~ = -grad f*(s): the z in int K* with -grad f(z) = s.

        Solving -grad f(z) = s reduces to one scalar equation (derived from
        the barrier formulas; the identity -grad f(z~) = s is checked by the
        jet derivatives in the tests).  The scalar root is found by plain
        bisection on its logarithm.

        exp:  with r = log(s3/s2) - s1/s2 > 0, find t > 0 with
              log(1 + 1/t) + 1/t = r; then z~ = (u, v, w) with u = -t/s2,
              w = (1 + t)/s3, v = 1/s2 + u + u log(w/(-u)).
        pow:  with C = 2 log|s3| - 2a log(a s1) - 2(1-a) log((1-a) s2), find
              y > 0 with 2a log(1+a+2ay) + 2(1-a) log(2-a+2(1-a)y)
              - log(1+y) - log y - log 4 + C = 0; then
              z~ = ((1+a+2ay)/s1, (2-a+2(1-a)y)/s2, -2y/s3)  (y = 0 if s3 = 0).
        Both left sides decrease strictly in t (resp. y).
        """
        N = s.shape[0]
        s1, s2, s3 = s[:, 0], s[:, 1], s[:, 2]
        ok = self.primal_interior(s)
        z = np.full((N, 3), np.nan)
        with np.errstate(all="ignore"):
            if self.kind == "exp":
                r = np.log(s3 / s2) - s1 / s2
                lo = np.full(N, -80.0)
                hi = np.full(N, 80.0)

                def gfun(lt):
                    t = np.exp(lt)
                    return np.log1p(1.0 / t) + 1.0 / t - r
                for _ in range(steps):
                    mid = 0.5 * (lo + hi)
                    pos = gfun(mid) > 0          # root lies above mid
                    lo = np.where(pos, mid, lo)
                    hi = np.where(pos, hi, mid)
                t = np.exp(0.5 * (lo + hi))
                u = -t / s2
                w = (1.0 + t) / s3
                v = 1.0 / s2 + u + u * np.log(w / (-u))
                z = np.stack([u, v, w], axis=1)
            else:
                a = self.alpha
                Cc = 2.0 * np.log(np.abs(s3)) - 2 * a * np.log(a * s1) - 2 * (1 - a) * np.log((1 - a) * s2)

                def hfun(ly):
                    y = np.exp(ly)
                    return (2 * a * np.log(1 + a + 2 * a * y) + 2 * (1 - a) * np.log(2 - a + 2 * (1 - a) * y)
                            - np.log1p(y) - ly - np.log(4.0) + Cc)
                lo = np.full(N, -200.0)
                hi = np.full(N, 200.0)
                for _ in range(steps):
                    mid = 0.5 * (lo + hi)
                    pos = hfun(mid) > 0
                    lo = np.where(pos, mid, lo)
                    hi = np.where(pos, hi, mid)
                y = np.where(s3 == 0, 0.0, np.exp(0.5 * (lo + hi)))
                z3 = np.where(s3 == 0, 0.0, -2.0 * y / np.where(s3 == 0, 1.0, s3))
                z = np.stack([(1 + a + 2 * a * y) / s1, (2 - a + 2 * (1 - a) * y) / s2, z3], axis=1)
        ok &= np.isfinite(z).all(axis=1)
        if with_status:
            return z, ok
        if not ok.all():
            raise np.linalg.LinAlgError("conjugate point of a point outside int K")
        return z

    def hess_factor(self, z):
        """G with G G' = Hess f(z), built from PSD rank-one pieces.

        exp: f = -log psi - log(-z1) - log z3 with psi concave and
             -Hess psi = c c', c = (1/sqrt(-z1), 0, sqrt(-z1)/z3); so
             Hess f = c c'/psi + grad psi grad psi'/psi^2 + e1 e1'/z1^2 + e3 e3'/z3^2.
        pow: with Pi = (z1/a)^a (z2/(1-a))^(1-a) (concave, -Hess Pi = Pi a(1-a) d d',
             d = (1/z1, -1/z2, 0)), f = -log(Pi - z3) - log(Pi + z3) - (1-a) log z1 - a log z2
             and Hess f = sum over +- of [Pi a(1-a) d d'/(Pi -+ z3)
             + grad(Pi -+ z3) grad(Pi -+ z3)'/(Pi -+ z3)^2] + diag((1-a)/z1^2, a/z2^2, 0).
        Near the boundary of K* the Hessian's condition number exceeds 1/eps;
        G has the square root of it, so its SVD yields accurate eigenpairs.
        """
        N = z.shape[0]
        z1, z2, z3 = z[:, 0], z[:, 1], z[:, 2]
        if self.kind == "exp":
            ell = np.log(z3 / (-z1))
            psi = z2 - z1 - z1 * ell
            gpsi = np.stack([-ell, np.ones(N), -z1 / z3], axis=1)
            c = np.stack([1.0 / np.sqrt(-z1), np.zeros(N), np.sqrt(-z1) / z3], axis=1)
            e1 = np.zeros((N, 3)); e1[:, 0] = 1.0 / (-z1)
            e3 = np.zeros((N, 3)); e3[:, 2] = 1.0 / z3
            cols = [c / np.sqrt(psi)[:, None], gpsi / psi[:, None], e1, e3]
        else:
            a = self.alpha
            Pi = (z1 / a) ** a * (z2 / (1 - a)) ** (1 - a)
            gPi = Pi[:, None] * np.stack([a / z1, (1 - a) / z2, np.zeros(N)], axis=1)
            d = np.stack([1.0 / z1, -1.0 / z2, np.zeros(N)], axis=1)
            e3 = np.zeros((N, 3)); e3[:, 2] = 1.0
            cols = []
            for sgn in (-1.0, 1.0):
                den = Pi + sgn * z3
                cols.append(np.sqrt(Pi * a * (1 - a) / den)[:, None] * d)
                cols.append((gPi + sgn * e3) / den[:, None])
            e1 = np.zeros((N, 3)); e1[:, 0] = np.sqrt(1 - a) / z1
            e2 = np.zeros((N, 3)); e2[:, 1] = np.sqrt(a) / z2
            cols += [e1, e2]
        return np.stack(cols, axis=2)

    def scale(self, s, z, mu, force_dual=False):
        """Primal-dual (rank-4 BFGS) scaling with the dual-scaling fallback.

        H_pd = s s'/<s,z> + ds ds'/<ds,dz> + mu u u'/(u' Hf^-1 u), with
        ds = s - mu_i s~, dz = z - mu_i z~, u = z x z~ (cross product); this
        equals S (S'Z)^-1 S' + Ha - Ha Z (Z'Ha Z)^-1 Z'Ha.  H_dual = mu Hf(z)
        when mu_i mu~_i - 1 < sqrt(eps) or when forced.  Both are returned in
        spectral form (eigenvalues = squared singular values of a factor).
        """
        g, _ = self.grad_hess(z)
        st = -g
        zt, ok = self.conj_grad_point(s, with_status=True)
        mu_i = np.sum(s * z, axis=1) / 3.0
        mut_i = np.sum(st * zt, axis=1) / 3.0
        with np.errstate(all="ignore"):
            dual = ~ok | ~(mu_i * mut_i - 1.0 >= THETA_PD) | force_dual
        G = self.hess_factor(z)
        Ug, sg, _ = np.linalg.svd(G, full_matrices=False)
        hinv = {"U": Ug, "sig": sg}
        dsv = s - mu_i[:, None] * st
        dzv = z - mu_i[:, None] * zt
        uu = np.cross(z, zt)
        with np.errstate(all="ignore"):
            uHu = np.sum((np.einsum("cji,cj->ci", Ug, uu) / sg) ** 2, axis=1)
            Gpd = np.stack([s / np.sqrt(np.sum(s * z, axis=1))[:, None],
                            dsv / np.sqrt(np.sum(dsv * dzv, axis=1))[:, None],
                            uu * np.sqrt(mu / uHu)[:, None]], axis=2)
        Gd = np.sqrt(mu) * G
        lam = np.empty((s.shape[0], 3))
        V = np.empty((s.shape[0], 3, 3))
        if np.any(dual):
            Ud, sd, _ = np.linalg.svd(Gd[dual], full_matrices=False)
            lam[dual], V[dual] = sd**2, Ud
        if np.any(~dual):
            Up, sp_, _ = np.linalg.svd(Gpd[~dual], full_matrices=False)
            lam[~dual], V[~dual] = sp_**2, Up
        H = np.einsum("cij,cj,ckj->cik", V, lam, V)
        return {"H": H, "lam": lam, "V": V, "st": st, "zt": zt, "branch": dual.astype(np.int32),
                "grad": g, "hinv": hinv}

    @staticmethod
    def hinv_apply(hinv, v):
        """Hess f(z)^-1 v from the SVD of its factor."""
        U, sg = hinv["U"], hinv["sig"]
        return np.einsum("cij,cj->ci", U, np.einsum("cji,cj->ci", U, v) / sg**2)

    def bfgs_raw(self, s, z, st, zt, Hf, mu):
        """The rank-4 formula S (S'Z)^-1 S' + Ha - Ha Z (Z'Ha Z)^-1 Z'Ha, evaluated literally."""
        S = np.stack([s, st], axis=2)
        Z = np.stack([z, zt], axis=2)
        Ha = mu * Hf
        SZ = np.einsum("cji,cjk->cik", S, Z)
        t1 = np.einsum("cij,cjk,clk->cil", S, np.linalg.inv(SZ), S)
        HaZ = np.einsum("cij,cjk->cik", Ha, Z)
        ZHZ = np.einsum("cji,cjk->cik", Z, HaZ)
        t2 = Ha - np.einsum("cij,cjk,clk->cil", HaZ, np.linalg.inv(ZHZ), HaZ)
        return t1 + t2


_EXP_UNIT = None


def _exp_unit_point():
    """Solve u = -grad f(u) for the exp-cone dual barrier by Newton's method."""
    global _EXP_UNIT
    if _EXP_UNIT is None:
        u = np.array([[-1.051383945322714, 0.556409619469370, 1.258967884768947]])
        for _ in range(50):
            g, H = jets.derivatives(f_exp, u)
            F = u + g
            J = np.eye(3)[None] + H
            u = u - np.linalg.solve(J, F[..., None])[..., 0]
        _EXP_UNIT = u[0].copy()
    return _EXP_UNIT


# ===========================================================================
# spectral forms of the symmetric-cone scalings
# ===========================================================================

def soc_spectral(wb, eta):
    """Eigenpairs of H = eta^2 (2 wb wb' - J) with wb'J wb = 1.

    With r = |wb_1| and u = wb_1 / r: (1, +-u)/sqrt(2) carry eta^2 (wb0 +- r)^2
    (the smaller one written as eta^2 / (wb0 + r)^2), and every (0, y) with
    y orthogonal to u carries eta^2.
    """
    N, d = wb.shape
    lam = np.empty((N, d))
    V = np.zeros((N, d, d))
    r = np.linalg.norm(wb[:, 1:], axis=1)
    big = wb[:, 0] + r
    lam[:, 0] = eta**2 * big**2
    lam[:, 1] = eta**2 / big**2
    lam[:, 2:] = (eta**2)[:, None]
    u = np.zeros((N, d - 1))
    pos = r > 0
    u[pos] = wb[pos, 1:] / r[pos, None]
    u[~pos, 0] = 1.0
    h = 1.0 / math.sqrt(2.0)
    V[:, 0, 0] = h
    V[:, 1:, 0] = h * u
    V[:, 0, 1] = h
    V[:, 1:, 1] = -h * u
    if d > 2:
        # Householder reflection mapping e_1 to u; its other columns span u-perp
        e1 = np.zeros(d - 1)
        e1[0] = 1.0
        w = u - e1[None]
        ww = np.sum(w * w, axis=1)
        Q = np.broadcast_to(np.eye(d - 1), (N, d - 1, d - 1)).copy()
        nz = ww > 0
        Q[nz] -= 2.0 * np.einsum("ci,cj->cij", w[nz], w[nz]) / ww[nz, None, None]
        V[:, 1:, 2:] = Q[:, :, 1:]
    return lam, V


def psd_spectral(R):
    """Eigenpairs of X -> M X M (M = R R') in svec coordinates.

    With M = sum_i m_i q_i q_i' (m_i = sigma_i(R)^2 from an SVD of R), the
    svec images of q_i q_i' and (q_i q_j' + q_j q_i')/sqrt(2) are orthonormal
    eigenvectors with eigenvalues m_i m_j.
    """
    N, k, _ = R.shape
    Ur, sig, _ = np.linalg.svd(R)
    m = sig**2
    idx = svec_index(k)
    sd = len(idx)
    lam = np.empty((N, sd))
    V = np.empty((N, sd, sd))
    col = 0
    for j in range(k):
        for i in range(j + 1):
            qi, qj = Ur[:, :, i], Ur[:, :, j]
            if i == j:
                E = np.einsum("ca,cb->cab", qi, qi)
            else:
                E = (np.einsum("ca,cb->cab", qi, qj) + np.einsum("ca,cb->cab", qj, qi)) / SQRT2
            V[:, :, col] = svec(E)
            lam[:, col] = m[:, i] * m[:, j]
            col += 1
    return lam, V
