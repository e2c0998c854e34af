"""The primal-dual interior-point method of the paper, plain FP64 on the CPU.

TEST INFRASTRUCTURE ONLY: this is the oracle.  It is called by tests/, by the
smoke check and by the benchmark's CPU-baseline leg, never by the product
path, and it shares no code with the GPU library.

Follows Algorithm 1 (Sec. 3.2) step by step:
  setup   equilibrate P, A, q, b; choose the initial point
  loop    residuals + termination (eq. residuals-objectives, termination-check,
          infeasibility-check) -> scaling H (Appendix A) -> factor K
          (eq. linsys_2x2) -> affine direction with d = (G, kappa tau, s)
          (eq. affine-step, step-direction) -> alpha_a -> sigma = (1-alpha_a)^3
          -> combined direction (eq. ds-correction-step with the Mehrotra /
          3rd-order corrections) -> alpha_c with the neighbourhood check ->
          v <- v + 0.99 alpha_c Delta_c.

Readings where the paper is silent or inconsistent (each also listed in the
design notes):
  * Delta tau uses the first printed form; the second drops kappa/tau.
  * affine d: d_kappa = kappa tau and d_s = s.
  * dual-infeasibility test multiplies by q'x (printed: b'z).
  * eps_feas = eps_inf = 1e-8, max_iter = 200.
  * equilibration: 10 modified Ruiz passes, factors clamped to [1e-4, 1e4],
    row factors averaged over the rows of each SOC/exp/pow/PSD cone, cost
    scale c = 1/max(1, mean_j |P^_j|_inf, |D q|_inf) clamped to [1e-4, 1e4].
  * initial point: symmetric cones only -> solve K with H = I (0 on zero
    rows) for [-q; b], s = -z, then shift s and z into the interior by
    (1 + alpha) e when alpha = max_i(-lambda_min) >= 0; with exp/pow cones ->
    x = 0 and s = z = the unit point of each cone.
  * step rule: alpha_0 = min(1, tau/kappa ratio tests, exact symmetric-cone
    boundary steps); backtrack x0.8 from alpha_0 while an exp/pow cone leaves
    its interior or (combined step) violates N(beta); stop below 1e-10.
  * alpha_c < 0.1 with a primal-dual exp/pow scaling -> redo the iteration
    with dual scaling; alpha_c < 1e-4 -> insufficient progress.
  * grad f* is evaluated through scalar bisection on a 1-d reduction of
    -grad f(z) = s (see cones.NonsymFamily.conj_grad_point).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from . import cones as C
from .linsys import KKT, SpectralBlocks

ZERO, NONNEG, SOC, EXP, POW, PSD = 0, 1, 2, 3, 4, 5

SOLVED, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, MAX_ITER, INSUFFICIENT_PROGRESS, NUMERICAL_ERROR = 1, 2, 3, 4, 5, 6
STATUS_NAMES = {0: "unsolved", 1: "solved", 2: "primal_infeasible", 3: "dual_infeasible",
                4: "max_iter", 5: "insufficient_progress", 6: "numerical_error"}


@dataclasses.dataclass
class Settings:
    eps_feas: float = 1e-8
    eps_inf: float = 1e-8
    max_iter: int = 200
    static_reg: float = 1e-8
    dyn_reg: float = 2.0 ** -104
    ir_abstol: float = 1e-12
    ir_reltol: float = 1e-12
    ir_max: int = 10
    beta: float = 1e-6
    backtrack: float = 0.8
    step_fraction: float = 0.99
    min_alpha: float = 1e-10
    insufficient_alpha: float = 1e-4
    dual_retry_alpha: float = 0.1
    equilibrate: bool = True
    equil_iters: int = 10
    equil_min: float = 1e-4
    equil_max: float = 1e4
    force_dual_scaling: bool = False
    verbose: bool = False


@dataclasses.dataclass
class Group:
    kind: int
    rows: np.ndarray          # (N, d) row indices of the cones of this family
    alpha: np.ndarray = None  # POW exponents
    k: int = 0                # PSD side

    @property
    def N(self):
        return self.rows.shape[0]

    @property
    def d(self):
        return self.rows.shape[1]

    def degree(self):
        if self.kind == ZERO:
            return 0
        if self.kind == NONNEG:
            return self.N
        if self.kind == SOC:
            return self.N
        if self.kind == PSD:
            return self.N * self.k
        return 3 * self.N


def build_groups(cones):
    """Cone list (kind, dim, alpha) in row order -> families of equal-size cones."""
    rows = {ZERO: [], NONNEG: [], EXP: [], POW: []}
    soc = {}
    psd = {}
    alphas = []
    r = 0
    for kind, dim, a in cones:
        if kind in (ZERO, NONNEG):
            rows[kind] += [[r + i] for i in range(dim)]
            r += dim
        elif kind == SOC:
            soc.setdefault(dim, []).append(list(range(r, r + dim)))
            r += dim
        elif kind in (EXP, POW):
            rows[kind].append(list(range(r, r + 3)))
            if kind == POW:
                alphas.append(a)
            r += 3
        elif kind == PSD:
            sd = dim * (dim + 1) // 2
            psd.setdefault(dim, []).append(list(range(r, r + sd)))
            r += sd
        else:
            raise ValueError(f"unknown cone kind {kind}")
    groups = []
    for kind in (ZERO, NONNEG):
        if rows[kind]:
            groups.append(Group(kind, np.array(rows[kind], dtype=np.int64)))
    for dim in sorted(soc):
        groups.append(Group(SOC, np.array(soc[dim], dtype=np.int64)))
    if rows[EXP]:
        groups.append(Group(EXP, np.array(rows[EXP], dtype=np.int64)))
    if rows[POW]:
        groups.append(Group(POW, np.array(rows[POW], dtype=np.int64), alpha=np.array(alphas)))
    for k in sorted(psd):   # PSD cones of several sides: one family per side
        groups.append(Group(PSD, np.array(psd[k], dtype=np.int64), k=k))
    return groups, r


def _fam(g):
    return C.NonsymFamily("exp" if g.kind == EXP else "pow", g.alpha if g.kind == POW else None)


def inf_norm(v):
    return float(np.max(np.abs(v))) if v.size else 0.0


# ===========================================================================
# setup: equilibration and initial point
# ===========================================================================

def equilibrate(P_full, A, q, groups, st: Settings):
    """Modified Ruiz equilibration; returns (D, E, c)."""
    n, m = A.shape[1], A.shape[0]
    D = np.ones(n)
    E = np.ones(m)
    if not st.equilibrate:
        return D, E, 1.0
    P_abs = abs(sp.csr_matrix(P_full))
    A_abs = abs(sp.csr_matrix(A))
    for _ in range(st.equil_iters):
        Ps = sp.diags(D) @ P_abs @ sp.diags(D)
        As = sp.diags(E) @ A_abs @ sp.diags(D)
        colP = np.asarray(Ps.max(axis=0).todense()).ravel() if n else np.zeros(0)
        colA = np.asarray(As.max(axis=0).todense()).ravel() if n else np.zeros(0)
        cn = np.maximum(colP, colA)
        d = np.where(cn > 0, 1.0 / np.sqrt(np.where(cn > 0, cn, 1.0)), 1.0)
        rn = np.asarray(As.max(axis=1).todense()).ravel() if m else np.zeros(0)
        e = np.where(rn > 0, 1.0 / np.sqrt(np.where(rn > 0, rn, 1.0)), 1.0)
        for g in groups:
            if g.kind in (SOC, EXP, POW, PSD):
                e[g.rows] = np.mean(e[g.rows], axis=1, keepdims=True)
        d = np.clip(d, st.equil_min, st.equil_max)
        e = np.clip(e, st.equil_min, st.equil_max)
        D = np.clip(D * d, st.equil_min, st.equil_max)
        E = np.clip(E * e, st.equil_min, st.equil_max)
    Ps = sp.diags(D) @ P_abs @ sp.diags(D)
    colP = np.asarray(Ps.max(axis=0).todense()).ravel() if n else np.zeros(0)
    mean_col = float(np.mean(colP)) if n else 0.0
    c = 1.0 / max(1.0, mean_col, inf_norm(D * q))
    c = min(max(c, st.equil_min), st.equil_max)
    return D, E, c


def unit_vector(groups, m):
    """The identity element e of the (symmetric part of the) cone product; 0 on zero rows."""
    e = np.zeros(m)
    for g in groups:
        if g.kind == NONNEG:
            e[g.rows[:, 0]] = 1.0
        elif g.kind == SOC:
            e[g.rows[:, 0]] = 1.0
        elif g.kind == PSD:
            for p, (i, j, f) in enumerate(C.svec_index(g.k)):
                if i == j:
                    e[g.rows[:, p]] = 1.0
        elif g.kind in (EXP, POW):
            e[g.rows] = _fam(g).unit_point(g.N)
    return e


def max_neg_eig(v, groups):
    """max over symmetric cones of -lambda_min(v_cone) (-inf if there are none)."""
    out = -np.inf
    for g in groups:
        x = v[g.rows]
        if g.kind == NONNEG:
            out = max(out, float(np.max(-x[:, 0])))
        elif g.kind == SOC:
            out = max(out, float(np.max(np.linalg.norm(x[:, 1:], axis=1) - x[:, 0])))
        elif g.kind == PSD:
            out = max(out, float(np.max(-np.linalg.eigvalsh(C.smat(x, g.k))[:, 0])))
    return out


# ===========================================================================
# the solver
# ===========================================================================

class Solver:
    def __init__(self, prob, settings: Settings | None = None):
        self.st = settings or Settings()
        self.prob = prob
        self.n, self.m = prob.n, prob.m
        P = sp.csr_matrix(prob.P)
        self.P_full = sp.csr_matrix(P + P.T - sp.diags(P.diagonal()))
        self.A = sp.csr_matrix(prob.A)
        self.q = prob.q.copy()
        self.b = prob.b.copy()
        self.groups, mm = build_groups(prob.cones)
        assert mm == self.m
        self.nu = sum(g.degree() for g in self.groups)
        self.has_nonsym = any(g.kind in (EXP, POW) for g in self.groups)
        self.D, self.E, self.c = equilibrate(self.P_full, self.A, self.q, self.groups, self.st)
        Dm, Em = sp.diags(self.D), sp.diags(self.E)
        self.Ps = sp.csr_matrix(self.c * (Dm @ self.P_full @ Dm))
        self.qs = self.c * self.D * self.q
        self.As = sp.csr_matrix(Em @ self.A @ Dm)
        self.bs = self.E * self.b
        self.history = []
        self.status = 0
        self.iterations = 0
        self.ir_solves = 0
        self.guard_hits = 0
        self.dual_switches = 0
        self._init_point()

    # -- helpers ---------------------------------------------------------------
    def _kkt(self, blocks):
        return KKT(self.Ps, self.As, blocks, self.st.static_reg, self.st.dyn_reg)

    def _solve(self, kkt, r1, r2):
        x, z, info = kkt.solve(r1, r2, self.st.ir_abstol, self.st.ir_reltol, self.st.ir_max)
        self.ir_solves += info["solves"]
        return x, z

    def _init_point(self):
        n, m = self.n, self.m
        if not self.has_nonsym:
            blocks = []
            for g in self.groups:
                lam = np.zeros((g.N, g.d)) if g.kind == ZERO else np.ones((g.N, g.d))
                blocks.append((g.rows, SpectralBlocks(lam, np.broadcast_to(np.eye(g.d), (g.N, g.d, g.d)).copy())))
            kkt = self._kkt(blocks)
            x, z = self._solve(kkt, -self.qs, self.bs)
            s = -z.copy()
            for g in self.groups:
                if g.kind == ZERO:
                    s[g.rows] = 0.0
            e = unit_vector(self.groups, m)
            ap = max_neg_eig(s, self.groups)
            if ap >= 0:
                s = s + (1.0 + ap) * e
            ad = max_neg_eig(z, self.groups)
            if ad >= 0:
                z = z + (1.0 + ad) * e
            self.x, self.s, self.z = x, s, z
        else:
            e = unit_vector(self.groups, m)
            self.x = np.zeros(n)
            self.s = e.copy()
            self.z = e.copy()
        self.tau, self.kappa = 1.0, 1.0

    def mu(self, s=None, z=None, tau=None, kappa=None):
        s = self.s if s is None else s
        z = self.z if z is None else z
        tau = self.tau if tau is None else tau
        kappa = self.kappa if kappa is None else kappa
        return (s @ z + kappa * tau) / (self.nu + 1)

    # -- residuals and termination on the unscaled data ---------------------------
    def residuals(self):
        t = self.tau
        xb = self.D * self.x / t
        sb = self.s / self.E / t
        zb = self.E * self.z / (self.c * t)
        Pxb = self.P_full @ xb
        rp = -(self.A @ xb) - sb + self.b
        rd = Pxb + self.A.T @ zb + self.q
        xPx = xb @ Pxb
        gp = 0.5 * xPx + self.q @ xb
        gd = -0.5 * xPx - self.b @ zb
        return dict(xb=xb, sb=sb, zb=zb, rp=rp, rd=rd, gp=gp, gd=gd,
                    nrp=inf_norm(rp), nrd=inf_norm(rd))

    def check(self, r):
        st = self.st
        eps = st.eps_feas
        b_n, q_n = inf_norm(self.b), inf_norm(self.q)
        xn, sn, zn = inf_norm(r["xb"]), inf_norm(r["sb"]), inf_norm(r["zb"])
        gap = abs(r["gp"] - r["gd"])
        if (r["nrp"] < eps * max(1.0, b_n + xn + sn) and r["nrd"] < eps * max(1.0, q_n + xn + zn)
                and gap < eps * max(1.0, min(abs(r["gp"]), abs(r["gd"])))):
            return SOLVED
        # certificates on the unnormalised (unscaled) iterate
        x = self.D * self.x
        z = self.E * self.z / self.c
        s = self.s / self.E
        ei = st.eps_inf
        bz = self.b @ z
        if bz < -ei and inf_norm(self.A.T @ z) < -ei * max(1.0, inf_norm(x) + inf_norm(z)) * bz:
            return PRIMAL_INFEASIBLE
        qx = self.q @ x
        if (qx < -ei and inf_norm(self.P_full @ x) < -ei * max(1.0, inf_norm(x)) * qx
                and inf_norm(self.A @ x + s) < -ei * max(1.0, inf_norm(x) + inf_norm(s)) * qx):
            return DUAL_INFEASIBLE
        return 0

    # -- cone layer ----------------------------------------------------------------
    def scale(self, mu, force_dual=False):
        """Per-family scaling state (aligned with self.groups); "Hb" is the H block operator."""
        out = []
        for g in self.groups:
            s, z = self.s[g.rows], self.z[g.rows]
            if g.kind == ZERO:
                sc = {"Hb": SpectralBlocks(np.zeros((g.N, 1)), np.ones((g.N, 1, 1)))}
            elif g.kind == NONNEG:
                sc = C.nn_scale(s, z)
                sc["Hb"] = SpectralBlocks(s / z, np.ones((g.N, 1, 1)))
            elif g.kind == SOC:
                sc = C.soc_scale(s, z)
                sc["Hb"] = SpectralBlocks(*C.soc_spectral(sc["wbar"], sc["eta"]))
            elif g.kind == PSD:
                sc = C.psd_scale(s, z, g.k)
                sc["Hb"] = SpectralBlocks(*C.psd_spectral(sc["R"]))
            else:
                sc = _fam(g).scale(s, z, mu, force_dual=force_dual or self.st.force_dual_scaling)
                sc["Hb"] = SpectralBlocks(sc["lam"], sc["V"])
            out.append(sc)
        return out

    def ds_combined(self, scal, dsa, dza, sigma, mu):
        """d_s of the combined step (eq. ds-correction-step), per family."""
        ds = np.zeros(self.m)
        for g, sc in zip(self.groups, scal):
            r = g.rows
            if g.kind == ZERO:
                continue
            ds[r] = ds_family(g.kind, self.s[r], self.z[r], sc, dsa[r], dza[r], sigma * mu,
                              k=g.k, fam=_fam(g) if g.kind in (EXP, POW) else None)
        return ds

    def H_apply(self, scal, v):
        out = np.zeros_like(v)
        for g, sc in zip(self.groups, scal):
            out[g.rows] = sc["Hb"].apply(v[g.rows])
        return out

    def step_length(self, d, combined):
        """Step rule: symmetric boundary steps, then x0.8 backtracking on exp/pow cones."""
        st = self.st
        a = 1.0
        if d["tau"] < 0:
            a = min(a, -self.tau / d["tau"])
        if d["kappa"] < 0:
            a = min(a, -self.kappa / d["kappa"])
        for g in self.groups:
            r = g.rows
            if g.kind == NONNEG:
                a = min(a, float(np.min(C.nn_step(self.s[r], d["s"][r]))),
                        float(np.min(C.nn_step(self.z[r], d["z"][r]))))
            elif g.kind == SOC:
                a = min(a, float(np.min(C.soc_step(self.s[r], d["s"][r]))),
                        float(np.min(C.soc_step(self.z[r], d["z"][r]))))
            elif g.kind == PSD:
                a = min(a, float(np.min(C.psd_step(self.s[r], d["s"][r], g.k))),
                        float(np.min(C.psd_step(self.z[r], d["z"][r], g.k))))
        if not self.has_nonsym:
            return a
        while True:
            if a < st.min_alpha:
                return 0.0
            ok = True
            for g in self.groups:
                if g.kind not in (EXP, POW):
                    continue
                fam = _fam(g)
                r = g.rows
                sa = self.s[r] + a * d["s"][r]
                za = self.z[r] + a * d["z"][r]
                if not (fam.primal_interior(sa).all() and fam.dual_interior(za).all()):
                    ok = False
                    break
            if ok and combined:
                mua = self.mu(self.s + a * d["s"], self.z + a * d["z"],
                              self.tau + a * d["tau"], self.kappa + a * d["kappa"])
                for g in self.groups:
                    if g.kind not in (EXP, POW):
                        continue
                    fam = _fam(g)
                    r = g.rows
                    sa = self.s[r] + a * d["s"][r]
                    za = self.z[r] + a * d["z"][r]
                    gz, _ = fam.grad_hess(za)
                    st_ = -gz
                    zt_, okz = fam.conj_grad_point(sa, with_status=True)
                    with np.errstate(all="ignore"):
                        inside = okz & (3.0 / np.sum(st_ * zt_, axis=1) >= st.beta * mua)
                    if not np.all(inside):
                        ok = False
                        break
            if ok:
                return a
            a *= st.backtrack

    # -- directions ------------------------------------------------------------------
    def G(self):
        Px = self.Ps @ self.x
        gx = -(Px + self.As.T @ self.z + self.qs * self.tau)
        gz = self.s + self.As @ self.x - self.bs * self.tau
        gt = self.kappa + self.qs @ self.x + self.bs @ self.z + (self.x @ Px) / self.tau
        return gx, gz, gt

    def direction(self, kkt, scal, dx_, dz_, dt_, ds_, dk_, c2):
        """Solve eq. linsys_2x2 for the RHS d and recover Delta (eq. step-direction)."""
        x1, z1 = self._solve(kkt, dx_, -(dz_ - ds_))
        x2, z2 = c2
        xi = self.x / self.tau
        Pxi = self.Ps @ xi
        w = 2.0 * Pxi + self.qs
        num = dt_ - dk_ / self.tau + w @ x1 + self.bs @ z1
        den = self.kappa / self.tau + xi @ Pxi - w @ x2 - self.bs @ z2
        dtau = num / den
        dx = x1 + dtau * x2
        dz = z1 + dtau * z2
        ds = -ds_ - self.H_apply(scal, dz)
        dk = -(dk_ + self.kappa * dtau) / self.tau
        return {"x": dx, "z": dz, "s": ds, "tau": dtau, "kappa": dk}

    def iterate(self):
        """One pass of the loop body; returns a status (0 = continue)."""
        st = self.st
        mu = self.mu()
        force_dual = False
        for attempt in range(2):
            scal = self.scale(mu, force_dual)
            kkt = self._kkt([(g.rows, sc["Hb"]) for g, sc in zip(self.groups, scal)])
            c2 = self._solve(kkt, -self.qs, self.bs)
            gx, gz, gt = self.G()
            # affine (predictor)
            da = self.direction(kkt, scal, gx, gz, gt, self.s.copy(), self.kappa * self.tau, c2)
            alpha_a = self.step_length(da, combined=False)
            sigma = (1.0 - alpha_a) ** 3
            # combined (predictor + corrector)
            dk = self.kappa * self.tau + da["kappa"] * da["tau"] - sigma * mu
            ds = self.ds_combined(scal, da["s"], da["z"], sigma, mu)
            f = 1.0 - sigma
            dc = self.direction(kkt, scal, f * gx, f * gz, f * gt, ds, dk, c2)
            alpha_c = self.step_length(dc, combined=True)
            pd_used = any(g.kind in (EXP, POW) and np.any(sc["branch"] == 0)
                          for g, sc in zip(self.groups, scal))
            if alpha_c < st.dual_retry_alpha and pd_used and not force_dual:
                force_dual = True
                self.dual_switches += 1
                continue
            break
        self.last = dict(mu=mu, sigma=sigma, alpha_a=alpha_a, alpha_c=alpha_c)
        if alpha_c < st.insufficient_alpha:
            return INSUFFICIENT_PROGRESS
        a = st.step_fraction * alpha_c
        self.x = self.x + a * dc["x"]
        self.s = self.s + a * dc["s"]
        self.z = self.z + a * dc["z"]
        self.tau = self.tau + a * dc["tau"]
        self.kappa = self.kappa + a * dc["kappa"]
        return 0

    def solve(self):
        st = self.st
        self.status = 0
        for k in range(st.max_iter + 1):
            r = self.residuals()
            status = self.check(r)
            self.history.append(dict(k=k, gp=r["gp"], gd=r["gd"], nrp=r["nrp"], nrd=r["nrd"],
                                     mu=self.mu(), tau=self.tau, kappa=self.kappa))
            if st.verbose:
                h = self.history[-1]
                print(f"{k:3d} gp={h['gp']:+.8e} gd={h['gd']:+.8e} rp={h['nrp']:.2e} rd={h['nrd']:.2e} mu={h['mu']:.2e}")
            if status:
                self.status = status
                break
            if k == st.max_iter:
                self.status = MAX_ITER
                break
            try:
                status = self.iterate()
            except np.linalg.LinAlgError:
                self.status = NUMERICAL_ERROR
                break
            self.iterations += 1
            if status:
                self.status = status
                break
        self.result = self.residuals()
        return self.status

    # -- results in user coordinates --------------------------------------------------
    @property
    def objective(self):
        return float(self.result["gp"])

    def solution(self):
        r = self.result
        return r["xb"], r["sb"], r["zb"]


def solve(prob, **kw):
    s = Solver(prob, Settings(**kw))
    s.solve()
    return s


def ds_family(kind, s, z, sc, dsa, dza, sm, k=0, fam=None):
    """d_s of the combined step (eq. ds-correction-step) for the cones of one family.

    s, z, dsa, dza: (N, d) rows of the N cones; sc: that family's scaling state
    (Solver.scale); sm = sigma * mu.
      nonneg/SOC/PSD: d_s = W'(lambda \\ (lambda o lambda + eta - sm e)) with the
        Mehrotra term eta = (W^-T ds_a) o (W dz_a);
      exp/pow: d_s = s + sm grad f(z) - 1/2 grad^3 f(z)[dz_a, grad^2 f(z)^-1 ds_a].
    """
    a, b_ = dsa, dza
    if kind == NONNEG:
        lam = sc["lam"]
        w = sc["w"]
        eta = (a / w) * (w * b_)
        v = lam * lam + eta - sm
        return w * (v / lam)
    if kind == SOC:
        W, Winv, lam = sc["W"], sc["Winv"], sc["lam"]
        Wi_ds = np.einsum("cji,cj->ci", Winv, a)       # W^-T ds
        W_dz = np.einsum("cij,cj->ci", W, b_)
        eta = C.soc_circ(Wi_ds, W_dz)
        e = np.zeros_like(lam)
        e[:, 0] = 1.0
        v = C.soc_circ(lam, lam) + eta - sm * e
        return np.einsum("cji,cj->ci", W, C.soc_inv_circ(lam, v))   # W' (lam \\ v)
    if kind == PSD:
        R, Rinv, lam = sc["R"], sc["Rinv"], sc["lam"]
        dS = C.smat(a, k)
        dZ = C.smat(b_, k)
        Aa = np.einsum("cij,cjk,clk->cil", Rinv, dS, Rinv)    # R^-1 dS R^-T
        Bb = np.einsum("cji,cjk,ckl->cil", R, dZ, R)          # R' dZ R
        eta = C.psd_circ(Aa, Bb)
        V = eta.copy()
        V += np.einsum("ci,ij->cij", lam * lam, np.eye(k))
        V -= sm * np.eye(k)[None]
        X = 2.0 * V / (lam[:, :, None] + lam[:, None, :])
        return C.svec(np.einsum("cij,cjk,clk->cil", R, X, R))   # R X R'
    g_ = sc["grad"]
    u = fam.hinv_apply(sc["hinv"], a)                       # Hf^-1 ds_a
    eta = -0.5 * fam.third(z, b_, u)
    return s + sm * g_ + eta
