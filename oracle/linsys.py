"""KKT solves of the oracle: quasi-definite LDL' by block elimination, and
iterative refinement.

TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Nothing in the product
path may import this package.

The reduced system (eq. linsys_2x2) is K [dx; dz] = rhs with
K = [[P, A'], [A, -H]], H block diagonal over the cones.  A regularisation
delta = delta_s + delta_d max_i |K_ii| makes K quasi-definite (Sec. 3.7
"Solving linear systems"): +delta on the P block and -delta on the -H block
(reading: adding +delta to the -H block as printed breaks quasi-definiteness).

Factorisation: the LDL' of K_reg with the cone rows ordered first.  Their
pivots are the blocks -(H_c + delta I) with inverses M_c; what remains is the positive definite Schur complement
S = P + delta I + A' M A over x, factored by a library Cholesky (dense S) or
sparse LU (large sparse S).  Symmetric-cone blocks are carried in spectral
form H_c = V diag(lam) V' and H_c v, M_c v are applied in that form:
near the cone boundary cond(H_c) exceeds 1/eps and an explicit M_c (entries
~1/delta) applied to a vector loses the component along H_c's largest
eigenvector, which H_c then amplifies into an O(1) residual.  Explicit
M_c entries are only used to assemble S, where that component is
negligible.

Iterative refinement (Sec. 3.7, the three-step loop): residual with the
*unregularised* K, correction with the regularised factor, stop when
||r||_inf <= t_abs + t_rel ||rhs||_inf, after T_max corrections, or when a
correction fails to halve the residual (the best iterate is kept).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class SpectralBlocks:
    """Per-cone H_c = V diag(lam) V' (V orthogonal), N cones of size d."""

    def __init__(self, lam, V):
        self.lam = lam
        self.V = V

    def apply(self, v):
        return np.einsum("cij,cj->ci", self.V, self.lam * np.einsum("cji,cj->ci", self.V, v))

    def inv_reg(self, delta):
        return np.einsum("cij,cj,ckj->cik", self.V, 1.0 / (self.lam + delta), self.V)

    def inv_reg_apply(self, v, delta):
        return np.einsum("cij,cj->ci", self.V, np.einsum("cji,cj->ci", self.V, v) / (self.lam + delta))

    def diag(self):
        return np.einsum("cij,cj,cij->ci", self.V, self.lam, self.V)

    def dense(self):
        return np.einsum("cij,cj,ckj->cik", self.V, self.lam, self.V)


class DenseBlocks:
    """Per-cone explicit H_c (N, d, d)."""

    def __init__(self, H):
        self.H = H

    def apply(self, v):
        return np.einsum("cij,cj->ci", self.H, v)

    def inv_reg(self, delta):
        d = self.H.shape[1]
        return np.linalg.inv(self.H + delta * np.eye(d)[None])

    def inv_reg_apply(self, v, delta):
        d = self.H.shape[1]
        return np.linalg.solve(self.H + delta * np.eye(d)[None], v[..., None])[..., 0]

    def diag(self):
        return np.diagonal(self.H, axis1=1, axis2=2)

    def dense(self):
        return self.H


class KKT:
    """The regularised reduced KKT system for one IPM iteration.

    P_full: full symmetric P (scipy sparse, n x n); A: (m x n) CSR;
    blocks: list of (rows (N, d) int array, SpectralBlocks | DenseBlocks)
    covering every constraint row (zero rows carry H = 0).
    """

    def __init__(self, P_full, A, blocks, delta_s, delta_d, dense_S_limit=30000, dense_row_nnz=512):
        self.P = sp.csr_matrix(P_full)
        self.A = sp.csr_matrix(A)
        self.n = A.shape[1]
        self.m = A.shape[0]
        self.blocks = blocks
        hdiag = np.zeros(self.m)
        for rows, Hb in blocks:
            hdiag[rows] = Hb.diag()
        maxdiag = max(np.max(np.abs(self.P.diagonal())) if self.n else 0.0,
                      np.max(np.abs(hdiag)) if self.m else 0.0)
        self.delta = delta_s + delta_d * maxdiag
        self._factor(dense_S_limit, dense_row_nnz)

    # -- unregularised operator -------------------------------------------
    def H_apply(self, v):
        out = np.zeros_like(v)
        for rows, Hb in self.blocks:
            out[rows] = Hb.apply(v[rows])
        return out

    def M_apply(self, v):
        """(H + delta I)^-1 v, block by block in each block's own form."""
        out = np.zeros_like(v)
        for rows, Hb in self.blocks:
            out[rows] = Hb.inv_reg_apply(v[rows], self.delta)
        return out

    def matvec(self, x, z):
        """K [x; z] with the unregularised K."""
        return self.P @ x + self.A.T @ z, self.A @ x - self.H_apply(z)

    # -- factorisation -------------------------------------------------------
    def _factor(self, dense_S_limit, dense_row_nnz):
        n, m = self.n, self.m
        rr, cc, vv = [], [], []
        mdiag = np.zeros(m)
        diag_rows = np.zeros(m, dtype=bool)
        for rows, Hb in self.blocks:
            d = rows.shape[1]
            M = Hb.inv_reg(self.delta)
            rr.append(np.repeat(rows, d, axis=1).ravel())
            cc.append(np.tile(rows, (1, d)).ravel())
            vv.append(M.ravel())
            if d == 1:
                mdiag[rows[:, 0]] = M[:, 0, 0]
                diag_rows[rows[:, 0]] = True
        self.Mbd = sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))), shape=(m, m))
        # rows with many nonzeros in diagonal-M blocks are multiplied out densely
        rownnz = np.diff(self.A.indptr)
        dense_rows = np.nonzero(diag_rows & (rownnz > dense_row_nnz))[0]
        keep = np.ones(m)
        keep[dense_rows] = 0.0
        Asp = sp.diags(keep) @ self.A
        S = self.P + self.delta * sp.identity(n) + Asp.T @ self.Mbd @ Asp
        if n <= dense_S_limit:
            S = S.toarray()
            if dense_rows.size:
                AD = self.A[dense_rows].toarray()
                S += AD.T @ (mdiag[dense_rows][:, None] * AD)
            self.S_chol = sla.cho_factor(S, lower=True, overwrite_a=True, check_finite=False)
            self.S_lu = None
        else:
            if dense_rows.size:
                AD = self.A[dense_rows]
                S = S + AD.T @ sp.diags(mdiag[dense_rows]) @ AD
            self.S_lu = spla.splu(sp.csc_matrix(S), permc_spec="MMD_AT_PLUS_A")
            self.S_chol = None

    def solve_reg(self, r1, r2):
        """Solve K_reg [x; z] = [r1; r2]:
        (P + d) x + A'z = r1, A x - (H + d) z = r2  =>  z = M (A x - r2),  S x = r1 + A' M r2."""
        rhs = r1 + self.A.T @ self.M_apply(r2)
        if self.S_chol is not None:
            x = sla.cho_solve(self.S_chol, rhs, check_finite=False)
        else:
            x = self.S_lu.solve(rhs)
        z = self.M_apply(self.A @ x - r2)
        return x, z

    def solve(self, r1, r2, abstol=1e-12, reltol=1e-12, max_ref=10):
        """Iterative refinement against the unregularised K.  Returns (x, z, info)."""
        nb = max(np.max(np.abs(r1)) if r1.size else 0.0, np.max(np.abs(r2)) if r2.size else 0.0)
        x = np.zeros(self.n)
        z = np.zeros(self.m)
        best = (x, z, nb)
        rx, rz = r1.copy(), r2.copy()
        rnorm = nb
        steps = 0
        for it in range(max_ref + 1):
            dx, dz = self.solve_reg(rx, rz)
            xn, zn = x + dx, z + dz
            kx, kz = self.matvec(xn, zn)
            rxn, rzn = r1 - kx, r2 - kz
            rn = max(np.max(np.abs(rxn)) if rxn.size else 0.0, np.max(np.abs(rzn)) if rzn.size else 0.0)
            steps += 1
            if rn < best[2]:
                best = (xn, zn, rn)
            if rn <= abstol + reltol * nb:
                break
            if it > 0 and rn > 0.5 * rnorm:
                break
            x, z, rx, rz, rnorm = xn, zn, rxn, rzn, rn
        return best[0], best[1], {"solves": steps, "resid": best[2]}
