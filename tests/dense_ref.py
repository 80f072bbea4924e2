"""A second, dense, matrix-style statement of one PISO step / SIMPLE
iteration for tiny meshes (a few dozen cells), used to pin the oracle.

Everything is assembled as dense N x N numpy matrices and solved with
numpy.linalg.solve, so a Krylov solver, a face-addressed product or a
scatter in the oracle that drops a term, flips a sign or swaps an index
shows up as a mismatch.  The discretisation is the one the oracle
implements (Section 3 of the paper, following Jasak/OpenFOAM): linear
interpolation, Gauss gradient, over-relaxed non-orthogonal split, implicit
Euler, Rhie-Chow-free compact pressure Laplacian.
"""
import numpy as np

FIXED, ZERO_GRAD, EMPTY = 0, 1, 2


class DenseMesh:
    def __init__(self, mesh, bcs):
        self.N = mesh.n_cells
        self.F = mesh.n_faces
        self.Fi = mesh.n_internal
        self.own = mesh.owner.astype(int)
        self.nei = mesh.neighbour.astype(int)
        self.S = mesh.Sf
        self.V = mesh.V
        Fi = self.Fi
        C, Cf, S = mesh.C, mesh.Cf, mesh.Sf
        d = C[self.nei] - C[self.own[:Fi]]
        Sd = np.einsum("ij,ij->i", S[:Fi], d)
        self.w = np.einsum("ij,ij->i", S[:Fi], C[self.nei] - Cf[:Fi]) / Sd
        self.dl = np.zeros(self.F)
        self.dl[:Fi] = np.einsum("ij,ij->i", S[:Fi], S[:Fi]) / Sd
        self.k = S[:Fi] - self.dl[:Fi, None] * d
        db = Cf[Fi:] - C[self.own[Fi:]]
        self.dl[Fi:] = np.einsum("ij,ij->i", S[Fi:], S[Fi:]) / np.einsum("ij,ij->i", S[Fi:], db)
        self.uk = np.zeros(self.F - Fi, int); self.pk = np.zeros(self.F - Fi, int)
        self.uv = np.zeros((self.F - Fi, 3)); self.pv = np.zeros(self.F - Fi)
        for p, (s, z) in enumerate(zip(mesh.patch_start, mesh.patch_size)):
            sl = slice(s - Fi, s - Fi + z)
            self.uk[sl] = bcs[p].u_kind; self.pk[sl] = bcs[p].p_kind
            self.uv[sl] = bcs[p].u_value; self.pv[sl] = bcs[p].p_value

    # Gauss gradient of a scalar with boundary kinds/values
    def grad(self, phi, bk, bv):
        g = np.zeros((self.N, 3))
        for f in range(self.Fi):
            P, Q = self.own[f], self.nei[f]
            pf = self.w[f] * phi[P] + (1 - self.w[f]) * phi[Q]
            g[P] += self.S[f] * pf
            g[Q] -= self.S[f] * pf
        for b in range(self.F - self.Fi):
            f = self.Fi + b; P = self.own[f]
            if bk[b] == EMPTY:
                continue
            g[P] += self.S[f] * (bv[b] if bk[b] == FIXED else phi[P])
        return g / self.V[:, None]

    def momentum(self, nu, dt, phi, U_old, U_now):
        N = self.N
        A = np.zeros((N, N)); b = np.zeros((N, 3))
        if dt > 0:
            A[np.arange(N), np.arange(N)] += self.V / dt
            b += self.V[:, None] * U_old / dt
        for f in range(self.Fi):
            P, Q, Fl, w, D = self.own[f], self.nei[f], phi[f], self.w[f], nu * self.dl[f]
            A[P, P] += Fl * w + D; A[P, Q] += Fl * (1 - w) - D
            A[Q, Q] += -Fl * (1 - w) + D; A[Q, P] += -Fl * w - D
        for bb in range(self.F - self.Fi):
            f = self.Fi + bb; P = self.own[f]; Fl = phi[f]
            if self.uk[bb] == FIXED:
                A[P, P] += nu * self.dl[f]
                b[P] += (nu * self.dl[f] - Fl) * self.uv[bb]
            elif self.uk[bb] == ZERO_GRAD:
                A[P, P] += Fl
        gU = [self.grad(U_now[:, c], self.uk, self.uv[:, c]) for c in range(3)]
        for f in range(self.Fi):
            P, Q, w = self.own[f], self.nei[f], self.w[f]
            for c in range(3):
                s = nu * self.k[f] @ (w * gU[c][P] + (1 - w) * gU[c][Q])
                b[P, c] += s; b[Q, c] -= s
        return A, b

    def pressure(self, rAU, phiH, gradp, pin, p_ref):
        N = self.N
        gam = np.zeros(self.F)
        gam[: self.Fi] = self.w * rAU[self.own[: self.Fi]] + (1 - self.w) * rAU[self.nei]
        gam[self.Fi:] = rAU[self.own[self.Fi:]]
        A = np.zeros((N, N)); b = np.zeros(N)
        for f in range(self.Fi):
            P, Q = self.own[f], self.nei[f]
            g = gam[f] * self.dl[f]
            A[P, P] += g; A[Q, Q] += g; A[P, Q] -= g; A[Q, P] -= g
            b[P] -= phiH[f]; b[Q] += phiH[f]
            w = self.w[f]
            t = gam[f] * self.k[f] @ (w * gradp[P] + (1 - w) * gradp[Q])
            b[P] += t; b[Q] -= t
        for bb in range(self.F - self.Fi):
            f = self.Fi + bb; P = self.own[f]
            if self.pk[bb] == EMPTY:
                continue
            b[P] -= phiH[f]
            if self.pk[bb] == FIXED:
                g = gam[f] * self.dl[f]
                A[P, P] += g; b[P] += g * self.pv[bb]
        if not np.any(self.pk == FIXED):
            a = A[pin, pin]; A[pin, pin] = 2 * a; b[pin] += a * p_ref
        return A, b, gam

    def corrector(self, A, src, U, p, pin, p_ref):
        D = np.diag(A).copy()
        H = src - (A - np.diag(D)) @ U
        HbyA = H / D[:, None]; rAU = self.V / D
        phiH = np.zeros(self.F)
        for f in range(self.Fi):
            P, Q, w = self.own[f], self.nei[f], self.w[f]
            phiH[f] = self.S[f] @ (w * HbyA[P] + (1 - w) * HbyA[Q])
        for bb in range(self.F - self.Fi):
            f = self.Fi + bb; P = self.own[f]
            phiH[f] = (self.S[f] @ self.uv[bb] if self.uk[bb] == FIXED
                       else self.S[f] @ HbyA[P] if self.uk[bb] == ZERO_GRAD else 0.0)
        gp0 = self.grad(p, self.pk, self.pv)
        Ap, bp, gam = self.pressure(rAU, phiH, gp0, pin, p_ref)
        pn = np.linalg.solve(Ap, bp)
        phi = np.zeros(self.F)
        for f in range(self.Fi):
            P, Q, w = self.own[f], self.nei[f], self.w[f]
            phi[f] = (phiH[f] - gam[f] * self.dl[f] * (pn[Q] - pn[P])
                      - gam[f] * self.k[f] @ (w * gp0[P] + (1 - w) * gp0[Q]))
        for bb in range(self.F - self.Fi):
            f = self.Fi + bb; P = self.own[f]
            phi[f] = phiH[f] - (gam[f] * self.dl[f] * (self.pv[bb] - pn[P]) if self.pk[bb] == FIXED else 0.0)
        return HbyA, rAU, pn, phi


def piso_step(mesh, bcs, nu, dt, n_corr, pin, p_ref, U, p, phi):
    dm = DenseMesh(mesh, bcs)
    A, src = dm.momentum(nu, dt, phi, U, U)
    gp = dm.grad(p, dm.pk, dm.pv)
    U = np.linalg.solve(A, src - dm.V[:, None] * gp)
    for _ in range(n_corr):
        HbyA, rAU, p, phi = dm.corrector(A, src, U, p, pin, p_ref)
        U = HbyA - rAU[:, None] * dm.grad(p, dm.pk, dm.pv)
    return U, p, phi


def simple_iteration(mesh, bcs, nu, alpha_u, alpha_p, pin, p_ref, U, p, phi):
    dm = DenseMesh(mesh, bcs)
    A, src = dm.momentum(nu, 0.0, phi, None, U)
    D0 = np.diag(A).copy()
    A[np.arange(dm.N), np.arange(dm.N)] = D0 / alpha_u
    src = src + ((1 - alpha_u) / alpha_u * D0)[:, None] * U
    gp = dm.grad(p, dm.pk, dm.pv)
    Un = np.linalg.solve(A, src - dm.V[:, None] * gp)
    HbyA, rAU, pn, phi = dm.corrector(A, src, Un, p, pin, p_ref)
    p_rel = p + alpha_p * (pn - p)
    Un = HbyA - rAU[:, None] * dm.grad(p_rel, dm.pk, dm.pv)
    return Un, p_rel, phi
