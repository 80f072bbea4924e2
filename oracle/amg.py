"""Oracle of the aggregation AMG preconditioner for the pressure CG.

TEST INFRASTRUCTURE ONLY: used by the tests and never by the product path.
Plain numpy, written from the textbook definitions (unsmoothed aggregation
AMG used as a CG preconditioner: piecewise-constant prolongation P, Galerkin
coarse operators P^T A P, a symmetric V-cycle with damped-Jacobi smoothing
and an exact solve on the coarsest level).  The paper names stronger
pressure preconditioners as future work (Section 5); the choices below are
this implementation's:

* aggregation, in cell index order: a cell none of whose neighbours is
  aggregated yet starts an aggregate with all of them (phase 1); every cell
  left over joins the aggregate of its lowest-index neighbour aggregated in
  phase 1 (phase 2; a cell without neighbours is its own aggregate);
* coarse faces: the distinct aggregate pairs joined by a fine face, in
  ascending (lower, upper) order;
* levels are added while a level has more than `coarse_max` cells and the
  aggregation shrinks it by at least 10%;
* V-cycle on level l for right-hand side b, from x = 0:
      x = w D^-1 b;  r = b - A x;  x += P V_{l+1}(P^T r);  x += w D^-1 (b - A x)
  with w = 2/3, and x = A^-1 b on the coarsest level.  Pre- and
  post-smoothing are the same symmetric operator, so the cycle is a
  symmetric linear map (positive definite for w < 2 / lambda_max(D^-1 A)).
"""
from __future__ import annotations

import numpy as np

OMEGA = 2.0 / 3.0


def aggregate(n: int, own, nei):
    """Aggregate index of every cell and the number of aggregates."""
    adj = [[] for _ in range(n)]
    for a, b in zip(np.asarray(own).tolist(), np.asarray(nei).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    for r in adj:
        r.sort()
    agg = [-1] * n
    phase1 = [False] * n
    na = 0
    for i in range(n):
        if agg[i] != -1:
            continue
        if all(agg[j] == -1 for j in adj[i]):
            agg[i] = na
            phase1[i] = True
            for j in adj[i]:
                agg[j] = na
                phase1[j] = True
            na += 1
    for i in range(n):
        if agg[i] != -1:
            continue
        cand = [j for j in adj[i] if phase1[j]]
        if cand:
            agg[i] = agg[cand[0]]
        else:
            agg[i] = na
            na += 1
    return np.array(agg, np.int32), na


def coarse_faces(agg, own, nei):
    """Distinct aggregate pairs (lower, upper) joined by a fine face."""
    pairs = set()
    for a, b in zip(np.asarray(own).tolist(), np.asarray(nei).tolist()):
        A, B = int(agg[a]), int(agg[b])
        if A != B:
            pairs.add((min(A, B), max(A, B)))
    pairs = sorted(pairs)
    return (np.array([p[0] for p in pairs], np.int32), np.array([p[1] for p in pairs], np.int32))


def build_hierarchy(n: int, own, nei, coarse_max: int = 128, max_levels: int = 20):
    """Topology of the levels: per level (n, own, nei, agg to the next level)."""
    levels = [dict(n=int(n), own=np.asarray(own, np.int32), nei=np.asarray(nei, np.int32), agg=None)]
    while levels[-1]["n"] > coarse_max and len(levels) < max_levels:
        L = levels[-1]
        agg, na = aggregate(L["n"], L["own"], L["nei"])
        if na > 0.9 * L["n"]:
            break
        L["agg"] = agg
        co, cn = coarse_faces(agg, L["own"], L["nei"])
        levels.append(dict(n=na, own=co, nei=cn, agg=None))
    return levels


def galerkin(level, diag, offd, coarse):
    """P^T A P of a symmetric face-addressed matrix (diag, offd per face) for
    piecewise-constant P: coarse diagonal = sum of the member diagonals plus
    twice the faces inside the aggregate; coarse face = sum of its fine faces."""
    agg = level["agg"]
    nc = coarse["n"]
    dc = np.zeros(nc)
    np.add.at(dc, agg, diag)
    A = agg[level["own"]]
    B = agg[level["nei"]]
    inside = A == B
    np.add.at(dc, A[inside], 2.0 * offd[inside])
    index = {(int(a), int(b)): k for k, (a, b) in enumerate(zip(coarse["own"], coarse["nei"]))}
    oc = np.zeros(len(coarse["own"]))
    for f in np.nonzero(~inside)[0]:
        a, b = int(A[f]), int(B[f])
        oc[index[(min(a, b), max(a, b))]] += offd[f]
    return dc, oc


def amul(n, own, nei, diag, offd, x):
    y = diag * x
    np.add.at(y, own, offd * x[nei])
    np.add.at(y, nei, offd * x[own])
    return y


def dense(n, own, nei, diag, offd):
    A = np.diag(np.asarray(diag, np.float64)).copy()
    A[own, nei] = offd
    A[nei, own] = offd
    return A


class Amg:
    """The hierarchy with matrix values: levels[l] gains diag and offd."""

    def __init__(self, n, own, nei, diag, offd, coarse_max: int = 128):
        self.levels = build_hierarchy(n, own, nei, coarse_max)
        self.levels[0]["diag"] = np.asarray(diag, np.float64)
        self.levels[0]["offd"] = np.asarray(offd, np.float64)
        for l in range(len(self.levels) - 1):
            L, C = self.levels[l], self.levels[l + 1]
            C["diag"], C["offd"] = galerkin(L, L["diag"], L["offd"], C)
        c = self.levels[-1]
        self.coarse = dense(c["n"], c["own"], c["nei"], c["diag"], c["offd"])

    def vcycle(self, b, l: int = 0):
        L = self.levels[l]
        if l == len(self.levels) - 1:
            return np.linalg.solve(self.coarse, b)
        A = lambda x: amul(L["n"], L["own"], L["nei"], L["diag"], L["offd"], x)
        x = OMEGA * b / L["diag"]
        r = b - A(x)
        bc = np.zeros(self.levels[l + 1]["n"])
        np.add.at(bc, L["agg"], r)
        x = x + self.vcycle(bc, l + 1)[L["agg"]]
        x = x + OMEGA * (b - A(x)) / L["diag"]
        return x


def pcg(n, own, nei, diag, offd, b, x0, tol, max_iter=10000, coarse_max=128):
    """CG (Barrett et al., the template the solver follows) preconditioned
    by the V-cycle, with the solver's stopping test: normalised L1 residual
    sum|b - Ax| / n_f <= tol, n_f = sum(|Ax - xbar A1| + |b - xbar A1|) +
    1e-20, tested before the first iteration and after every update."""
    M = Amg(n, own, nei, diag, offd, coarse_max)
    A = lambda v: amul(n, own, nei, diag, offd, v)
    x = np.array(x0, np.float64)
    Ax = A(x)
    a1 = A(np.ones(n))
    xb = x.mean()
    nf = np.sum(np.abs(Ax - xb * a1) + np.abs(b - xb * a1)) + 1e-20
    r = b - Ax
    res = np.sum(np.abs(r)) / nf
    it = 0
    if res <= tol:
        return x, dict(iters=0, res=res)
    z = M.vcycle(r)
    rho = r @ z
    p = z.copy()
    while it < max_iter:
        q = A(p)
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        res = np.sum(np.abs(r)) / nf
        if res <= tol:
            break
        z = M.vcycle(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, dict(iters=it, res=res)
