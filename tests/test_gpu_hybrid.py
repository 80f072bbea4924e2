"""Operators one at a time on the GPU, in the solver's face-major layout and
in the paper's hybrid layout (Section 3.1), against the oracle: Gauss
gradient, divergence, Laplacian assembly, A x, and (hybrid) A^T x of a
non-symmetric matrix.  Meshes span several 256-cell tiles; the slot counts
include rows longer than K (CRS part) and K = 1 (diagonals in the CRS
part)."""
import sys

import numpy as np
import pytest

from oracle import hybrid as oh
from oracle import oracle as orc
from paper_1207_1571_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [((10, 9, 8), None, 7, 0.0), ((10, 9, 8), 3, 4, 0.0), ((12, 11, 1), 5, 3, 0.0), ((8, 7, 6), 2, 1, 0.15),
         ((20, 20, 20), None, 7, 0.0)]


def _bkinds(case):
    m = case.mesh
    kinds = np.concatenate([np.full(z, case.bcs[i].p_kind) for i, z in enumerate(m.patch_size)]).astype(np.int32)
    vals = np.concatenate([np.full(z, case.bcs[i].p_value) for i, z in enumerate(m.patch_size)])
    return kinds, vals


@pytest.mark.parametrize("shape,perm,K,jitter", CASES)
def test_operators_against_oracle(shape, perm, K, jitter):
    import torch
    from paper_1207_1571_amd import fvm
    case = wl.cavity(shape, Re=100.0, dt=0.01, perm_seed=perm, jitter=jitter, jitter_seed=4).with_(hybrid_K=K)
    m = case.mesh
    N, F, Fi = m.V.shape[0], m.owner.shape[0], m.neighbour.shape[0]
    _say(f"hybrid ops: shape {shape} perm {perm} K {K} jitter {jitter}: N {N}")
    c = fvm.Case(case)
    rng = np.random.default_rng(17)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
    bk, bv = _bkinds(case)

    # gradient
    x = rng.normal(size=N)
    g_o = orc.grad(m, x, bk, bv)
    for op in (fvm.OP_GRAD, fvm.OP_HY_GRAD):
        out = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        fvm.operator(c, op, dev(x), out)
        g = out.cpu().numpy().reshape(3, N).T
        assert _rel(g, g_o) <= TOL, (op, _rel(g, g_o))

    # divergence (the oracle's pressure right-hand side of a flux is -div)
    flux = rng.normal(size=F)
    _, _, b = orc.pressure_system(m, np.zeros(F), bk, bv, phiH=flux)
    for op in (fvm.OP_DIV, fvm.OP_HY_DIV):
        out = torch.empty(N, dtype=torch.float64, device="cuda")
        fvm.operator(c, op, dev(flux), out)
        assert _rel(out.cpu().numpy(), -b) <= TOL, (op, _rel(out.cpu().numpy(), -b))

    # Laplacian (solve_pressure's matrix) and A x in both layouts
    gamma = rng.uniform(0.5, 2.0, F)
    diag, offd, _ = orc.pressure_system(m, gamma, bk, bv, pin_cell=case.p_ref_cell, p_ref=case.p_ref_value)
    x = rng.normal(size=N)
    y_o = orc.amul(m.owner[:Fi].copy(), m.neighbour.copy(), diag, offd, offd, x)
    out = torch.empty(N, dtype=torch.float64, device="cuda")
    fvm.operator(c, fvm.OP_LAP, dev(gamma), out)
    assert _rel(out.cpu().numpy(), diag) <= TOL
    fvm.operator(c, fvm.OP_SPMV, dev(x), out)
    assert _rel(out.cpu().numpy(), y_o) <= TOL
    h = oh.hybrid_structure(N, m.owner[:Fi], m.neighbour, K)
    nC = len(h["c_col"])
    V = torch.empty(K * N + nC, dtype=torch.float64, device="cuda")
    fvm.operator(c, fvm.OP_HY_LAP, dev(gamma), V)
    V = V.cpu().numpy()
    face_of = {}
    for f in range(Fi):
        face_of[(int(m.owner[f]), int(m.neighbour[f]))] = f
        face_of[(int(m.neighbour[f]), int(m.owner[f]))] = f

    def entry(i, j):
        return diag[i] if i == j else offd[face_of[(i, j)]]
    # expected values: row i in ascending column order, the first K entries
    # in slots 0..K-1 (slot-major), the rest in the CRS part; unused slots 0
    rows = [[i] for i in range(N)]
    for f in range(Fi):
        rows[m.owner[f]].append(int(m.neighbour[f]))
        rows[m.neighbour[f]].append(int(m.owner[f]))
    Ve = np.zeros(K * N + nC)
    for i in range(N):
        for t, j in enumerate(sorted(rows[i])):
            if t < K:
                Ve[t * N + i] = entry(i, j)
            else:
                Ve[K * N + h["c_start"][i] + t - K] = entry(i, j)
    assert _rel(V, Ve) <= TOL, _rel(V, Ve)
    fvm.operator(c, fvm.OP_HY_SPMV, dev(x), out)
    assert _rel(out.cpu().numpy(), y_o) <= TOL

    # a non-symmetric matrix through SETMAT: A x and A^T x
    dg, up, lo = rng.uniform(4.0, 6.0, N), rng.normal(size=Fi), rng.normal(size=Fi)
    fvm.operator(c, fvm.OP_HY_SETMAT, dev(np.concatenate([dg, up, lo])))
    for op, tr in ((fvm.OP_HY_SPMV, False), (fvm.OP_HY_STMVP, True)):
        fvm.operator(c, op, dev(x), out)
        y = orc.amul(m.owner[:Fi].copy(), m.neighbour.copy(), dg, up, lo, x, transpose=tr)
        assert _rel(out.cpu().numpy(), y) <= TOL, (op, _rel(out.cpu().numpy(), y))
    c.close()
