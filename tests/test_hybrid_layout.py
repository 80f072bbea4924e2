"""The paper's hybrid matrix layout (Section 3.1), host side.

The oracle's construction (oracle/hybrid.py) is pinned by the worked example
the paper prints and by the defining property of J (the transposed entry of
(i, k) is found at row I[i][k], slot J[i][k], and points back); the library's
own construction (fvm_mesh_hybrid) must equal it exactly on every mesh and
slot count, including rows longer than K (the CRS part) and K = 1 (diagonal
entries in the CRS part).
"""
import os

import numpy as np
import pytest

from oracle import hybrid as oh
from paper_1207_1571_amd import fvm
from paper_1207_1571_amd import meshgen as mg
from paper_1207_1571_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hybrid_worked_example.txt")


def _golden():
    K, I, J = None, {}, {}
    for line in open(GOLDEN):
        t = line.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "K":
            K = int(t[1])
        else:
            (I if t[0] == "I" else J)[int(t[1])] = [int(v) for v in t[2:]]
    n = len(I)
    return K, np.array([I[i] for i in range(n)]), np.array([J[i] for i in range(n)])


def test_worked_example():
    K, I, J = _golden()
    # the matrix's off-diagonal pattern as faces (lower index first)
    faces = sorted({(min(i, j), max(i, j)) for i in range(len(I)) for j in I[i] if j != i})
    own = np.array([f[0] for f in faces], np.int32)
    nei = np.array([f[1] for f in faces], np.int32)
    h = oh.hybrid_structure(len(I), own, nei, K)
    assert np.array_equal(h["I"], I)
    assert np.array_equal(h["J"], J)
    assert h["J"][1, 2] == 0            # the entry the paper's figure evaluates
    assert len(h["c_col"]) == 0         # every row fits: C is empty


def _meshes():
    yield "lex", wl.cavity((5, 4, 3), Re=10.0, dt=0.01).mesh
    yield "perm", wl.cavity((6, 5, 4), Re=10.0, dt=0.01, perm_seed=3).mesh
    yield "2d", wl.cavity((7, 6, 1), Re=10.0, dt=0.01, perm_seed=5).mesh
    yield "jitter", wl.cavity((4, 4, 4), Re=10.0, dt=0.01, jitter=0.2, jitter_seed=2, perm_seed=7).mesh


def _check_invariants(h, N, rows, K):
    I, J, cs, cc, ct_ = h["I"], h["J"], h["c_start"], h["c_col"], h["c_tr"]
    for i in range(N):
        full = list(I[i, :min(K, len(rows[i]))]) + list(cc[cs[i]:cs[i + 1]])
        assert full == rows[i]                                    # every entry once, ascending
        for k in range(K):
            j = I[i, k]
            if k >= len(rows[i]):
                assert j == i and J[i, k] == k                    # unused slot
                continue
            if J[i, k] >= 0:
                assert I[j, J[i, k]] == i and J[j, J[i, k]] == k  # transpose points back
            else:
                c = -1 - J[i, k]
                assert cc[c] == i and ct_[c] == K * i + k and cs[j] <= c < cs[j + 1]
        for c in range(cs[i], cs[i + 1]):
            j, t = cc[c], ct_[c]
            if t >= 0:
                assert I[t // K, t % K] == i and t // K == j and J[j, t % K] == -1 - c
            else:
                assert cc[-1 - t] == i and ct_[-1 - t] == -1 - c and cs[j] <= -1 - t < cs[j + 1]


@pytest.mark.parametrize("K", [7, 4, 3, 1])
def test_oracle_invariants(K):
    for name, m in _meshes():
        N, Fi = m.V.shape[0], len(m.neighbour)
        rows = [[i] for i in range(N)]
        for a, b in zip(m.owner[:Fi], m.neighbour):
            rows[a].append(int(b)); rows[b].append(int(a))
        rows = [sorted(r) for r in rows]
        h = oh.hybrid_structure(N, m.owner[:Fi], m.neighbour, K)
        _check_invariants(h, N, rows, K)
        Iq, Jq = oh.decode_q(h["Q"], K)
        ok = h["J"] >= 0
        assert np.array_equal(Iq[ok], h["I"][ok]) and np.array_equal(Jq[ok], h["J"][ok])
        assert np.all(h["Q"][~ok] == -1)


lib_required = pytest.mark.skipif(not os.path.exists(fvm.LIB_PATH), reason="libfvm.so not built")


@lib_required
@pytest.mark.parametrize("K", [7, 4, 3, 1])
def test_library_equals_oracle(K):
    for name, m in _meshes():
        case_bcs = [wl.PatchBC(wl.FIXED, wl.FIXED) for _ in m.patch_names]
        lm = fvm.Mesh(m, case_bcs)
        Fi = len(m.neighbour)
        o = oh.hybrid_structure(m.V.shape[0], m.owner[:Fi], m.neighbour, K)
        h = fvm.mesh_hybrid(lm, K)
        for key in ("I", "J", "Q", "c_start", "c_col", "c_tr"):
            assert np.array_equal(h[key], o[key]), (name, K, key)


@lib_required
def test_library_many_neighbours():
    """Rows longer than K on a line mesh with long-range faces."""
    n, reach = 40, 5
    own, nei = [], []
    for i in range(n):
        for k in range(1, reach + 1):
            if i + k < n:
                own.append(i); nei.append(i + k)
    Fi = len(own)
    S = np.array([(1.0 if (b - a) == 1 else 0.1, 0.0, 0.0) for a, b in zip(own, nei)] + [(-1.0, 0, 0), (1.0, 0, 0)])
    Cf = np.array([((a + b + 1) / 2.0, 0.5, 0.5) for a, b in zip(own, nei)] + [(0.0, 0.5, 0.5), (float(n), 0.5, 0.5)])
    m = mg.Mesh(owner=np.array(own + [0, n - 1], np.int32), neighbour=np.array(nei, np.int32), Sf=S, Cf=Cf,
                C=np.array([(i + 0.5, 0.5, 0.5) for i in range(n)]), V=np.ones(n), patch_names=["ends"],
                patch_start=np.array([Fi], np.int32), patch_size=np.array([2], np.int32), shape=(n, 1, 1),
                lex_of_cell=np.arange(n))
    lm = fvm.Mesh(m, [wl.PatchBC(wl.FIXED, wl.FIXED)])
    for K in (11, 6, 3):
        o = oh.hybrid_structure(n, m.owner[:Fi], m.neighbour, K)
        h = fvm.mesh_hybrid(lm, K)
        assert (len(o["c_col"]) > 0) == (K < 2 * reach + 1)
        for key in ("I", "J", "Q", "c_start", "c_col", "c_tr"):
            assert np.array_equal(h[key], o[key]), (K, key)


@lib_required
def test_library_rejects_bad_K():
    m = wl.cavity((3, 3, 3), Re=1.0, dt=1.0)
    lm = fvm.Mesh(m.mesh, m.bcs)
    with pytest.raises(fvm.FvmError):
        fvm.mesh_hybrid(lm, 0)
    c = m.with_(hybrid_K=-1)
    with pytest.raises(fvm.FvmError):
        fvm.workspace_bytes(lm, fvm.opts_from_case(c))
