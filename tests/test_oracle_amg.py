"""Pins of the AMG oracle (oracle/amg.py) against what the definitions fix:
the aggregation rule worked by hand on a chain, the Galerkin operator
against the dense product P^T A P, the V-cycle's symmetry and positivity,
exactness when the hierarchy has one level, and the preconditioned CG's
solution against a dense solve (with fewer iterations than Jacobi)."""
import numpy as np
import pytest

from oracle import amg
from oracle import oracle as orc
from paper_1207_1571_amd import workloads as wl


def test_aggregation_on_a_chain():
    # 0-1-2-3-4-5-6: cell 0 starts {0,1}; 2 has an aggregated neighbour;
    # 3 starts {2,3,4}; 5 has an aggregated neighbour; 6 starts {5,6}
    own = np.arange(6, dtype=np.int32)
    nei = own + 1
    agg, na = amg.aggregate(7, own, nei)
    assert na == 3 and agg.tolist() == [0, 0, 1, 1, 1, 2, 2]
    # a star: the centre takes everything
    agg, na = amg.aggregate(5, np.zeros(4, np.int32), np.arange(1, 5, dtype=np.int32))
    assert na == 1 and agg.tolist() == [0] * 5
    # phase 2 on the chain 0-1-2-3-4-5: {0,1} and {2,3,4} in phase 1; cell 5
    # is left over and joins the aggregate of its phase-1 neighbour 4
    own = np.array([0, 1, 2, 3, 4], np.int32)
    nei = np.array([1, 2, 3, 4, 5], np.int32)
    agg, na = amg.aggregate(6, own, nei)
    assert na == 2 and agg.tolist() == [0, 0, 1, 1, 1, 1]


def _pressure(case, rng):
    m = case.mesh
    F = m.owner.shape[0]
    gamma = rng.uniform(0.5, 2.0, F)
    pk = np.concatenate([np.full(z, case.bcs[i].p_kind) for i, z in enumerate(m.patch_size)]).astype(np.int32)
    diag, offd, _ = orc.pressure_system(m, gamma, pk, np.zeros(F - m.n_internal), pin_cell=case.p_ref_cell,
                                        p_ref=case.p_ref_value)
    return diag, offd


@pytest.mark.parametrize("shape,perm", [((9, 8, 7), None), ((10, 9, 1), 3), ((6, 6, 6), 5)])
def test_aggregates_partition_and_connect(shape, perm):
    m = wl.cavity(shape, Re=10.0, dt=0.01, perm_seed=perm).mesh
    Fi = m.n_internal
    own, nei = m.owner[:Fi], m.neighbour
    agg, na = amg.aggregate(m.n_cells, own, nei)
    assert agg.min() == 0 and agg.max() == na - 1 and len(set(agg.tolist())) == na
    # connected: union-find over the faces inside aggregates
    parent = list(range(m.n_cells))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in zip(own, nei):
        if agg[a] == agg[b]:
            parent[find(a)] = find(b)
    roots = {}
    for i in range(m.n_cells):
        roots.setdefault(int(agg[i]), set()).add(find(i))
    assert all(len(r) == 1 for r in roots.values())
    assert na < 0.5 * m.n_cells          # 3-D and 2-D hex meshes coarsen by well over 2


@pytest.mark.parametrize("shape,perm", [((9, 8, 7), None), ((10, 9, 1), 3)])
def test_galerkin_is_dense_ptap(shape, perm):
    case = wl.cavity(shape, Re=10.0, dt=0.01, perm_seed=perm)
    rng = np.random.default_rng(3)
    diag, offd = _pressure(case, rng)
    m = case.mesh
    levels = amg.build_hierarchy(m.n_cells, m.owner[:m.n_internal], m.neighbour, coarse_max=8)
    L, C = levels[0], levels[1]
    dc, oc = amg.galerkin(L, diag, offd, C)
    P = np.zeros((L["n"], C["n"]))
    P[np.arange(L["n"]), L["agg"]] = 1.0
    A = amg.dense(L["n"], L["own"], L["nei"], diag, offd)
    Ac = amg.dense(C["n"], C["own"], C["nei"], dc, oc)
    assert np.abs(Ac - P.T @ A @ P).max() <= 1e-12 * np.abs(A).max()


def test_vcycle_symmetric_positive_and_exact_on_one_level():
    case = wl.cavity((12, 11, 10), Re=10.0, dt=0.01, perm_seed=2)
    rng = np.random.default_rng(4)
    diag, offd = _pressure(case, rng)
    m = case.mesh
    own, nei = m.owner[:m.n_internal], m.neighbour
    M = amg.Amg(m.n_cells, own, nei, diag, offd, coarse_max=16)
    assert len(M.levels) >= 3
    u, w = rng.normal(size=m.n_cells), rng.normal(size=m.n_cells)
    a, b = u @ M.vcycle(w), w @ M.vcycle(u)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    for _ in range(5):
        v = rng.normal(size=m.n_cells)
        assert v @ M.vcycle(v) > 0.0
    # one level: the cycle is the exact inverse, CG stops after one iteration
    small = wl.cavity((4, 4, 3), Re=10.0, dt=0.01)
    d2, o2 = _pressure(small, rng)
    ms = small.mesh
    b = rng.normal(size=ms.n_cells)
    M1 = amg.Amg(ms.n_cells, ms.owner[:ms.n_internal], ms.neighbour, d2, o2, coarse_max=128)
    assert len(M1.levels) == 1
    A = amg.dense(ms.n_cells, ms.owner[:ms.n_internal], ms.neighbour, d2, o2)
    assert np.abs(M1.vcycle(b) - np.linalg.solve(A, b)).max() <= 1e-10 * np.abs(np.linalg.solve(A, b)).max()
    x, info = amg.pcg(ms.n_cells, ms.owner[:ms.n_internal], ms.neighbour, d2, o2, b, np.zeros(ms.n_cells), 1e-12)
    assert info["iters"] == 1


def test_pcg_solution_and_fewer_iterations_than_jacobi():
    case = wl.cavity((20, 20, 20), Re=10.0, dt=0.01)
    rng = np.random.default_rng(5)
    diag, offd = _pressure(case, rng)
    m = case.mesh
    own, nei = m.owner[:m.n_internal].copy(), m.neighbour.copy()
    b = rng.normal(size=m.n_cells)
    x, info = amg.pcg(m.n_cells, own, nei, diag, offd, b, np.zeros(m.n_cells), 1e-11)
    A = amg.dense(m.n_cells, own, nei, diag, offd)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    xj, ij = orc.pcg(own, nei, diag, offd, b, np.zeros(m.n_cells), 1e-11)
    assert info["iters"] < 0.5 * ij["iters"], (info["iters"], ij["iters"])


@pytest.mark.parametrize("shape,perm", [((9, 8, 7), None), ((10, 9, 1), 3), ((14, 13, 12), 5), ((30, 30, 30), None)])
def test_library_hierarchy_equals_oracle(shape, perm):
    """fvm_mesh_amg: the library's levels (sizes, coarse faces, aggregation)
    equal the oracle's exactly."""
    import os
    from paper_1207_1571_amd import fvm
    if not os.path.exists(fvm.LIB_PATH):
        pytest.skip("libfvm.so not built")
    case = wl.cavity(shape, Re=10.0, dt=0.01, perm_seed=perm)
    m = case.mesh
    lm = fvm.Mesh(m, case.bcs)
    lib_levels = fvm.mesh_amg(lm)
    ora = amg.build_hierarchy(m.n_cells, m.owner[:m.n_internal], m.neighbour, coarse_max=128)
    assert [L["n"] for L in lib_levels] == [L["n"] for L in ora]
    for l, (a, b) in enumerate(zip(lib_levels, ora)):
        if l > 0:
            assert np.array_equal(a["own"], b["own"]) and np.array_equal(a["nei"], b["nei"])
        if b["agg"] is not None:
            assert np.array_equal(a["agg"], b["agg"]), l
