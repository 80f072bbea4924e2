"""Host side of the C interface, without a GPU.

libfvm.so loads on a machine without a GPU; mesh ingest (validation,
canonical face order, level schedule) and the workspace planner are host
code, so their error behaviour and results are checked here through the
C-ABI itself.  Every function declared in the header must be exported.
"""
import ctypes as ct
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_1207_1571_amd import fvm
from paper_1207_1571_amd import meshgen as mg
from paper_1207_1571_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(fvm.LIB_PATH), reason="libfvm.so not built")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = set()
    for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M):
        head = m.group(0)
        if head.lstrip().startswith(("typedef", "struct", "#", "return", "enum")):
            continue
        names.add(m.group(1))
    return names


def test_header_functions_are_exported():
    names = _declared_functions()
    assert {"piso_step", "simple_iterate", "solve_pressure", "piso_step_batch", "fvm_mesh_create"} <= names
    L = ct.CDLL(fvm.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    # the binding covers exactly the declared interface
    assert set(fvm.EXPORTS) == names


def _mesh(case):
    return fvm.Mesh(case.mesh, case.bcs)


def test_sell_info_regular_and_explicit_slices():
    """A lexicographic 16^3 box: a slice of 256 cells is one z-layer, whose
    column offsets are among +-1, +-16, +-256, so no slice stores indices.
    A lower entry (offset -1, -16, -256) is read through a mirror when the
    neighbour's slices hold the opposite offset in one common slot.  Slice 0
    has no z-neighbour below, so its offsets (-16, -1, 1, 16, 256) sit in
    other slots than the interior slices' (-256, -16, -1, 1, 16, 256): its
    own in-layer lower entries (no lower slice at all) and slice 1's -1 and
    -16 entries (whose neighbours span slices 0 and 1) keep their own copies,
    2 x 2 x 240 entries; every other internal face is read once.  The
    7-point slices (all six offsets, the three lower slots mirrored, both
    neighbouring layers inside the box) are therefore layers 2 to 14: layer
    15 has no layer above it, and layer 1 reads its lower entries from layer
    0, whose slots differ.  A randomly renumbered box stores explicit columns
    in every slice: two entries per internal face, no 7-point slice."""
    m = _mesh(wl.cavity((16, 16, 16), Re=10.0, dt=0.01))
    si = fvm.mesh_sell_info(m)
    assert si["w_slots"] == 6 and si["n_slices"] == 16 and si["n_explicit_slices"] == 0
    assert si["explicit_entries"] == 0
    assert si["mirrored_entries"] == m.n_internal - 4 * 240
    assert si["n_7pt_slices"] == 13
    r = _mesh(wl.cavity((16, 16, 16), Re=10.0, dt=0.01, perm_seed=3))
    si = fvm.mesh_sell_info(r)
    assert si["n_explicit_slices"] == 16 and si["explicit_entries"] == 2 * r.n_internal
    assert si["mirrored_entries"] == 0 and si["n_7pt_slices"] == 0


def test_mesh_info_counts():
    c = wl.cavity((5, 4, 3), Re=10.0, dt=0.01)
    m = _mesh(c)
    assert m.n_cells == 60
    nxf = 4 * 4 * 3 + 5 * 3 * 3 + 5 * 4 * 2
    assert m.n_internal == nxf
    assert m.n_faces == nxf + 2 * (4 * 3 + 5 * 3 + 5 * 4)
    assert not m.non_orthogonal
    cj = wl.cavity((5, 4, 3), Re=10.0, dt=0.01, jitter=0.2, jitter_seed=1)
    assert _mesh(cj).non_orthogonal


def _desc_from(mesh, bcs, **over):
    arrs = dict(owner=np.array(mesh.owner, np.int32), neighbour=np.array(mesh.neighbour, np.int32),
                Sf=np.array(mesh.Sf, np.float64), Cf=np.array(mesh.Cf, np.float64), C=np.array(mesh.C, np.float64),
                V=np.array(mesh.V, np.float64))
    arrs.update(over)
    return dataclasses.replace(mesh, **arrs)


def _expect_einval(mesh, bcs, fragment):
    with pytest.raises(fvm.FvmError) as e:
        fvm.Mesh(mesh, bcs)
    assert e.value.code == -1
    assert fragment in str(e.value)


def test_mesh_validation_errors():
    c = wl.cavity((4, 4, 1), Re=10.0, dt=0.01)
    mesh, bcs = c.mesh, c.bcs
    Fi = len(mesh.neighbour)
    nb = np.array(mesh.neighbour, np.int32)
    nb[3] = mesh.owner[3]
    _expect_einval(_desc_from(mesh, bcs, neighbour=nb), bcs, "owner == neighbour")
    nb = np.array(mesh.neighbour, np.int32)
    nb[0] = mesh.V.shape[0]
    _expect_einval(_desc_from(mesh, bcs, neighbour=nb), bcs, "neighbour out of range")
    ow = np.array(mesh.owner, np.int32)
    ow[-1] = -1
    _expect_einval(_desc_from(mesh, bcs, owner=ow), bcs, "owner out of range")
    V = np.array(mesh.V, np.float64)
    V[2] = 0.0
    _expect_einval(_desc_from(mesh, bcs, V=V), bcs, "V <= 0")
    S = np.array(mesh.Sf, np.float64)
    S[1] *= -1.0
    _expect_einval(_desc_from(mesh, bcs, Sf=S), bcs, "S.d <= 0")
    S = np.array(mesh.Sf, np.float64)
    S[Fi + 1] *= -1.0
    _expect_einval(_desc_from(mesh, bcs, Sf=S), bcs, "S.d <= 0 at boundary")
    # duplicate internal face: face 1 repeats face 0's cell pair
    ow = np.array(mesh.owner, np.int32)
    nb = np.array(mesh.neighbour, np.int32)
    S = np.array(mesh.Sf, np.float64)
    Cf = np.array(mesh.Cf, np.float64)
    ow[1], nb[1], S[1], Cf[1] = ow[0], nb[0], S[0], Cf[0]
    _expect_einval(_desc_from(mesh, bcs, owner=ow, neighbour=nb, Sf=S, Cf=Cf), bcs, "duplicated face")


def test_patch_tiling_errors():
    c = wl.cavity((4, 4, 1), Re=10.0, dt=0.01)
    mesh = c.mesh
    ps = np.array(mesh.patch_size).copy()
    ps[0] -= 1
    bad = dataclasses.replace(mesh, patch_size=ps)
    _expect_einval(bad, c.bcs, "tile")
    bcs = list(c.bcs)
    bcs[0] = wl.PatchBC(7, wl.ZERO_GRAD)
    _expect_einval(mesh, bcs, "unknown boundary kind")


def _opts(case, **kw):
    return fvm.opts_from_case(case.with_(**kw))


def test_option_checks():
    c = wl.cavity((4, 4, 2), Re=10.0, dt=0.01)
    m = _mesh(c)
    good = fvm.workspace_bytes(m, fvm.opts_from_case(c))
    assert good > 0
    bad = [dict(nu=0.0), dict(n_corr=0), dict(n_corr=4, n_non_orth_corr=4), dict(p_ref_cell=m.n_cells),
           dict(precision=7), dict(convection=9), dict(p_ctl=wl.SolverCtl(1e-6, max_iter=0)),
           dict(u_ctl=wl.SolverCtl(-1.0)), dict(precision=wl.MIXED, p_ctl=wl.SolverCtl(1e-6, precond=wl.PC_DIC)),
           dict(precision=wl.MIXED, inner_rel_tol=1.0), dict(u_ctl=wl.SolverCtl(1e-6, precond=wl.PC_DIC)),
           dict(u_solver=7), dict(u_solver=wl.SOLVER_BICGSTAB, precision=wl.MIXED)]
    for kw in bad:
        with pytest.raises(fvm.FvmError):
            fvm.workspace_bytes(m, _opts(c, **kw))


def test_bicgstab_option_accepted_and_sized():
    """BiCGStab keeps two more Krylov vectors per component (p^, s^)."""
    c = wl.cavity((8, 8, 8), Re=10.0, dt=0.01)
    m = _mesh(c)
    base = fvm.workspace_bytes(m, fvm.opts_from_case(c))
    stab = fvm.workspace_bytes(m, _opts(c, u_solver=wl.SOLVER_BICGSTAB))
    assert stab - base == 6 * 8 * m.n_cells


def test_workspace_planner():
    """Workspace grows linearly in the mesh size; the FP32 copies and the DIC
    arrays add what they should; bytes per cell stay in the band of a
    few hundred bytes that a face-addressed FP64 PISO solver needs."""
    sizes = {}
    for n in (8, 16, 24):
        c = wl.cavity((n, n, n), Re=10.0, dt=0.01)
        m = _mesh(c)
        fp64 = fvm.workspace_bytes(m, fvm.opts_from_case(c))
        mixed = fvm.workspace_bytes(m, _opts(c, precision=wl.MIXED))
        dic = fvm.workspace_bytes(m, _opts(c, p_ctl=wl.SolverCtl(1e-6, precond=wl.PC_DIC)))
        assert mixed > fp64 and dic > fp64
        sizes[n] = (m.n_cells, fp64, mixed, dic)
        per_cell = fp64 / m.n_cells
        assert 300 < per_cell < 1500, per_cell
        # FP32 copies: between 1 and 4 floats per cell-face slot added
        assert 40 < (mixed - fp64) / m.n_cells < 400
        # DIC: z and D* in cell order, D*, y, z in level order (FP64), the cells
        # in level order and the dependencies in level order (positions, faces,
        # values)
        assert 100 <= (dic - fp64) / m.n_cells < 200
    # grows with the mesh; the marginal cost per added cell is in the same band
    (n1, a1, _, _), (n2, a2, _, _), (n3, a3, _, _) = sizes[8], sizes[16], sizes[24]
    assert a1 < a2 < a3
    assert 300 < (a3 - a2) / (n3 - n2) < 1500


def test_dic_workspace_is_per_cell():
    """PCG-DIC adds per-cell arrays only: z and D* in cell order, D*, y, z in
    level order (FP64), the cells in level order (int32), and for each of the
    3 lower and 3 upper dependency slots of a hex cell a position and a face
    (int32) and a coefficient (FP64)."""
    for n in (6, 9):
        c = wl.cavity((n, n, n), Re=10.0, dt=0.01, p_precond=wl.PC_DIC)
        m = _mesh(c)
        base = fvm.workspace_bytes(m, _opts(c, p_ctl=wl.SolverCtl(1e-6)))
        dic = fvm.workspace_bytes(m, fvm.opts_from_case(c))
        N = m.n_cells
        expect = 5 * 8 * N + 4 * N + 6 * (4 + 4 + 8) * N
        # each of the 12 arrays is aligned on 256 bytes
        assert expect <= dic - base <= expect + 12 * 256


def test_binding_arity_matches_the_header():
    """Every exported call's parameter count in include/fvm.h equals the
    number of argument types the ctypes binding declares for it (a call
    whose signature changed on one side only would pass garbage)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "fvm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    L = fvm.lib()
    checked = 0
    for name in fvm.EXPORTS:
        m = re.search(r"\b" + name + r"\s*\(([^;]*?)\)\s*;", text, flags=re.S)
        assert m, name
        params = [p for p in m.group(1).split(",") if p.strip()]
        n = 0 if params == ["void"] or [p.strip() for p in params] == ["void"] else len(params)
        argtypes = getattr(L, name).argtypes
        if argtypes is None:
            assert n == 0, name
            continue
        assert len(argtypes) == n, (name, n, len(argtypes))
        checked += 1
    assert checked >= len(fvm.EXPORTS) - 1
