"""solve_pressure_static (the allocation-free pressure solve) against
solve_pressure, called through the C interface: two calls in a row, the
second on a smaller case, each equal bit for bit to the existing entry
point's result (same kernels, same reduction order) and within the FP64
tolerance of the oracle."""
import ctypes as ct
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1207_1571_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _inputs(case, seed):
    rng = np.random.default_rng(seed)
    m = case.mesh
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    rhs = rng.normal(size=m.n_cells)
    rhs -= rhs.mean()
    p0 = rng.normal(size=m.n_cells) * 0.1
    return gamma, rhs, p0


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_solve_equals_solve_pressure(order):
    import torch
    from paper_1207_1571_amd import fvm
    cases = [("renumbered 24x20x16", wl.cavity((24, 20, 16), Re=100.0, dt=0.01, perm_seed=4, tol=1e-9), 1),
             ("lexicographic 12x10x8", wl.cavity((12, 10, 8), Re=100.0, dt=0.01, tol=1e-9), 2)]
    assert cases[1][1].mesh.n_cells < cases[0][1].mesh.n_cells
    for name, case, seed in cases:
        _say(f"solve_pressure_static vs solve_pressure: {name}, {case.mesh.n_cells} cells")
        gamma, rhs, p0 = _inputs(case, seed)
        c = fvm.Case(case)
        g_d, r_d = torch.from_numpy(gamma).cuda(), torch.from_numpy(rhs).cuda()
        p_ref = torch.from_numpy(p0.copy()).cuda()
        st_a, info_a = c.solve_pressure(g_d, r_d, p_ref, 1e-10)
        p_st = torch.from_numpy(p0.copy()).cuda()
        st_b, info_b = c.solve_pressure_static(g_d, r_d, p_st, 1e-10)
        torch.cuda.synchronize()
        a, b = p_ref.cpu().numpy(), p_st.cpu().numpy()
        po = p0.copy()
        st_o, info_o = orc.OracleCase(case).solve_pressure(gamma, rhs, po, 1e-10)
        rel = float(np.linalg.norm(b - po) / np.linalg.norm(po))
        _say(f"  iters static {info_b['iters']} solve_pressure {info_a['iters']} oracle {info_o['iters']}, "
             f"rel vs oracle {rel:.2e}")
        assert st_a == st_b == st_o == 0
        assert info_b["iters"] == info_a["iters"] == info_o["iters"]
        assert info_b["res_final"] == info_a["res_final"]
        assert np.array_equal(a, b)
        assert rel <= 1e-9
        # the case's own pressure field is left untouched
        _, p_case, _ = c.get_state_numpy()
        assert np.all(p_case == 0.0)
        c.close()


def test_static_solve_rejects_what_it_does_not_cover():
    import torch
    from paper_1207_1571_amd import fvm
    case = wl.cavity((6, 5, 4), Re=100.0, dt=0.01, tol=1e-9)
    gamma, rhs, p0 = _inputs(case, 3)
    c = fvm.Case(case)
    g_d, r_d, p_d = (torch.from_numpy(x).cuda() for x in (gamma, rhs, p0))
    L = fvm.lib()
    info = fvm.FvmSolveInfo()
    for precond in (fvm.PC_DIC, fvm.PC_AMG):
        ctl = fvm.FvmSolverCtl(1e-10, 0.0, 100, precond)
        st = L.solve_pressure_static(c.handle, ct.c_void_p(g_d.data_ptr()), ct.c_void_p(r_d.data_ptr()),
                                     ct.c_void_p(p_d.data_ptr()), ct.byref(ctl), None, ct.byref(info))
        assert st == fvm.FVM_EINVAL
        assert b"Jacobi" in L.fvm_last_error()
    mixed = fvm.Case(case.with_(precision=wl.MIXED))
    ctl = fvm.FvmSolverCtl(1e-10, 0.0, 100, fvm.PC_JACOBI)
    st = L.solve_pressure_static(mixed.handle, ct.c_void_p(g_d.data_ptr()), ct.c_void_p(r_d.data_ptr()),
                                 ct.c_void_p(p_d.data_ptr()), ct.byref(ctl), None, ct.byref(info))
    assert st == fvm.FVM_EINVAL
    assert np.array_equal(p_d.cpu().numpy(), p0)
    c.close()
    mixed.close()
