"""Python binding of libfvm (argument marshalling only).

Every step of the solver runs in the HIP library; this module converts numpy
/ torch arguments to the C interface of include/fvm.h and back.  torch is
used for device memory (each case's workspace is a uint8 CUDA tensor) and
for the stream handle.  There is no CPU fallback: if libfvm.so is missing,
loading fails with an error.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfvm.so")

FVM_OK, FVM_WARN_MAXITER, FVM_EINVAL, FVM_ENOMEM, FVM_ENUMERIC, FVM_EDEVICE = 0, 1, -1, -2, -3, -4
BC_FIXED, BC_ZERO_GRAD, BC_EMPTY = 0, 1, 2
PC_JACOBI, PC_DIC, PC_AMG = 0, 1, 2
STEP_AUTO, STEP_LAUNCHED = 0, 1
# fvm_case_operator: face-major layout, then the paper's hybrid layout
OP_GRAD, OP_DIV, OP_LAP, OP_SPMV = 0, 1, 2, 3
OP_HY_GRAD, OP_HY_DIV, OP_HY_LAP, OP_HY_SPMV, OP_HY_STMVP, OP_HY_SETMAT = 4, 5, 6, 7, 8, 9
FP64, MIXED = 0, 1

i32p = ct.POINTER(ct.c_int32)
f64p = ct.POINTER(ct.c_double)


class FvmPatch(ct.Structure):
    _fields_ = [("start", ct.c_int32), ("size", ct.c_int32), ("u_kind", ct.c_int32), ("p_kind", ct.c_int32),
                ("u_value", ct.c_double * 3), ("p_value", ct.c_double)]


class FvmMeshDesc(ct.Structure):
    _fields_ = [("n_cells", ct.c_int32), ("n_faces", ct.c_int32), ("n_internal_faces", ct.c_int32),
                ("n_patches", ct.c_int32), ("owner", i32p), ("neighbour", i32p), ("Sf", f64p), ("Cf", f64p),
                ("C", f64p), ("V", f64p), ("patches", ct.POINTER(FvmPatch))]


class FvmSolverCtl(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("rel_tol", ct.c_double), ("max_iter", ct.c_int32), ("precond", ct.c_int32)]


class FvmCaseOpts(ct.Structure):
    _fields_ = [("nu", ct.c_double), ("dt", ct.c_double), ("alpha_u", ct.c_double), ("alpha_p", ct.c_double),
                ("p_ref_value", ct.c_double), ("inner_rel_tol", ct.c_double), ("n_corr", ct.c_int32),
                ("n_non_orth_corr", ct.c_int32), ("convection", ct.c_int32), ("precision", ct.c_int32),
                ("p_ref_cell", ct.c_int32), ("inner_max_iter", ct.c_int32), ("p_ctl", FvmSolverCtl),
                ("u_ctl", FvmSolverCtl), ("u_solver", ct.c_int32), ("hybrid_K", ct.c_int32),
                ("step_kernel", ct.c_int32)]


class FvmSolveInfo(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("status", ct.c_int32), ("res_initial", ct.c_double),
                ("res_final", ct.c_double)]

    def as_dict(self):
        return dict(iters=self.iters, status=self.status, res_initial=self.res_initial, res_final=self.res_final)


class FvmStepInfo(ct.Structure):
    _fields_ = [("u", FvmSolveInfo * 3), ("p", FvmSolveInfo * 16), ("n_p_solves", ct.c_int32),
                ("status", ct.c_int32)]

    def as_dict(self):
        return dict(u=[self.u[c].as_dict() for c in range(3)],
                    p=[self.p[k].as_dict() for k in range(self.n_p_solves)], status=self.status)


class FvmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfvm error {code}: {msg}")
        self.code = code


_lib = None

EXPORTS = ("fvm_mesh_create", "fvm_mesh_destroy", "fvm_mesh_info", "fvm_case_workspace_bytes", "fvm_case_create",
           "fvm_case_destroy", "fvm_case_set_state", "fvm_case_get_state", "fvm_case_set_patch_value", "piso_step",
           "simple_iterate", "solve_pressure", "fvm_dic_apply", "piso_step_batch", "fvm_profile_enable", "fvm_profile_read",
           "fvm_last_error", "fvm_mesh_hybrid", "fvm_case_operator", "fvm_mesh_amg", "fvm_mesh_sell_info",
           "solve_pressure_static")


def lib():
    """Load libfvm.so (built in-tree by paper_1207_1571_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1207_1571_amd.build`")
        # torch first: libfvm then binds to the HIP runtime torch has loaded,
        # so both share one runtime (and one device context) in the process
        import torch  # noqa: F401
        L = ct.CDLL(LIB_PATH)
        vp = ct.c_void_p
        L.fvm_mesh_create.argtypes = [ct.POINTER(FvmMeshDesc), ct.POINTER(vp)]
        L.fvm_mesh_destroy.argtypes = [vp]
        L.fvm_mesh_destroy.restype = None
        L.fvm_mesh_info.argtypes = [vp, i32p, i32p, i32p, i32p]
        L.fvm_case_workspace_bytes.argtypes = [vp, ct.POINTER(FvmCaseOpts), ct.POINTER(ct.c_size_t)]
        L.fvm_case_create.argtypes = [vp, ct.POINTER(FvmCaseOpts), vp, ct.c_size_t, vp, ct.POINTER(vp)]
        L.fvm_case_destroy.argtypes = [vp]
        L.fvm_case_destroy.restype = None
        L.fvm_case_set_state.argtypes = [vp, vp, vp, vp, vp]
        L.fvm_case_get_state.argtypes = [vp, vp, vp, vp, vp]
        L.fvm_case_set_patch_value.argtypes = [vp, ct.c_int32, ct.POINTER(ct.c_double), ct.c_double, vp]
        L.piso_step.argtypes = [vp, ct.c_int32, vp, ct.POINTER(FvmStepInfo)]
        L.simple_iterate.argtypes = [vp, ct.c_int32, ct.c_double, vp, i32p, ct.POINTER(FvmStepInfo)]
        L.solve_pressure.argtypes = [vp, vp, vp, vp, ct.POINTER(FvmSolverCtl), vp, ct.POINTER(FvmSolveInfo)]
        L.solve_pressure_static.argtypes = [vp, vp, vp, vp, ct.POINTER(FvmSolverCtl), vp, ct.POINTER(FvmSolveInfo)]
        L.fvm_dic_apply.argtypes = [vp, vp, vp, vp, vp, vp]
        L.piso_step_batch.argtypes = [ct.POINTER(vp), ct.c_int32, ct.c_int32, vp, ct.POINTER(FvmStepInfo)]
        L.fvm_profile_enable.argtypes = [ct.c_int32]
        L.fvm_profile_read.argtypes = [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)]
        L.fvm_last_error.restype = ct.c_char_p
        L.fvm_mesh_hybrid.argtypes = [vp, ct.c_int32, i32p, i32p, i32p, i32p, i32p, i32p, i32p]
        L.fvm_case_operator.argtypes = [vp, ct.c_int32, vp, vp, vp]
        L.fvm_mesh_amg.argtypes = [vp, ct.c_int32, i32p, i32p, i32p, i32p, i32p, i32p]
        i64p = ct.POINTER(ct.c_int64)
        L.fvm_mesh_sell_info.argtypes = [vp, i32p, i32p, i32p, i64p, i64p, i32p]
        for name in ("fvm_mesh_create", "fvm_mesh_info", "fvm_case_workspace_bytes", "fvm_case_create",
                     "fvm_case_set_state", "fvm_case_get_state", "fvm_case_set_patch_value", "piso_step",
                     "simple_iterate", "solve_pressure", "solve_pressure_static", "fvm_dic_apply", "piso_step_batch",
                     "fvm_profile_enable",
                     "fvm_profile_read", "fvm_mesh_hybrid", "fvm_case_operator", "fvm_mesh_amg", "fvm_mesh_sell_info"):
            getattr(L, name).restype = ct.c_int32
        _lib = L
    return _lib


def _check(st: int, allow_warn: bool = True) -> int:
    if st < 0 or (st > 0 and not allow_warn):
        raise FvmError(st, lib().fvm_last_error().decode(errors="replace"))
    return st


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Mesh:
    """Host-side canonical mesh (fvm_mesh_create)."""

    def __init__(self, mesh, bcs):
        L = lib()
        self.owner = np.ascontiguousarray(mesh.owner, np.int32)
        self.neighbour = np.ascontiguousarray(mesh.neighbour, np.int32)
        self.Sf = np.ascontiguousarray(mesh.Sf, np.float64)
        self.Cf = np.ascontiguousarray(mesh.Cf, np.float64)
        self.C = np.ascontiguousarray(mesh.C, np.float64)
        self.V = np.ascontiguousarray(mesh.V, np.float64)
        npch = len(mesh.patch_start)
        self.patches = (FvmPatch * max(npch, 1))()
        for p in range(npch):
            b = bcs[p]
            self.patches[p] = FvmPatch(int(mesh.patch_start[p]), int(mesh.patch_size[p]), int(b.u_kind),
                                       int(b.p_kind), (ct.c_double * 3)(*b.u_value), float(b.p_value))
        self.desc = FvmMeshDesc(int(self.V.shape[0]), int(self.owner.shape[0]), int(self.neighbour.shape[0]), npch,
                                self.owner.ctypes.data_as(i32p), self.neighbour.ctypes.data_as(i32p),
                                self.Sf.ctypes.data_as(f64p), self.Cf.ctypes.data_as(f64p),
                                self.C.ctypes.data_as(f64p), self.V.ctypes.data_as(f64p), self.patches)
        h = ct.c_void_p()
        _check(L.fvm_mesh_create(ct.byref(self.desc), ct.byref(h)))
        self.handle = h
        a, b, c, d = ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(L.fvm_mesh_info(h, ct.byref(a), ct.byref(b), ct.byref(c), ct.byref(d)))
        self.n_cells, self.n_faces, self.n_internal, self.non_orthogonal = a.value, b.value, c.value, bool(d.value)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fvm_mesh_destroy(self.handle)
            self.handle = None


def opts_from_case(case) -> FvmCaseOpts:
    return FvmCaseOpts(case.nu, case.dt, case.alpha_u, case.alpha_p, case.p_ref_value, case.inner_rel_tol,
                       case.n_corr, case.n_non_orth_corr, case.convection, case.precision, case.p_ref_cell,
                       case.inner_max_iter,
                       FvmSolverCtl(case.p_ctl.tol, case.p_ctl.rel_tol, case.p_ctl.max_iter, case.p_ctl.precond),
                       FvmSolverCtl(case.u_ctl.tol, case.u_ctl.rel_tol, case.u_ctl.max_iter, case.u_ctl.precond),
                       getattr(case, "u_solver", 0), getattr(case, "hybrid_K", 0), getattr(case, "step_kernel", 0))


def workspace_bytes(mesh: Mesh, opts: FvmCaseOpts) -> int:
    n = ct.c_size_t()
    _check(lib().fvm_case_workspace_bytes(mesh.handle, ct.byref(opts), ct.byref(n)))
    return int(n.value)


class Case:
    """A resident case: its workspace is one CUDA uint8 tensor."""

    def __init__(self, case_spec, device="cuda", stream=None, mesh: Optional[Mesh] = None):
        import torch
        L = lib()
        self.spec = case_spec
        self.mesh = mesh if mesh is not None else Mesh(case_spec.mesh, case_spec.bcs)
        self.opts = opts_from_case(case_spec)
        self.bytes = workspace_bytes(self.mesh, self.opts)
        self.workspace = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.stream = stream
        h = ct.c_void_p()
        _check(L.fvm_case_create(self.mesh.handle, ct.byref(self.opts), ct.c_void_p(self.workspace.data_ptr()),
                                 self.bytes, ct.c_void_p(_stream_ptr(stream)), ct.byref(h)))
        self.handle = h
        self.n_cells, self.n_faces = self.mesh.n_cells, self.mesh.n_faces

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fvm_case_destroy(self.handle)
            self.handle = None

    def close(self):
        self.__del__()

    # ---- state
    def set_state(self, U=None, p=None, phi=None):
        _check(lib().fvm_case_set_state(self.handle, _dptr(U), _dptr(p), _dptr(phi),
                                        ct.c_void_p(_stream_ptr(self.stream))))

    def get_state(self):
        import torch
        dev = self.workspace.device
        U = torch.empty((self.n_cells, 3), dtype=torch.float64, device=dev)
        p = torch.empty(self.n_cells, dtype=torch.float64, device=dev)
        phi = torch.empty(self.n_faces, dtype=torch.float64, device=dev)
        _check(lib().fvm_case_get_state(self.handle, _dptr(U), _dptr(p), _dptr(phi),
                                        ct.c_void_p(_stream_ptr(self.stream))))
        return U, p, phi

    def get_state_numpy(self):
        import torch
        U, p, phi = self.get_state()
        torch.cuda.current_stream().synchronize() if self.stream is None else self.stream.synchronize()
        return U.cpu().numpy(), p.cpu().numpy(), phi.cpu().numpy()

    def set_patch_value(self, patch: int, u_value: Sequence[float], p_value: float):
        arr = (ct.c_double * 3)(*u_value)
        _check(lib().fvm_case_set_patch_value(self.handle, patch, arr, float(p_value),
                                              ct.c_void_p(_stream_ptr(self.stream))))

    # ---- algorithms
    def piso(self, n_steps: int, info: bool = True):
        si = FvmStepInfo()
        st = _check(lib().piso_step(self.handle, n_steps, ct.c_void_p(_stream_ptr(self.stream)),
                                    ct.byref(si) if info else None))
        return st, (si.as_dict() if info else None)

    def simple(self, max_iters: int, res_tol: float):
        si = FvmStepInfo()
        it = ct.c_int32()
        st = _check(lib().simple_iterate(self.handle, max_iters, res_tol, ct.c_void_p(_stream_ptr(self.stream)),
                                         ct.byref(it), ct.byref(si)))
        return st, it.value, si.as_dict()

    def solve_pressure(self, gamma, rhs, p, tol: float, rel_tol: float = 0.0, max_iter: int = 10000,
                       precond: int = PC_JACOBI):
        ctl = FvmSolverCtl(tol, rel_tol, max_iter, precond)
        info = FvmSolveInfo()
        st = _check(lib().solve_pressure(self.handle, _dptr(gamma), _dptr(rhs), _dptr(p), ct.byref(ctl),
                                         ct.c_void_p(_stream_ptr(self.stream)), ct.byref(info)))
        return st, info.as_dict()

    def solve_pressure_static(self, gamma, rhs, p, tol: float, rel_tol: float = 0.0, max_iter: int = 10000):
        """solve_pressure_static: the Jacobi pressure solve with its reduction
        state in the library's static device array (no allocation)."""
        ctl = FvmSolverCtl(tol, rel_tol, max_iter, PC_JACOBI)
        info = FvmSolveInfo()
        st = _check(lib().solve_pressure_static(self.handle, _dptr(gamma), _dptr(rhs), _dptr(p), ct.byref(ctl),
                                                ct.c_void_p(_stream_ptr(self.stream)), ct.byref(info)))
        return st, info.as_dict()


def mesh_sell_info(mesh: Mesh) -> dict:
    """Structure of the sliced-ELL copy the CG's product reads."""
    w, ns, nx, n7 = ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_int32()
    ex, mir = ct.c_int64(), ct.c_int64()
    _check(lib().fvm_mesh_sell_info(mesh.handle, ct.byref(w), ct.byref(ns), ct.byref(nx), ct.byref(ex), ct.byref(mir),
                                    ct.byref(n7)))
    return dict(w_slots=w.value, n_slices=ns.value, n_explicit_slices=nx.value, explicit_entries=ex.value,
                mirrored_entries=mir.value, n_7pt_slices=n7.value)


def mesh_amg(mesh: Mesh):
    """fvm_mesh_amg: the AMG hierarchy, one dict per level (n, own, nei, agg)."""
    import numpy as np
    nl = ct.c_int32()
    _check(lib().fvm_mesh_amg(mesh.handle, 0, ct.byref(nl), None, None, None, None, None))
    out = []
    for l in range(nl.value):
        n, nf = ct.c_int32(), ct.c_int32()
        _check(lib().fvm_mesh_amg(mesh.handle, l, None, ct.byref(n), ct.byref(nf), None, None, None))
        own, nei = np.empty(max(nf.value, 1), np.int32), np.empty(max(nf.value, 1), np.int32)
        agg = np.empty(max(n.value, 1), np.int32)
        last = l == nl.value - 1
        _check(lib().fvm_mesh_amg(mesh.handle, l, None, None, None, own.ctypes.data_as(i32p), nei.ctypes.data_as(i32p),
                                  None if last else agg.ctypes.data_as(i32p)))
        out.append(dict(n=n.value, own=own[:nf.value], nei=nei[:nf.value], agg=None if last else agg[:n.value]))
    return out


def mesh_hybrid(mesh: Mesh, K: int):
    """fvm_mesh_hybrid: the paper-form index arrays of the hybrid layout."""
    import numpy as np
    nC = ct.c_int32()
    _check(lib().fvm_mesh_hybrid(mesh.handle, K, ct.byref(nC), None, None, None, None, None, None))
    N = mesh.n_cells
    out = dict(I=np.empty((N, K), np.int32), J=np.empty((N, K), np.int32), Q=np.empty((N, K), np.int32),
               c_start=np.empty(N + 1, np.int32), c_col=np.empty(max(nC.value, 1), np.int32),
               c_tr=np.empty(max(nC.value, 1), np.int32))
    p = {k: v.ctypes.data_as(i32p) for k, v in out.items()}
    _check(lib().fvm_mesh_hybrid(mesh.handle, K, None, p["I"], p["J"], p["Q"], p["c_start"], p["c_col"], p["c_tr"]))
    out["c_col"] = out["c_col"][:nC.value]
    out["c_tr"] = out["c_tr"][:nC.value]
    return out


def operator(case: Case, op: int, x, out=None):
    """fvm_case_operator on the case's stream (device tensors)."""
    _check(lib().fvm_case_operator(case.handle, op, _dptr(x), _dptr(out), ct.c_void_p(_stream_ptr(case.stream))))


def dic_apply(case: Case, gamma, r, z, dstar=None):
    _check(lib().fvm_dic_apply(case.handle, _dptr(gamma), _dptr(r), _dptr(z), _dptr(dstar),
                               ct.c_void_p(_stream_ptr(case.stream))))


def piso_batch(cases: Sequence[Case], n_steps: int, stream=None, raise_on_case_failure: bool = True):
    """piso_step_batch.  A case whose solve failed is rolled back and left out
    of the remaining steps; its info carries the negative status.  With
    raise_on_case_failure=False such per-case failures are returned in the
    infos instead of raised (argument and device errors still raise)."""
    arr = (ct.c_void_p * len(cases))(*[c.handle for c in cases])
    infos = (FvmStepInfo * max(1, len(cases)))()
    st = lib().piso_step_batch(arr, len(cases), n_steps, ct.c_void_p(_stream_ptr(stream)), infos)
    out = [infos[i].as_dict() for i in range(len(cases))]
    case_failure = st < 0 and any(o["status"] < 0 for o in out) and st not in (-1, -2, -4)
    if not (case_failure and not raise_on_case_failure):
        _check(st)
    return st, out


def profile_enable(on: bool):
    _check(lib().fvm_profile_enable(1 if on else 0))


def profile_read(kernel_class: str):
    ms = ct.c_double()
    n = ct.c_int64()
    _check(lib().fvm_profile_read(kernel_class.encode(), ct.byref(ms), ct.byref(n)))
    return ms.value, n.value
