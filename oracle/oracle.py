"""ctypes shim of the FP64 CPU oracle (fvm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  This module imports
nothing from the HIP package; meshes and cases are accepted by duck typing
(objects with the attributes the seeded input generators produce).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fvm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

i32p = ct.POINTER(ct.c_int32)
f64p = ct.POINTER(ct.c_double)

ST_OK, ST_MAXITER, ST_EINVAL, ST_ENOMEM, ST_ENUMERIC = 0, 1, -1, -2, -3


class OrcMesh(ct.Structure):
    _fields_ = [("n_cells", ct.c_int32), ("n_faces", ct.c_int32), ("n_internal", ct.c_int32),
                ("n_patches", ct.c_int32), ("owner", i32p), ("neighbour", i32p), ("Sf", f64p), ("Cf", f64p),
                ("C", f64p), ("V", f64p), ("patch_start", i32p), ("patch_size", i32p), ("patch_u_kind", i32p),
                ("patch_p_kind", i32p), ("patch_u_value", f64p), ("patch_p_value", f64p)]


class OrcOpts(ct.Structure):
    _fields_ = [("nu", ct.c_double), ("dt", ct.c_double), ("alpha_u", ct.c_double), ("alpha_p", ct.c_double),
                ("p_ref_value", ct.c_double), ("p_tol", ct.c_double), ("p_rel_tol", ct.c_double),
                ("u_tol", ct.c_double), ("u_rel_tol", ct.c_double), ("n_corr", ct.c_int32),
                ("n_non_orth_corr", ct.c_int32), ("convection", ct.c_int32), ("p_ref_cell", ct.c_int32),
                ("p_max_iter", ct.c_int32), ("p_precond", ct.c_int32), ("u_max_iter", ct.c_int32),
                ("u_solver", ct.c_int32)]


class OrcSolveInfo(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("status", ct.c_int32), ("res_initial", ct.c_double),
                ("res_final", ct.c_double)]

    def as_dict(self):
        return dict(iters=self.iters, status=self.status, res_initial=self.res_initial, res_final=self.res_final)


class OrcStepInfo(ct.Structure):
    _fields_ = [("u", OrcSolveInfo * 3), ("p", OrcSolveInfo * 16), ("n_p_solves", ct.c_int32),
                ("status", ct.c_int32)]

    def as_dict(self):
        return dict(u=[self.u[c].as_dict() for c in range(3)],
                    p=[self.p[k].as_dict() for k in range(self.n_p_solves)], status=self.status)


_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")


def build(force: bool = False, native: bool = False) -> str:
    """Compile liboracle.so with gcc (ISO C99, no fast-math, no contraction
    of multiply-adds).  native=True builds liboracle_native.so for the host
    it runs on (-O3 -march=native), used to time the oracle as a CPU
    baseline; both give the same results (the same IEEE operations in the
    same order)."""
    out = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        subprocess.check_call(["gcc", "-std=c99", *opt, "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None
_use_native = False


def select_native() -> str:
    """Load the host-tuned build in this process (must come before the
    first use of the oracle); returns its path."""
    global _use_native
    if _lib is not None and not _use_native:
        raise RuntimeError("the oracle library is already loaded")
    _use_native = True
    return build(force=True, native=True)


def lib():
    global _lib
    if _lib is None:
        path = build(native=_use_native)
        L = ct.CDLL(path)
        M, O = ct.POINTER(OrcMesh), ct.POINTER(OrcOpts)
        SI, STI = ct.POINTER(OrcSolveInfo), ct.POINTER(OrcStepInfo)
        L.orc_flux_from_U.argtypes = [M, f64p, f64p]
        L.orc_face_coeffs.argtypes = [M, f64p, f64p, f64p, i32p]
        L.orc_grad.argtypes = [M, f64p, i32p, f64p, f64p]
        L.orc_momentum_system.argtypes = [M, ct.c_double, ct.c_double, ct.c_int32, f64p, f64p, f64p, f64p, f64p,
                                          f64p, f64p]
        L.orc_pressure_system.argtypes = [M, f64p, f64p, f64p, i32p, f64p, ct.c_int32, ct.c_double, f64p, f64p,
                                          f64p]
        L.orc_amul.argtypes = [ct.c_int32, ct.c_int32, i32p, i32p, f64p, f64p, f64p, f64p, f64p, ct.c_int32]
        L.orc_pcg.argtypes = [ct.c_int32, ct.c_int32, i32p, i32p, f64p, f64p, f64p, f64p, ct.c_double, ct.c_double,
                              ct.c_int32, ct.c_int32, SI]
        L.orc_pbicg.argtypes = [ct.c_int32, ct.c_int32, i32p, i32p, f64p, f64p, f64p, f64p, f64p, ct.c_double,
                                ct.c_double, ct.c_int32, SI]
        L.orc_pbicgstab.argtypes = L.orc_pbicg.argtypes
        L.orc_dic.argtypes = [ct.c_int32, ct.c_int32, i32p, i32p, f64p, f64p, f64p, f64p, f64p]
        L.orc_nres.argtypes = [ct.c_int32, ct.c_int32, i32p, i32p, f64p, f64p, f64p, f64p, f64p]
        L.orc_nres.restype = ct.c_double
        L.orc_piso.argtypes = [M, O, f64p, f64p, f64p, ct.c_int32, STI]
        L.orc_simple.argtypes = [M, O, f64p, f64p, f64p, ct.c_int32, ct.c_double, i32p, STI]
        L.orc_solve_pressure.argtypes = [M, O, f64p, f64p, f64p, ct.c_double, ct.c_double, ct.c_int32, ct.c_int32, SI]
        _lib = L
    return _lib


def _f(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(f64p)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(i32p)


def _nullf():
    return ct.cast(None, f64p)


class OMesh:
    """Keeps the numpy arrays of a mesh (+ patch BCs) alive behind an OrcMesh."""

    def __init__(self, mesh, bcs=None):
        self.owner = np.ascontiguousarray(mesh.owner, np.int32)
        self.neighbour = np.ascontiguousarray(mesh.neighbour, np.int32)
        self.Sf = np.ascontiguousarray(mesh.Sf, np.float64)
        self.Cf = np.ascontiguousarray(mesh.Cf, np.float64)
        self.C = np.ascontiguousarray(mesh.C, np.float64)
        self.V = np.ascontiguousarray(mesh.V, np.float64)
        self.pstart = np.ascontiguousarray(mesh.patch_start, np.int32)
        self.psize = np.ascontiguousarray(mesh.patch_size, np.int32)
        npch = self.pstart.shape[0]
        if bcs is None:
            bcs_uk = np.zeros(npch, np.int32); bcs_pk = np.ones(npch, np.int32)
            uv = np.zeros((npch, 3)); pv = np.zeros(npch)
        else:
            bcs_uk = np.array([b.u_kind for b in bcs], np.int32)
            bcs_pk = np.array([b.p_kind for b in bcs], np.int32)
            uv = np.array([b.u_value for b in bcs], np.float64).reshape(npch, 3)
            pv = np.array([b.p_value for b in bcs], np.float64)
        self.uk, self.pk = bcs_uk, bcs_pk
        self.uv, self.pv = np.ascontiguousarray(uv), np.ascontiguousarray(pv)
        self.N = self.V.shape[0]
        self.F = self.owner.shape[0]
        self.Fi = self.neighbour.shape[0]
        self.s = OrcMesh(self.N, self.F, self.Fi, npch, _i(self.owner), _i(self.neighbour), _f(self.Sf),
                         _f(self.Cf), _f(self.C), _f(self.V), _i(self.pstart), _i(self.psize), _i(self.uk),
                         _i(self.pk), _f(self.uv), _f(self.pv))

    def ref(self):
        return ct.byref(self.s)


def opts_from_case(case) -> OrcOpts:
    return OrcOpts(case.nu, case.dt, case.alpha_u, case.alpha_p, case.p_ref_value, case.p_ctl.tol,
                   case.p_ctl.rel_tol, case.u_ctl.tol, case.u_ctl.rel_tol, case.n_corr, case.n_non_orth_corr,
                   case.convection, case.p_ref_cell, case.p_ctl.max_iter, case.p_ctl.precond, case.u_ctl.max_iter,
                   case.u_solver)


# ---------------------------------------------------------------------------
# Case-level drivers
# ---------------------------------------------------------------------------

class OracleCase:
    """Oracle state (U[N,3], p[N], phi[F]) of one case, advanced in place."""

    def __init__(self, case, U=None, p=None, phi=None):
        self.case = case
        self.om = OMesh(case.mesh, case.bcs)
        self.opts = opts_from_case(case)
        N, F = self.om.N, self.om.F
        self.U = np.zeros((N, 3)) if U is None else np.array(U, np.float64, order="C").reshape(N, 3)
        self.p = np.zeros(N) if p is None else np.array(p, np.float64)
        if phi is None:
            self.phi = np.zeros(F)
            st = lib().orc_flux_from_U(self.om.ref(), _f(self.U), _f(self.phi))
            assert st == ST_OK, st
        else:
            self.phi = np.array(phi, np.float64)

    def piso(self, n_steps: int) -> Tuple[int, dict]:
        info = OrcStepInfo()
        st = lib().orc_piso(self.om.ref(), ct.byref(self.opts), _f(self.U), _f(self.p), _f(self.phi), n_steps,
                            ct.byref(info))
        return st, info.as_dict()

    def simple(self, max_iters: int, res_tol: float) -> Tuple[int, int, dict]:
        info = OrcStepInfo()
        it = ct.c_int32(0)
        st = lib().orc_simple(self.om.ref(), ct.byref(self.opts), _f(self.U), _f(self.p), _f(self.phi), max_iters,
                              res_tol, ct.byref(it), ct.byref(info))
        return st, it.value, info.as_dict()

    def solve_pressure(self, gamma: np.ndarray, rhs: np.ndarray, p: np.ndarray, tol: float, rel_tol: float = 0.0,
                       max_iter: int = 10000, precond: int = 0) -> Tuple[int, dict]:
        info = OrcSolveInfo()
        g = np.ascontiguousarray(gamma, np.float64); r = np.ascontiguousarray(rhs, np.float64)
        st = lib().orc_solve_pressure(self.om.ref(), ct.byref(self.opts), _f(g), _f(r), _f(p), tol, rel_tol, max_iter,
                                      precond, ct.byref(info))
        return st, info.as_dict()


# ---------------------------------------------------------------------------
# Operator-level access (for pins)
# ---------------------------------------------------------------------------

def face_coeffs(mesh):
    om = OMesh(mesh)
    w = np.zeros(om.Fi); dl = np.zeros(om.F); k = np.zeros((om.Fi, 3)); no = ct.c_int32(0)
    st = lib().orc_face_coeffs(om.ref(), _f(w), _f(dl), _f(k), ct.byref(no))
    assert st == ST_OK, st
    return w, dl, k, bool(no.value)


def grad(mesh, phi: np.ndarray, bkind: np.ndarray, bval: np.ndarray) -> np.ndarray:
    om = OMesh(mesh)
    out = np.zeros((om.N, 3))
    st = lib().orc_grad(om.ref(), _f(np.ascontiguousarray(phi, np.float64)), _i(np.ascontiguousarray(bkind, np.int32)),
                        _f(np.ascontiguousarray(bval, np.float64)), _f(out))
    assert st == ST_OK, st
    return out


def momentum_system(mesh, bcs, nu, dt, convection, phi, U_old=None, U_grad=None):
    om = OMesh(mesh, bcs)
    diag = np.zeros(om.N); up = np.zeros(om.Fi); lo = np.zeros(om.Fi); src = np.zeros((om.N, 3))
    Uo = _nullf() if U_old is None else _f(np.ascontiguousarray(U_old, np.float64))
    Ug = _nullf() if U_grad is None else _f(np.ascontiguousarray(U_grad, np.float64))
    st = lib().orc_momentum_system(om.ref(), nu, dt, convection, _f(np.ascontiguousarray(phi, np.float64)), Uo, Ug,
                                   _f(diag), _f(up), _f(lo), _f(src))
    assert st == ST_OK, st
    return diag, up, lo, src


def pressure_system(mesh, gamma, pbkind, pbval, phiH=None, gradp=None, pin_cell=-1, p_ref=0.0):
    om = OMesh(mesh)
    diag = np.zeros(om.N); offd = np.zeros(om.Fi); b = np.zeros(om.N)
    ph = _nullf() if phiH is None else _f(np.ascontiguousarray(phiH, np.float64))
    gp = _nullf() if gradp is None else _f(np.ascontiguousarray(gradp, np.float64))
    st = lib().orc_pressure_system(om.ref(), _f(np.ascontiguousarray(gamma, np.float64)), ph, gp,
                                   _i(np.ascontiguousarray(pbkind, np.int32)),
                                   _f(np.ascontiguousarray(pbval, np.float64)), pin_cell, p_ref, _f(diag), _f(offd),
                                   _f(b))
    assert st == ST_OK, st
    return diag, offd, b


def amul(own, nei, diag, upper, lower, x, transpose=False):
    N = diag.shape[0]
    y = np.zeros(N)
    lib().orc_amul(N, nei.shape[0], _i(own), _i(nei), _f(diag), _f(upper), _f(lower), _f(x), _f(y), int(transpose))
    return y


def pcg(own, nei, diag, offd, b, x0, tol, rel_tol=0.0, max_iter=10000, precond=0):
    x = np.array(x0, np.float64)
    info = OrcSolveInfo()
    lib().orc_pcg(diag.shape[0], nei.shape[0], _i(own), _i(nei), _f(diag), _f(offd), _f(b), _f(x), tol, rel_tol,
                  max_iter, precond, ct.byref(info))
    return x, info.as_dict()


def pbicg(own, nei, diag, upper, lower, b, x0, tol, rel_tol=0.0, max_iter=10000):
    x = np.array(x0, np.float64)
    info = OrcSolveInfo()
    lib().orc_pbicg(diag.shape[0], nei.shape[0], _i(own), _i(nei), _f(diag), _f(upper), _f(lower), _f(b), _f(x), tol,
                    rel_tol, max_iter, ct.byref(info))
    return x, info.as_dict()


def pbicgstab(own, nei, diag, upper, lower, b, x0, tol, rel_tol=0.0, max_iter=10000):
    x = np.array(x0, np.float64)
    info = OrcSolveInfo()
    lib().orc_pbicgstab(diag.shape[0], nei.shape[0], _i(own), _i(nei), _f(diag), _f(upper), _f(lower), _f(b), _f(x),
                        tol, rel_tol, max_iter, ct.byref(info))
    return x, info.as_dict()


def dic(own, nei, diag, offd, r=None):
    N = diag.shape[0]
    dstar = np.zeros(N)
    z = np.zeros(N)
    rr = _nullf() if r is None else _f(np.ascontiguousarray(r, np.float64))
    st = lib().orc_dic(N, nei.shape[0], _i(own), _i(nei), _f(diag), _f(offd), rr, _f(dstar),
                       _f(z) if r is not None else _nullf())
    assert st == ST_OK, st
    return dstar, (z if r is not None else None)


def nres(own, nei, diag, upper, lower, b, x):
    return lib().orc_nres(diag.shape[0], nei.shape[0], _i(own), _i(nei), _f(diag), _f(upper), _f(lower), _f(b), _f(x))
