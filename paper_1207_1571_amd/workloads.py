"""Seeded workload recipes: meshes plus boundary conditions and controls.

Everything here is an *input*: which mesh, which patch carries which
boundary kind and value, and the solver controls (viscosity, time step,
tolerances).  The recipes mirror the paper's own test problems (Section 4.1:
lid-driven cavities of increasing resolution, a laminar pipe/channel) at the
sizes the benchmark configurations name.  No solver arithmetic lives here.

Boundary kinds are small integers shared with the C interface:
FIXED = 0 (given value), ZERO_GRAD = 1 (owner-cell value), EMPTY = 2 (face
takes part in no sum; front/back of 2-D slabs).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

from . import meshgen as mg

FIXED, ZERO_GRAD, EMPTY = 0, 1, 2
PC_JACOBI, PC_DIC, PC_AMG = 0, 1, 2
STEP_AUTO, STEP_LAUNCHED = 0, 1
FP64, MIXED = 0, 1
CONV_LINEAR, CONV_UPWIND = 0, 1
SOLVER_BICG, SOLVER_BICGSTAB = 0, 1   # momentum solver


@dataclass
class PatchBC:
    u_kind: int
    p_kind: int
    u_value: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    p_value: float = 0.0


@dataclass
class SolverCtl:
    tol: float
    rel_tol: float = 0.0
    max_iter: int = 10000
    precond: int = PC_JACOBI


@dataclass
class CaseSpec:
    """A complete case: mesh, one BC per patch (in patch order), controls."""

    name: str
    mesh: mg.Mesh
    bcs: List[PatchBC]
    nu: float
    dt: float = 0.0
    alpha_u: float = 1.0
    alpha_p: float = 1.0
    p_ref_value: float = 0.0
    p_ref_cell: int = 0
    n_corr: int = 2
    n_non_orth_corr: int = 0
    convection: int = CONV_LINEAR
    precision: int = FP64
    inner_rel_tol: float = 1e-3
    inner_max_iter: int = 2000
    u_solver: int = SOLVER_BICG
    hybrid_K: int = 0            # > 0: the case also holds the paper's hybrid layout (comparison operators)
    step_kernel: int = 0         # 0: small cases run whole steps in one workgroup; 1: always launched phases
    p_ctl: SolverCtl = field(default_factory=lambda: SolverCtl(1e-6))
    u_ctl: SolverCtl = field(default_factory=lambda: SolverCtl(1e-6))
    mode: str = "piso"            # "piso" | "simple"
    n_steps: int = 1              # PISO steps, or SIMPLE max iterations
    res_tol: float = 1e-6         # SIMPLE stopping threshold on initial residuals

    def with_(self, **kw) -> "CaseSpec":
        return replace(self, **kw)


def _lex_image(mesh: mg.Mesh, lex_index: int) -> int:
    """Cell id that lexicographic cell `lex_index` carries after renumbering."""
    if mesh.lex_of_cell is None:
        return lex_index
    return int(np.nonzero(mesh.lex_of_cell == lex_index)[0][0])


def cavity(n: Tuple[int, int, int], Re: float, dt: float, *, perm_seed: Optional[int] = None,
           use_rcm: bool = False, tol: float = 1e-6, p_precond: int = PC_JACOBI,
           n_steps: int = 1, precision: int = FP64, jitter: float = 0.0, jitter_seed: Optional[int] = None,
           u_lid: float = 1.0, name: str = "cavity") -> CaseSpec:
    """Lid-driven cavity on the unit square/cube.  The lid is the y=1 face
    moving with U=(u_lid,0,0); the other walls are no-slip; p is zero-gradient
    everywhere (pressure level fixed by the reference cell).  A 2-D cavity
    (nz=1) has depth h=1/nx and empty front/back faces.  nu = u_lid*1/Re."""
    nx, ny, nz = n
    Lz = 1.0 / nx if nz == 1 else 1.0
    mesh = mg.box_mesh(nx, ny, nz, lengths=(1.0, 1.0, Lz), jitter=jitter, seed=jitter_seed)
    if perm_seed is not None:
        mesh = mg.random_permutation(mesh, perm_seed)
    if use_rcm:
        mesh = mg.rcm(mesh)
    wall = PatchBC(FIXED, ZERO_GRAD)
    bcs = []
    for side in mesh.patch_names:
        if side == "ymax":
            bcs.append(PatchBC(FIXED, ZERO_GRAD, (u_lid, 0.0, 0.0)))
        elif nz == 1 and side in ("zmin", "zmax"):
            bcs.append(PatchBC(EMPTY, EMPTY))
        else:
            bcs.append(wall)
    return CaseSpec(name=name, mesh=mesh, bcs=bcs, nu=u_lid / Re, dt=dt, p_ref_cell=_lex_image(mesh, 0),
                    p_ctl=SolverCtl(tol, precond=p_precond), u_ctl=SolverCtl(tol), n_steps=n_steps,
                    precision=precision)


def duct(n: Tuple[int, int, int], lengths: Tuple[float, float, float] = (4.0, 1.0, 1.0), Re: float = 50.0,
         *, u_in: float = 1.0, jitter: float = 0.0, jitter_seed: Optional[int] = None,
         mode: str = "simple", n_steps: int = 1, dt: float = 0.0, name: str = "duct") -> CaseSpec:
    """Straight duct along x: plug inlet U=(u_in,0,0) at x=0 (p zero-gradient),
    outlet at x=L with p=0 (U zero-gradient), no-slip side walls.  For nz=1
    the front/back faces are empty (a 2-D plane channel).  nu = u_in*H/Re with
    H the y-extent."""
    nx, ny, nz = n
    mesh = mg.box_mesh(nx, ny, nz, lengths=lengths, jitter=jitter, seed=jitter_seed)
    bcs = []
    for side in mesh.patch_names:
        if side == "xmin":
            bcs.append(PatchBC(FIXED, ZERO_GRAD, (u_in, 0.0, 0.0)))
        elif side == "xmax":
            bcs.append(PatchBC(ZERO_GRAD, FIXED, (0.0, 0.0, 0.0), 0.0))
        elif nz == 1 and side in ("zmin", "zmax"):
            bcs.append(PatchBC(EMPTY, EMPTY))
        else:
            bcs.append(PatchBC(FIXED, ZERO_GRAD))
    return CaseSpec(name=name, mesh=mesh, bcs=bcs, nu=u_in * lengths[1] / Re, dt=dt, mode=mode,
                    n_steps=n_steps, alpha_u=0.7 if mode == "simple" else 1.0,
                    alpha_p=0.3 if mode == "simple" else 1.0,
                    p_ctl=SolverCtl(1e-8, 0.05), u_ctl=SolverCtl(1e-8, 0.1))


# ---------------------------------------------------------------------------
# The benchmark configurations
# ---------------------------------------------------------------------------

def cav2d32() -> CaseSpec:
    """2-D cavity 32x32x1, cells renumbered by a seeded random permutation
    (seed 1), Re=100, PISO dt=0.005, 2 correctors, PCG-Jacobi / PBiCG-Jacobi
    at tol 1e-8, 100 steps, FP64."""
    return cavity((32, 32, 1), Re=100.0, dt=0.005, perm_seed=1, tol=1e-8, n_steps=100, name="cav2d32")


def cav100(n: int = 100, n_steps: int = 50) -> CaseSpec:
    """3-D cavity 100^3, seeded random renumbering (seed 2) then RCM,
    Re=400, PISO dt=0.002, 2 correctors, PCG-DIC pressure / PBiCG momentum at
    tol 1e-7, 50 steps, FP64."""
    return cavity((n, n, n), Re=400.0, dt=0.002, perm_seed=2, use_rcm=True, tol=1e-7, p_precond=PC_DIC,
                  n_steps=n_steps, name=f"cav{n}")


def duct256(shape: Tuple[int, int, int] = (256, 64, 64), max_iters: int = 5000) -> CaseSpec:
    """3-D square duct 256x64x64 on [0,4]x[0,1]^2 with interior-vertex jitter
    +-0.15h (seed 3), Re=50 plug inflow, steady SIMPLE (alpha_U=0.7,
    alpha_p=0.3) until every initial residual is <= 1e-6, FP64."""
    nx, ny, nz = shape
    return duct(shape, lengths=(nx / ny, 1.0, 1.0), jitter=0.15, jitter_seed=3, mode="simple",
                n_steps=max_iters, name="duct%d" % nx).with_(res_tol=1e-6)


def cav200(n: int = 200, n_steps: int = 20, precision: int = FP64) -> CaseSpec:
    """3-D cavity 200^3 lexicographic, Re=1000, PISO dt=0.001, 20 steps,
    PCG-Jacobi / PBiCG-Jacobi at tol 1e-6; FP64 or mixed (FP32 inner)."""
    return cavity((n, n, n), Re=1000.0, dt=0.001, tol=1e-6, n_steps=n_steps, precision=precision,
                  name=f"cav{n}")


def tp1m(nx: int = 3200, ny: int = 300, n_steps: int = 5000, tol: float = 1e-6) -> CaseSpec:
    """Transient 2-D pipe (plane channel) 0.16 m x 0.02 m, nx x ny x 1 cells
    (depth one cell height), nu = 3.3e-6, inlet u_in(t) = 0.01 sin(2 pi 0.5 t)
    set before every step (tp1m_inlet), p = 0 at the outlet, no-slip walls,
    PISO dt = 0.1 ms, 2 correctors, PCG-Jacobi / PBiCG-Jacobi at tol."""
    L, H = 0.16, 0.02
    mesh = mg.box_mesh(nx, ny, 1, lengths=(L, H, H / ny))
    bcs = []
    for side in mesh.patch_names:
        if side == "xmin":
            bcs.append(PatchBC(FIXED, ZERO_GRAD, (0.0, 0.0, 0.0)))
        elif side == "xmax":
            bcs.append(PatchBC(ZERO_GRAD, FIXED, (0.0, 0.0, 0.0), 0.0))
        elif side in ("zmin", "zmax"):
            bcs.append(PatchBC(EMPTY, EMPTY))
        else:
            bcs.append(PatchBC(FIXED, ZERO_GRAD))
    return CaseSpec(name=f"tp{nx}x{ny}", mesh=mesh, bcs=bcs, nu=3.3e-6, dt=1e-4, mode="piso", n_steps=n_steps,
                    p_ctl=SolverCtl(tol), u_ctl=SolverCtl(tol))


def tp1m_inlet(step: int, dt: float = 1e-4, u0: float = 0.01, freq: float = 0.5) -> Tuple[float, float, float]:
    """Inlet velocity for PISO step `step` (0-based): the value at the new
    time level t = (step + 1) dt of the implicit step."""
    t = (step + 1) * dt
    return (u0 * math.sin(2.0 * math.pi * freq * t), 0.0, 0.0)


@dataclass
class ServeRequest:
    rid: int
    arrival_s: float
    kind: str          # "cavity" | "duct"
    n: int
    Re: float
    dt: float
    n_steps: int


def serve_stream(n_requests: int = 512, rate_hz: float = 40.0, seed: int = 5, n_steps: int = 200,
                 side_range: Tuple[int, int] = (16, 96)) -> List[ServeRequest]:
    """Serving stream: each request is a cavity or a duct (Bernoulli 1/2) on an
    n^3 box, n = round(exp(U(ln lo, ln hi))), Re ~ U(10, 1000), dt = 0.2/n,
    Poisson arrivals at `rate_hz`; numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = side_range
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        kind = "cavity" if rng.random() < 0.5 else "duct"
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        Re = float(rng.uniform(10.0, 1000.0))
        out.append(ServeRequest(i, t, kind, n, Re, 0.2 / n, n_steps))
    return out


def serve_case(req: ServeRequest, precision: int = MIXED, tol: float = 1e-6) -> CaseSpec:
    """The case a serving request describes (Jacobi PCG/PBiCG at tol)."""
    if req.kind == "cavity":
        c = cavity((req.n,) * 3, Re=req.Re, dt=req.dt, tol=tol, n_steps=req.n_steps, precision=precision,
                   name=f"req{req.rid}")
    else:
        c = duct((req.n,) * 3, lengths=(1.0, 1.0, 1.0), Re=req.Re, mode="piso", n_steps=req.n_steps,
                 dt=req.dt, name=f"req{req.rid}")
        c = c.with_(p_ctl=SolverCtl(tol), u_ctl=SolverCtl(tol), precision=precision, alpha_u=1.0, alpha_p=1.0)
    return c
