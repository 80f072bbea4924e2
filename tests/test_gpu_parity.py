"""Parity of the HIP path (through the C interface) with the FP64 oracle.

Protocol: run the same seeded case on both sides and compare U, p and phi by
relative L2 error.  When every per-solve iteration count of the compared
step agrees, the fields must agree to 1e-9 (FP64).  A count that differs at
a threshold crossing moves the fields by about the tolerance; such cases are
rerun on both sides with the tolerance divided by 1e3 before comparing.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1207_1571_amd import meshgen as mg
from paper_1207_1571_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _gpu(case, steps=None, simple=False, res_tol=None, U=None, p=None, phi=None):
    import torch
    from paper_1207_1571_amd import fvm
    c = fvm.Case(case)
    if U is not None:
        c.set_state(torch.from_numpy(np.ascontiguousarray(U)).cuda(), torch.from_numpy(np.ascontiguousarray(p)).cuda(),
                    None if phi is None else torch.from_numpy(np.ascontiguousarray(phi)).cuda())
    if simple:
        st, it, info = c.simple(steps, res_tol)
    else:
        st, info = c.piso(steps)
        it = steps
    Ug, pg, phig = c.get_state_numpy()
    return dict(st=st, it=it, info=info, U=Ug, p=pg, phi=phig, case=c)


def _oracle(case, steps, simple=False, res_tol=None, U=None, p=None, phi=None):
    oc = orc.OracleCase(case, U=U, p=p, phi=phi)
    if simple:
        st, it, info = oc.simple(steps, res_tol)
    else:
        st, info = oc.piso(steps)
        it = steps
    return dict(st=st, it=it, info=info, U=oc.U, p=oc.p, phi=oc.phi)


def _counts(info):
    return [s["iters"] for s in info["u"]] + [s["iters"] for s in info["p"]]


def _compare(g, o, tol=TOL_FP64, what=""):
    eU, ep, ephi = _rel(g["U"], o["U"]), _rel(g["p"], o["p"]), _rel(g["phi"], o["phi"])
    _say(f"  {what}: relL2 U {eU:.2e} p {ep:.2e} phi {ephi:.2e}; iters gpu {_counts(g['info'])} "
         f"oracle {_counts(o['info'])}")
    assert eU <= tol and ep <= tol and ephi <= tol, (eU, ep, ephi)


def _parity(case, steps, simple=False, res_tol=None, what=""):
    _say(f"[parity] {what} N={case.mesh.n_cells} steps={steps}")
    g = _gpu(case, steps, simple, res_tol)
    o = _oracle(case, steps, simple, res_tol)
    assert g["st"] == o["st"], (g["st"], o["st"])
    if simple:
        assert g["it"] == o["it"], (g["it"], o["it"])
    if _counts(g["info"]) != _counts(o["info"]):
        _say(f"  iteration counts differ at a threshold: rerun with tolerances / 1e3")
        tight = case.with_(p_ctl=wl.SolverCtl(case.p_ctl.tol * 1e-3, case.p_ctl.rel_tol * 1e-3,
                                              case.p_ctl.max_iter, case.p_ctl.precond),
                           u_ctl=wl.SolverCtl(case.u_ctl.tol * 1e-3, case.u_ctl.rel_tol * 1e-3, case.u_ctl.max_iter))
        g = _gpu(tight, steps, simple, res_tol)
        o = _oracle(tight, steps, simple, res_tol)
    _compare(g, o, what=what)
    return g, o


def test_cav2d32_full_run():
    """The 2-D cavity configuration exactly: 32x32x1, random renumbering
    (seed 1), Re=100, dt=0.005, 2 correctors, tol 1e-8, 100 PISO steps."""
    case = wl.cav2d32()
    g, o = _parity(case, case.n_steps, what="cav2d32")
    # divergence-free corrected flux (identity of the pressure equation)
    m = case.mesh
    div = np.zeros(m.n_cells)
    np.add.at(div, m.owner, g["phi"])
    np.add.at(div, m.neighbour, -g["phi"][: m.n_internal])
    assert np.abs(div).max() <= 1e-6 * np.abs(g["phi"]).max()


@pytest.mark.parametrize("shape,perm", [((9, 7, 5), 3), ((17, 1, 13), None), ((6, 6, 6), 11)])
def test_cavity3d_parity_several_tiles(shape, perm):
    case = wl.cavity(shape, Re=200.0, dt=0.01, perm_seed=perm, tol=1e-9, n_steps=6)
    _parity(case, 6, what=f"cavity {shape}")


def test_noncanonical_face_order_and_orientation():
    case = wl.cavity((7, 6, 5), Re=150.0, dt=0.01, perm_seed=4, tol=1e-9)
    sh = case.with_(mesh=mg.shuffle_faces(case.mesh, seed=2))
    _parity(sh, 4, what="shuffled faces")


def test_upwind_and_rcm_parity():
    case = wl.cavity((12, 10, 8), Re=400.0, dt=0.01, perm_seed=2, use_rcm=True, tol=1e-9).with_(convection=1)
    _parity(case, 4, what="upwind rcm")


def test_simple_jittered_duct_parity():
    # relative inner tolerances let an early outer iteration cross a stopping
    # threshold on one side only; absolute tight tolerances keep every outer
    # iteration comparable
    case = wl.duct256((32, 8, 8)).with_(p_ctl=wl.SolverCtl(1e-12, 0.0), u_ctl=wl.SolverCtl(1e-12, 0.0))
    _parity(case, 12, simple=True, res_tol=0.0, what="SIMPLE jittered duct")


def test_piso_jittered_duct_nonorth_correctors():
    case = wl.duct((16, 6, 6), lengths=(2.0, 1.0, 1.0), Re=50.0, jitter=0.2, jitter_seed=7, mode="piso",
                   dt=0.01).with_(p_ctl=wl.SolverCtl(1e-10), u_ctl=wl.SolverCtl(1e-10), n_non_orth_corr=1)
    _parity(case, 3, what="PISO jittered, 1 non-orth corrector")


def test_bicgstab_momentum_parity():
    """The BiCGStab momentum solver (the paper's GPU choice) against the
    oracle's: PISO on a renumbered 3-D cavity, SIMPLE on the jittered duct."""
    case = wl.cavity((9, 7, 5), Re=300.0, dt=0.01, perm_seed=3, tol=1e-9).with_(u_solver=wl.SOLVER_BICGSTAB)
    _parity(case, 4, what="BiCGStab cavity")
    duct = wl.duct256((32, 8, 8)).with_(p_ctl=wl.SolverCtl(1e-12, 0.0), u_ctl=wl.SolverCtl(1e-12, 0.0),
                                        u_solver=wl.SOLVER_BICGSTAB)
    _parity(duct, 8, simple=True, res_tol=0.0, what="BiCGStab SIMPLE duct")


@pytest.mark.parametrize("variant", ["jacobi", "dic", "mixed", "bicgstab", "amg"])
def test_captured_iteration_chunks_equal_direct_launches(variant):
    """Krylov iterations launched through captured graphs (the default) and
    launched one by one (per-launch profiling turns capture off) give the
    same fields bit for bit, over several steps and many graph replays."""
    from paper_1207_1571_amd import fvm
    kw = dict(Re=300.0, dt=0.01, perm_seed=4, tol=1e-9)
    if variant == "dic":
        kw["p_precond"] = wl.PC_DIC
    if variant == "amg":
        kw["p_precond"] = wl.PC_AMG
    if variant == "mixed":
        kw["precision"] = wl.MIXED
    case = wl.cavity((14, 12, 10), **kw).with_(step_kernel=wl.STEP_LAUNCHED)
    if variant == "bicgstab":
        case = case.with_(u_solver=wl.SOLVER_BICGSTAB)
    out = []
    for profile in (False, True):
        fvm.profile_enable(profile)
        try:
            _say(f"  {variant}: per-launch profiling {profile}")
            c = fvm.Case(case)
            st, info = c.piso(4)
            out.append((c.get_state_numpy(), _counts(info)))
            c.close()
        finally:
            fvm.profile_enable(False)
    (a, ca), (b, cb) = out
    _say(f"  {variant}: iterations {ca}")
    assert ca == cb
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_solve_pressure_parity():
    import torch
    from paper_1207_1571_amd import fvm
    case = wl.cavity((15, 13, 9), Re=100.0, dt=0.01, perm_seed=6, tol=1e-9)
    rng = np.random.default_rng(0)
    m = case.mesh
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    rhs = rng.normal(size=m.n_cells)
    rhs -= rhs.mean()
    p0 = rng.normal(size=m.n_cells) * 0.1
    oc = orc.OracleCase(case)
    po = p0.copy()
    st_o, info_o = oc.solve_pressure(gamma, rhs, po, 1e-10)
    c = fvm.Case(case)
    pg = torch.from_numpy(p0.copy()).cuda()
    st_g, info_g = c.solve_pressure(torch.from_numpy(gamma).cuda(), torch.from_numpy(rhs).cuda(), pg, 1e-10)
    _say(f"  solve_pressure iters gpu {info_g['iters']} oracle {info_o['iters']}")
    assert st_g == st_o == 0
    assert info_g["iters"] == info_o["iters"]
    assert _rel(pg.cpu().numpy(), po) <= TOL_FP64
    # the case's own pressure field is left untouched
    _, p_case, _ = c.get_state_numpy()
    assert np.all(p_case == 0.0)


def test_zero_lid_exact_rest_and_zero_iterations():
    case = wl.cavity((8, 8, 8), Re=100.0, dt=0.01, tol=1e-8, u_lid=0.0).with_(nu=0.01)
    g = _gpu(case, 3)
    assert np.all(g["U"] == 0.0) and np.all(g["p"] == 0.0) and np.all(g["phi"] == 0.0)
    assert all(k == 0 for k in _counts(g["info"]))


def test_determinism_and_restart_bitwise():
    case = wl.cavity((10, 9, 7), Re=300.0, dt=0.01, perm_seed=1, tol=1e-8)
    a = _gpu(case, 6)
    b = _gpu(case, 6)
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["p"], b["p"]) and np.array_equal(a["phi"], b["phi"])
    h = _gpu(case, 3)
    r = _gpu(case, 3, U=h["U"], p=h["p"], phi=h["phi"])
    assert np.array_equal(a["U"], r["U"]) and np.array_equal(a["p"], r["p"]) and np.array_equal(a["phi"], r["phi"])


def test_maxiter_warning_and_breakdown_rollback():
    import torch
    from paper_1207_1571_amd import fvm
    case = wl.cavity((6, 6, 1), Re=100.0, dt=0.005, tol=1e-8).with_(p_ctl=wl.SolverCtl(0.0, max_iter=5))
    g = _gpu(case, 1)
    o = _oracle(case, 1)
    assert g["st"] == o["st"] == fvm.FVM_WARN_MAXITER
    assert g["info"]["p"][0]["iters"] == 5
    _compare(g, o, what="max_iter")
    # a non-finite state is reported and the step rolled back
    c = fvm.Case(wl.cavity((6, 6, 1), Re=100.0, dt=0.005, tol=1e-8))
    U = np.zeros((36, 3)); U[5, 0] = np.nan
    c.set_state(torch.from_numpy(U).cuda(), torch.zeros(36, dtype=torch.float64, device="cuda"), None)
    U0, p0, phi0 = c.get_state_numpy()
    with pytest.raises(fvm.FvmError) as e:
        c.piso(1)
    assert e.value.code == fvm.FVM_ENUMERIC
    U1, p1, phi1 = c.get_state_numpy()
    assert np.array_equal(np.isnan(U0), np.isnan(U1)) and np.array_equal(np.nan_to_num(U0), np.nan_to_num(U1))


def test_time_dependent_patch_value():
    from paper_1207_1571_amd import fvm
    case = wl.duct((24, 8, 1), lengths=(3.0, 1.0, 1.0 / 8), Re=20.0, mode="piso", dt=0.01)
    case = case.with_(p_ctl=wl.SolverCtl(1e-10), u_ctl=wl.SolverCtl(1e-10))
    c = fvm.Case(case)
    oc = orc.OracleCase(case)
    for k in range(4):
        u = 0.5 + 0.25 * k
        c.set_patch_value(0, (u, 0.0, 0.0), 0.0)
        case.bcs[0].u_value = (u, 0.0, 0.0)
        oc2 = orc.OracleCase(case, U=oc.U, p=oc.p, phi=oc.phi)
        c.piso(1)
        oc2.piso(1)
        oc = oc2
    Ug, pg, phig = c.get_state_numpy()
    assert _rel(Ug, oc.U) <= TOL_FP64 and _rel(pg, oc.p) <= TOL_FP64


def test_transient_pipe_sinusoidal_inlet_parity():
    """The transient pipe (tp1M's geometry, viscosity and time step at a
    reduced 160 x 15 resolution): the inlet velocity follows the sinusoid,
    set through fvm_case_set_patch_value before every step."""
    from paper_1207_1571_amd import fvm
    case = wl.tp1m(nx=160, ny=15, tol=1e-10)
    c = fvm.Case(case)
    oc = orc.OracleCase(case)
    for k in range(6):
        u = wl.tp1m_inlet(2500 + 400 * k)      # sweeps through the sinusoid
        c.set_patch_value(0, u, 0.0)
        case.bcs[0].u_value = u
        oc = orc.OracleCase(case, U=oc.U, p=oc.p, phi=oc.phi)
        st, info = c.piso(1)
        st_o, info_o = oc.piso(1)
        assert st == st_o == 0
        assert _counts(info) == _counts(info_o), (_counts(info), _counts(info_o))
    Ug, pg, phig = c.get_state_numpy()
    _say(f"  transient pipe: relL2 U {_rel(Ug, oc.U):.2e} p {_rel(pg, oc.p):.2e} phi {_rel(phig, oc.phi):.2e}")
    assert _rel(Ug, oc.U) <= TOL_FP64 and _rel(pg, oc.p) <= TOL_FP64 and _rel(phig, oc.phi) <= TOL_FP64


@pytest.mark.parametrize("shape,perm,rcm", [((11, 9, 7), 2, True), ((20, 20, 1), 1, False), ((8, 8, 8), None, False)])
def test_dic_pcg_piso_parity(shape, perm, rcm):
    case = wl.cavity(shape, Re=400.0, dt=0.005, perm_seed=perm, use_rcm=rcm, tol=1e-9, p_precond=wl.PC_DIC)
    _parity(case, 5, what=f"DIC cavity {shape}")


def test_dic_exact_on_chain_and_solve_pressure():
    import torch
    from paper_1207_1571_amd import fvm
    # a 1-D chain with a fixed-p end: tridiagonal SPD, DIC is exact -> 1 iteration
    case = wl.duct((40, 1, 1), lengths=(4.0, 0.1, 0.1), Re=10.0, mode="piso", dt=0.01)
    case = case.with_(p_ctl=wl.SolverCtl(1e-12, precond=wl.PC_DIC))
    rng = np.random.default_rng(3)
    m = case.mesh
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    rhs = rng.normal(size=m.n_cells)
    c = fvm.Case(case)
    pg = torch.zeros(m.n_cells, dtype=torch.float64, device="cuda")
    st, info = c.solve_pressure(torch.from_numpy(gamma).cuda(), torch.from_numpy(rhs).cuda(), pg, 1e-12,
                                precond=wl.PC_DIC)
    assert st == 0 and info["iters"] == 1, info
    oc = orc.OracleCase(case)
    po = np.zeros(m.n_cells)
    oc.solve_pressure(gamma, rhs, po, 1e-12, precond=wl.PC_DIC)
    assert _rel(pg.cpu().numpy(), po) <= 1e-12
    # a 3-D renumbered mesh: same iterations and solution as the oracle
    case = wl.cavity((13, 11, 9), Re=100.0, dt=0.01, perm_seed=5, use_rcm=True, tol=1e-9, p_precond=wl.PC_DIC)
    m = case.mesh
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    rhs = rng.normal(size=m.n_cells); rhs -= rhs.mean()
    c = fvm.Case(case)
    pg = torch.zeros(m.n_cells, dtype=torch.float64, device="cuda")
    st, info = c.solve_pressure(torch.from_numpy(gamma).cuda(), torch.from_numpy(rhs).cuda(), pg, 1e-10,
                                precond=wl.PC_DIC)
    po = np.zeros(m.n_cells)
    st_o, info_o = orc.OracleCase(case).solve_pressure(gamma, rhs, po, 1e-10, precond=wl.PC_DIC)
    _say(f"  DIC solve_pressure iters gpu {info['iters']} oracle {info_o['iters']}")
    assert info["iters"] == info_o["iters"]
    assert _rel(pg.cpu().numpy(), po) <= TOL_FP64


@pytest.mark.parametrize("shape,perm,rcm", [((40, 1, 1), None, False), ((9, 8, 7), 3, True), ((70, 60, 1), 4, False),
                                            ((130, 120, 1), 5, False), ((30, 30, 30), 6, True)])
def test_dic_apply_matches_oracle(shape, perm, rcm):
    """D* and z = M^-1 r of the GPU sweeps against the oracle's row-ordered
    recurrences on the same assembled matrix.  The two larger meshes are
    longer than the sweeps' gate distance (8192 positions), so their later
    waves wait on the gate before polling."""
    import torch
    from paper_1207_1571_amd import fvm
    case = wl.cavity(shape, Re=100.0, dt=0.01, perm_seed=perm, use_rcm=rcm, tol=1e-9, p_precond=wl.PC_DIC)
    m = case.mesh
    Fi = m.n_internal
    rng = np.random.default_rng(7)
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    r = rng.normal(size=m.n_cells)
    pk = np.concatenate([np.full(z, case.bcs[i].p_kind) for i, z in enumerate(m.patch_size)]).astype(np.int32)
    diag, offd, _ = orc.pressure_system(m, gamma, pk, np.zeros(m.n_faces - Fi), pin_cell=case.p_ref_cell,
                                        p_ref=case.p_ref_value)
    ds_o, z_o = orc.dic(m.owner[:Fi].copy(), m.neighbour.copy(), diag, offd, r)
    c = fvm.Case(case)
    zg = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    dg = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    fvm.dic_apply(c, torch.from_numpy(gamma).cuda(), torch.from_numpy(r).cuda(), zg, dg)
    zg, dg = zg.cpu().numpy(), dg.cpu().numpy()
    bad = np.nonzero(~np.isfinite(dg) | (np.abs(dg - ds_o) > 1e-12 * np.abs(ds_o)))[0]
    _say(f"  D*: {bad.size} mismatches; first {bad[:5]} gpu {dg[bad[:5]]} oracle {ds_o[bad[:5]]}")
    assert bad.size == 0
    bad = np.nonzero(~np.isfinite(zg) | (np.abs(zg - z_o) > 1e-10 * np.abs(z_o).max()))[0]
    _say(f"  z: {bad.size} mismatches; first {bad[:5]} gpu {zg[bad[:5]]} oracle {z_o[bad[:5]]}")
    assert bad.size == 0


def _long_range_mesh(n, reach):
    """Cells on a line (unit cubes at x = i + 1/2) with the regular faces
    between neighbours and extra faces of area 0.1 between cells i and i + k
    for k = 2..reach, so a cell has up to `reach` lower and upper neighbours;
    the two end faces form the only patch."""
    own, nei, S, Cf = [], [], [], []
    for i in range(n):
        for k in range(1, reach + 1):
            if i + k < n:
                a = 1.0 if k == 1 else 0.1
                own.append(i); nei.append(i + k)
                S.append((a, 0.0, 0.0)); Cf.append((i + 0.5 + k / 2.0, 0.5, 0.5))
    Fi = len(own)
    own += [0, n - 1]
    S += [(-1.0, 0.0, 0.0), (1.0, 0.0, 0.0)]
    Cf += [(0.0, 0.5, 0.5), (float(n), 0.5, 0.5)]
    C = np.array([(i + 0.5, 0.5, 0.5) for i in range(n)])
    return mg.Mesh(owner=np.array(own, np.int32), neighbour=np.array(nei, np.int32), Sf=np.array(S),
                   Cf=np.array(Cf), C=C, V=np.ones(n), patch_names=["ends"],
                   patch_start=np.array([Fi], np.int32), patch_size=np.array([2], np.int32), shape=(n, 1, 1),
                   lex_of_cell=np.arange(n))


@pytest.mark.parametrize("reach,perm,n", [(6, None, 300), (11, 9, 300), (6, None, 20000), (11, 9, 20000)])
def test_dic_apply_many_dependencies(reach, perm, n):
    """Cells with more dependencies than the 4 register slots (reach 6 in
    natural order: at most 6 per side, the 8-slot variant) or than 8 (reach
    11, permuted: the streaming path); the 20000-cell lines also pass the
    sweeps' gate distance."""
    import torch
    from paper_1207_1571_amd import fvm
    m = _long_range_mesh(n, reach)
    if perm is not None:
        m = mg.random_permutation(m, perm)
    bcs = [wl.PatchBC(wl.FIXED, wl.FIXED)]
    case = wl.CaseSpec(name="long-range", mesh=m, bcs=bcs, nu=0.1, dt=0.01, p_ref_cell=0,
                       p_ctl=wl.SolverCtl(1e-10, precond=wl.PC_DIC), u_ctl=wl.SolverCtl(1e-10))
    Fi = m.n_internal
    rng = np.random.default_rng(8)
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    r = rng.normal(size=m.n_cells)
    pk = np.full(m.n_faces - Fi, wl.FIXED, np.int32)
    diag, offd, _ = orc.pressure_system(m, gamma, pk, np.zeros(m.n_faces - Fi), pin_cell=case.p_ref_cell,
                                        p_ref=case.p_ref_value)
    ds_o, z_o = orc.dic(m.owner[:Fi].copy(), m.neighbour.copy(), diag, offd, r)
    c = fvm.Case(case)
    zg = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    dg = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    fvm.dic_apply(c, torch.from_numpy(gamma).cuda(), torch.from_numpy(r).cuda(), zg, dg)
    zg, dg = zg.cpu().numpy(), dg.cpu().numpy()
    _say(f"  reach {reach}: max |D* diff| {np.abs(dg - ds_o).max():.2e}, max |z diff| {np.abs(zg - z_o).max():.2e}")
    assert np.all(np.isfinite(dg)) and np.all(np.abs(dg - ds_o) <= 1e-12 * np.abs(ds_o))
    assert np.all(np.isfinite(zg)) and np.all(np.abs(zg - z_o) <= 1e-10 * np.abs(z_o).max())


TOL_MIXED = 1e-6


@pytest.mark.parametrize("shape,perm", [((12, 10, 9), 2), ((24, 24, 1), 1)])
def test_mixed_precision_parity_tight(shape, perm):
    """FP32 inner / FP64 refinement against the FP64 oracle, both run to an
    outer normalised residual of 1e-10: agreement within 1e-6."""
    case = wl.cavity(shape, Re=400.0, dt=0.01, perm_seed=perm, tol=1e-10, precision=wl.MIXED)
    _say(f"[mixed] cavity {shape}")
    g = _gpu(case, 5)
    o = _oracle(case, 5)
    assert g["st"] == o["st"] == 0
    _compare(g, o, tol=TOL_MIXED, what="mixed tight")


def test_mixed_precision_error_at_benchmark_tolerance():
    """At the 1e-6 stopping threshold the mixed result is stated, and bounded
    by what the threshold allows (the FP64 path itself differs from the exact
    solution by that much)."""
    case = wl.cavity((16, 16, 16), Re=1000.0, dt=0.001, tol=1e-6, precision=wl.MIXED)
    g = _gpu(case, 5)
    o = _oracle(case, 5)
    eU, ep = _rel(g["U"], o["U"]), _rel(g["p"], o["p"])
    _say(f"  mixed at tol 1e-6: relL2 U {eU:.2e} p {ep:.2e}; p iters gpu {_counts(g['info'])} oracle {_counts(o['info'])}")
    assert eU <= 1e-4 and ep <= 1e-3
    # against the FP64 path at the same stopping threshold the mixed result
    # is within the mixed-precision tolerance: both stop on the same
    # normalised residual, and the FP32 inner work changes only rounding
    f = _gpu(case.with_(precision=wl.FP64), 5)
    eU, ep = _rel(g["U"], f["U"]), _rel(g["p"], f["p"])
    _say(f"  mixed vs FP64 GPU at tol 1e-6: relL2 U {eU:.2e} p {ep:.2e}; iters {_counts(g['info'])} {_counts(f['info'])}")
    assert eU <= TOL_MIXED and ep <= TOL_MIXED


def _giant_cavity(precision, step_kernel):
    """An 8^3 cavity of side 1e12 at Re 100 with dt = 1e-6: the momentum
    diagonal V/dt (about 2e39) lies beyond the FP32 range while the pressure
    system (coefficients about 1e5) does not, so the FP32 inner momentum
    solve of the mixed path breaks down at its first step."""
    from paper_1207_1571_amd import meshgen as mgen
    L = 1e12
    base = wl.cavity((8, 8, 8), Re=100.0, dt=1e-6, tol=1e-10, precision=precision)
    mesh = mgen.box_mesh(8, 8, 8, lengths=(L, L, L))
    assert mesh.patch_names == base.mesh.patch_names
    return base.with_(mesh=mesh, nu=L / 100.0, step_kernel=step_kernel)


@pytest.mark.parametrize("step_kernel", [wl.STEP_AUTO, wl.STEP_LAUNCHED])
def test_mixed_momentum_falls_back_to_fp64(step_kernel):
    """Mixed precision: a momentum component whose FP32 inner solve breaks
    down continues as an FP64 BiCG solve from its current iterate (whole-step
    kernel and launched phases), instead of failing the step: the result
    agrees with the oracle within the mixed tolerance, and the momentum
    solves reach the oracle's residuals."""
    case = _giant_cavity(wl.MIXED, step_kernel)
    v = case.mesh.V[0]
    assert v / case.dt > 3.5e38 and case.mesh.n_cells <= 32768
    _say(f"[fallback] giant cavity, step kernel {step_kernel}")
    g = _gpu(case, 3)
    o = _oracle(case.with_(precision=wl.FP64), 3)
    assert g["st"] == 0 and o["st"] == 0
    for su, so in zip(g["info"]["u"], o["info"]["u"]):
        assert su["status"] == 0 and su["iters"] >= 1
        assert su["res_final"] <= case.u_ctl.tol
    _compare(g, o, tol=TOL_MIXED, what="mixed with FP64 momentum fallback")
    f = _gpu(case.with_(precision=wl.FP64), 3)
    _compare(f, o, what="FP64, same case")


@pytest.mark.timeout(600)
def test_cav200_settings_on_a_64_cube():
    """The 200^3 configuration's settings (lexicographic numbering, Re 1000,
    dt 0.001, Jacobi PCG / PBiCG, tol 1e-6) on 64^3 cells: the z-neighbour
    lies 4096 cells, 16 slices of the sliced-ELL copy, away, so the
    index-free regular slices and the mirrored lower-slot reads cross slices
    as they do at 200^3.  FP64 under the parity protocol (1e-9); the mixed
    path against the oracle with both at an outer tolerance of 1e-10 (1e-6);
    and mixed against FP64 at the configuration's 1e-6 (1e-6)."""
    case = wl.cavity((64, 64, 64), Re=1000.0, dt=0.001, tol=1e-6)
    g, _ = _parity(case, 3, what="64^3 lexicographic, FP64")
    m = _gpu(case.with_(precision=wl.MIXED), 3)
    eU, ep = _rel(m["U"], g["U"]), _rel(m["p"], g["p"])
    _say(f"  mixed vs FP64 at tol 1e-6: relL2 U {eU:.2e} p {ep:.2e}; iters {_counts(m['info'])} {_counts(g['info'])}")
    assert m["st"] == 0 and eU <= TOL_MIXED and ep <= TOL_MIXED
    tight = case.with_(p_ctl=wl.SolverCtl(1e-10), u_ctl=wl.SolverCtl(1e-10), precision=wl.MIXED)
    m = _gpu(tight, 3)
    o = _oracle(tight, 3)
    assert m["st"] == o["st"] == 0
    _compare(m, o, tol=TOL_MIXED, what="64^3 lexicographic, mixed at 1e-10")


def test_mixed_solve_pressure_and_simple():
    import torch
    from paper_1207_1571_amd import fvm
    case = wl.cavity((15, 13, 9), Re=100.0, dt=0.01, perm_seed=6, tol=1e-10, precision=wl.MIXED)
    rng = np.random.default_rng(0)
    m = case.mesh
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    rhs = rng.normal(size=m.n_cells); rhs -= rhs.mean()
    po = np.zeros(m.n_cells)
    orc.OracleCase(case).solve_pressure(gamma, rhs, po, 1e-11)
    c = fvm.Case(case)
    pg = torch.zeros(m.n_cells, dtype=torch.float64, device="cuda")
    st, info = c.solve_pressure(torch.from_numpy(gamma).cuda(), torch.from_numpy(rhs).cuda(), pg, 1e-11)
    _say(f"  mixed solve_pressure: {info}")
    assert st == 0 and info["res_final"] <= 1e-11
    assert _rel(pg.cpu().numpy(), po) <= TOL_MIXED
    sc = wl.duct256((24, 6, 6)).with_(p_ctl=wl.SolverCtl(1e-11, 0.0), u_ctl=wl.SolverCtl(1e-11, 0.0),
                                      precision=wl.MIXED)
    g = _gpu(sc, 8, simple=True, res_tol=0.0)
    o = _oracle(sc, 8, simple=True, res_tol=0.0)
    _compare(g, o, tol=TOL_MIXED, what="mixed SIMPLE")


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 1), (1, 1, 3), (3, 2, 1)])
@pytest.mark.parametrize("variant", ["jacobi", "dic", "mixed", "bicgstab", "amg"])
def test_degenerate_meshes(shape, variant):
    """One cell (no internal face), two cells (one face), a column of three
    and a 3x2 sheet: every solver variant against the oracle, 3 PISO steps.
    Some of these fields are zero analytically (the single internal flux of
    the two-cell cavity must vanish by continuity), so errors are measured
    against the lid's scale where the field itself is smaller: U against the
    lid speed 1, phi against the lid speed times the largest face area, p
    against 1."""
    case = wl.cavity(shape, Re=50.0, dt=0.01, tol=1e-10)
    if variant == "dic":
        case = case.with_(p_ctl=wl.SolverCtl(1e-10, precond=wl.PC_DIC))
    elif variant == "mixed":
        case = case.with_(precision=wl.MIXED)
    elif variant == "bicgstab":
        case = case.with_(u_solver=wl.SOLVER_BICGSTAB)
    _say(f"[degenerate] {shape} {variant}")
    g = _gpu(case.with_(p_ctl=wl.SolverCtl(1e-10, precond=wl.PC_AMG)) if variant == "amg" else case, 3)
    # the oracle's PISO has no AMG: with one level (these meshes) the
    # V-cycle is the exact inverse, so the fields equal the Jacobi oracle's
    # to solver tolerance
    o = _oracle(case, 3)
    assert g["st"] == o["st"] == 0, (g["st"], o["st"])
    if variant not in ("mixed", "amg"):
        assert _counts(g["info"]) == _counts(o["info"]), (_counts(g["info"]), _counts(o["info"]))
    if variant == "amg":
        assert all(s["iters"] <= 1 for s in g["info"]["p"])
    tol = TOL_MIXED if variant in ("mixed", "amg") else TOL_FP64
    smax = float(np.linalg.norm(case.mesh.Sf, axis=1).max())
    for k, floor in (("U", 1.0), ("p", 1.0), ("phi", smax)):
        a, b = g[k], o[k]
        assert np.all(np.isfinite(a))
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), floor)
        assert err <= tol, (k, err)


@pytest.mark.parametrize("precision", [wl.FP64, wl.MIXED])
@pytest.mark.parametrize("shape,perm", [((9, 7, 5), 3), ((32, 32, 1), 1), ((17, 1, 13), None), ((32, 32, 32), 2)])
def test_whole_step_kernel_against_launched_phases_and_oracle(shape, perm, precision):
    """Small cases run whole PISO steps in one workgroup (the default for
    them); the same case with every phase launched over the grid, and the
    oracle, give the same fields: FP64 under the parity protocol (1e-9),
    mixed precision within 1e-6 with both at an outer tolerance of 1e-10.
    32^3 is the largest size that runs whole steps."""
    tol = 1e-9 if precision == wl.FP64 else 1e-10
    case = wl.cavity(shape, Re=300.0, dt=0.01, perm_seed=perm, tol=tol, precision=precision)
    _say(f"[whole-step] {shape} precision {precision}")
    solo = _gpu(case, 4)
    launched = _gpu(case.with_(step_kernel=wl.STEP_LAUNCHED), 4)
    assert solo["st"] == launched["st"] == 0
    if precision == wl.FP64:
        _say(f"  iters whole-step {_counts(solo['info'])} launched {_counts(launched['info'])}")
        _compare(solo, launched, what="whole-step vs launched")
        _parity(case, 4, what="whole-step vs oracle")
    else:
        o = _oracle(case, 4)
        _compare(solo, o, tol=TOL_MIXED, what="whole-step mixed vs oracle")
        _compare(solo, launched, tol=TOL_MIXED, what="whole-step mixed vs launched")
