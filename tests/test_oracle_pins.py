"""Pins of the FP64 CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: a closed
form (linear fields), an invariant (symmetry, M-matrix, divergence-free
flux, mass balance, permutation equivariance), a special case that reduces
to a textbook result (BiCG == CG on symmetric systems, exact DIC on
tridiagonal systems), a library routine on tiny problems (dense
numpy.linalg.solve, and a dense matrix-style restatement of a full step),
or an analytic flow (plane and square-duct Poiseuille).
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1207_1571_amd import meshgen as mg
from paper_1207_1571_amd import workloads as wl
from tests import dense_ref

FIXED, ZERO_GRAD, EMPTY = 0, 1, 2


def _graded_mesh(seed=0, shape=(5, 4, 3), perm=True):
    rng = np.random.default_rng(seed)
    gr = tuple(rng.uniform(0.5, 2.0, n) for n in shape)
    m = mg.box_mesh(*shape, lengths=(1.3, 0.9, 0.7), grading=gr)
    return mg.random_permutation(m, seed + 1) if perm else m


# --------------------------------------------------------------------- T3

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_T3_gauss_gradient_exact_for_linear_field(seed):
    m = _graded_mesh(seed)
    a = np.array([1.7, -0.4, 2.3]); c0 = 0.9
    phi = m.C @ a + c0
    Fi = m.n_internal
    bk = np.full(m.n_faces - Fi, FIXED, np.int32)
    bv = m.Cf[Fi:] @ a + c0
    g = orc.grad(m, phi, bk, bv)
    assert np.abs(g - a).max() <= 1e-12 * np.abs(a).max()


def test_T3_gradient_of_constant_is_zero_with_zero_gradient_bcs_jittered():
    m = mg.box_mesh(4, 4, 4, jitter=0.25, seed=5)
    phi = np.full(m.n_cells, 3.25)
    bk = np.full(m.n_faces - m.n_internal, ZERO_GRAD, np.int32)
    g = orc.grad(m, phi, bk, np.zeros(m.n_faces - m.n_internal))
    assert np.abs(g).max() <= 1e-12


# --------------------------------------------------------------------- T4

@pytest.mark.parametrize("seed", [0, 3])
def test_T4_laplacian_of_linear_field_vanishes_on_orthogonal_mesh(seed):
    m = _graded_mesh(seed, shape=(6, 5, 4))
    a = np.array([0.3, -1.1, 0.8]); gam0 = 2.5
    phi = m.C @ a - 0.2
    Fi = m.n_internal
    pk = np.full(m.n_faces - Fi, FIXED, np.int32)
    pv = m.Cf[Fi:] @ a - 0.2
    diag, offd, b = orc.pressure_system(m, np.full(m.n_faces, gam0), pk, pv)
    Ap = orc.amul(m.owner[:Fi].copy(), m.neighbour, diag, offd, offd, phi)
    scale = np.abs(diag * phi).max()
    assert np.abs(Ap - b).max() <= 1e-13 * scale


# --------------------------------------------------------------------- T5

def _one_step_state(case, steps=3):
    oc = orc.OracleCase(case)
    st, _ = oc.piso(steps)
    assert st == 0
    return oc


def test_T5_pressure_matrix_symmetric_diagonally_dominant_M_matrix():
    case = wl.cavity((6, 5, 4), Re=50.0, dt=0.01, perm_seed=4, tol=1e-10)
    oc = _one_step_state(case)
    m = case.mesh
    Fi = m.n_internal
    rng = np.random.default_rng(0)
    rAU = rng.uniform(0.5, 2.0, m.n_cells)
    w, dl, k, _ = orc.face_coeffs(m)
    gam = np.concatenate([w * rAU[m.owner[:Fi]] + (1 - w) * rAU[m.neighbour], rAU[m.owner[Fi:]]])
    pk = np.array([case.bcs[p].p_kind for p in range(len(case.bcs))])
    pkf = np.concatenate([np.full(z, pk[i]) for i, z in enumerate(m.patch_size)]).astype(np.int32)
    diag, offd, b = orc.pressure_system(m, gam, pkf, np.zeros(m.n_faces - Fi), phiH=oc.phi,
                                        pin_cell=case.p_ref_cell)
    N = m.n_cells
    A = np.zeros((N, N)); A[np.arange(N), np.arange(N)] = diag
    A[m.owner[:Fi], m.neighbour] = offd; A[m.neighbour, m.owner[:Fi]] = offd
    assert np.array_equal(A, A.T)
    assert np.all(diag > 0) and np.all(offd <= 0)
    off_sum = np.abs(A).sum(axis=1) - diag
    assert np.all(diag >= off_sum * (1 - 1e-15))
    assert diag[case.p_ref_cell] > off_sum[case.p_ref_cell] * 1.5
    assert np.all(np.linalg.eigvalsh(A) > 0)


# --------------------------------------------------------------------- T6

def _div(m, phi):
    d = np.zeros(m.n_cells)
    np.add.at(d, m.owner, phi)
    np.add.at(d, m.neighbour, -phi[: m.n_internal])
    return d


def test_T6_corrected_flux_divergence_free_and_walls_zero():
    case = wl.cavity((8, 8, 4), Re=100.0, dt=0.01, perm_seed=3, tol=1e-13)
    oc = orc.OracleCase(case)
    st, info = oc.piso(2)
    assert st == 0
    m = case.mesh
    div = _div(m, oc.phi)
    scale = np.abs(oc.phi).max()
    assert np.abs(div).max() <= 1e-10 * scale
    assert np.all(oc.phi[m.n_internal:] == 0.0)


# --------------------------------------------------------------------- T7

def _tiny_cases():
    out = []
    out.append(wl.cavity((2, 2, 1), Re=20.0, dt=0.05, tol=1e-14))
    out.append(wl.cavity((3, 3, 1), Re=20.0, dt=0.05, perm_seed=7, tol=1e-14))
    out.append(wl.cavity((4, 4, 4), Re=20.0, dt=0.05, tol=1e-14))
    out.append(wl.cavity((3, 3, 3), Re=20.0, dt=0.05, perm_seed=9, jitter=0.2, jitter_seed=4, tol=1e-14))
    d = wl.duct((5, 3, 3), lengths=(2.0, 1.0, 1.0), Re=10.0, jitter=0.15, jitter_seed=2, mode="piso", dt=0.05)
    out.append(d.with_(p_ctl=wl.SolverCtl(1e-14), u_ctl=wl.SolverCtl(1e-14)))
    return out


def _warm_state(case, rng):
    """A non-trivial but boundary-consistent state: random U, p, and the
    flux of U (so the momentum matrix has non-zero convection)."""
    N = case.mesh.n_cells
    U = rng.normal(size=(N, 3)) * 0.3
    if case.mesh.shape[2] == 1:
        U[:, 2] = 0.0
    p = rng.normal(size=N)
    oc = orc.OracleCase(case, U=U, p=p)
    return oc


@pytest.mark.parametrize("ci", range(5))
def test_T7_krylov_vs_dense_solve(ci):
    case = _tiny_cases()[ci]
    rng = np.random.default_rng(ci)
    oc = _warm_state(case, rng)
    m = case.mesh
    Fi = m.n_internal
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    diag, up, lo, src = orc.momentum_system(m, case.bcs, case.nu, case.dt, 0, oc.phi, oc.U, oc.U)
    N = m.n_cells
    A = np.zeros((N, N)); A[np.arange(N), np.arange(N)] = diag
    A[own, nei] = up; A[nei, own] = lo
    b = src[:, 0] + rng.normal(size=N)
    x, info = orc.pbicg(own, nei, diag, up, lo, b, np.zeros(N), 1e-15, max_iter=500)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    # symmetric pressure-type system, Jacobi and DIC
    g = rng.uniform(0.5, 2.0, m.n_faces)
    pk = np.full(m.n_faces - Fi, ZERO_GRAD, np.int32)
    pd, po, pb = orc.pressure_system(m, g, pk, np.zeros(m.n_faces - Fi), pin_cell=0, p_ref=0.0)
    Ap = np.zeros((N, N)); Ap[np.arange(N), np.arange(N)] = pd
    Ap[own, nei] = po; Ap[nei, own] = po
    bp = rng.normal(size=N)
    xd = np.linalg.solve(Ap, bp)
    for pc in (0, 1):
        x, info = orc.pcg(own, nei, pd, po, bp, np.zeros(N), 1e-15, max_iter=500, precond=pc)
        assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd), (pc, info)


@pytest.mark.parametrize("ci", range(5))
def test_T7_full_piso_step_vs_dense_restatement(ci):
    case = _tiny_cases()[ci]
    rng = np.random.default_rng(10 + ci)
    oc = _warm_state(case, rng)
    U0, p0, phi0 = oc.U.copy(), oc.p.copy(), oc.phi.copy()
    st, info = oc.piso(1)
    assert st == 0, info
    Ud, pd, phid = dense_ref.piso_step(case.mesh, case.bcs, case.nu, case.dt, case.n_corr, case.p_ref_cell,
                                       case.p_ref_value, U0, p0, phi0)
    assert np.linalg.norm(oc.U - Ud) <= 1e-10 * np.linalg.norm(Ud)
    assert np.linalg.norm(oc.p - pd) <= 1e-10 * max(np.linalg.norm(pd), 1e-30)
    assert np.linalg.norm(oc.phi - phid) <= 1e-10 * np.linalg.norm(phid)


@pytest.mark.parametrize("ci", [3, 4])
def test_T7_simple_iteration_vs_dense_restatement(ci):
    case = _tiny_cases()[ci].with_(alpha_u=0.7, alpha_p=0.3, mode="simple")
    rng = np.random.default_rng(20 + ci)
    oc = _warm_state(case, rng)
    U0, p0, phi0 = oc.U.copy(), oc.p.copy(), oc.phi.copy()
    st, it, info = oc.simple(1, 0.0)
    assert st == 0 and it == 1
    Ud, pd, phid = dense_ref.simple_iteration(case.mesh, case.bcs, case.nu, 0.7, 0.3, case.p_ref_cell,
                                              case.p_ref_value, U0, p0, phi0)
    assert np.linalg.norm(oc.U - Ud) <= 1e-10 * np.linalg.norm(Ud)
    assert np.linalg.norm(oc.p - pd) <= 1e-10 * np.linalg.norm(pd)
    assert np.linalg.norm(oc.phi - phid) <= 1e-10 * np.linalg.norm(phid)


# --------------------------------------------------------------------- T8

def _developed_profile(case, oc, x0, x1):
    m = case.mesh
    sel = (m.C[:, 0] >= x0) & (m.C[:, 0] <= x1)
    return sel


def _run_simple(case, max_iters=4000, res_tol=1e-8):
    case = case.with_(p_ctl=wl.SolverCtl(res_tol * 1e-2, 0.05), u_ctl=wl.SolverCtl(res_tol * 1e-2, 0.1))
    oc = orc.OracleCase(case)
    st, it, info = oc.simple(max_iters, res_tol)
    assert st >= 0
    assert it < max_iters, info
    return oc


def test_T8_plane_poiseuille_second_order():
    errs = []
    for ny in (8, 16, 32):
        case = wl.duct((4 * ny, ny, 1), lengths=(4.0, 1.0, 1.0 / ny), Re=10.0)
        oc = _run_simple(case)
        m = case.mesh
        sel = _developed_profile(case, oc, 3.0, 3.5)
        eta = m.C[sel, 1]
        ua = 6.0 * eta * (1.0 - eta)           # mean velocity 1 (mass conservation)
        errs.append(np.abs(oc.U[sel, 0] - ua).max())
    assert errs[-1] < 2e-3
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def _duct_series(y, z, n_terms=40):
    """Fully developed laminar flow in the square duct |y|,|z| <= 1/2 under
    a unit pressure gradient, by the classical Fourier series (rectangular
    duct, e.g. White, Viscous Fluid Flow, ch. 3), normalised to unit mean."""
    a = b = 0.5
    u = np.zeros_like(y)
    for i in range(1, 2 * n_terms, 2):
        u += ((-1) ** ((i - 1) // 2) * (1 - np.cosh(i * math.pi * z / (2 * a)) / math.cosh(i * math.pi * b / (2 * a)))
              * np.cos(i * math.pi * y / (2 * a)) / i ** 3)
    # mean over the section of the same series
    mean = 0.0
    for i in range(1, 2 * n_terms, 2):
        mean += (1.0 / i ** 4) * (1 - (2 * a / (i * math.pi * b)) * math.tanh(i * math.pi * b / (2 * a)))
    mean *= 2.0 / math.pi
    return u / mean


def test_T8_square_duct_poiseuille_series():
    case = wl.duct((40, 10, 10), lengths=(4.0, 1.0, 1.0), Re=5.0)
    oc = _run_simple(case, res_tol=1e-7)
    m = case.mesh
    sel = (m.C[:, 0] >= 3.0) & (m.C[:, 0] <= 3.5)
    y = m.C[sel, 1] - 0.5; z = m.C[sel, 2] - 0.5
    ua = _duct_series(y, z)
    assert np.abs(oc.U[sel, 0] - ua).max() <= 0.05 * ua.max()
    # mass balance (T15)
    ps, zs = case.mesh.patch("xmin"), case.mesh.patch("xmax")
    q_in = oc.phi[ps[0]:ps[0] + ps[1]].sum(); q_out = oc.phi[zs[0]:zs[0] + zs[1]].sum()
    assert abs(q_in + q_out) <= 1e-6 * abs(q_in)


# --------------------------------------------------------------------- T9

def test_T9_reference_cell_holds_reference_pressure():
    case = wl.cavity((6, 6, 1), Re=100.0, dt=0.01, perm_seed=2, tol=1e-12).with_(p_ref_value=3.0)
    oc = orc.OracleCase(case)
    st, _ = oc.piso(3)
    assert st == 0
    assert abs(oc.p[case.p_ref_cell] - 3.0) <= 1e-9 * (np.abs(oc.p - 3.0).max() + 1.0)


# --------------------------------------------------------------------- T10

def test_T10_zero_lid_velocity_stays_exactly_at_rest():
    case = wl.cavity((5, 4, 3), Re=100.0, dt=0.01, tol=1e-8, u_lid=0.0).with_(nu=0.01)
    oc = orc.OracleCase(case)
    st, info = oc.piso(3)
    assert st == 0
    assert np.all(oc.U == 0.0) and np.all(oc.p == 0.0) and np.all(oc.phi == 0.0)
    assert all(s["iters"] == 0 for s in info["u"]) and all(s["iters"] == 0 for s in info["p"])


# --------------------------------------------------------------------- T11

def test_T11_permutation_equivariance():
    base = wl.cavity((10, 10, 1), Re=100.0, dt=0.005, tol=1e-13)
    perm = wl.cavity((10, 10, 1), Re=100.0, dt=0.005, tol=1e-13, perm_seed=1)
    a = orc.OracleCase(base); b = orc.OracleCase(perm)
    assert a.piso(10)[0] == 0 and b.piso(10)[0] == 0
    lex = perm.mesh.lex_of_cell
    Ub = np.empty_like(b.U); Ub[lex] = b.U
    pb = np.empty_like(b.p); pb[lex] = b.p
    assert np.abs(Ub - a.U).max() <= 1e-11 * np.abs(a.U).max()
    assert np.abs(pb - a.p).max() <= 1e-11 * np.abs(a.p).max()


def test_T11_face_order_and_orientation_invariance():
    case = wl.cavity((6, 5, 3), Re=100.0, dt=0.01, perm_seed=5, tol=1e-13)
    sh = mg.shuffle_faces(case.mesh, seed=9)
    a = orc.OracleCase(case); b = orc.OracleCase(case.with_(mesh=sh))
    assert a.piso(4)[0] == 0 and b.piso(4)[0] == 0
    assert np.abs(a.U - b.U).max() <= 1e-11 * np.abs(a.U).max()
    assert np.abs(a.p - b.p).max() <= 1e-11 * np.abs(a.p).max()


# --------------------------------------------------------------------- T12

def test_T12_bicg_equals_cg_on_symmetric_jacobi():
    m = mg.random_permutation(mg.box_mesh(6, 6, 3), 3)
    Fi = m.n_internal
    rng = np.random.default_rng(1)
    g = rng.uniform(0.5, 2.0, m.n_faces)
    pd, po, _ = orc.pressure_system(m, g, np.full(m.n_faces - Fi, FIXED, np.int32), np.zeros(m.n_faces - Fi))
    b = rng.normal(size=m.n_cells)
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    for k in (1, 2, 5, 9):
        x1, _ = orc.pcg(own, nei, pd, po, b, np.zeros(m.n_cells), 0.0, max_iter=k)
        x2, _ = orc.pbicg(own, nei, pd, po, po, b, np.zeros(m.n_cells), 0.0, max_iter=k)
        assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()


# --------------------------------------------------------------------- T17

@pytest.mark.parametrize("ci", range(5))
def test_T17_bicgstab_vs_dense_solve(ci):
    """PBiCGStab (Barrett Sec. 2.3.8, Jacobi) on the non-symmetric momentum
    matrix against a dense solve."""
    case = _tiny_cases()[ci]
    rng = np.random.default_rng(40 + ci)
    oc = _warm_state(case, rng)
    m = case.mesh
    Fi = m.n_internal
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    diag, up, lo, src = orc.momentum_system(m, case.bcs, case.nu, case.dt, 0, oc.phi, oc.U, oc.U)
    N = m.n_cells
    A = np.zeros((N, N)); A[np.arange(N), np.arange(N)] = diag
    A[own, nei] = up; A[nei, own] = lo
    b = src[:, 0] + rng.normal(size=N)
    x, info = orc.pbicgstab(own, nei, diag, up, lo, b, np.zeros(N), 1e-15, max_iter=500)
    assert info["status"] == 0, info
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_T17_bicgstab_terminates_with_two_eigenvalues():
    """With Jacobi, M^-1 A = B for A = D B (B unit-diagonal); B made of
    identical 2x2 non-symmetric blocks has two distinct eigenvalues, so the
    BiCG polynomial underlying BiCGStab terminates in at most two steps; a
    diagonal system is solved in the first half step."""
    nb = 20
    N = 2 * nb
    rng = np.random.default_rng(5)
    D = rng.uniform(1.0, 3.0, N)
    own = np.arange(0, N, 2, dtype=np.int32)
    nei = own + 1
    a, c = 0.4, -0.7          # block [[1, a], [c, 1]]: eigenvalues 1 +- sqrt(a c) (complex pair)
    up = D[own] * a
    lo = D[nei] * c
    A = np.diag(D); A[own, nei] = up; A[nei, own] = lo
    b = rng.normal(size=N)
    x, info = orc.pbicgstab(own, nei, D, up, lo, b, np.zeros(N), 1e-13, max_iter=50)
    assert info["status"] == 0 and info["iters"] <= 2, info
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-12 * np.linalg.norm(x)
    e = np.zeros(0, np.int32)
    x, info = orc.pbicgstab(e, e, D, np.zeros(0), np.zeros(0), b, np.zeros(N), 1e-14, max_iter=50)
    assert info["status"] == 0 and info["iters"] == 1, info
    assert np.abs(x - b / D).max() <= 1e-15 * np.abs(b / D).max()


@pytest.mark.parametrize("ci", range(5))
def test_T17_piso_step_with_bicgstab_vs_dense_restatement(ci):
    case = _tiny_cases()[ci].with_(u_solver=wl.SOLVER_BICGSTAB)
    rng = np.random.default_rng(10 + ci)
    oc = _warm_state(case, rng)
    U0, p0, phi0 = oc.U.copy(), oc.p.copy(), oc.phi.copy()
    st, info = oc.piso(1)
    assert st == 0, info
    Ud, pd, phid = dense_ref.piso_step(case.mesh, case.bcs, case.nu, case.dt, case.n_corr, case.p_ref_cell,
                                       case.p_ref_value, U0, p0, phi0)
    assert np.linalg.norm(oc.U - Ud) <= 1e-10 * np.linalg.norm(Ud)
    assert np.linalg.norm(oc.p - pd) <= 1e-10 * max(np.linalg.norm(pd), 1e-30)


# --------------------------------------------------------------------- T13

def test_T13_dic_exact_on_tridiagonal_and_jacobi_on_diagonal():
    m = mg.random_permutation(mg.box_mesh(30, 1, 1), 0)   # a chain, not in chain order
    m = mg.box_mesh(30, 1, 1)
    Fi = m.n_internal
    rng = np.random.default_rng(2)
    g = rng.uniform(0.5, 2.0, m.n_faces)
    pd, po, _ = orc.pressure_system(m, g, np.full(m.n_faces - Fi, FIXED, np.int32), np.zeros(m.n_faces - Fi))
    b = rng.normal(size=m.n_cells)
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    x, info = orc.pcg(own, nei, pd, po, b, np.zeros(m.n_cells), 1e-13, precond=1)
    assert info["iters"] == 1 and info["status"] == 0
    # Jacobi on a diagonal system (no faces)
    d = rng.uniform(1.0, 3.0, 17)
    e = np.zeros(0, np.int32)
    x, info = orc.pcg(e, e, d, np.zeros(0), rng.normal(size=17), np.zeros(17), 1e-14, precond=0)
    assert info["iters"] == 1


def test_T13_dic_reproduces_A_on_its_pattern():
    """M = (D*+L) D*^-1 (D*+U) equals A on the diagonal and on every face
    pair (the defining property of the diagonal-only incomplete
    factorisation), and dic applies M^-1."""
    m = mg.random_permutation(mg.box_mesh(5, 4, 3), 8)
    Fi = m.n_internal
    rng = np.random.default_rng(3)
    g = rng.uniform(0.5, 2.0, m.n_faces)
    pd, po, _ = orc.pressure_system(m, g, np.full(m.n_faces - Fi, FIXED, np.int32), np.zeros(m.n_faces - Fi))
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    N = m.n_cells
    r = rng.normal(size=N)
    dstar, z = orc.dic(own, nei, pd, po, r)
    L = np.zeros((N, N))
    hi, lo = np.maximum(own, nei), np.minimum(own, nei)
    L[hi, lo] = po
    Dm = np.diag(dstar)
    M = (Dm + L) @ np.diag(1 / dstar) @ (Dm + L.T)
    A = np.diag(pd); A[own, nei] = po; A[nei, own] = po
    mask = A != 0
    assert np.abs((M - A)[mask]).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(M @ z - r).max() <= 1e-12 * np.abs(r).max()


# --------------------------------------------------------------------- T14

def test_T14_cg_energy_norm_error_monotone():
    m = mg.random_permutation(mg.box_mesh(7, 6, 5), 4)
    Fi = m.n_internal
    rng = np.random.default_rng(5)
    g = rng.uniform(0.2, 3.0, m.n_faces)
    pd, po, _ = orc.pressure_system(m, g, np.full(m.n_faces - Fi, FIXED, np.int32), np.zeros(m.n_faces - Fi))
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    N = m.n_cells
    A = np.diag(pd); A[own, nei] = po; A[nei, own] = po
    b = rng.normal(size=N)
    xs = np.linalg.solve(A, b)
    for pc in (0, 1):
        e0 = math.sqrt(xs @ A @ xs)
        prev = e0
        for k in range(1, 60):
            x, _ = orc.pcg(own, nei, pd, po, b, np.zeros(N), 0.0, max_iter=k, precond=pc)
            e = x - xs
            en = math.sqrt(e @ A @ e)
            if en < 1e-9 * e0:          # rounding floor reached
                break
            assert en <= prev * (1 + 1e-12)
            prev = en
        assert en < 1e-9 * e0


# --------------------------------------------------------------------- T16

def test_T16_restart_is_bitwise():
    case = wl.cavity((8, 8, 1), Re=100.0, dt=0.005, perm_seed=1, tol=1e-8)
    a = orc.OracleCase(case)
    a.piso(10)
    b = orc.OracleCase(case)
    b.piso(5)
    c = orc.OracleCase(case, U=b.U, p=b.p, phi=b.phi)
    c.piso(5)
    assert np.array_equal(a.U, c.U) and np.array_equal(a.p, c.p) and np.array_equal(a.phi, c.phi)


# --------------------------------------------------------------------- status codes

def test_breakdown_and_maxiter_statuses():
    case = wl.cavity((6, 6, 1), Re=100.0, dt=0.005, tol=1e-8).with_(p_ctl=wl.SolverCtl(0.0, max_iter=5))
    oc = orc.OracleCase(case)
    st, info = oc.piso(1)
    assert st == 1 and info["p"][0]["iters"] == 5 and info["p"][0]["status"] == 1
    m = case.mesh
    Fi = m.n_internal
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    d = np.ones(m.n_cells); o = np.zeros(Fi)
    b = np.ones(m.n_cells); b[3] = np.nan
    _, info = orc.pcg(own, nei, d, o, b, np.zeros(m.n_cells), 1e-8)
    assert info["status"] == -3


# --------------------------------------------------------------------- O4 convection

def _per_face_patches(m):
    """The same mesh with every boundary face in a patch of its own, so that
    each can carry its own boundary value."""
    import dataclasses
    Fi, F = m.n_internal, m.n_faces
    return dataclasses.replace(m, patch_names=[f"b{f}" for f in range(Fi, F)],
                               patch_start=np.arange(Fi, F, dtype=np.int32),
                               patch_size=np.ones(F - Fi, np.int32))


def _convection_residual(m, bcs, u0, convection, phi_cell):
    """(A phi - b)_P for component 0 of the convection-only momentum system
    (nu = 0, steady) built from the uniform flux F_f = S_f . u0."""
    Fi = m.n_internal
    F = m.Sf @ u0
    diag, up, lo, src = orc.momentum_system(m, bcs, 0.0, 0.0, convection, F)
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    Ap = orc.amul(own, nei, diag, up, lo, phi_cell)
    scale = np.abs(diag * phi_cell).max() + np.abs(src[:, 0]).max()
    return Ap - src[:, 0], scale


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_O4_central_convection_of_linear_field_is_exact(seed):
    """Linear (central) convection, no diffusion, uniform velocity u0:
    Gauss's theorem gives sum_f s F_f phi_f = V (u0 . a) for phi = a.x + c,
    and linear interpolation reproduces a linear field at the face centre of
    an orthogonal (graded, renumbered) box.  Every boundary face is FIXED at
    the field's value there, except a random half that is ZERO_GRAD, whose
    faces carry the owner value: they add F_b (phi_P - phi(C_b)) to the
    identity.  A sign flip of the flux, w swapped with 1 - w on a graded
    mesh, or a dropped boundary term -F_b U_b breaks it."""
    rng = np.random.default_rng(40 + seed)
    m = _per_face_patches(_graded_mesh(seed, shape=(6, 5, 4)))
    Fi, F = m.n_internal, m.n_faces
    a = rng.normal(size=3); c0 = rng.normal(); u0 = rng.normal(size=3)
    phi_cell = m.C @ a + c0
    phi_b = m.Cf[Fi:] @ a + c0
    zg = rng.random(F - Fi) < 0.5
    bcs = [wl.PatchBC(ZERO_GRAD if zg[b] else FIXED, ZERO_GRAD, (float(phi_b[b]), 0.0, 0.0)) for b in range(F - Fi)]
    res, scale = _convection_residual(m, bcs, u0, 0, phi_cell)
    expect = m.V * (u0 @ a)
    Fb = m.Sf[Fi:] @ u0
    zg_term = np.where(zg, Fb * (phi_cell[m.owner[Fi:]] - phi_b), 0.0)
    np.add.at(expect, m.owner[Fi:], zg_term)
    assert np.abs(res - expect).max() <= 1e-13 * scale


@pytest.mark.parametrize("u0", [(0.7, -1.3, 0.4), (-0.2, 0.9, -1.1)])
def test_O4_upwind_convection_of_linear_field_on_uniform_box(u0):
    """Upwind convection on a uniform box: each interior cell takes, per
    axis, F (phi_P - phi_upstream) = h^2 u (a h), so sum_f s F_f phi_up =
    V (u0 . a) whatever the flow direction.  Cells touching the boundary
    see the FIXED face value half a cell away and are left out."""
    u0 = np.array(u0)
    m = _per_face_patches(mg.random_permutation(mg.box_mesh(6, 5, 4, lengths=(1.2, 1.0, 0.8)), 6))
    Fi, F = m.n_internal, m.n_faces
    a = np.array([0.8, -0.5, 1.9]); c0 = 0.3
    phi_cell = m.C @ a + c0
    phi_b = m.Cf[Fi:] @ a + c0
    bcs = [wl.PatchBC(FIXED, ZERO_GRAD, (float(phi_b[b]), 0.0, 0.0)) for b in range(F - Fi)]
    res, scale = _convection_residual(m, bcs, u0, 1, phi_cell)
    interior = np.ones(m.n_cells, bool)
    interior[m.owner[Fi:]] = False
    assert interior.sum() == 4 * 3 * 2
    expect = m.V * (u0 @ a)
    assert np.abs(res - expect)[interior].max() <= 1e-13 * scale
    # and the boundary cells do differ (the upwind face value is not exact there)
    assert np.abs(res - expect)[~interior].max() > 1e-6 * scale


def test_O4_convection_matrix_entries_hand_worked():
    """Two cells of a 2x1x1 box (unit cells, so w = 1/2), flux F = S.u0 with
    u0 = (2, 0, 0) and nu = 0.5: the internal face has |S| = 1 and delta = 1,
    F = 2, so a_PN = F (1 - w) - nu delta = 0.5, a_NP = -F w - nu delta =
    -1.5; with every boundary face a no-slip wall (FIXED 0, F_b = 0 apart
    from the x-faces: F_b = -2 in at x = 0 and +2 out at x = 2, each with
    delta_b = 2 on a unit cell) the diagonals are a_PP = F w + nu delta +
    nu (4 side faces x 2 + x-face 2) = 1 + 0.5 + 5 = 6.5 and a_NN =
    -F (1 - w) + nu delta + 5 = -1 + 0.5 + 5 = 4.5; a lid value
    U_b = (3, 0, 0) on the x = 0 face adds (nu delta_b - F_b) U_b =
    (1 + 2) 3 = 9 to b_P."""
    m = _per_face_patches(mg.box_mesh(2, 1, 1, lengths=(2.0, 1.0, 1.0)))
    Fi, F = m.n_internal, m.n_faces
    assert Fi == 1
    bcs = []
    for b in range(F - Fi):
        f = Fi + b
        on_x0 = m.Cf[f, 0] == 0.0
        bcs.append(wl.PatchBC(FIXED, ZERO_GRAD, (3.0 if on_x0 else 0.0, 0.0, 0.0)))
    phi = m.Sf @ np.array([2.0, 0.0, 0.0])
    diag, up, lo, src = orc.momentum_system(m, bcs, 0.5, 0.0, 0, phi)
    P = int(m.owner[0]); Q = int(m.neighbour[0])
    assert abs(m.C[P, 0] - 0.5) < 1e-15 and abs(m.C[Q, 0] - 1.5) < 1e-15
    assert up[0] == pytest.approx(0.5, abs=1e-14)
    assert lo[0] == pytest.approx(-1.5, abs=1e-14)
    assert diag[P] == pytest.approx(6.5, abs=1e-14)
    assert diag[Q] == pytest.approx(4.5, abs=1e-14)
    assert src[P, 0] == pytest.approx(9.0, abs=1e-14) and src[Q, 0] == 0.0
    assert np.all(src[:, 1:] == 0.0)


# --------------------------------------------------------------------- O12 normaliser

def test_O12_normalised_residual_hand_worked():
    """Three cells in a chain, a non-symmetric matrix
        A = [[2, -1, 0], [-0.5, 4, -2], [0, -1, 3]]
    (upper = A(own, nei) = (-1, -2), lower = A(nei, own) = (-0.5, -1)),
    x = (1, 2, 3), b = (1, 1, 1).  By hand: xbar = 2, A 1 = (1, 1.5, 2),
    A x = (0, 1.5, 7), so
        n_f = |0-2| + |1.5-3| + |7-4|  +  |1-2| + |1-3| + |1-4| = 6.5 + 6 = 12.5
        sum |b - A x| = 1 + 0.5 + 6 = 7.5,  nres = 7.5 / 12.5 = 0.6."""
    own = np.array([0, 1], np.int32); nei = np.array([1, 2], np.int32)
    diag = np.array([2.0, 4.0, 3.0]); up = np.array([-1.0, -2.0]); lo = np.array([-0.5, -1.0])
    b = np.ones(3); x = np.array([1.0, 2.0, 3.0])
    assert orc.nres(own, nei, diag, up, lo, b, x) == pytest.approx(0.6, rel=1e-15)
    # upper and lower swapped is A^T, another value: A^T x = (1, 4, 5), A^T 1 = (1.5, 2, 1),
    #   n_f = |1-3| + |4-4| + |5-2|  +  |1-3| + |1-4| + |1-2| = 5 + 6 = 11, sum|b - A^T x| = 0 + 3 + 4 = 7
    assert orc.nres(own, nei, diag, lo, up, b, x) == pytest.approx(7.0 / 11.0, rel=1e-15)
    # a solve reports this value as its initial residual and stops before
    # its first iteration when it is within the tolerance
    _, info = orc.pbicg(own, nei, diag, up, lo, b, x, 0.61)
    assert info["iters"] == 0 and info["res_initial"] == pytest.approx(0.6, rel=1e-15)
    _, info = orc.pbicg(own, nei, diag, up, lo, b, x, 0.59)
    assert info["iters"] >= 1 and info["res_initial"] == pytest.approx(0.6, rel=1e-15)
    # relative tolerance: stop when nres <= rel_tol * nres0
    _, info = orc.pbicg(own, nei, diag, up, lo, b, x, 0.0, rel_tol=0.5)
    assert info["iters"] >= 1 and info["res_final"] <= 0.3 + 1e-15


def test_O12_normaliser_is_scale_and_shift_invariant():
    """n_f makes the residual independent of the level of x on a singular
    (zero row sum) system: for A 1 = 0 the normaliser is sum|A x| + sum|b|,
    and nres(x + k 1) = nres(x) for every k.  Scaling A, b together leaves
    nres unchanged."""
    m = mg.box_mesh(5, 4, 1)
    Fi = m.n_internal
    own, nei = m.owner[:Fi].copy(), m.neighbour.copy()
    rng = np.random.default_rng(3)
    g = rng.uniform(0.5, 2.0, Fi)
    diag = np.zeros(m.n_cells)
    np.add.at(diag, own, g); np.add.at(diag, nei, g)
    off = -g
    x = rng.normal(size=m.n_cells)
    b = rng.normal(size=m.n_cells); b -= b.mean()
    r0 = orc.nres(own, nei, diag, off, off, b, x)
    Ax = orc.amul(own, nei, diag, off, off, x)
    assert r0 == pytest.approx(np.abs(b - Ax).sum() / (np.abs(Ax).sum() + np.abs(b).sum()), rel=1e-13)
    assert orc.nres(own, nei, diag, off, off, b, x + 7.5) == pytest.approx(r0, rel=1e-11)
    assert orc.nres(own, nei, 3 * diag, 3 * off, 3 * off, 3 * b, x) == pytest.approx(r0, rel=1e-13)


def _couette_startup(n, nu, dt, permute=None):
    """Fluid at rest between a wall at y = 0 and a wall at y = 1 that starts
    moving with U = (1, 0, 0): one cell across x and z, whose faces take no
    part (EMPTY), so the PISO step reduces to the time-implicit diffusion of
    u_x and the pressure stays at its reference level."""
    m = mg.box_mesh(1, n, 1, lengths=(1.0 / n, 1.0, 1.0 / n))
    if permute is not None:
        m = mg.random_permutation(m, permute)
    bcs = []
    for side in m.patch_names:
        if side == "ymin":
            bcs.append(wl.PatchBC(wl.FIXED, wl.ZERO_GRAD))
        elif side == "ymax":
            bcs.append(wl.PatchBC(wl.FIXED, wl.ZERO_GRAD, (1.0, 0.0, 0.0)))
        else:
            bcs.append(wl.PatchBC(wl.EMPTY, wl.EMPTY))
    return wl.CaseSpec(name="couette", mesh=m, bcs=bcs, nu=nu, dt=dt, p_ctl=wl.SolverCtl(1e-14),
                       u_ctl=wl.SolverCtl(1e-14))


@pytest.mark.parametrize("permute", [None, 5])
def test_T18_impulsive_couette_is_implicit_euler_diffusion(permute):
    """The time term and the wall diffusion (paper §3, PISO with Euler
    implicit time steps): on the start-up Couette flow every step solves
    (h/dt)(u' - u) = nu [(u'_(j+1) - u'_j) - (u'_j - u'_(j-1))]/h, the wall
    neighbours at half a cell (u = 0 below, u = 1 above).  That tridiagonal
    system is solved here with scipy's banded solver, step by step; the
    oracle's velocity must equal it to rounding, with v, w and p zero."""
    from scipy.linalg import solve_banded
    n, nu, dt, K = 16, 0.3, 0.01, 12
    spec = _couette_startup(n, nu, dt, permute)
    oc = orc.OracleCase(spec)
    st, _ = oc.piso(K)
    assert st == 0
    h = 1.0 / n
    ab = np.zeros((3, n))
    ab[0, 1:] = -nu / h
    ab[2, :-1] = -nu / h
    ab[1] = h / dt + 2 * nu / h
    ab[1, 0] += nu / h        # wall at half a cell: 2 nu / h towards it instead of nu / h
    ab[1, -1] += nu / h
    v = np.zeros(n)
    for _ in range(K):
        rhs = h / dt * v
        rhs[-1] += 2 * nu / h * 1.0
        v = solve_banded((1, 1), ab, rhs)
    order = np.argsort(spec.mesh.C[:, 1], kind="stable")
    assert np.abs(oc.U[order, 0] - v).max() <= 1e-13
    assert np.abs(oc.U[:, 1:]).max() == 0.0 and np.abs(oc.p).max() == 0.0


def test_T18_couette_startup_converges_to_the_series_solution():
    """Against the exact start-up solution u = y + sum_m 2 (-1)^m /(m pi)
    sin(m pi y) exp(-nu m^2 pi^2 t): halving h and quartering dt (second order
    in space, first in time) divides the error at t = 0.05 by about 4; and
    long after the start the discrete profile is the linear Couette profile
    u = y exactly (the two-point flux with half-cell wall distances is exact
    for a linear field)."""
    nu, T = 1.0, 0.05

    def exact(y, t):
        m = np.arange(1, 400)[:, None]
        return y + np.sum(2 * (-1.0) ** m / (m * np.pi) * np.sin(m * np.pi * y) * np.exp(-nu * (m * np.pi) ** 2 * t),
                          axis=0)

    errs = []
    for n, steps in ((16, 10), (32, 40)):
        spec = _couette_startup(n, nu, T / steps)
        oc = orc.OracleCase(spec)
        assert oc.piso(steps)[0] == 0
        y = spec.mesh.C[:, 1]
        errs.append(np.abs(oc.U[:, 0] - exact(y, T)).max())
    assert 3.0 <= errs[0] / errs[1] <= 5.0, errs
    spec = _couette_startup(16, nu, 0.05)
    oc = orc.OracleCase(spec)
    assert oc.piso(200)[0] == 0
    assert np.abs(oc.U[:, 0] - spec.mesh.C[:, 1]).max() <= 1e-12
