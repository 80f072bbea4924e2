"""Parity and properties at the benchmark configurations' full sizes.

The oracle finishes one PISO step of the 1M-cell benchmark cavity and two
SIMPLE iterations of the 1M-cell jittered duct in seconds, so those are
compared element by element (same protocol as tests/test_gpu_parity.py).
The 8M-cell cavity is checked through properties that hold at any size:
the corrected flux is divergence-free to solver tolerance, the flow is
mirror-symmetric about the mid-plane normal to the lid's side walls, and the
mixed-precision result agrees with the FP64 one within 1e-6; its pressure
CG, the path the benchmark times, is also compared value by value with the
oracle over 8 iterations of a seeded system (the oracle takes seconds for
that).
"""
import sys

import numpy as np
import pytest

from paper_1207_1571_amd import workloads as wl

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_parity import _gpu, _parity, _rel  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _div(mesh, phi):
    div = np.zeros(mesh.n_cells)
    np.add.at(div, mesh.owner, phi)
    np.add.at(div, mesh.neighbour, -phi[: mesh.n_internal])
    return div


@pytest.mark.timeout(300)
def test_cav100_benchmark_first_step_parity():
    """The benchmark case exactly (100^3, random renumbering then RCM,
    PCG-DIC / PBiCG tol 1e-7, FP64): first PISO step against the oracle."""
    case = wl.cav100(n=100, n_steps=1)
    g, o = _parity(case, 1, what="cav100 benchmark, step 1")
    assert np.abs(_div(case.mesh, g["phi"])).max() <= 1e-6 * np.abs(g["phi"]).max()


@pytest.mark.timeout(300)
def test_duct256_full_size_simple_parity():
    """The jittered 256x64x64 duct (non-orthogonal faces), two SIMPLE
    iterations with absolute inner tolerances, against the oracle."""
    case = wl.duct256().with_(p_ctl=wl.SolverCtl(1e-8, 0.0), u_ctl=wl.SolverCtl(1e-8, 0.0))
    _parity(case, 2, simple=True, res_tol=0.0, what="duct256 SIMPLE x2")


@pytest.mark.timeout(300)
def test_cav200_properties_fp64_and_mixed():
    """200^3 cavity, one PISO step in FP64 and in mixed precision:
    divergence-free flux, mirror symmetry in z, mixed within 1e-6 of FP64."""
    base = wl.cav200(n=200, n_steps=1)
    _say("[cav200] FP64 step")
    g = _gpu(base, 1)
    del g["case"]
    _say(f"  iters {[s['iters'] for s in g['info']['u']]} {[s['iters'] for s in g['info']['p']]}")
    _say("[cav200] mixed step")
    m = _gpu(base.with_(precision=wl.MIXED), 1)
    del m["case"]
    mesh = base.mesh
    for name, r in (("fp64", g), ("mixed", m)):
        div = _div(mesh, r["phi"])
        d = np.abs(div).max() / np.abs(r["phi"]).max()
        _say(f"  {name}: max |div phi| / max |phi| = {d:.2e}")
        # the pressure solves stop at a normalised residual of 1e-6
        assert d <= 1e-6
    eU, ep = _rel(m["U"], g["U"]), _rel(m["p"], g["p"])
    _say(f"  mixed vs fp64: relL2 U {eU:.2e} p {ep:.2e}")
    assert eU <= 1e-6 and ep <= 1e-6
    # mirror symmetry z -> 1 - z (lexicographic cells: index = x + n (y + n z))
    n = 200
    U = g["U"].reshape(n, n, n, 3)          # [z][y][x][component]
    Um = U[::-1].copy()
    Um[..., 2] *= -1.0
    sym = np.linalg.norm(U - Um) / np.linalg.norm(U)
    p = g["p"].reshape(n, n, n)
    psym = np.linalg.norm(p - p[::-1]) / np.linalg.norm(p - p.mean())
    _say(f"  z-mirror asymmetry: U {sym:.2e} p {psym:.2e}")
    # the mirror is exact for the converged solution; the reference-cell pin
    # at a z = 0 corner makes the unconverged remainder (solver tolerance
    # 1e-6, normalised) asymmetric
    assert sym <= 1e-6 and psym <= 1e-6


@pytest.mark.timeout(300)
def test_cav200_pressure_solve_against_oracle():
    """The headline path itself at full size: the Jacobi pressure CG on the
    8M-cell cavity (every product on the paired 7-point kernel, except the
    slices of the first and last planes), 8 iterations from a seeded start
    on a seeded system, against the oracle's 8 iterations: every one of the
    8M values within the parity protocol's 1e-9 (relative L2) and the same
    stopping status."""
    import torch
    from oracle import oracle as orc
    from paper_1207_1571_amd import fvm
    case = wl.cav200(n=200, n_steps=1)
    m = case.mesh
    mesh = fvm.Mesh(m, case.bcs)
    si = fvm.mesh_sell_info(mesh)
    assert 2 * si["n_7pt_slices"] >= si["n_slices"]
    rng = np.random.default_rng(4)
    gamma = rng.uniform(0.5, 2.0, m.n_faces)
    rhs = rng.normal(size=m.n_cells)
    rhs -= rhs.mean()
    p0 = rng.normal(size=m.n_cells) * 0.1
    _say("[cav200 solve] oracle, 8 CG iterations")
    po = p0.copy()
    st_o, info_o = orc.OracleCase(case).solve_pressure(gamma, rhs, po, 0.0, max_iter=8)
    _say("[cav200 solve] GPU, 8 CG iterations")
    c = fvm.Case(case, mesh=mesh)
    pg = torch.from_numpy(p0.copy()).cuda()
    st_g, info_g = c.solve_pressure(torch.from_numpy(gamma).cuda(), torch.from_numpy(rhs).cuda(), pg, 0.0,
                                    max_iter=8)
    pg = pg.cpu().numpy()
    c.close()
    err = _rel(pg, po)
    _say(f"  status gpu {st_g} oracle {st_o}; iters {info_g['iters']} {info_o['iters']}; relL2 {err:.2e}, "
         f"max |diff| {np.abs(pg - po).max():.2e}")
    assert st_g == st_o and info_g["iters"] == info_o["iters"] == 8
    assert err <= 1e-9


@pytest.mark.timeout(300)
def test_duct256_simple_to_convergence_matches_poiseuille():
    """The duct configuration run as configured: steady SIMPLE on the jittered
    256x64x64 duct until every initial residual is <= 1e-6.  The section
    3.5 <= x <= 3.75 matches the developed laminar square-duct series within
    2% of its peak (max norm), and the outflow balances the inflow (T15).
    (The plug inflow at Re 50 is still developing upstream: the max-norm
    difference is 3.9% at 2.5 <= x <= 3, 2.4% at 3 <= x <= 3.5 and 1.5% here,
    the same with and without the vertex jitter, so it is development, not
    discretisation.)"""
    from paper_1207_1571_amd import fvm
    from test_oracle_pins import _duct_series
    spec = wl.duct256(max_iters=4000)
    c = fvm.Case(spec)
    done, info = 0, None
    while done < 4000:
        st, it, info = c.simple(min(500, 4000 - done), spec.res_tol)
        assert st >= 0
        done += it
        res = [info["u"][k]["res_initial"] for k in range(3)] + [info["p"][0]["res_initial"]]
        _say(f"  duct256: {done} SIMPLE iterations, initial residuals {['%.2e' % r for r in res]}")
        if max(res) <= spec.res_tol:
            break
    assert max(res) <= spec.res_tol, res
    U, p, phi = c.get_state_numpy()
    m = spec.mesh
    sel = (m.C[:, 0] >= 3.5) & (m.C[:, 0] <= 3.75)
    ua = _duct_series(m.C[sel, 1] - 0.5, m.C[sel, 2] - 0.5)
    err = np.abs(U[sel, 0] - ua).max() / ua.max()
    s_in, n_in = m.patch("xmin")
    s_out, n_out = m.patch("xmax")
    q_in, q_out = phi[s_in:s_in + n_in].sum(), phi[s_out:s_out + n_out].sum()
    bal = abs(q_in + q_out) / abs(q_in)
    _say(f"  duct256 converged in {done} iterations: developed profile max error {err:.3%} of peak, "
         f"mass balance {bal:.2e}")
    assert err <= 0.02
    assert bal <= 1e-6
