"""Serving on the GPU: each case's result is the same alone and in the mix.

Cases of different kinds and sizes arrive at different times; the server
admits them as slots free up and advances the resident ones together in
shared launches, so the group a case is advanced with changes while it runs.
The fields of every case must equal, bit for bit, those of the same case
run alone through piso_step (the kernels reduce per case in a fixed order
and a case's block-to-XCD placement does not depend on the batch), and so
also lie within the mixed-precision tolerance of 1e-6.
"""
import sys

import numpy as np
import pytest

from paper_1207_1571_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _requests(precision, n_steps, tol=1e-6):
    rng = np.random.default_rng(11)
    specs = []
    for rid, (kind, n) in enumerate([("cavity", 9), ("duct", 7), ("cavity", 12), ("duct", 10), ("cavity", 6),
                                      ("cavity", 11)]):
        req = wl.ServeRequest(rid, 0.0, kind, n, float(rng.uniform(10.0, 1000.0)), 0.2 / n, n_steps)
        specs.append(wl.serve_case(req, precision=precision, tol=tol))
    return specs


@pytest.mark.parametrize("step_kernel", [wl.STEP_AUTO, wl.STEP_LAUNCHED])
@pytest.mark.parametrize("precision", [wl.MIXED, wl.FP64])
def test_alone_equals_in_the_mix(precision, step_kernel):
    import torch
    from paper_1207_1571_amd import fvm
    from paper_1207_1571_amd.serve import GpuBackend, Request, Server

    n_steps = 6
    specs = [s.with_(step_kernel=step_kernel) for s in _requests(precision, n_steps)]
    alone = {}
    for rid, spec in enumerate(specs):
        _say(f"alone rid={rid} N={spec.mesh.n_cells} precision={precision}")
        c = fvm.Case(spec)
        st, info = c.piso(n_steps)
        assert st == 0
        alone[rid] = c.get_state_numpy()
        c.close()
    torch.cuda.synchronize()

    # arrivals spread out so that cases join while others are resident; at
    # most 3 resident, advanced 2 steps at a time in groups of up to 3
    arrivals = [0.0, 0.0, 0.01, 0.03, 0.06, 0.09]
    reqs = [Request(rid, arrivals[rid], spec, n_steps) for rid, spec in enumerate(specs)]
    be = GpuBackend(keep_fields=True)
    budget = sum(be.footprint(s) for s in specs)
    _say(f"mix: {len(reqs)} requests, budget {budget} bytes")
    groups = []
    orig_advance = be.advance

    def advance(cases, steps, lane=None):
        groups.append(tuple(id(c) for c in cases))
        return orig_advance(cases, steps, lane)

    be.advance = advance
    res = Server(be, budget, slots=3, group=3, chunk=2).run(reqs)
    assert len(res) == len(specs)
    # the batch composition changed while cases were resident
    assert len(set(groups)) > 1 and max(len(g) for g in groups) > 1
    for r in res:
        assert r.status == 0, r
        U, p, phi = r.fields
        Ua, pa, phia = alone[r.rid]
        for name, a, b in (("U", U, Ua), ("p", p, pa), ("phi", phi, phia)):
            nb = np.linalg.norm(b)
            rel = np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
            assert rel <= 1e-6, (r.rid, name, rel)
            assert np.array_equal(a, b), (r.rid, name, rel)


def test_budget_admission_on_device():
    """A budget that holds only the largest case admits one case at a time,
    and every case still completes."""
    from paper_1207_1571_amd.serve import GpuBackend, Request, Server

    allspecs = _requests(wl.MIXED, 2)
    specs = [allspecs[i] for i in (0, 3, 5)]   # 9^3, 10^3, 11^3: no two fit in the largest one's footprint
    be = GpuBackend()
    foot = [be.footprint(s) for s in specs]
    assert max(foot) < sum(sorted(foot)[:2])
    reqs = [Request(rid, 0.0, s, 2) for rid, s in enumerate(specs)]
    res = Server(be, max(foot), slots=8, group=8, chunk=2).run(reqs)
    assert sorted(r.rid for r in res) == [0, 1, 2]
    spans = sorted((r.admitted_s, r.done_s) for r in res)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0   # never two resident at once


def test_batched_dic_cases_equal_their_solo_runs():
    """Several PCG-DIC cases (FP64) advanced in shared launches: each case
    elects its own XCD for its sweeps, and its fields equal its solo run bit
    for bit."""
    from paper_1207_1571_amd import fvm
    specs = [wl.cavity(sh, Re=300.0, dt=0.01, perm_seed=seed, use_rcm=True, tol=1e-8, p_precond=wl.PC_DIC)
             for sh, seed in (((9, 8, 7), 1), ((12, 6, 5), 2), ((7, 7, 7), 3))]
    alone = []
    for spec in specs:
        c = fvm.Case(spec)
        c.piso(3)
        alone.append(c.get_state_numpy())
        c.close()
    cases = [fvm.Case(spec) for spec in specs]
    st, infos = fvm.piso_batch(cases, 3)
    assert st == 0
    for c, a in zip(cases, alone):
        for x, y in zip(c.get_state_numpy(), a):
            assert np.array_equal(x, y)
        c.close()


def test_mixed_options_stream():
    """Requests with different precisions and pressure preconditioners
    (Jacobi, DIC, AMG) in one stream: the backend advances compatible cases
    together and AMG cases alone; every case equals its solo run."""
    from paper_1207_1571_amd import fvm
    from paper_1207_1571_amd.serve import GpuBackend, Request, Server
    specs = [wl.cavity((9, 8, 7), Re=300.0, dt=0.01, tol=1e-8),
             wl.cavity((8, 8, 8), Re=200.0, dt=0.01, tol=1e-8, precision=wl.MIXED),
             wl.cavity((10, 9, 8), Re=300.0, dt=0.01, tol=1e-8, p_precond=wl.PC_AMG),
             wl.cavity((7, 7, 7), Re=100.0, dt=0.01, tol=1e-8, p_precond=wl.PC_DIC),
             wl.cavity((11, 9, 7), Re=300.0, dt=0.01, tol=1e-8, p_precond=wl.PC_AMG),
             wl.cavity((9, 9, 9), Re=300.0, dt=0.01, tol=1e-8)]
    alone = []
    for spec in specs:
        c = fvm.Case(spec)
        st, _ = c.piso(4)
        assert st == 0
        alone.append(c.get_state_numpy())
        c.close()
    be = GpuBackend(keep_fields=True)
    budget = sum(be.footprint(s) for s in specs)
    res = Server(be, budget, slots=6, group=6, chunk=2).run([Request(k, 0.0, s, 4) for k, s in enumerate(specs)])
    assert sorted(r.rid for r in res) == list(range(len(specs)))
    for r in res:
        assert r.status == 0, r
        for a, b in zip(r.fields, alone[r.rid]):
            assert np.array_equal(a, b), r.rid


@pytest.mark.parametrize("precision", [wl.FP64, wl.MIXED])
def test_served_cases_match_the_oracle(precision):
    """Every case of a served stream against the FP64 oracle, all at an
    outer tolerance of 1e-10: FP64 within 1e-9, with the oracle's pressure
    iteration counts at the ends of the advances; mixed precision within
    1e-6."""
    from oracle import oracle as orc
    from paper_1207_1571_amd.serve import GpuBackend, Request, Server

    n_steps, chunk = 4, 2
    specs = _requests(precision, n_steps, tol=1e-10)
    be = GpuBackend(keep_fields=True)
    budget = sum(be.footprint(s) for s in specs)
    reqs = [Request(rid, 0.0, spec, n_steps) for rid, spec in enumerate(specs)]
    res = Server(be, budget, slots=len(specs), group=len(specs), chunk=chunk).run(reqs)
    assert sorted(r.rid for r in res) == list(range(len(specs)))
    tol = 1e-9 if precision == wl.FP64 else 1e-6
    for r in sorted(res, key=lambda r: r.rid):
        assert r.status == 0, r
        spec = specs[r.rid].with_(precision=wl.FP64)
        oc = orc.OracleCase(spec)
        p_iters = 0
        for k in range(n_steps):
            st, info = oc.piso(1)
            assert st == 0
            if (k + 1) % chunk == 0:
                p_iters += sum(s["iters"] for s in info["p"])
        errs = []
        for a, b in zip(r.fields, (oc.U, oc.p, oc.phi)):
            nb = np.linalg.norm(b)
            errs.append(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
        _say(f"  served rid={r.rid} N={r.n_cells}: relL2 U {errs[0]:.2e} p {errs[1]:.2e} phi {errs[2]:.2e}; "
             f"p iters {r.p_iters} oracle {p_iters}")
        assert max(errs) <= tol, (r.rid, errs)
        if precision == wl.FP64:
            assert r.p_iters == p_iters, (r.rid, r.p_iters, p_iters)
