"""Benchmark of the PISO hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (timed): 3-D lid-driven cavity, 100^3 = 1M hex cells, cells
renumbered by a seeded random permutation (seed 2) then reverse
Cuthill-McKee, Re = 400, PISO dt = 0.002 with 2 correctors, pressure CG with
DIC preconditioning and momentum BiCG with Jacobi, both to tol 1e-7, FP64.
A step is one PISO time step (momentum assembly and solve, two pressure
correctors with assembly, CG solve, flux and velocity correction).  Fields
start at rest; K steps are timed from t = 0 on a freshly created case (the
W warm-up steps run on a separate case).

value = cell-updates/s = cells * K / wall time of the K steps (inputs resident
in device memory before the timed region).

Also reported on the same JSON line:
  roofline      the kernel class with the largest device time in a profiled
                pass (HIP events around each launch, on the stream the kernel
                runs on): algorithmic bytes per working launch / device time
                per working launch (Krylov launches enqueued past a solve's
                convergence return at once and do no work);
  kernels       per-class device time, launches (all and working), mean time
                per launch and per working launch, algorithmic GB/s;
  cpu_baseline  the FP64 oracle on the host on a bounded sample (the first
                PISO step of the same case), in cell-updates/s;
  other_preconditioners  the same case with Jacobi and with the AMG V-cycle
                in place of DIC (time per step, CG iterations per step);
  cav200        the 200^3 cavity (Jacobi) in FP64, in mixed precision and in
                FP64 with AMG: time per step, iterations, per-kernel GB/s;
  serving       continuous batching of a reduced request stream: p50/p99;
  tp1m          the transient pipe with its time-dependent inlet;
  layouts       the assembly operators one at a time in the solver's layout
                and in the paper's hybrid ELL + J + CRS layout, normalised by
                each layout's SMVP as in the paper's Table 3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + PCG SpMV HBM GB/s (FP64 vs mixed); serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(cls: str, N: int, Fi: int, dic: bool) -> float:
    """Bytes per launch that the operation itself must move (FP64).

    Symmetric SpMV: diag, x, y (24 N) + one coefficient and two int32
    indices per internal face (16 Fi).  Other classes follow the same
    counting: every cell-sized array read or written once, every face
    coefficient once, plus two int32 per face where faces are walked."""
    table = {
        "pcg_spmv": 24 * N + 16 * Fi,
        "pcg_update": 56 * N,                      # x, p, r, q, diag in; x, r out
        "pcg_dir": (24 if dic else 32) * N,        # z (or r, diag), p in; p out
        "dic_fwd": 32 * N + 16 * Fi,               # r, D*, y out, z clear; lower faces
        "dic_bwd": 32 * N + 16 * Fi,               # y, D*, r, z out; upper faces
        "dic_setup": 16 * N + 16 * Fi,             # diag, D* out; lower faces
        "bicg_spmv": 104 * N + 24 * Fi,            # 3 components, A and A^T
        "bicgstab_spmv": 80 * N + 12 * Fi,         # 3 components: x in, y out, r~ or s in; diag, upper, lower, 2 int32
        "pcg32_spmv": 12 * N + 12 * Fi,            # FP32 inner: diag, x, y + coefficient + 2 int32
        "pcg32_update": 36 * N,                    # x (FP64) in/out, p, r, q, diag (FP32) in; r out
        "pcg32_dir": 16 * N,
        "bicg32_spmv": 52 * N + 16 * Fi,
        "mom_face": 32 * Fi,                       # phi, w, dl in; upper, lower out
        "mom_cell": 136 * N + 40 * Fi,
        "hbya": 104 * N + 24 * Fi,
        "p_face": 112 * N + 56 * Fi,
        "p_cell": 24 * N + 32 * Fi,
        "flux_corr": 16 * N + 48 * Fi,
        "U_corr": 80 * N + 64 * Fi,
    }
    return float(table.get(cls, 0))


KERNEL_CLASSES = ["pcg_spmv", "pcg_update", "pcg_dir", "dic_setup", "dic_fwd", "dic_bwd", "bicg_spmv", "mom_face",
                  "mom_cell", "hbya", "p_face", "p_cell", "flux_corr", "U_corr", "pcg32_spmv", "pcg32_update",
                  "pcg32_dir", "bicg32_spmv"]


# classes whose launches past a solve's convergence return at once (the
# host enqueues iterations ahead of the device's stop flag): their working
# launches are counted from the solvers' iteration counts.  A pressure CG
# solve of k iterations runs k direction/SpMV/update launches and k DIC
# applications (one at the start, one after each update but the last).
_P_WORK = ("pcg_spmv", "pcg_update", "pcg_dir", "dic_fwd", "dic_bwd", "pcg32_spmv", "pcg32_update", "pcg32_dir")
_U_WORK = ("bicg_spmv",)


def profile_classes(fvm, case, steps, N, Fi, dic):
    """Per-class device time of `steps` PISO steps (HIP events per launch).

    mean_us is over every launch (as a kernel trace reports it); us_per_work
    and alg_GBps are over the launches that did work."""
    import torch
    fvm.profile_enable(True)
    p_work = u_work = 0
    for _ in range(steps):
        st, info = case.piso(1)
        p_work += sum(s["iters"] for s in info["p"])
        u_work += max(s["iters"] for s in info["u"])
    torch.cuda.synchronize()
    out = {}
    for cls in KERNEL_CLASSES:
        ms, n = fvm.profile_read(cls)
        if n == 0:
            continue
        work = min(n, p_work if cls in _P_WORK else u_work if cls in _U_WORK else n)
        mean_us = 1e3 * ms / n
        work_us = 1e3 * ms / max(work, 1)
        b = algorithmic_bytes(cls, N, Fi, dic)
        out[cls] = dict(total_ms=round(ms, 4), launches=n, work_launches=work, mean_us=round(mean_us, 3),
                        us_per_work=round(work_us, 3),
                        alg_GBps=round(b / (work_us * 1e-6) / 1e9, 1) if b and work_us > 0 else None)
    fvm.profile_enable(False)
    return out


def measured_traffic(kernel_class: str, workload: str):
    """HBM bytes per working launch (median over dispatches) from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE summaries under profiles/
    (copy-calibrated), if they were taken on the current kernel source; else
    None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1207_1571_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic-json:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if (rec.get("kernel_class") == kernel_class and rec.get("workload") == workload
                    and rec.get("kernels_hip_sha256") == sha):
                return float(rec["bytes_per_working_launch"])
    return None


def vs_spmv(k, spmv_cls):
    """Assembly operators' device time per call relative to one SpMV (the
    analogue of the paper's Table 3 normalisation)."""
    if spmv_cls not in k or not k[spmv_cls]["us_per_work"]:
        return None
    sp = k[spmv_cls]["us_per_work"]

    def per_call(*names):
        if not all(n in k for n in names):
            return None
        return round(sum(k[n]["mean_us"] for n in names) / sp, 2)

    return {
        "momentum assembly (convection + Laplacian: mom_face + mom_cell)": per_call("mom_face", "mom_cell"),
        "H operator and rAU (hbya)": per_call("hbya"),
        "pressure Laplacian + flux divergence (p_face + p_cell)": per_call("p_face", "p_cell"),
        "flux correction (flux_corr)": per_call("flux_corr"),
        "Gauss gradient of p + velocity correction (U_corr)": per_call("U_corr"),
    }


def cav200_section(fvm, wl, steps, log, profile_steps=2):
    """200^3 cavity, FP64 and mixed (FP32 inner + FP64 refinement), `steps`
    PISO steps each from rest: time per step, pressure iterations, SpMV and
    CG-iteration bandwidth, and the mixed-vs-FP64 field difference."""
    import numpy as np
    import torch
    t = time.perf_counter()
    spec = wl.cav200(n=200, n_steps=steps)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N, Fi = mesh.n_cells, mesh.n_internal
    log(f"cav200 mesh: {N} cells in {time.perf_counter() - t:.1f}s")
    res = {}
    fields = {}
    for name, prec in (("fp64", wl.FP64), ("mixed", wl.MIXED), ("amg_fp64", wl.FP64)):
        sp = spec.with_(precision=prec)
        if name == "amg_fp64":
            sp = sp.with_(p_ctl=wl.SolverCtl(sp.p_ctl.tol, sp.p_ctl.rel_tol, sp.p_ctl.max_iter, wl.PC_AMG))
        c = fvm.Case(sp, mesh=mesh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_iters = 0
        for k in range(steps):
            st, info = c.piso(1)
            p_iters += sum(s["iters"] for s in info["p"])
            if steps <= 5 or (k + 1) % 5 == 0:
                log(f"cav200 {name}: step {k + 1}/{steps}, p iters so far {p_iters}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fields[name] = c.get_state_numpy()
        del c
        k = {}
        if profile_steps > 0:
            pc = fvm.Case(sp, mesh=mesh)
            k = profile_classes(fvm, pc, profile_steps, N, Fi, False)
            del pc
        pre = "pcg32" if prec == wl.MIXED else "pcg"
        it_us = sum(k[c]["us_per_work"] for c in (pre + "_dir", pre + "_spmv", pre + "_update") if c in k)
        it_bytes = (112 * N + 16 * Fi) if prec == wl.FP64 else (64 * N + 12 * Fi)
        res[name] = dict(ms_per_step=round(1e3 * wall / steps, 2), cell_updates_per_s=round(N * steps / wall, 1),
                         p_iters_total=p_iters, ms_per_p_solve=round(1e3 * wall / (2 * steps), 2),
                         spmv_GBps=k.get(pre + "_spmv", {}).get("alg_GBps"),
                         spmv_us=k.get(pre + "_spmv", {}).get("us_per_work"),
                         cg_iter_us=round(it_us, 2) if it_us else None, cg_iter_GBps=round(it_bytes / (it_us * 1e-6) / 1e9, 1) if it_us else None,
                         assembly_vs_spmv=vs_spmv(k, pre + "_spmv"), kernels=k)
        log(f"cav200 {name}: {res[name]['ms_per_step']} ms/step, p iters {p_iters}, SpMV {res[name]['spmv_GBps']} GB/s, "
            f"CG iteration {res[name]['cg_iter_GBps']} GB/s")
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    res["mixed_vs_fp64_relL2"] = dict(U=rel(fields["mixed"][0], fields["fp64"][0]), p=rel(fields["mixed"][1], fields["fp64"][1]))
    res["amg_vs_fp64_relL2"] = dict(U=rel(fields["amg_fp64"][0], fields["fp64"][0]),
                                    p=rel(fields["amg_fp64"][1], fields["fp64"][1]))
    res["workload"] = (f"cav200: 3-D lid-driven cavity 200^3 hex cells, lexicographic, Re=1000, PISO dt=0.001, "
                       f"{steps} steps, PCG-Jacobi / PBiCG-Jacobi tol 1e-6; mixed = FP32 inner (eta 1e-3) + FP64 "
                       f"refinement; amg_fp64 = FP64 with the AMG V-cycle preconditioning the pressure CG")
    return res


def tp_section(fvm, wl, steps, log):
    """tp1M: the transient 2-D pipe, 3200 x 300 cells (960 000), sinusoidal
    inlet set before every step, `steps` PISO steps from rest (the paper
    runs 5000), FP64, PCG-Jacobi / PBiCG-Jacobi tol 1e-6."""
    import numpy as np
    import torch
    t = time.perf_counter()
    spec = wl.tp1m(n_steps=steps)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N, Fi = mesh.n_cells, mesh.n_internal
    log(f"tp1M mesh: {N} cells, {mesh.n_faces} faces in {time.perf_counter() - t:.1f}s")
    c = fvm.Case(spec, mesh=mesh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_iters = 0
    for k in range(steps):
        c.set_patch_value(0, wl.tp1m_inlet(k), 0.0)
        st, info = c.piso(1)
        p_iters += sum(s["iters"] for s in info["p"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    U, p, phi = c.get_state_numpy()
    del c
    res = dict(workload=f"tp1M: 2-D pipe 3200x300 ({N} cells, {mesh.n_faces} faces), nu 3.3e-6, inlet 0.01 sin(pi t), "
                        f"dt 0.1 ms, {steps} PISO steps from rest, FP64, Jacobi PCG/PBiCG tol 1e-6",
               ms_per_step=round(1e3 * wall / steps, 2), cell_updates_per_s=round(N * steps / wall, 1),
               p_iters_per_step=round(p_iters / steps, 1), finite=bool(np.isfinite(U).all() and np.isfinite(p).all()))
    log(f"tp1M: {res['ms_per_step']} ms/step, {res['p_iters_per_step']} pressure CG iterations per step")
    return res


# the paper's Table 3 (C2070, its hybrid layout): SMVP time and the
# divergence, gradient and Laplacian times normalised by it
PAPER_TABLE3 = {"cav100": dict(smvp_us=1103, div=2.9, grad=10.7, lap=2.4),
                "tp1M": dict(smvp_us=775, div=2.8, grad=10.4, lap=2.3)}


def precond_section(fvm, wl, mesh, steps, log):
    """The benchmark case with the pressure preconditioner switched to
    Jacobi and to the aggregation AMG V-cycle: the same PISO steps from rest,
    time per step and CG iterations (the benchmark configuration itself uses
    DIC)."""
    import torch
    out = {}
    for name, pc in (("jacobi", wl.PC_JACOBI), ("amg", wl.PC_AMG)):
        spec = wl.cav100(n=100, n_steps=steps)
        spec = spec.with_(p_ctl=wl.SolverCtl(spec.p_ctl.tol, spec.p_ctl.rel_tol, spec.p_ctl.max_iter, pc))
        t = time.perf_counter()
        c = fvm.Case(spec, mesh=mesh)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            st, info = c.piso(1)
            its += sum(s["iters"] for s in info["p"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = dict(ms_per_step=round(1e3 * wall / steps, 2), p_iters_per_step=round(its / steps, 1),
                         cell_updates_per_s=round(mesh.n_cells * steps / wall, 1), case_setup_s=round(setup, 2))
        log(f"precond {name}: {out[name]['ms_per_step']} ms/step, {out[name]['p_iters_per_step']} CG iterations "
            f"per step (case set-up {setup:.1f}s)")
        del c
    out["workload"] = f"cav100, {steps} PISO steps from rest, pressure CG with Jacobi or AMG instead of DIC"
    return out


def layout_section(fvm, wl, log, reps=20):
    """The assembly operators one at a time in the solver's face-major layout
    and in the paper's hybrid layout (ELL + J + CRS, K = 7), normalised by
    each layout's own SMVP as in the paper's Table 3 (device time per launch,
    HIP events; the conversion of the inputs into each layout is excluded)."""
    import numpy as np
    import torch
    out = {}
    specs = (("cav100", "cav100 (random + RCM numbering)", wl.cav100(n=100, n_steps=1)),
             ("cav100_lex", "100^3 cavity, lexicographic", wl.cavity((100, 100, 100), Re=400.0, dt=0.002)),
             ("tp1M", "tp1M 3200x300 pipe, lexicographic", wl.tp1m(n_steps=1)))
    for key, desc, spec in specs:
        spec = spec.with_(hybrid_K=7)
        t = time.perf_counter()
        c = fvm.Case(spec)
        N, F = spec.mesh.V.shape[0], spec.mesh.owner.shape[0]
        log(f"layouts {key}: case with both layouts in {time.perf_counter() - t:.1f}s")
        rng = np.random.default_rng(9)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
        x, flux, gamma = dev(rng.normal(size=N)), dev(rng.normal(size=F)), dev(rng.uniform(0.5, 2.0, F))
        y, g3 = torch.empty(N, dtype=torch.float64, device="cuda"), torch.empty(3 * N, dtype=torch.float64, device="cuda")
        V = torch.empty(7 * N + 2 * F, dtype=torch.float64, device="cuda")
        ops = [(fvm.OP_LAP, gamma, y), (fvm.OP_GRAD, x, g3), (fvm.OP_DIV, flux, y), (fvm.OP_SPMV, x, y),
               (fvm.OP_HY_LAP, gamma, V), (fvm.OP_HY_GRAD, x, g3), (fvm.OP_HY_DIV, flux, y), (fvm.OP_HY_SPMV, x, y),
               (fvm.OP_HY_STMVP, x, y)]
        for op, a, o in ops:
            fvm.operator(c, op, a, o)
        torch.cuda.synchronize()
        fvm.profile_enable(True)
        for _ in range(reps):
            for op, a, o in ops:
                fvm.operator(c, op, a, o)
        torch.cuda.synchronize()
        us = {}
        for cls in ("op_spmv", "op_grad", "op_div", "op_lap", "hy_spmv", "hy_stmvp", "hy_grad", "hy_div", "hy_lap"):
            ms, n = fvm.profile_read(cls)
            us[cls] = round(1e3 * ms / max(n, 1), 2)
        fvm.profile_enable(False)
        res = dict(workload=desc, cells=N)
        for lay, pre in (("face_major", "op"), ("hybrid", "hy")):
            sm = us[pre + "_spmv"]
            res[lay] = dict(smvp_us=sm, div=round(us[pre + "_div"] / sm, 2), grad=round(us[pre + "_grad"] / sm, 2),
                            lap=round(us[pre + "_lap"] / sm, 2))
        res["hybrid"]["stmvp"] = round(us["hy_stmvp"] / us["hy_spmv"], 2)
        res["us"] = us
        base = "tp1M" if key == "tp1M" else "cav100"
        res["paper_table3"] = PAPER_TABLE3[base]
        log(f"layouts {key}: face-major {res['face_major']}, hybrid {res['hybrid']}")
        out[key] = res
        del c
    return out


def serve_section(fvm, wl, n_requests, n_steps, log):
    """Serving stream (cavity/duct cases, cube side log-uniform 16..96,
    Re U(10, 1000), Poisson arrivals at 40 req/s), reduced to `n_requests`
    requests of `n_steps` PISO steps, run once in FP64 and once mixed: p50 /
    p99 time from arrival to converged result, throughput."""
    import torch
    from paper_1207_1571_amd.serve import GpuBackend, Request, Server, summarize
    reqs = wl.serve_stream(n_requests=n_requests, n_steps=n_steps)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    out = dict(workload=f"serve: {n_requests} requests of the 512-request stream (seed 5; cavity/duct, side "
                        f"log-uniform 16..96, Re U(10,1000), Poisson 40 req/s), {n_steps} PISO steps each, "
                        f"tol 1e-6, Jacobi; slots 32, groups of 16, 10 steps per advance",
               budget_bytes=budget)
    for name, prec in (("fp64", wl.FP64), ("mixed", wl.MIXED)):
        t = time.perf_counter()
        specs = [wl.serve_case(r, precision=prec) for r in reqs]
        log(f"serve {name}: {len(specs)} case meshes in {time.perf_counter() - t:.1f}s")
        be = GpuBackend()
        res = Server(be, budget, slots=32, group=16, chunk=10).run(
            [Request(r.rid, r.arrival_s, s, r.n_steps) for r, s in zip(reqs, specs)])
        torch.cuda.synchronize()
        sm = summarize(res)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sm.items()}
        log(f"serve {name}: p50 {sm['p50_s']:.3f}s p99 {sm['p99_s']:.3f}s, makespan {sm['makespan_s']:.2f}s, "
            f"{sm['cell_updates_per_s']:.4g} cell-updates/s, failed {sm['failed']}")
        del be, specs, res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100, help="cube side (100 = the benchmark configuration)")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cav200-steps", type=int, default=20, help="steps of the 200^3 FP64-vs-mixed section (0: skip)")
    ap.add_argument("--cav200-profile-steps", type=int, default=2,
                    help="steps of the per-kernel-class timing pass of the 200^3 section (0: skip)")
    ap.add_argument("--tp-steps", type=int, default=10, help="PISO steps of the tp1M transient pipe section (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=32, help="requests of the serving section (0: skip)")
    ap.add_argument("--no-precond-compare", dest="precond_compare", action="store_false",
                    help="skip the runs of the benchmark case with Jacobi and AMG in place of DIC")
    ap.add_argument("--no-layouts", dest="layouts", action="store_false",
                    help="skip the face-major vs hybrid layout operator comparison")
    ap.add_argument("--serve-steps", type=int, default=20, help="PISO steps per serving request")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1207_1571_amd import fvm
    from paper_1207_1571_amd import workloads as wl

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")
        del src, dst
    t = time.perf_counter()
    spec = wl.cav100(n=args.n, n_steps=args.steps)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N, Fi = mesh.n_cells, mesh.n_internal
    log(f"mesh {args.n}^3: {N} cells, {Fi} internal faces, built in {time.perf_counter() - t:.1f}s")

    if args.warmup > 0:
        w = fvm.Case(spec, mesh=mesh)
        w.piso(args.warmup)
        torch.cuda.synchronize()
        del w
        log(f"warm-up {args.warmup} steps done")

    case = fvm.Case(spec, mesh=mesh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = case.piso(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = N * args.steps / wall
    p_iters_last = [s["iters"] for s in info["p"]]
    log(f"timed {args.steps} steps in {wall:.3f}s: {value:.4g} cell-updates/s; last step p iters {p_iters_last}, "
        f"U iters {[s['iters'] for s in info['u']]}, status {st}")
    U, p, phi = case.get_state_numpy()
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(p)), "non-finite fields"
    del case

    # profiled pass: per-kernel-class device time
    kernels = {}
    if args.profile_steps > 0:
        pc = fvm.Case(spec, mesh=mesh)
        kernels = profile_classes(fvm, pc, args.profile_steps, N, Fi, spec.p_ctl.precond == wl.PC_DIC)
        del pc
        log("kernel classes: " + json.dumps(kernels))
    jacobi = precond_section(fvm, wl, mesh, args.steps, log) if args.precond_compare else None
    del mesh
    cav200 = (cav200_section(fvm, wl, args.cav200_steps, log, args.cav200_profile_steps)
              if args.cav200_steps > 0 else None)
    serving = serve_section(fvm, wl, args.serve_requests, args.serve_steps, log) if args.serve_requests > 0 else None
    tp = tp_section(fvm, wl, args.tp_steps, log) if args.tp_steps > 0 else None
    layouts = layout_section(fvm, wl, log) if args.layouts else None
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"]) if kernels else None
    roofline = None
    if dom:
        ach = kernels[dom]["alg_GBps"]
        tb = measured_traffic(dom, f"cav{args.n}")
        roofline = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(ach / HBM_PEAK_GBS, 4) if ach else None,
                        traffic=round(tb) if tb else None,
                        traffic_GBps=round(tb / (kernels[dom]["us_per_work"] * 1e-6) / 1e9, 1) if tb else None,
                        algorithmic_bytes=algorithmic_bytes(dom, N, Fi, spec.p_ctl.precond == wl.PC_DIC))
        if dom.startswith("dic"):
            roofline["note"] = ("dependency-latency bound: the sweep is a chain of one step per level of the "
                                "lower-triangular graph; HBM fraction shown for reference")
    spmv = kernels.get("pcg_spmv")

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        oc = orc.OracleCase(spec)
        t = time.perf_counter()
        oc.piso(1)
        dt = time.perf_counter() - t
        cpu = dict(value=round(N / dt, 1), unit="cell-updates/s", cores=1, kind="oracle",
                   sample=f"first PISO step of the same {args.n}^3 case, single-threaded C oracle ({dt:.1f}s)")
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cav{args.n}: 3-D lid-driven cavity {args.n}^3 hex cells, random renumbering "
                               f"(seed 2) + RCM, Re=400, PISO dt=0.002, 2 correctors, PCG-DIC / PBiCG tol 1e-7",
                   "cells": N, "internal_faces": Fi, "precision": "fp64"},
        "pcg_spmv_GBps": spmv["alg_GBps"] if spmv else None,
        "cav200": cav200,
        "serving": serving,
        "tp1m": tp,
        "layouts": layouts,
        "other_preconditioners": jacobi,
        "p_iters_last_step": p_iters_last,
        "roofline": roofline,
        "assembly_vs_spmv": vs_spmv(kernels, "pcg_spmv") if kernels else None,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
