"""Benchmark of the PISO / SIMPLE hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload (timed): the 3-D lid-driven cavity of 200^3 = 8M hex
cells, lexicographic numbering, Re = 1000, PISO dt = 0.001 with 2
correctors, pressure CG and momentum BiCG with Jacobi preconditioning, both
to a normalised residual of 1e-6, FP64.  A step is one PISO time step
(momentum assembly and solve, two pressure correctors with assembly, CG
solve, flux and velocity correction).  Fields start at rest; K steps are
timed from t = 0 on a freshly created case (the W warm-up steps run on a
separate case).

value = cell-updates/s = cells * K / wall time of the K steps (inputs
resident in device memory before the timed region).

Also reported on the same JSON line:
  mixed         the same K steps with FP32 inner Krylov iterations inside
                FP64 refinement: cell-updates/s, time per step and per
                pressure solve, speedup over FP64, field difference;
  roofline      the FP64 run's kernel class with the largest device time in
                a profiled pass (HIP events around each launch on the stream
                the kernel runs on): algorithmic bytes per working launch /
                device time per working launch, and the HBM bytes the
                rocprofv3 counters measured for that kernel (committed
                summaries under profiles/, used while the kernel source is
                the one profiled);
  cav200        per-class kernel times, SpMV and CG-iteration bandwidth
                (algorithmic and counter-measured) for FP64 and mixed, and
                FP64 with the AMG-preconditioned pressure CG;
  cpu_baseline  the FP64 oracle on the host (compiled for it, one thread)
                on a stated prefix of the same case, extrapolated to a full
                step, with the GPU's time for the identical prefix beside it;
  cav2d32, cav100, duct256, tp1m
                the other configurations: the 2-D cavity (100 steps), the
                1M-cell cavity with PCG-DIC (and Jacobi / AMG in its place),
                steady SIMPLE on the jittered duct to initial residuals of
                1e-6, the transient pipe with its time-dependent inlet;
  serving       continuous batching of the 512-request stream (a stated
                number of PISO steps per request), FP64 and mixed: p50/p99
                (--serving-only runs this section alone, e.g. with the
                configuration's 200 steps per request);
  layouts       the assembly operators one at a time in the solver's layout
                and in the paper's hybrid ELL + J + CRS layout, normalised by
                each layout's SMVP as in the paper's Table 3.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + PCG SpMV HBM GB/s (FP64 vs mixed); serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def diag_read_cells(spec, sell: dict) -> int:
    """Cells whose CG product reads the stored diagonal (FP64) or row sum
    (FP32): those of the 256-cell slices holding a cell with a
    fixed-pressure boundary face, or the reference pin when no patch fixes
    the pressure, and those of the slices with explicit columns (the other
    slices form each diagonal from the row's coefficients, and their row
    sums are zero)."""
    import numpy as np
    m = spec.mesh
    N = m.n_cells
    marked = np.zeros((N + 255) // 256, dtype=bool)
    fixed = [k for k, bc in enumerate(spec.bcs) if bc.p_kind == 0]
    for k in fixed:
        st, sz = int(m.patch_start[k]), int(m.patch_size[k])
        marked[np.asarray(m.owner[st:st + sz]) // 256] = True
    if not fixed:
        marked[spec.p_ref_cell // 256] = True
    return int(min(N, marked.sum() * 256 + sell.get("n_explicit_slices", 0) * 256))


def algorithmic_bytes(cls: str, N: int, Fi: int, sell: dict | None = None, diag_cells: int | None = None) -> float:
    """Bytes per launch that the operation itself must move.

    Symmetric SpMV (the CG's q = A p on the sliced-ELL copy): x and y, one
    coefficient per internal face (the matrix is symmetric; regular slices
    read the lower triangle through mirror slots), the diagonal where it is
    read (diag_cells cells: FP64 diagonals or FP32 row sums),
    and one int32 column index per entry of the slices that store explicit
    columns (regular slices store none).  Other classes: every cell-sized
    array read or written once, every face coefficient once, plus two int32
    per face where faces are walked through index lists."""
    ex = 4 * (sell["explicit_entries"] if sell else 2 * Fi)
    dcells = N if diag_cells is None else diag_cells
    table = {
        "pcg_spmv": 16 * N + 8 * dcells + 8 * Fi + ex,
        "pcg_update": 56 * N,                      # x, p, r, q, diag in; x, r out
        "pcg_dir": 32 * N,                         # r, diag, p in; p out (Jacobi)
        "pcg_dir_dic": 24 * N,                     # z, p in; p out
        "dic_fwd": 32 * N + 16 * Fi,               # r, D*, y out, z clear; lower faces
        "dic_bwd": 32 * N + 16 * Fi,               # y, D*, r, z out; upper faces
        "dic_setup": 16 * N + 16 * Fi,             # diag, D* out; lower faces
        "bicg_spmv": 104 * N + 24 * Fi,            # 3 components, A and A^T
        "bicgstab_spmv": 80 * N + 12 * Fi,         # 3 components: x in, y out, r~ or s in; diag, upper, lower, 2 int32
        "pcg32_spmv": 8 * N + 4 * dcells + 4 * Fi + ex,   # FP32 inner: x, y, row sums where read + coefficient (+ explicit indices)
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


def cg_iteration_bytes(N: int, Fi: int, sell: dict, mixed: bool, diag_cells: int | None = None) -> float:
    """One Jacobi CG iteration: direction, SpMV, update."""
    if mixed:
        return sum(algorithmic_bytes(c, N, Fi, sell, diag_cells) for c in ("pcg32_dir", "pcg32_spmv", "pcg32_update"))
    return sum(algorithmic_bytes(c, N, Fi, sell, diag_cells) for c in ("pcg_dir", "pcg_spmv", "pcg_update"))


KERNEL_CLASSES = ["pcg_spmv", "pcg_update", "pcg_dir", "dic_setup", "dic_fwd", "dic_bwd", "bicg_spmv", "mom_face",
                  "mom_cell", "hbya", "p_face", "p_cell", "flux_corr", "U_corr", "pcg32_spmv", "pcg32_update",
                  "pcg32_dir", "bicg32_spmv"]

# rocprofv3 kernel names of the classes whose HBM traffic the committed
# counter summaries hold
KERNEL_OF_CLASS = {"pcg_spmv": "k_cg_spmv<double", "pcg_update": "k_cg_update<", "pcg_dir": "k_cg_dir<double",
                   "pcg32_spmv": "k_cg_spmv<float", "pcg32_update": "k_rr_update<", "pcg32_dir": "k_cg_dir<float",
                   "dic_fwd": "k_dic_sweep<1", "dic_bwd": "k_dic_sweep<2"}


# classes whose launches past a solve's convergence return at once (the
# host enqueues iterations ahead of the device's stop flag): their working
# launches are counted from the solvers' iteration counts.  A pressure CG
# solve of k iterations runs k direction/SpMV/update launches and k DIC
# applications (one at the start, one after each update but the last).
_P_WORK = ("pcg_spmv", "pcg_update", "pcg_dir", "dic_fwd", "dic_bwd", "pcg32_spmv", "pcg32_update", "pcg32_dir")
_U_WORK = ("bicg_spmv",)


def profile_classes(fvm, case, steps, N, Fi, dic, sell, diag_cells=None):
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
        b = algorithmic_bytes("pcg_dir_dic" if (cls == "pcg_dir" and dic) else cls, N, Fi, sell, diag_cells)
        out[cls] = dict(total_ms=round(ms, 4), launches=n, work_launches=work, mean_us=round(mean_us, 3),
                        us_per_work=round(work_us, 3),
                        alg_bytes=b or None,
                        alg_GBps=round(b / (work_us * 1e-6) / 1e9, 1) if b and work_us > 0 else None)
    fvm.profile_enable(False)
    return out


def kernels_sha256() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_1207_1571_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def measured_traffic(kernel_class: str, workload: str):
    """HBM bytes and median duration per working launch from the rocprofv3
    FETCH_SIZE / WRITE_SIZE summaries under profiles/ (copy-calibrated), if
    they were taken on the current kernel source; else None."""
    import glob
    sha = kernels_sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic-json:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if (rec.get("kernel_class") == kernel_class and rec.get("workload") == workload
                    and rec.get("kernels_hip_sha256") == sha):
                return rec
    return None


def counter_GBps(rec):
    """HBM GB/s of a kernel from its counter record: counted bytes over the
    median duration of its working launches in the same profile."""
    if not rec or not rec.get("median_us"):
        return None
    return round(rec["bytes_per_working_launch"] / (rec["median_us"] * 1e-6) / 1e9, 1)


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


def run_steps(fvm, spec, mesh, steps, log, name, every=5):
    """`steps` PISO steps from rest on a fresh case; wall time between two
    device synchronisations."""
    import torch
    c = fvm.Case(spec, mesh=mesh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_iters = []
    u_iters = []
    st_all = 0
    for k in range(steps):
        st, info = c.piso(1)
        st_all = max(st_all, st)
        p_iters.append([s["iters"] for s in info["p"]])
        u_iters.append([s["iters"] for s in info["u"]])
        if steps <= 5 or (k + 1) % every == 0:
            log(f"{name}: step {k + 1}/{steps}, p iters so far {sum(map(sum, p_iters))}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return c, wall, p_iters, u_iters, st_all


def cav200_section(fvm, wl, n, steps, warmup, profile_steps, log):
    """The headline configuration, FP64 and mixed, plus FP64 with the AMG
    V-cycle preconditioning the pressure CG."""
    import numpy as np
    import torch
    t = time.perf_counter()
    spec = wl.cav200(n=n, n_steps=steps)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N, Fi = mesh.n_cells, mesh.n_internal
    sell = fvm.mesh_sell_info(mesh)
    dcells = diag_read_cells(spec, sell)
    log(f"cav{n} mesh: {N} cells, {Fi} internal faces in {time.perf_counter() - t:.1f}s; sliced ELL {sell}; "
        f"FP64 product reads the diagonal of {dcells} cells")
    if warmup > 0:
        w = fvm.Case(spec, mesh=mesh)
        w.piso(warmup)
        torch.cuda.synchronize()
        del w
        log(f"cav{n}: {warmup} warm-up steps done")
    res = {}
    fields = {}
    for name, prec in (("fp64", wl.FP64), ("mixed", wl.MIXED), ("amg_fp64", wl.FP64)):
        sp = spec.with_(precision=prec)
        if name == "amg_fp64":
            sp = sp.with_(p_ctl=wl.SolverCtl(sp.p_ctl.tol, sp.p_ctl.rel_tol, sp.p_ctl.max_iter, wl.PC_AMG))
        c, wall, p_iters, u_iters, st = run_steps(fvm, sp, mesh, steps, log, f"cav{n} {name}")
        U, p, phi = c.get_state_numpy()
        assert np.all(np.isfinite(U)) and np.all(np.isfinite(p)), f"non-finite fields ({name})"
        fields[name] = (U, p)
        del c
        k = {}
        if profile_steps > 0:
            pc = fvm.Case(sp, mesh=mesh)
            k = profile_classes(fvm, pc, profile_steps, N, Fi, False, sell, dcells)
            del pc
        pre = "pcg32" if prec == wl.MIXED else "pcg"
        it_us = sum(k[c_]["us_per_work"] for c_ in (pre + "_dir", pre + "_spmv", pre + "_update") if c_ in k)
        it_bytes = cg_iteration_bytes(N, Fi, sell, prec == wl.MIXED, dcells)
        ptot = int(sum(map(sum, p_iters)))
        spmv_cls = pre + "_spmv"
        tr = measured_traffic(spmv_cls, f"cav{n}") if name != "amg_fp64" else None
        r = dict(ms_per_step=round(1e3 * wall / steps, 2), cell_updates_per_s=round(N * steps / wall, 1),
                 status=st, p_iters_total=ptot, p_iters_per_solve=round(ptot / (steps * spec.n_corr), 1),
                 u_iters_first_last=[u_iters[0], u_iters[-1]],
                 ms_per_p_iteration=round(1e3 * wall / max(ptot, 1), 4),
                 spmv_us=k.get(spmv_cls, {}).get("us_per_work"),
                 spmv_alg_bytes=algorithmic_bytes(spmv_cls, N, Fi, sell, dcells),
                 spmv_alg_GBps=k.get(spmv_cls, {}).get("alg_GBps"),
                 spmv_counter_bytes=round(tr["bytes_per_working_launch"]) if tr else None,
                 spmv_counter_GBps=counter_GBps(tr),
                 cg_iter_us=round(it_us, 2) if it_us else None,
                 cg_iter_alg_bytes=it_bytes,
                 cg_iter_alg_GBps=round(it_bytes / (it_us * 1e-6) / 1e9, 1) if it_us else None,
                 assembly_vs_spmv=vs_spmv(k, spmv_cls), kernels=k)
        res[name] = r
        log(f"cav{n} {name}: {r['ms_per_step']} ms/step ({r['cell_updates_per_s']:.4g} cell-updates/s), p iters "
            f"{ptot}, SpMV {r['spmv_us']} us = {r['spmv_alg_GBps']} GB/s algorithmic, "
            f"{r['spmv_counter_GBps']} GB/s counters; CG iteration {r['cg_iter_us']} us = {r['cg_iter_alg_GBps']} GB/s")
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    res["mixed_vs_fp64_relL2"] = dict(U=rel(fields["mixed"][0], fields["fp64"][0]),
                                      p=rel(fields["mixed"][1], fields["fp64"][1]))
    res["amg_vs_fp64_relL2"] = dict(U=rel(fields["amg_fp64"][0], fields["fp64"][0]),
                                    p=rel(fields["amg_fp64"][1], fields["fp64"][1]))
    res["sliced_ell"] = dict(sell, fp64_diag_read_cells=dcells)
    res["workload"] = (f"cav{n}: 3-D lid-driven cavity {n}^3 hex cells, lexicographic, Re=1000, PISO dt=0.001, 2 "
                       f"correctors, {steps} steps from rest, PCG-Jacobi / PBiCG-Jacobi tol 1e-6 (normalised "
                       f"residual); mixed = FP32 inner (eta 1e-3) + FP64 refinement; amg_fp64 = FP64 with the "
                       f"AMG V-cycle preconditioning the pressure CG")
    return spec, mesh, res


def cpu_baseline_section(fvm, wl, spec, mesh, iters_per_step, log, k1=4, k2=16):
    """The FP64 oracle (compiled for this host, -O3 -march=native, one
    thread: its loops run in a fixed sequential order) on a prefix of the
    headline case: the first PISO step from rest with each pressure solve
    stopped after k1, then k2, CG iterations.  The difference of the two
    times gives the oracle's time per CG iteration, the rest its time for
    everything else in a step; a full step is extrapolated to the GPU run's
    mean pressure iterations per step (the oracle takes the same counts: the
    parity tests check them).  The GPU's time for the identical k2 prefix
    (same case, same cap, one step from rest) is reported beside it."""
    import torch
    from oracle import oracle as orc
    path = orc.select_native()
    log(f"cpu baseline: oracle built for this host ({path})")
    times = {}
    for K in (k1, k2):
        sp = spec.with_(p_ctl=wl.SolverCtl(spec.p_ctl.tol, spec.p_ctl.rel_tol, K, spec.p_ctl.precond))
        oc = orc.OracleCase(sp)
        t = time.perf_counter()
        st, info = oc.piso(1)
        times[K] = time.perf_counter() - t
        log(f"cpu baseline: oracle first step with pressure solves capped at {K} iterations: {times[K]:.2f}s "
            f"(p iters {[s['iters'] for s in info['p']]}, U iters {[s['iters'] for s in info['u']]})")
        del oc
    n_solves = spec.n_corr
    t_iter = (times[k2] - times[k1]) / (n_solves * (k2 - k1))
    t_rest = times[k1] - n_solves * k1 * t_iter
    t_step = t_rest + iters_per_step * t_iter
    N = mesh.n_cells
    sp = spec.with_(p_ctl=wl.SolverCtl(spec.p_ctl.tol, spec.p_ctl.rel_tol, k2, spec.p_ctl.precond))
    c = fvm.Case(sp, mesh=mesh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    c.piso(1)
    torch.cuda.synchronize()
    gpu_prefix = time.perf_counter() - t
    del c
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    model = model or platform.processor()
    out = dict(value=round(N / t_step, 1), unit="cell-updates/s", cores=1, kind="oracle",
               sample=(f"first PISO step from rest of the same {round(N ** (1 / 3))}^3 case with each pressure "
                       f"solve capped at {k1} and at {k2} CG iterations ({times[k1]:.2f}s and {times[k2]:.2f}s); "
                       f"per step extrapolated to the GPU run's {iters_per_step:.0f} CG iterations per step: "
                       f"{t_iter * 1e3:.1f} ms per CG iteration, {t_rest:.2f}s for the rest of a step, "
                       f"{t_step:.1f}s per step"),
               extrapolated=True, oracle_s_per_step=round(t_step, 3), oracle_ms_per_cg_iteration=round(t_iter * 1e3, 3),
               identical_prefix=dict(oracle_s=round(times[k2], 3), gpu_s=round(gpu_prefix, 4),
                                     what=f"first step from rest, pressure solves capped at {k2} iterations"),
               host_nproc=os.cpu_count(), host_cpu=model, build="gcc -std=c99 -O3 -march=native -ffp-contract=off",
               threads_note="the oracle is sequential by construction (its face loops scatter into cells and the "
                            "order of its sums defines its result)")
    log(f"cpu baseline: {out}")
    return out


def cav100_section(fvm, wl, steps, profile_steps, precond_compare, log):
    """The 1M-cell cavity with PCG-DIC (the configuration as named), its
    per-class kernel times, and the same steps with Jacobi and with the AMG
    V-cycle in place of DIC."""
    import torch
    t = time.perf_counter()
    spec = wl.cav100(n=100, n_steps=steps)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N, Fi = mesh.n_cells, mesh.n_internal
    sell = fvm.mesh_sell_info(mesh)
    log(f"cav100 mesh: {N} cells in {time.perf_counter() - t:.1f}s")
    out = {}
    variants = [("dic", wl.PC_DIC)] + ([("jacobi", wl.PC_JACOBI), ("amg", wl.PC_AMG)] if precond_compare else [])
    for name, pc in variants:
        sp = spec.with_(p_ctl=wl.SolverCtl(spec.p_ctl.tol, spec.p_ctl.rel_tol, spec.p_ctl.max_iter, pc))
        c, wall, p_iters, _, st = run_steps(fvm, sp, mesh, steps, log, f"cav100 {name}", every=10)
        del c
        its = sum(map(sum, p_iters))
        out[name] = dict(ms_per_step=round(1e3 * wall / steps, 2), cell_updates_per_s=round(N * steps / wall, 1),
                         p_iters_per_step=round(its / steps, 1), status=st)
        log(f"cav100 {name}: {out[name]['ms_per_step']} ms/step, {out[name]['p_iters_per_step']} CG iterations/step")
    if profile_steps > 0:
        pc_ = fvm.Case(spec, mesh=mesh)
        k = profile_classes(fvm, pc_, profile_steps, N, Fi, True, sell, diag_read_cells(spec, sell))
        del pc_
        out["kernels"] = k
        tr = {cls: measured_traffic(cls, "cav100") for cls in ("dic_fwd", "dic_bwd")}
        out["dic_sweeps"] = {cls: dict(us_per_work=k[cls]["us_per_work"], alg_GBps=k[cls]["alg_GBps"],
                                       counter_bytes=round(tr[cls]["bytes_per_working_launch"]) if tr[cls] else None)
                             for cls in ("dic_fwd", "dic_bwd") if cls in k}
        out["assembly_vs_spmv"] = vs_spmv(k, "pcg_spmv")
    out["workload"] = (f"cav100: 3-D lid-driven cavity 100^3 hex cells, random renumbering (seed 2) + RCM, Re=400, "
                       f"PISO dt=0.002, 2 correctors, PCG-DIC / PBiCG tol 1e-7, {steps} steps from rest, FP64 "
                       f"(jacobi, amg: the same with that pressure preconditioner)")
    return out


def cav2d32_section(fvm, wl, log):
    """The 2-D cavity configuration as named: 100 PISO steps from rest."""
    spec = wl.cav2d32()
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    c, wall, p_iters, _, st = run_steps(fvm, spec, mesh, spec.n_steps, log, "cav2d32", every=50)
    del c
    N = mesh.n_cells
    out = dict(workload="cav2d32: 2-D cavity 32x32x1, random renumbering (seed 1), Re=100, PISO dt=0.005, 2 "
                        "correctors, PCG-Jacobi / PBiCG tol 1e-8, 100 steps from rest, FP64",
               ms_per_step=round(1e3 * wall / spec.n_steps, 3), cell_updates_per_s=round(N * spec.n_steps / wall, 1),
               p_iters_per_step=round(sum(map(sum, p_iters)) / spec.n_steps, 1), status=st)
    log(f"cav2d32: {out}")
    return out


def duct_section(fvm, wl, max_iters, log, chunk=250):
    """Steady SIMPLE on the jittered 256x64x64 duct until every initial
    residual (U_x, U_y, U_z, p) of an iteration is <= 1e-6."""
    import numpy as np
    import torch
    t = time.perf_counter()
    spec = wl.duct256(max_iters=max_iters)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N = mesh.n_cells
    log(f"duct256 mesh: {N} cells (non-orthogonal: {mesh.non_orthogonal}) in {time.perf_counter() - t:.1f}s")
    c = fvm.Case(spec, mesh=mesh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    info = None
    while done < max_iters:
        st, it, info = c.simple(min(chunk, max_iters - done), spec.res_tol)
        done += it
        res = [info["u"][k]["res_initial"] for k in range(3)] + [info["p"][0]["res_initial"]]
        log(f"duct256: {done} SIMPLE iterations, initial residuals {['%.2e' % r for r in res]}")
        if max(res) <= spec.res_tol or it < min(chunk, max_iters - done + it):
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    U, p, phi = c.get_state_numpy()
    del c
    m = spec.mesh
    s_in, n_in = m.patch("xmin")
    s_out, n_out = m.patch("xmax")
    q_in, q_out = phi[s_in:s_in + n_in].sum(), phi[s_out:s_out + n_out].sum()
    res = [info["u"][k]["res_initial"] for k in range(3)] + [info["p"][0]["res_initial"]]
    out = dict(workload="duct256: square duct 256x64x64 on [0,4]x[0,1]^2, interior vertices jittered +-0.15h "
                        "(seed 3), Re=50 plug inflow, steady SIMPLE (alpha_U 0.7, alpha_p 0.3; p PCG-Jacobi tol 1e-8 "
                        "rel 0.05, U PBiCG-Jacobi tol 1e-8 rel 0.1) until every initial residual <= 1e-6, FP64",
               iterations=done, converged=bool(max(res) <= spec.res_tol), final_initial_residuals=res,
               seconds_to_converge=round(wall, 2), cell_updates_per_s=round(N * done / wall, 1),
               ms_per_iteration=round(1e3 * wall / max(done, 1), 3),
               mass_balance=float(abs(q_in + q_out) / abs(q_in)), finite=bool(np.isfinite(U).all()))
    log(f"duct256: {out}")
    return out


def tp_section(fvm, wl, steps, log):
    """tp1M: the transient 2-D pipe, 3200 x 300 cells (960 000), sinusoidal
    inlet set before every step, `steps` PISO steps from rest (the paper
    runs 5000), FP64, PCG-Jacobi / PBiCG-Jacobi tol 1e-6."""
    import numpy as np
    import torch
    t = time.perf_counter()
    spec = wl.tp1m(n_steps=steps)
    mesh = fvm.Mesh(spec.mesh, spec.bcs)
    N = mesh.n_cells
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


def serve_section(fvm, wl, n_requests, n_steps, log, precisions=("fp64", "mixed")):
    """Serving stream (cavity/duct cases, cube side log-uniform 16..96,
    Re U(10, 1000), Poisson arrivals at 40 req/s), `n_requests` requests of
    `n_steps` PISO steps, run once in FP64 and once mixed: p50 / p99 time
    from arrival to converged result, throughput."""
    import torch
    from paper_1207_1571_amd.serve import GpuBackend, Request, Server, summarize
    reqs = wl.serve_stream(n_requests=n_requests, n_steps=n_steps)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    out = dict(workload=f"serve: {n_requests} requests of the 512-request stream (seed 5; cavity/duct, side "
                        f"log-uniform 16..96, Re U(10,1000), Poisson 40 req/s), {n_steps} PISO steps each (the "
                        f"configuration names 200), tol 1e-6, Jacobi",
               budget_bytes=budget, steps_per_request=n_steps)
    for name, prec in (("fp64", wl.FP64), ("mixed", wl.MIXED)):
        if name not in precisions:
            continue
        t = time.perf_counter()
        specs = [wl.serve_case(r, precision=prec) for r in reqs]
        log(f"serve {name}: {len(specs)} case meshes in {time.perf_counter() - t:.1f}s")
        be = GpuBackend()
        done = [0]

        def progress(msg):
            done[0] += 1
            if done[0] % 32 == 0:
                log(f"serve {name}: {done[0]} requests done ({msg})")

        srv = Server(be, budget, slots=256, group=32, chunk=40)
        res = srv.run([Request(r.rid, r.arrival_s, s, r.n_steps) for r, s in zip(reqs, specs)], log=progress)
        torch.cuda.synchronize()
        sm = summarize(res)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sm.items()}
        out[name]["server"] = getattr(srv, "describe", lambda: None)()
        log(f"serve {name}: p50 {sm['p50_s']:.3f}s p99 {sm['p99_s']:.3f}s, makespan {sm['makespan_s']:.2f}s, "
            f"{sm['cell_updates_per_s']:.4g} cell-updates/s, failed {sm['failed']}")
        del be, specs, res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="PISO steps of the headline 200^3 cavity")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=200, help="cube side of the headline cavity (200 = the configuration)")
    ap.add_argument("--profile-steps", type=int, default=2, help="steps of the per-kernel-class timing passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cav100-steps", type=int, default=50, help="steps of the 1M-cell PCG-DIC cavity (0: skip)")
    ap.add_argument("--no-precond-compare", dest="precond_compare", action="store_false",
                    help="skip the runs of the 1M-cell cavity with Jacobi and AMG in place of DIC")
    ap.add_argument("--no-cav2d32", dest="cav2d32", action="store_false")
    ap.add_argument("--duct-iters", type=int, default=4000,
                    help="SIMPLE iteration cap of the 256x64x64 duct (stops at residual 1e-6; 0: skip)")
    ap.add_argument("--tp-steps", type=int, default=10, help="PISO steps of the tp1M transient pipe section (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=512, help="requests of the serving section (0: skip)")
    ap.add_argument("--serve-steps", type=int, default=20, help="PISO steps per serving request")
    ap.add_argument("--serving-only", choices=["fp64", "mixed", "both"], default=None,
                    help="run only the serving stream (in that precision) and print its JSON section")
    ap.add_argument("--no-layouts", dest="layouts", action="store_false",
                    help="skip the face-major vs hybrid layout operator comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1207_1571_amd import fvm
    from paper_1207_1571_amd import workloads as wl

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.serving_only:
        precs = ("fp64", "mixed") if args.serving_only == "both" else (args.serving_only,)
        serving = serve_section(fvm, wl, args.serve_requests, args.serve_steps, log, precs)
        print(json.dumps({"serving": serving}), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")
        del src, dst

    spec, mesh, cav = cav200_section(fvm, wl, args.n, args.steps, args.warmup, args.profile_steps, log)
    N, Fi = mesh.n_cells, mesh.n_internal
    fp, mx = cav["fp64"], cav["mixed"]
    wall = fp["ms_per_step"] * args.steps / 1e3
    value = fp["cell_updates_per_s"]
    k = fp["kernels"]
    roofline = None
    if k:
        dom = max(k, key=lambda c_: k[c_]["total_ms"])
        tr = measured_traffic(dom, f"cav{args.n}")
        ach = k[dom]["alg_GBps"]
        roofline = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(ach / HBM_PEAK_GBS, 4) if ach else None,
                        traffic=round(tr["bytes_per_working_launch"]) if tr else None,
                        traffic_GBps=counter_GBps(tr),
                        traffic_frac=round(counter_GBps(tr) / HBM_PEAK_GBS, 4) if counter_GBps(tr) else None,
                        algorithmic_bytes=k[dom]["alg_bytes"], us_per_working_launch=k[dom]["us_per_work"])
    iters_per_step = fp["p_iters_total"] / args.steps
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_section(fvm, wl, spec, mesh, iters_per_step, log)
    del mesh
    c2d = cav2d32_section(fvm, wl, log) if args.cav2d32 else None
    c100 = (cav100_section(fvm, wl, args.cav100_steps, args.profile_steps, args.precond_compare, log)
            if args.cav100_steps > 0 else None)
    duct = duct_section(fvm, wl, args.duct_iters, log) if args.duct_iters > 0 else None
    tp = tp_section(fvm, wl, args.tp_steps, log) if args.tp_steps > 0 else None
    layouts = layout_section(fvm, wl, log) if args.layouts else None
    serving = serve_section(fvm, wl, args.serve_requests, args.serve_steps, log) if args.serve_requests > 0 else None

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
        "config": {"workload": f"cav{args.n}: 3-D lid-driven cavity {args.n}^3 hex cells, lexicographic, Re=1000, "
                               f"PISO dt=0.001, 2 correctors, PCG-Jacobi / PBiCG-Jacobi to normalised residual 1e-6, "
                               f"{args.steps} steps from rest",
                   "cells": N, "internal_faces": Fi, "precision": "fp64"},
        "mixed": dict(cell_updates_per_s=mx["cell_updates_per_s"], ms_per_step=mx["ms_per_step"],
                      speedup_vs_fp64=round(fp["ms_per_step"] / mx["ms_per_step"], 3),
                      ms_per_p_iteration=mx["ms_per_p_iteration"], p_iters_total=mx["p_iters_total"],
                      fp64_p_iters_total=fp["p_iters_total"], relL2_vs_fp64=cav["mixed_vs_fp64_relL2"],
                      dtype="f32 inner Krylov / f64 refinement, dots, corrections"),
        "pcg_spmv": dict(fp64_alg_GBps=fp["spmv_alg_GBps"], fp64_counter_GBps=fp["spmv_counter_GBps"],
                         mixed_alg_GBps=mx["spmv_alg_GBps"], mixed_counter_GBps=mx["spmv_counter_GBps"],
                         fp64_frac_of_peak_counter=(round(fp["spmv_counter_GBps"] / HBM_PEAK_GBS, 4)
                                                    if fp["spmv_counter_GBps"] else None)),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cav200": cav,
        "cav2d32": c2d,
        "cav100": c100,
        "duct256": duct,
        "tp1m": tp,
        "serving": serving,
        "layouts": layouts,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
