"""Serving loop: many independent cases resident on one GPU.

Requests arrive over time (each: a case and a number of PISO steps).  The
server admits a request when a slot is free and its exact device footprint
(fvm_case_workspace_bytes) fits in the memory budget next to the cases
already resident; admitted cases keep their fields and matrices on the device
until they finish, and requests that arrive while others are running are
admitted as soon as slots and memory free up (continuous batching: the set
of cases on the device changes while work is in flight).

Small cases cannot fill the GPU alone, so resident cases are advanced
together: the slots are served round-robin in groups, and each group's PISO
steps are issued through piso_step_batch, whose kernels process all the
cases of the group in shared launches.  A case's result does not depend on
which other cases share its launches (per-case reductions, fixed order).

Time is wall-clock from the start of run(); arrival times are honoured (a
request is not admitted before it arrives).  latency = completion - arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    spec: object                 # a workloads.CaseSpec
    n_steps: int


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    admitted_s: float
    done_s: float
    n_cells: int
    n_steps: int
    bytes: int
    status: int
    p_iters: int                 # pressure CG iterations of the last step of each advance
    fields: Optional[tuple] = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class GpuBackend:
    """Cases in libfvm; advances groups of resident cases with piso_step_batch.

    The host mesh (validation, canonical faces, sliced-ELL structure) built
    to price a request is kept and reused when the request is admitted."""

    def __init__(self, device="cuda", keep_fields: bool = False):
        import torch
        from . import fvm
        self.torch = torch
        self.fvm = fvm
        self.device = device
        self.keep_fields = keep_fields
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self._meshes: Dict[int, object] = {}

    def footprint(self, spec) -> int:
        m = self._meshes.get(id(spec))
        if m is None:
            m = self._meshes[id(spec)] = self.fvm.Mesh(spec.mesh, spec.bcs)
        return self.fvm.workspace_bytes(m, self.fvm.opts_from_case(spec))

    def create(self, spec):
        mesh = self._meshes.pop(id(spec), None)
        with self.torch.cuda.stream(self.stream):
            return self.fvm.Case(spec, device=self.device, stream=self.stream, mesh=mesh)

    def advance(self, cases: Sequence, n_steps: int) -> List[dict]:
        """piso_step_batch over sub-batches of cases that may share launches
        (same precision, correctors, pressure preconditioner and momentum
        solver; AMG cases one at a time)."""
        fvm = self.fvm
        subs: Dict[tuple, List[int]] = {}
        for k, c in enumerate(cases):
            o = c.opts
            key = (o.precision, o.n_corr, o.n_non_orth_corr, o.p_ctl.precond, o.u_solver)
            if o.p_ctl.precond == fvm.PC_AMG:
                key = key + (k,)
            subs.setdefault(key, []).append(k)
        infos: List[dict] = [None] * len(cases)
        for idx in subs.values():
            st, part = fvm.piso_batch([cases[k] for k in idx], n_steps, stream=self.stream,
                                      raise_on_case_failure=False)
            for k, info in zip(idx, part):
                infos[k] = info
        return infos

    def finish(self, case):
        fields = case.get_state_numpy() if self.keep_fields else None
        case.close()
        return fields


# status of a request that was never admitted (the values of the C interface)
STATUS_EINVAL, STATUS_ENOMEM = -1, -2


class Server:
    """Admission by device footprint and slots; round-robin stepping of
    resident cases in groups of `group` cases, `chunk` steps at a time."""

    def __init__(self, backend, budget_bytes: int, slots: int = 32, group: int = 16, chunk: int = 10,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        if slots < 1 or group < 1 or chunk < 1:
            raise ValueError("slots, group and chunk must be positive")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.group = int(group)
        self.chunk = int(chunk)
        self.clock = clock
        self.sleep = sleep

    def _rejected(self, req: Request, t0: float, status: int, why: str) -> Result:
        now = self.clock() - t0
        self.rejections.append((req.rid, why))
        return Result(req.rid, req.arrival_s, now, now, getattr(req.spec.mesh, "n_cells", 0), req.n_steps, 0, status,
                      0, None)

    def run(self, requests: Sequence[Request], log: Optional[Callable[[str], None]] = None) -> List[Result]:
        """Serve every request; one that cannot be admitted (invalid, larger
        than the whole budget, or failing at creation) comes back at once
        with a negative status, and the others go on."""
        self.rejections = []
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        active: Dict[int, dict] = {}
        results: List[Result] = []
        used = 0
        t0 = self.clock()
        rr = 0
        foot_cache: Dict[int, int] = {}
        while pending or active:
            now = self.clock() - t0
            # admit in arrival order while a slot and memory are free
            while pending and pending[0].arrival_s <= now and len(active) < self.slots:
                req = pending[0]
                need = foot_cache.get(req.rid)
                if need is None:
                    try:
                        need = foot_cache[req.rid] = int(self.backend.footprint(req.spec))
                    except Exception as e:   # invalid mesh or options: reject this request only
                        pending.popleft()
                        results.append(self._rejected(req, t0, STATUS_EINVAL, f"footprint: {e}"))
                        continue
                if need > self.budget:
                    pending.popleft()
                    results.append(self._rejected(req, t0, STATUS_ENOMEM,
                                                  f"needs {need} bytes, more than the whole budget {self.budget}"))
                    continue
                if used + need > self.budget:
                    break
                pending.popleft()
                try:
                    case = self.backend.create(req.spec)
                except Exception as e:       # e.g. a hierarchy that cannot be built for this mesh
                    results.append(self._rejected(req, t0, STATUS_EINVAL, f"create: {e}"))
                    continue
                used += need
                active[req.rid] = dict(req=req, case=case, bytes=need, left=req.n_steps, admitted=self.clock() - t0,
                                       p_iters=0, status=0)
            if not active:
                if not pending:
                    break
                # idle until the next arrival
                wait = pending[0].arrival_s - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 0.05))
                continue
            # advance one group of resident cases (round-robin)
            ids = sorted(active)
            take = [ids[(rr + k) % len(ids)] for k in range(min(self.group, len(ids)))]
            rr = (rr + len(take)) % max(1, len(ids))
            steps = min(self.chunk, min(active[i]["left"] for i in take))
            infos = self.backend.advance([active[i]["case"] for i in take], steps)
            for i, info in zip(take, infos):
                a = active[i]
                a["left"] -= steps
                a["p_iters"] += sum(s["iters"] for s in info["p"]) if info else 0
                if info and info["status"] < 0:
                    a["status"] = info["status"]
                    a["left"] = 0
            for i in take:
                a = active[i]
                if a["left"] <= 0:
                    fields = self.backend.finish(a["case"])
                    done = self.clock() - t0
                    req = a["req"]
                    results.append(Result(req.rid, req.arrival_s, a["admitted"], done, req.spec.mesh.n_cells,
                                          req.n_steps, a["bytes"], a["status"], a["p_iters"], fields))
                    used -= a["bytes"]
                    del active[i]
                    if log:
                        log(f"done rid={req.rid} N={req.spec.mesh.n_cells} latency={done - req.arrival_s:.3f}s")
        return results


def summarize(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency_s for r in results])
    if lat.size == 0:
        return {}
    span = max(r.done_s for r in results) - min(r.arrival_s for r in results)
    cu = sum(r.n_cells * r.n_steps for r in results)
    return dict(n=len(results), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), max_s=float(lat.max()), makespan_s=float(span),
                cases_per_s=float(len(results) / span) if span > 0 else None,
                cell_updates_per_s=float(cu / span) if span > 0 else None,
                failed=int(sum(1 for r in results if r.status < 0)))
