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

Lanes: a backend may sort cases into lanes that advance independently and
concurrently (one host thread and one stream each).  The GPU backend has
two: small cases that run whole PISO steps in one workgroup each (one launch
advances up to 32 of them by several steps, side by side on separate
compute units), and the others, advanced by launched phases; so the small
cases of a stream overlap with the large ones on the device instead of
waiting for them.

Time is wall-clock from the start of run(); arrival times are honoured (a
request is not admitted before it arrives).  latency = completion - arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
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

    # lane -> (cases per advance, steps per advance)
    LANES = {"solo": (32, 40), "launched": (32, 20)}

    def __init__(self, device="cuda", keep_fields: bool = False, lanes: bool = True):
        import torch
        from . import fvm
        self.torch = torch
        self.fvm = fvm
        self.device = device
        self.keep_fields = keep_fields
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.lane_streams = {k: torch.cuda.Stream(device=device) for k in self.LANES}
        self._meshes: Dict[int, object] = {}
        self._mu = threading.Lock()
        if not lanes:
            self.lane_of = None

    def lane_of(self, spec) -> str:
        """'solo' for a case that runs whole steps in one workgroup
        (FVM_STEP_AUTO: at most 32 768 cells, orthogonal, Jacobi CG, BiCG,
        at most 4 correctors), else 'launched'."""
        fvm = self.fvm
        with self._mu:
            m = self._meshes.get(id(spec))
        solo = (getattr(spec, "step_kernel", 0) == fvm.STEP_AUTO and spec.mesh.n_cells <= 32768
                and spec.n_non_orth_corr == 0 and spec.n_corr <= 4 and spec.p_ctl.precond == fvm.PC_JACOBI
                and getattr(spec, "u_solver", 0) == 0 and not (m.non_orthogonal if m is not None else False))
        return "solo" if solo else "launched"

    def footprint(self, spec) -> int:
        with self._mu:
            m = self._meshes.get(id(spec))
        if m is None:
            m = self.fvm.Mesh(spec.mesh, spec.bcs)
            with self._mu:
                self._meshes[id(spec)] = m
        return self.fvm.workspace_bytes(m, self.fvm.opts_from_case(spec))

    def create(self, spec):
        """The case's workspace and uploads are enqueued on the admission
        stream; the call returns once they are complete, because the case is
        then advanced on a lane's stream."""
        with self._mu:
            mesh = self._meshes.pop(id(spec), None)
        with self.torch.cuda.stream(self.stream):
            case = self.fvm.Case(spec, device=self.device, stream=self.stream, mesh=mesh)
        self.stream.synchronize()
        return case

    def advance(self, cases: Sequence, n_steps: int, lane: Optional[str] = None) -> List[dict]:
        """piso_step_batch over sub-batches of cases that may share launches
        (same precision, correctors, pressure preconditioner, momentum
        solver and step kernel; AMG cases one at a time), on the lane's
        stream."""
        fvm = self.fvm
        stream = self.lane_streams.get(lane, self.stream)
        subs: Dict[tuple, List[int]] = {}
        for k, c in enumerate(cases):
            o = c.opts
            key = (o.precision, o.n_corr, o.n_non_orth_corr, o.p_ctl.precond, o.u_solver, lane)
            if o.p_ctl.precond == fvm.PC_AMG:
                key = key + (k,)
            subs.setdefault(key, []).append(k)
        infos: List[dict] = [None] * len(cases)
        for idx in subs.values():
            st, part = fvm.piso_batch([cases[k] for k in idx], n_steps, stream=stream,
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
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 order: str = "size"):
        if slots < 1 or group < 1 or chunk < 1:
            raise ValueError("slots, group and chunk must be positive")
        if order not in ("size", "id"):
            raise ValueError("order must be 'size' or 'id'")
        # lanes walk their resident cases round-robin in this order: by cell
        # count ("size"), so a group holds cases of similar size, whose
        # solves end after similar iteration counts (a shared launch runs
        # until its slowest case is done), or by request id
        self.order = order
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

    def describe(self) -> dict:
        lanes = getattr(self.backend, "LANES", None) if getattr(self.backend, "lane_of", None) else None
        return dict(slots=self.slots, group=self.group, chunk=self.chunk, order=self.order,
                    lanes={k: dict(group=min(g, self.group), chunk=min(c, self.chunk)) for k, (g, c) in lanes.items()}
                    if lanes else None)

    def run(self, requests: Sequence[Request], log: Optional[Callable[[str], None]] = None) -> List[Result]:
        """Serve every request; one that cannot be admitted (invalid, larger
        than the whole budget, or failing at creation) comes back at once
        with a negative status, and the others go on."""
        if getattr(self.backend, "lane_of", None):
            return self._run_lanes(requests, log)
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


    def _run_lanes(self, requests: Sequence[Request], log) -> List[Result]:
        """Admission on the calling thread; one worker thread per lane
        advances the lane's resident cases round-robin (the backend's group
        size and step count per lane, capped by the server's).  Shared state is guarded by one
        condition variable; device work and case set-up run outside it."""
        self.rejections = []
        lanes = dict(self.backend.LANES)
        cv = threading.Condition()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        active: Dict[int, dict] = {}
        results: List[Result] = []
        state = dict(used=0, stop=False, error=None)
        foot_cache: Dict[int, int] = {}
        t0 = self.clock()

        def finish(batch):
            for a in batch:
                fields = self.backend.finish(a["case"])
                done = self.clock() - t0
                req = a["req"]
                res = Result(req.rid, req.arrival_s, a["admitted"], done, req.spec.mesh.n_cells, req.n_steps,
                             a["bytes"], a["status"], a["p_iters"], fields)
                with cv:
                    results.append(res)
                    state["used"] -= a["bytes"]
                    del active[req.rid]
                    cv.notify_all()
                if log:
                    log(f"done rid={req.rid} N={req.spec.mesh.n_cells} latency={done - req.arrival_s:.3f}s")

        def worker(lane):
            group, chunk = min(lanes[lane][0], self.group), min(lanes[lane][1], self.chunk)
            rr = 0
            try:
                while True:
                    with cv:
                        while True:
                            ids = sorted((r for r, a in active.items() if a["lane"] == lane),
                                         key=(lambda r: (active[r]["req"].spec.mesh.n_cells, r)) if self.order == "size"
                                         else None)
                            if ids or state["stop"]:
                                break
                            cv.wait(0.05)
                        if not ids or state["error"] is not None:
                            return
                        take = [ids[(rr + k) % len(ids)] for k in range(min(group, self.slots, len(ids)))]
                        rr = (rr + len(take)) % max(1, len(ids))
                        steps = min(chunk, min(active[i]["left"] for i in take))
                        batch = [active[i] for i in take]
                    infos = self.backend.advance([a["case"] for a in batch], steps, lane)
                    done = []
                    with cv:
                        for a, info in zip(batch, infos):
                            a["left"] -= steps
                            a["p_iters"] += sum(s["iters"] for s in info["p"]) if info else 0
                            if info and info["status"] < 0:
                                a["status"] = info["status"]
                                a["left"] = 0
                            if a["left"] <= 0:
                                done.append(a)
                    finish(done)
            except BaseException as e:     # surfaced by run()
                with cv:
                    state["error"] = e
                    state["stop"] = True
                    cv.notify_all()

        threads = [threading.Thread(target=worker, args=(k,), daemon=True) for k in lanes]
        for t in threads:
            t.start()
        try:
            while True:
                with cv:
                    if state["error"] is not None:
                        break
                    if not pending and not active:
                        break
                    now = self.clock() - t0
                    req = pending[0] if pending and pending[0].arrival_s <= now and len(active) < self.slots else None
                    if req is None:
                        wait = (pending[0].arrival_s - now) if pending and len(active) < self.slots else 0.05
                        cv.wait(max(1e-3, min(wait, 0.05)))
                        continue
                    need = foot_cache.get(req.rid)
                # price and create outside the lock (host mesh work, uploads)
                if need is None:
                    try:
                        need = foot_cache[req.rid] = int(self.backend.footprint(req.spec))
                    except Exception as e:
                        with cv:
                            pending.popleft()
                            results.append(self._rejected(req, t0, STATUS_EINVAL, f"footprint: {e}"))
                        continue
                with cv:
                    if need > self.budget:
                        pending.popleft()
                        results.append(self._rejected(req, t0, STATUS_ENOMEM,
                                                      f"needs {need} bytes, more than the whole budget {self.budget}"))
                        continue
                    if state["used"] + need > self.budget:
                        cv.wait(0.05)
                        continue
                    pending.popleft()
                    state["used"] += need
                try:
                    case = self.backend.create(req.spec)
                    lane = self.backend.lane_of(req.spec)
                except Exception as e:
                    with cv:
                        state["used"] -= need
                        results.append(self._rejected(req, t0, STATUS_EINVAL, f"create: {e}"))
                    continue
                with cv:
                    active[req.rid] = dict(req=req, case=case, bytes=need, left=req.n_steps, lane=lane,
                                           admitted=self.clock() - t0, p_iters=0, status=0)
                    cv.notify_all()
        finally:
            with cv:
                state["stop"] = True
                cv.notify_all()
            for t in threads:
                t.join()
        if state["error"] is not None:
            raise state["error"]
        return results


def summarize(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency_s for r in results])
    if lat.size == 0:
        return {}
    span = max(r.done_s for r in results) - min(r.arrival_s for r in results)
    cu = sum(r.n_cells * r.n_steps for r in results if r.status >= 0)
    return dict(n=len(results), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), max_s=float(lat.max()), makespan_s=float(span),
                cases_per_s=float(len(results) / span) if span > 0 else None,
                cell_updates_per_s=float(cu / span) if span > 0 else None,
                failed=int(sum(1 for r in results if r.status < 0)),
                failures=[dict(rid=r.rid, n_cells=r.n_cells, status=r.status) for r in results if r.status < 0])
