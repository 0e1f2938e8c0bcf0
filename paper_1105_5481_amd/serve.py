"""Continuous-batching server for KPM density-of-states requests.

Requests (a lattice or CSR Hamiltonian, M moments, R start vectors) arrive over time.  The
loop below admits them first-come first-served while their device footprint (operator plus
workspace, from the C ABI's kpm_request_bytes) fits the HBM budget and a batch slot is free.
An admitted request gets its spectral bounds (device Gershgorin, or the tighter device Lanczos
interval on request), its operator (kpm_build) and
a begun solve whose vector state stays resident in its workspace.  Every loop iteration
enqueues one chunk of recursion steps through kpm_batch_advance: each launch of the chunk covers
all in-flight solves of an operator class, each at its own step, so requests that arrive while
others run share the device immediately.  Finished solves leave the batch, run the moment
reduction and the Jackson DoS, and are retired once their completion event has fired; their
memory returns to the budget.  A solve whose moments come back non-finite or above 1 in modulus
(a scale that does not enclose the spectrum) is reported with status "bounds" without
disturbing its neighbours.

All device work goes through the C ABI (paper_1105_5481_amd); this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import F32, F64, VEC_RADEMACHER, Batch, Hamiltonian, KPMError, Solve, dos, gershgorin, lanczos_scale, \
    request_bytes, scale_from_bounds


@dataclass(eq=False)
class KPMRequest:
    op: object                      # workloads.Lattice or workloads.CSR
    M: int
    R: int
    vec: int = VEC_RADEMACHER
    seed: int = 0
    instance: int = 0
    K_dos: int = 0                  # DoS points (0: 2M)
    eps: float = 0.01               # spectral margin of the scale
    scale: Optional[Tuple[float, float]] = None   # explicit (a, b); else from `bounds`
    bounds: str = "gershgorin"      # "gershgorin" or "lanczos" (interval from lanczos_k steps)
    lanczos_k: int = 100
    arrival: float = 0.0            # seconds (wall clock) or chunk index (chunk clock)
    rid: int = -1


@dataclass
class KPMResult:
    rid: int
    status: str                     # ok | bounds | oom | cancelled | error
    mu: Optional[np.ndarray] = None
    omega: Optional[np.ndarray] = None
    rho: Optional[np.ndarray] = None
    a: float = 0.0
    b: float = 0.0
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    message: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass(eq=False)
class _Live:
    req: KPMRequest
    bytes: int
    ham: Hamiltonian
    solve: Solve
    t_admit: float
    mu: object = None
    om: object = None
    rho: object = None
    event: object = None
    keep: List = field(default_factory=list)


class Server:
    """prec: recursion precision (F32 served path, F64 plain path); max_active: batch slots;
    chunk: recursion steps per loop iteration; hbm_budget: bytes (default 80% of free memory)."""

    def __init__(self, prec: int = F32, max_active: int = 64, chunk: int = 32, hbm_budget: Optional[int] = None,
                 device: str = "cuda"):
        import torch
        self.torch = torch
        self.prec, self.max_active, self.chunk, self.device = prec, max_active, chunk, device
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.hbm_budget = int(hbm_budget)
        self.used = 0
        self.batch = Batch(capacity=max_active)
        self.stream = torch.cuda.current_stream()
        self.pending: deque = deque()
        self.active: List[_Live] = []
        self.retiring: List[_Live] = []
        self.results: Dict[int, KPMResult] = {}
        self.arrivals: Dict[int, float] = {}
        self.chunk_log: List[Tuple[float, List[int]]] = []   # (time, rids in the chunk's launches)
        self.max_concurrent = 0
        self._next_rid = 0
        self._cancel = set()
        self._clock0 = time.perf_counter()
        self._chunks = 0
        self._clock_mode = "wall"
        self._inflight = deque()

    # ------------------------------------------------------------------ clock
    def now(self) -> float:
        if self._clock_mode == "chunks":
            return float(self._chunks)
        return time.perf_counter() - self._clock0

    # --------------------------------------------------------------- requests
    def submit(self, req: KPMRequest) -> int:
        if req.rid < 0:
            req.rid = self._next_rid
        self._next_rid = max(self._next_rid, req.rid) + 1
        self.arrivals[req.rid] = self.now()
        self.pending.append(req)
        return req.rid

    def cancel(self, rid: int):
        self._cancel.add(rid)

    # ------------------------------------------------------------- scheduling
    def _footprint(self, req: KPMRequest) -> int:
        op = req.op
        inputs = 0
        if getattr(op, "onsite", None) is not None:
            inputs += op.onsite.nbytes
        if getattr(op, "spinor", None) is not None:
            inputs += op.spinor.nbytes
        if hasattr(op, "row_ptr"):
            inputs += op.row_ptr.nbytes + op.col.nbytes + op.val_re.nbytes + (op.val_im.nbytes if op.val_im is not None else 0)
        K = req.K_dos or 2 * req.M
        return request_bytes(op, self.prec, req.M, req.R, req.vec) + inputs + 8 * (req.M + 2 * K)

    def _admit(self):
        while self.pending and len(self.active) < self.max_active:
            req = self.pending[0]
            if req.rid in self._cancel:
                self.pending.popleft()
                self._finish_result(req, "cancelled", t_admit=self.now())
                continue
            try:
                need = self._footprint(req)
            except KPMError as e:
                self.pending.popleft()
                self._finish_result(req, "error", message=str(e))
                continue
            if need > self.hbm_budget:
                self.pending.popleft()
                self._finish_result(req, "oom", message=f"needs {need} bytes, budget {self.hbm_budget}")
                continue
            if self.used + need > self.hbm_budget:
                break                                   # first come, first served
            self.pending.popleft()
            t_admit = self.now()
            ham = solve = None
            try:
                if req.scale is not None:
                    a, b = req.scale
                elif req.bounds == "lanczos":
                    a, b = lanczos_scale(req.op, req.lanczos_k, req.eps, device=self.device)
                else:
                    lo, hi = gershgorin(req.op, self.device)
                    a, b = scale_from_bounds(lo, hi, req.eps)
                ham = Hamiltonian(req.op, a, b, self.prec, self.device)
                solve = Solve(ham, req.M, req.R, req.vec, req.seed, req.instance)
            except KPMError as e:          # e.g. a CSR structure the device check rejects
                if solve is not None:
                    solve.close()
                if ham is not None:
                    ham.free()
                self._finish_result(req, "error", t_admit=t_admit, message=str(e))
                continue
            live = _Live(req=req, bytes=need, ham=ham, solve=solve, t_admit=t_admit)
            self.used += need
            if solve.remaining > 0:
                self.batch.add(solve)
            self.active.append(live)

    def _launch_chunk(self):
        members = [lv for lv in self.active if lv.solve.remaining > 0]
        self.max_concurrent = max(self.max_concurrent, len(members))
        if members:
            self.batch.advance(self.chunk)
            self.chunk_log.append((self.now(), [lv.req.rid for lv in members]))
        self._chunks += 1

    def _retire(self):
        torch = self.torch
        still = []
        for lv in self.active:
            cancelled = lv.req.rid in self._cancel
            if lv.solve.remaining > 0 and not cancelled:
                still.append(lv)
                continue
            if lv.solve in self.batch.members:
                self.batch.remove(lv.solve)
            if cancelled:
                lv.event = torch.cuda.Event()
                lv.event.record(self.stream)
                lv.mu = None
            else:
                K = lv.req.K_dos or 2 * lv.req.M
                lv.mu = lv.solve.finish()
                lv.om, lv.rho = dos(lv.mu, K, lv.ham.a, lv.ham.b)
                lv.event = torch.cuda.Event()
                lv.event.record(self.stream)
            self.retiring.append(lv)
        self.active = still
        done = []
        for lv in self.retiring:
            if not lv.event.query():
                continue
            done.append(lv)
            if lv.mu is None:
                self._finish_result(lv.req, "cancelled", t_admit=lv.t_admit, a=lv.ham.a, b=lv.ham.b)
            else:
                mu = lv.mu.cpu().numpy()
                ok = bool(np.all(np.isfinite(mu)) and np.abs(mu).max() <= 1.0 + (1e-4 if self.prec == F32 else 1e-9))
                self._finish_result(lv.req, "ok" if ok else "bounds", mu=mu, omega=lv.om.cpu().numpy(),
                                    rho=lv.rho.cpu().numpy(), t_admit=lv.t_admit, a=lv.ham.a, b=lv.ham.b,
                                    message="" if ok else "moments diverged: the scale does not enclose the spectrum")
            lv.solve.close()
            lv.ham.free()
            lv.solve = lv.ham = lv.mu = lv.om = lv.rho = None
            self.used -= lv.bytes
        done_ids = {id(lv) for lv in done}
        self.retiring = [lv for lv in self.retiring if id(lv) not in done_ids]

    def _finish_result(self, req, status, mu=None, omega=None, rho=None, t_admit=0.0, a=0.0, b=0.0, message=""):
        self.results[req.rid] = KPMResult(rid=req.rid, status=status, mu=mu, omega=omega, rho=rho, a=a, b=b,
                                          t_arrival=self.arrivals.get(req.rid, 0.0), t_admit=t_admit,
                                          t_done=self.now(), message=message)

    def busy(self) -> bool:
        return bool(self.pending or self.active or self.retiring)

    def step(self):
        """One scheduling iteration: admit, enqueue one chunk, retire what completed.  The host
        keeps at most two chunks in flight so admission decisions follow the device."""
        self._admit()
        self._launch_chunk()
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self._inflight.append(ev)
        while len(self._inflight) > 2:
            self._inflight.popleft().synchronize()
        self._retire()

    def run(self, requests: List[KPMRequest], clock: str = "wall", timeout: float = 3600.0, progress=None,
            progress_every: float = 30.0) -> List[KPMResult]:
        """Serve `requests` (arrival in seconds for clock="wall", in chunks for clock="chunks").
        progress: optional callable receiving a status line every `progress_every` seconds."""
        self._clock_mode = clock
        self._clock0 = time.perf_counter()
        self._chunks = 0
        queue = deque(sorted(requests, key=lambda r: r.arrival))
        t_start = time.perf_counter()
        t_note = t_start
        while queue or self.busy():
            now = self.now()
            while queue and queue[0].arrival <= now:
                req = queue.popleft()
                rid = self.submit(req)
                self.arrivals[rid] = req.arrival      # latency counts from the nominal arrival
            if self.active or self.pending or self.retiring:
                self.step()
                if not self.active and self.retiring:
                    self.torch.cuda.current_stream().synchronize()
            elif queue:
                if clock == "wall":
                    time.sleep(max(0.0, min(queue[0].arrival - now, 0.01)))
                else:
                    self._chunks += 1
            t = time.perf_counter()
            if progress is not None and t - t_note >= progress_every:
                t_note = t
                progress(f"serve: {len(self.results)}/{len(requests)} done, {len(self.active)} active, "
                         f"{len(self.pending) + len(queue)} waiting, {t - t_start:.0f} s")
            if t - t_start > timeout:
                raise KPMError("serving trace timed out")
        self.torch.cuda.synchronize()
        self._retire()
        return [self.results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]

    def close(self):
        self.batch.free()


def latency_stats(results: List[KPMResult]) -> dict:
    lat = np.array([r.latency for r in results if r.status == "ok"])
    if len(lat) == 0:
        return {"n": 0}
    return {"n": int(len(lat)), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
