"""Serving loop for setup + solve requests (continuous batching on one GPU).

A request brings a sparse SPD matrix (CSR, original order), the integer grid
coordinates of its unknowns and 1..16 right-hand sides.  The server builds
the cluster and block trees, H^2(A), the H^2-Cholesky factor and solves every
right-hand side by PCG; the result is the solution block.

Scheduling (host side only; every numerical step runs in the h2lr library):

* admission: a waiting request is admitted first-come first-served when its
  device bytes (``h2_estimate_bytes`` plus an allowance for task lists and
  PCG vectors) fit the HBM budget next to everything still held; a request
  larger than the whole budget is rejected;
* launch slots: each slot owns a HIP stream; admitted requests are
  factorised together in one batched launch (``h2_cholesky_launch``, one
  workgroup per problem) on a free slot, so launches made while others run
  overlap on the device;
* completion: a finished launch is checked, and all right-hand sides of its
  requests are solved by one batched PCG (``h2_pcg_batched``: one CG
  iteration per column; per iteration the preconditioner applications of
  all requests, all columns of a request at once, in one launch; with
  pcg_graph the iteration is captured once as a HIP graph and replayed);
* release: a request's device memory returns to the budget as soon as its
  own results are back ("eager", the default): the library frees matrix
  memory in stream order (hipFreeAsync on the matrix's stream), so a release
  does not wait for launches still running on other streams and requests
  are admitted into the freed memory while those launches continue.
  "idle" frees only when no launch is in flight (for comparison).

Latency of a request = completion time - arrival time.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import h2lr

TASK_BYTES_PER_DOF = 2048     # allowance for task lists and PCG vectors per unknown


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    A: object                      # scipy CSR, SPD
    coords: np.ndarray             # n x dim int32
    B: np.ndarray                  # n x nrhs right-hand sides
    result: np.ndarray | None = None
    iters: list = field(default_factory=list)
    status: str = "waiting"        # waiting, admitted, running, done, rejected, failed
    error: str = ""
    t_admit: float = -1.0
    t_done: float = -1.0
    nbytes: int = 0
    # device objects while the request is held
    _ct: object = None
    _bt: object = None
    _L: object = None
    _csr: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Server:
    def __init__(self, budget_bytes: int, eps: float = 1e-4, eta: float = 2.0, leaf: int = 32,
                 rtol: float = 1e-8, maxit: int = 500, slots: int = 2, max_batch: int = 32,
                 device: int = 0, release: str = "eager", pcg_graph: bool = False):
        self.budget = int(budget_bytes)
        self.tr = h2lr.trunc(eps, "block_rel", 32)
        self.eta, self.leaf, self.rtol, self.maxit = eta, leaf, rtol, maxit
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.ctxs = [h2lr.h2_ctx_create(device, s.cuda_stream) for s in self.streams]
        self.host_ctx = h2lr.h2_ctx_create(-1)
        self.used = 0                  # bytes held by admitted, unreleased requests
        self.peak = 0
        self.launches = 0
        self.max_inflight = 0
        self.admitted_in_flight = 0    # requests admitted while another launch was running
        if release not in ("idle", "eager"):
            raise ValueError("release must be 'idle' or 'eager'")
        self.release = release
        self.pcg_graph = pcg_graph     # batched PCG iterations replayed from a captured HIP graph
        self.release_s = 0.0           # host time spent freeing device memory

    # ------------------------------------------------------------ helpers
    def _estimate(self, r: Request) -> int:
        r._ct = h2lr.h2_ctree_build(self.host_ctx, r.coords, self.leaf)
        r._bt = h2lr.h2_btree_build(self.host_ctx, r._ct, self.eta)
        n = r.A.shape[0]
        return h2lr.h2_estimate_bytes(r._bt, True) + TASK_BYTES_PER_DOF * n

    def _materialise(self, r: Request, slot: int):
        ctx = self.ctxs[slot]
        # trees again on the slot's context (the host-only trees hold no device data)
        ct = h2lr.h2_ctree_build(ctx, r.coords, self.leaf)
        bt = h2lr.h2_btree_build(ctx, ct, self.eta)
        r._ct, r._bt = ct, bt
        r._L = h2lr.h2_mat_from_csr(ctx, bt, r.A, lower=True)
        r._csr = h2lr.h2_csr_create(ctx, r.A)

    def _release(self, r: Request):
        t = time.perf_counter()
        for name in ("_L", "_csr", "_bt", "_ct"):
            obj = getattr(r, name)
            if obj is not None:
                obj.close()
            setattr(r, name, None)
        self.used -= r.nbytes
        self.release_s += time.perf_counter() - t

    def _solve(self, reqs, slot: int):
        """All right-hand sides of the finished requests in one batched PCG
        (each request's columns share its preconditioner applications)."""
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            bs = [torch.tensor(np.ascontiguousarray(r.B.T), device="cuda") for r in reqs]
            xs = [torch.zeros_like(b) for b in bs]
            stream.synchronize()
            its, _, codes = h2lr.h2_pcg_batched([r._csr for r in reqs], [r._L for r in reqs], bs, xs,
                                                self.rtol, self.maxit, check=False, graph=self.pcg_graph)
            pos = 0
            for r, x in zip(reqs, xs):
                k = r.B.shape[1]
                r.result = np.ascontiguousarray(x.cpu().numpy().T)
                r.iters = its[pos:pos + k]
                bad = [c for c in codes[pos:pos + k] if c != 0]
                if bad and r.status != "failed":
                    r.status, r.error = "failed", h2lr.STATUS.get(bad[0], str(bad[0]))
                pos += k

    # --------------------------------------------------------------- loop
    def run(self, requests, poll: float = 5e-4, log=None):
        """Serve the requests (arrival times relative to the start); returns
        them with results, status and timestamps."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: list[Request] = []
        admitted: list[list[Request]] = [[] for _ in self.ctxs]   # per slot, not yet launched
        jobs: dict[int, tuple] = {}                               # slot -> (job, requests)
        to_release: list[Request] = []
        nxt = 0
        t0 = time.perf_counter()
        done = 0
        while done < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                waiting.append(pending[nxt])
                nxt += 1
            # release finished requests (at once, or when nothing is in flight)
            if to_release and (not jobs or self.release == "eager"):
                for r in to_release:
                    self._release(r)
                to_release = []
            # admission, first come first served, onto free slots
            free = [s for s in range(len(self.ctxs)) if s not in jobs]
            while waiting and free:
                r = waiting[0]
                if r.nbytes == 0:
                    r.nbytes = self._estimate(r)
                if r.nbytes > self.budget:
                    waiting.pop(0)
                    r.status, r.error, r.t_done = "rejected", "larger than the HBM budget", now
                    done += 1
                    continue
                if self.used + r.nbytes > self.budget:
                    break
                slot = min(free, key=lambda s: len(admitted[s]))
                if len(admitted[slot]) >= self.max_batch:
                    break
                waiting.pop(0)
                try:
                    self._materialise(r, slot)
                except h2lr.H2Error as e:          # e.g. the device is out of memory
                    r.status, r.error, r.t_done = "failed", str(e), time.perf_counter() - t0
                    self._release(r)
                    self.used += r.nbytes          # _release subtracted what was never added
                    done += 1
                    continue
                self.used += r.nbytes
                self.peak = max(self.peak, self.used)
                if jobs:
                    self.admitted_in_flight += 1
                r.status, r.t_admit = "admitted", time.perf_counter() - t0
                admitted[slot].append(r)
            # launch every free slot that holds admitted requests
            for s in free:
                if admitted[s]:
                    reqs = admitted[s]
                    admitted[s] = []
                    try:
                        job = h2lr.h2_cholesky_launch([r._L for r in reqs], self.tr)
                    except h2lr.H2Error as e:
                        for r in reqs:
                            r.status, r.error, r.t_done = "failed", str(e), time.perf_counter() - t0
                            to_release.append(r)
                            done += 1
                        continue
                    for r in reqs:
                        r.status = "running"
                    jobs[s] = (job, reqs)
                    self.launches += 1
                    self.max_inflight = max(self.max_inflight, len(jobs))
                    if log:
                        log(f"launch {self.launches}: slot {s}, {len(reqs)} problems, {len(jobs)} in flight, "
                            f"{self.used / 2**30:.2f} GiB held")
            # completions
            progressed = False
            for s in list(jobs):
                job, reqs = jobs[s]
                if not job.done():
                    continue
                progressed = True
                del jobs[s]
                codes = job.finish(check=False)
                ok = []
                for r, c in zip(reqs, codes):
                    if c == 0:
                        ok.append(r)
                    else:
                        r.status, r.error = "failed", h2lr.STATUS.get(c, str(c))
                if ok:
                    self._solve(ok, s)
                tnow = time.perf_counter() - t0
                for r in reqs:
                    if r.status == "running":
                        r.status = "done"
                    r.t_done = tnow
                    to_release.append(r)
                    done += 1
            if not progressed and nxt >= len(pending) and not waiting and not any(admitted) and not jobs:
                break
            if not progressed:
                time.sleep(poll)
        for r in to_release:
            self._release(r)
        return requests


def latency_summary(requests):
    lat = np.array([r.latency for r in requests if r.status == "done"])
    if lat.size == 0:
        return {"p50_s": None, "p99_s": None, "completed": 0}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "completed": int(lat.size)}
