"""Continuous-batching request loop for the reaction + SDC stage.

Independent simulations (tissue or cell sweeps with their own vertex count,
cell model, precision and dt) arrive over time.  The loop keeps every admitted
simulation's ionic state resident in HBM and advances all simulations of one
class (cell model x precision x node count, the unit one kernel instantiation
serves) together: each round launches one batched kernel per class over a
chunk of steps (reaction_sdc_step_batch), on one stream per class so the
classes overlap on the GPU.  A chunk is at least chunk_steps steps and at least
quantum_vertices * chunk_steps vertex-steps, so a small request finishes in
one round instead of waiting out as many rounds as a large one; with
split_small, requests below quantum_vertices form classes (and streams) of
their own, so a new small request does not wait for the round of the large
ones of its kind.  Between chunks it retires finished requests
(their final V is copied to the host) and admits arrivals in FIFO order while
the resident footprint stays within the HBM budget and a slot is free; neither
step waits for the device.  A request computes exactly what it computes alone:
every vertex's arithmetic is independent of what else shares the launch.

Latency of a request = time its result (final V on the host) is ready minus
its arrival time.  Throughput = total vertex-steps / (last completion - first
arrival).
"""
from __future__ import annotations

import sys
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


# ---- admission policy (pure host logic) ------------------------------------------
class Admission:
    """FIFO admission against a byte budget and a slot count."""

    def __init__(self, budget_bytes: float, slots: int):
        self.budget = float(budget_bytes)
        self.slots = int(slots)
        self.resident = 0.0
        self.active = 0

    def fits(self, footprint: float) -> bool:
        return self.active < self.slots and self.resident + footprint <= self.budget

    def admit(self, footprint: float):
        if not self.fits(footprint):
            raise RuntimeError("admission over budget or slots")
        self.resident += footprint
        self.active += 1

    def release(self, footprint: float):
        self.resident -= footprint
        self.active -= 1

    def take(self, waiting: deque, footprint_of):
        """Pop the arrived requests that may start now (head-of-line FIFO).
        A request larger than the whole budget is rejected (returned apart)."""
        admitted, rejected = [], []
        while waiting:
            fp = footprint_of(waiting[0])
            if fp > self.budget:
                rejected.append(waiting.popleft())
                continue
            if not self.fits(fp):
                break
            self.admit(fp)
            admitted.append(waiting.popleft())
        return admitted, rejected


def chunk_for(n: int, remaining: int, chunk_steps: int, quantum_vertices: int) -> int:
    """Steps a job of n vertices takes in one round: chunk_steps, or more for a
    job smaller than quantum_vertices, so that it does chunk_steps *
    quantum_vertices vertex-steps; never more than it has left."""
    steps = chunk_steps
    if quantum_vertices > 0 and n > 0:
        steps = max(steps, (chunk_steps * quantum_vertices) // n)
    return max(0, min(remaining, steps))


@dataclass
class _Job:
    req: object
    sim: object
    inputs: tuple          # device tensors kept alive while the job runs
    footprint: float
    remaining: int
    t_admit: float
    ready: object          # event on the upload stream: state and inputs in place
    waited: bool = False   # the class stream has been made to wait for `ready`
    host_v: object = None  # pinned host copy of V once the job has finished
    copied: object = None  # event: host_v is complete
    state: Optional[np.ndarray] = None


@dataclass
class Result:
    rid: int
    model: str
    precision: str
    n: int
    n_steps: int
    arrival: float
    admitted: float
    done: float
    V: Optional[np.ndarray] = None
    state: Optional[np.ndarray] = None

    @property
    def latency(self):
        return self.done - self.arrival


@dataclass
class Server:
    budget_bytes: float = 200e9
    slots: int = 128
    chunk_steps: int = 25
    quantum_vertices: int = 1_000_000   # jobs below this many vertices take longer chunks
    split_small: bool = True            # small jobs (below quantum_vertices) get streams of their own
    keep_state: bool = False            # keep each result's full state (tests)
    results: List[Result] = field(default_factory=list)
    rejected: List[int] = field(default_factory=list)
    trace_log: List[tuple] = field(default_factory=list)  # (class, t_launch) per batched launch

    def run(self, trace, verbose=False, time_scale=1.0):
        """Serve the requests of `trace` (arrival times in seconds, replayed in
        wall-clock time divided by time_scale).  Returns the list of Results.

        Nothing on the admit or retire path waits for the device: a request's
        state and inputs are built on the GPU on an upload stream (the initial
        state shared by every vertex is broadcast there, the diffusion current
        travels from pinned host memory) and its class stream waits for that
        upload by an event; a finished request's V (plane 0 of the state, double
        in both precision layouts) is copied to pinned host memory
        asynchronously, and the request completes once that copy's event has
        fired.  Its handle is closed, and its memory and slot released, at the
        next point where its class stream has no chunk in flight (closing waits
        for the streams the handle has used).""" 
        import torch

        from . import ionic as I

        policy = Admission(self.budget_bytes, self.slots)
        streams: Dict[tuple, "torch.cuda.Stream"] = {}
        upload = torch.cuda.Stream()
        active: Dict[tuple, List[_Job]] = {}
        retiring: List[tuple] = []
        closing: List[tuple] = []
        inflight: Dict[tuple, "torch.cuda.Event"] = {}
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        waiting: deque = deque()
        t0 = time.perf_counter()

        def now():
            return (time.perf_counter() - t0) * time_scale

        def start(req):
            x0c, amp, n_stim, (t_on, t_off), diff_np = req.compact_inputs()
            n = req.n
            with torch.cuda.stream(upload):
                x0 = torch.as_tensor(x0c).to("cuda", non_blocking=True)[:, None].expand(-1, n)
                x0 = x0.contiguous()
                stim = torch.zeros(n, dtype=torch.float64, device="cuda")
                stim[:n_stim] = amp
                diff = torch.from_numpy(diff_np).pin_memory().to("cuda", non_blocking=True)
                sim = I.Simulation(req.model, x0, precision=req.precision, stream=upload)
                ready = torch.cuda.Event()
                ready.record(upload)
            I.ionic_set_inputs(sim.handle, 0.0, req.dt, req.n_nodes, req.n_sweeps, stim, t_on,
                               t_off, diff)
            return _Job(req, sim, (x0, stim, diff), req.footprint_bytes(), req.n_steps, now(),
                        ready)

        def begin_finish(cls, job):
            """Enqueue the copy of the result; the class stream is idle here."""
            st = streams[cls]
            n = job.sim.n
            if not job.waited:           # a request with no steps: its upload still orders
                st.wait_event(job.ready)
                job.waited = True
            if self.keep_state:
                ns = job.sim.n_states
                if ns * n * 8 <= (8 << 20):   # through the library's static staging buffer
                    job.state = I.state_readback_noalloc(job.sim.handle, ns, 0, n, stream=st)
                else:
                    job.state = job.sim.readback(stream=st)
            with torch.cuda.stream(st):
                v_dev = job.sim.state[: n * 8].view(torch.float64)
                job.host_v = torch.empty(n, dtype=torch.float64, pin_memory=True)
                job.host_v.copy_(v_dev, non_blocking=True)
                job.copied = torch.cuda.Event()
                job.copied.record(st)
            retiring.append((cls, job))

        def complete(cls, job):
            r = job.req
            self.results.append(Result(r.rid, r.model, r.precision, r.n, r.n_steps, r.arrival,
                                       job.t_admit, now(), job.host_v.numpy().copy(), job.state))
            closing.append((cls, job))

        def close(job):
            job.sim.close()
            job.sim.state = None
            job.inputs = None
            policy.release(job.footprint)

        while pending or waiting or any(active.values()) or retiring or closing:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            progressed = False
            # chunks that completed
            for cls in list(inflight):
                if inflight[cls].query():
                    del inflight[cls]
                    progressed = True
            # results that reached the host
            for item in list(retiring):
                if item[1].copied.query():
                    retiring.remove(item)
                    complete(*item)
                    progressed = True
            # handles of completed requests whose class has nothing in flight
            for item in list(closing):
                if item[0] not in inflight:
                    closing.remove(item)
                    close(item[1])
                    progressed = True
            # finished jobs of idle classes start their result copy
            for cls, jobs in active.items():
                if cls in inflight:
                    continue
                for job in [j for j in jobs if j.remaining == 0]:
                    begin_finish(cls, job)
                    jobs.remove(job)
                    progressed = True
            # admit arrivals
            adm, rej = policy.take(waiting, lambda r: r.footprint_bytes())
            self.rejected += [r.rid for r in rej]
            for req in adm:
                cls = (req.model, req.precision, req.n_nodes,
                       bool(self.split_small and req.n < self.quantum_vertices))
                if cls not in streams:
                    streams[cls] = torch.cuda.Stream()
                active.setdefault(cls, []).append(start(req))
                progressed = True
                if verbose:
                    print("[serve] t=%.2fs admit req %d (%s %s N=%d steps=%d), active %d" % (
                        now(), req.rid, req.model, req.precision, req.n, req.n_steps,
                        policy.active), file=sys.stderr, flush=True)
            # launch the next chunk of every idle class
            for cls, jobs in active.items():
                if cls in inflight or not jobs:
                    continue
                st = streams[cls]
                for j in jobs:
                    if not j.waited:
                        st.wait_event(j.ready)
                        j.waited = True
                steps = [chunk_for(j.sim.n, j.remaining, self.chunk_steps, self.quantum_vertices)
                         for j in jobs]
                I.reaction_sdc_step_batch([j.sim.handle for j in jobs], steps, stream=st)
                ev = torch.cuda.Event()
                ev.record(st)
                inflight[cls] = ev
                self.trace_log.append((cls, now()))
                for j, k in zip(jobs, steps):
                    j.remaining -= k
                progressed = True
            if not progressed:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        return self.results


def summarize(results, rejected=()):
    lat = np.array([r.latency for r in results])
    work = sum(r.n * r.n_steps for r in results)
    t_first = min(r.arrival for r in results)
    t_last = max(r.done for r in results)
    return {
        "requests": len(results),
        "rejected": len(rejected),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in results])),
        "makespan_s": t_last - t_first,
        "throughput_vertex_steps_per_s": work / (t_last - t_first),
        "total_vertex_steps": int(work),
    }


def run_trace(trace, verbose=False, **server_kw):
    srv = Server(**server_kw)
    res = srv.run(trace, verbose=verbose)
    out = summarize(res, srv.rejected)
    out.update({"budget_bytes": srv.budget_bytes, "slots": srv.slots, "chunk_steps": srv.chunk_steps,
                "quantum_vertices": srv.quantum_vertices,
                "trace": "256 requests, Poisson 20/s, N log-uniform [1e3, 2e6], LR91/TT06, "
                         "fp64/mixed, dt {0.01, 0.02}, steps U{100..1000}, M=3, K=2"})
    return out
