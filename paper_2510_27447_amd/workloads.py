"""Seeded synthetic inputs shaped like the paper's workloads.

This module serves both the library and the tests; it holds no arithmetic of
the method: initial states come from a stored table (data/initial_states.json,
written by an oracle script), everything else is random numbers and index
bookkeeping.  The paper measures on its own meshes (a 2D square of 100^2 to
1000^2 cells, a 600x60x20 slab, a rabbit ventricle; sections 4.1-4.5), not on
a public dataset; these vertex sets stand in for them.  Vertex index
i + nx*(j + ny*k), x fastest.  NumPy PCG64, seed recorded with each workload.

Configurations (stimulus amplitudes in the cell-model sign convention:
negative depolarises; the paper's +100 uA/cm^2 reads -100 here):
  C1  LR91 (paper conductances), 64x64 = 4096 vertices, rest + U(-0.5, 0.5) mV
      on V, -80 uA/cm^2 on vertices 0..409 for t in [0, 1) ms, no diffusion
      input; dt 0.02 ms, 1000 steps, 3 nodes, 2 sweeps.
  C2  TT06 epi, 100^3 slab, rest + U(-1, 1) mV, -100 uA/cm^2 on the x = 0 face
      for [0, 2) ms, I_diff ~ N(0, 0.5^2) fixed; dt 0.02, 500 steps, 3 nodes,
      3 sweeps, Newton tol 1e-10.
  C3  C2 in mixed precision.
  C4  TT06 epi, 200^3, spiral V field -85 + 110 max(0, sin(theta - r/8)) mV
      (gates then set to steady state by the library), I_diff ~ N(0, 1)
      redrawn every 50 steps; dt 0.01, 1000 steps, 4 nodes, 3 sweeps.
  C5  serving trace: 256 requests, Poisson arrivals at 20/s, N log-uniform in
      [1e3, 2e6], LR91/TT06 50/50, dt in {0.01, 0.02}, steps U{100..1000},
      fp64/mixed 50/50; 3 nodes, 2 sweeps, stimulus on the first 10% of the
      vertices for 1 ms, I_diff ~ N(0, 0.5^2) per request.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "initial_states.json")
STATE_NAMES = {
    "LR91": ("V", "Cai", "m", "h", "j", "d", "f", "X"),
    "TT06": ("V", "Cai", "CaSR", "CaSS", "Nai", "Ki", "m", "h", "j", "xr1", "xr2", "xs", "r",
             "s", "d", "f", "f2", "fCass", "Rbar"),
}


def initial_state(model: str) -> np.ndarray:
    with open(_DATA) as f:
        tab = json.load(f)
    return np.array([tab[model][k] for k in STATE_NAMES[model]], dtype=np.float64)


@dataclass
class Workload:
    name: str
    model: str                 # "LR91" | "TT06"
    precision: str             # "fp64" | "mixed"
    x0: np.ndarray             # (n_states, N) float64
    dt: float
    n_steps: int
    n_nodes: int
    n_sweeps: int
    newton_tol: float = 1e-10
    newton_maxit: int = 10
    i_stim: Optional[np.ndarray] = None
    stim_t_on: float = 0.0
    stim_t_off: float = 0.0
    # diffusion current: one field held for the whole run, or a list of fields
    # each held for `diff_period` steps
    i_diff: Optional[np.ndarray] = None
    i_diff_series: List[np.ndarray] = field(default_factory=list)
    diff_period: int = 0
    steady_gates: bool = False  # set gates to steady state at V before stepping
    seed: int = 0
    grid: tuple = ()

    @property
    def n(self):
        return self.x0.shape[1]

    def subset(self, idx):
        """The same workload restricted to vertices idx (vertices are independent)."""
        idx = np.asarray(idx)
        return Workload(self.name + "[subset]", self.model, self.precision, self.x0[:, idx].copy(),
                        self.dt, self.n_steps, self.n_nodes, self.n_sweeps, self.newton_tol,
                        self.newton_maxit,
                        None if self.i_stim is None else self.i_stim[idx].copy(),
                        self.stim_t_on, self.stim_t_off,
                        None if self.i_diff is None else self.i_diff[idx].copy(),
                        [d[idx].copy() for d in self.i_diff_series], self.diff_period,
                        self.steady_gates, self.seed, ())


def blocked_order(nx, ny, nz, b=4, by=None, bz=None):
    """A processing order of a structured grid's vertices (index i + nx (j + ny k))
    in which each run of b * by * bz consecutive entries is a block of b x by x bz
    neighbouring vertices, x fastest inside a block (partial blocks at the far
    faces), for ionic_set_vertex_order; by and bz default to b, so that a
    wavefront of 64 lanes holds one 4 x 4 x 4 block."""
    by = b if by is None else by
    bz = b if bz is None else bz
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    parts = [idx[k:k + bz, j:j + by, i:i + b].ravel()
             for k in range(0, nz, bz) for j in range(0, ny, by) for i in range(0, nx, b)]
    return np.concatenate(parts).astype(np.int32)


def c1_lr91(seed=0, nx=64, ny=64, n_steps=1000):
    rng = np.random.Generator(np.random.PCG64(seed))
    N = nx * ny
    x0 = np.tile(initial_state("LR91")[:, None], (1, N))
    x0[0] += rng.uniform(-0.5, 0.5, N)
    stim = np.zeros(N)
    stim[:min(410, N)] = -80.0
    return Workload("C1-LR91-fp64", "LR91", "fp64", x0, 0.02, n_steps, 3, 2, 1e-10, 10,
                    stim, 0.0, 1.0, None, seed=seed, grid=(nx, ny))


def c2_tt06(seed=0, nx=100, ny=100, nz=100, n_steps=500, precision="fp64"):
    rng = np.random.Generator(np.random.PCG64(seed))
    N = nx * ny * nz
    x0 = np.tile(initial_state("TT06")[:, None], (1, N))
    x0[0] += rng.uniform(-1.0, 1.0, N)
    stim = np.zeros(N)
    stim[np.arange(N) % nx == 0] = -100.0
    diff = rng.normal(0.0, 0.5, N)
    name = "C2-TT06-fp64" if precision == "fp64" else "C3-TT06-mixed"
    return Workload(name, "TT06", precision, x0, 0.02, n_steps, 3, 3, 1e-10, 10,
                    stim, 0.0, 2.0, diff, seed=seed, grid=(nx, ny, nz))


def c3_tt06_mixed(seed=0, nx=100, ny=100, nz=100, n_steps=500):
    return c2_tt06(seed, nx, ny, nz, n_steps, precision="mixed")


def spiral_voltage(nx, ny, nz, c=None):
    """V = -85 + 110 max(0, sin(theta - r/8)), theta and r about the grid centre
    in index units, invariant in z."""
    c = (nx - 1) / 2.0 if c is None else c
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    theta = np.arctan2(j - c, i - c)
    r = np.hypot(i - c, j - c)
    v2 = -85.0 + 110.0 * np.maximum(0.0, np.sin(theta - r / 8.0))   # (ny, nx)
    return np.broadcast_to(v2[None], (nz, ny, nx)).reshape(-1)


def c4_tt06_spiral(seed=0, nx=200, ny=200, nz=200, n_steps=1000, precision="fp64"):
    rng = np.random.Generator(np.random.PCG64(seed))
    N = nx * ny * nz
    x0 = np.tile(initial_state("TT06")[:, None], (1, N))
    x0[0] = spiral_voltage(nx, ny, nz)
    period = 50
    series = [rng.normal(0.0, 1.0, N) for _ in range((n_steps + period - 1) // period)]
    return Workload("C4-TT06-spiral-" + precision, "TT06", precision, x0, 0.01, n_steps, 4, 3,
                    1e-10, 10, None, 0.0, 0.0, None, series, period, True, seed,
                    (nx, ny, nz))


@dataclass
class Request:
    """One serving request; its arrays are generated only when it is admitted."""
    rid: int
    arrival: float      # seconds after the trace starts
    model: str
    precision: str
    n: int
    dt: float
    n_steps: int
    seed: int
    n_nodes: int = 3
    n_sweeps: int = 2

    def footprint_bytes(self):
        n_states = len(STATE_NAMES[self.model])
        n_fp64 = 2 if self.model == "LR91" else 6
        stride = (self.n + 63) // 64 * 64
        per = n_states * 8 if self.precision == "fp64" else n_fp64 * 8 + (n_states - n_fp64) * 4
        return stride * per + 2 * 8 * self.n          # state + stimulus + diffusion input

    def compact_inputs(self):
        """The request's inputs in compact form: the initial state shared by every
        vertex (n_states,), the stimulus amplitude and the number of stimulated
        leading vertices, the stimulus window, and the diffusion current (n,)."""
        rng = np.random.Generator(np.random.PCG64(self.seed))
        amp = -80.0 if self.model == "LR91" else -100.0
        diff = rng.normal(0.0, 0.5, self.n)
        return initial_state(self.model), amp, max(1, self.n // 10), (0.0, 1.0), diff

    def materialize(self) -> Workload:
        x0c, amp, n_stim, (t_on, t_off), diff = self.compact_inputs()
        x0 = np.tile(x0c[:, None], (1, self.n))
        stim = np.zeros(self.n)
        stim[:n_stim] = amp
        return Workload("C5-req%d" % self.rid, self.model, self.precision, x0, self.dt,
                        self.n_steps, self.n_nodes, self.n_sweeps, 1e-10, 10, stim, t_on, t_off,
                        diff, seed=self.seed)


def c5_trace(seed=0, n_requests=256, rate_per_s=20.0, n_min=1e3, n_max=2e6):
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(n_requests):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        model = "LR91" if rng.random() < 0.5 else "TT06"
        dt = 0.01 if rng.random() < 0.5 else 0.02
        steps = int(rng.integers(100, 1001))
        precision = "fp64" if rng.random() < 0.5 else "mixed"
        reqs.append(Request(k, float(arrivals[k]), model, precision, n, dt, steps,
                            int(rng.integers(0, 2 ** 31))))
    return reqs
