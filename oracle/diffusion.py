"""Diffusion current of the parabolic equation on a structured grid, fp64
(oracle; test infrastructure).

Paper section 3.1 (spatial discretisation, equations semi-elliptic and
semi-parabolic): piecewise (multi)linear finite elements on a structured grid
of quadrilaterals / hexahedra give stiffness matrices A_i (sigma_i) and
A_ie (sigma_i + sigma_e) and the mass matrix M.  Section 4 uses scalar
conductivities sigma_i = sigma_e = 1.5e-3 everywhere.

* Assembly here is the plain definition: element matrices from the Q1 basis
  on [0, h]^d by Gauss-Legendre quadrature (two points per direction, exact
  for these polynomials), summed into global sparse matrices over every
  element of an nx x ny x nz grid of nodes (d = number of extents > 1);
  the lumped mass is the row sum of the consistent mass.
* Reading (bidomain -> monodomain for the paper's conductivities): with
  sigma_e = lambda sigma_i the discrete elliptic equation A_ie u = -A_i v has
  the solution u = -v / (1 + lambda) + const, so -A_i v - A_i u =
  -(lambda / (1 + lambda)) A_i v: the monodomain with
  sigma_m = sigma_i sigma_e / (sigma_i + sigma_e) (0.75e-3 for the paper's
  values) is the same semi-discrete system.  test_oracle_diffusion checks this
  against a sparse solve of the elliptic equation.
* The diffusion current entering dV/dt (R2 of the build's readings) is
  I_diff = -sigma_m M_L^{-1} A v with A the unit-conductivity stiffness;
  homogeneous Neumann boundaries (equation bcpde1) are natural in the
  assembly.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAUSS2 = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def monodomain_sigma(sigma_i, sigma_e):
    return sigma_i * sigma_e / (sigma_i + sigma_e)


def grid_dims(shape):
    """Extents > 1, in x, y, z order (x fastest in the vertex index)."""
    return [k for k, n in enumerate(shape) if n > 1]


def element_matrices(d, h, sig=None):
    """Stiffness K (conductivity diag(sig) over the element's d directions, unit
    if None) and mass Mm of the Q1 element [0, h]^d, local nodes in
    lexicographic order of their corner bits (bit k = upper end along axis k)."""
    sig = np.ones(d) if sig is None else np.asarray(sig, dtype=np.float64)
    corners = list(itertools.product((0, 1), repeat=d))
    nloc = len(corners)
    K = np.zeros((nloc, nloc))
    Mm = np.zeros((nloc, nloc))
    w = 0.5 * h  # Gauss weights on [0, h]: two points of weight h/2
    for q in itertools.product(GAUSS2, repeat=d):
        x = np.array(q)  # reference coordinates in [0, 1]
        phi = np.empty(nloc)
        grad = np.empty((nloc, d))
        for a, c in enumerate(corners):
            f = [x[k] if c[k] else 1.0 - x[k] for k in range(d)]
            df = [1.0 if c[k] else -1.0 for k in range(d)]
            phi[a] = np.prod(f)
            for k in range(d):
                grad[a, k] = df[k] * np.prod([f[j] for j in range(d) if j != k]) / h
        wq = w ** d
        K += wq * (grad * sig[None, :]) @ grad.T
        Mm += wq * np.outer(phi, phi)
    return corners, K, Mm


def assemble(shape, h, sigma=None):
    """Stiffness A (unit conductivity, or the diagonal tensor sigma = (sx, sy,
    sz)) and consistent mass M (scipy CSR) and the lumped mass (row sums of M)
    for the node grid `shape` = (nx, ny, nz)."""
    shape = tuple(int(n) for n in shape)
    dims = grid_dims(shape)
    d = len(dims)
    N = int(np.prod(shape))
    if d == 0:
        return sp.csr_matrix((N, N)), sp.identity(N, format="csr"), np.ones(N)
    sig = None if sigma is None else np.asarray(sigma, dtype=np.float64)[dims]
    corners, K, Mm = element_matrices(d, h, sig)
    strides = (1, shape[0], shape[0] * shape[1])
    rows, cols, kv, mv = [], [], [], []
    ranges = [range(shape[k] - 1) for k in dims]
    for e in itertools.product(*ranges):
        base = sum(e[j] * strides[dims[j]] for j in range(d))
        nodes = [base + sum(c[j] * strides[dims[j]] for j in range(d)) for c in corners]
        for a, na in enumerate(nodes):
            for b, nb in enumerate(nodes):
                rows.append(na)
                cols.append(nb)
                kv.append(K[a, b])
                mv.append(Mm[a, b])
    A = sp.csr_matrix((kv, (rows, cols)), shape=(N, N))
    M = sp.csr_matrix((mv, (rows, cols)), shape=(N, N))
    return A, M, np.asarray(M.sum(axis=1)).ravel()


class Diffusion:
    """I_diff = -sigma_m M_L^{-1} A v on one grid."""

    def __init__(self, shape, h, sigma_m):
        self.shape, self.h, self.sigma_m = tuple(shape), float(h), float(sigma_m)
        self.A, self.M, self.ml = assemble(shape, h)

    def current(self, v):
        return -self.sigma_m * (self.A @ v) / self.ml


class Bidomain:
    """The partitioned step's spatial part for diagonal conductivity tensors
    sigma_i, sigma_e (paper section 3.1: A_i with sigma_i, A_ie with
    sigma_i + sigma_e; section 3.3.2, Algorithm 2: the elliptic equation
    A_ie u = -A_i v is solved with v fixed, then the parabolic-ODE system with u
    fixed).  Neumann boundaries leave u defined up to a constant; the lumped-mass
    mean of u is fixed to zero (a bordered system, solved directly).  The
    current entering dV/dt is -M_L^{-1} A_i (v + u)."""

    def __init__(self, shape, h, sigma_i, sigma_e):
        self.shape, self.h = tuple(shape), float(h)
        self.sigma_i = np.asarray(sigma_i, dtype=np.float64)
        self.sigma_e = np.asarray(sigma_e, dtype=np.float64)
        self.Ai, _, self.ml = assemble(shape, h, self.sigma_i)
        self.Aie, _, _ = assemble(shape, h, self.sigma_i + self.sigma_e)
        ml = sp.csr_matrix(self.ml[None, :])
        self.bordered = sp.bmat([[self.Aie, ml.T], [ml, None]], format="csc")
        self.lu = spla.splu(self.bordered)

    def elliptic(self, v):
        rhs = np.concatenate([-(self.Ai @ v), [0.0]])
        return self.lu.solve(rhs)[:-1]

    def current(self, v, u):
        return -(self.Ai @ (v + u)) / self.ml


def advance_bidomain(model, X0, bidomain, *, t0=0.0, dt, n_steps, n_nodes, n_sweeps,
                     i_stim=None, stim_on=0.0, stim_off=0.0, tol=1e-10, maxit=10,
                     predictor="newton"):
    """One pass of the partitioned step per time step: u from the elliptic
    equation with v^n fixed, the current -M_L^{-1} A_i (v^n + u) held over one
    reaction step.  Returns (X, u of the last step, Stats)."""
    from .lobatto import integration_matrix, nodes
    from .sdc import Stats, sdc_step, stimulus_on

    X = np.array(X0, dtype=np.float64, copy=True)
    n, N = X.shape
    stim_amp = np.zeros(N) if i_stim is None else np.asarray(i_stim, dtype=np.float64)
    c = nodes(n_nodes)
    S = integration_matrix(n_nodes)
    stats = Stats(per_vertex_iters=np.zeros(N, dtype=np.int64))
    u = np.zeros(N)
    for step in range(n_steps):
        u = bidomain.elliptic(X[0])
        i_diff = bidomain.current(X[0], u)
        stim = stim_amp if stimulus_on(t0, dt, step, stim_on, stim_off) else np.zeros(N)
        X, _ = sdc_step(model, X, stim, dt, n_nodes, n_sweeps, i_diff, tol, maxit, False, stats,
                        S, c, predictor)
    stats.n_nonfinite = int((~np.isfinite(X).all(axis=0)).sum())
    return X, u, stats


def advance_coupled(model, X0, diffusion, *, t0=0.0, dt, n_steps, n_nodes, n_sweeps,
                    i_stim=None, stim_on=0.0, stim_off=0.0, tol=1e-10, maxit=10,
                    predictor="newton", record=None):
    """Per step: the diffusion current from V at the start of the step, held
    over the step, then one reaction step (sdc_step).  `record`, if given, is a
    callable(step_index_after, t, X) invoked after every step."""
    from .lobatto import integration_matrix, nodes
    from .sdc import Stats, sdc_step, stimulus_on

    X = np.array(X0, dtype=np.float64, copy=True)
    n, N = X.shape
    stim_amp = np.zeros(N) if i_stim is None else np.asarray(i_stim, dtype=np.float64)
    c = nodes(n_nodes)
    S = integration_matrix(n_nodes)
    stats = Stats(per_vertex_iters=np.zeros(N, dtype=np.int64))
    for step in range(n_steps):
        i_diff = diffusion.current(X[0])
        stim = stim_amp if stimulus_on(t0, dt, step, stim_on, stim_off) else np.zeros(N)
        X, _ = sdc_step(model, X, stim, dt, n_nodes, n_sweeps, i_diff, tol, maxit, False, stats,
                        S, c, predictor)
        if record is not None:
            record(step + 1, t0 + (step + 1) * dt, X)
    stats.n_nonfinite = int((~np.isfinite(X).all(axis=0)).sum())
    return X, stats
