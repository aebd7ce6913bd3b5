"""Pins of the oracle's partitioned step with the parabolic term inside ROS2 and
the inner iterations of Algorithm 2 (oracle/partitioned.py; paper section
3.3.2, Algorithm 2; section 3.3.1, equation rb_system; equation sdc).

* Without intracellular coupling (sigma_i = 0) the global systems fall apart
  into the vertices' own, u = 0, and one step is the per-vertex ROS2 step with
  one trapezoidal correction (oracle.sdc with the ROS2 predictor, M = 2, K = 1).
* On a cable with a linear cell model every cosine mode of the lumped Q1
  Neumann Laplacian is an eigenvector of the whole step: the step multiplies it
  by the fixed point of one pass of the scheme written for that mode alone
  (the pinned scalar ROS2 step of oracle.ros2 with the frozen u-term as a
  forcing, then the correction of equation sdc solved by hand), at every mode
  up to the highest one -- where an explicit parabolic term at this step and
  grid (tau = 0.05 ms, h = 0.01 cm) is unstable -- with |amplification| < 1.
* On LR91 and TT06 sheets at tau = 0.05 ms, h = 0.01 cm the inner iterations
  contract and stop within 16 passes at tol 1e-8; the field stays finite and
  physiological.
"""
import numpy as np
import pytest

from oracle import tt06
from oracle.diffusion import Bidomain
from oracle.models import LR91, TEST_LINEAR, TT06
from oracle.partitioned import advance_partitioned
from oracle.ros2 import ros2_step
from oracle.sdc import advance


def test_without_coupling_it_is_the_per_vertex_ros2_step():
    shape = (4, 3, 1)
    N = 12
    rng = np.random.Generator(np.random.PCG64(3))
    X0 = np.tile(tt06.published_initial()[:, None], (1, N))
    X0[0] += rng.uniform(-5.0, 40.0, N)
    stim = np.where(np.arange(N) < 4, -60.0, 0.0)
    bd = Bidomain(shape, 0.01, (0.0, 0.0, 0.0), (1.5e-3,) * 3)
    u0 = bd.elliptic(X0[0])
    assert np.max(np.abs(u0)) == 0.0
    X, u, st = advance_partitioned(TT06, X0, u0, bd, dt=0.05, n_steps=3, i_stim=stim,
                                   stim_on=0.0, stim_off=0.1, tol=1e-12)
    ref, _ = advance(TT06, X0, dt=0.05, n_steps=3, n_nodes=2, n_sweeps=1, i_stim=stim,
                     stim_on=0.0, stim_off=0.1, predictor="ros2")
    scale = np.maximum(np.abs(ref), TT06.newton_scale[:, None])
    assert np.max(np.abs(X - ref) / scale) < 1e-12
    assert st.inner_iterations == [2, 2, 2]   # the second pass reproduces the first


def _mode_amplification(lam, mu, tau):
    """One step of the scheme on a single mode v = w e_k of a linear cell model
    y' = lam y + I_diff with sigma_e = sigma_i (so u = -v/2 + const) and
    M_L^{-1} A_i e_k = mu e_k, written for that mode: ROS2 on
    y' = (lam - mu) y + f with f = (mu/2) w frozen (w the end-of-step value),
    the correction with G(y^n; u^n) = (lam - mu/2) y^n, then the fixed point in w."""
    def one_pass(w):
        m = TEST_LINEAR.with_params(lam=lam - mu, b=0.5 * mu * w)
        y0 = np.ones((1, 1))
        yt, _, Ft0 = ros2_step(m, y0, tau, np.zeros(1), np.zeros(1))
        yt = float(yt[0, 0])
        a = lam - mu
        g_n = (lam - 0.5 * mu) * 1.0
        g_t = a * yt + 0.5 * mu * w
        eps = (1.0 - yt + 0.5 * tau * (g_n + g_t)) / (1.0 - tau * a)
        return yt + eps
    p0 = one_pass(0.0)
    p1 = one_pass(1.0)
    return p0 / (1.0 - (p1 - p0))          # w = p0 + (p1 - p0) w


@pytest.mark.parametrize("k", [0, 1, 5, 16, 32])
def test_linear_cable_modes(k):
    nx, h, sig, tau, lam = 33, 0.01, 1.5e-3, 0.05, -0.3
    bd = Bidomain((nx, 1, 1), h, (sig,) * 3, (sig,) * 3)
    phi = np.cos(k * np.pi * np.arange(nx) / (nx - 1))
    L = (bd.Ai @ phi) / bd.ml
    mu = sig * 2.0 / h ** 2 * (1.0 - np.cos(k * np.pi / (nx - 1)))
    np.testing.assert_allclose(L, mu * phi, rtol=0, atol=1e-9 * max(mu, 1.0))
    model = TEST_LINEAR.with_params(lam=lam, b=0.0)
    X0 = phi[None, :].copy()
    u0 = bd.elliptic(X0[0])
    X, u, st = advance_partitioned(model, X0, u0, bd, dt=tau, n_steps=1, tol=1e-14, max_inner=200)
    R = _mode_amplification(lam, mu, tau)
    assert st.converged
    np.testing.assert_allclose(X[0], R * phi, rtol=0, atol=1e-12)
    assert abs(R) < 1.0
    # the elliptic solution is -v/2 shifted to lumped-mass mean zero
    vend = X[0]
    shift = -0.5 * vend - u
    assert np.ptp(shift) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("model", [LR91, TT06], ids=["LR91", "TT06"])
def test_sheet_inner_iterations_contract_at_the_papers_step(model):
    shape = (12, 10, 1)
    N = 120
    from oracle import rest
    x = rest.lr91_rest() if model is LR91 else tt06.published_initial()
    X0 = np.tile(x[:, None], (1, N))
    stim = np.where(np.arange(N) % shape[0] < 2, -100.0, 0.0)
    bd = Bidomain(shape, 0.01, (1.5e-3,) * 3, (1.5e-3,) * 3)
    u0 = bd.elliptic(X0[0])
    X, u, st = advance_partitioned(model, X0, u0, bd, dt=0.05, n_steps=40, i_stim=stim,
                                   stim_on=0.0, stim_off=1.0, tol=1e-8, max_inner=30)
    assert st.converged
    # the lagged u contracts the error by at most 1/2 per pass on the stiffest
    # modes (tau a / (2 (1 + tau a)) for a Laplacian eigenvalue a): 1e-8 within 16
    assert max(st.inner_iterations) <= 16
    assert np.all(np.isfinite(X))
    assert -95.0 < X[0].min() and X[0].max() < 70.0
    assert X[0].max() > -40.0            # the stimulated edge is depolarising
