"""Pins of the oracle's cell models (LR91, TT06).

* exact Jacobian (paper section 3.3.2, after equation rb_system) against
  central finite differences of F;
* the compile-time sparsity of the local Jacobian (paper, CTSM, section
  3.3.2): the pattern each row may touch, stated here from the structure of
  the model equations, is checked three ways -- AD zeros, finite perturbations
  that leave F_i bit-identical, and tightness;
* the removable singularities are continuous;
* TT06 conserves charge: the gradient of the invariant Q is orthogonal to F.
"""
import numpy as np
import pytest

from oracle import lr91, rest, tt06
from oracle.models import LR91, TT06

# Row -> set of columns a model equation can depend on.
LR91_PATTERN = {
    "V": set(LR91.state_names),
    "Cai": {"V", "d", "f", "Cai"},
    **{g: {"V", g} for g in ("m", "h", "j", "d", "f", "X")},
}
TT06_PATTERN = {
    "V": set(TT06.state_names) - {"CaSR", "Rbar"},
    "Cai": {"V", "Nai", "Cai", "CaSR", "CaSS"},
    "CaSR": {"Cai", "CaSR", "CaSS", "Rbar"},
    "CaSS": {"V", "d", "f", "f2", "fCass", "CaSS", "CaSR", "Rbar", "Cai"},
    "Nai": {"V", "m", "h", "j", "Nai", "Cai"},
    "Ki": {"V", "r", "s", "xr1", "xr2", "xs", "Nai", "Ki"},
    **{g: {"V", g} for g in tt06.V_GATES},
    "fCass": {"CaSS", "fCass"},
    "Rbar": {"CaSS", "CaSR", "Rbar"},
}


def random_states(model, N, seed):
    rng = np.random.default_rng(seed)
    if model is LR91:
        base = rest.lr91_rest()
    else:
        base = tt06.published_initial()
    X = np.tile(base[:, None], (1, N))
    X[0] = rng.uniform(-90.0, 40.0, N)
    for i, name in enumerate(model.state_names):
        if name == "V":
            continue
        if name in model.fp64_states:
            X[i] *= rng.uniform(0.5, 2.0, N)
        else:
            X[i] = rng.uniform(0.02, 0.98, N)
    # keep away from the h/j branch point for finite differences
    X[0][np.abs(X[0] + 40.0) < 1e-2] += 0.1
    return X


def fd_jacobian(model, X, i_stim, i_diff):
    n, N = X.shape
    J = np.zeros((N, n, n))
    s = np.maximum(np.abs(X), model.newton_scale[:, None])
    for k in range(n):
        h = 1e-6 * s[k]
        Xp, Xm = X.copy(), X.copy()
        Xp[k] += h
        Xm[k] -= h
        J[:, :, k] = ((model.F(Xp, i_stim, i_diff) - model.F(Xm, i_stim, i_diff)) / (2 * h)).T
    return J, s


@pytest.mark.parametrize("model", [LR91, TT06], ids=["LR91", "TT06"])
def test_jacobian_matches_finite_differences(model):
    X = random_states(model, 64, 3)
    i_stim = np.full(64, -10.0)
    i_diff = np.linspace(-1, 1, 64)
    _, J = model.FJ(X, i_stim, i_diff)
    Jfd, s = fd_jacobian(model, X, i_stim, i_diff)
    # compare J_ik * s_k (change of F_i per relative change of X_k), row-scaled
    A = J * s.T[:, None, :]
    B = Jfd * s.T[:, None, :]
    rowscale = np.max(np.abs(A), axis=2, keepdims=True) + 1e-300
    assert np.max(np.abs(A - B) / rowscale) < 1e-6


@pytest.mark.parametrize("model,pattern", [(LR91, LR91_PATTERN), (TT06, TT06_PATTERN)], ids=["LR91", "TT06"])
def test_sparsity_pattern(model, pattern):
    names = model.state_names
    n = len(names)
    mask = np.zeros((n, n), dtype=bool)
    for i, row in pattern.items():
        for k in row:
            mask[names.index(i), names.index(k)] = True
    X = random_states(model, 200, 5)
    i_stim = np.full(200, -5.0)
    i_diff = np.full(200, 0.3)
    _, J = model.FJ(X, i_stim, i_diff)
    # AD zeros outside the pattern
    assert np.all(J[:, ~mask] == 0.0)
    # tight: every declared entry is nonzero somewhere
    assert np.all(np.any(J != 0.0, axis=0)[mask])
    # independent of AD: moving X_k leaves F_i bit-identical outside the pattern
    F0 = model.F(X, i_stim, i_diff)
    for k in range(n):
        Xp = X.copy()
        Xp[k] *= 1.001
        Xp[k] += 1e-7
        F1 = model.F(Xp, i_stim, i_diff)
        for i in range(n):
            if not mask[i, k]:
                assert np.array_equal(F0[i], F1[i]), (names[i], names[k])
    assert int(mask.sum()) == {8: 24, 19: 76}[n]


@pytest.mark.parametrize("model,v_sing", [(LR91, -47.13), (LR91, -77.0), (TT06, 15.0)],
                         ids=["LR91-alpha_m", "LR91-Xi", "TT06-ICaL"])
def test_removable_singularities_are_continuous(model, v_sing):
    X = random_states(model, 3, 7)
    X[0] = [v_sing, v_sing + 1e-6, v_sing - 1e-6]
    z = np.zeros(3)
    F, J = model.FJ(X, z, z)
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(J))
    # X columns differ in V only by 1e-6 and share the other states
    X[1:, 1] = X[1:, 0]
    X[1:, 2] = X[1:, 0]
    F, J = model.FJ(X, z, z)
    np.testing.assert_allclose(F[:, 0], F[:, 1], rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(F[:, 0], F[:, 2], rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(J[0, :, 0], J[1, :, 0], rtol=1e-4, atol=1e-9)


def test_tt06_charge_is_conserved():
    X = random_states(TT06, 50, 11)
    rng = np.random.default_rng(12)
    i_stim = rng.normal(0, 20, 50)
    i_diff = rng.normal(0, 1, 50)
    from oracle.ad import seed
    q = rest.tt06_charge(seed(X))
    F = TT06.F(X, i_stim, i_diff)
    terms = q.d * F
    assert np.max(np.abs(terms.sum(axis=0)) / np.max(np.abs(terms), axis=0)) < 1e-13
