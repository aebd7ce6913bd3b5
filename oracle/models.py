"""Model registry of the oracle (test infrastructure).

A model provides: NAME, STATE_NAMES, N_STATES, FP64_STATES, NEWTON_SCALE,
default parameters and rhs(x, i_stim, i_diff, p, clamp_v) returning the list
of n right-hand sides (paper equations parabolic, odes_con and odes with the
diffusion term held fixed; section 3.3 equation genODE with M~ = I).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from . import lr91, tt06
from .ad import seed, split
from .testmodels import Linear, Logistic


@dataclass
class Model:
    name: str
    state_names: tuple
    fp64_states: tuple
    newton_scale: np.ndarray
    params: dict
    _rhs: Callable = field(repr=False)

    @property
    def n(self):
        return len(self.state_names)

    def with_params(self, **overrides):
        p = dict(self.params)
        p.update(overrides)
        return Model(self.name, self.state_names, self.fp64_states, self.newton_scale, p, self._rhs)

    def F(self, X, i_stim, i_diff, clamp_v=False):
        """Right-hand side at X (n, N) -> (n, N)."""
        out = self._rhs(list(X), i_stim, i_diff, self.params, clamp_v)
        N = X.shape[1]
        return np.array([np.broadcast_to(np.asarray(o, dtype=np.float64), (N,)) for o in out])

    def FJ(self, X, i_stim, i_diff, clamp_v=False):
        """Right-hand side and exact Jacobian: F (n, N), J (N, n, n)."""
        n, N = X.shape
        out = self._rhs(seed(X), i_stim, i_diff, self.params, clamp_v)
        return split(out, n, N)


LR91 = Model(lr91.NAME, lr91.STATE_NAMES, lr91.FP64_STATES, lr91.NEWTON_SCALE,
             dict(lr91.PARAMS_PAPER), lr91.rhs)
LR91_ORIGINAL = LR91.with_params(**lr91.PARAMS_ORIGINAL)
TT06 = Model(tt06.NAME, tt06.STATE_NAMES, tt06.FP64_STATES, tt06.NEWTON_SCALE,
             dict(tt06.PARAMS), tt06.rhs)
TEST_LINEAR = Model(Linear.NAME, Linear.STATE_NAMES, Linear.FP64_STATES, Linear.NEWTON_SCALE,
                    dict(Linear.DEFAULT_PARAMS), Linear.rhs)
TEST_LOGISTIC = Model(Logistic.NAME, Logistic.STATE_NAMES, Logistic.FP64_STATES,
                      Logistic.NEWTON_SCALE, dict(Logistic.DEFAULT_PARAMS), Logistic.rhs)

BY_NAME = {m.name: m for m in (LR91, TT06, TEST_LINEAR, TEST_LOGISTIC)}
