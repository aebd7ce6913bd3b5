"""Scalar test problems with closed-form solutions (oracle; test infrastructure).

They are not in the paper: they exist to pin the SDC machinery of section
3.3.2 (equations picard_form ... sdc) to textbook results, independently of
the cell models.

TEST_LINEAR    y' = lam * y + b + i_diff        params (lam, b)
TEST_LOGISTIC  y' = rate * y * (1 - y) + i_diff params (rate,)
The per-vertex diffusion input adds to the right-hand side and the stimulus
is ignored, so both problems use the same inputs as the cell models.
"""
from __future__ import annotations

import numpy as np


class Linear:
    NAME = "TEST_LINEAR"
    STATE_NAMES = ("y",)
    N_STATES = 1
    FP64_STATES = ("y",)
    NEWTON_SCALE = np.array([1.0])
    DEFAULT_PARAMS = dict(lam=-1.0, b=0.0)

    @staticmethod
    def rhs(x, i_stim, i_diff, p=DEFAULT_PARAMS, clamp_v=False):
        (y,) = x
        return [p["lam"] * y + p["b"] + i_diff]

    @staticmethod
    def exact(y0, t, p=DEFAULT_PARAMS):
        lam, b = p["lam"], p["b"]
        if lam == 0.0:
            return y0 + b * t
        return (y0 + b / lam) * np.exp(lam * t) - b / lam


class Logistic:
    NAME = "TEST_LOGISTIC"
    STATE_NAMES = ("y",)
    N_STATES = 1
    FP64_STATES = ("y",)
    NEWTON_SCALE = np.array([1.0])
    DEFAULT_PARAMS = dict(rate=1.0)

    @staticmethod
    def rhs(x, i_stim, i_diff, p=DEFAULT_PARAMS, clamp_v=False):
        (y,) = x
        return [p["rate"] * y * (1.0 - y) + i_diff]

    @staticmethod
    def exact(y0, t, p=DEFAULT_PARAMS):
        e = np.exp(p["rate"] * t)
        return y0 * e / (1.0 - y0 + y0 * e)
