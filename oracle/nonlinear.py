"""Nonlinearity catalogue (oracle side): f, its derivative f', and its
antiderivative F with F(0) = 0, so that F' = f.

Assumption A (Section 2) asks f(x, .) to be monotone and Lipschitz in a weak
sense; every entry below is nondecreasing in u:
    zero          f = 0
    linear        f = c u, c >= 0
    cubic         f = u^3                       (Example 1, Section 4)
    u_plus_sin    f = u + sin u                 (f' = 1 + cos u >= 0)
    abs_u_u       f = |u| u                     (f' = 2|u|)
    signed_pow    f = sign(u) |u|^q, q >= 1     (Example 3 with q = 3/2)
    neg_exp       f = -exp(-u)                  (Example 2, moved to the left side)

Example 3 prints f = -u^{3/2} for u < 0, which is undefined for real u < 0;
it is read as the odd extension sign(u)|u|^{3/2}.  Example 2 prints
-Laplace(u) - e^{-u} = 1, i.e. f(u) = -e^{-u}, which is increasing.
"""
from __future__ import annotations

import numpy as np

from paper_1611_05677_amd.workloads import (F_ABS_U_U, F_CUBIC, F_LINEAR, F_NEG_EXP,
                                            F_SIGNED_POW, F_U_PLUS_SIN, F_ZERO)


class Nonlinearity:
    def __init__(self, kind: int, param: float = 0.0):
        self.kind = int(kind)
        self.param = float(param)
        if kind == F_LINEAR and param < 0:
            raise ValueError("linear f needs c >= 0 (Assumption A)")
        if kind == F_SIGNED_POW and param < 1:
            raise ValueError("signed_pow needs q >= 1")

    def f(self, u):
        k, c = self.kind, self.param
        if k == F_ZERO:
            return np.zeros_like(u)
        if k == F_LINEAR:
            return c * u
        if k == F_CUBIC:
            return u * u * u
        if k == F_U_PLUS_SIN:
            return u + np.sin(u)
        if k == F_ABS_U_U:
            return np.abs(u) * u
        if k == F_SIGNED_POW:
            return np.sign(u) * np.abs(u) ** c
        if k == F_NEG_EXP:
            return -np.exp(-u)
        raise ValueError(k)

    def df(self, u):
        k, c = self.kind, self.param
        if k == F_ZERO:
            return np.zeros_like(u)
        if k == F_LINEAR:
            return np.full_like(u, c)
        if k == F_CUBIC:
            return 3.0 * u * u
        if k == F_U_PLUS_SIN:
            return 1.0 + np.cos(u)
        if k == F_ABS_U_U:
            return 2.0 * np.abs(u)
        if k == F_SIGNED_POW:
            return c * np.abs(u) ** (c - 1.0)
        if k == F_NEG_EXP:
            return np.exp(-u)
        raise ValueError(k)

    def F(self, u):
        k, c = self.kind, self.param
        if k == F_ZERO:
            return np.zeros_like(u)
        if k == F_LINEAR:
            return 0.5 * c * u * u
        if k == F_CUBIC:
            return 0.25 * u ** 4
        if k == F_U_PLUS_SIN:
            return 0.5 * u * u + 1.0 - np.cos(u)
        if k == F_ABS_U_U:
            return np.abs(u) ** 3 / 3.0
        if k == F_SIGNED_POW:
            return np.abs(u) ** (c + 1.0) / (c + 1.0)
        if k == F_NEG_EXP:
            return np.exp(-u) - 1.0
        raise ValueError(k)
