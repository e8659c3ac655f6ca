"""Closed-form solutions the paper fixes (test-side only)."""
from __future__ import annotations

import math

from scipy.optimize import brentq
from scipy.special import erf, erfc


def neumann_melting_k(Ste_l: float) -> float:
    """Root of Ste_l / (exp(k^2) erf(k)) = k sqrt(pi), Eq. (61)."""
    return brentq(lambda k: Ste_l / (math.exp(k * k) * erf(k)) - k * math.sqrt(math.pi),
                  1e-9, 5.0, xtol=1e-15)


def neumann_melting_front(t: float, chi_l: float, Ste_l: float) -> float:
    """Interface position X(t) = 2 k sqrt(t chi_l), Eq. (61)."""
    return 2.0 * neumann_melting_k(Ste_l) * math.sqrt(t * chi_l)


def neumann_melting_T(x: float, t: float, chi_l: float, Ste_l: float, T_h=1.0, T_m=0.0):
    """Temperature of Eq. (60)."""
    k = neumann_melting_k(Ste_l)
    X = 2.0 * k * math.sqrt(t * chi_l)
    if x > X:
        return T_m
    return T_h - (T_h - T_m) / erf(k) * erf(x / (2.0 * math.sqrt(t * chi_l)))


def solidification_k(Ste_s, Ste_l, chi_s, chi_l):
    """Root of Eq. (63)."""
    r = math.sqrt(chi_s / chi_l)

    def fn(k):
        return (Ste_s / (math.exp(k * k) * erf(k))
                - Ste_l * math.sqrt(chi_l / chi_s) / (math.exp(k * k * chi_s / chi_l) * erfc(k * r))
                - k * math.sqrt(math.pi))
    return brentq(fn, 1e-9, 3.0, xtol=1e-15)
