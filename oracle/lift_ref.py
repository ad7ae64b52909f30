"""FP64 reference of the surrogate's lift from (rho^N, u) back to colour
densities.  TEST INFRASTRUCTURE ONLY.

The phase field (defined below Eq. 8) scales each colour by its initial
density: with a = rho_R/rho_R^in and b = rho_B/rho_B^in, rho^N = (a - b)/(a + b).
The pressure is the sum of the colour pressures p_k = rho_k (c_s^k)^2 with
(c_s^k)^2 = (1 - alpha_k)/2, and the initial densities are in pressure
balance, rho_R^in cs2R = rho_B^in cs2B = p_in.  Then p = p_in (a + b), so a
target phase field v and pressure p fix a = (p/p_in)(1 + v)/2,
b = (p/p_in)(1 - v)/2, i.e. rho_R = p (1 + v)/(2 cs2R), rho_B = p (1 - v)/(2 cs2B).
"""
from __future__ import annotations

import numpy as np


def phase_field(rR, rB, rR_in, rB_in):
    a, b = np.asarray(rR, dtype=np.float64) / rR_in, np.asarray(rB, dtype=np.float64) / rB_in
    return (a - b) / (a + b)


def lift(rhoN, p, cs2R, cs2B):
    v = np.clip(np.asarray(rhoN, dtype=np.float64), -1.0, 1.0)
    p = np.asarray(p, dtype=np.float64)
    return 0.5 * p * (1.0 + v) / cs2R, 0.5 * p * (1.0 - v) / cs2B
