"""Pins of the lift reference: the lifted densities reproduce the requested
phase field (the scaled definition below Eq. 8) and pressure, and pure
phases at the balanced pressure give the initial densities."""
import numpy as np

from oracle import lift_ref as L

CS2 = (0.05, 0.15)        # alpha 0.9 / 0.7
RIN = (3.0, 1.0)          # pressure balance: 3 * 0.05 = 1 * 0.15


def test_lift_reproduces_phase_field_and_pressure():
    rng = np.random.default_rng(3)
    v = rng.uniform(-1, 1, 1000)
    p = rng.uniform(0.1, 0.2, 1000)
    rR, rB = L.lift(v, p, *CS2)
    assert np.all(rR >= 0) and np.all(rB >= 0)
    assert np.allclose(L.phase_field(rR, rB, *RIN), v, rtol=0, atol=1e-14)
    assert np.allclose(rR * CS2[0] + rB * CS2[1], p, rtol=1e-14, atol=0)


def test_lift_pure_phases_and_clipping():
    rR, rB = L.lift(np.array([1.0, -1.0, 1.5, -2.0, 0.0]), 0.15, *CS2)
    assert np.allclose(rR, [3.0, 0.0, 3.0, 0.0, 1.5]) and np.allclose(rB, [0.0, 1.0, 0.0, 1.0, 0.5])
