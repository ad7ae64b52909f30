"""CPU pins of the result metrics on constructed fields."""
import numpy as np

import result_metrics as RM


def _p(nx, ny, nz, alpha=(0.9, 0.7)):
    return {"nx": nx, "ny": ny, "nz": nz, "alpha": alpha}


def test_pressure_and_laplace_jump():
    p = _p(4, 4, 4)
    rR = np.zeros(64); rB = np.ones(64)
    rR[:8] = 3.0; rB[:8] = 0.0
    f = {"rhoR": rR, "rhoB": rB}
    pr = RM.pressure(f, p)
    assert np.allclose(pr[:8], 0.15) and np.allclose(pr[8:], 0.15)
    rR[:8] = 3.3
    assert abs(RM.laplace_jump(f, p, np.arange(64) < 8, np.arange(64) >= 8) - 0.015) < 1e-12


def test_channel_profile_averages_planes():
    p = _p(2, 3, 4)
    ux = np.repeat(np.arange(4.0), 6)
    assert np.allclose(RM.channel_profile({"ux": ux}, p), np.arange(4.0))


def test_fronts_interpolate_first_crossing():
    p = _p(4, 4, 8)
    z = np.arange(8.0)
    col_b = np.tanh(z - 5.25)          # crossing at 5.25 (interpolated linearly)
    col_s = np.tanh(z - 2.5)
    rn = np.zeros((8, 4, 4))
    rn[:, :, :] = -1.0
    rn[:, 0, 0] = col_b
    rn[:, 2, 2] = col_s
    b, s = RM.fronts(rn.ravel(), p)
    i = 5
    assert abs(b - (i + col_b[i] / (col_b[i] - col_b[i + 1]))) < 1e-12 and 5.0 < b < 6.0
    assert 2.0 < s < 3.0
