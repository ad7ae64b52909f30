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


def test_droplet_shape_of_a_wrapped_ellipse():
    """A sharp ellipse (semi-axes 20 and 16, major axis at 30 deg to x) whose
    centre sits 4.7 nodes from the periodic x edge: the second moments of an
    ellipse of semi-axes a, b are a^2/4 and b^2/4, so the aspect ratio is
    a/b = 1.25 up to the staircase of the grid; the centre and angle come back.
    A circle gives 1."""
    nx, ny, nz = 140, 120, 2
    p = dict(nx=nx, ny=ny, nz=nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, t = 135.3, 60.7, np.radians(30.0)
    dx = x - cx
    dx = dx - nx * np.round(dx / nx)
    dy = y - cy
    u = dx * np.cos(t) + dy * np.sin(t)
    v = -dx * np.sin(t) + dy * np.cos(t)
    rhoN = np.where((u / 20.0) ** 2 + (v / 16.0) ** 2 <= 1.0, 1.0, -1.0).reshape(-1)
    s = RM.droplet_shape(rhoN, p)
    assert abs(s["xc"] - cx) < 0.1 and abs(s["yc"] - cy) < 0.1, s
    assert abs(s["aspect"] - 1.25) < 0.01, s
    assert abs(s["incl"] - 30.0) < 1.0, s
    circ = np.where(dx * dx + dy * dy <= 18.0 ** 2, 1.0, -1.0).reshape(-1)
    c = RM.droplet_shape(circ, p)
    assert abs(c["aspect"] - 1.0) < 0.005 and abs(c["xc"] - cx) < 0.05, c


def test_spreading_diameters():
    """A sharp lamella (disk of radius 40, two layers thick) under a
    hemisphere of radius 25: contact and lateral diameter 80.  A sphere of
    radius 20 resting on the wall: lateral diameter 40, contact only its
    lowest nodes.  Grid staircase below 1 %."""
    nx, ny, nz = 120, 110, 60
    p = dict(nx=nx, ny=ny, nz=nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - 60.3) ** 2 + (y - 54.6) ** 2
    drop = ((r2 <= 40.0 ** 2) & (z < 2)) | (r2 + z ** 2 <= 25.0 ** 2)
    c, l = RM.spreading(np.where(drop, 1.0, -1.0).reshape(-1), p)
    assert abs(c / 80.0 - 1.0) < 0.01 and abs(l / 80.0 - 1.0) < 0.01, (c, l)
    ball = r2 + (z - 20.0) ** 2 <= 20.0 ** 2
    c, l = RM.spreading(np.where(ball, 1.0, -1.0).reshape(-1), p)
    assert abs(l / 40.0 - 1.0) < 0.01 and c < 10.0, (c, l)


def test_asai_correlation_values():
    """The correlation at We = 28.8 (the paper's impact): D_max/D_0 rises from
    1.74 at Re = 75 to 2.25 at Re = 1000 (hand-evaluated: We^0.5 = 5.367,
    We^0.22 = 2.094, Re^-0.21 = 0.404 and 0.234)."""
    assert abs(RM.asai_spreading(28.8, 75.0) - 1.7366) < 1e-3
    assert abs(RM.asai_spreading(28.8, 1000.0) - 2.2455) < 1e-3
