"""Seeded synthetic workloads: case parameters and initial fields.

This module holds no arithmetic of the lattice Boltzmann method itself.  It
only builds inputs -- lattice sizes, fluid parameters and the initial density
and velocity fields -- for the experiments of the paper (Sec. IV) scaled to the
benchmark shapes.  Both the GPU library and the CPU oracle receive exactly
these inputs; neither computes them.

A case is ``(params, fields)``:
  params  plain dict: nx, ny, nz, bc[3] (0 periodic / 1 wall), theta_deg[2],
          rho_in[2], alpha[2], tau_v[2], A[2], beta, delta, tau_e, tau_q,
          tau_pi, force[3], grav[3], rho_ref, improved, meq4 (rows 16-18 of
          the moment equilibria: 0 = M f^eq, 1 = the Appendix as printed), wall_u[2][3]
          (tangential velocity of the wall at the low and the high end of the
          wall axis)
  fields  dict of float64 arrays of length nx*ny*nz in x-fastest order:
          rhoR, rhoB, ux, uy, uz  (the initial colour densities and velocity)

Pressure balance between the two fluids (Sec. IV.A: rho_R^in/rho_B^in =
(1 - alpha_B)/(1 - alpha_R)) is imposed when alpha_R is derived.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(bc=(0, 0, 0), theta_deg=(90.0, 90.0), beta=0.5, delta=0.98,
                tau_e=1.0, tau_q=1.0, tau_pi=1.0, force=(0.0, 0.0, 0.0),
                grav=(0.0, 0.0, 0.0), rho_ref=0.0, improved=1, meq4=0,
                wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))


def _params(**kw) -> dict:
    p = dict(DEFAULTS)
    p.update(kw)
    return p


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1).astype(np.float64), y.reshape(-1).astype(np.float64), z.reshape(-1).astype(np.float64)


def _periodic_d2(coord, centre, n, periodic):
    d = coord - centre
    if periodic:
        d = d - n * np.round(d / n)
    return d * d


def droplet_fields(p: dict, centre, radius, rho_in, u_in=(0.0, 0.0, 0.0), u_out=(0.0, 0.0, 0.0)):
    """Sharp +-1 sphere: red (rho_R^in, 0) where the periodic distance to the
    centre is <= radius (inclusive), blue (0, rho_B^in) elsewhere."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    x, y, z = _grid(nx, ny, nz)
    d2 = (_periodic_d2(x, centre[0], nx, p["bc"][0] == 0) +
          _periodic_d2(y, centre[1], ny, p["bc"][1] == 0) +
          _periodic_d2(z, centre[2], nz, p["bc"][2] == 0))
    inside = d2 <= radius * radius
    f = dict(rhoR=np.where(inside, rho_in[0], 0.0), rhoB=np.where(inside, 0.0, rho_in[1]))
    for a, name in enumerate(("ux", "uy", "uz")):
        f[name] = np.where(inside, u_in[a], u_out[a]).astype(np.float64)
    return f


def static_droplet(n=32, radius=8.0, rho_in=(1.0, 1.0), alpha=(1 / 3, 1 / 3), tau=1.0, A=0.01):
    """Static droplet on a periodic cube (Laplace jump, mass conservation).
    Default: 32^3, density and viscosity ratio 1, tau = 1, A_R = A_B = 0.01,
    radius 8 at the centre, zero velocity."""
    p = _params(nx=n, ny=n, nz=n, rho_in=rho_in, alpha=alpha, tau_v=(tau, tau), A=(A, A),
                tau_e=tau, tau_q=tau, tau_pi=tau)
    return p, droplet_fields(p, (n / 2, n / 2, n / 2), radius, rho_in)


def paper_fluids_droplet(n=32, radius=8.0):
    """The same droplet with the fluid pair of Sec. IV.A (rho^in 3/1, alpha
    0.9/0.7, A = 0.01, beta = 0.5, all relaxation times 1): exercises the
    improved equilibrium and the correction term, which vanish at alpha = 1/3."""
    return static_droplet(n=n, radius=radius, rho_in=(3.0, 1.0), alpha=(0.9, 0.7), tau=1.0, A=0.01)


def galilean_droplet(n=128, radius=20.0, seed=1904, u0=(0.05, 0.05, 0.05), rho_in=(1.0, 1.0),
                     alpha=(1 / 3, 1 / 3), A=0.01):
    """Droplet advected by a uniform flow on a periodic cube.  The centre is
    drawn uniformly in the box and tau_v (both fluids) uniformly in [0.6, 1.0]
    from the seed; the whole lattice starts at velocity u0."""
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0.0, n, size=3)
    tau = float(rng.uniform(0.6, 1.0))
    p = _params(nx=n, ny=n, nz=n, rho_in=rho_in, alpha=alpha, tau_v=(tau, tau), A=(A, A))
    return p, droplet_fields(p, centre, radius, rho_in, u_in=u0, u_out=u0)


def channel_alpha(ratio: float, alpha_B: float = 0.2):
    """alpha pair with rho_R^in = ratio, rho_B^in = 1 in pressure balance."""
    return 1.0 - (1.0 - alpha_B) / ratio, alpha_B


def layered_channel(nx=64, ny=64, nz=256, ratio=1.0, visc_ratio=1.0, G=1e-6, alpha_B=0.2,
                    tau_min=1.5, A=1e-4, three_layer=False):
    """Layered two-phase channel flow: walls at z (halfway bounce-back),
    periodic in x and y, body-force density (G, 0, 0).  Red below mid-height,
    blue above (or the paper's symmetric red core when three_layer=True).
    The dynamic viscosity ratio M = mu_R/mu_B equals (tau_R-1/2)/(tau_B-1/2)
    because both fluids share rho_k (c_s^k)^2; the less viscous fluid gets
    tau_min."""
    aR, aB = channel_alpha(ratio, alpha_B)
    if visc_ratio >= 1.0:
        tB = tau_min
        tR = 0.5 + visc_ratio * (tau_min - 0.5)
    else:
        tR = tau_min
        tB = 0.5 + (tau_min - 0.5) / visc_ratio
    p = _params(nx=nx, ny=ny, nz=nz, bc=(0, 0, 1), rho_in=(ratio, 1.0), alpha=(aR, aB),
                tau_v=(tR, tB), A=(A, A), force=(G, 0.0, 0.0))
    x, y, z = _grid(nx, ny, nz)
    if three_layer:
        red = np.abs(z + 0.5 - nz / 2.0) <= nz / 4.0
    else:
        red = z < nz / 2.0
    f = dict(rhoR=np.where(red, ratio, 0.0), rhoB=np.where(red, 0.0, 1.0),
             ux=np.zeros_like(x), uy=np.zeros_like(x), uz=np.zeros_like(x))
    return p, f


def rayleigh_taylor(nx=128, ny=None, nz=None, g=2e-5, Re=1024.0, amp=0.05, rho_in=(3.0, 1.0),
                    alpha=(0.9, 0.7), A=1e-4):
    """3D Rayleigh-Taylor instability (Sec. IV.C) in [0,L]^2 x [0,4L], walls at
    z, periodic sides.  Atwood number 0.5 (rho^in 3/1), identical kinematic
    viscosity nu = L sqrt(gL)/Re, single-mode interface Eq. (56) with amplitude
    amp*L; heavy red on top; buoyancy F = (rho - rho_ref) g with g along -z and
    rho_ref the mean of the two densities."""
    ny = nx if ny is None else ny
    nz = 4 * nx if nz is None else nz
    L = float(nx)
    nu = L * math.sqrt(g * L) / Re
    tau = tuple(0.5 + nu / (0.5 * (1.0 - a)) for a in alpha)
    p = _params(nx=nx, ny=ny, nz=nz, bc=(0, 0, 1), rho_in=rho_in, alpha=alpha, tau_v=tau,
                A=(A, A), grav=(0.0, 0.0, -g), rho_ref=0.5 * (rho_in[0] + rho_in[1]))
    x, y, z = _grid(nx, ny, nz)
    h = amp * L * (np.cos(2 * np.pi * x / L) + np.cos(2 * np.pi * y / L))
    red = z >= nz / 2.0 + h
    f = dict(rhoR=np.where(red, rho_in[0], 0.0), rhoB=np.where(red, 0.0, rho_in[1]),
             ux=np.zeros_like(x), uy=np.zeros_like(x), uz=np.zeros_like(x))
    return p, f


def galilean_plates(nx=140, ny=140, nz=4, radius=30.0, improved=1, U=0.0):
    """Moving droplet between two plates (Sec. IV.A): walls at y, periodic x
    and z, a circular (z-invariant) droplet of radius 30 at the centre of the
    x-y plane, rho^in 3/1, alpha 0.9/0.7, A_R = A_B = 0.01, beta = 0.5,
    mu_R = mu_B = 0.075.  With (c_s^k)^2 = (1 - alpha_k)/2 both fluids have
    rho_k^in (c_s^k)^2 = 0.15, so nu_k = (c_s^k)^2 (tau_v^k - 1/2) gives
    tau_v = 1 for both; the other relaxation times are 1.  Both plates move
    along x with velocity U (0 while the droplet relaxes at rest)."""
    p = _params(nx=nx, ny=ny, nz=nz, bc=(0, 1, 0), rho_in=(3.0, 1.0), alpha=(0.9, 0.7),
                tau_v=(1.0, 1.0), A=(0.01, 0.01), improved=improved,
                wall_u=((U, 0.0, 0.0), (U, 0.0, 0.0)))
    x, y, _ = _grid(nx, ny, nz)
    cx, cy = nx / 2.0 - 0.5, ny / 2.0 - 0.5
    inside = _periodic_d2(x, cx, nx, True) + (y - cy) ** 2 <= radius * radius
    f = dict(rhoR=np.where(inside, 3.0, 0.0), rhoB=np.where(inside, 0.0, 1.0),
             ux=np.zeros_like(x), uy=np.zeros_like(x), uz=np.zeros_like(x))
    return p, f


def smooth_droplet_fields(p: dict, centre, radius, rho_in, u_in=(0.0, 0.0, 0.0), width=1.5):
    """Droplet with a tanh interface of the given width: red fraction
    phi = (1 - tanh((d - R)/width))/2 with d the (periodic) distance to the
    centre; rho_R = phi rho_R^in, rho_B = (1 - phi) rho_B^in, and the droplet
    velocity carried by the red fraction (u = phi u_in)."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    x, y, z = _grid(nx, ny, nz)
    d = np.sqrt(_periodic_d2(x, centre[0], nx, p["bc"][0] == 0) +
                _periodic_d2(y, centre[1], ny, p["bc"][1] == 0) +
                _periodic_d2(z, centre[2], nz, p["bc"][2] == 0))
    ph = 0.5 * (1.0 - np.tanh((d - radius) / width))
    f = dict(rhoR=rho_in[0] * ph, rhoB=rho_in[1] * (1.0 - ph))
    for a, name in enumerate(("ux", "uy", "uz")):
        f[name] = u_in[a] * ph
    return f


def impact_case(case: int, seed=1904, lmin=48, lmax=128, A=0.00225, width=1.5):
    """One droplet-impact case of the batch: cube of side L ~ U{lmin..lmax},
    wall at z (bottom wetting theta ~ U(60, 150) deg, top 90 deg), periodic x,y,
    droplet radius U(0.2, 0.3) L centred at (L/2, L/2, R+2) moving at -U0,
    U0 ~ U(0.01, 0.05), density ratio ~ U(10, 100), alpha_B = 0.2, tau = 1.
    The droplet starts with a tanh interface (width 1.5) and its velocity is
    carried by the red fraction: with the heavy phase's sound speed
    sqrt(0.4/ratio), a sharp start at these Mach numbers is unstable."""
    rng = np.random.default_rng([seed, case])
    L = int(rng.integers(lmin, lmax + 1))
    R = float(rng.uniform(0.2, 0.3)) * L
    U0 = float(rng.uniform(0.01, 0.05))
    ratio = float(rng.uniform(10.0, 100.0))
    theta = float(rng.uniform(60.0, 150.0))
    aR, aB = 1.0 - 0.8 / ratio, 0.2
    rho_in = (1.0, 1.0 / ratio)
    p = _params(nx=L, ny=L, nz=L, bc=(0, 0, 1), theta_deg=(theta, 90.0), rho_in=rho_in,
                alpha=(aR, aB), tau_v=(1.0, 1.0), A=(A, A))
    f = smooth_droplet_fields(p, (L / 2.0, L / 2.0, R + 2.0), R, rho_in, u_in=(0.0, 0.0, -U0), width=width)
    return p, f


def impact_paper(Re, D0=100.0, nx=300, ny=300, nz=150, U0=0.006, ratio=100.0, alpha_B=0.2, A=0.00225,
                 width=1.5, visc_ratio=10.0):
    """Droplet impact of Sec. IV.D: 300 x 300 x 150, walls at z (the droplet's
    flat surface at the bottom, theta = 90 deg on both), periodic x and y.  A
    droplet of diameter D0 = 100 touches the bottom wall at the centre of the
    box and moves down at U0 = 0.006; rho^in 8/0.08 (ratio 100), alpha_B =
    0.2 and alpha_R from pressure balance, A_R = A_B = 0.00225 (sigma =
    2(A_R + A_B)/9 = 0.001, We = rho_R U0^2 D0/sigma = 28.8).  Re = rho_R U0
    D0/mu_R sets tau_R through mu_k = rho_k^in (c_s^k)^2 (tau_k - 1/2); the
    paper does not give mu_B: the gas takes mu_B = mu_R / visc_ratio (default
    10; both fluids share rho_k^in (c_s^k)^2, so tau_B - 1/2 =
    (tau_R - 1/2)/visc_ratio).  The droplet starts with a tanh interface of the
    given width and its velocity carried by the red fraction."""
    rho_in = (8.0, 8.0 / ratio)
    aR = 1.0 - (1.0 - alpha_B) / ratio
    p_k = rho_in[0] * 0.5 * (1.0 - aR)
    tau = 0.5 + rho_in[0] * U0 * D0 / (Re * p_k)
    tau_B = 0.5 + (tau - 0.5) / visc_ratio
    p = _params(nx=nx, ny=ny, nz=nz, bc=(0, 0, 1), theta_deg=(90.0, 90.0), rho_in=rho_in,
                alpha=(aR, alpha_B), tau_v=(tau, tau_B), A=(A, A))
    R = 0.5 * D0
    f = smooth_droplet_fields(p, (nx / 2.0 - 0.5, ny / 2.0 - 0.5, R), R, rho_in, u_in=(0.0, 0.0, -U0),
                              width=width)
    return p, f


def impact_batch(ncases=256, seed=1904, lmin=48, lmax=128):
    return [impact_case(c, seed=seed, lmin=lmin, lmax=lmax) for c in range(ncases)]


def random_state_case(nx, ny, nz, seed=0, bc=(0, 0, 0), rho_in=(3.0, 1.0), alpha=(0.9, 0.7),
                      tau=(0.8, 0.65), theta=(70.0, 120.0), improved=1, force=(0.0, 0.0, 0.0),
                      grav=(0.0, 0.0, 0.0), rho_ref=0.0, u_scale=0.02):
    """Smooth random two-colour state for parity tests: a few random blobs,
    a diffuse interface and a small random velocity field."""
    rng = np.random.default_rng(seed)
    p = _params(nx=nx, ny=ny, nz=nz, bc=bc, theta_deg=theta, rho_in=rho_in, alpha=alpha,
                tau_v=tau, A=(0.01, 0.008), improved=improved, force=force, grav=grav,
                rho_ref=rho_ref, tau_e=0.9, tau_q=1.1, tau_pi=1.2)
    x, y, z = _grid(nx, ny, nz)
    phase = np.zeros_like(x)
    for _ in range(3):
        c = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
        r = rng.uniform(0.2, 0.4) * min(nx, ny, nz) + 1.0
        d = np.sqrt(_periodic_d2(x, c[0], nx, bc[0] == 0) + _periodic_d2(y, c[1], ny, bc[1] == 0) +
                    _periodic_d2(z, c[2], nz, bc[2] == 0))
        phase = np.maximum(phase, 0.5 * (1.0 - np.tanh((d - r) / 1.5)))
    f = dict(rhoR=rho_in[0] * phase, rhoB=rho_in[1] * (1.0 - phase))
    for name in ("ux", "uy", "uz"):
        f[name] = u_scale * rng.uniform(-1, 1, x.size) * (0.5 + 0.5 * np.sin(2 * np.pi * x / nx))
    return p, f
