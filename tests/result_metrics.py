"""Paper-level results computed from macroscopic fields (numpy, any source):
the Laplace pressure jump of a droplet, the velocity profile of a layered
channel, the bubble/spike fronts of a Rayleigh-Taylor column, the shape of
a z-invariant droplet carried along a periodic x axis and the spreading of a
droplet on the bottom wall.  Used to
state the error of each storage format against the FP64 oracle."""
import numpy as np


def pressure(fields, p):
    """p = sum_k rho_k (c_s^k)^2 with (c_s^k)^2 = (1 - alpha_k)/2."""
    cs2 = [0.5 * (1.0 - a) for a in p["alpha"]]
    return fields["rhoR"] * cs2[0] + fields["rhoB"] * cs2[1]


def laplace_jump(fields, p, inside, outside):
    """Mean pressure inside minus outside (boolean node masks)."""
    pr = pressure(fields, p)
    return float(pr[inside].mean() - pr[outside].mean())


def channel_profile(fields, p):
    """u_x averaged over each z plane (x fastest layout)."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    return fields["ux"].reshape(nz, ny, nx).mean(axis=(1, 2))


def fronts(rhoN, p):
    """(bubble, spike): first rho^N = 0 crossing from the bottom along the
    column x = y = 0 and along x = y = L/2, linearly interpolated."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    col = np.asarray(rhoN, dtype=np.float64).reshape(nz, ny, nx)
    out = []
    for (x, y) in ((0, 0), (nx // 2, ny // 2)):
        c = col[:, y, x]
        k = np.nonzero((c[:-1] < 0) & (c[1:] >= 0))[0]
        if k.size == 0:
            out.append(float("nan"))
            continue
        i = int(k[0])
        out.append(i + c[i] / (c[i] - c[i + 1]))
    return tuple(out)


def droplet_shape(rhoN, p):
    """Centre, aspect ratio and inclination of a droplet in the x-y plane.

    The phase fraction (1 + rho^N)/2, clipped to [0, 1] and averaged over z,
    weights the nodes.  x is periodic: the centre along x is the circular mean
    of the weights, and distances along x are taken modulo nx.  The aspect
    ratio is sqrt(l1/l2) of the eigenvalues l1 >= l2 of the weighted second
    moment tensor (a/b for an ellipse with semi-axes a >= b); the inclination
    is the angle of the major axis to x, in degrees within (-90, 90]."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    w = np.clip(0.5 * (1.0 + np.asarray(rhoN, dtype=np.float64).reshape(nz, ny, nx)), 0.0, 1.0).mean(axis=0)
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    m = w.sum()
    ang = 2.0 * np.pi * x / nx
    xc = (np.arctan2((w * np.sin(ang)).sum(), (w * np.cos(ang)).sum()) * nx / (2.0 * np.pi)) % nx
    yc = float((w * y).sum() / m)
    dx = x - xc
    dx = dx - nx * np.round(dx / nx)
    dy = y - yc
    ixx, iyy, ixy = (w * dx * dx).sum() / m, (w * dy * dy).sum() / m, (w * dx * dy).sum() / m
    lam, vec = np.linalg.eigh(np.array([[ixx, ixy], [ixy, iyy]]))
    major = vec[:, 1]
    incl = float(np.degrees(np.arctan2(major[1], major[0])))
    if incl <= -90.0:
        incl += 180.0
    elif incl > 90.0:
        incl -= 180.0
    return dict(xc=float(xc), yc=yc, aspect=float(np.sqrt(lam[1] / lam[0])), incl=incl)


def spreading(rhoN, p):
    """(contact, lateral) diameter of a droplet on the bottom wall (z = 0).

    The phase fraction (1 + rho^N)/2, clipped to [0, 1], gives areas: the
    contact diameter is 2 sqrt(A/pi) of the fraction summed over the first
    layer, the lateral diameter the same of the droplet's footprint seen along
    z (the largest fraction over z at each (x, y))."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    ph = np.clip(0.5 * (1.0 + np.asarray(rhoN, dtype=np.float64).reshape(nz, ny, nx)), 0.0, 1.0)
    contact = 2.0 * np.sqrt(ph[0].sum() / np.pi)
    lateral = 2.0 * np.sqrt(ph.max(axis=0).sum() / np.pi)
    return float(contact), float(lateral)


def asai_spreading(We, Re):
    """Maximum spreading factor D_max/D_0 of the Asai et al. correlation
    quoted in Sec. IV.D: 1 + 0.48 We^0.5 exp(-1.48 We^0.22 Re^-0.21)."""
    return 1.0 + 0.48 * We ** 0.5 * np.exp(-1.48 * We ** 0.22 * Re ** -0.21)
