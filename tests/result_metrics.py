"""Paper-level results computed from macroscopic fields (numpy, any source):
the Laplace pressure jump of a droplet, the velocity profile of a layered
channel and the bubble/spike fronts of a Rayleigh-Taylor column.  Used to
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
