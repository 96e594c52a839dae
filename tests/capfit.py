"""Contact angle of a drop on a flat wall: the phi = 0 crossings along grid
lines, a least-squares circle through them, and the angle that circle makes
with the wall line.  Shared by the oracle's and the GPU's wetting tests."""
import math

import numpy as np

from paper_2311_05097_amd import workloads as W


def interface_points(phi, ymin, ymax):
    """Sub-node crossings of phi = 0 along grid lines, ymin < y < ymax."""
    pts = []
    ny, nx = phi.shape
    for j in range(ny - 1):
        for i in range(nx):
            a, b = phi[j, i], phi[j + 1, i]
            if a * b < 0 and ymin < j + 0.5 < ymax:
                pts.append((i, j + a / (a - b)))
            if i < nx - 1:
                c = phi[j, i + 1]
                if a * c < 0 and ymin < j < ymax:
                    pts.append((i + a / (a - c), j))
    return np.array(pts)


def cap_angle(phi, ys):
    p = interface_points(phi, ys + 3.0, phi.shape[0] - 4.0)
    x, y = p[:, 0], p[:, 1]
    A = np.c_[2 * x, 2 * y, np.ones_like(x)]
    cx, cy, c = np.linalg.lstsq(A, x * x + y * y, rcond=None)[0]
    R = math.sqrt(c + cx * cx + cy * cy)
    return math.degrees(math.acos(np.clip((ys - cy) / R, -1.0, 1.0)))


def cap_state(nx, ny, ys, R0, theta_param, theta_shape):
    """A circular cap of contact angle theta_shape and area pi R0^2 / 2 on
    the flat diffuse slab of rows y < ys (the wall line), with the wetting
    parameter theta_param; density and viscosity ratios 1, sigma = 1e-2."""
    t0 = math.radians(theta_shape)
    Rc = math.sqrt(0.5 * math.pi * R0 * R0 / (t0 - math.sin(t0) * math.cos(t0)))
    yc = ys - Rc * math.cos(t0)
    w = W.droplet_on_slab(nx=nx, ny=ny, slab_rows=16, R=Rc, theta_deg=theta_param, rho_ratio=1.0,
                          mu_ratio=1.0, mu1=0.1, tau_phi=1.0, sigma=1e-2)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = (1 - w.phi0) * np.tanh((Rc - np.hypot(x - nx / 2, y - yc)) / (w.params["D"] / 2))
    return w, phi


def interface_points_3d(phi, zmin, zmax):
    """Sub-node crossings of phi = 0 along the grid lines in x, y and z,
    zmin < z < zmax; phi is (nz, ny, nx)."""
    pts = []
    for axis in range(3):
        a = phi
        b = np.roll(phi, -1, axis=axis)
        m = a * b < 0
        idx = np.argwhere(m)
        if axis == 0:  # no wrap in z
            idx = idx[idx[:, 0] < phi.shape[0] - 1]
        k, j, i = idx[:, 0], idx[:, 1], idx[:, 2]
        va, vb = a[k, j, i], b[k, j, i]
        s = va / (va - vb)
        z = k + (s if axis == 0 else 0.0)
        y = j + (s if axis == 1 else 0.0)
        x = i + (s if axis == 2 else 0.0)
        keep = (z > zmin) & (z < zmax) & (x < phi.shape[2] - 1) & (y < phi.shape[1] - 1)
        pts.append(np.c_[x[keep], y[keep], z[keep]])
    return np.concatenate(pts)


def cap_angle_3d(phi, zs):
    """Contact angle of a drop on the wall plane z = zs: the least-squares
    sphere through the phi = 0 crossings more than 3 nodes above the wall,
    and the angle it makes with the plane (inside the liquid)."""
    p = interface_points_3d(phi, zs + 3.0, phi.shape[0] - 4.0)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    A = np.c_[2 * x, 2 * y, 2 * z, np.ones_like(x)]
    cx, cy, cz, c = np.linalg.lstsq(A, x * x + y * y + z * z, rcond=None)[0]
    R = math.sqrt(c + cx * cx + cy * cy + cz * cz)
    return math.degrees(math.acos(np.clip((zs - cz) / R, -1.0, 1.0)))


def cap_state_3d(nx, ny, nz, slab, R0, theta_param, theta_shape, **kw):
    """A spherical cap of contact angle theta_shape and the volume of a
    hemisphere of radius R0, on the diffuse slab of rows z < slab (wall plane
    z = slab - 1/2), with the wetting parameter theta_param; density and
    viscosity ratios 1, sigma = 1e-2 unless given."""
    t0 = math.radians(theta_shape)
    ct = math.cos(t0)
    Rc = R0 * (2.0 / ((2.0 + ct) * (1.0 - ct) ** 2)) ** (1.0 / 3.0)
    zs = slab - 0.5
    zc = zs - Rc * ct
    opts = dict(rho_ratio=1.0, mu_ratio=1.0, mu1=0.1, sigma=1e-2)
    opts.update(kw)
    w = W.drop_on_slab_3d(nx, ny, nz, slab=slab, R=Rc, theta_deg=theta_param, **opts)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - zc) ** 2)
    phi = (1 - w.phi0) * np.tanh((Rc - r) / (w.params["D"] / 2))
    import dataclasses
    return dataclasses.replace(w, phi=phi), zs
