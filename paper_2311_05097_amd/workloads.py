"""Seeded synthetic inputs (geometry, initial fields, parameters).

This module only builds inputs: the smooth solid indicator phi0, the initial
order parameter phi, the per-node contact angle, the initial velocity and the
parameter set of each workload.  It holds none of the lattice Boltzmann
arithmetic, imports nothing else from this package, and is the one piece
shared by the GPU path and the CPU oracle (both receive the same arrays).

Shapes follow the paper's experiments (Sec. 4): a tanh indicator
phi0 = [1 + tanh(2 zeta / D)] / 2 of the signed distance zeta to the solid
surface (Sec. 2.1, equilibrium profile), and initial droplets
phi = (1 - phi0) tanh((R - r) / (D / 2)) (Sec. 4.2).  Every array is
(ny, nx), x fastest, float64.  Random draws use numpy's PCG64 generator with
a fixed draw order, so a seed fixes the input bit for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Parameters shared by all of the paper's runs (Sec. 4.1: M = 0.1,
# sigma = 0.001, D = 4, d0 = 0.4, s_i = 1, dx = dt = 1).
PAPER_DEFAULTS = dict(
    d0=0.4, sigma=1e-3, D=4.0, M=0.1,
    rho1=1.0, rho2=1.0, mu1=0.1, mu2=0.1,
    tau_phi=1.0, s0=1.0, s1=1.0, s2=1.0, s3=1.0, s4=1.0,
    gx=0.0, gy=0.0, rho_ref=0.0, fbx=0.0, fby=0.0,
    solid_eps=1e-2,
    # free particles: repulsion threshold and stiffness (eps <= 0: none),
    # wall planes for the particle-wall repulsion (bit 0: y0, 1: y1, 2: x0, 3: x1)
    rep_xi=0.0, rep_eps=0.0, walls=0, wall_x0=0.0, wall_x1=0.0, wall_y0=0.0, wall_y1=0.0,
    # no-flux (bounce-back) walls below the first and above the last row,
    # left of the first and right of the last column
    bounce_y=0, bounce_x=0,
    # H of the pressure recovery: 0 from the model's first-order moments,
    # 1 as printed (Sec. 3.2, after Eq. u)
    h_form=0,
)

# Columns of a particle array: centre, translational and angular velocity,
# radius, density, cos of the contact angle of phase 1 on the particle.
PARTICLE_COLUMNS = ("x", "y", "ux", "uy", "omega", "R", "rho_p", "cos_theta")


def params(nx: int, ny: int, **kw) -> dict:
    p = dict(PAPER_DEFAULTS)
    unknown = set(kw) - set(p)
    if unknown:
        raise KeyError(f"unknown parameters {sorted(unknown)}")
    p.update(kw)
    p["nx"], p["ny"] = int(nx), int(ny)
    return p


@dataclass
class Workload:
    name: str
    params: dict
    phi: np.ndarray
    phi0: np.ndarray
    cos_theta: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    meta: dict = field(default_factory=dict)
    particles: np.ndarray | None = None  # (np, 8), columns PARTICLE_COLUMNS

    @property
    def shape(self):
        return self.phi.shape

    def arrays(self):
        return self.phi, self.phi0, self.cos_theta, self.ux, self.uy


def indicator(zeta: np.ndarray, D: float) -> np.ndarray:
    """Smooth indicator [1 + tanh(2 zeta / D)] / 2 of a signed distance."""
    return 0.5 * (1.0 + np.tanh(2.0 * zeta / D))


def _grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def _per_dist(a: np.ndarray, c: float, n: int) -> np.ndarray:
    d = np.abs(a - c) % n
    return np.minimum(d, n - d)


def _zeros(nx, ny):
    return np.zeros((ny, nx))


# ------------------------------------------------------------------ configs
def droplet_on_slab(nx: int = 64, ny: int = 64, slab_rows: int = 8, R: float = 16.0,
                    theta_deg: float = 90.0, rho_ratio: float = 10.0, mu_ratio: float = 10.0,
                    tau: float = 0.8, tau_phi: float = 0.8, mu1: float | None = None,
                    xc: float | None = None, name: str = "droplet_on_slab", **kw) -> Workload:
    """Semicircular drop resting on a flat solid slab (rows 0 .. slab_rows-1).

    The slab is a periodic band centred at (slab_rows-1)/2 whose tanh
    indicator crosses 1/2 at y = -1/2 and y = slab_rows - 1/2; the drop centre
    sits on the upper surface.  With the defaults this is the 64 x 64, W = 4,
    R = 16, 90 degree, density ratio 10, viscosity ratio 10, M = 0.1,
    relaxation time 0.8 case.  mu1 defaults to rho1 (tau - 1/2) d0 (liquid
    bulk relaxation time tau on the shear rate).
    """
    p = params(nx, ny, **kw)
    d0 = p["d0"]
    rho1 = p["rho1"] if "rho1" in kw else 1.0
    if mu1 is None:
        mu1 = rho1 * (tau - 0.5) * d0
    p.update(rho1=rho1, rho2=rho1 / rho_ratio, mu1=mu1, mu2=mu1 / mu_ratio, tau_phi=tau_phi)
    x, y = _grid(nx, ny)
    half = slab_rows / 2.0
    zeta = half - _per_dist(y, (slab_rows - 1) / 2.0, ny)
    phi0 = indicator(zeta, p["D"])
    xc = nx / 2.0 if xc is None else xc
    yc = slab_rows - 0.5
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    phi = (1.0 - phi0) * np.tanh((R - r) / (p["D"] / 2.0))
    ct = np.full((ny, nx), math.cos(math.radians(theta_deg)))
    return Workload(name, p, phi, phi0, ct, _zeros(nx, ny), _zeros(nx, ny),
                    dict(R=R, theta_deg=theta_deg, slab_rows=slab_rows, xc=xc, yc=yc))


def config1() -> Workload:
    """64 x 64 periodic, slab rows 0-7 (W = 4), R = 16 drop, 90 degrees,
    density ratio 10, viscosity ratio 10, M = 0.1, relaxation times 0.8."""
    return droplet_on_slab(name="C1 drop-on-slab 64x64 fp64")


def cylinder_drop(n: int = 1024, Rp: float = 128.0, R0: float = 160.0, theta_deg: float = 60.0,
                  rho_ratio: float = 100.0, mu_ratio: float = 50.0, g: float = 1e-6,
                  name: str | None = None, **kw) -> Workload:
    """Fixed circular cylinder (radius Rp, centre of an n x n periodic box)
    with a drop of radius R0 tangent to its top (Sec. 4.2 geometry)."""
    p = params(n, n, **kw)
    rho1, mu1 = 1.0, 0.1
    p.update(rho1=rho1, rho2=rho1 / rho_ratio, mu1=mu1, mu2=mu1 / mu_ratio,
             gx=0.0, gy=-g, rho_ref=rho1 / rho_ratio)
    x, y = _grid(n, n)
    c = n / 2.0
    rc = np.sqrt((x - c) ** 2 + (y - c) ** 2)
    phi0 = indicator(Rp - rc, p["D"])
    rd = np.sqrt((x - c) ** 2 + (y - (c + Rp + R0)) ** 2)
    phi = (1.0 - phi0) * np.tanh((R0 - rd) / (p["D"] / 2.0))
    ct = np.full((n, n), math.cos(math.radians(theta_deg)))
    return Workload(name or f"cylinder+drop {n}x{n}", p, phi, phi0, ct, _zeros(n, n), _zeros(n, n),
                    dict(Rp=Rp, R0=R0, theta_deg=theta_deg))


def drop_on_cylinder(n: int = 256, Rp: float = 50.0, R0: float = 50.0, theta_deg: float = 90.0,
                     rho_ratio: float = 10.0, name: str | None = None, **kw) -> Workload:
    """The drop-on-cylinder case of Sec. 4.2: an n x n box (the paper's
    [-L/2, L/2] x [-L/4, 3L/4], cylinder at the origin, i.e. lattice (n/2,
    n/4)), cylinder radius Rp, a drop of radius R0 centred on the top of the
    cylinder surface, phi = (1 - phi0) tanh((R0 - r)/(D/2)); rho1 = 1,
    rho2 = rho1 / rho_ratio and the Sec. 4.1 parameters otherwise.  Periodic in
    y as well (the paper's top and bottom walls are far from the drop)."""
    p = params(n, n, **kw)
    p.update(rho1=1.0, rho2=1.0 / rho_ratio)
    x, y = _grid(n, n)
    cx, cy = n / 2.0, n / 4.0
    phi0 = indicator(Rp - np.hypot(x - cx, y - cy), p["D"])
    phi = (1.0 - phi0) * np.tanh((R0 - np.hypot(x - cx, y - (cy + Rp))) / (p["D"] / 2.0))
    ct = np.full((n, n), math.cos(math.radians(theta_deg)))
    return Workload(name or f"drop on cylinder {n}x{n} theta={theta_deg:g}", p, phi, phi0, ct,
                    _zeros(n, n), _zeros(n, n), dict(Rp=Rp, R0=R0, theta_deg=theta_deg, cx=cx, cy=cy))


def config2() -> Workload:
    """1024 x 1024, cylinder R = 128 at the centre, drop R = 160 on top,
    60 degrees, density ratio 100, viscosity ratio 50, gravity 1e-6."""
    return cylinder_drop(1024, 128.0, 160.0, name="C2 cylinder+drop 1024x1024")


def roofline_grid() -> Workload:
    """The same physics scaled to 4096 x 4096 (working set far above the
    256 MB last-level cache)."""
    return cylinder_drop(4096, 512.0, 640.0, name="R cylinder+drop 4096x4096")


def porous_channel(nx: int = 2048, ny: int = 1024, n_obstacles: int = 200, seed: int = 3,
                   r_range=(8.0, 24.0), theta_range=(45.0, 135.0), wall_rows: int = 8,
                   liquid_frac: float = 0.3, rho_ratio: float = 1000.0, mu_ratio: float = 100.0,
                   body_force: float = 1e-6, max_tries: int = 100000, name: str | None = None,
                   **kw) -> Workload:
    """Channel with diffuse walls (rows 0..wall_rows-1 and the last wall_rows
    rows), circular obstacles placed by rejection, liquid in the left part,
    driven along x by a uniform body force per unit mass: F_b = rho g with
    g = (body_force, 0) (the gravity term with rho_ref = 0).  Applied per
    unit volume instead, the same 1e-6 would accelerate a gas of density
    1e-3 by 1e-3 per step, to |u| ~ 0.5 within 500 steps."""
    p = params(nx, ny, **kw)
    rho1, mu1 = 1.0, 0.1
    p.update(rho1=rho1, rho2=rho1 / rho_ratio, mu1=mu1, mu2=mu1 / mu_ratio,
             gx=body_force, gy=0.0, rho_ref=0.0)
    D = p["D"]
    rng = np.random.default_rng(seed)
    gap = 2.0 * D
    circles = []
    y_lo, y_hi = wall_rows - 0.5, ny - wall_rows - 0.5
    for _ in range(n_obstacles):
        for _t in range(max_tries):
            r = rng.uniform(*r_range)
            cx = rng.uniform(0.0, nx)
            cy = rng.uniform(0.0, ny)
            if cy - r < y_lo + gap or cy + r > y_hi - gap:
                continue
            ok = True
            for (ox, oy, orr) in circles:
                dx = abs(cx - ox) % nx
                dx = min(dx, nx - dx)
                if math.hypot(dx, cy - oy) < r + orr + gap:
                    ok = False
                    break
            if ok:
                circles.append((cx, cy, r))
                break
    thetas = rng.uniform(*theta_range, size=len(circles))
    x, y = _grid(nx, ny)
    # walls: one periodic band of 2*wall_rows rows centred on the y wrap
    phi0 = indicator(wall_rows - _per_dist(y, ny - 0.5, ny), D)
    best = phi0.copy()
    ct = np.zeros((ny, nx))  # neutral walls
    # Each obstacle's indicator is exactly 0 more than 12 D outside its rim
    # (tanh saturates), so it is evaluated on its bounding box only; the sum
    # runs over the obstacles in draw order and the per-node contact angle
    # goes to the largest indicator, ties to the earlier one.
    for (cx, cy, r), th in zip(circles, thetas):
        m = r + 12.0 * D
        rows = np.arange(max(0, math.floor(cy - m)), min(ny, math.ceil(cy + m) + 1))
        if 2 * m + 1 >= nx:
            cols = np.arange(nx)
        else:
            cols = np.arange(math.floor(cx - m), math.ceil(cx + m) + 1) % nx
        box = np.ix_(rows, cols)
        dx = _per_dist(cols.astype(np.float64), cx, nx)[None, :]
        dy = rows.astype(np.float64)[:, None] - cy
        ind = indicator(r - np.sqrt(dx ** 2 + dy ** 2), D)
        phi0[box] += ind
        b = best[box]
        up = ind > b
        best[box] = np.where(up, ind, b)
        ct[box] = np.where(up, math.cos(math.radians(th)), ct[box])
    phi0 = np.clip(phi0, 0.0, 1.0)
    xc = liquid_frac * nx / 2.0
    zeta_l = xc - _per_dist(x, xc, nx)
    phi = (1.0 - phi0) * np.tanh(zeta_l / (D / 2.0))
    return Workload(name or f"C3 porous channel {nx}x{ny}", p, phi, phi0, ct,
                    _zeros(nx, ny), _zeros(nx, ny),
                    dict(circles=circles, thetas=list(map(float, thetas)), seed=seed))


def config3() -> Workload:
    return porous_channel()


def porous_random(n: int = 256, n_obstacles: int = 20, seed: int = 1, theta_deg: float = 90.0,
                  r_range=(8.0, 20.0), **kw) -> Workload:
    """Synthetic stand-in for the micro-CT porous medium of Sec. 4.1: random
    circles and phi = (1 - phi0) rand(-1, 1); rho1 = rho2 = 1, mu = 0.1."""
    p = params(n, n, **kw)
    D = p["D"]
    rng = np.random.default_rng(seed)
    x, y = _grid(n, n)
    phi0 = np.zeros((n, n))
    for _ in range(n_obstacles):
        r = rng.uniform(*r_range)
        cx, cy = rng.uniform(0, n), rng.uniform(0, n)
        dx, dy = _per_dist(x, cx, n), _per_dist(y, cy, n)
        phi0 = phi0 + indicator(r - np.sqrt(dx ** 2 + dy ** 2), D)
    phi0 = np.clip(phi0, 0.0, 1.0)
    phi = (1.0 - phi0) * rng.uniform(-1.0, 1.0, size=(n, n))
    ct = np.full((n, n), math.cos(math.radians(theta_deg)))
    return Workload(f"X1-synthetic porous {n}x{n} theta={theta_deg:g}", p, phi, phi0, ct,
                    _zeros(n, n), _zeros(n, n), dict(seed=seed))


def voxel_solid(nx: int = 256, ny: int = 256, n_grains: int = 40, seed: int = 7,
                r_range=(6.0, 18.0), periodic: bool = True) -> np.ndarray:
    """Synthetic stand-in for a segmented micro-CT image (Sec. 4.1): a binary
    voxel solid (1 in the grains, 0 in the pores) of random disks, rasterised
    node by node, with the staircase boundaries of voxel data.  Draw order per
    grain: r, x, y.  With periodic=False the disks are not wrapped."""
    rng = np.random.default_rng(seed)
    s = np.zeros((ny, nx))
    for _ in range(n_grains):
        r = rng.uniform(*r_range)
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        # the grain's bounding box, wrapped (or cut) at the edges
        xs = np.arange(int(np.floor(cx - r)), int(np.ceil(cx + r)) + 1)
        ys = np.arange(int(np.floor(cy - r)), int(np.ceil(cy + r)) + 1)
        if not periodic:
            xs = xs[(xs >= 0) & (xs < nx)]
            ys = ys[(ys >= 0) & (ys < ny)]
        dx, dy = xs - cx, ys - cy
        inside = dy[:, None] ** 2 + dx[None, :] ** 2 <= r * r
        yy, xx = np.nonzero(inside)
        s[ys[yy] % ny, xs[xx] % nx] = 1.0
    return s


def static_drop(n: int = 64, R: float = 16.0, **kw) -> Workload:
    """Free circular drop in a periodic box, no solid."""
    p = params(n, n, **kw)
    x, y = _grid(n, n)
    c = (n - 1) / 2.0
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2)
    phi = np.tanh((R - r) / (p["D"] / 2.0))
    z = _zeros(n, n)
    return Workload(f"static drop n={n} R={R}", p, phi, z.copy(), z.copy(), z.copy(), z.copy(),
                    dict(R=R, centre=c))


def flat_interface(nx: int = 8, ny: int = 64, **kw) -> Workload:
    """Two planar interfaces at y = ny/4 and 3 ny/4 (tanh profile)."""
    p = params(nx, ny, **kw)
    x, y = _grid(nx, ny)
    c = ny / 2.0
    zeta = ny / 4.0 - _per_dist(y, c - 0.5, ny)
    phi = np.tanh(2.0 * zeta / p["D"])
    z = _zeros(nx, ny)
    return Workload("flat interface", p, phi, z.copy(), z.copy(), z.copy(), z.copy(), {})


def random_state(nx: int, ny: int, seed: int = 0, solid: bool = True, theta_range=(30.0, 150.0),
                 amp_u: float = 1e-3, **kw) -> Workload:
    """Seeded random-but-smooth state for parity tests: a few circular solids
    with random contact angles, random drops, and a small random velocity."""
    p = params(nx, ny, **kw)
    D = p["D"]
    rng = np.random.default_rng(seed)
    x, y = _grid(nx, ny)
    phi0 = np.zeros((ny, nx))
    ct = np.zeros((ny, nx))
    best = np.zeros((ny, nx))
    if solid:
        for _ in range(3):
            r = rng.uniform(3.0, max(3.5, min(nx, ny) / 6.0))
            cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
            part = indicator(r - np.sqrt(_per_dist(x, cx, nx) ** 2 + _per_dist(y, cy, ny) ** 2), D)
            c = math.cos(math.radians(rng.uniform(*theta_range)))
            ct = np.where(part > best, c, ct)
            best = np.maximum(best, part)
            phi0 += part
    phi0 = np.clip(phi0, 0.0, 1.0)
    field_ = -np.ones((ny, nx))
    for _ in range(3):
        r = rng.uniform(3.0, max(3.5, min(nx, ny) / 4.0))
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        d = np.sqrt(_per_dist(x, cx, nx) ** 2 + _per_dist(y, cy, ny) ** 2)
        field_ = np.maximum(field_, np.tanh((r - d) / (D / 2.0)))
    phi = (1.0 - phi0) * field_
    ux = amp_u * rng.standard_normal((ny, nx)) * (1.0 - phi0)
    uy = amp_u * rng.standard_normal((ny, nx)) * (1.0 - phi0)
    return Workload(f"random state {nx}x{ny} seed={seed}", p, phi, phi0, ct, ux, uy, dict(seed=seed))


# ------------------------------------------------------------ served stream
@dataclass
class JobSpec:
    job_id: int
    side: int
    theta_deg: float
    rho_ratio: float
    steps: int
    arrival_s: float = 0.0

    def workload(self, mu1: float = 1.0, mu_ratio: float = 10.0, **kw) -> Workload:
        """Drop-on-slab job: L x L periodic, slab rows [0, L/8), drop radius
        L/4 on the slab, density ratio r with rho2 = 1/r; viscosities mu1 and
        mu2 = mu1 / mu_ratio (the stream fixes no viscosity; with 1.0 and 10
        the jobs of density ratio up to 100 stay finite over 20 000 steps
        except strongly spreading ones on the smallest grid: 2 of the 256 jobs
        of the seeded stream, 128^2 at 34 and 43 degrees, ratios 61 and 88)."""
        L = self.side
        return droplet_on_slab(nx=L, ny=L, slab_rows=L // 8, R=L / 4.0, theta_deg=self.theta_deg,
                               rho_ratio=self.rho_ratio, mu_ratio=mu_ratio, mu1=mu1,
                               tau_phi=1.0, name=f"job{self.job_id} {L}x{L}", **kw)


def job_stream(n_jobs: int = 256, seed: int = 4, sides=(128, 256, 512, 1024),
               theta_range=(30.0, 150.0), ratio_range=(10.0, 1000.0),
               steps_range=(2000, 20000), rate_per_s: float | None = None):
    """Seeded stream of drop-on-slab jobs.  Arrival times are a Poisson
    process of the given rate (all at t = 0 when rate is None)."""
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for j in range(n_jobs):
        side = int(sides[rng.integers(0, len(sides))])
        th = float(rng.uniform(*theta_range))
        ratio = float(rng.uniform(*ratio_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        gap = float(rng.exponential(1.0))
        if rate_per_s is not None:
            t += gap / rate_per_s
        jobs.append(JobSpec(j, side, th, ratio, steps, t if rate_per_s is not None else 0.0))
    return jobs


# ------------------------------------------------------------ free particles
def particle(x, y, R, rho_p, theta_deg=90.0, ux=0.0, uy=0.0, omega=0.0) -> list:
    """One row of a particle array (columns PARTICLE_COLUMNS)."""
    return [float(x), float(y), float(ux), float(uy), float(omega), float(R), float(rho_p),
            math.cos(math.radians(theta_deg))]


def particles_in_fluid(n: int = 48, parts=None, phi_value: float = 0.0, ux: float = 0.0,
                       uy: float = 0.0, name: str = "particles in fluid", **kw) -> Workload:
    """Periodic n x n box of one fluid state phi = phi_value everywhere (0: the
    50/50 mixture, where the chemical potential and mu_phi0 vanish), uniform
    velocity, no stationary solid, the given particles."""
    p = params(n, n, **kw)
    z = _zeros(n, n)
    phi = np.full((n, n), float(phi_value))
    return Workload(name, p, phi, z.copy(), z.copy(), np.full((n, n), float(ux)),
                    np.full((n, n), float(uy)), {}, np.array(parts if parts is not None else [], float).reshape(-1, 8))


def pool_with_particles(nx: int = 1024, ny: int = 2048, n_particles: int = 64, seed: int = 5,
                        r_range=(12.0, 20.0), rho_ratio_p: float = 2.0, theta_deg: float = 70.0,
                        rho2: float = 0.1, mu1: float = 0.3, mu_ratio: float = 10.0, g: float = 1e-6,
                        wall: int = 8, name: str | None = None, **kw) -> Workload:
    """Gas-liquid-particle box: diffuse walls of `wall` rows/columns on all four
    sides (90 degrees), a liquid pool filling the lower half, n particles of
    radius U[r_range] and density rho_ratio_p * rho1 placed without overlap
    (gap >= 2 D, also from the walls and the pool surface) in the gas above,
    contact angle theta on every particle, gravity (0, -g) on fluid and
    particles (rho_ref = rho2), particle-particle and particle-wall repulsion
    with threshold D/2 and a stiffness that makes the repulsion at half the
    threshold about ten times a particle's weight."""
    rng = np.random.default_rng(seed)
    p = params(nx, ny, **kw)
    D = p["D"]
    p.update(rho1=1.0, rho2=rho2, mu1=mu1, mu2=mu1 / mu_ratio, gy=-g, rho_ref=rho2,
             rep_xi=D / 2.0, rep_eps=2e-3 / g, walls=15,
             wall_x0=wall - 0.5, wall_x1=nx - wall - 0.5, wall_y0=wall - 0.5, wall_y1=ny - wall - 0.5)
    x, y = _grid(nx, ny)
    # distance into the walls, positive inside the solid band
    zeta = np.maximum.reduce([wall - 0.5 - x, x - (nx - wall - 0.5), wall - 0.5 - y, y - (ny - wall - 0.5)])
    phi0 = indicator(zeta, D)
    level = ny / 2.0
    parts = []
    tries = 0
    while len(parts) < n_particles and tries < 200000:
        tries += 1
        R = float(rng.uniform(*r_range))
        xc = float(rng.uniform(wall + R + 2 * D, nx - wall - R - 2 * D))
        yc = float(rng.uniform(level + R + 2 * D, ny - wall - R - 2 * D))
        if all(math.hypot(xc - q[0], yc - q[1]) >= R + q[5] + 2 * D for q in parts):
            parts.append(particle(xc, yc, R, rho_ratio_p * p["rho1"], theta_deg))
    parts = np.array(parts, float).reshape(-1, 8)
    phi = (1.0 - phi0) * np.tanh((level - y) / (D / 2.0))
    for q in parts:  # phi = 0 inside the particles (Sec. 4.5 initial condition)
        r = np.hypot(x - q[0], y - q[1])
        phi *= 1.0 - indicator(q[5] - r, D)
    ct = np.zeros((ny, nx))
    return Workload(name or f"C5 pool + {len(parts)} particles {nx}x{ny}", p, phi, phi0, ct,
                    _zeros(nx, ny), _zeros(nx, ny), dict(seed=seed, n_particles=len(parts)), parts)


# ------------------------------------------------------- three dimensions
PAPER_DEFAULTS_3D = dict(
    d0=0.4, sigma=1e-3, D=4.0, M=0.1,
    rho1=1.0, rho2=1.0, mu1=0.1, mu2=0.1,
    tau_phi=1.0, s0=1.0, s1=1.0, s2=1.0, s3=1.0, s4=1.0,
    gx=0.0, gy=0.0, gz=0.0, rho_ref=0.0, fbx=0.0, fby=0.0, fbz=0.0,
    solid_eps=1e-2,
)


def params3(nx: int, ny: int, nz: int, **kw) -> dict:
    """Parameters of the three-dimensional path (the Sec. 4.1 values)."""
    p = dict(PAPER_DEFAULTS_3D)
    unknown = set(kw) - set(p)
    if unknown:
        raise KeyError(f"unknown parameters {sorted(unknown)}")
    p.update(kw)
    p["nx"], p["ny"], p["nz"] = int(nx), int(ny), int(nz)
    return p


@dataclass
class Workload3:
    name: str
    params: dict
    phi: np.ndarray       # (nz, ny, nx)
    phi0: np.ndarray
    cos_theta: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    meta: dict = field(default_factory=dict)

    def arrays(self):
        return self.phi, self.phi0, self.cos_theta, self.ux, self.uy, self.uz


def drop_on_slab_3d(nx: int = 64, ny: int | None = None, nz: int | None = None, slab: int = 8,
                    R: float = 16.0, theta_deg: float = 90.0, rho_ratio: float = 10.0, mu_ratio: float = 10.0,
                    mu1: float = 0.1, name: str | None = None, **kw) -> Workload3:
    """A spherical drop of radius R resting on a solid slab (z < slab, tanh
    indicator of width D), contact angle theta on the slab, periodic box;
    rho1 = 1, rho2 = 1/rho_ratio, mu2 = mu1/mu_ratio."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    p = params3(nx, ny, nz, **kw)
    p.update(rho1=1.0, rho2=1.0 / rho_ratio, mu1=mu1, mu2=mu1 / mu_ratio)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    phi0 = indicator(slab - 0.5 - z, p["D"])
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - slab) ** 2)
    phi = (1.0 - phi0) * np.tanh((R - r) / (p["D"] / 2.0))
    zero = np.zeros_like(phi)
    ct = np.full_like(phi, math.cos(math.radians(theta_deg)))
    return Workload3(name or f"3-D drop on slab {nx}x{ny}x{nz}", p, phi, phi0, ct, zero, zero.copy(), zero.copy(),
                     dict(R=R, slab=slab, theta_deg=theta_deg))


def bench_3d() -> Workload3:
    """The 3-D benchmark domain: 256^3 (16.8M nodes), a drop of radius 64 on a
    slab of 16 rows, contact angle 60 degrees, density ratio 10."""
    return drop_on_slab_3d(256, slab=16, R=64.0, theta_deg=60.0, rho_ratio=10.0, mu_ratio=10.0,
                           mu1=0.1, name="3-D drop on slab 256^3, theta=60, rho ratio 10")
