"""Pins of the oracle's free-particle path (Sec. 2.4, procedure steps 7-10,
Sec. 4.5 repulsion) against what the model and the mathematics fix: the
stationary-solid limit, Galilean translation, a discrete momentum balance
between fluid and particle, the first updates from rest under gravity, the
sense of rotational drag and the repulsion's properties.

Most cases use phi = 0 everywhere (the 50/50 mixture) with a 90 degree
contact angle: there the chemical potential, the mass flux and mu_phi0 all
vanish (Eq. muPhi0 and the remark after it), so only the particle coupling
acts on the flow.
"""
import math

import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W


def _oracle(orc, w):
    return orc.Oracle(w.params, *w.arrays(), particles=w.particles)


def _disk(n, xc, yc, R, D):
    """Indicator of a disk with the nearest periodic image, at every node."""
    y, x = np.mgrid[0:n, 0:n].astype(float)
    dx = (x - xc + n / 2) % n - n / 2
    dy = (y - yc + n / 2) % n - n / 2
    r = np.hypot(dx, dy)
    return W.indicator(R - r, D)


def test_heavy_particle_is_a_stationary_solid(orc):
    """A particle of enormous density cannot move: the flow past it equals the
    flow past the same disk given as a stationary solid."""
    n, R = 40, 7.0
    kw = dict(fbx=2e-6, mu1=0.1, mu2=0.1)
    wp = W.particles_in_fluid(n, [W.particle(17.3, 21.6, R, 1e30)], **kw)
    ws = W.particles_in_fluid(n, None, **kw)
    ws.phi0[:] = _disk(n, 17.3, 21.6, R, wp.params["D"])
    a, b = _oracle(orc, wp), _oracle(orc, ws)
    assert np.abs(a.field("phi0") - b.field("phi0")).max() < 1e-15
    a.step(150)
    b.step(150)
    for fa, fb in zip(a.read()[1:], b.read()[1:]):
        assert np.abs(fa - fb).max() <= 1e-12 * np.abs(fb).max()
    st, out = a.particles()
    assert abs(st[0, 2]) < 1e-20 and abs(st[0, 3]) < 1e-20
    # the drag on it is along the driving force
    assert out[0, 0] > 0 and abs(out[0, 1]) < 1e-3 * out[0, 0]


def test_particle_carried_by_uniform_flow(orc):
    """Galilean case: a neutrally buoyant particle moving with a uniform flow
    feels no force; it moves at exactly that velocity (explicit Euler),
    crosses the periodic boundary, and its regenerated indicator follows."""
    n, R, U = 36, 6.0, (0.07, -0.03)
    w = W.particles_in_fluid(n, [W.particle(31.2, 3.4, R, 1.0, ux=U[0], uy=U[1])], ux=U[0], uy=U[1])
    o = _oracle(orc, w)
    steps = 120
    o.step(steps)
    st, out = o.particles()
    xe, ye = (31.2 + steps * U[0]) % n, (3.4 + steps * U[1]) % n
    assert abs(st[0, 0] - xe) < 1e-10 and abs(st[0, 1] - ye) < 1e-10
    assert abs(st[0, 2] - U[0]) < 1e-13 and abs(st[0, 3] - U[1]) < 1e-13 and abs(st[0, 4]) < 1e-13
    _, ux, uy, P = o.read()
    assert np.abs(ux - U[0]).max() < 1e-13 and np.abs(uy - U[1]).max() < 1e-13
    assert np.abs(P).max() < 1e-13
    assert np.abs(o.field("phi0") - _disk(n, st[0, 0], st[0, 1], R, w.params["D"])).max() < 1e-13


def _fluid_momentum(o):
    g, f = o.pops()
    w, cx, cy = orc_lattice(o)
    return np.array([np.tensordot(cx, f, axes=(0, 0)).sum(), np.tensordot(cy, f, axes=(0, 0)).sum()])


def orc_lattice(o):
    from oracle import oracle as O
    return O.lattice(o.params["d0"])


@pytest.mark.parametrize("rho_p", [0.6, 3.0])
def test_fluid_particle_momentum_balance(orc, rho_p):
    """Newton's third law through the coupling.  The fluid gains sum rho f per
    collision; the particle gains F_f = -sum rho f plus the internal-fluid
    correction F^in of the previous update.  Hence
        J = P_fluid - F_f + (M_p - rho_in V_p) u_p + F^in
    is the same after every update (derived from Eqs. particle, Ff, Ffin and
    the forcing of Sec. 3.2; the other forces sum to zero on a periodic box)."""
    n, R = 40, 6.5
    parts = [W.particle(15.2, 19.7, R, rho_p, ux=0.02, uy=-0.011, omega=0.003),
             W.particle(29.0, 30.5, 5.0, rho_p, ux=-0.015, uy=0.004)]
    w = W.particles_in_fluid(n, parts, mu1=0.05, mu2=0.05)
    o = _oracle(orc, w)
    J = []
    for k in range(40):
        o.step(1)
        if k < 1:
            continue
        st, out = o.particles()
        Pf = _fluid_momentum(o)
        j = Pf.copy()
        for q, r in zip(st, out):
            V = math.pi * q[5] ** 2
            M = q[6] * V
            j += -r[0:2] + (M - r[6] * V) * q[2:4] + r[3:5]
        J.append(j)
    J = np.array(J)
    scale = np.abs(J).max()
    assert np.abs(J - J[0]).max() <= 1e-12 * scale, np.abs(J - J[0]).max() / scale
    # and the particles did exchange momentum with the fluid
    assert np.abs(_fluid_momentum(o)).max() > 1e-3 * scale


def test_first_updates_from_rest_under_gravity(orc):
    """From rest in a neutral fluid (rho_ref = rho = 1, so the fluid itself
    feels no gravity): the first update sees no hydrodynamic force, so
    u_p = (1 - rho/rho_p) g; the position still uses the old velocity (0); the
    second update adds the drag of the fluid held by the moving indicator,
    -sum_owned phi0 * u_p, and the internal-fluid correction rho V_p u_p."""
    n, R, rp, g = 40, 6.0, 2.5, (0.0, -2e-4)
    w = W.particles_in_fluid(n, [W.particle(20.4, 19.1, R, rp)], gx=g[0], gy=g[1], rho_ref=1.0)
    o = _oracle(orc, w)
    o.step(1)
    st, out = o.particles()
    u1 = (1.0 - 1.0 / rp) * np.array(g)
    assert np.allclose(st[0, 2:4], u1, rtol=0, atol=1e-18)
    assert st[0, 0] == 20.4 and st[0, 1] == 19.1
    assert np.allclose(out[0, :3], 0.0, atol=1e-18) and abs(out[0, 6] - 1.0) < 1e-14
    own = o.field("owner") == 0
    S0 = o.field("phi0")[own].sum()
    V = math.pi * R * R
    M = rp * V
    o.step(1)
    st2, out2 = o.particles()
    u2 = u1 + (-S0 * u1 + V * u1 + (1.0 - 1.0 / rp) * M * np.array(g)) / M
    assert np.allclose(out2[0, :2], -S0 * u1, rtol=1e-12, atol=1e-30)
    assert np.allclose(st2[0, 2:4], u2, rtol=1e-12, atol=1e-30)
    assert abs(st2[0, 1] - (19.1 + u1[1])) < 1e-15


def test_rotating_particle_slows_and_drives_the_fluid(orc):
    """Rotational drag: a spinning particle in fluid at rest slows down
    without reversing, and the fluid around it turns in the same sense."""
    n, R, om = 44, 8.0, 4e-3
    w = W.particles_in_fluid(n, [W.particle(22.0, 22.0, R, 2.0, omega=om)])
    o = _oracle(orc, w)
    prev = om
    for _ in range(6):
        o.step(10)
        st, out = o.particles()
        assert 0.0 < st[0, 4] < prev
        prev = st[0, 4]
    assert out[0, 2] < 0  # the torque opposes the spin
    _, ux, uy, _ = o.read()
    y, x = np.mgrid[0:n, 0:n].astype(float)
    rx, ry = x - 22.0, y - 22.0
    ring = (np.hypot(rx, ry) > R + 2) & (np.hypot(rx, ry) < R + 8)
    assert (rx * uy - ry * ux)[ring].sum() > 0


def test_repulsion_properties(orc):
    """Sec. 4.5 repulsion: zero beyond the threshold, along the line of
    centres, odd in the separation, vanishing continuously at the outer
    threshold and growing as the gap closes."""
    xi, eps, rs = 2.0, 50.0, 20.0
    d = np.array([0.6, 0.8])
    for gap in (xi + 1e-9, 3.0, 10.0):
        assert np.all(orc.repulsion(*(d * (rs + gap)), rs, xi, eps) == 0.0)
    vals = []
    for gap in (1.9, 1.5, 1.0, 0.5, 0.01):
        f = orc.repulsion(*(d * (rs + gap)), rs, xi, eps)
        assert f[0] > 0 and abs(f[0] * d[1] - f[1] * d[0]) < 1e-15 * abs(f).max()
        assert np.allclose(orc.repulsion(*(-d * (rs + gap)), rs, xi, eps), -f, rtol=0, atol=0)
        vals.append(np.hypot(*f))
    assert all(a < b for a, b in zip(vals, vals[1:]))
    near = np.hypot(*orc.repulsion(*(d * (rs + xi - 1e-6)), rs, xi, eps))
    assert near < 1e-9


def test_wall_repulsion_pushes_particle_away(orc):
    """A particle at rest just inside the repulsion range of a wall plane is
    pushed away from it (mirror image across the plane, Sec. 4.5)."""
    n, R = 40, 6.0
    w = W.particles_in_fluid(n, [W.particle(20.0, 12.7, R, 2.0)], rep_xi=2.0, rep_eps=50.0,
                             walls=1, wall_y0=6.0)
    o = _oracle(orc, w)
    o.step(1)
    st, _ = o.particles()
    assert st[0, 3] > 0 and abs(st[0, 2]) < 1e-12 * st[0, 3]


def _interface_case(orc, theta, n=40, H=64, R=9.0, steps=800):
    """Neutral particle centred on the upper of two flat interfaces: phase 1
    (phi = +1) fills |y - H/2| < H/4, equal densities and viscosities."""
    p = W.params(n, H)
    D = p["D"]
    y, x = np.mgrid[0:H, 0:n].astype(float)
    phi = np.tanh((H / 4.0 - np.abs(y - H / 2.0)) / (D / 2.0))
    dy = (y - 0.75 * H + H / 2.0) % H - H / 2.0  # nearest periodic image
    phi = phi * (1.0 - W.indicator(R - np.hypot(x - n / 2.0, dy), D))
    o = orc.Oracle(p, phi, np.zeros_like(phi), particles=[W.particle(n / 2.0, 0.75 * H, R, 1.0, theta)])
    o.step(steps)
    return o


def test_particle_at_interface_moves_into_the_wetting_phase(orc):
    """Capillarity on a free particle (mu_phi0 grad phi0, Eq. muPhi0, and the
    wetting terms): a particle wetted preferentially by phase 1 (60 degrees)
    sinks into phase 1, its mirror case (120 degrees) rises into phase 2 by the
    same distance.  Reflecting about the interface and swapping the phases maps
    one case onto the other exactly (the lattice, stencils, energy and equal
    fluid properties are all symmetric), so the two displacements are opposite
    to round-off; equilibrium (centre R cos(theta) into phase 1, the zero-Bond
    limit of the single-particle balance of Sec. 4.4) is far slower than this
    run."""
    H = 64
    a = _interface_case(orc, 60.0, H=H)
    b = _interface_case(orc, 120.0, H=H)
    ya = a.particles()[0][0, 1] - 0.75 * H
    yb = b.particles()[0][0, 1] - 0.75 * H
    assert ya < -0.01
    assert abs(ya + yb) < 1e-10 * abs(ya)
    # the fields are mirror images with phi -> -phi
    pa, pb = a.field("phi"), b.field("phi")
    mirror = (2 * (3 * H // 4) - np.arange(H)) % H
    assert np.abs(pa + pb[mirror, :]).max() < 1e-11


def test_prescribed_rotation_couette_torque_balance(orc):
    """A solid of prescribed motion (rho_p <= 0: the rotating inner cylinder
    of Sec. 4.5) inside a stationary ring: its angular velocity is held, the
    fluid turns with it and reaches a steady circular Couette flow, and at
    steady state the torque the fluid exerts on the cylinder (reported by the
    particle update, Eq. Ff) balances the torque of the ring's penalty force
    on the fluid (angular-momentum balance: viscous and pressure forces are
    internal)."""
    n, Rin, Rout, om = 64, 10.0, 28.0, 2e-3
    p = W.params(n, n)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    c = n / 2.0
    r = np.hypot(x - c, y - c)
    zb = W.indicator(r - Rout, p["D"])
    o = orc.Oracle(p, np.zeros((n, n)), zb, particles=[W.particle(c, c, Rin, -1.0, 90.0, omega=om)])
    o.step(3000)
    st, out = o.particles()
    assert st[0, 4] == om and st[0, 2] == 0.0 and st[0, 3] == 0.0 and st[0, 0] == c
    own = o.field("owner") < 0
    rho = o.field("rho")
    fx, fy = rho * o.field("asx"), rho * o.field("asy")
    t_ring = ((x - c) * fy - (y - c) * fx)[own].sum()  # torque of the ring on the fluid
    assert out[0, 2] < 0  # the fluid brakes the cylinder
    # balanced up to what is left of the start-up transient (the slowest
    # viscous mode of the gap decays over ~(Rout - Rin)^2 / (nu pi^2) ~ 330
    # steps; a wrong sign or lever arm would be off by 50-200%)
    assert abs(out[0, 2] - t_ring) <= 1e-3 * abs(t_ring)
    # and the fluid between turns with the cylinder, fastest near it
    _, ux, uy, _ = o.read()
    ut = (-(y - c) * ux + (x - c) * uy) / np.maximum(r, 1e-9)
    prof = [ut[np.abs(r - rr) < 0.5].mean() for rr in (14.0, 19.0, 24.0)]
    assert prof[0] > prof[1] > prof[2] > 0
