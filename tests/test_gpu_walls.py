"""No-flux bounce-back walls in y on the GPU against the FP64 CPU oracle,
element by element, on a ragged domain (every tile shape leaves a partial
tile row next to the upper wall), with two phases of different density and
viscosity, a wetting stationary solid, gravity, a body force and a shear
flow; free particles between walls; the discrete channel flow in closed
form; walled and periodic domains in one batch.

Bars: FP64 <= 1e-12 relative on phi, u and P; FP32 <= 1e-5 relative;
FP16-dev within its storage quantisation (1e-3 on phi) and with the phase
mass conserved exactly.
"""
import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W
from parity import BAR, check, errors, fmt, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_05097_amd import lbmgls
    lbmgls.lib()
    return lbmgls


def wall_case(nx=67, ny=45):
    """A drop sitting on the lower wall, a smaller one touching the upper
    wall, a wetting cylinder between them, gravity, a body force along x and
    a shear flow."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = np.tanh((9.0 - np.hypot(x - 20.0, y + 0.5)) / 1.5)
    phi = np.maximum(phi, np.tanh((6.0 - np.hypot(x - 45.0, y - (ny - 4.0))) / 1.5))
    ux = 0.004 * (y + 0.5) / ny
    p = W.params(nx, ny, bounce_y=1, rho1=1.0, rho2=0.3, mu1=0.1, mu2=0.04, gy=-1e-5, rho_ref=0.5,
                 D=3.0, fbx=2e-6)
    z = W.indicator(4.0 - np.hypot(x - 55.0, y - 20.0), 3.0)
    return p, phi, z, np.full((ny, nx), 0.3), ux


def _pair(gpu, storage, steps, tile=0, case=wall_case):
    from oracle.oracle import Oracle
    p, phi, z, ct, ux = case()
    o = Oracle(p, phi, z, ct, ux, None)
    d = gpu.Domain(p, phi, z, ct, ux, None, storage=storage, tile=tile)
    o.step(steps)
    d.step(steps)
    errs = errors(d.read(), o.read())
    print(f"\nwalls {storage} tile {tile} {steps} steps: " + fmt(errs))
    return d, o, errs


@pytest.mark.parametrize("tile", [4, 16])
def test_walls_fp64_parity(gpu, tile):
    d, o, errs = _pair(gpu, "fp64", 300, tile)
    check(errs, BAR["fp64"])
    assert abs(d.mass() - o.mass()) <= 1e-11 * np.abs(o.field("phi")).sum()


def test_walls_fp32_parity(gpu):
    d, o, errs = _pair(gpu, "fp32", 300, 8)
    check(errs, BAR["fp32"])


def test_walls_fp16dev_exact_mass(gpu):
    d, o, errs = _pair(gpu, "fp16dev", 300, 8)
    assert errs["phi"][0] <= 1e-3
    p, phi, z, ct, ux = wall_case()
    d0 = gpu.Domain(p, phi, z, ct, ux, None, storage="fp16dev", tile=8)
    assert d.mass() == d0.mass()  # the fixed-point total, exact in 16-bit modes


def test_walls_tile_shapes_bitwise(gpu):
    p, phi, z, ct, ux = wall_case()
    ref = None
    for ty in (4, 8, 16, 32):
        d = gpu.Domain(p, phi, z, ct, ux, None, storage="fp32", tile=ty)
        d.step(41)
        got = d.read()
        if ref is None:
            ref = got
        else:
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), ty


def test_walls_domain_lower_than_a_tile(gpu):
    """ny = 8 under 64 x 32 tiles: the ghost rows fold back into the domain
    for the tile rows beyond both walls."""
    def small():
        p, phi, z, ct, ux = wall_case(70, 8)
        return p, phi, z, ct, ux
    d, o, errs = _pair(gpu, "fp32", 60, 32, case=small)
    check(errs, BAR["fp32"])


def test_poiseuille_closed_form_gpu(gpu):
    """The discrete steady channel flow between bounce-back walls (derived in
    the oracle's wall pins): u_j = F/(2 nu)(j + 1/2)(H - 1/2 - j) + F/(2 d0)
    - F/2 - F/(8 nu) for the third-order rate 1, in FP64."""
    H, nx, mu, F, d0 = 16, 64, 0.125, 1e-8, 0.4
    p = W.params(nx, H, mu1=mu, mu2=mu, fbx=F, bounce_y=1)
    phi = np.ones((H, nx))
    d = gpu.Domain(p, phi, np.zeros_like(phi), storage="fp64")
    d.step(6000)
    _, ux, uy, _ = d.read()
    j = np.arange(H)
    ue = F / (2 * mu) * (j + 0.5) * (H - 0.5 - j) + F / (2 * d0) - F / 2 - F / (8 * mu)
    assert np.abs(ux - ue[:, None]).max() <= 1e-9 * ue.max()


def test_particles_between_walls_fp64(gpu):
    """Free particles next to both walls (one pressed against the upper wall
    plane by its velocity, one of prescribed motion), wall repulsion at the
    bounce-back planes; fields, particle state and forces against the
    oracle."""
    from oracle.oracle import Oracle
    nx, ny = 67, 45
    p = W.params(nx, ny, bounce_y=1, rho2=0.5, mu2=0.05, gy=-2e-5, rho_ref=0.5, rep_xi=2.0, rep_eps=50.0,
                 walls=3, wall_y0=-0.5, wall_y1=ny - 0.5)
    D = p["D"]
    parts = np.array([W.particle(14.3, 5.2, 5.5, 1.6, 60.0, ux=0.002, uy=-0.003),
                      W.particle(40.5, 39.9, 7.0, 0.9, 120.0, omega=1e-3, uy=0.002),
                      W.particle(30.0, 22.0, 4.0, -1.0, 75.0, ux=0.001, omega=-2e-3)])
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = np.tanh((22.0 - y) / (D / 2))
    for q in parts:
        dx = (x - q[0] + nx / 2) % nx - nx / 2
        phi *= 1.0 - W.indicator(q[5] - np.hypot(dx, y - q[1]), D)
    z = np.zeros_like(phi)
    o = Oracle(p, phi, z, None, None, None, particles=parts)
    d = gpu.Domain(p, phi, z, storage="fp64", tile=8, particles=parts)
    o.step(300)
    d.step(300)
    for a, b in zip(d.read(), o.read()):
        assert rel(a, b) <= 1e-12
    ds, do = d.particles()
    os_, oo = o.particles()
    assert np.abs(ds - os_).max() <= 1e-10
    assert np.abs(do[:, :3] - oo[:, :3]).max() <= 1e-10 * np.abs(oo[:, :3]).max()


def test_walled_and_periodic_domains_in_one_batch(gpu):
    """A batch holds each member's boundary kind: a walled and a periodic
    domain stepped together equal their solo runs bit for bit."""
    p, phi, z, ct, ux = wall_case()
    pp = dict(p, bounce_y=0)
    batch = gpu.Batch(storage="fp32", tile=8, max_members=2)
    a = batch.domain(p, phi, z, ct, ux, None, tile=8)
    b = batch.domain(pp, phi, z, ct, ux, None, tile=8)
    batch.add(a)
    batch.add(b)
    batch.step(37)
    for q, ref_p in ((a, p), (b, pp)):
        solo = gpu.Domain(ref_p, phi, z, ct, ux, None, storage="fp32", tile=8)
        solo.step(37)
        for u, v in zip(q.read(), solo.read()):
            assert np.array_equal(u, v)
    assert not np.array_equal(a.read()[0], b.read()[0])


def box_case(bx=1, by=1, nx=67, ny=45):
    """Walls in x (and y): a drop in the lower left corner, one at the right
    wall, one at the upper wall, a wetting cylinder, gravity with a sideways
    component and a swirling initial flow; ragged in both directions."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = np.maximum(np.tanh((10.0 - np.hypot(x + 0.5, y + 0.5)) / 1.5),
                     np.tanh((6.0 - np.hypot(x - (nx - 8.0), y - 20.0)) / 1.5))
    phi = np.maximum(phi, np.tanh((5.0 - np.hypot(x - 30.0, y - (ny - 2.0))) / 1.5))
    ux = 0.003 * np.sin(np.pi * (y + 0.5) / ny)
    uy = -0.002 * np.sin(np.pi * (x + 0.5) / nx)
    p = W.params(nx, ny, bounce_x=bx, bounce_y=by, rho1=1.0, rho2=0.3, mu1=0.1, mu2=0.04, gy=-1e-5, gx=3e-6,
                 rho_ref=0.5, D=3.0)
    z = W.indicator(4.0 - np.hypot(x - 45.0, y - 14.0), 3.0)
    return p, phi, z, np.full((ny, nx), 0.3), ux, uy


def _box_pair(gpu, storage, steps, tile, bx=1, by=1):
    from oracle.oracle import Oracle
    p, phi, z, ct, ux, uy = box_case(bx, by)
    o = Oracle(p, phi, z, ct, ux, uy)
    d = gpu.Domain(p, phi, z, ct, ux, uy, storage=storage, tile=tile)
    o.step(steps)
    d.step(steps)
    errs = errors(d.read(), o.read())
    print(f"\nbox x={bx} y={by} {storage} tile {tile} {steps} steps: "
          + fmt(errs))
    return d, o, errs


@pytest.mark.parametrize("bx,by,tile", [(1, 1, 8), (1, 0, 16), (1, 1, 4)])
def test_side_walls_and_closed_box_fp64_parity(gpu, bx, by, tile):
    d, o, errs = _box_pair(gpu, "fp64", 300, tile, bx, by)
    check(errs, BAR["fp64"])


def test_closed_box_fp32_parity_and_tiles_bitwise(gpu):
    d, o, errs = _box_pair(gpu, "fp32", 300, 8)
    check(errs, BAR["fp32"])
    p, phi, z, ct, ux, uy = box_case()
    ref = None
    for ty in (4, 8, 16, 32):
        d = gpu.Domain(p, phi, z, ct, ux, uy, storage="fp32", tile=ty)
        d.step(41)
        got = d.read()
        if ref is None:
            ref = got
        else:
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), ty


def test_closed_box_fp16dev_exact_mass(gpu):
    d, o, errs = _box_pair(gpu, "fp16dev", 300, 16)
    assert errs["phi"][0] <= 1e-3
    p, phi, z, ct, ux, uy = box_case()
    d0 = gpu.Domain(p, phi, z, ct, ux, uy, storage="fp16dev", tile=16)
    assert d.mass() == d0.mass()


def test_particles_in_a_closed_box_fp64(gpu):
    """Particles next to every wall of a closed box (repulsion planes on the
    wall lines), one of prescribed motion; fields, state and forces against
    the oracle."""
    from oracle.oracle import Oracle
    nx, ny = 67, 45
    p = W.params(nx, ny, bounce_x=1, bounce_y=1, rho2=0.5, mu2=0.05, gy=-2e-5, gx=4e-6, rho_ref=0.5,
                 rep_xi=2.0, rep_eps=50.0, walls=15, wall_y0=-0.5, wall_y1=ny - 0.5, wall_x0=-0.5,
                 wall_x1=nx - 0.5)
    D = p["D"]
    parts = np.array([W.particle(5.1, 5.2, 5.5, 1.6, 60.0, ux=-0.002, uy=-0.003),
                      W.particle(61.5, 38.9, 6.0, 0.9, 120.0, omega=1e-3, ux=0.003),
                      W.particle(30.0, 22.0, 4.0, -1.0, 75.0, ux=0.001, omega=-2e-3)])
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = np.tanh((22.0 - y) / (D / 2))
    for q in parts:
        phi *= 1.0 - W.indicator(q[5] - np.hypot(x - q[0], y - q[1]), D)
    z = np.zeros_like(phi)
    o = Oracle(p, phi, z, None, None, None, particles=parts)
    d = gpu.Domain(p, phi, z, storage="fp64", tile=16, particles=parts)
    o.step(300)
    d.step(300)
    for a, b in zip(d.read(), o.read()):
        assert rel(a, b) <= 1e-12
    ds, do = d.particles()
    os_, oo = o.particles()
    assert np.abs(ds - os_).max() <= 1e-10
    assert np.abs(do[:, :3] - oo[:, :3]).max() <= 1e-10 * np.abs(oo[:, :3]).max()


def test_closed_box_checkpoint_bitwise(gpu):
    """Export/import of a walled domain: a resumed run gives the same bits."""
    p, phi, z, ct, ux, uy = box_case()
    a = gpu.Domain(p, phi, z, ct, ux, uy, storage="fp32", tile=8)
    a.step(20)
    s = a.export_state()
    a.step(17)
    b = gpu.Domain(p, phi, z, ct, ux, uy, storage="fp32", tile=8)
    b.import_state(s)
    b.step(17)
    for x, y in zip(a.read(), b.read()):
        assert np.array_equal(x, y)
