"""Three-dimensional path on the GPU (lbmgls3d.h) against the FP64 CPU
oracle in three dimensions (oracle/lbm3d_oracle.c), element by element.

Bars (tests/parity.py): FP64 storage <= 1e-12 relative, FP32 storage <= 1e-5
relative, on phi, u (three components) and P, in the 2-norm over the field and
in the max-norm.  Domains are ragged (node counts not multiples of the 256-node
block or of the 64-entry plane pitch) and periodic; the full-size 256^3 domain
of the benchmark is checked against the oracle on a 128^3 cut of the same
recipe and through properties that hold at any size.
"""
import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W
from parity import BAR, check, errors, fmt

pytestmark = pytest.mark.gpu
NAMES3 = ("phi", "ux", "uy", "uz", "P")


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_05097_amd import lbmgls
    lbmgls.lib()
    return lbmgls


def _pair(gpu, w, storage, steps):
    from oracle.oracle3d import Oracle3
    d = gpu.Domain3(w.params, *w.arrays(), storage=storage)
    o = Oracle3(w.params, *w.arrays())
    m0 = d.mass()
    d.step(steps)
    o.step(steps)
    errs = errors(d.read(), o.read(), NAMES3)
    drift = abs(d.mass() - m0) / np.abs(w.phi).sum()
    print(f"\n{w.name} {storage} {steps} steps (2-norm/max-norm): {fmt(errs)} mass_drift={drift:.2e}")
    return d, o, errs, drift


def _small():
    return W.drop_on_slab_3d(20, 16, 12, slab=3, R=5.0, theta_deg=60.0, rho_ratio=10.0)


def _ragged():
    # 70 x 36 x 21 = 52920 nodes: 206.7 blocks of 256, pitch padding 8
    return W.drop_on_slab_3d(70, 36, 21, slab=4, R=9.0, theta_deg=120.0, rho_ratio=10.0, mu_ratio=5.0,
                             sigma=5e-3, gz=-2e-6, rho_ref=0.1)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_initial_level_matches(gpu, storage):
    w = _small()
    from oracle.oracle3d import Oracle3
    d = gpu.Domain3(w.params, *w.arrays(), storage=storage)
    errs = errors(d.read(), Oracle3(w.params, *w.arrays()).read(), NAMES3)
    print(fmt(errs))
    check(errs, BAR[storage], ("phi",))
    for k in ("ux", "uy", "uz", "P"):
        assert errs[k][1] == 0.0  # at rest, P = 0 (procedure step 1)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_small_drop_on_wetting_slab_300_steps(gpu, storage):
    d, o, errs, drift = _pair(gpu, _small(), storage, 300)
    check(errs, BAR[storage])
    assert drift < (1e-13 if storage == "fp64" else 1e-9)
    ef, ek = d.energy()
    ef0, ek0 = o.energy()
    assert abs(ef - ef0) <= BAR[storage] * abs(ef0) and abs(ek - ek0) <= max(BAR[storage] * 10, 1e-12) * abs(ek0)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_ragged_domain_with_gravity_100_steps(gpu, storage):
    _, _, errs, drift = _pair(gpu, _ragged(), storage, 100)
    check(errs, BAR[storage])
    assert drift < (1e-13 if storage == "fp64" else 1e-9)


def _moving(nx, ny, nz, seed=11):
    """A drop on a slab with a seeded smooth periodic initial velocity."""
    import dataclasses
    w = W.drop_on_slab_3d(nx, ny, nz, slab=max(1, nz // 5), R=max(1.5, min(nx, ny, nz) / 3.0), theta_deg=75.0,
                          rho_ratio=10.0)
    rng = np.random.default_rng(seed)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    a, b, c = rng.uniform(0.0, 2.0 * np.pi, 3)
    return dataclasses.replace(w, name=f"moving drop {nx}x{ny}x{nz}",
                               ux=1e-3 * np.sin(2.0 * np.pi * y / ny + a),
                               uy=1e-3 * np.sin(2.0 * np.pi * z / nz + b),
                               uz=1e-3 * np.sin(2.0 * np.pi * x / nx + c))


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(67, 23, 19), (3, 3, 3)])
def test_partial_columns_and_the_smallest_grid(gpu, storage, shape):
    """The node update marches along z over 64 x 4 columns of 16 slices:
    67 x 23 x 19 leaves a 3-column, 3-row and 3-slice remainder, and 3^3 (the
    smallest grid) puts one column over a grid whose every neighbour wraps;
    moving initial state, 60 steps, against the oracle."""
    _, _, errs, drift = _pair(gpu, _moving(*shape), storage, 60)
    check(errs, BAR[storage])
    assert drift < (1e-13 if storage == "fp64" else 1e-9)


def test_runs_of_steps_compose(gpu):
    """Stepping 7 + 13 + 1 equals stepping 21 at once, bit for bit."""
    w = _small()
    a = gpu.Domain3(w.params, *w.arrays(), storage="fp64")
    b = gpu.Domain3(w.params, *w.arrays(), storage="fp64")
    a.step(7)
    a.step(13)
    a.step(1)
    b.step(21)
    for x, y in zip(a.read(), b.read()):
        assert np.array_equal(x, y)


def test_benchmark_recipe_at_128_cubed_against_the_oracle(gpu):
    """The benchmark's recipe (drop on a slab, theta 60, ratio 10) at 128^3,
    3 steps, FP64 and FP32 storage."""
    from oracle.oracle3d import Oracle3
    w = W.drop_on_slab_3d(128, slab=8, R=32.0, theta_deg=60.0, rho_ratio=10.0)
    o = Oracle3(w.params, *w.arrays())
    o.step(3)
    ref = o.read()
    for storage in ("fp64", "fp32"):
        d = gpu.Domain3(w.params, *w.arrays(), storage=storage)
        d.step(3)
        errs = errors(d.read(), ref, NAMES3)
        print(f"\n128^3 {storage}: {fmt(errs)}")
        check(errs, BAR[storage])
        d.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_full_size_properties(gpu, storage):
    """256^3 benchmark domain, 50 steps: finite, mass conserved, and the
    mirror symmetries of the centred drop (x -> nx - x, y -> ny - y, x <-> y)
    kept to rounding."""
    w = W.bench_3d()
    d = gpu.Domain3(w.params, *w.arrays(), storage=storage)
    m0 = d.mass()
    d.step(50)
    phi, ux, uy, uz, P = d.read()
    drift = abs(d.mass() - m0) / np.abs(w.phi).sum()
    n = w.params["nx"]
    idx = (-np.arange(n)) % n  # x -> n - x (mod n): the reflection about x = n/2
    sym_phi = max(np.abs(phi - phi[:, :, idx]).max(), np.abs(phi - phi[:, idx, :]).max(),
                  np.abs(phi - np.swapaxes(phi, 1, 2)).max())
    sym_u = max(np.abs(ux + ux[:, :, idx]).max(), np.abs(ux - np.swapaxes(uy, 1, 2)).max()) / np.abs(ux).max()
    print(f"\n256^3 {storage}: mass drift {drift:.2e}, symmetry defect phi {sym_phi:.2e} u {sym_u:.2e}, "
          f"|u|max {np.sqrt(ux ** 2 + uy ** 2 + uz ** 2).max():.2e}, step {d.last_step_ms:.3f} ms")
    assert np.isfinite(phi).all() and np.isfinite(P).all()
    assert drift < (1e-12 if storage == "fp64" else 1e-8)
    assert sym_phi < (1e-12 if storage == "fp64" else 1e-6)
    assert sym_u < (1e-9 if storage == "fp64" else 1e-3)
    d.close()


def _cap_angle_after(gpu, R0, n, nz, theta, steps):
    from capfit import cap_angle_3d, cap_state_3d
    w, zs = cap_state_3d(n, n, nz, 12, R0, theta, theta)
    d = gpu.Domain3(w.params, *w.arrays(), storage="fp32")
    d.step(steps)
    got = cap_angle_3d(d.read()[0], zs)
    d.close()
    return got


def test_young_angle_hydrophilic_cap(gpu):
    """Young's law in three dimensions (Sec. 2.1's wetting condition on a flat
    diffuse slab, no oracle): a spherical cap of 60 degrees given 60 degrees
    (hemisphere volume of radius 24, density and viscosity ratios 1, sigma
    1e-2) stays within 2 degrees of it over 30000 steps (measured: 58.6)."""
    got = _cap_angle_after(gpu, 24.0, 128, 72, 60.0, 30000)
    print(f"\n3-D Young 60: {got:.2f}")
    assert abs(got - 60.0) < 2.0, got


def test_young_angle_hydrophobic_cap_converges_with_size(gpu):
    """A cap of 120 degrees given 120 degrees settles below it by an amount
    that falls with the drop's size, as a diffuse-interface correction of
    order D / R does: hemisphere radius 24 and 36 (interface width D = 4),
    60000 steps (measured: 114.9 and 117.0 degrees, deficits near the ratio
    of the radii).  The larger drop ends within 4 degrees."""
    small = _cap_angle_after(gpu, 24.0, 128, 72, 120.0, 60000)
    large = _cap_angle_after(gpu, 36.0, 176, 96, 120.0, 60000)
    print(f"\n3-D Young 120: R0 24 -> {small:.2f}, R0 36 -> {large:.2f}")
    assert small < large < 120.0, (small, large)
    assert (120.0 - large) < 0.8 * (120.0 - small), (small, large)
    assert 120.0 - large < 4.0, large


@pytest.mark.parametrize("R,n", [(12.0, 48), (20.0, 80), (32.0, 128)])
def test_laplace_law_sphere_gpu(gpu, R, n):
    """Static sphere at density ratio 10 (FP64, sigma 1e-2, no solid): the
    pressure jump equals 2 sigma / R (the Laplace law in three dimensions) on
    grids the oracle would take hours for (its own pin runs R = 7), within 5%
    (measured: 1.038, 0.999, 0.987), and the drop stays at rest (spurious
    currents below 2e-5)."""
    p = W.params3(n, n, n, sigma=1e-2, M=0.1)
    p.update(rho1=1.0, rho2=0.1, mu1=0.3, mu2=0.3)
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    d = gpu.Domain3(p, np.tanh((R - r) / 2.0), np.zeros((n, n, n)), storage="fp64")
    d.step(int(6 * n * n / 100) + 4000)
    dps = []
    for _ in range(4):  # average over the remaining acoustic oscillation
        d.step(50)
        phi, ux, uy, uz, P = d.read()
        c = n // 2
        dps.append(P[c - 1:c + 2, c - 1:c + 2, c - 1:c + 2].mean() - P[:3, :3, :3].mean())
    Re = (3 * ((phi + 1) / 2).sum() / (4 * np.pi)) ** (1 / 3)
    ratio = float(np.mean(dps)) / (2 * 1e-2 / Re)
    umax = max(float(np.abs(a).max()) for a in (ux, uy, uz))
    print(f"\n3-D Laplace R={R}: dp / (2 sigma/R) = {ratio:.4f}, max |u| {umax:.1e}")
    d.close()
    assert abs(ratio - 1) < 0.05
    assert umax < 2e-5


def test_zero_steps_change_nothing_and_negative_steps_are_refused(gpu):
    w = _small()
    d = gpu.Domain3(w.params, *w.arrays(), storage="fp32")
    d.step(2)
    before = d.read()
    d.step(0)
    with pytest.raises(gpu.LbmError):
        d.step(-1)
    for a, b in zip(before, d.read()):
        assert np.array_equal(a, b)
