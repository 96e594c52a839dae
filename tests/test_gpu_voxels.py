"""Voxel solids on the GPU: the Cahn-Hilliard smoothing of a binary solid
(lbm_smooth_solid) against the FP64 oracle, and the porous-medium phase
separation of Sec. 4.1 started from it (no-flux walls on every side, random
initial phase in the pores): parity with the oracle over the first steps,
exact mass and the energy decay the paper reports, on the 256 x 256 grid.
"""
import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_05097_amd import lbmgls
    lbmgls.lib()
    return lbmgls


@pytest.mark.parametrize("nx,ny,bx,by", [(67, 45, 0, 0), (67, 45, 1, 1), (300, 70, 1, 0), (256, 256, 1, 1)])
def test_smoothing_matches_the_oracle(gpu, nx, ny, bx, by):
    from oracle import oracle as O
    s = W.voxel_solid(nx, ny, n_grains=max(8, nx * ny // 3000), seed=3, periodic=not (bx or by))
    p = W.params(nx, ny, bounce_x=bx, bounce_y=by)
    g = gpu.smooth_solid(p, s, 20)
    o = O.smooth_solid(s, p["D"], 20, bounce_x=bx, bounce_y=by)
    assert np.abs(g - o).max() <= 1e-13
    assert np.abs(o - s).max() > 0.3  # it did smooth


def test_smoothing_with_a_given_step(gpu):
    from oracle import oracle as O
    s = W.voxel_solid(100, 64, n_grains=10, seed=4)
    p = W.params(100, 64, bounce_y=1)
    g = gpu.smooth_solid(p, s, 35, dtau=0.004)
    o = O.smooth_solid(s, p["D"], 35, dtau=0.004, bounce_y=1)
    assert np.abs(g - o).max() <= 1e-13


def test_smoothing_arguments(gpu):
    p = W.params(32, 32)
    with pytest.raises(gpu.LbmError):
        gpu.smooth_solid(p, np.zeros((32, 32)), -1)
    with pytest.raises(gpu.LbmError):
        gpu.smooth_solid(dict(p, bounce_x=3), np.zeros((32, 32)), 5)
    assert np.array_equal(gpu.smooth_solid(p, np.ones((32, 32)), 7), np.ones((32, 32)))


def _porous(gpu, n, seed, theta):
    """Sec. 4.1: a voxel porous medium smoothed by 20 CH steps, walls on
    every side, phi = (1 - phi0) rand(-1, 1), rho1 = rho2, mu = 0.1."""
    s = W.voxel_solid(n, n, n_grains=n * n // 2200, seed=seed, r_range=(6.0, 16.0), periodic=False)
    p = W.params(n, n, bounce_x=1, bounce_y=1)
    phi0 = gpu.smooth_solid(p, s, 20)
    rng = np.random.default_rng(seed + 100)
    phi = (1.0 - phi0) * rng.uniform(-1.0, 1.0, size=(n, n))
    ct = np.full((n, n), np.cos(np.radians(theta)))
    return p, phi, phi0, ct


def test_porous_phase_separation_fp64_parity(gpu):
    from oracle.oracle import Oracle
    p, phi, phi0, ct = _porous(gpu, 96, 11, 45.0)
    o = Oracle(p, phi, phi0, ct, None, None)
    d = gpu.Domain(p, phi, phi0, ct, storage="fp64", tile=8)
    o.step(100)
    d.step(100)
    for a, b in zip(d.read(), o.read()):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("theta", [45.0, 135.0])
def test_porous_phase_separation_energy_decays(gpu, theta):
    """The total energy of Sec. 2.3 (free energy with the wetting term plus
    kinetic energy) does not increase along the run (the energy law the paper
    proves and plots for this case), and the phase mass is kept, on 256^2."""
    p, phi, phi0, ct = _porous(gpu, 256, 7, theta)
    d = gpu.Domain(p, phi, phi0, ct, storage="fp64", tile=8)
    m0 = d.mass()
    e = [sum(d.energy())]
    for _ in range(20):
        d.step(500)
        e.append(sum(d.energy()))
    e = np.array(e)
    print(f"\nporous theta={theta}: E {e[0]:.5f} -> {e[-1]:.5f}, max rise {np.max(np.diff(e)):.2e}")
    assert np.all(np.diff(e) <= 1e-9 * abs(e[0]))
    assert e[-1] < 0.9 * e[0]
    assert abs(d.mass() - m0) <= 1e-12 * np.abs(phi).sum()
