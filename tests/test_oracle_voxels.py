"""Pins of the oracle's voxel-solid smoothing (Sec. 4.1: the binary micro-CT
solid is smoothed by a few iterations of a standard Cahn-Hilliard equation
before it serves as phi0): fixed points, conservation, the discrete energy,
the linear decay of a Fourier mode against the stencil's symbol in closed
form, the near-stationarity of the equilibrium profile, and the exact
equivalence of mirrored walls with a reflected periodic domain.
"""
import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W


def _lap(c):
    """Isotropic 9-point Laplacian (weights 4/9, 1/9, 1/36 with c_s^2 = 1/3),
    periodic, written with numpy rolls."""
    r = lambda dy, dx: np.roll(np.roll(c, -dy, 0), -dx, 1)
    ax = r(0, 1) + r(0, -1) + r(1, 0) + r(-1, 0)
    dg = r(1, 1) + r(1, -1) + r(-1, 1) + r(-1, -1)
    return 6.0 * ((ax - 4 * c) / 9.0 + (dg - 4 * c) / 36.0)


def test_uniform_solid_and_pore_are_fixed(orc):
    for v in (0.0, 1.0):
        s = np.full((20, 24), v)
        assert np.array_equal(orc.smooth_solid(s, 4.0), s)


def test_smoothing_conserves_the_solid_and_lowers_the_energy(orc):
    """chi = 2 s - 1 follows a conservative gradient flow of
    E = sum (chi^2 - 1)^2 / 4 - kappa/2 chi lap(chi), kappa = D^2/8: the total
    of chi is kept to rounding and E does not increase step by step."""
    s = W.voxel_solid(64, 48, n_grains=10, seed=2)
    chi0 = 2 * s - 1
    D = 4.0
    kappa = D * D / 8

    def energy(c):
        return float(np.sum((c * c - 1) ** 2 / 4 - kappa / 2 * c * _lap(c)))
    prev = energy(chi0)
    for it in range(1, 21):
        c = orc.smooth_chi(chi0, D, it)
        e = energy(c)
        assert e <= prev + 1e-12 * abs(prev)
        prev = e
        assert abs(c.sum() - chi0.sum()) <= 1e-11 * np.abs(chi0).sum()
    assert energy(c) < 0.8 * energy(chi0)


@pytest.mark.parametrize("kx,ky", [(1, 0), (3, 2), (8, 8), (16, 16)])
def test_mode_decay_matches_the_stencil_symbol(orc, kx, ky):
    """About chi = 1 the step is linear: a mode of wave vector k decays by
    1 - dtau L (2 + kappa L) per step, L = -symbol of the Laplacian, here in
    closed form: L = 6 [ (2/9)(2 - cos a - cos b) + (1/36)(4 - 2 cos(a + b)
    - 2 cos(a - b)) ].  At k = (pi, pi), L = 16/3 and the default step halves
    the mode."""
    n, D, eps = 32, 4.0, 1e-8
    kappa = D * D / 8
    y, x = np.mgrid[0:n, 0:n].astype(float)
    a, b = 2 * np.pi * kx / n, 2 * np.pi * ky / n
    mode = np.cos(a * x + b * y)
    c = orc.smooth_chi(1.0 + eps * mode, D, 1)
    L = 6 * ((2 / 9) * (2 - np.cos(a) - np.cos(b)) + (1 / 36) * (4 - 2 * np.cos(a + b) - 2 * np.cos(a - b)))
    dtau = orc.vox_dtau(D)
    ratio = 1 - dtau * L * (2 + kappa * L)
    got = np.sum((c - 1.0) * mode) / np.sum(eps * mode * mode)
    assert abs(got - ratio) <= 1e-6
    if (kx, ky) == (16, 16):
        assert abs(L - 16 / 3) < 1e-12 and abs(ratio - 0.5) < 1e-12


def test_equilibrium_profile_hardly_moves(orc):
    """tanh(2 z / D) solves mu = 0 for the continuous equation; on the
    lattice it changes by the stencil's truncation error only, far less than
    a voxel step does."""
    n, D = 64, 4.0
    y, x = np.mgrid[0:8, 0:n].astype(float)
    # a slab of phase -1 between x = 20.3 and 52.7
    smooth = np.tanh(2 * (np.abs(x - 36.5) - 16.2) / D)
    step = np.where(np.abs(x - 36.5) >= 16.2, 1.0, -1.0)
    ds = np.abs(orc.smooth_chi(smooth, D, 20) - smooth).max()
    dv = np.abs(orc.smooth_chi(step, D, 20) - step).max()
    assert ds < 0.02 and dv > 0.3, (ds, dv)


def test_mirrored_walls_equal_a_reflected_periodic_domain(orc):
    """With no-flux walls the ghost nodes mirror the field, so smoothing a
    walled domain equals smoothing the periodic domain of twice the size that
    holds the mask and its mirror images."""
    s = W.voxel_solid(40, 30, n_grains=8, seed=5, periodic=False)
    walled = orc.smooth_solid(s, 4.0, 20, bounce_x=1, bounce_y=1)
    s2 = np.concatenate([s, s[::-1]], axis=0)
    s4 = np.concatenate([s2, s2[:, ::-1]], axis=1)
    per = orc.smooth_solid(s4, 4.0, 20)
    assert np.abs(walled - per[:30, :40]).max() <= 1e-13
    assert np.abs(walled - orc.smooth_solid(s, 4.0, 20)).max() > 1e-3
