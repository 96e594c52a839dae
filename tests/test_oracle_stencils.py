"""Pins of the oracle's finite differences, chemical potential and energy.

* gradient / Laplacian: exact on quadratics; second-order convergence to the
  analytic identities of the tanh indicator (Sec. 2.1, Eq. phi0Eq);
* chemical potential: zero on the planar equilibrium profile tanh(2z/D)
  (Sec. 2.1), and equal to the variational derivative of the discrete free
  energy (Eq. potential = delta E_F / delta phi) taken by finite differences
  of the oracle's own energy, with solid and wetting terms active;
* free energy: a planar interface stores sigma per unit length.
"""
import numpy as np
import pytest


def test_fd_exact_on_quadratics(orc):
    n = 24
    y, x = np.mgrid[0:n, 0:n].astype(float)
    a, b, c, d, e, f = 0.3, -1.2, 0.7, 0.05, -0.11, 0.08
    chi = a + b * x + c * y + d * x * x + e * x * y + f * y * y
    gx, gy = orc.grad(chi)
    lap = orc.lap(chi)
    sl = (slice(2, -2), slice(2, -2))  # away from the periodic seam
    assert np.allclose(gx[sl], (b + 2 * d * x + e * y)[sl], atol=1e-12)
    assert np.allclose(gy[sl], (c + e * x + 2 * f * y)[sl], atol=1e-12)
    assert np.allclose(lap[sl], 2 * d + 2 * f, atol=1e-12)


def test_fd_periodic_wrap(orc):
    n = 16
    x = np.arange(n)
    k = 2 * np.pi / n
    chi = np.tile(np.sin(k * x), (8, 1))
    gx, gy = orc.grad(chi)
    lap = orc.lap(chi)
    # discrete symbols of the isotropic stencils on a 1-D mode
    assert np.allclose(gx, np.sin(k) * np.cos(k * x), atol=1e-14)
    assert np.allclose(gy, 0.0, atol=1e-14)
    assert np.allclose(lap, -4 * np.sin(k / 2) ** 2 * chi, atol=1e-14)


def _ind_err(orc, D):
    ny, nx = 512, 4
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    zeta = 128.0 - np.abs(y - 255.5)
    p0 = 0.5 * (1 + np.tanh(2 * zeta / D))
    gx, gy = orc.grad(p0)
    lap = orc.lap(p0)
    lap_ex = 16 * p0 * (1 - p0) * (1 - 2 * p0) / D ** 2
    gn_ex = 4 * p0 * (1 - p0) / D
    return (np.abs(lap - lap_ex).max() / np.abs(lap_ex).max(),
            np.abs(np.hypot(gx, gy) - gn_ex).max() / gn_ex.max())


def test_indicator_identities(orc):
    """Eq. phi0Eq: lap(phi0) = 16 phi0(1-phi0)(1-2 phi0)/D^2 and
    |grad phi0| = 4 phi0(1-phi0)/D hold for the tanh indicator of a planar
    signed distance; the stencils reproduce them to second order in dx/D."""
    errs = {D: _ind_err(orc, D) for D in (4.0, 8.0, 16.0)}
    for D, (e_lap, e_gn) in errs.items():
        assert e_lap < 0.5 * (2 / D) ** 2 and e_gn < 0.5 * (2 / D) ** 2
    for a, b in ((4.0, 8.0), (8.0, 16.0)):
        for k in (0, 1):
            assert 3.0 < errs[a][k] / errs[b][k] < 5.0


@pytest.mark.parametrize("D", [4.0, 8.0])
def test_mu_vanishes_on_planar_profile(orc, D):
    from paper_2311_05097_amd.workloads import flat_interface
    w = flat_interface(nx=4, ny=128, D=D)
    z = np.zeros_like(w.phi)
    mu = orc.mu(w.params, w.phi, z, z)
    scale = 3 * w.params["sigma"] / D  # bulk scale of mu
    # the residual is the truncation error of the discrete Laplacian
    assert np.abs(mu).max() / scale < 0.5 * (2 / D) ** 2
    # a wrong relative weight of the bulk and gradient terms is O(1)
    mu_bad = orc.mu(dict(w.params, D=D * 1.2), w.phi, z, z)
    assert np.abs(mu_bad).max() / scale > 0.05


def _var_err(orc, n, sigma=1e-2):
    """max |dE/dphi_j - mu_j| / max|mu| over a few nodes, smooth fields with
    wavelength n (so dx/wavelength halves when n doubles)."""
    from paper_2311_05097_amd.workloads import params
    from oracle.oracle import Oracle
    y, x = np.mgrid[0:n, 0:n].astype(float)
    k = 2 * np.pi / n
    phi = 0.6 * np.tanh(np.sin(k * x + 1.3) * 3) * np.cos(k * y) + 0.1
    phi0 = 0.5 + 0.45 * np.sin(k * x) * np.cos(k * y + 0.4)
    cth = 0.5 + 0.3 * np.cos(k * x)
    D = n / 4.0
    p = params(n, n, D=D, sigma=sigma)
    mu = orc.mu(p, phi, phi0, cth * phi0)

    def energy(ph):
        return Oracle(p, ph, phi0, cth).energy()[0]

    h, s = 1e-6, n // 32
    errs = []
    for (j, i) in [(5 * s, 7 * s), (16 * s, 16 * s), (12 * s, 20 * s), (20 * s, 9 * s), (25 * s, 25 * s)]:
        a, b = phi.copy(), phi.copy()
        a[j, i] += h
        b[j, i] -= h
        errs.append(abs((energy(a) - energy(b)) / (2 * h) - mu[j, i]))
    return max(errs) / np.abs(mu).max()


def test_mu_is_variational_derivative_of_energy(orc):
    """Eq. (potential) = delta E_F / delta phi: perturb phi at single nodes and
    difference the oracle's discrete energy, with the solid penalty and the
    wetting terms active (varying phi0 and contact angle).  The two differ
    only by the compact-versus-wide Laplacian, which is second order."""
    e64, e128 = _var_err(orc, 64), _var_err(orc, 128)
    assert e64 < 0.05 and e128 < 0.015
    assert e64 / e128 > 2.5


def test_planar_interface_energy_is_sigma(orc):
    """A flat interface stores sigma_12 per unit length (Eq. 2energyDensity
    with the tanh(2z/D) profile); two interfaces across nx columns."""
    from paper_2311_05097_amd.workloads import flat_interface
    from oracle.oracle import Oracle
    for D in (4.0, 8.0):
        w = flat_interface(nx=4, ny=256, D=D, sigma=2e-3)
        o = Oracle(w.params, *w.arrays())
        ef, ek = o.energy()
        assert ek == 0.0
        assert abs(ef / (2 * 4 * 2e-3) - 1.0) < 0.25 * (2 / D) ** 2
