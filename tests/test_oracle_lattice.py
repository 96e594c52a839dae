"""Pins of the oracle's lattice, matrices and collision operator (Sec. 4).

Each check compares the oracle with something it does not compute itself:
the printed matrices (golden file), the textbook D2Q9 weights, lattice
isotropy identities, Hermite polynomials evaluated here, or an algebraic
property the paper states (BGK reduction, the equivalence of the two forms of
the collision matrix).
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hermite_matrices.txt")
D0S = [1.0 / 3.0, 0.4, 0.25, 0.6]


def _read_golden(d0):
    cs2 = d0
    mats, cur = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("M0", "NH"):
            cur = mats.setdefault(line, [])
            continue
        row = []
        for tok in line.split():
            row.append({"cs2": cs2, "-cs2": -cs2, "cs4": cs2 * cs2}.get(tok, None)
                       if "cs" in tok else float(tok))
        cur.append(row)
    return np.array(mats["M0"]), np.array(mats["NH"])


@pytest.mark.parametrize("d0", D0S)
def test_weights_moments(orc, d0):
    w, cx, cy = orc.lattice(d0)
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    assert np.isclose((w * cx).sum(), 0.0, atol=1e-15)
    assert np.isclose((w * cx * cx).sum(), d0, atol=1e-15)  # c_s^2 = d0 c^2
    assert np.isclose((w * cy * cy).sum(), d0, atol=1e-15)
    assert np.isclose((w * cx * cy).sum(), 0.0, atol=1e-15)
    assert np.isclose((w * cx ** 4).sum(), d0, atol=1e-15)
    assert np.isclose((w * cx ** 2 * cy ** 2).sum(), d0 * d0, atol=1e-15)
    # the weights are the tensor product of the 1-D three-point rule
    w1 = {0: 1.0 - d0, 1: d0 / 2.0, -1: d0 / 2.0}
    for i in range(9):
        assert np.isclose(w[i], w1[cx[i]] * w1[cy[i]], atol=1e-15)


def test_classical_weights(orc):
    # d0 = 1/3 is the classical D2Q9 lattice: 4/9, 1/9, 1/36
    w, cx, cy = orc.lattice(1.0 / 3.0)
    assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-15)
    assert sorted(zip(cx, cy)) == sorted([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                                          (1, 1), (-1, 1), (-1, -1), (1, -1)])


@pytest.mark.parametrize("d0", D0S)
def test_matrices_match_printed(orc, d0):
    M0g, NHg = _read_golden(d0)
    M0, NH, MH, MHinv = orc.matrices(d0)
    assert np.array_equal(M0, M0g)
    assert np.allclose(NH, NHg, atol=0, rtol=0)
    assert np.allclose(MH, NHg @ M0g, atol=1e-15)  # c = 1: C_d = I


@pytest.mark.parametrize("d0", D0S)
def test_MH_rows_are_hermite_polynomials(orc, d0):
    _, cx, cy = orc.lattice(d0)
    a = d0
    H = np.array([np.ones(9), cx, cy, cx ** 2 - a, cy ** 2 - a, cx * cy,
                  cx * (cy ** 2 - a), cy * (cx ** 2 - a), (cx ** 2 - a) * (cy ** 2 - a)], float)
    _, _, MH, MHinv = orc.matrices(d0)
    assert np.allclose(MH, H, atol=1e-15)
    assert np.allclose(MH @ MHinv, np.eye(9), atol=1e-13)
    # N_H is unit lower triangular, so det M_H = det M_0 (= 64 for D2Q9)
    assert np.isclose(np.linalg.det(MH), 64.0, rtol=1e-12)
    # discrete orthogonality with the lattice weights
    w, _, _ = orc.lattice(d0)
    G = MH @ np.diag(w) @ MH.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-15)


@pytest.mark.parametrize("d0", D0S)
@pytest.mark.parametrize("s", [0.3, 1.0, 1.7])
def test_bgk_reduction(orc, d0, s):
    lam = orc.collision_matrix(d0, [s] * 9)
    assert np.allclose(lam, s * np.eye(9), atol=1e-14)


@pytest.mark.parametrize("d0", D0S)
def test_two_forms_of_collision_matrix(orc, d0):
    # Lam = M_H^-1 S_H M_H = M_0^-1 S_0 M_0 with S_0 = C_d^-1 N_H^-1 S_H N_H C_d
    # lower triangular (Sec. 4).
    rng = np.random.default_rng(7)
    s = rng.uniform(0.2, 1.9, 9)
    lam = orc.collision_matrix(d0, s)
    M0, NH, _, _ = orc.matrices(d0)
    S0 = np.linalg.inv(NH) @ np.diag(s) @ NH
    assert np.allclose(np.triu(S0, 1), 0.0, atol=1e-15)
    assert np.allclose(np.diag(S0), s, atol=1e-15)
    assert np.allclose(lam, np.linalg.inv(M0) @ S0 @ M0, atol=1e-13)
    # eigenvalues of Lam are the relaxation rates
    ev = np.sort(np.linalg.eigvals(lam).real)
    assert np.allclose(ev, np.sort(s), atol=1e-12)
