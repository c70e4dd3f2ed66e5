"""Pins of the oracle's phi^4 action (Sec. 2, Eq. (1))."""

import numpy as np
import pytest

import synth
from oracle import action as act


@pytest.mark.parametrize("L", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("c", [-1.3, 0.0, 0.25, 2.0])
def test_constant_field_closed_form(L, c):
    m2, lam = -4.0, 8.0
    phi = np.full((1, L * L), c)
    expect = L * L * (0.5 * m2 * c * c + lam * c ** 4)
    assert act.action(phi, L, m2, lam)[0] == pytest.approx(expect, rel=1e-14, abs=1e-14)


@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_z2_symmetry_bitwise(L):
    phi = synth.fields(1, 32, L).astype(np.float64)
    assert np.array_equal(act.action(phi, L, -4.0, 8.0), act.action(-phi, L, -4.0, 8.0))


@pytest.mark.parametrize("L,k0,k1", [(4, 1, 0), (4, 1, 2), (8, 3, 5), (6, 0, 1), (16, 7, 2)])
def test_plane_wave_is_laplacian_eigenvector(L, k0, k1):
    x0, x1 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    phi = np.cos(2 * np.pi * (k0 * x0 + k1 * x1) / L).reshape(1, -1)
    lam_k = 4 * np.sin(np.pi * k0 / L) ** 2 + 4 * np.sin(np.pi * k1 / L) ** 2
    expect = 0.5 * lam_k * np.sum(phi ** 2)
    assert act.action(phi, L, 0.0, 0.0)[0] == pytest.approx(expect, rel=1e-12, abs=1e-12)


def _dense_kinetic(L):
    """K = sum_mu (I - T_mu)^T (I - T_mu) built from explicit shift matrices."""
    d = L * L
    K = np.zeros((d, d))
    for dx0, dx1 in ((1, 0), (0, 1)):
        T = np.zeros((d, d))
        for a in range(L):
            for b in range(L):
                T[a * L + b, ((a + dx0) % L) * L + (b + dx1) % L] = 1.0
        D = np.eye(d) - T
        K += D.T @ D
    return K


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 8])
def test_dense_quadratic_form_route(L):
    m2, lam = -4.0, 8.0
    phi = synth.fields(2, 16, L).astype(np.float64)
    K = _dense_kinetic(L)
    quad = 0.5 * np.einsum("ni,ij,nj->n", phi, K + m2 * np.eye(L * L), phi)
    expect = quad + lam * np.sum(phi ** 4, axis=1)
    np.testing.assert_allclose(act.action(phi, L, m2, lam), expect, rtol=1e-12, atol=1e-12)


def test_L1_has_no_kinetic_term():
    phi = np.array([[0.7], [-1.1]])
    expect = 0.5 * 2.0 * phi[:, 0] ** 2 + 3.0 * phi[:, 0] ** 4
    np.testing.assert_allclose(act.action(phi, 1, 2.0, 3.0), expect, rtol=1e-15)


def test_L2_counts_each_bond_twice():
    a, b, c, d = 0.3, -0.8, 1.1, 0.05
    phi = np.array([[a, b, c, d]])          # sites (0,0) (0,1) (1,0) (1,1)
    kin = (a - b) ** 2 + (c - d) ** 2 + (a - c) ** 2 + (b - d) ** 2   # 1/2 * 2 per bond
    assert act.action(phi, 2, 0.0, 0.0)[0] == pytest.approx(kin, rel=1e-15)


def test_row_major_site_layout():
    # a field varying only along x1 (fast index) has no x0 bonds
    L = 4
    phi = np.tile(np.array([0.0, 1.0, 0.0, 1.0]), L).reshape(1, -1)
    # x1 bonds: each row has 4 bonds of |1| -> 1/2 * 4 per row
    assert act.action(phi, L, 0.0, 0.0)[0] == pytest.approx(0.5 * 4 * L)


def test_magnetisation_and_u0():
    phi = np.array([[1.0, 2.0, 3.0, 6.0]])
    assert act.magnetisation(phi)[0] == 3.0
    assert act.u0(phi)[0] == 25.0
