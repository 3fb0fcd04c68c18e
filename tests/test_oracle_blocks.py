"""Pins of the oracle's building blocks against what the paper fixes.

- Product-form equilibria (Sec. 2.4, eq prod): moments {1, c, cc} give
  {1, xi, xi xi + zeta I}; the diagonal third moment equals xi (the lattice
  constraint c^3 = c discussed in Sec. 3.4.2); at xi = 0, zeta = 1/3 they are
  the textbook D3Q27 weights (golden file).
- Energy-lattice ansatz (Sec. 3.4.1, eqs gansatz..Bi): reproduces {M0, m, M}
  for any theta; reduces to Grad's form at theta = 1/3.
- Correction vectors A_i (eq Ai) and B_i (eq Bi): the moments used in the
  paper's construction.
- Isotropic derivative (Sec. 4.1 reading): exact symbol sin(k) on Fourier modes.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _c(O):
    return O.velocities().astype(np.float64)


def test_velocity_set(oracle_mod):
    c = _c(oracle_mod)
    assert c.shape == (27, 3)
    assert len({tuple(v) for v in c}) == 27
    assert set(np.unique(c)) == {-1.0, 0.0, 1.0}
    # index convention i = 9 (cx+1) + 3 (cy+1) + (cz+1); opposite is 26 - i
    for i in range(27):
        assert np.all(c[26 - i] == -c[i])


def test_psi_weights_golden(oracle_mod):
    """Psi_i(0, 1/3) equals the D3Q27 weights, and so do w_i(1/3)."""
    c = _c(oracle_mod)
    table = {}
    with open(os.path.join(GOLDEN, "d3q27_weights.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                c2, w = line.split()
                table[int(c2)] = float(Fraction(w))
    psi = oracle_mod.psi([0.0, 0.0, 0.0], 1.0 / 3.0)
    w = oracle_mod.weights(1.0 / 3.0)
    for i in range(27):
        expect = table[int((c[i] ** 2).sum())]
        assert psi[i] == pytest.approx(expect, rel=1e-14)
        assert w[i] == pytest.approx(expect, rel=1e-14)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_psi_moments(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-0.3, 0.3, 3)
    zeta = rng.uniform(0.01, 0.6)
    rho = rng.uniform(0.2, 3.0)
    f = rho * oracle_mod.psi(xi, zeta)
    c = _c(oracle_mod)
    assert f.sum() == pytest.approx(rho, rel=1e-14)
    np.testing.assert_allclose(f @ c, rho * xi, rtol=1e-13, atol=1e-15)
    P = np.einsum("i,ia,ib->ab", f, c, c)
    np.testing.assert_allclose(P, rho * (np.outer(xi, xi) + zeta * np.eye(3)), rtol=1e-13, atol=1e-15)
    # diagonal third moment collapses to the momentum (c^3 = c)
    np.testing.assert_allclose(np.einsum("i,ia->a", f, c ** 3), rho * xi, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("theta", [0.01, 0.05, 0.1, 0.2, 1.0 / 3.0, 0.45, 0.6])
def test_gansatz_moments(oracle_mod, theta):
    rng = np.random.default_rng(int(theta * 1000))
    c = _c(oracle_mod)
    for _ in range(3):
        M0 = rng.uniform(0.1, 2.0)
        m = rng.uniform(-0.5, 0.5, 3)
        S = rng.uniform(-0.3, 0.3, (3, 3))
        Mt = 0.5 * (S + S.T) + M0 * theta * np.eye(3)
        g = oracle_mod.gansatz(theta, M0, m, Mt)
        scale = max(M0, 1.0) / theta ** 2
        assert g.sum() == pytest.approx(M0, abs=1e-13 * scale)
        np.testing.assert_allclose(g @ c, m, atol=1e-13 * scale)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", g, c, c), Mt, atol=1e-13 * scale)


def test_gansatz_reduces_to_grad_at_reference_temperature(oracle_mod):
    """At theta = 1/3 the B.Z term vanishes (Z = 0): G is Grad's expansion."""
    c = _c(oracle_mod)
    w = oracle_mod.weights(1.0 / 3.0)
    th = 1.0 / 3.0
    M0 = 1.3
    m = np.array([0.1, -0.2, 0.05])
    Mt = np.array([[0.5, 0.02, -0.01], [0.02, 0.4, 0.03], [-0.01, 0.03, 0.45]])
    grad = np.array([w[i] * (M0 + m @ c[i] / th +
                             np.sum((Mt - M0 * th * np.eye(3)) * (np.outer(c[i], c[i]) - th * np.eye(3)))
                             / (2 * th * th)) for i in range(27)])
    np.testing.assert_allclose(oracle_mod.gansatz(th, M0, m, Mt), grad, rtol=1e-13, atol=1e-15)


def test_correction_vectors(oracle_mod):
    """A_i: zero mass, unit first moment (adds X to the momentum), no second
    moment. B_i: zero mass and momentum; second moment -delta (cancels the
    (1-3 theta)/(2 theta) deficit of the weights)."""
    c = _c(oracle_mod)
    A, B = oracle_mod.tables()
    np.testing.assert_array_equal(A.sum(axis=0), 0.0)
    np.testing.assert_array_equal(np.einsum("ia,ib->ab", A, c), np.eye(3))
    np.testing.assert_array_equal(np.einsum("ia,ib,ic->abc", A, c, c), 0.0)
    np.testing.assert_array_equal(B.sum(axis=0), 0.0)
    np.testing.assert_array_equal(np.einsum("ia,ib->ab", B, c), 0.0)
    np.testing.assert_array_equal(np.einsum("ia,ib,ic->abc", B, c, c)[:, [0, 1, 2], [0, 1, 2]], -np.eye(3))
    off = np.einsum("ia,ib,ic->abc", B, c, c)
    for a in range(3):
        for b in range(3):
            for d in range(3):
                if b != d:
                    assert off[a, b, d] == 0.0


@pytest.mark.parametrize("k", [1, 3, 7])
def test_isotropic_gradient_symbol(oracle_mod, k):
    """On a Fourier mode exp(i k.x) the operator 3 sum_i w_i c_i phi(x + c_i) with
    the product weights (2/3, 1/6, 1/6) has the exact symbol
    i sin(k_a) prod_{b != a} (2 + cos k_b) / 3 -- second-order accurate."""
    nx, ny, nz = 32, 16, 8
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kx, ky, kz = 2 * np.pi * k / nx, 2 * np.pi / ny, 2 * np.pi / nz
    phi = np.sin(kx * x + ky * y + kz * z)
    g = oracle_mod.gradient(phi)
    cosv = np.cos(kx * x + ky * y + kz * z)
    ks = [kx, ky, kz]
    for comp in range(3):
        others = np.prod([(2.0 + np.cos(ks[b])) / 3.0 for b in range(3) if b != comp])
        np.testing.assert_allclose(g[comp], np.sin(ks[comp]) * others * cosv, atol=1e-13)
