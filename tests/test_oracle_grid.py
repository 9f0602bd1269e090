"""Pins of the oracle's 1D building blocks against textbook values and library
routines (numpy.polynomial.chebyshev, numpy.fft) and closed-form integrals."""

import os

import numpy as np
import numpy.polynomial.chebyshev as C
import pytest

from oracle import grid as og

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


def test_cheb_matrix_textbook_3pt():
    D = og.cheb_diff_matrix(3, -1.0, 1.0)
    np.testing.assert_allclose(D, _gold("cheb_D3.txt"), rtol=0, atol=1e-15)


@pytest.mark.parametrize("n_r", [5, 17, 33, 65])
def test_cheb_matrix_exact_on_chebyshev_polynomials(n_r):
    r_in, r_out = 1.0, 3.0
    r = og.cgl_nodes(n_r, r_in, r_out)
    assert r[0] == pytest.approx(r_in, abs=1e-15) and r[-1] == pytest.approx(r_out, abs=1e-15)
    xi = (2 * r - r_in - r_out) / (r_out - r_in)
    D = og.cheb_diff_matrix(n_r, r_in, r_out)
    for n in range(n_r):
        c = np.zeros(n + 1)
        c[n] = 1.0
        f = C.chebval(xi, c)
        df = C.chebval(xi, C.chebder(c)) * 2.0 / (r_out - r_in) if n else 0 * xi
        err = np.max(np.abs(D @ f - df))
        scale = max(1.0, np.max(np.abs(df)))
        # the collocation matrix has entries of size N^2, so rounding grows as N^2 eps
        assert err <= 1e-15 * (n_r - 1) ** 2 * scale, (n, err, scale)


def test_cheb_matrix_constant_exact():
    D = og.cheb_diff_matrix(33, 1.0, 3.0)
    assert np.max(np.abs(D @ np.ones(33))) <= 1e-12


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_fourier_matrix_exact_on_trig_polynomials(n):
    D = og.fourier_diff_matrix(n)
    x = 2 * np.pi * np.arange(n) / n
    for k in range(n // 2):
        np.testing.assert_allclose(D @ np.cos(k * x), -k * np.sin(k * x), atol=1e-13 * max(k, 1))
        np.testing.assert_allclose(D @ np.sin(k * x), k * np.cos(k * x), atol=1e-13 * max(k, 1))
    # Nyquist mode is annihilated
    assert np.max(np.abs(D @ np.cos(n // 2 * x))) <= 1e-12
    # antisymmetric
    np.testing.assert_allclose(D, -D.T, atol=0)


@pytest.mark.parametrize("n", [16, 32, 64])
def test_fourier_matrix_matches_fft_derivative(n):
    rng = np.random.default_rng(3)
    f = rng.normal(size=n)
    k = np.fft.fftfreq(n, d=1.0 / n)
    k[n // 2] = 0.0  # Nyquist derivative set to zero
    ref = np.real(np.fft.ifft(1j * k * np.fft.fft(f)))
    np.testing.assert_allclose(og.fourier_diff_matrix(n) @ f, ref, atol=1e-12)


def test_fourier_matrix_half_shifted_grid():
    # shift invariance: same matrix on (j + 1/2) h nodes
    n = 32
    x = (np.arange(n) + 0.5) * 2 * np.pi / n
    D = og.fourier_diff_matrix(n)
    for k in range(1, n // 2):
        np.testing.assert_allclose(D @ np.sin(k * x), k * np.cos(k * x), atol=1e-12)


def test_fejer_textbook_and_exactness():
    np.testing.assert_allclose(og.fejer_weights(3), _gold("fejer_n3.txt"), atol=1e-15)
    for n in (2, 5, 8, 16, 17, 32):
        w = og.fejer_weights(n)
        mu = np.cos((np.arange(n) + 0.5) * np.pi / n)
        assert np.sum(w) == pytest.approx(2.0, abs=1e-14)
        for p in range(n):
            exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
            assert np.sum(w * mu ** p) == pytest.approx(exact, abs=1e-14), (n, p)


def test_clenshaw_curtis_textbook_and_exactness():
    np.testing.assert_allclose(og.clenshaw_curtis_weights(5), _gold("clenshaw_curtis_n5.txt"), atol=1e-15)
    np.testing.assert_allclose(og.clenshaw_curtis_weights(3), [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    for n_r in (4, 9, 17, 33, 65):
        w = og.clenshaw_curtis_weights(n_r)
        x = -np.cos(np.pi * np.arange(n_r) / (n_r - 1))
        for p in range(n_r):
            exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
            assert np.sum(w * x ** p) == pytest.approx(exact, abs=2e-14), (n_r, p)


def test_grid_nodes_and_dt():
    g = og.make_grid(1, 17, 8, 16, 8, 16)
    assert g.dt_default() == pytest.approx(3.842944e-3, rel=1e-6)
    assert og.make_grid(1, 33, 2, 4, 2, 4).dt_default() == pytest.approx(9.630547e-4, rel=1e-6)
    assert og.make_grid(1, 65, 2, 4, 2, 4).dt_default() == pytest.approx(2.409088e-4, rel=1e-6)
    # no Theta node at pi/2 for even n_Theta, no theta node at a pole
    assert np.min(np.abs(np.cos(g.Theta))) > 0.1
    assert np.min(np.sin(g.theta)) > 0.1
