"""Pins of the oracle's angular transform Y = P Phi (Sec. 4.1), CPU only."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import angular


@pytest.mark.parametrize("nt,nphi", [(4, 5), (8, 9), (12, 7)])
def test_y_is_unitary(nt, nphi):
    Y = angular.dense_matrix(nt, nphi)
    np.testing.assert_allclose(Y.conj().T @ Y, np.eye(nt * nphi), atol=1e-13)
    np.testing.assert_allclose(Y @ Y.conj().T, np.eye(nt * nphi), atol=1e-13)


@pytest.mark.parametrize("l,m", [(0, 0), (1, 0), (1, 1), (1, -1), (3, 2), (5, -4), (7, 3), (7, -7)])
def test_sampled_harmonic_gives_one_coefficient(l, m):
    # a spherical harmonic (library routine) with l <= N_theta - 1 sampled with the
    # quadrature weights sqrt(w_j dphi) has the single coefficient 1 at (l, m):
    # Gauss-Legendre integrates these products exactly, so the orthonormalisation
    # leaves the low functions unchanged
    nt, nphi = 8, 17
    eta, w, phi = angular.grid(nt, nphi)
    th = np.arccos(eta)
    psi = special.sph_harm_y(l, m, th[:, None], phi[None, :]) * np.sqrt(w)[:, None] * math.sqrt(2 * math.pi / nphi)
    c = angular.forward(psi[:, :, None], nt, nphi)[:, :, 0]
    ref = np.zeros_like(c)
    M = (nphi - 1) // 2
    ref[m + M, l - abs(m)] = 1.0
    np.testing.assert_allclose(c, ref, atol=1e-13)


def test_round_trip_and_linearity_over_radius():
    rng = np.random.default_rng(3)
    nt, nphi, nr = 6, 11, 5
    psi = rng.standard_normal((nt, nphi, nr)) + 1j * rng.standard_normal((nt, nphi, nr))
    c = angular.forward(psi, nt, nphi)
    np.testing.assert_allclose(angular.inverse(c, nt, nphi), psi, atol=1e-13)
    # each radial point is transformed independently
    np.testing.assert_allclose(angular.forward(psi[:, :, 2:3], nt, nphi)[:, :, 0], c[:, :, 2], atol=1e-14)


def test_negative_m_is_the_condon_shortley_mirror():
    P = angular.p_tables(6, 9)
    M = 4
    for m in range(1, M + 1):
        np.testing.assert_allclose(P[M - m], (-1) ** m * P[M + m], atol=1e-14)


@pytest.mark.parametrize("nt,nphi,ms", [(8, 17, (8, -8, 3, 0)), (14, 27, (13, -13, 6, -1))])
def test_blocks_match_exact_rational_orthonormalisation(nt, nphi, ms):
    # the Lanczos blocks against Gram-Schmidt in exact rationals (same nodes and
    # weights), including the largest |m|, where Gram-Schmidt on the sampled
    # functions in FP64 loses up to 1e-5
    P = angular.p_tables(nt, nphi)
    M = (nphi - 1) // 2
    for m, B in angular.p_tables_exact(nt, nphi, ms).items():
        np.testing.assert_allclose(P[m + M], B, atol=1e-13)


def test_low_blocks_are_the_library_functions():
    # where the quadrature integrates the products exactly (l, l' <= N_theta - 1),
    # the orthonormalised functions are the library's normalised Pbar_l^m
    nt, nphi = 10, 9
    eta, w, _ = angular.grid(nt, nphi)
    P = angular.p_tables(nt, nphi)
    for m in range(-4, 5):
        for t in range(nt - abs(m)):
            l = abs(m) + t
            ref = math.sqrt(2 * math.pi) * special.sph_harm_y(l, m, np.arccos(eta), 0.0).real * np.sqrt(w)
            np.testing.assert_allclose(P[m + 4, t], ref, atol=1e-13)
