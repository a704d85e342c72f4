"""Pins of the dense FP64 DSBT oracle against library routines, closed forms and
the paper's invariants (CPU only)."""
import math

import numpy as np
import pytest
import scipy.fft

from oracle import dsbt, sbf


@pytest.mark.parametrize("N", [8, 64, 256])
@pytest.mark.parametrize("ell", [0, 1, 2, 3, 6, 7])
def test_fourier_matrix_is_orthonormal_dct_dst(N, ell):
    # reading R1: F equals SciPy's orthonormal DCT-II (odd l) / DST-II (even l),
    # times sigma_l (reading R3); F F^T = I.
    F = dsbt.fourier_matrix(N, ell)
    x = np.random.default_rng(N + ell).standard_normal(N)
    ref = (scipy.fft.dst(x, type=2, norm="ortho") if ell % 2 == 0
           else scipy.fft.dct(x, type=2, norm="ortho"))
    assert np.max(np.abs(F @ x - dsbt.sigma(ell) * ref)) < 1e-13
    assert np.max(np.abs(F @ F.T - np.eye(N))) < 1e-13


@pytest.mark.parametrize("N,ells", [(64, range(0, 127)), (256, range(0, 16)), (512, [31, 63, 64, 127])])
def test_T_orthogonal(N, ells):
    # Appendix A: T T^T = I
    for ell in ells:
        T = dsbt.ftb_matrix(N, ell)
        assert np.max(np.abs(T @ T.T - np.eye(N))) < 1e-13, ell


@pytest.mark.slow
@pytest.mark.parametrize("N,ell", [(2048, 63), (2048, 127), (4096, 31)])
def test_T_orthogonal_large(N, ell):
    T = dsbt.ftb_matrix(N, ell)
    assert np.max(np.abs(T @ T.T - np.eye(N))) < 1e-13


def test_ell0_is_identity_and_ell1_kernel():
    # Sec. 2.1: c_0 = c~_0, so T = I for l = 0.  For l = 1 the DDLOP is the
    # constant P'_1(i, 2n) = -1/n, so L_nm = w_m/n below the diagonal and
    # L_nn = 1/(2n) (theta(0) = 1/2).
    N = 32
    assert np.array_equal(dsbt.ftb_matrix(N, 0), np.eye(N))
    T = dsbt.ftb_matrix(N, 1)
    w = dsbt.weights_w(N, 1)
    for n in range(1, N):  # p = 0, slot = n
        row = np.zeros(N)
        row[:n] = -w[:n] / n
        row[n] = 1.0 - 1.0 / (2 * n)
        row /= np.linalg.norm(row)
        assert np.max(np.abs(T[n] - row)) < 1e-14
    # completion row n = 0: l(0) = 0, the constant DLOP
    assert np.max(np.abs(T[0] - w / np.linalg.norm(w))) < 1e-14


def _gauss_case(ell, rmax, dr=0.4, a=0.5):
    N = int(round(rmax / dr))
    r = dsbt.grid_r(N, rmax)
    psi = r ** (ell + 1) * np.exp(-a * r * r) * math.sqrt(rmax / N)
    b = dsbt.forward(psi, ell)
    p = dsbt.parity_p(ell)
    dk = dsbt.delta_k(rmax)
    k = np.arange(p, p + N) * dk
    nz = dsbt.n0(ell)
    c = sbf.gaussian_sbt(k, ell, a) * math.sqrt(dk)
    return b, c, nz - p, dk


@pytest.mark.parametrize("ell", [1, 2, 3, 5])
def test_gaussian_closed_form_converges_as_dk2(ell):
    # Sec. 3 (Fig. 1): |c_nl - c_l(k_n)| falls as dk^2: x4 per doubling of rmax
    # at dr = 0.4; rmax = 51.2, 102.4, 204.8.  Regular rows only.
    errs = []
    for rmax in (51.2, 102.4, 204.8):
        b, c, s0, dk = _gauss_case(ell, rmax)
        errs.append(np.max(np.abs(b[s0:] - c[s0:])) / math.sqrt(dk))
    assert errs[0] < 0.05
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.8 < e1 / e2 < 4.2, errs


def test_gaussian_closed_form_ell0_exact_to_rounding():
    b, c, s0, dk = _gauss_case(0, 51.2)
    assert np.max(np.abs(b - c)) < 1e-12


@pytest.mark.parametrize("ell", [1, 2, 3, 4, 5, 7, 11])
def test_completion_coefficients_vanish_for_smooth_input(ell):
    # Sec. 2.5: for psi ~ r^(l+1) at the origin the rows n < n_0 give b_n ~ 0
    # (measured: 2e-12 at l = 1 rising to 4e-7 at l = 11 on dr = 0.4).
    b, c, s0, dk = _gauss_case(ell, 102.4)
    assert np.max(np.abs(b[:s0])) <= 1e-6 * np.max(np.abs(b))


def test_bruteforce_quadrature_agrees_to_order_dk2():
    # O(N^2) midpoint quadrature of eq. BesselProj at the grid momenta: the
    # difference to the DSBT shrinks ~x4 per rmax doubling (dr fixed).
    ell, a = 2, 0.5
    diffs = []
    for rmax in (12.8, 25.6):
        N = int(round(rmax / 0.2))
        r = dsbt.grid_r(N, rmax)
        dk = dsbt.delta_k(rmax)
        psi = r ** (ell + 1) * np.exp(-a * r * r) * math.sqrt(rmax / N)
        b = dsbt.forward(psi, ell)
        p = dsbt.parity_p(ell)
        s0 = dsbt.n0(ell) - p
        k = np.arange(p, p + N)[s0:40] * dk
        q = sbf.quadrature_sbt(lambda x: x ** (ell + 1) * np.exp(-a * x * x), N, rmax, ell, k)
        diffs.append(np.max(np.abs(b[s0:40] / math.sqrt(dk) - q)))
    assert diffs[1] < diffs[0] / 3.0


def test_basis_functions_approach_sbf():
    # Sec. 3 (Figs. 2, 4, 5): column n of (T F)^T, scaled by sqrt(N/2), tends to
    # chi_l(k_n r) at fixed k: on a fixed window r < 20 the error falls ~x4 per
    # doubling of rmax (dk^2); over the whole box it grows with r, and the
    # corrected momentum k_nl of eq. kcorr cuts it by about an order of magnitude.
    ell, dr = 3, 0.4
    k_fixed = math.pi / 6.4
    win, full, full_c = [], [], []
    for rmax in (51.2, 102.4):
        N = int(round(rmax / dr))
        B = dsbt.dsbt_matrix(N, ell)
        dk = dsbt.delta_k(rmax)
        n = int(round(k_fixed / dk))
        p = dsbt.parity_p(ell)
        r = dsbt.grid_r(N, rmax)
        chit = B[n - p] * math.sqrt(N / 2)
        e = np.abs(chit - sbf.chi(ell, n * dk * r))
        kc = sbf.corrected_momenta(N, rmax, ell)[n - dsbt.n0(ell)]
        win.append(e[r < 20].max())
        full.append(e.max())
        full_c.append(np.abs(chit - sbf.chi(ell, kc * r)).max())
    assert win[1] < win[0] / 3.0
    assert full_c[0] < full[0] / 5.0 and full_c[1] < full[1] / 5.0


@pytest.mark.parametrize("ell", [0, 1, 6, 31])
def test_roundtrip_and_norm(ell):
    N = 256
    rng = np.random.default_rng(ell)
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    b = dsbt.forward(psi, ell)
    assert abs(np.linalg.norm(b) - np.linalg.norm(psi)) < 1e-12 * np.linalg.norm(psi)  # eq. conservNorm
    back = dsbt.inverse(b, ell)
    assert np.max(np.abs(back - psi)) < 1e-12


def test_sign_option_only_flips_sigma():
    N, ell = 64, 3
    x = np.random.default_rng(1).standard_normal(N)
    assert np.allclose(dsbt.forward(x, ell, sign=False), dsbt.sigma(ell) * dsbt.forward(x, ell))
