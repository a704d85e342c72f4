"""Pins of the paper-literal monomial fast multiplication (Sec. 2.6) in the oracle (CPU only)."""
import numpy as np
import pytest

from oracle import dsbt, exact, monomial


@pytest.mark.parametrize("ell", [1, 2, 3, 6, 9])
def test_xi_expansion_is_the_ddlop(ell):
    # eq. DP_expan: -sum_nu xi_nu(n) m^nu equals the DDLOP of the definition
    # (eq. backDiff, exact rationals) at every m = 0..n, and the coefficients of
    # the wrong parity vanish (the DDLOP parity, Sec. 2.6)
    for n in (dsbt.n0(ell), dsbt.n0(ell) + 3, 17):
        xe = monomial.xi_exact(ell, n)
        assert len(xe) == ell
        for m in range(n + 1):
            assert -sum(x * m ** nu for nu, x in enumerate(xe)) == exact.ddlop(ell, n - m, 2 * n)
        for nu in range(ell):
            if nu not in monomial.nonzero_nus(ell):
                assert xe[nu] == 0
    assert len(monomial.nonzero_nus(ell)) == dsbt.n_extra(ell)


@pytest.mark.parametrize("N", [64, 128])
@pytest.mark.parametrize("ell", [0, 1, 2, 3, 4, 5, 8])
def test_literal_matches_dense_transform_where_stable(N, ell):
    # at small l the monomial sums lose little, so the printed algorithm gives
    # T f and T^T b of the dense definition to rounding
    rng = np.random.default_rng(100 + ell)
    T = dsbt.ftb_matrix(N, ell)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = T @ f
    assert np.linalg.norm(monomial.forward_literal(f, ell) - ref) <= 2e-14 * np.linalg.norm(ref)
    assert np.linalg.norm(monomial.inverse_literal(ref, ell) - f) <= 2e-14 * np.linalg.norm(f)


def test_literal_error_grows_with_l():
    # the monomial coefficients grow like a power of l and the sums cancel them
    # (reading of Sec. 2.6: the printed form is exact in exact arithmetic but not
    # stable in FP64); measured: l = 8 5e-15, l = 16 9e-12, l = 24 5e-8 at N = 128
    N = 128
    rng = np.random.default_rng(7)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    err = {}
    for ell in (8, 16, 24):
        ref = dsbt.ftb_matrix(N, ell) @ f
        err[ell] = np.linalg.norm(monomial.forward_literal(f, ell) - ref) / np.linalg.norm(ref)
    assert err[8] < 1e-13
    assert 1e-13 < err[16] < 1e-9
    assert err[24] > 1e3 * err[16] and err[24] > 1e-9
