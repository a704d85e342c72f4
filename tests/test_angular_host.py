"""Host tables of the angular transform (Sec. 4.1) against the oracle (CPU only)."""
import numpy as np
import pytest

from oracle import angular


@pytest.mark.parametrize("nt,nphi,tol", [(1, 1, 1e-15), (4, 5, 1e-14), (8, 17, 1e-13), (16, 31, 1e-13),
                                         (24, 47, 1e-13), (64, 63, 1e-12)])
def test_grid_and_tables_match_oracle(built_lib, nt, nphi, tol):
    # both build the blocks by the Lanczos recurrence on the weighted nodes (in
    # independent code); the oracle's form is pinned to exact rationals
    from paper_1509_07115_amd import sht_grid, sht_host_tables
    eta, w, phi = sht_grid(nt, nphi)
    e0, w0, p0 = angular.grid(nt, nphi)
    np.testing.assert_allclose(eta, e0, atol=1e-15)
    np.testing.assert_allclose(w, w0, rtol=5e-12)   # two FP64 Newton solutions
    np.testing.assert_allclose(phi, p0, atol=1e-15)
    P = sht_host_tables(nt, nphi)
    np.testing.assert_allclose(P, angular.p_tables(nt, nphi), atol=tol)


def test_rejects_unsupported_sizes(built_lib):
    from paper_1509_07115_amd import DsbtError, sht_grid
    for nt, nphi in ((0, 5), (65, 5), (8, 4), (8, 65)):
        with pytest.raises(DsbtError, match="UNSUPPORTED"):
            sht_grid(nt, nphi)
