"""Host tables of the monomial-moment variant (Sec. 2.6) against the oracle (CPU only)."""
import numpy as np
import pytest

from oracle import dsbt, monomial


@pytest.mark.parametrize("N,ell", [(64, 0), (64, 1), (64, 2), (64, 7), (128, 16), (128, 24), (256, 33)])
def test_monomial_tables_match_oracle(built_lib, N, ell):
    # xi from the library's binary128 expansion equals the oracle's exact
    # rationals rounded to FP64 (to one unit in the last place); alpha_n and the
    # completion rows of eq. Tadd agree with the dense FP64 T
    from paper_1509_07115_amd import host_monomial_tables
    xi, alpha, comp = host_monomial_tables(N, ell)
    k, nz = dsbt.n_extra(ell), dsbt.n0(ell)
    xo, ao, co = monomial.tables(N, ell)
    rows = sorted(xo)
    assert rows[0] == nz and xi.size == len(rows) * k and alpha.size == len(rows) and comp.size == k * N
    X = np.array([[xo[n][nu] for nu in monomial.nonzero_nus(ell)] for n in rows]).reshape(-1)
    if X.size:
        np.testing.assert_allclose(xi, X, rtol=2.5e-16, atol=0)
    np.testing.assert_allclose(alpha, [ao[n] for n in rows], rtol=1e-14, atol=0)
    if k:
        np.testing.assert_allclose(comp.reshape(k, N), co, rtol=0, atol=1e-14)
