"""Pins of the oracle's DLOP and T against exact rational arithmetic (CPU only).

Each identity checked here is one the paper states (Sec. 2.3-2.5, Appendix A);
the exact values come from the defining falling-factorial sums, not from any
recurrence the FP64 oracle uses.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import dsbt, exact


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8, 13])
def test_dlop_orthogonality_and_norm(M):
    # eq. DLOPortho with the norm factor of eq. DLOPnormfac, and P_l(0, M) = 1
    P = {l: [exact.dlop(l, i, M) for i in range(M + 1)] for l in range(M + 1)}
    for l in range(M + 1):
        assert P[l][0] == 1
        for mu in range(l + 1):
            s = sum(a * b for a, b in zip(P[l], P[mu]))
            assert s == (exact.norm_factor(l, M) if mu == l else 0)


@pytest.mark.parametrize("M", [4, 7, 10])
def test_dlop_parity_and_moments(M):
    # eq. DLOPparity (Appendix A) and eq. intDPx
    for l in range(M + 1):
        P = [exact.dlop(l, i, M) for i in range(M + 1)]
        for i in range(M + 1):
            assert P[i] == (-1) ** l * P[M - i]
        for s in range(l):
            assert sum(P[i] * i ** s for i in range(M + 1)) == 0


@pytest.mark.parametrize("M", [3, 6, 9])
def test_ddlop_weighted_sum_identity(M):
    # eq. sumDDPp: sum_i P'_l(i, M) p(i) w_i(M) = (-1)^l p(M) - p(0) for deg p < l
    rng = np.random.default_rng(5)
    for l in range(1, M):
        for mu in range(l):
            C = [Fraction(int(c)) for c in rng.integers(-5, 6, size=mu + 1)]
            p = lambda i: sum(c * i ** s for s, c in enumerate(C))  # noqa: E731
            lhs = Fraction(0)
            for i in range(M + 1):
                wi = Fraction(1, 2) if i in (0, M) else Fraction(1)
                lhs += exact.ddlop(l, i, M) * p(i) * wi
            assert lhs == (-1) ** l * p(M) - p(0)


@pytest.mark.parametrize("N", [3, 5, 8])
def test_rows_of_I_minus_L_orthogonal(N):
    # eq. orthoImL: rows n, m >= n_0 of I - L are orthogonal (theta(0) = 1/2)
    for ell in range(0, 2 * N - 1):
        rows = exact.imL_rows(N, ell)
        keys = sorted(rows)
        for a in keys:
            for b in keys:
                if b <= a:
                    continue
                g = sum(exact.w_sq(m) * rows[a][m] * rows[b].get(m, 0) for m in rows[a])
                assert g == 0, (ell, a, b)


@pytest.mark.parametrize("N", [3, 5, 8])
def test_completion_rows(N):
    # eq. Tadd: completion rows are orthogonal to every regular row and to each
    # other, and their squared weighted norm is N(l(n), 2N_l)/2 (alpha_n = sqrt(2/N)).
    for ell in range(1, 2 * N - 1):
        p = dsbt.parity_p(ell)
        Nl = dsbt.n_top(N, ell)
        reg = exact.imL_rows(N, ell)
        ext = exact.completion_rows(N, ell)
        for n, row in ext.items():
            nrm = sum(exact.w_sq(m) * row[m] ** 2 for m in row)
            assert nrm == exact.norm_factor(2 * n - p, 2 * Nl) / 2
            for r in reg.values():
                assert sum(exact.w_sq(m) * row[m] * r.get(m, 0) for m in row) == 0
            for n2, row2 in ext.items():
                if n2 > n:
                    assert sum(exact.w_sq(m) * row[m] * row2[m] for m in row) == 0


@pytest.mark.parametrize("N", [4, 7])
def test_regular_row_is_positive_multiple_of_v(N):
    # reading R4: (I - L)_n = 2/(1 + P_l(-1, 2n-1)) v_n with v_nn = 1 and
    # v_nm = w_m [P_l(n-m, 2n-1) - P_l(n-m-1, 2n-1)]; the factor is positive.
    for ell in range(0, 2 * N - 1):
        for n, row in exact.imL_rows(N, ell).items():
            c = (1 + exact.dlop(ell, -1, 2 * n - 1)) / 2
            assert c > 0
            for m, R in row.items():
                expect = 1 if m == n else exact.dlop(ell, n - m, 2 * n - 1) - exact.dlop(ell, n - m - 1, 2 * n - 1)
                assert R * c == expect


def test_fp64_dlop_matches_exact():
    worst = 0.0
    for M in range(1, 34):
        for ell in range(M + 1):
            xmax = M // 2 + 1
            P = dsbt.dlop(ell, M, xmax)
            E = np.array([float(exact.dlop(ell, i, M)) for i in range(xmax + 1)])
            worst = max(worst, np.max(np.abs(P - E)) / np.max(np.abs(E)))
    assert worst < 1e-13


@pytest.mark.parametrize("N", [2, 4, 6, 9])
def test_fp64_T_matches_exact(N):
    for ell in range(0, 2 * N - 1):
        p = dsbt.parity_p(ell)
        T = dsbt.ftb_matrix(N, ell)
        Te = np.zeros((N, N))
        for rows in (exact.imL_rows(N, ell), exact.completion_rows(N, ell)):
            for n, row in rows.items():
                g = sum(exact.w_sq(m) * v ** 2 for m, v in row.items())
                a = float(1 / g) ** 0.5
                for m, v in row.items():
                    Te[n - p, m - p] = a * float(exact.w_sq(m)) ** 0.5 * float(v)
        assert np.max(np.abs(T - Te)) < 1e-13, ell
