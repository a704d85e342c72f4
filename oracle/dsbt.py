"""Dense FP64 oracle of the orthogonal discrete spherical Bessel transform (DSBT).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``; never by the product library.

Everything here is the plain definition written out as dense matrices:

* the sine/cosine Fourier matrix F of Sec. 2.2 (eq. csFourierBasis, k_grid),
* the DLOP P_l(i, N) of Sec. 2.3 (eq. DLOPortho, DLOPnormfac and the
  falling-factorial expansion), evaluated by two recurrences that are
  identities for that definition (checked against exact rationals in
  ``oracle.exact`` by the tests),
* the Fourier-to-Bessel matrix T of Sec. 2.4 (eq. Tdef, Ldef, orthoImL) and
  its completion rows of Sec. 2.5 (eq. Tadd),
* forward b = T F psi and inverse psi = F^T T^T b (eq. f_vs_psi, b_vs_f,
  f_vs_b, and T^{-1} = T^T).

There is no FFT, no fast algorithm and no tiling: a reader can hold each
function against the paper.  Readings of passages that are garbled or silent
(numbered as in the library's design notes):

R1  F is orthonormal: scale sqrt((2 - delta_{n0})/N), and sqrt(1/N) for the
    n = N sine row of even l (the printed 1/sqrt((2-delta)N) is not orthonormal).
R3  F carries the sign sigma_l = (-1)^ceil(l/2) so that f_n = c~_l(k_n) sqrt(w_n)
    as the text after eq. weight_dk states (``sign=False`` drops it).
R4  The diagonal of I - L is not formed as 1 - L_nn (it cancels to all digits
    at large l): the regular row n is v_n / |v_n| with v_nn = 1 and
    v_nm = w_m [P_l(n-m, 2n-1) - P_l(n-m-1, 2n-1)], m < n, which equals
    alpha_n (delta - L) exactly because 2/(1 + P_l(-1, 2n-1)) > 0 factors out.
R5  alpha_n of the completion rows is taken as the numerical row norm, which is
    sqrt(2 / N(l(n), 2 N_l)) exactly but does not overflow.
R6  P_l(x, M) uses the degree recurrence when l^2 <= 2M and otherwise the
    difference equation in x marched from x = 0 (where P = 1).
"""
from __future__ import annotations

import functools
import math

import numpy as np

__all__ = [
    "parity_p", "n0", "n_extra", "n_top", "weights_w", "grid_r", "delta_k",
    "dlop", "fourier_matrix", "ftb_matrix", "dsbt_matrix", "forward", "inverse",
    "sigma",
]


# ---------------------------------------------------------------------------
# index conventions (Sec. 2.2, eq. k_grid; Sec. 2.4, n_0)
# ---------------------------------------------------------------------------

def parity_p(ell: int) -> int:
    """p_l = (1 + (-1)^l)/2: 1 for even l, 0 for odd l (Sec. 2.2, eq. k_grid)."""
    return 1 if ell % 2 == 0 else 0


def n0(ell: int) -> int:
    """n_0l = ceil((l+1)/2): first regular row of T (Sec. 2.4)."""
    return (ell + 2) // 2


def n_extra(ell: int) -> int:
    """Number of completion rows n_0l - p_l = ceil(l/2) (Sec. 2.5)."""
    return n0(ell) - parity_p(ell)


def n_top(N: int, ell: int) -> int:
    """N_l = N + p_l - 1: last momentum index (Sec. 2.2, eq. k_grid)."""
    return N + parity_p(ell) - 1


def sigma(ell: int) -> int:
    """(-1)^ceil(l/2), the sign in eq. tilde_c_def."""
    return -1 if ((ell + 1) // 2) % 2 else 1


def weights_w(N: int, ell: int) -> np.ndarray:
    """sqrt(1 - delta_m0/2) for m = p_l..N_l in slot order j = m - p_l (eq. Ldef)."""
    w = np.ones(N)
    if parity_p(ell) == 0:
        w[0] = math.sqrt(0.5)
    return w


def grid_r(N: int, rmax: float) -> np.ndarray:
    """r_i = (i - 1/2) dr, i = 1..N, dr = rmax/N (Sec. 2.2, eq. r_grid)."""
    dr = rmax / N
    return (np.arange(1, N + 1) - 0.5) * dr


def delta_k(rmax: float) -> float:
    """dk = pi / rmax (Sec. 2.2)."""
    return math.pi / rmax


# ---------------------------------------------------------------------------
# DLOP P_l(x, M), x = 0..xmax  (Sec. 2.3)
# ---------------------------------------------------------------------------

def _dlop_degree_recurrence(ell: int, M: int, x: np.ndarray) -> np.ndarray:
    # (j+1)(M-j) P_{j+1} = (2j+1)(M-2x) P_j - j(M+j+1) P_{j-1},
    # P_0 = 1, P_1 = 1 - 2x/M.
    p_prev = np.ones_like(x)
    if ell == 0:
        return p_prev
    p_cur = 1.0 - 2.0 * x / M
    for j in range(1, ell):
        p_next = ((2 * j + 1) * (M - 2.0 * x) * p_cur - j * (M + j + 1.0) * p_prev) / ((j + 1.0) * (M - j))
        p_prev, p_cur = p_cur, p_next
    return p_cur


def _dlop_difference_march(ell: int, M: int, xmax: int) -> np.ndarray:
    # B(x) y(x+1) = [l(l+1) + B(x) + D(x)] y(x) - D(x) y(x-1),
    # B(x) = (x+1)(x-M), D(x) = x(x-M-1), y(0) = 1.
    y = np.empty(xmax + 1)
    y[0] = 1.0
    if xmax >= 1:
        y[1] = 1.0 - ell * (ell + 1.0) / M
    lam = ell * (ell + 1.0)
    for xx in range(1, xmax):
        B = (xx + 1.0) * (xx - M)
        D = xx * (xx - M - 1.0)
        y[xx + 1] = ((lam + B + D) * y[xx] - D * y[xx - 1]) / B
    return y


def dlop(ell: int, M: int, xmax: int) -> np.ndarray:
    """P_l(x, M) for integer x = 0..xmax, FP64 (reading R6).

    Requires 0 <= l <= M and xmax <= M.  P_l(0, M) = 1 (Sec. 2.3).
    """
    if ell < 0 or ell > M:
        raise ValueError(f"DLOP degree {ell} not defined on {M + 1} points")
    if xmax > M:
        raise ValueError("xmax beyond the grid")
    if M == 0:
        return np.ones(xmax + 1)
    if ell * ell <= 2 * M:
        return _dlop_degree_recurrence(ell, M, np.arange(xmax + 1, dtype=np.float64))
    return _dlop_difference_march(ell, M, xmax)


# ---------------------------------------------------------------------------
# F: sine / cosine transform (Sec. 2.2, eq. csFourierBasis)
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=64)
def fourier_matrix(N: int, ell: int, sign: bool = True) -> np.ndarray:
    """F[j, i], row j = n - p_l (n = p_l..N_l), column i = 0..N-1 (r_{i+1}).

    k_n r_i = pi n (i + 1/2) / N.  Sine rows for even l, cosine rows for odd l,
    orthonormal scale (R1), times sigma_l unless ``sign`` is False (R3).
    """
    p = parity_p(ell)
    n = np.arange(p, p + N, dtype=np.int64)[:, None]
    i = np.arange(N, dtype=np.int64)[None, :]
    # k_n r_i = pi n (2i + 1) / (2N); the integer n (2i + 1) is reduced mod 4N
    # first so the angle stays in [0, 2 pi) without rounding of a large argument.
    arg = math.pi * ((n * (2 * i + 1)) % (4 * N)).astype(np.float64) / (2 * N)
    F = np.sin(arg) if p == 1 else np.cos(arg)
    scale = np.full(N, math.sqrt(2.0 / N))
    if p == 0:
        scale[0] = math.sqrt(1.0 / N)      # cosine row n = 0
    else:
        scale[N - 1] = math.sqrt(1.0 / N)  # sine row n = N
    F = F * scale[:, None]
    if sign:
        F = F * sigma(ell)
    F.setflags(write=False)
    return F


# ---------------------------------------------------------------------------
# T: Fourier-to-Bessel matrix (Sec. 2.4 eq. Tdef/Ldef; Sec. 2.5 eq. Tadd)
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=64)
def ftb_matrix(N: int, ell: int) -> np.ndarray:
    """T[j, j'] with j = n - p_l, j' = m - p_l.  Orthogonal (Appendix A)."""
    p = parity_p(ell)
    nz = n0(ell)
    Nl = n_top(N, ell)
    if ell > 2 * N - 2:
        raise ValueError("need ceil(l/2) <= N - 1 so that a regular row exists")
    w = weights_w(N, ell)
    T = np.zeros((N, N))
    # regular rows n = n_0..N_l (R4): v_nn = 1, v_nm = w_m [P(n-m) - P(n-m-1)]
    for n in range(nz, Nl + 1):
        P = dlop(ell, 2 * n - 1, n)          # P_l(x, 2n-1), x = 0..n
        m = np.arange(p, n)
        v = np.empty(n - p + 1)
        v[: n - p] = w[m - p] * (P[n - m] - P[n - m - 1])
        v[n - p] = 1.0
        T[n - p, : n - p + 1] = v / np.linalg.norm(v)
    # completion rows n = p..n_0-1 (eq. Tadd), l(n) = 2n - p, normalised (R5)
    for n in range(p, nz):
        d = 2 * n - p
        P = dlop(d, 2 * Nl, Nl - p)          # x = N_l - m for m = p..N_l
        m = np.arange(p, Nl + 1)
        row = P[Nl - m] * w
        T[n - p, :] = row / np.linalg.norm(row)
    T.setflags(write=False)
    return T


def dsbt_matrix(N: int, ell: int, sign: bool = True) -> np.ndarray:
    """B = T F (the radial block of eq. BYpsi)."""
    return ftb_matrix(N, ell) @ fourier_matrix(N, ell, sign)


# ---------------------------------------------------------------------------
# transforms
# ---------------------------------------------------------------------------

def _apply(M: np.ndarray, x: np.ndarray) -> np.ndarray:
    """M x for a real matrix M: complex x is transformed linearly, real and
    imaginary parts separately (the same products as a complex product)."""
    if np.iscomplexobj(x):
        # interleaved (re, im) columns of a contiguous complex128 array
        xc = np.ascontiguousarray(x, dtype=np.complex128)
        cols = xc.view(np.float64).reshape(x.shape[0], -1)
        return np.ascontiguousarray(M @ cols).view(np.complex128).reshape(x.shape)
    return M @ x


def forward(psi: np.ndarray, ell: int, sign: bool = True) -> np.ndarray:
    """b = T (F psi) for psi of shape (N,) or (N, C); complex or real, FP64."""
    N = psi.shape[0]
    return _apply(ftb_matrix(N, ell), _apply(fourier_matrix(N, ell, sign), psi))


def inverse(b: np.ndarray, ell: int, sign: bool = True) -> np.ndarray:
    """psi = F^T (T^T b): the inverse because both factors are orthogonal."""
    N = b.shape[0]
    return _apply(fourier_matrix(N, ell, sign).T, _apply(ftb_matrix(N, ell).T, b))
