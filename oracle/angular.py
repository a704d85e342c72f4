"""Angular layer of the DSBT-DVR solver: the transform Y = P Phi between grid values
on (eta_j, phi_k) and spherical-harmonic coefficients (l, m), at every radial point.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 4.1 discretises the angles on N_theta Gauss-Legendre nodes eta_j (weights
w_j) and N_phi uniform azimuths phi_k = 2 pi k / N_phi, with grid values carrying
sqrt(w_j dphi).  Y is the product of

* Phi: per eta_j, the unitary DFT over phi_k to the azimuthal orders m
  (m = -M..M, N_phi = 2M + 1), entries exp(-i m phi_k) / sqrt(N_phi);
* P: per m, the N_theta x N_theta matrix of associated Legendre functions
  Pbar_l^m(eta_j) sqrt(w_j), l = |m| .. |m| + N_theta - 1, orthonormalised on the
  quadrature (in l order).

Pbar_l^m(eta) is (1 - eta^2)^{|m|/2} times a polynomial of degree l - |m| whose
leading coefficient has the sign (-1)^m for m > 0 and + for m <= 0 (Condon-
Shortley phase, Pbar_l^{-m} = (-1)^m Pbar_l^m).  So the first t + 1 functions
on the nodes span {sqrt(W_j) p(eta_j): deg p <= t}, W_j = w_j (1 - eta_j^2)^|m|,
and their orthonormalisation in order is sqrt(W) times the orthonormal
polynomials of the discrete weights W, with that sign.  p_tables builds them
by the Lanczos recurrence on the weighted nodes (multiply by eta, subtract the
projections twice, normalise), which is accurate where Gram-Schmidt on the
sampled Pbar loses digits (for large |m| those vectors are nearly dependent);
p_tables_exact does the same Gram-Schmidt in exact rationals, for the pins.
Coefficient layout: [m index q][l index t][radial i] with m = q - M and
l = |m| + t; grid layout [j][k][i] with eta ascending.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np

__all__ = ["grid", "m_values", "p_tables", "p_tables_exact", "phi_matrix", "forward", "inverse", "dense_matrix"]


def grid(n_theta: int, n_phi: int):
    """(eta, w, phi): Gauss-Legendre nodes (ascending) and weights, azimuths."""
    eta, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    return eta, w, phi


def m_values(n_phi: int) -> np.ndarray:
    if n_phi % 2 != 1:
        raise ValueError("N_phi must be odd (m = -M..M)")
    M = (n_phi - 1) // 2
    return np.arange(-M, M + 1)


def _sign(m: int) -> int:
    return (-1) ** m if m > 0 else 1


@functools.lru_cache(maxsize=16)
def p_tables(n_theta: int, n_phi: int) -> np.ndarray:
    """P[q, t, j] = the orthonormalised Pbar_{|m|+t}^m(eta_j) sqrt(w_j) (Lanczos on the weighted nodes)."""
    eta, w, _ = grid(n_theta, n_phi)
    out = np.zeros((n_phi, n_theta, n_theta))
    for q, m in enumerate(m_values(n_phi)):
        U = out[q]
        sw = np.sqrt(w) * np.sqrt(1.0 - eta ** 2) ** abs(int(m))
        U[0] = sw / np.linalg.norm(sw)
        for t in range(1, n_theta):
            v = eta * U[t - 1]
            for _ in range(2):
                v = v - U[:t].T @ (U[:t] @ v)
            U[t] = v / np.linalg.norm(v)
        U *= _sign(int(m))
    return out


def p_tables_exact(n_theta: int, n_phi: int, ms) -> dict:
    """{m: block} by Gram-Schmidt of the monomials in exact rationals with the weights
    W_j = w_j (1 - eta_j^2)^|m| (the FP64 nodes and weights taken as exact binary
    fractions), evaluated in FP64 at the end.  Slow: small sizes only."""
    eta, w, _ = grid(n_theta, n_phi)
    E = [Fraction(float(x)) for x in eta]
    out = {}
    for m in ms:
        W = [Fraction(float(wj)) * (1 - e * e) ** abs(m) for wj, e in zip(w, E)]
        qs, norms = [], []
        for t in range(n_theta):
            v = [e ** t for e in E]
            for qv, nq in zip(qs, norms):
                c = sum(Wj * a * b for Wj, a, b in zip(W, qv, v)) / nq
                v = [a - c * b for a, b in zip(v, qv)]
            qs.append(v)
            norms.append(sum(Wj * a * a for Wj, a in zip(W, v)))
        B = np.zeros((n_theta, n_theta))
        for t in range(n_theta):
            nrm = math.sqrt(float(norms[t]))
            for j in range(n_theta):
                B[t, j] = _sign(m) * math.sqrt(w[j]) * math.sqrt(1 - eta[j] ** 2) ** abs(m) * float(qs[t][j]) / nrm
        out[m] = B
    return out


def phi_matrix(n_phi: int) -> np.ndarray:
    """Phi[q, k] = exp(-i m_q phi_k) / sqrt(N_phi)."""
    _, _, phi = grid(1, n_phi)
    return np.exp(-1j * np.outer(m_values(n_phi), phi)) / math.sqrt(n_phi)


def forward(psi: np.ndarray, n_theta: int, n_phi: int) -> np.ndarray:
    """c[q, t, i] = sum_j P[q, t, j] sum_k Phi[q, k] psi[j, k, i]."""
    P, F = p_tables(n_theta, n_phi), phi_matrix(n_phi)
    a = np.einsum("qk,jki->jqi", F, psi)          # per eta_j: DFT over phi
    return np.einsum("qtj,jqi->qti", P, a)         # per m: associated Legendre functions


def inverse(c: np.ndarray, n_theta: int, n_phi: int) -> np.ndarray:
    """psi = Y^H c (Y is unitary)."""
    P, F = p_tables(n_theta, n_phi), phi_matrix(n_phi)
    a = np.einsum("qtj,qti->jqi", P, c)
    return np.einsum("qk,jqi->jki", F.conj(), a)


def dense_matrix(n_theta: int, n_phi: int) -> np.ndarray:
    """Y as a dense (N_phi N_theta) x (N_theta N_phi) matrix, rows (q, t), columns (j, k)."""
    P, F = p_tables(n_theta, n_phi), phi_matrix(n_phi)
    Y = np.einsum("qtj,qk->qtjk", P, F)
    return Y.reshape(n_phi * n_theta, n_theta * n_phi)
