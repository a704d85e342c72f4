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

The normalised Pbar_l^m are read from a library routine: Pbar_l^m(eta) =
sqrt(2 pi) Y_l^m(arccos eta, 0) (Condon-Shortley phase, so Pbar_l^{-m} =
(-1)^m Pbar_l^m).  Coefficient layout: [m index q][l index t][radial i] with
m = q - M and l = |m| + t; grid layout [j][k][i] with eta ascending.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy import special

__all__ = ["grid", "m_values", "p_tables", "phi_matrix", "forward", "inverse", "dense_matrix"]


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


def _gram_schmidt_rows(V: np.ndarray) -> np.ndarray:
    Q = np.array(V, dtype=np.float64)
    for t in range(Q.shape[0]):
        for s in range(t):
            Q[t] -= np.dot(Q[s], Q[t]) * Q[s]
        Q[t] /= np.linalg.norm(Q[t])
    return Q


@functools.lru_cache(maxsize=16)
def p_tables(n_theta: int, n_phi: int) -> np.ndarray:
    """P[q, t, j] = Pbar_{|m|+t}^m(eta_j) sqrt(w_j), rows orthonormalised in t."""
    eta, w, _ = grid(n_theta, n_phi)
    theta = np.arccos(eta)
    out = np.zeros((n_phi, n_theta, n_theta))
    for q, m in enumerate(m_values(n_phi)):
        V = np.zeros((n_theta, n_theta))
        for t in range(n_theta):
            l = abs(int(m)) + t
            V[t] = math.sqrt(2.0 * math.pi) * special.sph_harm_y(l, int(m), theta, 0.0).real * np.sqrt(w)
        out[q] = _gram_schmidt_rows(V)
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
