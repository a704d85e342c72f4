"""Dense split-operator step of the 3D DSBT-DVR solver in the coordinate gauge.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 4.1 with zero vector potential: on grid values psi[j][k][i] (Gauss-Legendre
node eta_j, azimuth phi_k, radius r_i)

    psi <- exp(-i U tau/2) Y^H B^T exp(-i K tau) B Y exp(-i U tau/2) psi,

U = U(r_i, theta_j, phi_k, t + tau/2) the potential on the grid, Y the angular
transform, B the radial DSBT of each (l, m) channel and K the kinetic diagonal
(the two half kinetic factors of the printed sequence merge when the vector
potential is zero).  Here U = V0 + F V1 with fixed grid fields V0, V1 and the
step's scalar strength F.
"""
from __future__ import annotations

import numpy as np

from . import angular, dsbt, tdse

__all__ = ["step3d", "expect_z", "grid_r_eta"]


def grid_r_eta(nr: int, rmax: float, nt: int, nphi: int):
    """r[i], eta[j] and the grid shape (nt, nphi, nr)."""
    eta, _, _ = angular.grid(nt, nphi)
    return dsbt.grid_r(nr, rmax), eta


def step3d(psi: np.ndarray, rmax: float, V0: np.ndarray, V1: np.ndarray, F: float, dt: float,
           corrected: bool = False) -> np.ndarray:
    nt, nphi, nr = psi.shape
    ph = np.exp(-1j * (V0 + F * V1) * dt / 2.0)
    c = angular.forward(ph * psi, nt, nphi)
    M = (nphi - 1) // 2
    for q in range(nphi):
        for t in range(nt):
            ell = abs(q - M) + t
            E = tdse.kinetic_energies(nr, rmax, ell, corrected)
            b = dsbt.forward(c[q, t], ell)
            c[q, t] = dsbt.inverse(np.exp(-1j * E * dt) * b, ell)
    return ph * angular.inverse(c, nt, nphi)


def expect_z(psi: np.ndarray, r: np.ndarray, eta: np.ndarray) -> float:
    """<z> = sum |psi_jki|^2 r_i eta_j (the grid values carry the volume weights)."""
    return float(np.sum(np.abs(psi) ** 2 * r[None, None, :] * eta[:, None, None]))
