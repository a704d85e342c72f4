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

import functools
import math

import numpy as np

from . import angular, dsbt, tdse

__all__ = ["step3d", "expect_z", "grid_r_eta", "to_momentum_order", "from_momentum_order", "step3d_velocity",
           "oscillator_exact"]


def grid_r_eta(nr: int, rmax: float, nt: int, nphi: int):
    """r[i], eta[j] and the grid shape (nt, nphi, nr)."""
    eta, _, _ = angular.grid(nt, nphi)
    return dsbt.grid_r(nr, rmax), eta


@functools.lru_cache(maxsize=256)
def _kinetic(nr: int, rmax: float, ell: int, corrected: bool) -> np.ndarray:
    E = tdse.kinetic_energies(nr, rmax, ell, corrected)
    E.setflags(write=False)
    return E


def step3d(psi: np.ndarray, rmax: float, V0: np.ndarray, V1: np.ndarray, F: float, dt: float,
           corrected: bool = False) -> np.ndarray:
    nt, nphi, nr = psi.shape
    ph = np.exp(-1j * (V0 + F * V1) * dt / 2.0)
    c = angular.forward(ph * psi, nt, nphi)
    M = (nphi - 1) // 2
    for q in range(nphi):
        for t in range(nt):
            ell = abs(q - M) + t
            E = _kinetic(nr, rmax, ell, corrected)
            b = dsbt.forward(c[q, t], ell)
            c[q, t] = dsbt.inverse(np.exp(-1j * E * dt) * b, ell)
    return ph * angular.inverse(c, nt, nphi)


def expect_z(psi: np.ndarray, r: np.ndarray, eta: np.ndarray) -> float:
    """<z> = sum |psi_jki|^2 r_i eta_j (the grid values carry the volume weights)."""
    return float(np.sum(np.abs(psi) ** 2 * r[None, None, :] * eta[:, None, None]))


# --- velocity gauge (Sec. 4.1, the printed nine-line sequence) ---------------
#
# With a vector potential A(t) along z the step passes through the momentum
# DVR: c = B Y psi, a half kinetic factor, phi = Ytilde^H c on the unified
# momentum grid k~_n = n dk (n = 1..N, eq. tilde_k_grid), the factor
# exp(i A k~_n eta_j tau), back with Ytilde, the second half kinetic factor,
# psi = Y^H B^T c.  Ytilde = i^l Y (modified spherical harmonics).  On the
# unified grid the slots of even l (n = 1..N) stay in place; for odd l the slot
# of n = 0 moves to n = N (reading: it stands for the top momentum).


def to_momentum_order(c: np.ndarray, ell: int) -> np.ndarray:
    """Channel coefficients in slot order -> unified order n = 1..N."""
    return c if ell % 2 == 0 else np.roll(c, -1, axis=-1)


def from_momentum_order(u: np.ndarray, ell: int) -> np.ndarray:
    return u if ell % 2 == 0 else np.roll(u, 1, axis=-1)


def step3d_velocity(psi: np.ndarray, rmax: float, V0: np.ndarray, A: float, dt: float,
                    corrected: bool = False) -> np.ndarray:
    nt, nphi, nr = psi.shape
    M = (nphi - 1) // 2
    eta, _, _ = angular.grid(nt, nphi)
    ktil = np.arange(1, nr + 1) * dsbt.delta_k(rmax)
    pu = np.exp(-1j * V0 * dt / 2.0)
    c = angular.forward(pu * psi, nt, nphi)
    ls = [[abs(q - M) + t for t in range(nt)] for q in range(nphi)]
    half = {}
    for q in range(nphi):
        for t in range(nt):
            ell = ls[q][t]
            half[ell] = np.exp(-1j * _kinetic(nr, rmax, ell, corrected) * dt / 2.0)
            c[q, t] = to_momentum_order(half[ell] * dsbt.forward(c[q, t], ell), ell) * (1j) ** (-ell)
    phi = angular.inverse(c, nt, nphi)                                 # Ytilde^H on the momentum grid
    phi *= np.exp(1j * A * ktil[None, None, :] * eta[:, None, None] * dt)
    c = angular.forward(phi, nt, nphi)
    for q in range(nphi):
        for t in range(nt):
            ell = ls[q][t]
            b = from_momentum_order(c[q, t] * (1j) ** ell, ell)
            c[q, t] = dsbt.inverse(half[ell] * b, ell)
    return pu * angular.inverse(c, nt, nphi)


def oscillator_exact(nr: int, rmax: float, nt: int, nphi: int, t: float, omega: float, A0: float) -> np.ndarray:
    """Grid values of the exact solution for U = r^2/2 - F(t) z, F = omega A0 cos(omega t),
    from the ground state at t = 0 (Sec. 4.2): the ground state moved to the classical
    point (z_c, p_c), times exp(i p_c (z - z_c) + i S(t) - 3 i t / 2), with S the classical
    action integral of p_c^2/2 - z_c^2/2 + F z_c (library quadrature)."""
    from scipy.integrate import quad
    w1 = omega * A0 / (1.0 - omega ** 2)
    zc_f = lambda s: w1 * (math.cos(omega * s) - math.cos(s))
    pc_f = lambda s: w1 * (math.sin(s) - omega * math.sin(omega * s))
    lag = lambda s: 0.5 * pc_f(s) ** 2 - 0.5 * zc_f(s) ** 2 + omega * A0 * math.cos(omega * s) * zc_f(s)
    S = quad(lag, 0.0, t, epsabs=1e-14, epsrel=1e-13, limit=500)[0]
    zc, pc = zc_f(t), pc_f(t)
    dr = rmax / nr
    r = dsbt.grid_r(nr, rmax)
    eta, w, _ = angular.grid(nt, nphi)
    z = r[None, None, :] * eta[:, None, None]
    rho2 = r[None, None, :] ** 2 * (1 - eta[:, None, None] ** 2)
    psi = math.pi ** -0.75 * np.exp(-rho2 / 2 - (z - zc) ** 2 / 2 + 1j * (pc * (z - zc) + S - 1.5 * t))
    wts = r[None, None, :] * math.sqrt(dr) * np.sqrt(w * 2 * math.pi / nphi)[:, None, None]
    return psi * wts * np.ones((1, nphi, 1))
