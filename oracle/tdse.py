"""Dense FP64 split-operator step of the DSBT-DVR solver, and its adjoint.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

One step for a radial channel of angular momentum l with zero vector
potential (Sec. 4.1, the split-operator sequence with A = 0, where the two
half kinetic factors are adjacent and merge):

    psi <- exp(-i s V tau/2) F^T T^T exp(-i E tau) T F exp(-i s V tau/2) psi

with the diagonal kinetic energy E_n = k_nl^2 / 2 (eq. KinMat).  k_nl is
n dk (plain mode, eq. tilde_k_grid) or the root of eq. kcorr (corrected mode)
for the regular rows n >= n_0l; the completion rows (n < n_0l, which include
n = 0 of odd l) take (N dk)^2/2 (reading R7: they are the highest-momentum
components, Sec. 2.5 and the remark after eq. tilde_k_grid).

The adjoint follows the PyTorch convention: the gradient with respect to a
complex tensor is 2 dL/d(conj psi), so for L = |<phi|psi_T>|^2 it starts at
2 z phi with z = <phi|psi_T>, runs backwards through U_t^H = U_t^{-1}
(all factors are unitary), and dL/ds_t = (tau/2) sum_i V_i
Im(conj(lam_{t+1}) psi_{t+1} + conj(lam_t) psi_t).
"""
from __future__ import annotations

import numpy as np

from . import dsbt
from .sbf import corrected_momenta

__all__ = ["kinetic_energies", "hamiltonian", "step", "propagate", "loss_and_grad", "loss_and_grad_blocks",
           "imag_step", "orthonormalize", "energy_terms", "imag_time"]


def kinetic_energies(N: int, rmax: float, ell: int, corrected: bool = False) -> np.ndarray:
    """E in slot order j = n - p_l."""
    p = dsbt.parity_p(ell)
    nz = dsbt.n0(ell)
    dk = dsbt.delta_k(rmax)
    E = np.empty(N)
    E[: nz - p] = 0.5 * (N * dk) ** 2
    if corrected:
        k = corrected_momenta(N, rmax, ell)
    else:
        k = np.arange(nz, N + p) * dk
    E[nz - p:] = 0.5 * k ** 2
    return E


def hamiltonian(N: int, rmax: float, ell: int, V: np.ndarray, corrected: bool = False) -> np.ndarray:
    """Dense H = B^T diag(E) B + diag(V) (eq. H_DVR with A = 0, one channel)."""
    B = dsbt.dsbt_matrix(N, ell)
    E = kinetic_energies(N, rmax, ell, corrected)
    return B.T @ (E[:, None] * B) + np.diag(V)


def step(psi: np.ndarray, ell: int, V: np.ndarray, E: np.ndarray, dt: float,
         s: float = 1.0, adjoint: bool = False) -> np.ndarray:
    """One split-operator step U (or U^H when ``adjoint``) on psi of shape (N,) or (N, C)."""
    sg = 1.0 if adjoint else -1.0
    pv = np.exp(sg * 1j * s * V * dt / 2.0)
    pk = np.exp(sg * 1j * E * dt)
    if psi.ndim == 2:
        pv = pv[:, None]
        pk = pk[:, None]
    x = pv * psi
    b = dsbt.forward(x, ell)
    x = dsbt.inverse(pk * b, ell)
    return pv * x


def propagate(psi0: np.ndarray, ell: int, V: np.ndarray, E: np.ndarray, dt: float,
              s: np.ndarray, keep: bool = False):
    """Apply steps t = 0..len(s)-1 with potential strengths s[t]."""
    x = np.array(psi0, dtype=np.complex128)
    states = [x] if keep else None
    for st in s:
        x = step(x, ell, V, E, dt, st)
        if keep:
            states.append(x)
    return states if keep else x


def loss_and_grad(psi0: np.ndarray, phi: np.ndarray, ell: int, V: np.ndarray, E: np.ndarray,
                  dt: float, s: np.ndarray):
    """L = |<phi|psi_T>|^2 and its gradients (PyTorch convention) wrt psi0 and s."""
    states = propagate(psi0, ell, V, E, dt, s, keep=True)
    z = np.vdot(phi, states[-1])
    L = float(abs(z) ** 2)
    lam = 2.0 * z * np.asarray(phi, dtype=np.complex128)
    gs = np.zeros(len(s))
    Vb = V[:, None] if psi0.ndim == 2 else V
    for t in range(len(s) - 1, -1, -1):
        lam_next = lam
        lam = step(lam_next, ell, V, E, dt, s[t], adjoint=True)
        acc = np.conj(lam_next) * states[t + 1] + np.conj(lam) * states[t]
        gs[t] = 0.5 * dt * float(np.sum(Vb * acc.imag))
    return L, lam, gs


def loss_and_grad_blocks(blocks, dt: float, s: np.ndarray):
    """L = |<phi|psi_T>|^2 over several channel blocks and its gradients.

    blocks: list of (ell, V, E, psi0, phi) with psi0, phi of shape (N,) or (N, C)
    (channels of one l).  The overlap z sums over every block, so the adjoint
    of each block starts from 2 z phi.  Returns (L, [grad psi0 per block], grad s).
    """
    states = [propagate(p0, ell, V, E, dt, s, keep=True) for ell, V, E, p0, _ in blocks]
    z = sum(np.vdot(b[4], st[-1]) for b, st in zip(blocks, states))
    L = float(abs(z) ** 2)
    gs = np.zeros(len(s))
    grads = []
    for (ell, V, E, p0, phi), st in zip(blocks, states):
        lam = 2.0 * z * np.asarray(phi, dtype=np.complex128)
        Vb = V[:, None] if np.ndim(p0) == 2 else V
        for t in range(len(s) - 1, -1, -1):
            lam_next = lam
            lam = step(lam_next, ell, V, E, dt, s[t], adjoint=True)
            acc = np.conj(lam_next) * st[t + 1] + np.conj(lam) * st[t]
            gs[t] += 0.5 * dt * float(np.sum(Vb * acc.imag))
        grads.append(lam)
    return L, grads, gs


# --- Imaginary-time method (Sec. 4.3) -------------------------------------
#
# Bound states are found by propagating in imaginary time: t -> -i t turns
# every unitary factor exp(-i X tau) of the step into the real decay
# exp(-X tau), so the component along an eigenvector of energy E shrinks like
# exp(-E tau) per step and the lowest state dominates.  Excited states of one
# l are obtained by orthogonalising each state to the lower ones after every
# step (Sec. 4.3), and the energy is the expectation of the dense
# Hamiltonian of eq. H_DVR: <psi|B^T diag(E) B + diag(V)|psi> / <psi|psi>.


def imag_step(psi: np.ndarray, ell: int, V: np.ndarray, E: np.ndarray, dt: float) -> np.ndarray:
    """One imaginary-time step exp(-V tau/2) F^T T^T exp(-E tau) T F exp(-V tau/2) on
    psi of shape (N,) or (N, C)."""
    pv = np.exp(-V * dt / 2.0)
    pk = np.exp(-E * dt)
    if psi.ndim == 2:
        pv = pv[:, None]
        pk = pk[:, None]
    x = pv * psi
    b = dsbt.forward(x, ell)
    x = dsbt.inverse(pk * b, ell)
    return pv * x


def orthonormalize(X: np.ndarray) -> np.ndarray:
    """Gram-Schmidt over the columns of X (N, m) in column order: column j loses
    its components along the already orthonormalised columns 0..j-1 one at a
    time (modified form), then is scaled to unit norm."""
    Y = np.array(X, dtype=np.complex128)
    for j in range(Y.shape[1]):
        for i in range(j):
            Y[:, j] -= np.vdot(Y[:, i], Y[:, j]) * Y[:, i]
        Y[:, j] /= np.linalg.norm(Y[:, j])
    return Y


def energy_terms(psi: np.ndarray, ell: int, V: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Per column of psi (N,) or (N, C): [<psi|psi>, <psi|V|psi>, <psi|B^T E B|psi>]
    (the kinetic term from b = T F psi, eq. H_DVR)."""
    P = psi[:, None] if psi.ndim == 1 else psi
    b = dsbt.forward(P, ell)
    a2 = np.abs(P) ** 2
    out = np.stack([a2.sum(0), (V[:, None] * a2).sum(0), (E[:, None] * np.abs(b) ** 2).sum(0)], 1)
    return out[0] if psi.ndim == 1 else out


def imag_time(X0: np.ndarray, ell: int, V: np.ndarray, E: np.ndarray, dt: float, nsteps: int) -> np.ndarray:
    """nsteps imaginary-time steps of the states X0 (N, m) of one l, each followed by
    orthonormalisation in column order (state j is kept orthogonal to states < j)."""
    X = orthonormalize(X0)
    for _ in range(nsteps):
        X = orthonormalize(imag_step(X, ell, V, E, dt))
    return X
