"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the transform: it only samples analytic
radial functions on the grid r_i = (i - 1/2) dr (the input layout of Sec. 2.2,
psi_i = psi(r_i) sqrt(dr)) and draws random numbers.  It imports nothing from
the library or the oracle.

Workloads (all inputs FP64 on the host, in channel order):

* ``gaussian_orbitals``  N = 256, rmax = 20, l = 0..7, psi = r^(l+1) exp(-a r^2),
  a ~ U[0.5, 2] drawn in l order (the Gaussian atomic orbitals of Sec. 3).
* ``batched_all_m``      N = 2048, rmax = 100, l = 0..63 with 2l+1 channels each
  (4096), each channel a sum of 4 terms c_j r^(l+1) exp(-a_j (r - r0_j)^2),
  a ~ U[0.05, 1], r0 ~ U[0, 50], c ~ N(0,1) + i N(0,1), each term scaled to
  unit norm on the grid (evaluated in log space).
* ``uneven``             512 channels, N ~ {512 .. 8192}, l ~ U{0..127}, rmax = 0.05 N,
  the same Gaussian sums with r0 ~ U[0, min(50, rmax/2)].
* ``tdse``               N = 4096, rmax = 200, l = 0..31 with all m (1024 channels):
  r exp(-r) in (0, 0) plus Gaussian sums of norm 1e-3 elsewhere, total norm 1;
  V = -1/sqrt(r^2 + 0.01) + l(l+1)/(2 r^2).
* ``adjoint``            N = 2048, rmax = 100, l = 0..15 with all m (256 channels),
  psi0 and V as in ``tdse``; 200 strengths s_t ~ U[0.9, 1.1], dt = 0.01, and a
  target phi with N(0,1) + i N(0,1) entries, norm 1 (loss |<phi|psi_T>|^2).
* ``hydrogen``           rmax = 102.4, N = rmax/dr (dr = 0.2, 0.1, 0.05 give 512, 1024,
  2048): two l = 1 channels and one l = 2 channel (the l > 0 states of the
  bound-state table of Sec. 4.3), V = -1/r, starting states either generic
  (r^(l+1) exp(-r/2), r^(l+2) exp(-r/3)) or the hydrogen functions r^2 exp(-r/2),
  r^2 (1 - r/6) exp(-r/3), r^3 exp(-r/3), each scaled to norm 1; the channel sets
  [0, 2, 3] group the two l = 1 states.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

__all__ = ["Workload", "gaussian_orbitals", "batched_all_m", "uneven", "tdse", "adjoint", "hydrogen", "grid",
           "gaussian_sum"]


@dataclass
class Workload:
    name: str
    channels: List[Tuple[int, int, float, int]]   # (N, l, rmax, offset)
    psi: np.ndarray                                # complex128, packed
    extra: dict = field(default_factory=dict)

    @property
    def elems(self) -> int:
        return max(off + N for N, _, _, off in self.channels)

    @property
    def points(self) -> int:
        return sum(N for N, _, _, _ in self.channels)


def grid(N: int, rmax: float) -> np.ndarray:
    return (np.arange(1, N + 1) - 0.5) * (rmax / N)


def gaussian_sum(rng, N: int, rmax: float, ell: int, r0_max: float, nterms: int = 4) -> np.ndarray:
    """sum_j c_j g_j with g_j = r^(l+1) exp(-a_j (r - r0_j)^2) / |g_j| on the grid."""
    r = grid(N, rmax)
    out = np.zeros(N, dtype=np.complex128)
    for _ in range(nterms):
        a = rng.uniform(0.05, 1.0)
        r0 = rng.uniform(0.0, r0_max)
        c = rng.standard_normal() + 1j * rng.standard_normal()
        lg = (ell + 1) * np.log(r) - a * (r - r0) ** 2
        g = np.exp(lg - lg.max())
        g /= np.linalg.norm(g)
        out += c * g
    return out


def _pack(chs):
    channels, parts, off = [], [], 0
    for N, ell, rmax, data in chs:
        channels.append((N, ell, rmax, off))
        parts.append(data)
        off += N
    return channels, np.concatenate(parts)


def gaussian_orbitals(seed: int = 1, N: int = 256, rmax: float = 20.0, lmax: int = 7) -> Workload:
    rng = np.random.default_rng(seed)
    r = grid(N, rmax)
    chs, aa = [], []
    for ell in range(lmax + 1):
        a = rng.uniform(0.5, 2.0)
        aa.append(a)
        chs.append((N, ell, rmax, (r ** (ell + 1) * np.exp(-a * r * r) * math.sqrt(rmax / N)).astype(np.complex128)))
    channels, psi = _pack(chs)
    return Workload("gaussian orbitals N=256 rmax=20 l=0..7 (FP64)", channels, psi, {"a": aa})


def batched_all_m(seed: int = 2, N: int = 2048, rmax: float = 100.0, lmax: int = 63,
                  ells=None) -> Workload:
    rng = np.random.default_rng(seed)
    chs = []
    for ell in (range(lmax + 1) if ells is None else ells):
        for _ in range(2 * ell + 1):
            chs.append((N, ell, rmax, gaussian_sum(rng, N, rmax, ell, 50.0)))
    channels, psi = _pack(chs)
    return Workload(f"batched all-m N={N} rmax={rmax} lmax={lmax} ({len(channels)} channels)", channels, psi)


def uneven(seed: int = 3, count: int = 512) -> Workload:
    rng = np.random.default_rng(seed)
    Ns = rng.choice([512, 1024, 2048, 4096, 8192], size=count)
    ells = rng.integers(0, 128, size=count)
    chs = []
    for N, ell in zip(Ns, ells):
        N, ell = int(N), int(ell)
        rmax = 0.05 * N
        chs.append((N, ell, rmax, gaussian_sum(rng, N, rmax, ell, min(50.0, rmax / 2))))
    channels, psi = _pack(chs)
    return Workload(f"uneven batch of {count} transforms, N in 512..8192, l in 0..127", channels, psi)


def tdse(seed: int = 4, N: int = 4096, rmax: float = 200.0, lmax: int = 31, dt: float = 0.01,
         small: float = 1e-3) -> Workload:
    rng = np.random.default_rng(seed)
    r = grid(N, rmax)
    chs, Vs = [], []
    for ell in range(lmax + 1):
        for m in range(2 * ell + 1):
            if ell == 0:
                d = (r * np.exp(-r) * math.sqrt(rmax / N)).astype(np.complex128)
                d /= np.linalg.norm(d)
            else:
                d = gaussian_sum(rng, N, rmax, ell, 50.0)
                d *= small / np.linalg.norm(d)
            chs.append((N, ell, rmax, d))
            Vs.append(-1.0 / np.sqrt(r * r + 0.01) + ell * (ell + 1) / (2.0 * r * r))
    channels, psi = _pack(chs)
    psi /= np.linalg.norm(psi)
    return Workload(f"split step N={N} rmax={rmax} lmax={lmax} ({len(channels)} channels)", channels, psi,
                    {"V": np.concatenate(Vs), "dt": dt})


def adjoint(seed: int = 5, N: int = 2048, rmax: float = 100.0, lmax: int = 15, nsteps: int = 200,
            dt: float = 0.01) -> Workload:
    w = tdse(seed=seed, N=N, rmax=rmax, lmax=lmax, dt=dt)
    rng = np.random.default_rng(seed + 1000)
    s = rng.uniform(0.9, 1.1, nsteps)
    phi = rng.standard_normal(w.elems) + 1j * rng.standard_normal(w.elems)
    phi /= np.linalg.norm(phi)
    w.name = f"adjoint N={N} rmax={rmax} lmax={lmax} ({len(w.channels)} channels, {nsteps} steps)"
    w.extra.update({"s": s, "phi": phi})
    return w


def hydrogen(dr: float = 0.2, rmax: float = 102.4, start: str = "generic") -> Workload:
    N = int(round(rmax / dr))
    r = grid(N, rmax)
    if start == "generic":
        funcs = [(1, r ** 2 * np.exp(-r / 2)), (1, r ** 3 * np.exp(-r / 3)), (2, r ** 3 * np.exp(-r / 2))]
    elif start == "hydrogen":
        funcs = [(1, r ** 2 * np.exp(-r / 2)), (1, r ** 2 * (1 - r / 6) * np.exp(-r / 3)), (2, r ** 3 * np.exp(-r / 3))]
    else:
        raise ValueError(start)
    chs = [(N, ell, rmax, (f / np.linalg.norm(f)).astype(np.complex128)) for ell, f in funcs]
    channels, psi = _pack(chs)
    V = np.concatenate([-1.0 / r] * len(chs))
    return Workload(f"hydrogen l>0 states dr={dr} rmax={rmax} ({start} start)", channels, psi,
                    {"V": V, "sets": [0, 2, 3], "states": [(1, 0), (1, 1), (2, 0)]})
