"""MI355X orthogonal discrete spherical Bessel transform (Serov, arXiv 1509.07115).

A thin Python binding over the C ABI of ``libdsbt.so`` (include/dsbt.h):
PyTorch supplies device memory and streams; every step of the transform runs
in the library's HIP kernels.  There is no CPU fallback: if the library is not
built, or no GPU is present, the calls raise.

    from paper_1509_07115_amd import Plan
    plan = Plan.uniform(N=2048, rmax=100.0, ells=range(64), all_m=True)
    b = plan.forward(psi)          # psi: torch.complex64 on cuda, plan.elems elements
    psi2 = plan.inverse(b)
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional, Sequence

import numpy as np

from . import _lib

__all__ = ["Plan", "AngularTransform", "DsbtError", "exported_symbols"]

DsbtError = _lib.DsbtError


def exported_symbols() -> list:
    return list(_lib.EXPORTED)


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """A DSBT plan over a set of radial channels (``dsbt_plan_create``).

    channels: sequence of (N, ell, rmax, offset) tuples (offset in complex elements).
    precision: "c64" (complex64 data, FP32 arithmetic), "c128", or "c64x"
    (complex64 data, FP64 arithmetic and tables).
    mode: "batched" (default) or "plain" (one launch per channel and stage).
    plan_where: "device" (default, FP64 plan kernels on the GPU) or "host".
    kinetic: "plain" (k_n = n dk) or "corrected" (roots of eq. kcorr) momenta of the step.
    algorithm: "tiled" (default, the stable tiled moment form) or "monomial" (the paper's own
        monomial-moment fast multiplication of Sec. 2.6, FP64, complex128 plans only).
    check_finite: scan transform and step inputs for NaN / infinities (``DSBT_ERR_NONFINITE``;
        checked calls synchronise).
    allocator: None (the library's hipMalloc), "torch" (PyTorch's caching allocator on the
        current device and stream), or a pair (alloc(nbytes) -> int pointer or 0, free(ptr)) of
        Python callables, passed as the plan's ``dev_alloc`` / ``dev_free``.
    """

    def __init__(self, channels: Sequence, precision: str = "c64", mode: str = "batched", tile: int = 0,
                 chans_per_block: int = 0, sign: bool = True, plan_where: str = "device", kinetic: str = "plain",
                 algorithm: str = "tiled", check_finite: bool = False, allocator=None, stream=None, _create=True):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        self.precision = precision
        self.channels = [tuple(c) for c in channels]
        if not _create:
            return
        arr = (_lib.Channel * len(self.channels))()
        for i, (N, ell, rmax, off) in enumerate(self.channels):
            arr[i] = _lib.Channel(int(N), int(ell), float(rmax), int(off))
        opts = self._opts(precision, mode, tile, chans_per_block, sign, plan_where, kinetic, algorithm)
        opts.check_finite = 1 if check_finite else 0
        self._alloc_cbs = self._allocator(allocator, stream)
        if self._alloc_cbs is not None:
            opts.dev_alloc, opts.dev_free = self._alloc_cbs
        _lib.check(self._lib.dsbt_plan_create(ctypes.byref(self._h), arr, len(self.channels), ctypes.byref(opts),
                                              _stream_handle(stream)), "dsbt_plan_create")
        self._info()

    @staticmethod
    def _allocator(allocator, stream):
        """ctypes callbacks for dsbt_plan_opts.dev_alloc / dev_free (kept alive by the plan)."""
        if allocator is None:
            return None
        if allocator == "torch":
            import torch
            dev = torch.cuda.current_device()
            st = torch.cuda.current_stream() if stream is None else stream

            def alloc(nbytes):
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=st)

            def free(ptr):
                torch.cuda.caching_allocator_delete(ptr)
        else:
            alloc, free = allocator

        def c_alloc(nbytes, _ctx):
            try:
                return int(alloc(nbytes)) or None
            except Exception:   # reported to the library as a failed allocation (DSBT_ERR_OOM)
                return None

        def c_free(ptr, _ctx):
            if ptr:
                free(int(ptr))
        return _lib.ALLOC_FN(c_alloc), _lib.FREE_FN(c_free)

    @staticmethod
    def _opts(precision, mode, tile, chans_per_block, sign, plan_where="device", kinetic="plain", algorithm="tiled"):
        o = _lib.PlanOpts()
        o.precision = {"c64": _lib.DSBT_C64, "c128": _lib.DSBT_C128, "c64x": _lib.DSBT_C64_FP64}[precision]
        o.mode = {"batched": _lib.DSBT_MODE_BATCHED, "plain": _lib.DSBT_MODE_PLAIN}[mode]
        o.tile = int(tile)
        o.chans_per_block = int(chans_per_block)
        o.sign = _lib.DSBT_SIGN_C if sign else _lib.DSBT_SIGN_PRINTED_F
        o.plan_where = {"device": _lib.DSBT_PLAN_ON_DEVICE, "host": _lib.DSBT_PLAN_ON_HOST}[plan_where]
        o.kinetic = {"plain": _lib.DSBT_K_PLAIN, "corrected": _lib.DSBT_K_CORRECTED}[kinetic]
        o.algorithm = {"tiled": _lib.DSBT_ALG_TILED, "monomial": _lib.DSBT_ALG_MONOMIAL}[algorithm]
        return o

    @classmethod
    def autotuned(cls, channels: Sequence, nrep: int = 10, cache: Optional[str] = None, stream=None, **kw) -> "Plan":
        """A plan with the tile and channels per work item chosen by measurement (``dsbt_autotune``);
        ``cache``: JSON-lines file of earlier results.  The choice is in ``plan.tuning``."""
        lib = _lib.load()
        chans = [tuple(c) for c in channels]
        arr = (_lib.Channel * len(chans))()
        for i, (N, ell, rmax, off) in enumerate(chans):
            arr[i] = _lib.Channel(int(N), int(ell), float(rmax), int(off))
        opts = cls._opts(kw.get("precision", "c64"), kw.get("mode", "batched"), 0, 0, kw.get("sign", True),
                         kw.get("plan_where", "device"), kw.get("kinetic", "plain"), kw.get("algorithm", "tiled"))
        best = _lib.PlanOpts()
        ms = ctypes.c_double()
        _lib.check(lib.dsbt_autotune(arr, len(chans), ctypes.byref(opts), int(nrep),
                                     cache.encode() if cache else None, ctypes.byref(best), ctypes.byref(ms),
                                     _stream_handle(stream)), "dsbt_autotune")
        kw = dict(kw)
        kw["tile"], kw["chans_per_block"] = best.tile, best.chans_per_block
        plan = cls(chans, stream=stream, **kw)
        plan.tuning = {"tile": best.tile, "chans_per_block": best.chans_per_block, "ms_per_fwd_inv": ms.value}
        return plan

    @classmethod
    def uniform(cls, N: int, rmax: float, ells: Iterable[int], all_m: bool = False, **kw) -> "Plan":
        ells = [int(e) for e in ells]
        ch, off = [], 0
        for e in ells:
            for _ in range(2 * e + 1 if all_m else 1):
                ch.append((N, e, rmax, off))
                off += N
        return cls(ch, **kw)

    def _info(self):
        nch, elems, prec, tb = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _lib.check(self._lib.dsbt_plan_info(self._h, ctypes.byref(nch), ctypes.byref(elems), ctypes.byref(prec),
                                            ctypes.byref(tb)), "dsbt_plan_info")
        self.nch, self.elems, self.table_bytes = nch.value, elems.value, tb.value

    # -- buffers ---------------------------------------------------------
    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.precision == "c128" else torch.complex64

    def _check_buf(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}, got {t.dtype}")
        if not t.is_contiguous() or t.numel() < self.elems:
            raise ValueError(f"{name} must be contiguous with at least {self.elems} elements")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self):
        import torch
        return torch.empty(self.elems, dtype=self.dtype, device="cuda")

    # -- transforms ------------------------------------------------------
    def forward(self, psi, out=None, stream=None):
        """b = T F psi for every channel (``dsbt_forward``)."""
        out = self.empty() if out is None else out
        _lib.check(self._lib.dsbt_forward(self._h, self._check_buf(psi, "psi"), self._check_buf(out, "out"),
                                          _stream_handle(stream)), "dsbt_forward")
        return out

    def inverse(self, b, out=None, stream=None):
        """psi = F^T T^T b for every channel (``dsbt_inverse``)."""
        out = self.empty() if out is None else out
        _lib.check(self._lib.dsbt_inverse(self._h, self._check_buf(b, "b"), self._check_buf(out, "out"),
                                          _stream_handle(stream)), "dsbt_inverse")
        return out

    def set_potential(self, V: np.ndarray, dt: float, imaginary: bool = False):
        """Radial potential in data layout (FP64 host array) and time step (``dsbt_set_potential_ex``);
        ``imaginary``: real decay factors exp(-V tau/2), exp(-K tau) (imaginary-time method)."""
        V = np.ascontiguousarray(V, dtype=np.float64)
        if V.size < self.elems:
            raise ValueError("potential shorter than the data layout")
        flags = _lib.DSBT_TIME_IMAGINARY if imaginary else 0
        _lib.check(self._lib.dsbt_set_potential_ex(self._h, V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                   float(dt), flags), "dsbt_set_potential_ex")

    def energy(self, psi, work=None, out=None, stream=None):
        """Per-channel energy terms (``dsbt_energy``): cuda float64 tensor (nch, 3) holding
        <psi|psi>, <psi|V|psi>, <psi|K|psi>; work receives b = T F psi."""
        import torch
        work = self.empty() if work is None else work
        if out is None:
            out = torch.empty((len(self.channels), 3), dtype=torch.float64, device="cuda")
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                and out.numel() >= 3 * len(self.channels)):
            raise TypeError("out must be a contiguous cuda float64 tensor with 3 values per channel")
        _lib.check(self._lib.dsbt_energy(self._h, self._check_buf(psi, "psi"), self._check_buf(work, "work"),
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "dsbt_energy")
        return out

    def orthonormalize(self, psi, sets: Sequence[int], stream=None):
        """Gram-Schmidt within channel sets [sets[k], sets[k+1]) in place (``dsbt_orthonormalize``)."""
        key = tuple(int(x) for x in sets)
        if getattr(self, "_sets_key", None) != key:    # marshal a set table once, not per call
            self._sets_arr = (ctypes.c_int32 * len(key))(*key)
            self._sets_key = key
        _lib.check(self._lib.dsbt_orthonormalize(self._h, self._check_buf(psi, "psi"), self._sets_arr, len(key) - 1,
                                                 _stream_handle(stream)), "dsbt_orthonormalize")
        return psi

    def kinetic_step(self, psi, nsteps: int = 1, s=None, adjoint: bool = False, graph: bool = False,
                     resident: bool = False, stream=None):
        """nsteps split-operator steps in place (``dsbt_kinetic_step``); s: cuda float32 strengths."""
        import torch
        sp = None
        if s is not None:
            if not (isinstance(s, torch.Tensor) and s.is_cuda and s.dtype == torch.float32 and s.is_contiguous()
                    and s.numel() >= nsteps):
                raise TypeError("s must be a contiguous cuda float32 tensor with nsteps entries")
            sp = ctypes.c_void_p(s.data_ptr())
        flags = ((_lib.DSBT_STEP_ADJOINT if adjoint else 0) | (_lib.DSBT_STEP_GRAPH if graph else 0)
                 | (_lib.DSBT_STEP_RESIDENT if resident else 0))
        _lib.check(self._lib.dsbt_kinetic_step(self._h, self._check_buf(psi, "psi"), int(nsteps), sp, flags,
                                               _stream_handle(stream)), "dsbt_kinetic_step")
        return psi

    def step_grad_s(self, psi_t, psi_t1, lam_t, lam_t1, out, stream=None):
        """out[0] = (tau/2) sum V Im(conj(lam_t1) psi_t1 + conj(lam_t) psi_t) (``dsbt_step_grad_s``)."""
        import torch
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.numel() >= 1):
            raise TypeError("out must be a cuda float64 tensor")
        _lib.check(self._lib.dsbt_step_grad_s(self._h, self._check_buf(psi_t, "psi_t"),
                                              self._check_buf(psi_t1, "psi_t1"), self._check_buf(lam_t, "lam_t"),
                                              self._check_buf(lam_t1, "lam_t1"), ctypes.c_void_p(out.data_ptr()),
                                              _stream_handle(stream)), "dsbt_step_grad_s")
        return out

    def adjoint_segment(self, psi_a, nsteps: int, s, lam, gs, graph: bool = False, stream=None):
        """Backward pass of one checkpoint segment (``dsbt_adjoint_segment``): lam_{a+n} -> lam_a in
        place in lam, gs[t-a] = dL/ds_t; psi_a is the state before the segment; s and gs: cuda float32 and
        float64 tensors of nsteps values."""
        import torch
        if not (isinstance(s, torch.Tensor) and s.is_cuda and s.dtype == torch.float32 and s.is_contiguous()
                and s.numel() >= nsteps):
            raise TypeError("s must be a contiguous cuda float32 tensor with nsteps entries")
        if not (isinstance(gs, torch.Tensor) and gs.is_cuda and gs.dtype == torch.float64 and gs.is_contiguous()
                and gs.numel() >= nsteps):
            raise TypeError("gs must be a contiguous cuda float64 tensor with nsteps entries")
        _lib.check(self._lib.dsbt_adjoint_segment(self._h, self._check_buf(psi_a, "psi_a"), int(nsteps),
                                                  ctypes.c_void_p(s.data_ptr()), self._check_buf(lam, "lam"),
                                                  ctypes.c_void_p(gs.data_ptr()),
                                                  _lib.DSBT_STEP_GRAPH if graph else 0, _stream_handle(stream)),
                   "dsbt_adjoint_segment")
        return lam

    def profile(self, enable: bool = True, clear: bool = True):
        """Start or stop per-stage HIP-event timing (``dsbt_profile_enable``);
        ``clear=False`` resumes without clearing what was recorded."""
        mode = (1 if clear else 2) if enable else 0
        _lib.check(self._lib.dsbt_profile_enable(self._h, mode), "dsbt_profile_enable")

    def profile_read(self) -> dict:
        """{stage: (milliseconds summed, launches)} for "sincos" and "moment" (``dsbt_profile_read``)."""
        ms = (ctypes.c_double * 2)()
        n = (ctypes.c_int64 * 2)()
        _lib.check(self._lib.dsbt_profile_read(self._h, ms, n, 2), "dsbt_profile_read")
        return {"sincos": (ms[0], n[0]), "moment": (ms[1], n[1])}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dsbt_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_ftb_tables(N: int, ell: int, B: int) -> np.ndarray:
    """FP64 moment-tile blocks of the plan (``dsbt_host_ftb_tables``), shape (N/B, R, R)."""
    lib = _lib.load()
    need = ctypes.c_int64()
    _lib.check(lib.dsbt_host_ftb_tables(N, ell, B, None, 0, ctypes.byref(need)), "dsbt_host_ftb_tables")
    out = np.empty(need.value, dtype=np.float64)
    _lib.check(lib.dsbt_host_ftb_tables(N, ell, B, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        need.value, ctypes.byref(need)), "dsbt_host_ftb_tables")
    k = (ell + 1) // 2
    R = B + k
    return out.reshape(N // B, R, R)


class AngularTransform:
    """The angular transform Y = P Phi of Sec. 4.1 at every radial point (``dsbt_sht_*``).

    grid  [j][k][i]: Gauss-Legendre node eta_j (ascending), azimuth phi_k, radial point i;
    coef  [q][t][i]: m = q - M, l = |m| + t (N_phi = 2M + 1), i.e. channel q*N_theta + t of a
    DSBT plan built from ``channels(rmax)``.
    """

    def __init__(self, Nr: int, n_theta: int, n_phi: int, precision: str = "c64"):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        self.Nr, self.n_theta, self.n_phi, self.precision = int(Nr), int(n_theta), int(n_phi), precision
        prec = {"c64": _lib.DSBT_C64, "c128": _lib.DSBT_C128}[precision]
        _lib.check(self._lib.dsbt_sht_create(ctypes.byref(self._h), self.Nr, self.n_theta, self.n_phi, prec),
                   "dsbt_sht_create")

    @property
    def size(self) -> int:
        return self.Nr * self.n_theta * self.n_phi

    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.precision == "c128" else torch.complex64

    def lm(self):
        """[(l, m)] per coefficient channel, in channel order."""
        M = (self.n_phi - 1) // 2
        return [(abs(q - M) + t, q - M) for q in range(self.n_phi) for t in range(self.n_theta)]

    def channels(self, rmax: float):
        """DSBT channels (Nr, l, rmax, offset) of the coefficient layout."""
        return [(self.Nr, l, float(rmax), c * self.Nr) for c, (l, _) in enumerate(self.lm())]

    def _buf(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.dtype:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor of {self.dtype}")
        if not t.is_contiguous() or t.numel() < self.size:
            raise ValueError(f"{name} must be contiguous with at least {self.size} elements")
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, grid, out=None, stream=None):
        import torch
        out = torch.empty(self.size, dtype=self.dtype, device="cuda") if out is None else out
        _lib.check(self._lib.dsbt_sht_forward(self._h, self._buf(grid, "grid"), self._buf(out, "out"),
                                              _stream_handle(stream)), "dsbt_sht_forward")
        return out

    def inverse(self, coef, out=None, stream=None):
        import torch
        out = torch.empty(self.size, dtype=self.dtype, device="cuda") if out is None else out
        _lib.check(self._lib.dsbt_sht_inverse(self._h, self._buf(coef, "coef"), self._buf(out, "out"),
                                              _stream_handle(stream)), "dsbt_sht_inverse")
        return out

    def potential_phase(self, grid, V0=None, V1=None, F: float = 0.0, dt: float = 0.0, stream=None):
        """grid *= exp(-i (V0 + F V1) dt/2) in place (``dsbt_sht_potential_phase``);
        V0, V1: cuda float64 tensors in grid layout, or None."""
        import torch

        def ptr(v, name):
            if v is None:
                return None
            if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
                    and v.numel() >= self.size):
                raise TypeError(f"{name} must be a contiguous cuda float64 tensor of the grid size")
            return ctypes.c_void_p(v.data_ptr())
        _lib.check(self._lib.dsbt_sht_potential_phase(self._h, self._buf(grid, "grid"), ptr(V0, "V0"), ptr(V1, "V1"),
                                                      float(F), float(dt), _stream_handle(stream)),
                   "dsbt_sht_potential_phase")
        return grid

    def momentum_order(self, src, dst=None, inverse: bool = False, stream=None):
        """Channels <-> the unified momentum order with i^-l / i^l (``dsbt_sht_momentum_order``)."""
        import torch
        dst = torch.empty(self.size, dtype=self.dtype, device="cuda") if dst is None else dst
        _lib.check(self._lib.dsbt_sht_momentum_order(self._h, self._buf(src, "src"), self._buf(dst, "dst"),
                                                     1 if inverse else 0, _stream_handle(stream)),
                   "dsbt_sht_momentum_order")
        return dst

    def kinetic(self, rmax: float, kinetic: str = "plain", stream=None):
        """K_n = k_n^2/2 per channel slot (cuda float64, coefficient layout; ``dsbt_sht_kinetic``)."""
        import torch
        out = torch.empty(self.size, dtype=torch.float64, device="cuda")
        kin = {"plain": _lib.DSBT_K_PLAIN, "corrected": _lib.DSBT_K_CORRECTED}[kinetic]
        _lib.check(self._lib.dsbt_sht_kinetic(self._h, float(rmax), kin, ctypes.c_void_p(out.data_ptr()),
                                              _stream_handle(stream)), "dsbt_sht_kinetic")
        return out

    def momentum_pz(self, rmax: float, stream=None):
        """-2 k~_n eta_j on the momentum grid [j][k][n] (cuda float64; ``dsbt_sht_momentum_pz``): with it
        as V1 and F = A, ``potential_phase`` multiplies by exp(i A k~_n eta_j dt)."""
        import torch
        out = torch.empty(self.size, dtype=torch.float64, device="cuda")
        _lib.check(self._lib.dsbt_sht_momentum_pz(self._h, float(rmax), ctypes.c_void_p(out.data_ptr()),
                                                  _stream_handle(stream)), "dsbt_sht_momentum_pz")
        return out

    def close(self):
        if self._h:
            self._lib.dsbt_sht_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f64_ptr(v, n, name):
    import torch
    if v is None:
        return None
    if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
            and v.numel() >= n):
        raise TypeError(f"{name} must be a contiguous cuda float64 tensor of the grid size")
    return ctypes.c_void_p(v.data_ptr())


def step3d(Y: "AngularTransform", plan: "Plan", grid, V0, V1, F: float, dt: float, coef=None, stream=None):
    """One 3D split step in the coordinate gauge (Sec. 4.1) in place on ``grid`` (``dsbt_step3d``):
    exp(-i U dt/2) Y^H B^T exp(-i K dt) B Y exp(-i U dt/2), U = V0 + F V1.  ``plan`` is a
    Plan over ``Y.channels(rmax)`` whose potential was set to zero with the same dt."""
    import torch
    coef = torch.empty_like(grid) if coef is None else coef
    _lib.check(Y._lib.dsbt_step3d(Y._h, plan._h, Y._buf(grid, "grid"), Y._buf(coef, "coef"),
                                  _f64_ptr(V0, Y.size, "V0"), _f64_ptr(V1, Y.size, "V1"), float(F), float(dt),
                                  _stream_handle(stream)), "dsbt_step3d")
    return grid


def step3d_velocity(Y: "AngularTransform", plan: "Plan", grid, V0, K, Pz, A: float, dt: float, w1=None, w2=None,
                    stream=None):
    """One 3D split step in the velocity gauge (Sec. 4.1, the printed sequence) in place on ``grid``
    (``dsbt_step3d_velocity``).  K = ``Y.kinetic(rmax)``, Pz = ``Y.momentum_pz(rmax)``, ``plan`` a Plan
    over ``Y.channels(rmax)``; w1, w2: optional work buffers of Y's size."""
    import torch
    w1 = torch.empty_like(grid) if w1 is None else w1
    w2 = torch.empty_like(grid) if w2 is None else w2
    _lib.check(Y._lib.dsbt_step3d_velocity(Y._h, plan._h, Y._buf(grid, "grid"), Y._buf(w1, "w1"), Y._buf(w2, "w2"),
                                           _f64_ptr(V0, Y.size, "V0"), _f64_ptr(K, Y.size, "K"),
                                           _f64_ptr(Pz, Y.size, "Pz"), float(A), float(dt), _stream_handle(stream)),
               "dsbt_step3d_velocity")
    return grid


def sht_grid(n_theta: int, n_phi: int):
    """(eta, w, phi) of the angular grid (``dsbt_sht_grid``)."""
    lib = _lib.load()
    eta, w, phi = np.zeros(n_theta), np.zeros(n_theta), np.zeros(n_phi)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _lib.check(lib.dsbt_sht_grid(n_theta, n_phi, dp(eta), dp(w), dp(phi)), "dsbt_sht_grid")
    return eta, w, phi


def sht_host_tables(n_theta: int, n_phi: int) -> np.ndarray:
    """P[q, t, j] of the angular transform (``dsbt_sht_host_tables``)."""
    lib = _lib.load()
    out = np.zeros((n_phi, n_theta, n_theta))
    _lib.check(lib.dsbt_sht_host_tables(n_theta, n_phi, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "dsbt_sht_host_tables")
    return out


def host_monomial_tables(N: int, ell: int):
    """(xi, alpha, comp) of the monomial variant for one (N, l) (``dsbt_host_monomial_tables``)."""
    lib = _lib.load()
    sz = (ctypes.c_int64 * 3)()
    _lib.check(lib.dsbt_host_monomial_tables(N, ell, None, None, None, sz), "dsbt_host_monomial_tables")
    out = [np.zeros(max(int(n), 1)) for n in sz]
    ptr = [o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for o in out]
    _lib.check(lib.dsbt_host_monomial_tables(N, ell, *ptr, sz), "dsbt_host_monomial_tables")
    return tuple(o[: int(n)] for o, n in zip(out, sz))


def device_ftb_tables(N: int, ell: int, B: int, stream=None) -> np.ndarray:
    """The same blocks from the FP64 GPU plan generator (``dsbt_device_ftb_tables``)."""
    lib = _lib.load()
    need = ctypes.c_int64()
    _lib.check(lib.dsbt_device_ftb_tables(N, ell, B, None, 0, ctypes.byref(need), None), "dsbt_device_ftb_tables")
    out = np.empty(need.value, dtype=np.float64)
    _lib.check(lib.dsbt_device_ftb_tables(N, ell, B, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          need.value, ctypes.byref(need), _stream_handle(stream)),
               "dsbt_device_ftb_tables")
    k = (ell + 1) // 2
    R = B + k
    return out.reshape(N // B, R, R)


def kinetic_momenta(N: int, ell: int, rmax: float, kinetic: str = "plain") -> np.ndarray:
    """Momenta of the kinetic diagonal in slot order (``dsbt_kinetic_momenta``), host FP64."""
    lib = _lib.load()
    out = np.empty(N, dtype=np.float64)
    kin = {"plain": _lib.DSBT_K_PLAIN, "corrected": _lib.DSBT_K_CORRECTED}[kinetic]
    _lib.check(lib.dsbt_kinetic_momenta(N, ell, float(rmax), kin, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "dsbt_kinetic_momenta")
    return out
