"""Benchmark: batched complex64 DSBT forward + inverse on one MI355X.

Workload: N = 2048 radial points, rmax = 100, l = 0..63 with all 2l+1 m
channels (4096 channels, 8.4 M radial points), each channel a seeded sum of four
Gaussians r^(l+1) exp(-a (r - r0)^2) with complex amplitudes (synthetic data).
One step = one forward transform and one inverse transform of the whole batch,
inputs resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "mfma_fp32_TFLOPs": 157.3}
PROFILE_EVERY = 10   # steps of the timed region whose stage launches carry HIP events

# HBM traffic of one moment-stage launch (forward and inverse averaged) on this
# workload, from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of this
# script, each scaled by what the same counter reads for a device copy of known
# size (--copy-calibration).  The record holds the SHA-256 of the kernel's
# sources and of the host code that builds and schedules its work items at the
# time of the measurement; after any change to them the figure no longer
# applies and the roofline reports traffic as null.
MOMENT_TRAFFIC = {"sources": ["paper_1509_07115_amd/csrc/mstage_chain.hip", "paper_1509_07115_amd/csrc/kernels.h",
                              "paper_1509_07115_amd/csrc/capi.cpp"],
                  "sha256": "1c669beaf6aa8ff7bbb6fe284e792422aecaf6657f1f03e6c87fd52ea51efca4",
                  "fetch_bytes": 147867056, "write_bytes": 67482496}


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def algorithmic_counts(channels):
    """Per launch of each stage, from the operation model of the method.

    Points: sum of N.  Flops per point: 5 log2 N + 8 for the sine/cosine stage
    (an N-point complex FFT plus the pre/post steps), 12 ceil(l/2) for the
    moment stage (a complex x real update, contraction and completion row per
    moment).  Bytes: 16 per point for each stage (complex64 in and out) plus
    the tables once per launch: for the moment stage the minimal state
    ceil(l/2) + 1 FP32 words per row for each distinct l (up to its largest N)
    and ceil(l/2) N words of completion rows per distinct (l, N); for the
    sine/cosine stage two complex64 tables of N entries per distinct N.
    """
    pts = sum(N for N, _, _, _ in channels)
    f_sincos = sum(N * (5 * math.log2(N) + 8) for N, _, _, _ in channels)
    f_moment = sum(N * 12 * ((l + 1) // 2) for N, l, _, _ in channels)
    maxn_l, pairs, ns = {}, set(), set()
    for N, l, _, _ in channels:
        maxn_l[l] = max(maxn_l.get(l, 0), N)
        pairs.add((N, l))
        ns.add(N)
    tab_m = 4 * (sum(((l + 1) // 2 + 1) * n for l, n in maxn_l.items()) + sum(((l + 1) // 2) * N for N, l in pairs))
    tab_f = sum(2 * 8 * N for N in ns)
    return {"points": pts, "flops_sincos": f_sincos, "flops_moment": f_moment,
            "bytes_sincos": 16.0 * pts + tab_f, "bytes_moment": 16.0 * pts + tab_m}


def roofline(kind, flops, nbytes, avg_ms, traffic):
    """The binding roofline of a kernel (the larger time at peak) and the
    achieved rate on it from the live average launch time."""
    t_hbm = nbytes / (PEAK["hbm_GBps"] * 1e9)
    t_mfma = flops / (PEAK["mfma_fp32_TFLOPs"] * 1e12)
    s = avg_ms * 1e-3
    if t_hbm >= t_mfma:
        a = nbytes / s / 1e9
        r = {"bound": "hbm", "achieved": a, "peak": PEAK["hbm_GBps"], "unit": "GB/s", "frac": a / PEAK["hbm_GBps"]}
    else:
        a = flops / s / 1e12
        r = {"bound": "mfma", "achieved": a, "peak": PEAK["mfma_fp32_TFLOPs"], "unit": "TFLOP/s",
             "frac": a / PEAK["mfma_fp32_TFLOPs"]}
    r.update({"traffic": traffic, "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
              "kernel": kind, "avg_launch_ms": avg_ms, "algorithmic_bytes": nbytes, "algorithmic_flops": flops,
              "mfma_TFLOPs_algorithmic": flops / s / 1e12, "hbm_GBps_algorithmic": nbytes / s / 1e9,
              "time_at_peak_ms": {"hbm": t_hbm * 1e3, "mfma": t_mfma * 1e3}})
    return r


def cpu_baseline(w, b_gpu=None, reps=300):
    """The CPU-baseline leg: time the FP64 oracle (dense F and T) on whole l groups of the
    workload and, given the GPU forward result b_gpu (complex128 host array), its largest
    per-channel relative error against the oracle on the groups l = 1, 32, 63.
    Returns (baseline record, error or None)."""
    import numpy as np
    from oracle import dsbt as odsbt
    worst = None
    if b_gpu is not None:
        worst = 0.0
        for N_, l, _, off in w.channels:
            if l in (1, 32, 63):
                ref = odsbt.forward(w.psi[off:off + N_], l)
                worst = max(worst, float(np.linalg.norm(b_gpu[off:off + N_] - ref) / np.linalg.norm(ref)))
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    groups = {}
    for N, l, _, off in w.channels:
        groups.setdefault(l, []).append(off)
    N = w.channels[0][0]
    sample_ells = (63, 47, 31, 15, 62, 46, 30, 14)
    blocks = {}
    for l in sample_ells:
        blocks[l] = np.stack([w.psi[o:o + N] for o in groups[l]], axis=1)
        odsbt.forward(blocks[l][:, :1], l)     # builds and caches F and T (plan time, not timed)
    pts = sum(N * blocks[l].shape[1] for l in sample_ells) * reps
    t = time.perf_counter()
    for _ in range(reps):
        for l in sample_ells:
            odsbt.inverse(odsbt.forward(blocks[l], l), l)
    spent = time.perf_counter() - t
    return ({"value": pts / spent, "unit": "radial points/s", "cores": cores, "kind": "oracle",
             "sample": f"dense FP64 oracle forward+inverse, {reps} passes over the l groups {list(sample_ells)} "
                       f"with all m ({pts // reps} points per pass, N={N}), {spent:.1f} s; matrix build excluded"},
            worst)


def _timed(fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def other_workloads(progress):
    """The uneven batch, the 1000-step split-operator propagation and the adjoint
    pass (synthetic seeded inputs of the same shapes), timed on the GPU."""
    import time as _t
    import numpy as np
    import torch
    from paper_1509_07115_amd import Plan, workloads
    from paper_1509_07115_amd.autograd import propagate
    res = {}
    # uneven batch: 512 transforms, N in 512..8192, l in 0..127, rmax = 0.05 N
    progress("uneven batch")
    w = workloads.uneven()
    t = _t.perf_counter()
    plan = Plan(w.channels)
    t_plan = _t.perf_counter() - t
    x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
    b, y = plan.empty(), plan.empty()
    step = lambda: (plan.forward(x, b), plan.inverse(b, y))
    step()
    ms = _timed(step, 10)
    rt = float(max(torch.linalg.vector_norm(y[o:o + N] - x[o:o + N]).item() / torch.linalg.vector_norm(x[o:o + N]).item()
                   for N, _, _, o in w.channels))
    res["uneven_batch"] = {"workload": w.name, "points": w.points, "ms_per_fwd_inv": ms,
                           "points_per_s": w.points / (ms * 1e-3), "transforms_per_s": len(w.channels) / (ms * 1e-3),
                           "plan_s_fp64_on_gpu": t_plan, "roundtrip_max_rel": rt}
    del plan, x, b, y
    # split-operator propagation: 1000 steps from a captured graph
    progress("1000-step split-operator propagation")
    w = workloads.tdse()
    for prec in ("c64", "c64x"):
        plan = Plan(w.channels, precision=prec)
        plan.set_potential(w.extra["V"], w.extra["dt"])
        x0 = torch.from_numpy(w.psi).to(torch.complex64).cuda()
        x = x0.clone()
        plan.kinetic_step(x, 1000, graph=True)      # captures, runs once
        x.copy_(x0)
        ms = _timed(lambda: plan.kinetic_step(x, 1000, graph=True), 1)
        n2 = float(torch.sum(torch.abs(x.to(torch.complex128)) ** 2).item())
        res[f"tdse_1000_steps_{prec}"] = {"workload": w.name, "ms_per_1000_steps": ms, "norm_drift": abs(n2 - 1.0)}
        del plan
    # adjoint through 200 steps, checkpoints every 20, against the plain per-channel form
    progress("adjoint pass")
    w = workloads.adjoint()
    plan = Plan(w.channels)
    plan.set_potential(w.extra["V"], w.extra["dt"])
    phi = torch.from_numpy(w.extra["phi"]).to(torch.complex64).cuda()
    s = torch.from_numpy(w.extra["s"]).to(torch.float32).cuda()

    def grad_pass(pl):
        p0 = torch.from_numpy(w.psi).to(torch.complex64).cuda().requires_grad_(True)
        st = s.clone().requires_grad_(True)
        z = torch.vdot(phi, propagate(pl, p0, st, checkpoint_every=20, graph=True))
        ((z * z.conj()).real).backward()
    grad_pass(plan)
    ms = _timed(lambda: grad_pass(plan), 2)
    pplan = Plan(w.channels, mode="plain")
    pplan.set_potential(w.extra["V"], w.extra["dt"])
    xp = torch.from_numpy(w.psi).to(torch.complex64).cuda()
    ms_plain_20 = _timed(lambda: pplan.kinetic_step(xp, 20), 1)
    ms_batched_20 = _timed(lambda: plan.kinetic_step(xp, 20), 3)
    res["adjoint_200_steps"] = {"workload": w.name, "ms_per_loss_and_gradient": ms,
                                "ms_per_step_batched": ms_batched_20 / 20, "ms_per_step_plain_form": ms_plain_20 / 20}
    return res


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # defaults: the headline run times 200 steps after 2000 untimed ones (about
    # 0.4 s: the first ~10 ms of a burst run ~7% slower than the sustained
    # rate, while clock and power state ramp up); the single-workload modes
    # below default to 50 and 5
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (uneven batch, 1000-step TDSE, adjoint)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run device copies of 256 MiB (for scaling memory counters)")
    ap.add_argument("--split-step-profile", action="store_true",
                    help="only run --steps split steps of the 1000-step TDSE workload per precision "
                         "(c64, c64x), launched one by one, for a kernel trace")
    ap.add_argument("--imag-time-profile", action="store_true",
                    help="only time the imaginary-time method: the hydrogen l > 0 states (dr = 0.05, "
                         "10 --steps steps per graph replay, then Gram-Schmidt) in c64 and c128, and the "
                         "energy and orthonormalisation calls on the 1024-channel TDSE batch")
    ap.add_argument("--monomial-profile", action="store_true",
                    help="only time the paper-literal monomial moment stage against the tiled one (complex128, "
                         "N = 1024, l = 0..31 with all m) and report its error per l")
    ap.add_argument("--autotune-profile", action="store_true",
                    help="only run the autotuner on the batched all-m and the uneven workloads and compare the "
                         "tuned plan with the default one")
    ap.add_argument("--angular-profile", action="store_true",
                    help="only time the angular transform Y = P Phi (N_r = 4096, N_theta = 64, N_phi = 17, "
                         "complex64) forward and inverse, and B Y psi with the radial transform")
    ap.add_argument("--uneven-profile", action="store_true",
                    help="only run --steps forward + inverse pairs of the uneven batch (512 transforms, N 512..8192, "
                         "l 0..127) after --warmup untimed pairs, for a kernel trace")
    ap.add_argument("--adjoint-profile", action="store_true",
                    help="only run --steps loss-and-gradient passes through 200 split steps (checkpoints every 20, "
                         "graph-replayed segments) after --warmup untimed ones, for a kernel trace")
    args = ap.parse_args()
    headline_defaults = (args.steps is None, args.warmup is None)
    if args.steps is None:
        args.steps = 50
    if args.warmup is None:
        args.warmup = 5
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU per process; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1509_07115_amd import Plan, _lib, workloads

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 4}))
        return

    if args.uneven_profile:
        w = workloads.uneven()
        plan = Plan(w.channels)
        x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
        b, y = plan.empty(), plan.empty()
        step = lambda: (plan.forward(x, b), plan.inverse(b, y))
        for _ in range(max(args.warmup, 1)):
            step()
        ms = _timed(step, args.steps)
        print(json.dumps({"workload": w.name, "ms_per_fwd_inv": ms, "pairs": args.steps,
                          "points_per_s": w.points / (ms * 1e-3)}))
        return

    if args.adjoint_profile:
        from paper_1509_07115_amd.autograd import propagate
        w = workloads.adjoint()
        plan = Plan(w.channels)
        plan.set_potential(w.extra["V"], w.extra["dt"])
        phi = torch.from_numpy(w.extra["phi"]).to(torch.complex64).cuda()
        s = torch.from_numpy(w.extra["s"]).to(torch.float32).cuda()

        def grad_pass():
            p0 = torch.from_numpy(w.psi).to(torch.complex64).cuda().requires_grad_(True)
            st = s.clone().requires_grad_(True)
            z = torch.vdot(phi, propagate(plan, p0, st, checkpoint_every=20, graph=True))
            ((z * z.conj()).real).backward()
        for _ in range(max(args.warmup, 1)):
            grad_pass()
        ms = _timed(grad_pass, args.steps)
        print(json.dumps({"workload": w.name, "ms_per_loss_and_gradient": ms, "passes": args.steps}))
        return

    if args.split_step_profile:
        w = workloads.tdse()
        out = {}
        for prec in ("c64", "c64x"):
            plan = Plan(w.channels, precision=prec)
            plan.set_potential(w.extra["V"], w.extra["dt"])
            x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
            plan.kinetic_step(x, args.warmup)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.kinetic_step(x, args.steps)
            e1.record()
            torch.cuda.synchronize()
            out[prec] = {"workload": w.name, "ms_per_step": e0.elapsed_time(e1) / args.steps, "steps": args.steps}
            del plan
        print(json.dumps(out))
        return

    if args.angular_profile:
        from paper_1509_07115_amd import AngularTransform, sht_grid

        def timed(fn, n):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n
        nr, nt, nphi, rmax = 4096, 64, 17, 200.0
        Y = AngularTransform(nr, nt, nphi)
        plan = Plan(Y.channels(rmax))
        g = torch.randn(Y.size, dtype=torch.complex64, device="cuda")
        c, b = torch.empty_like(g), torch.empty_like(g)
        steps = max(args.steps, 1)

        def step3d_ms():
            # one split step of U = r^2/2 - F z on this grid (the potential factor twice, Y, the radial
            # kinetic step, Y^H)
            from paper_1509_07115_amd import step3d
            r = (torch.arange(nr, dtype=torch.float64, device="cuda") + 0.5) * (rmax / nr)
            eta = torch.from_numpy(sht_grid(nt, nphi)[0]).cuda()
            v0 = (0.5 * r * r).repeat(nt * nphi).contiguous()
            v1 = (-eta[:, None, None] * r[None, None, :]).expand(nt, nphi, nr).contiguous().reshape(-1)
            step_plan = Plan(Y.channels(rmax))
            step_plan.set_potential(np.zeros(step_plan.elems), 0.01)
            x = g.clone()
            return timed(lambda: step3d(Y, step_plan, x, v0, v1, 0.3, 0.01, c), steps)

        def step3d_velocity_ms():
            # one velocity-gauge step (the printed sequence through the momentum grid), A along z
            from paper_1509_07115_amd import step3d_velocity
            r = (torch.arange(nr, dtype=torch.float64, device="cuda") + 0.5) * (rmax / nr)
            v0 = (0.5 * r * r).repeat(nt * nphi).contiguous()
            K, Pz = Y.kinetic(rmax), Y.momentum_pz(rmax)
            x, w1, w2 = g.clone(), torch.empty_like(g), torch.empty_like(g)
            return timed(lambda: step3d_velocity(Y, plan, x, v0, K, Pz, 0.1, 0.01, w1, w2), steps)
        out = {"workload": f"angular transform N_r={nr} N_theta={nt} N_phi={nphi} ({nt * nphi} channels, "
                           f"l <= {nt - 1 + (nphi - 1) // 2}), complex64",
               "ms_forward": timed(lambda: Y.forward(g, c), steps),
               "ms_inverse": timed(lambda: Y.inverse(c, g), steps),
               "ms_B_Y_psi": timed(lambda: plan.forward(Y.forward(g, c), b), steps),
               "ms_step3d": step3d_ms(),
               "ms_step3d_velocity": step3d_velocity_ms(),
               "flops_per_direction": 8 * nt * nphi * nphi * nr + 4 * nphi * nt * nt * nr,
               "bytes_per_direction": 4 * Y.size * 8}
        # the same grid in complex128 (vector kernels, FP64), and N_phi = 63, whose azimuthal DFT
        # (2 N_phi > 64) takes the vector kernel in complex64 as well
        Y2 = AngularTransform(nr, nt, nphi, "c128")
        g2 = torch.randn(Y2.size, dtype=torch.complex128, device="cuda")
        c2 = torch.empty_like(g2)
        out["complex128"] = {"ms_forward": timed(lambda: Y2.forward(g2, c2), steps),
                             "ms_inverse": timed(lambda: Y2.inverse(c2, g2), steps)}
        del Y2, g2, c2
        Y3 = AngularTransform(1024, nt, 63)
        g3 = torch.randn(Y3.size, dtype=torch.complex64, device="cuda")
        c3 = torch.empty_like(g3)
        out["n_phi_63"] = {"workload": f"N_r=1024 N_theta={nt} N_phi=63, complex64",
                           "ms_forward": timed(lambda: Y3.forward(g3, c3), steps),
                           "ms_inverse": timed(lambda: Y3.inverse(c3, g3), steps)}
        print(json.dumps(out))
        return

    if args.autotune_profile:
        def timed(fn, n):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n
        out = {}
        for w in (workloads.batched_all_m(), workloads.uneven()):
            t0 = time.time()
            tuned = Plan.autotuned(w.channels, nrep=max(args.steps, 1))
            t_tune = time.time() - t0
            default = Plan(w.channels)
            x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
            b = torch.empty_like(x)
            res = {"tuning": tuned.tuning, "tune_seconds": t_tune}
            for name, p in (("default", default), ("tuned", tuned)):
                res[f"ms_fwd_inv_{name}"] = timed(lambda: (p.forward(x, b), p.inverse(b, x)), max(args.steps, 1))
            out[w.name] = res
            del tuned, default
        print(json.dumps(out))
        return

    if args.monomial_profile:
        def timed(fn, n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n
        N, rmax = 1024, 102.4
        chs, off = [], 0
        for ell in range(32):
            for _ in range(2 * ell + 1):
                chs.append((N, ell, rmax, off))
                off += N
        rng = np.random.default_rng(9)
        psi = torch.from_numpy(rng.standard_normal(off) + 1j * rng.standard_normal(off)).cuda()
        out = {"workload": f"N={N} rmax={rmax} l=0..31 all m ({len(chs)} channels), complex128"}
        res = {}
        for alg in ("tiled", "monomial"):
            plan = Plan(chs, precision="c128", algorithm=alg)
            b, x = plan.empty(), plan.empty()
            timed(lambda: plan.forward(psi, b), max(args.warmup, 1))
            out[alg] = {"ms_forward": timed(lambda: plan.forward(psi, b), args.steps),
                        "ms_inverse": timed(lambda: plan.inverse(b, x), args.steps)}
            res[alg] = b.clone()
            del plan
        err = {}
        for c, (N_, ell, _, o) in enumerate(chs):
            if ell in err:
                continue
            d = torch.linalg.vector_norm(res["monomial"][o:o + N] - res["tiled"][o:o + N])
            err[ell] = float(d / torch.linalg.vector_norm(res["tiled"][o:o + N]))
        out["monomial_error_vs_tiled"] = {str(k): v for k, v in sorted(err.items())}
        print(json.dumps(out))
        return

    if args.imag_time_profile:
        def timed(fn, n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n
        out = {}
        w = workloads.hydrogen(dr=0.05, start="hydrogen")
        for prec in ("c64", "c128"):
            plan = Plan(w.channels, precision=prec, kinetic="corrected")
            plan.set_potential(w.extra["V"], 0.01, imaginary=True)
            x = torch.from_numpy(w.psi).to(plan.dtype).cuda()
            sets = w.extra["sets"]

            def block():
                plan.kinetic_step(x, 10, graph=True)
                plan.orthonormalize(x, sets)
            timed(block, max(args.warmup, 1))
            ms = timed(block, args.steps) / 10
            e = plan.energy(x).cpu().numpy()
            out[prec] = {"workload": w.name, "ms_per_step": ms, "steps": 10 * args.steps,
                         "energies": [float(v) for v in (e[:, 1] + e[:, 2]) / e[:, 0]]}
            del plan
        w = workloads.tdse()
        plan = Plan(w.channels, kinetic="corrected")
        plan.set_potential(w.extra["V"], w.extra["dt"], imaginary=True)
        x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
        work = plan.empty()
        eo = torch.empty((len(w.channels), 3), dtype=torch.float64, device="cuda")
        single = list(range(len(w.channels) + 1))
        timed(lambda: plan.energy(x, work, eo), max(args.warmup, 1))
        timed(lambda: plan.orthonormalize(x, single), max(args.warmup, 1))
        out["batch"] = {"workload": w.name,
                        "ms_energy": timed(lambda: plan.energy(x, work, eo), args.steps),
                        "ms_orthonormalize_single": timed(lambda: plan.orthonormalize(x, single), args.steps),
                        "calls": args.steps}
        print(json.dumps(out))
        return

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1509_07115_amd import build
        build.build()

    progress("building the workload and the plan")
    if headline_defaults[0]:
        args.steps = 200
    if headline_defaults[1]:
        args.warmup = 2000
    w = workloads.batched_all_m()
    plan = Plan(w.channels)
    x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
    b = plan.empty()
    y = plan.empty()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.forward(x, b)
        plan.inverse(b, y)
    torch.cuda.synchronize()

    progress("warmup done; timing")
    # timed region: K steps.  Per-stage HIP events on the launch stream bracket
    # the launches of every PROFILE_EVERY-th step (events on every launch would
    # add their own gaps to the step time).
    plan.profile(True)
    plan.profile(False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        sample = i % PROFILE_EVERY == 0
        if sample:
            plan.profile(True, clear=False)
        plan.forward(x, b)
        plan.inverse(b, y)
        if sample:
            plan.profile(False)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    stages = plan.profile_read()
    ms_step = total_ms / args.steps
    alg = algorithmic_counts(w.channels)
    pts = alg["points"]
    value = pts / (ms_step * 1e-3)

    # dominant stage and its roofline (algorithmic flops / bytes per launch)
    (ms_f, n_f), (ms_m, n_m) = stages["sincos"], stages["moment"]
    avg_f, avg_m = ms_f / max(n_f, 1), ms_m / max(n_m, 1)
    if avg_m >= avg_f:
        traffic = None
        if MOMENT_TRAFFIC["sha256"] and MOMENT_TRAFFIC["sha256"] == sources_sha256(MOMENT_TRAFFIC["sources"]):
            traffic = MOMENT_TRAFFIC["fetch_bytes"] + MOMENT_TRAFFIC["write_bytes"]
        roof = roofline("moment stage (dsbt::mstage_chain)", alg["flops_moment"], alg["bytes_moment"], avg_m, traffic)
    else:
        roof = roofline("sine/cosine stage (dsbt::fstage_n)", alg["flops_sincos"], alg["bytes_sincos"], avg_f, None)
    roof["stages_ms_per_launch"] = {"sincos": avg_f, "moment": avg_m}
    roof["stage_launches_timed"] = {"sincos": n_f, "moment": n_m, "every_nth_step": PROFILE_EVERY}

    progress(f"timed {args.steps} steps: {ms_step:.4f} ms per step")
    bh = b.cpu().numpy().astype(np.complex128)   # checked against the oracle in the CPU-baseline leg
    rt = float((y - x).abs().max().item() / x.abs().max().item())

    out = {
        "metric": "complex64 DSBT fwd+inv radial points/sec vs plain GPU form, at <=1e-5 rel err",
        "value": value, "unit": "radial points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded Gaussian sums)",
        "config": {"workload": "batched all-m DSBT, N=2048, rmax=100, l=0..63 with 2l+1 m each (4096 channels), "
                               "complex64 data, FP64-built plan", "channels": len(w.channels), "N": 2048,
                   "points": pts, "parallelism": "single GPU"},
        "transforms_per_s": 2 * len(w.channels) / (ms_step * 1e-3),
        "max_rel_err_vs_oracle": None, "roundtrip_max_rel": rt,
        "roofline": roof,
    }
    if not args.no_plain:
        progress("timing the plain per-channel form")
        pplan = Plan(w.channels, mode="plain")
        pplan.forward(x, b)
        pplan.inverse(b, y)
        torch.cuda.synchronize()
        reps = 2
        e0.record(stream)
        for _ in range(reps):
            pplan.forward(x, b)
            pplan.inverse(b, y)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / reps
        out["plain_gpu_form"] = {"value": pts / (pms * 1e-3), "ms_per_step": pms,
                                 "form": "one launch per channel and stage (4 launches per channel per step)"}
        out["speedup_vs_plain"] = out["value"] / out["plain_gpu_form"]["value"]
    if not args.no_extra:
        out["other_workloads"] = other_workloads(progress)
    if not args.no_cpu_baseline:
        progress("timing the FP64 oracle on the host and checking l = 1, 32, 63 against it")
        out["cpu_baseline"], out["max_rel_err_vs_oracle"] = cpu_baseline(w, bh)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
