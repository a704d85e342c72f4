"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import dsbt as odsbt
from oracle import sbf, tdse
from paper_1509_07115_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def Plan(*a, **k):
    from paper_1509_07115_amd import Plan as P
    return P(*a, **k)


def to_dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def per_channel_rel(got, ref, channels):
    out = []
    for N, _, _, off in channels:
        a, b = got[off:off + N], ref[off:off + N]
        nb = np.linalg.norm(b)
        out.append(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
    return np.array(out)


def oracle_apply(channels, x, inverse=False, ells=None):
    y = np.zeros_like(x, dtype=np.complex128)
    for N, ell, _, off in channels:
        if ells is not None and ell not in ells:
            continue
        seg = x[off:off + N].astype(np.complex128)
        y[off:off + N] = odsbt.inverse(seg, ell) if inverse else odsbt.forward(seg, ell)
    return y


def run(plan, x, inverse=False):
    d = to_dev(x, plan.dtype)
    out = plan.inverse(d) if inverse else plan.forward(d)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


# --- FP64 path: Gaussian orbitals N = 256, rmax = 20, l = 0..7 -------------

def test_c128_gaussian_orbitals_parity_and_closed_form():
    w = workloads.gaussian_orbitals()
    plan = Plan(w.channels, precision="c128")
    b = run(plan, w.psi)
    ref = oracle_apply(w.channels, w.psi)
    rel = per_channel_rel(b, ref, w.channels)
    assert rel.max() < 1e-12, rel
    back = run(plan, b, inverse=True)
    assert np.max(np.abs(back - w.psi)) < 1e-12 * np.max(np.abs(w.psi))
    # closed form of Sec. 3 (regular rows), error O(dk^2) on this coarse box
    for (N, ell, rmax, off), a in zip(w.channels, w.extra["a"]):
        p = odsbt.parity_p(ell)
        dk = odsbt.delta_k(rmax)
        k = np.arange(p, p + N) * dk
        c = sbf.gaussian_sbt(k, ell, a) * math.sqrt(dk)
        s0 = odsbt.n_extra(ell)
        err = np.max(np.abs(b[off + s0:off + N] - c[s0:])) / np.max(np.abs(c))
        assert err < 5e-2, (ell, err)


# --- complex64 path at small and ragged sizes --------------------------------

SMALL_CASES = [
    (16, [0, 1, 2, 3, 7, 14, 30]),
    (64, [0, 5, 6, 31, 63, 126]),
    (256, [1, 2, 17, 40, 127, 255]),
    (1024, [0, 33, 64, 127]),
]


@pytest.mark.parametrize("N,ells", SMALL_CASES)
@pytest.mark.parametrize("mode,precision", [("batched", "c64"), ("plain", "c64"), ("batched", "c64x"),
                                            ("batched", "c128"), ("plain", "c128")])
def test_c64_parity_small(N, ells, mode, precision):
    rng = np.random.default_rng(N)
    chans, parts, off = [], [], 0
    for ell in ells:
        # ragged channel counts per l exercise partial work items
        for _ in range(1 + (ell % 3) + (17 if ell == ells[-1] else 0)):
            chans.append((N, ell, 10.0 + ell, off))
            parts.append(rng.standard_normal(N) + 1j * rng.standard_normal(N))
            off += N
    x = np.concatenate(parts)
    plan = Plan(chans, mode=mode, precision=precision)
    # c64x rounds only the stored input and output to FP32: two roundings;
    # c128 is FP64 throughout (four-wave pipeline for l <= 63, generic kernel above)
    tol = {"c64": 2e-6, "c64x": 2.5e-7, "c128": 1e-12}[precision]
    b = run(plan, x)
    ref = oracle_apply(chans, x)
    assert per_channel_rel(b, ref, chans).max() < tol
    y = run(plan, x, inverse=True)
    refi = oracle_apply(chans, x, inverse=True)
    assert per_channel_rel(y, refi, chans).max() < tol


def test_plain_and_batched_agree_bitwise():
    w = workloads.batched_all_m(seed=7, N=512, rmax=25.0, ells=[0, 3, 8, 21])
    x = to_dev(w.psi, torch.complex64)
    a = Plan(w.channels).forward(x)
    b = Plan(w.channels, mode="plain").forward(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fused_step_stages_agree_bitwise_with_separate_launches():
    # batched split steps run one step's inverse sine/cosine stage and the next
    # step's forward one as one launch; the plain form launches them
    # separately: the products are the same, so the results agree bitwise
    # (strengths per step, forward and adjoint order)
    w = workloads.batched_all_m(seed=9, N=512, rmax=25.0, ells=[0, 1, 6, 13])
    V = np.concatenate([-1.0 / np.sqrt(workloads.grid(N, rmax) ** 2 + 0.1) for N, _, rmax, _ in w.channels])
    pb, pp = Plan(w.channels), Plan(w.channels, mode="plain")
    for p in (pb, pp):
        p.set_potential(V, 0.01)
    x = to_dev(w.psi, torch.complex64)
    a, b = x.clone(), x.clone()
    s = torch.tensor([1.0, 0.97, 1.03, 1.1], dtype=torch.float32, device="cuda")
    pb.kinetic_step(a, 4, s)
    pp.kinetic_step(b, 4, s)
    pb.kinetic_step(a, 3, s, adjoint=True)
    pp.kinetic_step(b, 3, s, adjoint=True)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_steps_of_two_block_items_agree_bitwise_with_plain():
    # l = 0..63 with all m (4096 channels) gives 288 items of 16 channels, more
    # than the device's compute units, so the batched moment stage runs items
    # of two 16-column blocks; the plain form runs one channel per launch.
    # Split steps with the kinetic factors (forward and adjoint): same products
    # per channel, bitwise equal results
    w = workloads.batched_all_m(seed=12, N=256, rmax=25.6, lmax=63)
    V = np.concatenate([-1.0 / np.sqrt(workloads.grid(N, rmax) ** 2 + 0.1) for N, _, rmax, _ in w.channels])
    pb, pp = Plan(w.channels), Plan(w.channels, mode="plain")
    for p in (pb, pp):
        p.set_potential(V, 0.01)
    x = to_dev(w.psi, torch.complex64)
    a, b = x.clone(), x.clone()
    s = torch.tensor([1.0, 0.9], dtype=torch.float32, device="cuda")
    pb.kinetic_step(a, 2, s)
    pp.kinetic_step(b, 2, s)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    pb.kinetic_step(a, 2, s, adjoint=True)
    pp.kinetic_step(b, 2, s, adjoint=True)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # two steps and their adjoint return the input to rounding
    assert float(torch.max(torch.abs(a - x)).item()) < 1e-5 * float(torch.max(torch.abs(x)).item())


def test_in_place_and_offsets_with_gaps():
    rng = np.random.default_rng(3)
    chans = [(128, 5, 12.0, 7), (256, 12, 30.0, 400), (128, 0, 5.0, 1000)]
    x = np.zeros(1200, dtype=np.complex128)
    for N, _, _, off in chans:
        x[off:off + N] = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    plan = Plan(chans)
    d = to_dev(x, torch.complex64)
    plan.forward(d, out=d)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    ref = oracle_apply(chans, x)
    assert per_channel_rel(got, ref, chans).max() < 2e-6
    # untouched gaps stay untouched
    assert np.all(got[:7] == 0) and np.all(got[135:400] == 0)
    plan.inverse(d, out=d)
    torch.cuda.synchronize()
    back = d.cpu().numpy()
    assert per_channel_rel(back, x, chans).max() < 4e-6


def test_max_sizes_n8192_l127():
    rng = np.random.default_rng(11)
    chans = [(8192, 127, 409.6, 0), (8192, 126, 409.6, 8192), (8192, 1, 409.6, 16384)]
    x = rng.standard_normal(3 * 8192) + 1j * rng.standard_normal(3 * 8192)
    plan = Plan(chans)
    b = run(plan, x)
    ref = oracle_apply(chans, x)
    assert per_channel_rel(b, ref, chans).max() < 1e-5


# --- batched workload at its full size: every l group -----------------------

def test_c64_batched_all_m_full_size_every_l():
    # N = 2048, rmax = 100, l = 0..63 with all m (4096 channels), the launch
    # configuration the benchmark times.  Every l group is compared with the
    # FP64 oracle, forward on the workload and inverse on the GPU's own b (the
    # oracle's T and F are built once per l and applied to all 2l+1 columns),
    # so a wrong table at any l fails even if it keeps T orthogonal.
    w = workloads.batched_all_m()
    plan = Plan(w.channels)
    b = run(plan, w.psi)
    back = run(plan, b, inverse=True)
    groups = {}
    for N, ell, _, off in w.channels:
        groups.setdefault(ell, []).append(off)
    N = w.channels[0][0]
    worst_f = worst_i = 0.0
    for ell, offs in sorted(groups.items()):
        cols = np.stack([w.psi[o:o + N] for o in offs], axis=1)
        ref_f = odsbt.forward(cols, ell)
        got_f = np.stack([b[o:o + N] for o in offs], axis=1)
        ef = np.linalg.norm(got_f - ref_f, axis=0) / np.linalg.norm(ref_f, axis=0)
        bcols = got_f
        ref_i = odsbt.inverse(bcols, ell)
        got_i = np.stack([back[o:o + N] for o in offs], axis=1)
        ei = np.linalg.norm(got_i - ref_i, axis=0) / np.linalg.norm(ref_i, axis=0)
        worst_f, worst_i = max(worst_f, ef.max()), max(worst_i, ei.max())
        assert ef.max() < 1e-5 and ei.max() < 1e-5, (ell, ef.max(), ei.max())
    print(f"every l: forward max rel {worst_f:.2e}, inverse max rel {worst_i:.2e}")
    # norm conservation on every channel (eq. conservNorm), and roundtrip
    for N, _, _, off in w.channels:
        assert abs(np.linalg.norm(b[off:off + N]) / np.linalg.norm(w.psi[off:off + N]) - 1) < 1e-5
    assert per_channel_rel(back, w.psi, w.channels).max() < 1e-5


# --- split step --------------------------------------------------------------

def _small_tdse(N=256, rmax=25.6, lmax=3, dt=0.01):
    return workloads.tdse(seed=5, N=N, rmax=rmax, lmax=lmax, dt=dt, small=0.1)


@pytest.mark.parametrize("N,rmax,lmax", [(256, 25.6, 3), (64, 12.8, 6)])
def test_step_matches_oracle_and_is_unitary(N, rmax, lmax):
    # N = 64: two tiles of 32 per channel, fewer than a pipeline loop
    # iteration (the tail variant), with the kinetic factors on the inverse
    w = _small_tdse(N=N, rmax=rmax, lmax=lmax)
    plan = Plan(w.channels)
    plan.set_potential(w.extra["V"], w.extra["dt"])
    d = to_dev(w.psi, torch.complex64)
    plan.kinetic_step(d, nsteps=5)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    ref = w.psi.copy()
    for N, ell, rmax, off in w.channels:
        V = w.extra["V"][off:off + N]
        E = tdse.kinetic_energies(N, rmax, ell)
        x = w.psi[off:off + N]
        for _ in range(5):
            x = tdse.step(x, ell, V, E, w.extra["dt"])
        ref[off:off + N] = x
    assert per_channel_rel(got, ref, w.channels).max() < 2e-5
    assert abs(np.linalg.norm(got) - np.linalg.norm(w.psi)) < 1e-5


def test_adjoint_step_inverts_and_graph_is_identical():
    w = _small_tdse()
    plan = Plan(w.channels)
    plan.set_potential(w.extra["V"], w.extra["dt"])
    s = torch.tensor([1.0, 0.95, 1.05, 1.1], dtype=torch.float32, device="cuda")
    d0 = to_dev(w.psi, torch.complex64)
    d = d0.clone()
    plan.kinetic_step(d, nsteps=4, s=s)
    e = d0.clone()
    plan.kinetic_step(e, nsteps=4, s=s, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(d, e)
    plan.kinetic_step(d, nsteps=4, s=s, adjoint=True)
    torch.cuda.synchronize()
    assert (d - d0).abs().max().item() < 1e-5


def test_step_grad_s_matches_oracle():
    w = _small_tdse(N=128, rmax=12.8, lmax=2)
    plan = Plan(w.channels, precision="c128")
    V, dt = w.extra["V"], w.extra["dt"]
    plan.set_potential(V, dt)
    rng = np.random.default_rng(2)
    n = w.elems
    a, b_, c, e = (rng.standard_normal(n) + 1j * rng.standard_normal(n) for _ in range(4))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.step_grad_s(*(to_dev(v, torch.complex128) for v in (a, b_, c, e)), out)
    torch.cuda.synchronize()
    ref = 0.5 * dt * np.sum(V * (np.conj(e) * b_ + np.conj(c) * a).imag)
    assert abs(out.item() - ref) < 1e-10 * max(1.0, abs(ref))
