"""FP64 plan generation on the GPU, and the uneven batch built from it."""
import time

import numpy as np
import pytest

from oracle import dsbt as odsbt
from paper_1509_07115_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(x, dtype=torch.complex64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("N,ell,B", [(256, 0, 32), (256, 1, 32), (256, 2, 32), (512, 7, 32), (512, 40, 32),
                                     (2048, 62, 32), (2048, 63, 32), (4096, 100, 64), (8192, 126, 64),
                                     (8192, 127, 64)])
def test_device_tables_match_host(N, ell, B):
    # the GPU generator (DLOP recurrences, tile bases, weighted inner products
    # in FP64) against the host generator, which the CPU tests pin to the
    # oracle's T
    from paper_1509_07115_amd import device_ftb_tables, host_ftb_tables
    d = device_ftb_tables(N, ell, B)
    h = host_ftb_tables(N, ell, B)
    err = np.max(np.abs(d - h)) / np.max(np.abs(h))
    print(f"N={N} l={ell} B={B}: max |device - host| / max |host| = {err:.2e}")
    assert err < 1e-11


def test_device_and_host_plans_agree_and_match_oracle():
    from paper_1509_07115_amd import Plan
    w = workloads.batched_all_m(N=512, lmax=9)
    x = dev(w.psi)
    outs = []
    for where in ("device", "host"):
        plan = Plan(w.channels, plan_where=where)
        outs.append(plan.forward(x).cpu().numpy().astype(np.complex128))
    torch.cuda.synchronize()
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-6 * np.max(np.abs(outs[1]))
    for N, ell, _, off in w.channels[::7]:
        ref = odsbt.forward(w.psi[off:off + N], ell)
        assert np.linalg.norm(outs[0][off:off + N] - ref) <= 1e-5 * np.linalg.norm(ref)


def test_uneven_batch_device_plan():
    # 512 transforms, N in {512 .. 8192}, l in 0..127, rmax = 0.05 N (seed 3):
    # one plan, FP64 tables generated on the GPU; per-channel round trip for
    # every channel, forward against the FP64 oracle on the smallest and the
    # largest l of every N
    from paper_1509_07115_amd import Plan
    w = workloads.uneven()
    t = time.perf_counter()
    plan = Plan(w.channels)
    print(f"plan for {len(w.channels)} channels: {time.perf_counter() - t:.2f} s, "
          f"{plan.table_bytes / 1e6:.1f} MB of tables")
    x = dev(w.psi)
    b = plan.forward(x)
    y = plan.inverse(b)
    torch.cuda.synchronize()
    bh = b.cpu().numpy().astype(np.complex128)
    yh = y.cpu().numpy().astype(np.complex128)
    worst_rt = 0.0
    for N, ell, _, off in w.channels:
        nx = np.linalg.norm(w.psi[off:off + N])
        worst_rt = max(worst_rt, np.linalg.norm(yh[off:off + N] - w.psi[off:off + N]) / nx)
    print(f"round trip: max per-channel relative error {worst_rt:.2e}")
    assert worst_rt < 1e-5
    # forward and inverse against the FP64 oracle: the smallest and the largest
    # l of every N, and one channel (the smallest N) of every distinct l, so
    # that every l's tables are checked
    pick = {}
    for N, ell, _, off in w.channels:
        lo, hi = pick.get(N, ((999, 0), (-1, 0)))
        pick[N] = (min(lo, (ell, off)), max(hi, (ell, off)))
    sel = {(N, ell, off) for N, s in pick.items() for ell, off in s}
    per_l = {}
    for N, ell, _, off in w.channels:
        if ell not in per_l or N < per_l[ell][0]:
            per_l[ell] = (N, off)
    sel |= {(N, ell, off) for ell, (N, off) in per_l.items()}
    worst_f = worst_i = 0.0
    for N, ell, off in sorted(sel):
        ref = odsbt.forward(w.psi[off:off + N], ell)
        err = np.linalg.norm(bh[off:off + N] - ref) / np.linalg.norm(ref)
        ref_i = odsbt.inverse(bh[off:off + N], ell)
        err_i = np.linalg.norm(yh[off:off + N] - ref_i) / np.linalg.norm(ref_i)
        worst_f, worst_i = max(worst_f, err), max(worst_i, err_i)
        assert err < 1e-5 and err_i < 1e-5, (N, ell, err, err_i)
    print(f"{len(sel)} channels ({len(per_l)} distinct l): forward max rel {worst_f:.2e}, "
          f"inverse max rel {worst_i:.2e}")
