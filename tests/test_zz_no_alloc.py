"""The allocation-free entry point dsbt_step_grad_s_noalloc against
dsbt_step_grad_s, called through the C ABI: two calls in a row on one device,
the second with a plan of fewer channels (the fixed scratch array keeps the
first call's partial sums, which the second must not read)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _case(nch, N, precision, seed):
    from paper_1509_07115_amd import Plan
    rng = np.random.default_rng(seed)
    chans = [(N, c % 7, 0.05 * N, c * N) for c in range(nch)]
    plan = Plan(chans, precision=precision)
    plan.set_potential(rng.uniform(-2.0, 2.0, nch * N), 0.01)
    dtype = plan.dtype
    bufs = [torch.from_numpy(rng.standard_normal(nch * N) + 1j * rng.standard_normal(nch * N)).to(dtype).cuda()
            for _ in range(4)]
    return plan, bufs


def _call(lib, name, plan, bufs, out):
    fn = getattr(lib, name)
    return fn(plan._h, *(ctypes.c_void_p(b.data_ptr()) for b in bufs), ctypes.c_void_p(out.data_ptr()), None)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_noalloc_grad_s_matches_the_allocating_entry_point(precision):
    from paper_1509_07115_amd import _lib
    lib = _lib.load()
    for nch, N, seed in ((300, 256, 1), (7, 64, 2)):     # second call: fewer channels, smaller grid
        plan, bufs = _case(nch, N, precision, seed)
        ref = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        got = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        assert _call(lib, "dsbt_step_grad_s", plan, bufs, ref) == 0
        assert _call(lib, "dsbt_step_grad_s_noalloc", plan, bufs, got) == 0
        torch.cuda.synchronize()
        r, g = ref.item(), got.item()
        print(f"{precision} nch={nch}: grad_s {r:.17g}, no-alloc {g:.17g}")
        assert np.isfinite(r) and abs(g - r) <= 1e-12 * max(1.0, abs(r)), (r, g)


def test_noalloc_grad_s_rejects_plans_above_its_limit():
    from paper_1509_07115_amd import Plan, _lib
    lib = _lib.load()
    n = 65537
    plan = Plan([(16, 0, 1.0, 16 * c) for c in range(n)])
    plan.set_potential(np.zeros(16 * n), 0.01)
    x = torch.zeros(16 * n, dtype=torch.complex64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = _call(lib, "dsbt_step_grad_s_noalloc", plan, [x, x, x, x], out)
    assert st == -2
    assert b"DSBT_NOALLOC_MAX_CHANNELS" in lib.dsbt_last_error()
