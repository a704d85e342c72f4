"""Error paths of the C ABI that need a device (plan creation validates on the
host before any launch); each failing call leaves the library usable."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def Plan(*a, **k):
    from paper_1509_07115_amd import Plan as P
    return P(*a, **k)


@pytest.mark.parametrize("chans,status", [
    ([(100, 3, 10.0, 0)], "UNSUPPORTED"),          # N not a power of two
    ([(8, 1, 10.0, 0)], "UNSUPPORTED"),            # N below 16
    ([(16384, 1, 10.0, 0)], "UNSUPPORTED"),        # N above 8192
    ([(64, 127, 10.0, 0)], "UNSUPPORTED"),         # l > 2N - 2: no regular row
    ([(1024, 256, 10.0, 0)], "UNSUPPORTED"),       # l above 255
    ([(64, 3, 0.0, 0)], "INVALID_ARG"),            # rmax not positive
    ([(64, 3, 10.0, -1)], "INVALID_ARG"),          # negative offset
    ([(64, 3, 10.0, 0), (64, 2, 10.0, 63)], "INVALID_ARG"),   # overlapping channels
])
def test_plan_create_rejects(chans, status):
    from paper_1509_07115_amd import DsbtError
    with pytest.raises(DsbtError, match=status):
        Plan(chans)


def test_step_and_buffer_errors_leave_the_plan_usable():
    from paper_1509_07115_amd import DsbtError, _lib
    chans = [(64, 2, 6.4, 0), (64, 30, 6.4, 64)]
    plan = Plan(chans)
    x = torch.zeros(128, dtype=torch.complex64, device="cuda")
    x[3] = 1.0
    with pytest.raises(DsbtError, match="PLAN_MISMATCH"):      # no potential yet
        plan.kinetic_step(x, 1)
    with pytest.raises(DsbtError, match="INVALID_ARG"):
        plan.set_potential(np.zeros(128), 0.0)                # dt must be positive
    V = np.zeros(128)
    V[5] = np.nan
    with pytest.raises(DsbtError, match="INVALID_ARG"):
        plan.set_potential(V, 0.01)                           # non-finite potential
    plan.set_potential(np.zeros(128), 0.01)
    with pytest.raises(DsbtError, match="UNSUPPORTED"):
        plan.kinetic_step(x, 1, resident=True)                # resident step not built
    lib = _lib.load()
    st = lib.dsbt_kinetic_step(plan._h, ctypes.c_void_p(x.data_ptr()), 1, None, 64, None)
    assert st == -1                                           # unknown step flag
    with pytest.raises(TypeError):
        plan.forward(torch.zeros(128, dtype=torch.complex128, device="cuda"))   # wrong data precision
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(100, dtype=torch.complex64, device="cuda"))    # shorter than the layout
    # the plan still transforms correctly: norm preserved, inverse restores
    b = plan.forward(x)
    back = plan.inverse(b)
    torch.cuda.synchronize()
    assert abs(torch.linalg.vector_norm(b).item() - 1.0) < 1e-6
    assert torch.allclose(back, x, atol=1e-6)


def test_check_finite_reports_nonfinite_data():
    # checked plans scan the input of a transform or step for NaN and
    # infinities; the output is not touched when one is found
    from paper_1509_07115_amd import DsbtError
    chans = [(256, 3, 25.6, 0), (512, 20, 51.2, 256), (256, 0, 25.6, 768)]
    for precision, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        plan = Plan(chans, precision=precision, check_finite=True)
        x = torch.randn(1024, dtype=dtype, device="cuda")
        b = plan.forward(x)                     # finite: transforms as an unchecked plan
        ref = Plan(chans, precision=precision).forward(x)
        torch.cuda.synchronize()
        assert torch.equal(b, ref)
        for pos, bad in ((300, float("nan")), (1023, float("inf")), (0, float("-inf"))):
            y = x.clone()
            y[pos] = bad
            out = torch.full_like(x, 7.0)
            with pytest.raises(DsbtError, match="NONFINITE"):
                plan.forward(y, out=out)
            with pytest.raises(DsbtError, match="NONFINITE"):
                plan.inverse(y, out=out)
            assert torch.all(out == 7.0)
        plan.set_potential(np.zeros(1024), 0.01)
        y = x.clone()
        y[700] = float("nan")
        with pytest.raises(DsbtError, match="NONFINITE"):
            plan.kinetic_step(y, 2, graph=True)
        z = x.clone()
        plan.kinetic_step(z, 2, graph=True)     # finite input and result
        torch.cuda.synchronize()


def test_plan_memory_through_the_caller_allocator():
    # dev_alloc / dev_free: every device buffer of the plan comes from the
    # caller's allocator and goes back to it; a failing allocation (injected
    # after k successes) gives DSBT_ERR_OOM and hands back what was obtained
    from paper_1509_07115_amd import DsbtError
    chans = [(256, 5, 25.6, 0), (256, 6, 25.6, 256), (512, 33, 51.2, 512)]
    live = {}

    def alloc(n):
        t = torch.empty(int(n), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr):
        del live[ptr]

    x = torch.randn(1024, dtype=torch.complex64, device="cuda")
    ref = Plan(chans).forward(x)
    plan = Plan(chans, allocator=(alloc, free))
    n_plan = len(live)
    assert n_plan > 5
    assert sum(t.numel() for t in live.values()) >= plan.table_bytes
    b = plan.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(b, ref)
    plan.set_potential(np.zeros(1024), 0.01)     # potential tables come from the allocator too
    assert len(live) > n_plan
    plan.close()
    assert not live
    for k in (0, 3, n_plan - 1):
        count = [0]

        def failing(n):
            count[0] += 1
            return 0 if count[0] > k else alloc(n)
        with pytest.raises(DsbtError, match="OOM"):
            Plan(chans, allocator=(failing, free))
        assert not live, k
    # PyTorch's caching allocator
    plan = Plan(chans, allocator="torch")
    b = plan.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(b, ref)
    plan.close()


def test_angular_diagonal_tables_from_the_library():
    # K = k_n^2/2 per coefficient slot (eq. KinMat) and -2 k~_n eta_j on the
    # momentum grid, built behind the C ABI, against their definitions
    from paper_1509_07115_amd import AngularTransform, kinetic_momenta, sht_grid
    Nr, nt, nphi, rmax = 64, 6, 5, 12.8
    Y = AngularTransform(Nr, nt, nphi)
    for kin in ("plain", "corrected"):
        K = Y.kinetic(rmax, kin).cpu().numpy().reshape(nphi, nt, Nr)
        M = (nphi - 1) // 2
        for q in range(nphi):
            for t in range(nt):
                ell = abs(q - M) + t
                k = kinetic_momenta(Nr, ell, rmax, kin)
                assert np.array_equal(K[q, t], 0.5 * k * k), (kin, q, t)
    P = Y.momentum_pz(rmax).cpu().numpy().reshape(nt, nphi, Nr)
    eta = sht_grid(nt, nphi)[0]
    kt = np.arange(1, Nr + 1) * (np.pi / rmax)
    assert np.allclose(P, -2.0 * eta[:, None, None] * kt[None, None, :], rtol=1e-15, atol=0)
