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
