"""The paper's monomial-moment fast multiplication (Sec. 2.6) on the GPU through
the C ABI: parity with the oracle's FP64 run of the same printed algorithm, and
its error envelope against the stable transform."""
import numpy as np
import pytest

from oracle import dsbt, monomial, tdse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def Plan(*a, **k):
    from paper_1509_07115_amd import Plan as P
    return P(*a, **k)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.complex128).cuda()


def channels(spec, gap=8):
    chs, off = [], 0
    for N, ell in spec:
        chs.append((N, ell, 0.1 * N, off))
        off += N + gap
    return chs, off


def random_state(chs, elems, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros(elems, dtype=np.complex128)
    for N, _, _, off in chs:
        v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        x[off:off + N] = v / np.linalg.norm(v)
    return x


SPEC = [(64, 0), (64, 1), (64, 2), (128, 3), (128, 6), (128, 9), (256, 12), (256, 16), (128, 20), (128, 24),
        (256, 1), (64, 5)]


def test_forward_and_inverse_match_the_printed_algorithm():
    # GPU and oracle run the same FP64 recurrences (eqs. rec_sum_b_f and
    # rec_sum_f_b) with the same xi; they differ only in rounding order, which
    # the cancellation amplifies as much as the algorithm's own error against
    # the dense T.  Bound per channel: 20 x that error + 1e-14.
    chs, elems = channels(SPEC)
    psi = random_state(chs, elems, 21)
    plan = Plan(chs, precision="c128", algorithm="monomial")
    b = plan.forward(dev(psi), torch.zeros(plan.elems, dtype=torch.complex128, device="cuda")).cpu().numpy()
    back = plan.inverse(dev(b)).cpu().numpy()
    for N, ell, _, off in chs:
        F = dsbt.fourier_matrix(N, ell)
        T = dsbt.ftb_matrix(N, ell)
        f = F @ psi[off:off + N]
        exact = T @ f
        lit = monomial.forward_literal(f, ell)
        env = np.linalg.norm(lit - exact) / np.linalg.norm(exact)
        gb = b[off:off + N]
        tol = 20 * env + 1e-14
        assert np.linalg.norm(gb - lit) <= tol * np.linalg.norm(exact), (N, ell, env)
        # inverse of the GPU's b: F^T applied to the literal T^T b
        ref_inv = F.T @ monomial.inverse_literal(gb, ell)
        env_i = np.linalg.norm(ref_inv - F.T @ (T.T @ gb)) / np.linalg.norm(gb)
        assert np.linalg.norm(back[off:off + N] - ref_inv) <= (20 * env_i + 1e-14) * np.linalg.norm(gb), (N, ell)
    # gaps between channels stay untouched
    mask = np.ones(plan.elems, bool)
    for N, _, _, off in chs:
        mask[off:off + N] = False
    assert np.all(b[mask] == 0)


def test_in_place_and_kinetic_step_match_oracle():
    chs, elems = channels([(128, 1), (128, 4), (64, 7), (64, 0)], gap=0)
    psi = random_state(chs, elems, 22)
    plan = Plan(chs, precision="c128", algorithm="monomial")
    x = dev(psi)
    ref = plan.forward(x)
    plan.forward(x, x)                       # in place
    assert torch.equal(x, ref)
    plan.inverse(x, x)
    np.testing.assert_allclose(x.cpu().numpy(), psi, atol=1e-13)
    # a split step with the kinetic phase fused into the monomial stage
    V = np.zeros(elems)
    for N, ell, rmax, off in chs:
        r = dsbt.grid_r(N, rmax)
        V[off:off + N] = -1.0 / np.sqrt(r * r + 0.01)
    plan.set_potential(V, 0.05)
    y = dev(psi)
    plan.kinetic_step(y, 2)
    got = y.cpu().numpy()
    for N, ell, rmax, off in chs:
        E = tdse.kinetic_energies(N, rmax, ell)
        r = psi[off:off + N]
        for _ in range(2):
            r = tdse.step(r, ell, V[off:off + N], E, 0.05)
        assert np.linalg.norm(got[off:off + N] - r) <= 1e-12, (N, ell)


def test_error_envelope_against_the_tiled_transform():
    # the printed algorithm's FP64 error grows quickly with l (the reason for the
    # tiled form); measured here against the stable complex128 path at N = 1024
    N, ells = 1024, [2, 4, 8, 12, 16, 20, 24, 28]
    chs, elems = channels([(N, ell) for ell in ells], gap=0)
    psi = random_state(chs, elems, 23)
    mono = Plan(chs, precision="c128", algorithm="monomial")
    tiled = Plan(chs, precision="c128")
    bm = mono.forward(dev(psi)).cpu().numpy()
    bt = tiled.forward(dev(psi)).cpu().numpy()
    err = {}
    for N_, ell, _, off in chs:
        err[ell] = np.linalg.norm(bm[off:off + N] - bt[off:off + N]) / np.linalg.norm(bt[off:off + N])
    print("monomial FP64 forward error vs tiled, N=1024: " + ", ".join(f"l={e}: {v:.1e}" for e, v in err.items()))
    assert err[2] < 1e-13 and err[4] < 1e-13
    assert err[16] > 10 * err[4]
    assert err[28] > 1e3 * err[12]


def test_unsupported_requests():
    from paper_1509_07115_amd import DsbtError
    with pytest.raises(DsbtError, match="UNSUPPORTED"):
        Plan([(64, 3, 6.4, 0)], precision="c64", algorithm="monomial")
    with pytest.raises(DsbtError, match="UNSUPPORTED"):
        Plan([(8192, 200, 100.0, 0)], precision="c128", algorithm="monomial")
