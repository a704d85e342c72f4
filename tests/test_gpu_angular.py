"""The angular transform Y = P Phi (Sec. 4.1) on the GPU through the C ABI,
against the FP64 oracle, and composed with the radial DSBT."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import angular, dsbt as odsbt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(dtype).cuda()


# tolerances: FP32 arithmetic, or FP64.  The complex64 cases take every matrix-core
# tile count of both axis steps (16 to 64 rows; the DFT up to 128), and N_phi = 63
# in complex128 the vector kernel of the azimuthal step (2 N_phi > 64).
CASES = [(8, 9, 100, "c64", 2e-6), (16, 17, 256, "c64", 2e-6), (64, 63, 70, "c64", 2e-6), (1, 1, 64, "c64", 1e-6),
         (33, 31, 130, "c64", 2e-6), (20, 5, 64, "c64", 2e-6),
         # 64 < 2 N_phi <= 128: the DFT matrix in LDS, 5, 6, 7 and 8 row blocks
         (8, 33, 100, "c64", 2e-6), (4, 45, 70, "c64", 2e-6), (3, 53, 130, "c64", 2e-6),
         # fewer radial points than one block: every load past the last point is clamped
         (5, 3, 3, "c64", 2e-6), (33, 31, 1, "c64", 2e-6), (5, 3, 3, "c128", 1e-12), (40, 31, 1, "c128", 1e-12),
         (8, 9, 100, "c128", 1e-12), (16, 31, 130, "c128", 1e-12), (64, 63, 65, "c128", 1e-12)]


@pytest.mark.parametrize("nt,nphi,nr,precision,tol", CASES)
def test_forward_inverse_match_oracle(nt, nphi, nr, precision, tol):
    from paper_1509_07115_amd import AngularTransform
    rng = np.random.default_rng(nt * 100 + nphi)
    psi = rng.standard_normal((nt, nphi, nr)) + 1j * rng.standard_normal((nt, nphi, nr))
    Y = AngularTransform(nr, nt, nphi, precision)
    c = Y.forward(dev(psi, Y.dtype)).cpu().numpy().reshape(nphi, nt, nr)
    ref = angular.forward(psi, nt, nphi)
    assert np.linalg.norm(c - ref) <= tol * np.linalg.norm(ref)
    back = Y.inverse(dev(c, Y.dtype)).cpu().numpy().reshape(nt, nphi, nr)
    assert np.linalg.norm(back - psi) <= 2 * tol * np.linalg.norm(psi)
    refi = angular.inverse(ref, nt, nphi)
    got_i = Y.inverse(dev(ref, Y.dtype)).cpu().numpy().reshape(nt, nphi, nr)
    assert np.linalg.norm(got_i - refi) <= tol * np.linalg.norm(refi)


@pytest.mark.parametrize("nt,nphi,nr,precision,tol", [(64, 17, 4096, "c64", 2e-6), (64, 63, 1024, "c64", 2e-6),
                                                      (64, 17, 4096, "c128", 1e-12)])
def test_timed_sizes_match_oracle(nt, nphi, nr, precision, tol):
    """The sizes the angular timing runs: there each matrix-core workgroup loops
    over several point blocks with its loads prefetched (3 and 4 blocks at
    64 x 17 x 4096 in complex64, 2 for the FP64 Legendre step; 2 for the
    Legendre step at 64 x 63 x 1024), which the small cases above do not reach.
    Element by element against the oracle."""
    from paper_1509_07115_amd import AngularTransform
    rng = np.random.default_rng(nr + nphi)
    psi = rng.standard_normal((nt, nphi, nr)) + 1j * rng.standard_normal((nt, nphi, nr))
    Y = AngularTransform(nr, nt, nphi, precision)
    ref = angular.forward(psi, nt, nphi)
    c = Y.forward(dev(psi, Y.dtype)).cpu().numpy().reshape(nphi, nt, nr)
    scale = np.abs(ref).max()
    assert np.abs(c - ref).max() <= tol * scale * math.sqrt(nt)
    assert np.linalg.norm(c - ref) <= tol * np.linalg.norm(ref)
    refi = angular.inverse(ref, nt, nphi)
    got_i = Y.inverse(dev(ref, Y.dtype)).cpu().numpy().reshape(nt, nphi, nr)
    assert np.abs(got_i - refi).max() <= tol * np.abs(refi).max() * math.sqrt(nt)
    assert np.linalg.norm(got_i - refi) <= tol * np.linalg.norm(refi)


@pytest.mark.parametrize("l,m", [(0, 0), (2, -1), (5, 3), (8, -7), (8, 8)])
def test_sampled_harmonic_has_one_coefficient(l, m):
    # Y_lm (library routine) sampled with sqrt(w_j dphi), l <= N_theta - 1: the
    # transform puts all of it on channel (l, m), at every radial point
    from paper_1509_07115_amd import AngularTransform
    nt, nphi, nr = 9, 17, 3
    eta, w, phi = angular.grid(nt, nphi)
    h = special.sph_harm_y(l, m, np.arccos(eta)[:, None], phi[None, :]) * np.sqrt(w)[:, None] * math.sqrt(2 * math.pi / nphi)
    psi = h[:, :, None] * np.array([1.0, -2.0, 0.5j])[None, None, :]
    Y = AngularTransform(nr, nt, nphi, "c128")
    c = Y.forward(dev(psi, Y.dtype)).cpu().numpy().reshape(nphi, nt, nr)
    ref = np.zeros_like(c)
    ref[m + 8, l - abs(m), :] = [1.0, -2.0, 0.5j]
    np.testing.assert_allclose(c, ref, atol=1e-12)


def test_composed_with_the_radial_transform():
    # c = B Y psi (eq. BYpsi): the coefficient layout is a DSBT channel layout
    from paper_1509_07115_amd import AngularTransform, Plan
    nt, nphi, nr, rmax = 6, 9, 128, 12.8
    rng = np.random.default_rng(8)
    psi = rng.standard_normal((nt, nphi, nr)) + 1j * rng.standard_normal((nt, nphi, nr))
    Y = AngularTransform(nr, nt, nphi)
    plan = Plan(Y.channels(rmax))
    b = plan.forward(Y.forward(dev(psi, torch.complex64))).cpu().numpy().reshape(nphi, nt, nr)
    a = angular.forward(psi, nt, nphi)
    for q in range(nphi):
        for t in range(nt):
            l = abs(q - 4) + t
            ref = odsbt.forward(a[q, t], l)
            assert np.linalg.norm(b[q, t] - ref) <= 1e-5 * np.linalg.norm(ref), (q, t)
    assert Y.lm()[0] == (4, -4) and Y.lm()[4 * nt] == (0, 0)


def test_rejected_sizes_and_buffers():
    from paper_1509_07115_amd import AngularTransform, DsbtError
    for nt, nphi in ((0, 5), (65, 5), (8, 4), (8, 65)):
        with pytest.raises(DsbtError, match="UNSUPPORTED"):
            AngularTransform(16, nt, nphi)
    Y = AngularTransform(16, 4, 5)
    with pytest.raises(TypeError):
        Y.forward(torch.zeros(16 * 20, dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        Y.forward(torch.zeros(10, dtype=torch.complex64, device="cuda"))
