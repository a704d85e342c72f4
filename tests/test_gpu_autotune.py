"""The tile and batch-shape autotuner (dsbt_autotune) on a device."""
import json

import numpy as np
import pytest

from oracle import dsbt as odsbt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def test_autotuned_plan_is_correct_and_cached(tmp_path):
    from paper_1509_07115_amd import Plan
    chans, off = [], 0
    for ell in (3, 20, 40):
        for _ in range(2 * ell + 1):
            chans.append((512, ell, 51.2, off))
            off += 512
    cache = str(tmp_path / "tune.jsonl")
    plan = Plan.autotuned(chans, nrep=3, cache=cache)
    t = plan.tuning
    assert t["tile"] in (0, 32, 64) and t["chans_per_block"] in (0, 8, 4) and t["ms_per_fwd_inv"] > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["tile"] == t["tile"]
    # the tuned plan transforms correctly (per-channel relative error vs the oracle)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(off) + 1j * rng.standard_normal(off)
    b = plan.forward(torch.from_numpy(x).to(torch.complex64).cuda()).cpu().numpy()
    for N, ell, _, o in chans[:: 7]:
        ref = odsbt.forward(x[o:o + N], ell)
        assert np.linalg.norm(b[o:o + N] - ref) <= 1e-5 * np.linalg.norm(ref)
    # a second call is answered from the cache: same choice and time, no new line
    again = Plan.autotuned(chans, nrep=3, cache=cache).tuning
    assert (again["tile"], again["chans_per_block"]) == (t["tile"], t["chans_per_block"])
    assert again["ms_per_fwd_inv"] == pytest.approx(t["ms_per_fwd_inv"], abs=1e-6)   # stored with 6 decimals
    assert len(open(cache).read().splitlines()) == 1


def test_autotune_rejects_bad_arguments():
    from paper_1509_07115_amd import DsbtError, Plan
    with pytest.raises(DsbtError, match="INVALID_ARG"):
        Plan.autotuned([(64, 3, 6.4, 0)], nrep=0)
