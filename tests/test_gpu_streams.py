"""Every call enqueues on the stream it is given: results on a side stream are
bitwise those of the default stream (the kernels are deterministic)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(built_lib):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def on_side(fn):
    """Run fn(stream) on a fresh default-priority stream, ordered after the current one."""
    side = torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    side.wait_stream(cur)
    with torch.cuda.stream(side):
        out = fn(side)
    cur.wait_stream(side)
    torch.cuda.synchronize()
    return out


def test_transforms_steps_and_state_kernels_on_a_side_stream():
    from paper_1509_07115_amd import Plan, workloads
    w = workloads.batched_all_m(seed=9, N=512, rmax=40.0, ells=[0, 5, 20, 40])
    plan = Plan(w.channels)
    x = torch.from_numpy(w.psi).to(torch.complex64).cuda()
    ref_b = plan.forward(x)
    ref_x = plan.inverse(ref_b)
    b = on_side(lambda s: plan.forward(x, stream=s))
    back = on_side(lambda s: plan.inverse(b, stream=s))
    assert torch.equal(b, ref_b) and torch.equal(back, ref_x)
    V = np.zeros(plan.elems)
    plan.set_potential(V - 0.1, 0.01)
    y0, y1 = x.clone(), x.clone()
    plan.kinetic_step(y0, 7, graph=True)
    on_side(lambda s: plan.kinetic_step(y1, 7, graph=True, stream=s))
    assert torch.equal(y0, y1)
    e0 = plan.energy(x)
    e1 = on_side(lambda s: plan.energy(x, stream=s))
    assert torch.equal(e0, e1)
    sets = [0, 1, 12, len(w.channels)]
    z0, z1 = x.clone(), x.clone()
    plan.orthonormalize(z0, sets)
    on_side(lambda s: plan.orthonormalize(z1, sets, stream=s))
    assert torch.equal(z0, z1)


def test_angular_transform_and_3d_step_on_a_side_stream():
    from paper_1509_07115_amd import AngularTransform, Plan, step3d
    nr, nt, nphi, rmax = 64, 6, 7, 12.8
    Y = AngularTransform(nr, nt, nphi)
    plan = Plan(Y.channels(rmax))
    plan.set_potential(np.zeros(plan.elems), 0.02)
    g = torch.randn(Y.size, dtype=torch.complex64, device="cuda")
    c0 = Y.forward(g)
    c1 = on_side(lambda s: Y.forward(g, stream=s))
    assert torch.equal(c0, c1)
    v0 = torch.rand(Y.size, dtype=torch.float64, device="cuda")
    v1 = torch.rand(Y.size, dtype=torch.float64, device="cuda")
    a, b = g.clone(), g.clone()
    for k in range(3):
        step3d(Y, plan, a, v0, v1, math.cos(k), 0.02)
    on_side(lambda s: [step3d(Y, plan, b, v0, v1, math.cos(k), 0.02, stream=s) for k in range(3)])
    assert torch.equal(a, b)


def test_3d_steps_replay_from_a_captured_graph():
    # dsbt_step3d / dsbt_step3d_velocity only enqueue kernels (no memsets, no host
    # synchronisation), so a caller can capture them; replays with eager work in
    # between must each match the eager steps
    from paper_1509_07115_amd import AngularTransform, Plan, step3d, step3d_velocity
    nr, nt, nphi, rmax, dt = 64, 6, 5, 12.8, 0.02
    Y = AngularTransform(nr, nt, nphi)
    plan = Plan(Y.channels(rmax))
    plan.set_potential(np.zeros(plan.elems), dt)
    v0 = torch.rand(Y.size, dtype=torch.float64, device="cuda")
    v1 = torch.rand(Y.size, dtype=torch.float64, device="cuda")
    K, Pz = Y.kinetic(rmax), Y.momentum_pz(rmax)
    g = torch.randn(Y.size, dtype=torch.complex64, device="cuda")
    static = g.clone()
    w1, w2 = torch.empty_like(g), torch.empty_like(g)
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm the library's one-time setup outside the capture
        step3d(Y, plan, g.clone(), v0, v1, 0.3, dt, w1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        step3d(Y, plan, static, v0, v1, 0.3, dt, w1)
        step3d_velocity(Y, plan, static, v0, K, Pz, -0.2, dt, w1, w2)
    ref = g.clone()
    for rep in range(3):
        static.copy_(ref)
        graph.replay()
        eager = ref.clone()
        step3d(Y, plan, eager, v0, v1, 0.3, dt, torch.empty_like(g))
        step3d_velocity(Y, plan, eager, v0, K, Pz, -0.2, dt)
        torch.cuda.synchronize()
        assert torch.equal(static, eager), rep
        ref = eager * (1.0 + rep)
