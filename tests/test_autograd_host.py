"""Host logic of the adjoint propagation (checkpoint segments, step order,
strength indexing) with a CPU stand-in for the plan built from the oracle,
checked against torch's own autograd through the dense FP64 step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dsbt as odsbt
from oracle import tdse
from paper_1509_07115_amd.autograd import propagate


class OraclePlan:
    """The two Plan methods the propagation uses, on CPU complex128 tensors."""

    def __init__(self, channels, V, dt):
        self.channels, self.V, self.dt = channels, V, dt
        self.E = {off: tdse.kinetic_energies(N, rmax, ell) for N, ell, rmax, off in channels}
        self.calls = []

    def kinetic_step(self, psi, nsteps, s=None, adjoint=False, graph=False):
        self.calls.append(("step", nsteps, adjoint))
        return self._steps(psi, s[:nsteps], adjoint)

    def _steps(self, psi, s, adjoint=False):
        nsteps = len(s)
        x = psi.numpy()
        sv = s.numpy().astype(np.float64)
        order = range(nsteps - 1, -1, -1) if adjoint else range(nsteps)
        for N, ell, _, off in self.channels:
            seg = x[off:off + N].copy()
            for t in order:
                seg = tdse.step(seg, ell, self.V[off:off + N], self.E[off], self.dt, sv[t], adjoint=adjoint)
            x[off:off + N] = seg
        return psi

    def step_grad_s(self, psi_t, psi_t1, lam_t, lam_t1, out):
        a, b, c, d = (v.numpy() for v in (psi_t, psi_t1, lam_t, lam_t1))
        out[0] = 0.5 * self.dt * float(np.sum(self.V * (np.conj(d) * b + np.conj(c) * a).imag))
        return out

    def adjoint_segment(self, psi_a, nsteps, s, lam, gs, graph=False):
        """The library's segment call: recompute psi_a .. psi_a+n, then
        lam_t = U_t^H lam_t+1 and gs[t - a] for t = a+n-1 .. a."""
        self.calls.append(("segment", nsteps, graph))
        states = [psi_a.clone()]
        for t in range(nsteps):
            x = states[-1].clone()
            self._steps(x, s[t:t + 1])
            states.append(x)
        for t in range(nsteps - 1, -1, -1):
            lam_next = lam.clone()
            self._steps(lam, s[t:t + 1], adjoint=True)
            self.step_grad_s(states[t], states[t + 1], lam, lam_next, gs[t:t + 1])
        return lam


def _case(seed=0):
    channels, off = [], 0
    for N, ell in ((32, 0), (32, 3), (64, 2)):
        channels.append((N, ell, 0.25 * N, off))
        off += N + 3                      # gaps between channels
    rng = np.random.default_rng(seed)
    V = rng.uniform(-1.0, 1.0, off)
    psi0 = rng.standard_normal(off) + 1j * rng.standard_normal(off)
    phi = rng.standard_normal(off) + 1j * rng.standard_normal(off)
    for x in (psi0, phi):
        mask = np.zeros(off, bool)
        for N, _, _, o in channels:
            mask[o:o + N] = True
        x[~mask] = 0.0
        x /= np.linalg.norm(x)
    return channels, V, psi0, phi


def _dense_torch_grads(channels, V, dt, psi0, phi, s):
    """L = |<phi|psi_n>|^2 through dense per-channel matrices, differentiated by torch."""
    p0 = torch.tensor(psi0, requires_grad=True)
    st = torch.tensor(s, requires_grad=True)
    out = []
    for N, ell, rmax, off in channels:
        B = torch.tensor(odsbt.dsbt_matrix(N, ell), dtype=torch.complex128)
        E = torch.tensor(tdse.kinetic_energies(N, rmax, ell))
        v = torch.tensor(V[off:off + N])
        x = p0[off:off + N]
        for t in range(len(s)):
            pv = torch.exp(-0.5j * dt * st[t] * v)
            x = pv * (B.T @ (torch.exp(-1j * dt * E) * (B @ (pv * x))))
        out.append(torch.vdot(torch.tensor(phi[off:off + N]), x))
    z = sum(out)
    L = (z * z.conj()).real
    L.backward()
    return L.item(), p0.grad.numpy(), st.grad.numpy()


@pytest.mark.parametrize("nsteps,every", [(7, 3), (6, 3), (5, 1), (4, 10)])
def test_checkpointed_adjoint_matches_torch_autograd(nsteps, every):
    channels, V, psi0, phi = _case()
    dt = 0.05
    s = np.random.default_rng(5).uniform(0.9, 1.1, nsteps)
    plan = OraclePlan(channels, V, dt)
    p0 = torch.tensor(psi0, requires_grad=True)
    st = torch.tensor(s, dtype=torch.float32, requires_grad=True)
    psi_n = propagate(plan, p0, st, checkpoint_every=every)
    z = torch.vdot(torch.tensor(phi), psi_n)
    L = (z * z.conj()).real
    L.backward()
    # the stand-in plan sees float32 strengths, as the library does
    Lr, gp, gs = _dense_torch_grads(channels, V, dt, psi0, phi, s.astype(np.float32).astype(np.float64))
    assert abs(L.item() - Lr) < 1e-12
    assert np.max(np.abs(p0.grad.numpy() - gp)) < 1e-12
    assert np.max(np.abs(st.grad.numpy().astype(np.float64) - gs)) < 1e-6 * max(1.0, np.max(np.abs(gs)))
    # forward: one multi-step call per segment; backward: one segment call per
    # segment, last segment first
    nseg = -(-nsteps // every)
    fwd = plan.calls[:nseg]
    assert all(c[0] == "step" and not c[2] for c in fwd)
    assert sum(c[1] for c in fwd) == nsteps
    bwd = plan.calls[nseg:]
    assert [c[0] for c in bwd] == ["segment"] * nseg
    assert [c[1] for c in bwd] == [min(every, nsteps - a) for a in range(0, nsteps, every)][::-1]


def test_gradient_matches_oracle_adjoint():
    channels, V, psi0, phi = _case(seed=4)
    N, ell, rmax, off = channels[1]
    seg = slice(off, off + N)
    dt, s = 0.05, np.random.default_rng(6).uniform(0.9, 1.1, 5).astype(np.float32).astype(np.float64)
    phi1 = np.zeros_like(phi)
    phi1[seg] = phi[seg] / np.linalg.norm(phi[seg])
    plan = OraclePlan(channels, V, dt)
    p0 = torch.tensor(psi0, requires_grad=True)
    st = torch.tensor(s, requires_grad=True)
    z = torch.vdot(torch.tensor(phi1), propagate(plan, p0, st, checkpoint_every=2))
    ((z * z.conj()).real).backward()
    E = tdse.kinetic_energies(N, rmax, ell)
    L, gpsi, gs = tdse.loss_and_grad(psi0[seg], phi1[seg], ell, V[seg], E, dt, s)
    assert np.max(np.abs(p0.grad.numpy()[seg] - gpsi)) < 1e-12
    # channels outside the support of phi get no gradient
    rest = np.ones(len(psi0), bool)
    rest[seg] = False
    assert np.max(np.abs(p0.grad.numpy()[rest])) == 0.0
    assert np.max(np.abs(st.grad.numpy() - gs)) < 1e-12


def test_rejects_bad_arguments():
    plan = OraclePlan([(32, 0, 8.0, 0)], np.zeros(32), 0.1)
    p0 = torch.zeros(32, dtype=torch.complex128)
    with pytest.raises(ValueError):
        propagate(plan, p0, torch.ones(3), checkpoint_every=0)
    with pytest.raises(ValueError):
        propagate(plan, p0, torch.ones(0))
