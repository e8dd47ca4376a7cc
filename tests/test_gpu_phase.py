"""GPU parity of the generalized iteration with per-iteration phases and of its adjoint gradient
(grover_phase_*), against the oracle (binary64, states kept for the reverse sweep) and, at n = 6, against
dense complex128 matrices differentiated by torch autograd.

Tolerances, derived from the arithmetic (u = 2^-24, complex64 storage; binary64 sums and element math):
  - every stored state is rounded once per iteration (2-norm error <= sqrt(2) u) and the steps are
    unitary, so after k iterations the state is within e_f(k) = k sqrt(2) u of the exact one, and the loss
    within 2 e_f(K) + e_f(K)^2;
  - the reverse sweep rebuilds a state from the next one with the inverse steps, each rounding again, and
    re-reads it from a checkpoint every `every` iterations: its error stays below e_f(K) + every sqrt(2) u;
    the adjoint state (norm <= |g|) picks up sqrt(2) u |g| per step;
  - each gradient entry is 2 Re <lambda, (dU/dp) c> with ||dU/dp|| <= 1, so its error is at most
    2 |g| ((K + 1) sqrt(2) u + 2 e_f(K) + every sqrt(2) u).
A factor 2 of margin is applied to each bound.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def forward_bound(K: int) -> float:
    e = K * math.sqrt(2.0) * U
    return 2.0 * e


def loss_bound(K: int) -> float:
    e = forward_bound(K) / 2.0
    return 2.0 * (2.0 * e + e * e) + 1e-15


def grad_bound(K: int, every: int, g: float = 1.0) -> float:
    e = K * math.sqrt(2.0) * U
    return 2.0 * 2.0 * abs(g) * ((K + 1) * math.sqrt(2.0) * U + 2.0 * e + every * math.sqrt(2.0) * U) + 1e-15


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def cuda(a):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


CASES = [  # (n, marks, K, B, every, team or 0 for the default)
    (6, [3, 17, 40], 16, 3, 4, 0),
    (12, list(range(2000, 2012)) + [5, 4095], 20, 2, 5, 0),
    (15, [7, 20000], 10, 2, 1, 2),
    (15, [32767], 10, 2, 10, 4),
    (17, [1, 65536, 131071], 9, 1, 3, 4),
    (16, [], 6, 2, 2, 1),
]


@pytest.mark.parametrize("form", ["streamed", "held"])
@pytest.mark.parametrize("n,marks,K,B,every,team", CASES)
def test_forward_and_gradient_match_oracle(G, orc, n, marks, K, B, every, team, form):
    """Both forms: states streamed from memory each iteration (team = workgroups per schedule, 0 for the
    default) or held on chip by teams sized from the state (`team` unused)."""
    phi, theta = workloads.phase_schedule(K, seed=100 + n, spread=0.3, batch=B)
    g = np.array([1.0, -0.5, 2.0][:B])
    eng = G.GroverPhase(n, marks, K, batch=B, checkpoint_every=every)
    assert eng.query(G.grover.PQ_EVERY) == every
    assert eng.query(G.grover.PQ_CHECKPOINTS) == (K - 1) // every
    assert eng.query(G.grover.PQ_FORM) == G.grover.GROVER_PHASE_FORM_HELD  # the default when it fits
    eng.set_form(form)
    assert eng.query(G.grover.PQ_FORM) == (G.grover.GROVER_PHASE_FORM_HELD if form == "held"
                                           else G.grover.GROVER_PHASE_FORM_STREAMED)
    # the held teams: the power of two of workgroups whose threads hold 16 vectors (forward) or 8 + 8
    nvec = 1 << (n - 1)
    assert eng.query(G.grover.PQ_HELD_TEAM_F) == max(1, 1 << max(0, (nvec - 1).bit_length() - 14))
    assert eng.query(G.grover.PQ_HELD_TEAM_A) == max(1, 1 << max(0, (nvec - 1).bit_length() - 13))
    if team:
        G.grover_phase_set_team(eng.p, team)
    loss = eng.forward(cuda(phi), cuda(theta))
    eng.sync()
    loss = loss.cpu().numpy()
    for b in range(B):
        want = orc.phase_search(n, marks, phi[b], theta[b])
        got = eng.read_state(b).astype(np.complex128)
        assert np.max(np.abs(got - want)) <= forward_bound(K), (b, np.max(np.abs(got - want)))
        assert abs(loss[b] - orc.phase_loss(want, marks)) <= loss_bound(K), b
    dphi, dtheta = eng.backward(cuda(g))
    eng.sync()
    dphi, dtheta = dphi.cpu().numpy(), dtheta.cpu().numpy()
    for b in range(B):
        wphi, wtheta = orc.phase_grad_adjoint(n, marks, phi[b], theta[b])
        tol = grad_bound(K, every, g[b])
        assert np.max(np.abs(dphi[b] - g[b] * wphi)) <= tol, (b, np.max(np.abs(dphi[b] - g[b] * wphi)), tol)
        assert np.max(np.abs(dtheta[b] - g[b] * wtheta)) <= tol, (b, np.max(np.abs(dtheta[b] - g[b] * wtheta)), tol)
    # after the sweep the states are back at the uniform superposition (re-read from the start)
    amp = np.float32(orc.uniform_amplitude(n))
    assert np.all(eng.read_state(0) == np.complex64(amp))
    eng.close()


@pytest.mark.parametrize("form", ["streamed", "held"])
@pytest.mark.parametrize("n,marks,K,every", [(22, [1, 4000000], 3, 1), (1, [1], 3, 2), (2, [0, 3], 4, 1)])
def test_extreme_sizes_in_both_forms(G, orc, n, marks, K, every, form):
    """The largest held state (n = 22: forward teams of 128 workgroups and adjoint teams of the whole grid,
    so the team barrier gathers over several waves) and the smallest ones (one or two vectors)."""
    phi, theta = workloads.phase_schedule(K, seed=300 + n, spread=0.3, batch=1)
    eng = G.GroverPhase(n, marks, K, batch=1, checkpoint_every=every)
    if form == "held" and eng.query(G.grover.PQ_HELD_TEAM_F) == 0:
        eng.close()
        pytest.skip("the grid is too small to hold this state")
    eng.set_form(form)
    loss = eng.forward(cuda(phi), cuda(theta))
    eng.sync()
    want = orc.phase_search(n, marks, phi[0], theta[0])
    got = eng.read_state(0).astype(np.complex128)
    assert np.max(np.abs(got - want)) <= forward_bound(K)
    assert abs(float(loss.cpu()[0]) - orc.phase_loss(want, marks)) <= loss_bound(K)
    dphi, dtheta = eng.backward(cuda([1.0]))
    eng.sync()
    wphi, wtheta = orc.phase_grad_adjoint(n, marks, phi[0], theta[0])
    tol = grad_bound(K, every)
    assert np.max(np.abs(dphi.cpu().numpy()[0] - wphi)) <= tol
    assert np.max(np.abs(dtheta.cpu().numpy()[0] - wtheta)) <= tol
    eng.close()


def test_dense_torch_autograd_at_n6(G):
    from test_oracle_phase import dense_loss_and_grad

    n, marks, K = 6, [3, 17, 40], 16
    phi, theta = workloads.phase_schedule(K, seed=3, spread=0.3, batch=1)
    _, loss, gphi, gtheta = dense_loss_and_grad(n, marks, phi[0], theta[0])
    eng = G.GroverPhase(n, marks, K, batch=1)
    ph, th = cuda(phi).requires_grad_(), cuda(theta).requires_grad_()
    out = eng.loss(ph, th)
    out.sum().backward()
    assert abs(float(out.detach().cpu()[0]) - loss) <= loss_bound(K)
    tol = grad_bound(K, eng.query(G.grover.PQ_EVERY))
    assert np.max(np.abs(ph.grad.cpu().numpy()[0] - gphi)) <= tol
    assert np.max(np.abs(th.grad.cpu().numpy()[0] - gtheta)) <= tol
    eng.close()


def test_autograd_scales_with_the_upstream_gradient_and_checks_order(G, orc):
    import torch

    n, marks, K, B = 10, [1, 500, 1023], 12, 4
    phi, theta = workloads.phase_schedule(K, seed=77, spread=0.2, batch=B)
    eng = G.GroverPhase(n, marks, K, batch=B)
    ph, th = cuda(phi).requires_grad_(), cuda(theta).requires_grad_()
    w = torch.tensor([1.0, 2.0, -1.0, 0.0], dtype=torch.float64, device="cuda")
    (eng.loss(ph, th) * w).sum().backward()
    for b in range(B):
        wphi, wtheta = orc.phase_grad_adjoint(n, marks, phi[b], theta[b])
        tol = grad_bound(K, eng.query(G.grover.PQ_EVERY), float(w[b]))
        assert np.max(np.abs(ph.grad[b].cpu().numpy() - float(w[b]) * wphi)) <= tol
        assert np.max(np.abs(th.grad[b].cpu().numpy() - float(w[b]) * wtheta)) <= tol
    # a forward run between forward and backward invalidates the first graph's checkpoints
    out = eng.loss(ph, th)
    eng.forward(cuda(phi), cuda(theta))
    with pytest.raises(RuntimeError):
        out.sum().backward()
    eng.close()


def test_backward_needs_a_forward_run(G):
    n, marks, K = 8, [9], 5
    phi, theta = workloads.phase_schedule(K, seed=1, batch=1)
    eng = G.GroverPhase(n, marks, K, batch=1)
    with pytest.raises(G.GroverError):
        eng.backward(cuda([1.0]))
    eng.forward(cuda(phi), cuda(theta))
    eng.backward(cuda([1.0]))
    with pytest.raises(G.GroverError):
        eng.backward(cuda([1.0]))
    eng.sync()
    with pytest.raises(G.GroverError):
        G.grover_phase_set_team(eng.p, 0)
    eng.close()


def test_phases_at_pi_reproduce_the_standard_search(G, orc):
    n, marks, K = 14, [100, 9000], 40
    eng = G.GroverPhase(n, marks, K, batch=2)
    ph = np.full((2, K), math.pi)
    loss = eng.forward(cuda(ph), cuda(ph)).cpu().numpy()
    eng.sync()
    want = orc.search(n, marks, K)
    assert np.max(np.abs(eng.read_state(1).astype(np.complex128) - want)) <= forward_bound(K)
    assert abs(loss[0] - (1.0 - sum(abs(want[i]) ** 2 for i in marks))) <= loss_bound(K)
    eng.close()


def test_team_sizes_agree_and_runs_reproduce(G):
    n, marks, K, B = 16, [12, 40000], 8, 2
    phi, theta = workloads.phase_schedule(K, seed=8, spread=0.3, batch=B)
    results = {}
    for team in (1, 2, 4, "held"):
        eng = G.GroverPhase(n, marks, K, batch=B)
        if team == "held":
            eng.set_form("held")
        else:
            eng.set_form("streamed")
            G.grover_phase_set_team(eng.p, team)
        runs = []
        for _ in range(2):
            loss = eng.forward(cuda(phi), cuda(theta))
            dphi, dtheta = eng.backward(cuda([1.0, 1.0]))
            eng.sync()
            runs.append((loss.cpu().numpy(), dphi.cpu().numpy(), dtheta.cpu().numpy()))
        for a, b in zip(runs[0], runs[1]):
            assert np.array_equal(a, b), team
        results[team] = runs[0]
        eng.close()
    tol = grad_bound(K, 3)
    for team in (2, 4, "held"):
        assert np.max(np.abs(results[team][0] - results[1][0])) <= 2 * loss_bound(K)
        assert np.max(np.abs(results[team][1] - results[1][1])) <= 2 * tol
        assert np.max(np.abs(results[team][2] - results[1][2])) <= 2 * tol


def test_forms_mix_between_forward_and_backward(G, orc):
    """Both forms keep the same checkpoints and final state: a backward run in either form after a forward
    run in either form gives the oracle's gradient."""
    n, marks, K, B, every = 14, [5, 9000, 16383], 12, 2, 3
    phi, theta = workloads.phase_schedule(K, seed=21, spread=0.3, batch=B)
    want = [orc.phase_grad_adjoint(n, marks, phi[b], theta[b]) for b in range(B)]
    for f_form, b_form in (("held", "streamed"), ("streamed", "held")):
        eng = G.GroverPhase(n, marks, K, batch=B, checkpoint_every=every)
        eng.set_form(f_form)
        loss = eng.forward(cuda(phi), cuda(theta))
        eng.set_form(b_form)
        dphi, dtheta = eng.backward(cuda([1.0, 1.0]))
        eng.sync()
        loss, dphi, dtheta = loss.cpu().numpy(), dphi.cpu().numpy(), dtheta.cpu().numpy()
        for b in range(B):
            ref = orc.phase_search(n, marks, phi[b], theta[b])
            assert abs(loss[b] - orc.phase_loss(ref, marks)) <= loss_bound(K)
            assert np.max(np.abs(dphi[b] - want[b][0])) <= grad_bound(K, every)
            assert np.max(np.abs(dtheta[b] - want[b][1])) <= grad_bound(K, every)
        assert np.all(eng.read_state(1) == np.complex64(np.float32(orc.uniform_amplitude(n))))
        eng.close()


def test_form_selection_limits(G):
    eng = G.GroverPhase(8, [3], 4, batch=1)
    with pytest.raises(G.GroverError) as e:
        G.grover_phase_set_form(eng.p, 3)
    assert e.value.status == G.grover.GROVER_E_INVAL
    eng.set_form("streamed")
    assert eng.query(G.grover.PQ_FORM) == G.grover.GROVER_PHASE_FORM_STREAMED
    eng.set_form("auto")
    assert eng.query(G.grover.PQ_FORM) == G.grover.GROVER_PHASE_FORM_HELD
    eng.close()
    # n = 23: the adjoint's team of 2^22 / 8192 = 512 workgroups exceeds the grid, so only streaming is left
    big = G.GroverPhase(23, [1], 1, batch=1)
    if big.query(G.grover.PQ_GRID) < 512:
        assert big.query(G.grover.PQ_HELD_TEAM_F) == 0 and big.query(G.grover.PQ_HELD_TEAM_A) == 0
        assert big.query(G.grover.PQ_FORM) == G.grover.GROVER_PHASE_FORM_STREAMED
        with pytest.raises(G.GroverError) as e:
            big.set_form("held")
        assert e.value.status == G.grover.GROVER_E_UNSUPPORTED
    big.close()


@pytest.mark.parametrize("form", ["streamed", "held"])
def test_barrier_timeout_is_reported(G, monkeypatch, form):
    monkeypatch.setenv("GROVER_BARRIER_TIMEOUT_MS", "0")
    n, marks, K = 17, [5], 6
    phi, theta = workloads.phase_schedule(K, seed=2, batch=1)
    eng = G.GroverPhase(n, marks, K, batch=1)
    eng.set_form(form)
    G.grover_phase_set_team(eng.p, 8)  # streamed: 8 workgroups; held: 4 from the state size
    eng.forward(cuda(phi), cuda(theta))
    with pytest.raises(G.GroverError) as e:
        eng.sync()
    assert e.value.status == G.grover.GROVER_E_TIMEOUT
    eng.close()
