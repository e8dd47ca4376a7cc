"""Pins of the oracle's generalized iteration with per-iteration phases (CPU only).

The paper fixes both phases at pi; the generalization (phase phi_j on the marked amplitudes, diffusion
D(theta) = (1 - e^{i theta}) |psi><psi| - I) is this project's convention.  It is pinned by:
  - phi = theta = pi reproducing the pinned Algorithm 3 + Eq. 2 path;
  - dense matrices built from the definition (torch complex128 on the CPU), with torch autograd giving
    the reference gradient at n <= 6;
  - central finite differences of the oracle's own loss;
  - a two-amplitude reduction of the uniform-start dynamics in 50-digit arithmetic (mpmath);
  - the inverse and unitarity identities D(theta)^-1 = D(-theta), O(phi)^-1 = O(-phi), unit norm;
  - the tangent (forward-mode) and the stored-state adjoint gradients agreeing with each other.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads


def schedule(K: int, seed: int, spread: float = 0.1):
    phi, theta = workloads.phase_schedule(K, seed, spread)
    return phi[0], theta[0]


def dense_loss_and_grad(n, marks, phi, theta):
    """The definition as matrices: O = diag(e^{i phi} on marked, 1 else), D = (1 - e^{i theta}) J / N - I,
    c_K = prod_j D_j O_j c_0, L = 1 - sum_marked |c|^2; torch autograd for dL/dphi, dL/dtheta."""
    import torch

    N = 1 << n
    ph = torch.tensor(np.asarray(phi), dtype=torch.float64, requires_grad=True)
    th = torch.tensor(np.asarray(theta), dtype=torch.float64, requires_grad=True)
    mask = torch.zeros(N, dtype=torch.complex128)
    mask[list(marks)] = 1.0
    J = torch.ones(N, N, dtype=torch.complex128) / N
    eye = torch.eye(N, dtype=torch.complex128)
    c = torch.full((N,), 1.0 / math.sqrt(N), dtype=torch.complex128)
    for j in range(len(phi)):
        o_diag = 1.0 + mask * (torch.exp(1j * ph[j].to(torch.complex128)) - 1.0)
        O = torch.diag(o_diag)
        D = (1.0 - torch.exp(1j * th[j].to(torch.complex128))) * J - eye
        c = D @ (O @ c)
    loss = 1.0 - torch.sum(torch.abs(c[list(marks)]) ** 2)
    loss.backward()
    return c.detach().numpy(), float(loss.detach()), ph.grad.numpy().copy(), th.grad.numpy().copy()


def test_phases_at_pi_are_the_standard_iteration(orc):
    for n, marks, K in [(3, [5], 2), (7, [0, 9, 100], 6), (10, [1023], 25)]:
        want = orc.search(n, marks, K)
        got = orc.phase_search(n, marks, [math.pi] * K, [math.pi] * K)
        # e^{i pi} carries sin(pi) = 1.2e-16 in binary64: the difference stays at rounding level
        assert np.max(np.abs(got - want)) < 1e-14


def test_fig2_through_the_generalized_iteration(orc):
    psi = orc.phase_search(3, [5], [math.pi] * 2, [math.pi] * 2)
    assert abs(abs(psi[5]) ** 2 - 121 / 128) < 1e-15
    assert abs(orc.phase_loss(psi, [5]) - 7 / 128) < 1e-15


@pytest.mark.parametrize("n,marks,K,seed", [(3, [2], 3, 1), (5, [1, 30], 5, 2), (6, [3, 17, 40], 8, 3)])
def test_dense_matrices_and_torch_autograd(orc, n, marks, K, seed):
    phi, theta = schedule(K, seed, spread=0.3)
    c, loss, gphi, gtheta = dense_loss_and_grad(n, marks, phi, theta)
    psi = orc.phase_search(n, marks, phi, theta)
    assert np.max(np.abs(psi - c)) < 1e-14
    assert abs(orc.phase_loss(psi, marks) - loss) < 1e-14
    for grad in (orc.phase_grad_tangent, orc.phase_grad_adjoint):
        dphi, dtheta = grad(n, marks, phi, theta)
        assert np.max(np.abs(dphi - gphi)) < 1e-13, grad.__name__
        assert np.max(np.abs(dtheta - gtheta)) < 1e-13, grad.__name__


def test_central_finite_differences(orc):
    n, marks, K = 6, [3, 17, 40], 16
    phi, theta = schedule(K, 11)
    dphi, dtheta = orc.phase_grad_adjoint(n, marks, phi, theta)
    h = 1e-5

    def loss(ph, th):
        return orc.phase_loss(orc.phase_search(n, marks, ph, th), marks)

    for j in range(K):
        for vec, grad in ((phi, dphi), (theta, dtheta)):
            up, dn = vec.copy(), vec.copy()
            up[j] += h
            dn[j] -= h
            if vec is phi:
                fd = (loss(up, theta) - loss(dn, theta)) / (2 * h)
            else:
                fd = (loss(phi, up) - loss(phi, dn)) / (2 * h)
            # truncation ~ h^2 |L'''| / 6 and cancellation ~ 1e-16 / h: both below 1e-9 here
            assert abs(fd - grad[j]) < 1e-8, (j, fd, grad[j])


def test_two_amplitude_reduction_in_50_digits(orc):
    """From the uniform start every marked amplitude equals a and every unmarked one b; the iteration
    maps (a, b) by the same two operators restricted to that plane."""
    import mpmath

    mpmath.mp.dps = 50
    n, marks, K = 12, [7, 1000, 2049, 4000], 30
    M, N = len(marks), 1 << n
    phi, theta = schedule(K, 5, spread=0.5)
    a = b = mpmath.mpf(1) / mpmath.sqrt(N)
    for j in range(K):
        ya = mpmath.expjpi(mpmath.mpf(float(phi[j])) / mpmath.pi) * a
        mean = (M * ya + (N - M) * b) / N
        f = (1 - mpmath.expjpi(mpmath.mpf(float(theta[j])) / mpmath.pi)) * mean
        a, b = f - ya, f - b
    psi = orc.phase_search(n, marks, phi, theta)
    mask = np.zeros(N, dtype=bool)
    mask[marks] = True
    assert np.max(np.abs(psi[mask] - complex(a))) < 1e-15
    assert np.max(np.abs(psi[~mask] - complex(b))) < 1e-15
    assert abs(orc.phase_loss(psi, marks) - float(1 - M * abs(a) ** 2)) < 1e-14


def test_inverses_and_unitarity(orc):
    n = 7
    psi0 = workloads.random_state(n, 77)
    marks = [0, 5, 64, 127]
    for ang in (0.3, math.pi, -2.0):
        psi = orc.phase_diffusion(psi0.copy(), ang)
        assert abs(np.linalg.norm(psi) - 1.0) < 1e-14
        back = orc.phase_diffusion(psi, -ang)
        assert np.max(np.abs(back - psi0)) < 1e-14
        psi = orc.phase_oracle(psi0.copy(), marks, ang)
        assert np.max(np.abs(orc.phase_oracle(psi, marks, -ang) - psi0)) < 1e-15
    phi, theta = schedule(20, 9, spread=1.0)
    assert abs(np.linalg.norm(orc.phase_search(9, marks, phi, theta)) - 1.0) < 1e-13


def test_tangent_and_adjoint_agree(orc):
    for n, marks, K, seed in [(4, [15], 12, 21), (9, [1, 2, 3], 20, 22), (11, [2047, 5], 9, 23)]:
        phi, theta = schedule(K, seed)
        t = orc.phase_grad_tangent(n, marks, phi, theta)
        a = orc.phase_grad_adjoint(n, marks, phi, theta)
        assert np.max(np.abs(t[0] - a[0])) < 1e-13 and np.max(np.abs(t[1] - a[1])) < 1e-13


def test_zero_gradient_for_empty_marked_set(orc):
    """With no marked index the loss is identically 1."""
    phi, theta = schedule(6, 4)
    for grad in (orc.phase_grad_tangent, orc.phase_grad_adjoint):
        dphi, dtheta = grad(5, [], phi, theta)
        assert np.all(dphi == 0.0) and np.max(np.abs(dtheta)) < 1e-16
