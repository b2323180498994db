"""Pins of the oracle's second material law: the neo-Hookean solid of Eq. 62
reinforced by one family of fibres along a unit reference direction a0,
W = W_NH + k1/2 (|F a0|^2 - 1)^2 (the anisotropic extension that the paper's
outlook names, Sec. 6; P = dW/dF, Eq. 4).

- the stress is the energy gradient and the tangent its Hessian (torch
  autograd of the energy written here), with major symmetry;
- at F = I the acoustic tensor (Eq. 19) along the fibre has the longitudinal
  speed^2 lambda + 2 mu + 4 k1 and the shear speed^2 mu; across the fibre the
  neo-Hookean speeds;
- a manufactured finite-strain plane wave of the fibre law (body acceleration
  from tests/refsol.piola_fibre, written independently of the oracle)
  converges at second order at omega = 2 in the full scheme.
"""
import numpy as np
import pytest
import torch

import refsol
import workloads as W


def _W_fibre(F, mu, lam, k1, a0):
    D = F.shape[0]
    J = torch.det(F)
    a = torch.tensor(a0, dtype=torch.float64)
    fa = F @ a
    I4 = (fa * fa).sum()
    return (0.5 * mu * ((F * F).sum() - D) - (mu + 0.5 * lam) * torch.log(J) + 0.25 * lam * (J * J - 1.0)
            + 0.5 * k1 * (I4 - 1.0) ** 2)


def _unit(rng, D):
    a = rng.standard_normal(D)
    return a / np.linalg.norm(a)


def _rand_F(rng, D, scale=0.3):
    while True:
        F = np.eye(D) + scale * rng.standard_normal((D, D))
        if np.linalg.det(F) > 0.2:
            return F


@pytest.mark.parametrize("D", [2, 3])
def test_fibre_stress_is_energy_gradient_and_tangent_its_hessian(orc, D):
    rng = np.random.default_rng(31)
    for _ in range(10):
        F = _rand_F(rng, D)
        a0 = _unit(rng, D)
        mu, lam, k1 = rng.uniform(0.3, 3.0), rng.uniform(0.1, 20.0), rng.uniform(0.1, 5.0)
        Ft = torch.tensor(F, dtype=torch.float64, requires_grad=True)
        (g,) = torch.autograd.grad(_W_fibre(Ft, mu, lam, k1, a0), Ft)
        P = orc.piola_law(F, mu, lam, k1, a0)
        assert np.allclose(P, g.numpy(), rtol=1e-12, atol=1e-12 * np.abs(P).max())
        H = torch.autograd.functional.hessian(lambda X: _W_fibre(X, mu, lam, k1, a0),
                                              torch.tensor(F, dtype=torch.float64)).numpy()
        dF1, dF2 = rng.standard_normal((D, D)), rng.standard_normal((D, D))
        d1 = orc.piola_law_jvp(F, dF1, mu, lam, k1, a0)
        d2 = orc.piola_law_jvp(F, dF2, mu, lam, k1, a0)
        ref = np.einsum("iakb,kb->ia", H, dF1)
        assert np.allclose(d1, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
        assert abs(np.sum(d1 * dF2) - np.sum(d2 * dF1)) < 1e-11 * np.abs(d1).max() * np.abs(dF2).max() * D * D


@pytest.mark.parametrize("D", [2, 3])
def test_fibre_acoustic_tensor_at_reference(orc, D):
    mu, lam, k1 = 1.3, 4.1, 0.7
    a0 = np.zeros(D)
    a0[0] = 1.0

    def Q(n):
        out = np.zeros((D, D))
        for k in range(D):
            dF = np.outer(np.eye(D)[k], n)
            out[:, k] = orc.piola_law_jvp(np.eye(D), dF, mu, lam, k1, a0) @ n
        return out
    ev = np.sort(np.linalg.eigvalsh(Q(a0)))
    assert np.allclose(ev, sorted([lam + 2 * mu + 4 * k1] + [mu] * (D - 1)), rtol=1e-13)
    n = np.zeros(D)
    n[1] = 1.0
    ev = np.sort(np.linalg.eigvalsh(Q(n)))
    assert np.allclose(ev, sorted([lam + 2 * mu] + [mu] * (D - 1)), rtol=1e-13)


def _mms_fibre(orc, N, k1=0.8, a0=(np.cos(0.5), np.sin(0.5))):
    D = 2
    m = refsol.PlaneWaveMMS(D, (1, 1), (1, 0.3), 0.02, 2 * np.pi, 1.0, 2.0, fibre=(k1, np.array(a0)))
    n = [N] * D
    dx = 1 / N
    dt = dx / 10
    X = W.node_coords(n, dx, [0.0] * D)
    s = orc.Sim(D, n, dx, dt, 1.0, 2.0, omega=2.0)
    s.set_fibres(k1, a0)
    U0, u0 = m.fields(X, 0.0)
    s.set_body_force(m.body(X, 0.0))
    s.set_state(U0, u0=u0, dU0=m.gradients(X, 0.0))
    nst = int(round(0.2 / dt))
    for it in range(nst):
        s.set_body_force(m.body(X, it * dt))
        s.step(1)
    U, u, _ = s.moments()
    Ue, ue = m.fields(X, nst * dt)
    Fi = np.eye(D).reshape(-1)[:, None]
    return np.array([np.linalg.norm(U[:D] - Ue[:D]) / np.linalg.norm(Ue[:D]),
                     np.linalg.norm(U[D:] - Ue[D:]) / np.linalg.norm(Ue[D:] - Fi),
                     np.linalg.norm(u - ue) / np.linalg.norm(ue)])


def test_fibre_manufactured_wave_second_order(orc):
    errs = [_mms_fibre(orc, N) for N in (16, 32, 64)]
    orders = [np.log2(e0 / e1) for e0, e1 in zip(errs, errs[1:])]
    assert np.all(orders[0] > 1.75) and np.all(orders[1] > 1.9), (errs, orders)
    # the neo-Hookean scheme with the fibre law's body acceleration is not
    # a solution: the fibre term is in effect
    m = refsol.PlaneWaveMMS(2, (1, 1), (1, 0.3), 0.02, 2 * np.pi, 1.0, 2.0, fibre=(0.8, np.array([np.cos(0.5), np.sin(0.5)])))
    X = W.node_coords([32, 32], 1 / 32, [0.0, 0.0])
    s = orc.Sim(2, [32, 32], 1 / 32, 1 / 320, 1.0, 2.0, omega=2.0)
    U0, u0 = m.fields(X, 0.0)
    s.set_body_force(m.body(X, 0.0))
    s.set_state(U0, u0=u0, dU0=m.gradients(X, 0.0))
    for it in range(64):
        s.set_body_force(m.body(X, it / 320))
        s.step(1)
    U, _, _ = s.moments()
    Ue, _ = m.fields(X, 64 / 320)
    assert np.linalg.norm(U[:2] - Ue[:2]) / np.linalg.norm(Ue[:2]) > 10 * errs[1][0]
