"""Pins of the oracle's thermal stretch, the thermal distortion through which
the outlook introduces thermoelasticity (Sec. 6): a per-node isotropic
stretch th from the temperature field enters the multiplicative split
F = F_e (th I), with the energy per reference volume th^D W(F / th), so that
P(F) = th^(D-1) P_W(F / th) (P = dPsi/dF, Eq. 4; W of Eq. 62, with fibres).

- the stress is the gradient of that energy and the tangent its Hessian
  (torch autograd of the energy written here);
- th times a rotation is stress free, whatever the law;
- a periodic lattice at rest under a uniform stretch keeps its state, and its
  stress output is the closed form th^(D-1) [mu (1/th - th) + lam/2
  (th^(-2D) - 1) th] I;
- a traction-free disk under a uniform stretch relaxes to the stress-free
  affine expansion F = th I, u = (th - 1)(X - mean X), which the embedded
  scheme (traction closure, LSQ, projection) holds exactly;
- th = 1 everywhere is bit for bit no stretch; values <= 0, a Maxwell branch
  and the reverse mode are refused.
"""
import numpy as np
import pytest
import torch


def _W(F, mu, lam, k1, a0):
    D = F.shape[0]
    J = torch.det(F)
    a = torch.tensor(a0, dtype=torch.float64)
    fa = F @ a
    I4 = (fa * fa).sum()
    return (0.5 * mu * ((F * F).sum() - D) - (mu + 0.5 * lam) * torch.log(J) + 0.25 * lam * (J * J - 1.0)
            + 0.5 * k1 * (I4 - 1.0) ** 2)


def _psi(F, mu, lam, k1, a0, th):
    D = F.shape[0]
    return th ** D * _W(F / th, mu, lam, k1, a0)


def _rand_F(rng, D, scale=0.3):
    while True:
        F = np.eye(D) + scale * rng.standard_normal((D, D))
        if np.linalg.det(F) > 0.2:
            return F


def _rotation(rng, D):
    Qm, R = np.linalg.qr(rng.standard_normal((D, D)))
    Qm = Qm * np.sign(np.diag(R))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] = -Qm[:, 0]
    return Qm


@pytest.mark.parametrize("D", [2, 3])
def test_thermal_stress_is_energy_gradient_and_tangent_its_hessian(orc, D):
    rng = np.random.default_rng(47)
    for _ in range(10):
        F = _rand_F(rng, D)
        a = rng.standard_normal(D)
        a0 = a / np.linalg.norm(a)
        mu, lam = rng.uniform(0.3, 3.0), rng.uniform(0.1, 20.0)
        k1 = rng.choice([0.0, rng.uniform(0.1, 5.0)])
        th = rng.uniform(0.8, 1.3)
        Ft = torch.tensor(F, dtype=torch.float64, requires_grad=True)
        (g,) = torch.autograd.grad(_psi(Ft, mu, lam, k1, a0, th), Ft)
        P = orc.thermal_piola(F, mu, lam, th, k1, a0)
        assert np.allclose(P, g.numpy(), rtol=1e-12, atol=1e-12 * np.abs(P).max())
        H = torch.autograd.functional.hessian(lambda X: _psi(X, mu, lam, k1, a0, th),
                                              torch.tensor(F, dtype=torch.float64)).numpy()
        dF = rng.standard_normal((D, D))
        d = orc.thermal_piola_jvp(F, dF, mu, lam, th, k1, a0)
        ref = np.einsum("iakb,kb->ia", H, dF)
        assert np.allclose(d, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
        # th = 1: the law itself, bit for bit
        assert np.array_equal(orc.thermal_piola(F, mu, lam, 1.0, k1, a0), orc.piola_law(F, mu, lam, k1, a0))


@pytest.mark.parametrize("D", [2, 3])
def test_stretched_rotation_is_stress_free(orc, D):
    rng = np.random.default_rng(5)
    for k1 in (0.0, 2.0):
        for _ in range(5):
            th = rng.uniform(0.7, 1.4)
            Rm = _rotation(rng, D)
            a = rng.standard_normal(D)
            P = orc.thermal_piola(th * Rm, 1.3, 7.0, th, k1, a / np.linalg.norm(a))
            assert np.abs(P).max() < 1e-13


def _grid(n, dx, off=0):
    ix, iy = np.tile(np.arange(n), n), np.repeat(np.arange(n), n)
    return (ix - off + 0.5) * dx, (iy - off + 0.5) * dx


@pytest.mark.parametrize("D", [2, 3])
def test_uniform_stretch_periodic_rest_state(orc, D):
    n, dx, mu, lam, th = 8, 1 / 8, 1.0, 2.0, 1.05
    N = n ** D
    o = orc.Sim(D, (n,) * D, dx, dx / 10, mu, lam)
    U0 = np.zeros((D + D * D, N))
    for a in range(D):
        U0[D + a * (D + 1)] = 1.0
    o.set_thermal(np.full(N, th))
    o.set_state(U0)
    o.step(50)
    U, _, _ = o.moments()
    assert np.abs(U - U0).max() < 1e-14
    P, _ = o.stress()
    p = th ** (D - 1) * (mu * (1 / th - th) + 0.5 * lam * (th ** (-2 * D) - 1.0) * th)
    Pex = np.zeros(D * D)
    Pex[:: D + 1] = p
    assert abs(p) > 0.1
    assert np.abs(P - Pex[:, None]).max() < 1e-13


def _disk(orc, th_field, steps, extra=None):
    N = 32
    n, dx = N + 2, 1 / N
    X, Y = _grid(n, dx, off=1)
    phi = np.hypot(X - 0.5, Y - 0.5) - 0.3
    o = orc.Sim(2, (n, n), dx, dx / 10, 1.0, 2.0, origin=(-dx, -dx), periodic_mask=0, gamma=10.0, proj_every=20)
    o.set_levelset(phi, np.ones(n * n, np.uint8))
    o.set_bc(1, orc.NEUMANN)
    if th_field is not None:
        o.set_thermal(th_field(n * n))
    U0 = np.zeros((6, n * n))
    U0[2] = U0[5] = 1.0
    o.set_state(U0)
    o.step(steps)
    return o, X, Y, phi <= 0


def test_free_disk_relaxes_to_stress_free_expansion(orc):
    th = 1.02
    o, X, Y, act = _disk(orc, lambda N: np.full(N, th), 1600)
    U, u, _ = o.moments()
    Xa = np.stack([X[act], Y[act]])
    ue = (th - 1.0) * (Xa - Xa.mean(axis=1, keepdims=True))
    assert np.abs(U[2:, act] - th * np.array([1.0, 0.0, 0.0, 1.0])[:, None]).max() < 1e-11
    assert np.abs(U[:2, act]).max() < 1e-11
    assert np.abs(u[:, act] - ue).max() < 1e-11
    assert o.stats()["newton_fail"] == 0


def test_unit_stretch_is_no_stretch_and_refusals(orc):
    a, _, _, act = _disk(orc, None, 60)
    b, _, _, _ = _disk(orc, lambda N: np.ones(N), 60)
    assert np.array_equal(a.get_f(), b.get_f())
    with pytest.raises(orc.OracleError):
        b.set_thermal(np.zeros(b.N))
    with pytest.raises(orc.OracleError):
        b.set_viscous(0.5, 1.0)
    with pytest.raises(orc.OracleError):
        b.adjoint(1, dLdu=np.zeros((2, b.N)))
    c = orc.Sim(2, (8, 8), 1 / 8, 1 / 80, 1.0, 2.0)
    c.set_viscous(0.5, 1.0)
    with pytest.raises(orc.OracleError):
        c.set_thermal(np.ones(64))
