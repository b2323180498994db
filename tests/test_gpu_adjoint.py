"""GPU reverse mode (project extension) against the oracle's reverse mode.

Same cases as the oracle's finite-difference pins (periodic 2D with damping,
periodic 3D, Dirichlet annulus, Neumann annulus with and without the
projection, Neumann sphere).  The GPU adjoint (checkpointed forward,
recomputed segments, transposed kernels) must reproduce the oracle's
gradients dL/d(mu, lambda), dL/dv0 and dL/du0: FP64 populations to 1e-9
relative (the two sides solve the projection to different CG tolerances,
1e-14 against 1e-15; measured <= 3e-12), FP32 populations to 1e-4 (FP32
rounding accumulated over the steps; measured <= 1e-5).  Different checkpoint
segment lengths give the same result (the recomputation is deterministic).
"""
import numpy as np
import pytest

from parity import check
from test_oracle_adjoint import CASES, _make

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    from paper_2606_20646_amd import tlvlbm
    torch.cuda.set_device(0)
    return tlvlbm


def _solver(T, cfg, precision):
    s = T.Solver(cfg["D"], cfg["n"], cfg["dx"], cfg["dt"], cfg["mu"], cfg["lam"], omega=cfg["omega"],
                 gamma=cfg["gamma"], origin=cfg.get("origin"), periodic_mask=cfg.get("pm", cfg.get("periodic_mask")),
                 proj_every=cfg.get("proj_every", 20), precision=precision, track_u=1,
                 proj_sweeps=cfg.get("proj_sweeps", 20), fibre=cfg.get("fibre"))
    if "phi" in cfg:
        s.set_levelset(cfg["phi"], cfg["bid"])
        for bid, bc in cfg["bcs"].items():
            bc = dict(bc)
            s.set_boundary(bid, bc.pop("type"), **bc)
    return s


def _weights(cfg):
    rng = np.random.default_rng(11)
    D, N = cfg["D"], int(np.prod(cfg["n"]))
    M = D + D * D
    act = (cfg["phi"] <= 0).reshape(-1) if "phi" in cfg else np.ones(N, bool)
    return rng.standard_normal((M, N)) * act, rng.standard_normal((D, N)) * act


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_oracle(T, orc, name, precision, tol):
    _say(f"adjoint {name} {precision}")
    make, n = CASES[name]
    cfg = make()
    wU, wu = _weights(cfg)
    u0 = cfg.get("u0")
    o = _make(cfg, cfg["mu"], cfg["lam"])
    o.set_state(cfg["U0"], u0=u0, dU0=cfg.get("dU0"))
    gm_o, gv_o, g0_o, gd_o = o.adjoint(n, wU, wu, with_dU0=True)
    s = _solver(T, cfg, precision)
    s.set_state(cfg["U0"], u0=u0, dU0=cfg.get("dU0"))
    # the two-call reverse mode: record the run, then the backward pass
    s.adjoint_record(n)
    assert s.stats()["step"] == n
    gm, gv, g0, gd = s.adjoint_backward(wU, wu, grad_dU0=True)
    assert s.stats()["step"] == n
    print(f"mu,lam: gpu {gm} oracle {gm_o}; v0 rel {_rel(gv, gv_o):.2e}; u0 rel {_rel(g0, g0_o):.2e}; "
          f"dU0 rel {_rel(gd, gd_o):.2e}", flush=True)
    assert _rel(gd, gd_o) <= tol
    scale = np.abs(gm_o).max()
    assert np.all(np.abs(gm - gm_o) <= tol * scale)
    assert _rel(gv, gv_o) <= tol
    if np.linalg.norm(g0_o) > 1e-12 * np.linalg.norm(gv_o):
        assert _rel(g0, g0_o) <= tol
    else:
        assert np.linalg.norm(g0) <= tol * np.linalg.norm(gv_o)
    # the context ends at step n with the forward state
    U, u, _ = s.moments()
    Uo, uo, _ = o.moments()
    act = (cfg["phi"] <= 0).reshape(-1) if "phi" in cfg else None
    # exact projection: CG stopped at a residual of 1e-14 (GPU) / 1e-15 (oracle)
    # relative to the larger of |b| and the initial residual, which the
    # random initial displacement of these cases makes large
    ftol = 1e-5 if precision == "fp32" else (1e-12 if cfg.get("proj_sweeps", 20) > 0 else 1e-9)
    check(U, Uo, cfg["D"], ftol, mask=act, label=f"adjoint forward {name} {precision}", pops=o.get_f(), steps=n,
          stress=(cfg["mu"], cfg["lam"], 1.0, cfg["dx"] / cfg["dt"], cfg["omega"]))


@pytest.mark.parametrize("name", ["neumann_annulus_projection", "periodic2d_damped"])
def test_adjoint_segments_agree(T, name):
    _say(f"adjoint segments {name}")
    make, n = CASES[name]
    cfg = make()
    wU, wu = _weights(cfg)
    out = []
    # 0: every step taped in the first pass; -3: three taped final steps
    # and the rest checkpointed; > 0: checkpoints only
    for seg in (0, -3, 1, 4, n):
        s = _solver(T, cfg, "fp64")
        s.set_state(cfg["U0"], u0=cfg.get("u0"), dU0=cfg.get("dU0"))
        out.append(s.adjoint(n, wU, wu, segment=seg))
    for gm, gv, g0 in out[1:]:
        assert np.array_equal(gm, out[0][0])
        assert np.array_equal(gv, out[0][1])
        assert np.array_equal(g0, out[0][2])


def test_record_backward_repeat_and_order(T):
    """The backward pass can be repeated on one record (same gradients bit
    for bit as the one-call reverse mode); any step after the record makes
    the backward refuse."""
    _say("adjoint record/backward repeat neumann_annulus_projection fp64")
    make, n = CASES["neumann_annulus_projection"]
    cfg = make()
    wU, wu = _weights(cfg)
    s = _solver(T, cfg, "fp64")
    s.set_state(cfg["U0"], u0=cfg.get("u0"), dU0=cfg.get("dU0"))
    s.adjoint_record(n)
    a = s.adjoint_backward(wU, wu)
    b = s.adjoint_backward(wU, wu)
    r = _solver(T, cfg, "fp64")
    r.set_state(cfg["U0"], u0=cfg.get("u0"), dU0=cfg.get("dU0"))
    c = r.adjoint(n, wU, wu)
    for x, y, z in zip(a[:3], b[:3], c):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    U1, u1, _ = s.moments()
    U2, u2, _ = r.moments()
    assert np.array_equal(U1, U2) and np.array_equal(u1, u2)
    s.step(1)
    with pytest.raises(T.TlvlbmError) as e:
        s.adjoint_backward(wU, wu)
    assert e.value.code == T.ERR_CALL_ORDER


def test_adjoint_requires_fresh_state(T):
    make, n = CASES["periodic2d_damped"]
    cfg = make()
    s = _solver(T, cfg, "fp64")
    s.set_state(cfg["U0"], dU0=cfg["dU0"])
    s.step(1)
    with pytest.raises(T.TlvlbmError):
        s.adjoint(2, np.ones((6, s.N)))


def test_adjoint_sphere_32(T, orc):
    """Reverse mode on the sphere recipe at 32^3 (+frame), 21 steps with two
    projections, FP64, against the oracle's adjoint."""
    import workloads as W
    _say("adjoint sphere 32^3 fp64 21 steps")
    c = W.config_c5(32)
    cfg = dict(c, pm=0, proj_every=20)
    wU, wu = _weights(cfg)
    o = _make(cfg, cfg["mu"], cfg["lam"])
    o.set_state(cfg["U0"], dU0=cfg["dU0"])
    gm_o, gv_o, g0_o = o.adjoint(21, wU, wu)
    s = _solver(T, cfg, "fp64")
    s.set_state(cfg["U0"], dU0=cfg["dU0"])
    gm, gv, g0 = s.adjoint(21, wU, wu)
    print(f"mu,lam: gpu {gm} oracle {gm_o}; v0 rel {_rel(gv, gv_o):.2e}; u0 rel {_rel(g0, g0_o):.2e}", flush=True)
    assert np.all(np.abs(gm - gm_o) <= 1e-9 * np.abs(gm_o).max())
    assert _rel(gv, gv_o) <= 1e-9
    assert _rel(g0, g0_o) <= 1e-9


def test_autograd_function_matches_adjoint(T):
    """The torch.autograd wrapper returns the reverse mode's gradients."""
    import torch
    _say("autograd wrapper neumann_annulus_projection fp64")
    make, n = CASES["neumann_annulus_projection"]
    cfg = make()
    wU, wu = _weights(cfg)
    D = cfg["D"]
    s = _solver(T, cfg, "fp64")
    mat = torch.tensor([cfg["mu"], cfg["lam"]], dtype=torch.float64, requires_grad=True)
    v0 = torch.tensor(cfg["U0"][:D], dtype=torch.float64, requires_grad=True)
    U, u = T.run_differentiable(s, mat, v0, n, cfg["U0"], dU0=cfg.get("dU0"))
    loss = (torch.from_numpy(wU) * U).sum() + (torch.from_numpy(wu) * u).sum()
    loss.backward()
    r = _solver(T, cfg, "fp64")
    r.set_state(cfg["U0"], dU0=cfg.get("dU0"))
    gm, gv, _ = r.adjoint(n, wU, wu)
    Ur, ur, _ = r.moments()
    assert np.array_equal(U.detach().numpy(), Ur) and np.array_equal(u.detach().numpy(), ur)
    assert np.array_equal(mat.grad.numpy(), gm)
    assert np.array_equal(v0.grad.numpy(), gv)


def test_autograd_with_consistent_initial_gradient(T):
    """Device tensors end to end, with the initial velocity gradient built
    from v0 by a torch difference operator: autograd's dL/dv0 (through
    dL/dv0 and dL/d dv0) matches central differences of runs in which v0 and
    its gradient move together.  The partial dL/dv0 at fixed dv0 does not."""
    import torch
    _say("autograd with dv0 = grad(v0) periodic2d_damped fp64 (device tensors)")
    make, n = CASES["periodic2d_damped"]
    cfg = make()
    D, N = cfg["D"], int(np.prod(cfg["n"]))
    nx, ny = cfg["n"]
    dx = cfg["dx"]
    dev = torch.device("cuda")
    wU, wu = (torch.from_numpy(w).to(dev) for w in _weights(cfg))

    def grad_op(v):  # periodic central differences: [A][i][nodes]
        vv = v.reshape(D, ny, nx)
        gx = (torch.roll(vv, -1, 2) - torch.roll(vv, 1, 2)) / (2 * dx)
        gy = (torch.roll(vv, -1, 1) - torch.roll(vv, 1, 1)) / (2 * dx)
        return torch.stack([gx.reshape(D, N), gy.reshape(D, N)])

    mat = torch.tensor([cfg["mu"], cfg["lam"]], dtype=torch.float64, device=dev)
    s = _solver(T, cfg, "fp64")

    def loss(v, dv=True):
        U, u = T.run_differentiable(s, mat, v, n, cfg["U0"], dU0=cfg["dU0"], dv0=grad_op(v) if dv else None)
        return (wU * U).sum() + (wu * u).sum()

    v0 = torch.tensor(cfg["U0"][:D], device=dev, requires_grad=True)
    loss(v0).backward()
    g_total = v0.grad.clone()
    v1 = torch.tensor(cfg["U0"][:D], device=dev, requires_grad=True)
    loss(v1, dv=False).backward()
    g_partial = v1.grad.clone()
    rng = np.random.default_rng(4)
    delta = torch.from_numpy(rng.standard_normal((D, N))).to(dev)
    base = torch.tensor(cfg["U0"][:D], device=dev)
    with torch.no_grad():
        def L(h):
            return float(loss(base + h * delta))
        h = 1e-3
        d1 = (L(h) - L(-h)) / (2 * h)
        d2 = (L(h / 2) - L(-h / 2)) / h
        fd = (4 * d2 - d1) / 3
    ad = float((g_total * delta).sum())
    ap = float((g_partial * delta).sum())
    print(f"total {ad} partial {ap} fd {fd}", flush=True)
    assert abs(ad - fd) <= 1e-7 * abs(fd)
    assert abs(ap - fd) > 100 * abs(ad - fd)
