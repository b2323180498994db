"""Degenerate inputs through the C ABI, against the oracle: a level set with
no active node (every step is a no-op), a body of one node whose four
links are all cut (Dirichlet and Neumann closures on every direction; the
traction closure's stencil is the node alone), and zero-step calls."""
import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def T():
    from paper_2606_20646_amd import tlvlbm
    return tlvlbm


def _grid2(n):
    """node coordinates of an n x n grid of spacing 1/n (x fastest)"""
    return (np.tile(np.arange(n), n) + 0.5) / n, (np.repeat(np.arange(n), n) + 0.5) / n


@pytest.mark.parametrize("D", [2, 3])
def test_empty_body(T, orc, D):
    """phi > 0 everywhere: no active node, no cut link; steps, moments and
    the checkpoint calls succeed and leave nothing to compare."""
    n = 16
    N = n ** D
    M = D + D * D
    _say(f"empty body {D}D")
    g = T.Solver(D, (n,) * D, 1 / n, 0.1 / n, 1.0, 2.0, periodic_mask=0, precision="fp64")
    o = orc.Sim(D, (n,) * D, 1 / n, 0.1 / n, 1.0, 2.0, periodic_mask=0)
    U0 = np.zeros((M, N))
    for a in range(D):
        U0[D + a * (D + 1)] = 1.0
    for s in (g, o):
        s.set_levelset(np.ones(N))
        s.set_state(U0)
        s.step(5)
    st = g.stats()
    assert st["active_nodes"] == 0 == o.num_active()
    assert st["cut_links"] == 0 == len(o.links()["node"])
    assert st["step"] == 5 and st["newton_failures"] == 0
    g.moments()
    f, us, step = g.get_state()
    g.put_state(f, us, step)
    g.step(1)
    assert g.stats()["step"] == 6


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
def test_single_node_body(T, orc, kind):
    """One active node at the centre of a 16^2 grid, all four of its links
    cut: the closures supply every incoming population (Dirichlet velocity,
    or a constant nominal traction whose LSQ stencil is the node alone and
    whose projection has one unknown)."""
    n = 16
    X, Y = _grid2(n)
    phi = np.hypot(X - 8.5 / n, Y - 8.5 / n) - 0.3 / n
    kw = dict(gamma=1.0, periodic_mask=0, proj_every=20)
    g = T.Solver(2, (n, n), 1 / n, 0.1 / n, 1.0, 2.0, precision="fp64", **kw)
    o = orc.Sim(2, (n, n), 1 / n, 0.1 / n, 1.0, 2.0, **kw)
    bid = np.ones(n * n, np.uint8)
    for s in (g, o):
        s.set_levelset(phi, bid)
    g.set_boundary(1, kind, a=(0.01, 0.0))
    o.set_bc(1, orc.DIRICHLET if kind == "dirichlet" else orc.NEUMANN, a=(0.01, 0.0))
    U0 = np.zeros((6, n * n))
    U0[2] = U0[5] = 1.0
    _say(f"single-node body {kind}")
    for s in (g, o):
        s.set_state(U0)
        s.step(45)
    Ug, ug, _ = g.moments()
    Uo, uo, _ = o.moments()
    act = phi <= 0
    assert act.sum() == 1 and g.stats()["cut_links"] == 4
    check(Ug, Uo, 2, 1e-12, ug, uo, mask=act, label=f"single node {kind}", pops=o.get_f(), steps=45,
          stress=(1.0, 2.0, 1.0, 10.0, 1.8))
    assert g.stats()["newton_failures"] == 0


def test_zero_steps(T, orc):
    """step(0) changes nothing; a negative count is an invalid argument."""
    n = 16
    X, Y = _grid2(n)
    U0 = np.zeros((6, n * n))
    U0[0] = 1e-3 * np.sin(2 * np.pi * X)
    U0[2] = U0[5] = 1.0
    g = T.Solver(2, (n, n), 1 / n, 0.1 / n, 1.0, 2.0, precision="fp64")
    g.set_state(U0)
    _say("zero steps")
    f0, u0, s0 = g.get_state()
    g.step(0)
    f1, u1, s1 = g.get_state()
    assert s0 == s1 == 0 and np.array_equal(f0, f1)
    with pytest.raises(T.TlvlbmError) as e:
        g.step(-1)
    assert e.value.code == T.ERR_INVALID_ARG
