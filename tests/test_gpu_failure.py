"""The failure path of the traction closure, on both sides.

One instance of the batched random-hole recipe drawn without the redraw of
narrow ligaments (instance 54 at 64^2 cells: two holes 0.0023 apart, a
sub-cell sliver of material) drives the local Newton solve of a Neumann cut
link (Sec. 3.4, Eqs. 53-56) to an inadmissible root (det F_b <= 0).  The
oracle and the GPU library (FP64) must both report it as ERR_NEWTON at the
same step, and leave the error sticky until a new state is set."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

K, N = 54, 64


def _oracle(c):
    from oracle import oracle as O
    kinds = {"dirichlet": O.DIRICHLET, "neumann": O.NEUMANN}
    ramps = {"const": O.RAMP_CONST, "sin2": O.RAMP_SIN2}
    o = O.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
              origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"])
    o.set_levelset(c["phi"], c["bid"])
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        t = kinds[bc.pop("type")]
        if "ramp" in bc:
            bc["ramp"] = ramps[bc["ramp"]]
        o.set_bc(bid, t, **bc)
    o.set_state(c["U0"])
    return o


def test_sliver_newton_failure_same_step():
    from oracle import oracle as O
    from paper_2606_20646_amd import tlvlbm as T
    print(f"[gpu-case] sliver instance {K} at {N}^2, FP64", flush=True)
    c = W.config_c4_instance(K, N=N, redraw=False)
    o = _oracle(c)
    with pytest.raises(O.OracleError) as e:
        o.step(c["steps"])
    assert e.value.code == 5  # ORC_ERR_NEWTON
    fail_orc = o.stats()["step"]
    g = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                 origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"], precision="fp64")
    g.set_levelset(c["phi"], c["bid"])
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        g.set_boundary(bid, bc.pop("type"), **bc)
    g.set_state(c["U0"])
    fail_gpu = None
    for k in range(c["steps"]):
        try:
            g.step(1)
        except T.TlvlbmError as err:
            assert err.code == T.ERR_NEWTON
            fail_gpu = g.stats()["step"]
            break
    print(f"ERR_NEWTON at step {fail_orc} (oracle), {fail_gpu} (GPU)", flush=True)
    assert fail_gpu == fail_orc
    # sticky until a new state
    with pytest.raises(T.TlvlbmError) as err:
        g.step(1)
    assert err.value.code == T.ERR_NEWTON
    g.set_state(c["U0"])
    g.step(10)
    # the recipe's redraw removes the sliver: the same instance runs through
    c2 = W.config_c4_instance(K, N=N)
    assert not np.array_equal(c2["hole_centres"], c["hole_centres"])
