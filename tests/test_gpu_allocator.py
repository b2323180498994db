"""Device memory through the caller's allocator (tlvlbm_options.dev_alloc /
dev_free), here torch's caching allocator: every buffer the context keeps
comes from it (torch's allocated-bytes counter grows by at least the two
population buffers and falls back when the context is destroyed), and the
results equal those of a context on hipMalloc bit for bit (forward steps
with cut links and projection, and the reverse mode's arena)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _annulus(T, c, stream, allocator):
    s = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                 origin=c["origin"], periodic_mask=0, proj_every=20, precision="fp64", stream=stream,
                 allocator=allocator)
    s.set_levelset(c["phi"], c["bid"])
    s.set_boundary(1, "dirichlet", ramp="sin2", T_r=2.0, given_as_displacement=True, p_radial=0.05, X0=(0.5, 0.5))
    s.set_boundary(2, "neumann")
    s.set_state(c["U0"])
    return s


def test_context_memory_from_torch_allocator():
    import torch
    from paper_2606_20646_amd import tlvlbm as T
    torch.cuda.set_device(0)
    _say("annulus 48 fp64 on torch's caching allocator")
    stream = torch.cuda.Stream()
    c = W.config_c2(48)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    # torch's allocator behind a ledger of the library's calls
    live = {}
    talloc, tfree = T.torch_allocator(stream)

    def alloc(nbytes, user):
        p = talloc(nbytes, user)
        if p:
            live[p] = nbytes
        return p

    def free(ptr, user):
        live.pop(ptr, None)
        tfree(ptr, user)

    hooks = (T.ALLOC_FN(alloc), T.FREE_FN(free))
    s = _annulus(T, c, stream, hooks)
    grown = torch.cuda.memory_allocated() - base
    assert grown >= 2 * s.population_bytes(), (grown, s.population_bytes())
    s.step(45)
    r = _annulus(T, c, stream.cuda_stream, None)
    r.step(45)
    for a, b in zip(s.moments(), r.moments()):
        assert np.array_equal(a, b)
    # the reverse mode's arena and tables come from the same allocator
    s.set_state(c["U0"])
    r.set_state(c["U0"])
    rng = np.random.default_rng(3)
    act = c["phi"] <= 0
    wu = rng.standard_normal((2, act.size)) * act
    before = torch.cuda.memory_allocated()
    ga = s.adjoint(25, None, wu)
    assert torch.cuda.memory_allocated() > before
    gb = r.adjoint(25, None, wu)
    for a, b in zip(ga, gb):
        assert np.array_equal(a, b)
    s.close()
    r.close()
    torch.cuda.synchronize()
    assert not live, f"blocks not returned: {sorted(live.values())}"
    assert torch.cuda.memory_allocated() == base


def test_allocator_needs_both_hooks():
    from paper_2606_20646_amd import tlvlbm as T
    c = W.config_c1()
    alloc, _ = T.torch_allocator()
    with pytest.raises(T.TlvlbmError) as e:
        T.Solver(2, c["n"], c["dx"], c["dt"], 1.0, 2.0, allocator=(alloc, T.FREE_FN()))
    assert e.value.code == T.ERR_INVALID_ARG
