"""The allocation-free entry point tlvlbm_cut_links_noalloc against the
allocating path it stands in for (tlvlbm_set_levelset + tlvlbm_get_links):
the same records in the same order, bit for bit, on three calls in a row
(the second and third on smaller grids, the third in 3D), and the
capacity error path."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _reference(T, c):
    s = T.Solver(c["D"], c["n"], c["dx"], c["dt"], c["mu"], c["lam"], origin=c["origin"], periodic_mask=0)
    s.set_levelset(c["phi"], c["bid"])
    L = s.links()
    s.close()
    return L


def _no_alloc(T, c, cap, stream):
    import torch
    dev = torch.device("cuda")
    phi = torch.from_numpy(np.ascontiguousarray(c["phi"], np.float64)).to(dev)
    bid = torch.from_numpy(np.ascontiguousarray(c["bid"], np.uint8)).to(dev)
    out = dict(node=torch.full((cap,), -1, dtype=torch.int64, device=dev),
               q=torch.full((cap,), -1, dtype=torch.int32, device=dev),
               eta=torch.full((cap,), -1.0, dtype=torch.float64, device=dev),
               Nb=torch.full((cap, 3), -1.0, dtype=torch.float64, device=dev),
               bid_out=torch.full((cap,), -1, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    n = T.cut_links_noalloc(c["D"], c["n"], c["dx"], phi, cap, bid=bid, origin=c["origin"],
                            stream=stream.cuda_stream, **out)
    return n, {k: v.cpu().numpy() for k, v in out.items()}


def test_no_alloc_links_equal_the_allocating_path():
    import torch
    from paper_2606_20646_amd import tlvlbm as T
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    for c, what in ((W.config_c2(512), "annulus 512^2"), (W.config_c2(96), "annulus 96^2"),
                    (W.config_c5(40), "sphere 40^3")):
        _say(f"no-alloc cut links: {what}")
        ref = _reference(T, c)
        n_ref = len(ref["node"])
        n, out = _no_alloc(T, c, n_ref + 7, stream)
        assert n == n_ref
        assert np.array_equal(out["node"][:n], ref["node"]) and np.array_equal(out["q"][:n], ref["q"])
        assert np.array_equal(out["bid_out"][:n], ref["bid"])
        assert np.array_equal(out["eta"][:n], ref["eta"])
        assert np.array_equal(out["Nb"][:n, :c["D"]], ref["N"])
        # nothing written past the table
        assert np.all(out["node"][n:] == -1) and np.all(out["eta"][n:] == -1.0)


def test_no_alloc_capacity_error():
    import torch
    from paper_2606_20646_amd import tlvlbm as T
    torch.cuda.set_device(0)
    c = W.config_c2(64)
    n_ref = len(_reference(T, c)["node"])
    _say("no-alloc cut links: capacity one short")
    with pytest.raises(T.TlvlbmError) as e:
        _no_alloc(T, c, n_ref - 1, torch.cuda.Stream())
    assert e.value.code == T.ERR_INVALID_ARG and e.value.n_links == n_ref
