"""The oracle's failure path of the traction closure: a random-hole instance
drawn without the recipe's redraw of narrow ligaments (instance 54 at 64^2
cells, a 0.0023-wide sliver between two holes) drives the Neumann Newton
solve (Sec. 3.4, Eqs. 53-56) to an inadmissible root; the oracle reports
ORC_ERR_NEWTON, keeps it, and the redrawn instance runs through."""
import pytest

import workloads as W
from test_gpu_failure import _oracle


def test_oracle_reports_newton_failure_on_sliver():
    from oracle import oracle as O
    c = W.config_c4_instance(54, N=64, redraw=False)
    o = _oracle(c)
    with pytest.raises(O.OracleError) as e:
        o.step(c["steps"])
    assert e.value.code == 5  # ORC_ERR_NEWTON
    st = o.stats()
    assert st["status"] == 5 and st["newton_fail"] >= 1 and 0 < st["step"] < c["steps"]
    with pytest.raises(O.OracleError):
        o.step(1)
    ok = _oracle(W.config_c4_instance(54, N=64))
    ok.step(st["step"] + 20)
    assert ok.stats()["newton_fail"] == 0
