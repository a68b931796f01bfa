"""The metric's workload in the launch configuration bench.py times: 64
cavities at 1024^2 with the sweep's parameter draws, FP64-table form, one
batch configured from the committed tuning cache (grouped passes, graphs of
64 trips), the graphs captured ahead by lsr_batch_prepare and calls of 20
trips replayed from whole-call graphs; sampled cavities against the FP64
oracle at the single-cavity bar after 50 trips, every cavity finite and
bitwise the one-cavity path."""
import os

import numpy as np
import pytest

import oracle
from paper_1410_2855_amd.inputs import initial_state, oracle_params, sweep_1024

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_1410_2855_amd", "tune_cache.json")
SAMPLED = (0, 21, 42, 63)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.timeout(900)
def test_bench_configuration_against_the_oracle(monkeypatch):
    monkeypatch.setenv("LSR_TUNE_CACHE", CACHE)
    cavs = sweep_1024(64)
    stream = torch.cuda.current_stream()
    plans = [lsr.Plan(c, stream=stream) for c in cavs]
    st = [p.state(*initial_state(c)) for p, c in zip(plans, cavs)]
    Es, Ns = [x[0] for x in st], [x[1] for x in st]
    b = lsr.lsr_batch_create([p.handle for p in plans])
    cfg = lsr.lsr_batch_configure(b)   # no change: the configuration the cache gave
    assert cfg["engine"] == 1 and cfg["graph_k"] == 64 and cfg["shape"] == 0, cfg
    lsr.lsr_batch_prepare(b, 20)
    lsr.lsr_batch_prepare(b, 10)
    for k in (20, 20, 10):
        lsr.lsr_batch_roundtrips(b, Es, Ns, k)
    for p in plans:
        p.sync()
    traces = {i: plans[i].trace(10) for i in SAMPLED}
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()
    assert all(bool(torch.isfinite(e).all()) for e in Es)
    # a sampled cavity on the one-cavity path: bitwise the same
    q = lsr.Plan(cavs[SAMPLED[1]])
    e1, n1 = q.state(*initial_state(cavs[SAMPLED[1]]))
    q.roundtrips(e1, n1, 50)
    q.sync()
    q.close()
    assert torch.equal(e1, Es[SAMPLED[1]]) and torch.equal(n1, Ns[SAMPLED[1]])
    for i in SAMPLED:
        eo, no, to = oracle.run(oracle_params(cavs[i]), *initial_state(cavs[i]), 50)
        err_e, err_n = rel(Es[i].cpu().numpy(), eo), rel(Ns[i].cpu().numpy(), no)
        print("cavity %d: E %.2e N %.2e trace %.2e" % (i, err_e, err_n, rel(traces[i], to[-10:])))
        assert err_e <= 1e-5 and err_n <= 1e-5, i
        assert rel(traces[i], to[-10:]) <= 1e-5, i
