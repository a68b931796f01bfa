"""The structured-gain workload at its full size (4096^2, periodic pump of
Sec. 3 with M = 45 and 89 periods across the window) batched for 50 round
trips against the FP64 oracle, element by element.  The oracle runs in child
processes started when this test is collected (tests/oracle_jobs.py)."""
import os
import sys

import numpy as np
import pytest

from paper_1410_2855_amd.inputs import initial_state, structured_4096

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle_jobs  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.timeout(1500)
def test_structured_4096_fifty_trips_vs_oracle():
    trips = 50
    idx = (0, 15)
    cavs = [structured_4096()[i] for i in idx]
    plans = [lsr.Plan(c) for c in cavs]
    st = [p.state(*initial_state(c)) for p, c in zip(plans, cavs)]
    Es, Ns = [x[0] for x in st], [x[1] for x in st]
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_roundtrips(b, Es, Ns, trips)
    for p in plans:
        p.sync()
    got = [(e.cpu().numpy(), n.cpu().numpy(), p.trace(trips)) for p, e, n in zip(plans, Es, Ns)]
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()
    del Es, Ns, st
    for i, (eg, ng, tg) in zip(idx, got):
        eo, no, to = oracle_jobs.result("structured4096", i, trips)
        errs = rel(eg, eo), rel(ng, no), rel(tg, to)
        print("4096^2 cavity %d (M = %d), %d trips: rel L2 E %.2e, N %.2e, trace %.2e"
              % (i, structured_4096()[i].mod_periods, trips, *errs))
        assert max(errs) <= 1e-5, errs
