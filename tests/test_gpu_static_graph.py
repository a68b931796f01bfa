"""The allocation-free entry point under HIP graph capture, the use it is
for: its launches recorded into a graph (through torch's graph capture on
a side stream) and replayed several times, with the program's own eager
work and synchronisations between the replays; every replay must equal the
eager call bitwise."""
import math

import numpy as np
import pytest

from paper_1410_2855_amd.inputs import initial_state, plain_256

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402


def static_call(cav, e, n, trips, tr, stream):
    focal = cav.focal if math.isfinite(cav.focal) else 0.0
    ap = lsr.lsr_aperture(cav.ap_kind, cav.ap_radius, cav.ap_order, None)
    lsr.lsr_roundtrips_static(cav.N, cav.dx, cav.lam, cav.L, focal, cav.R, ap, cav.N0, cav.T1,
                              cav.mod_amp, cav.mod_period, cav.model, e, n, trips, tr, stream)


def test_static_entry_point_replays_from_a_captured_graph():
    cav = plain_256().with_(mod_amp=0.3, mod_periods=20)
    trips = 6
    e0, n0 = initial_state(cav)
    e0 = torch.from_numpy(e0).to("cuda", torch.complex64)
    n0 = torch.from_numpy(n0).to("cuda", torch.float32)
    # eager reference (also the first call on this device: the array's
    # address is looked up here, outside the capture)
    e, n = e0.clone(), n0.clone()
    tr = torch.zeros((trips, 4), dtype=torch.float64, device="cuda")
    static_call(cav, e, n, trips, tr, torch.cuda.current_stream())
    torch.cuda.synchronize()
    ref = (e.clone(), n.clone(), tr.clone())

    eg, ng = e0.clone(), n0.clone()
    trg = torch.zeros_like(tr)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=side):
        static_call(cav, eg, ng, trips, trg, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        # the program's own eager work between replays: reset the state
        eg.copy_(e0)
        ng.copy_(n0)
        trg.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(eg, ref[0]) and torch.equal(ng, ref[1]), rep
        assert torch.equal(trg, ref[2]), rep
        # an eager call between replays, on another state
        e2, n2 = e0.clone(), n0.clone()
        static_call(cav, e2, n2, 2, None, torch.cuda.current_stream())
        torch.cuda.synchronize()
    assert np.isfinite(eg.cpu().numpy()).all()
