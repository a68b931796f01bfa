"""The allocation-free entry point lsr_roundtrips_static against the plan
path (lsr_plan_create + lsr_roundtrips) on the same seeded inputs, through
the C ABI: two calls in a row, the second on a smaller grid."""
import ctypes
import math

import numpy as np
import pytest

from paper_1410_2855_amd.inputs import initial_state, plain_256, sweep_1024

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def run_plan(cav, trips):
    p = lsr.Plan(cav)
    e, n = p.state(*initial_state(cav))
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    p.close()
    return e.cpu().numpy(), n.cpu().numpy(), tr


def run_static(cav, trips):
    e0, n0 = initial_state(cav)
    e = torch.from_numpy(e0).to("cuda", torch.complex64).contiguous()
    n = torch.from_numpy(n0).to("cuda", torch.float32).contiguous()
    tr = torch.zeros((trips, 4), dtype=torch.float64, device="cuda")
    focal = cav.focal if math.isfinite(cav.focal) else 0.0
    ap = lsr.lsr_aperture(cav.ap_kind, cav.ap_radius, cav.ap_order, None)
    lsr.lsr_roundtrips_static(cav.N, cav.dx, cav.lam, cav.L, focal, cav.R, ap, cav.N0, cav.T1,
                              cav.mod_amp, cav.mod_period, cav.model, e, n, trips, tr,
                              torch.cuda.current_stream())
    torch.cuda.synchronize()
    return e.cpu().numpy(), n.cpu().numpy(), tr.cpu().numpy()


def test_static_entry_point_matches_the_plan_path_twice():
    big = sweep_1024(2)[1].with_(mod_amp=0.3, mod_periods=60, focal=0.35)
    small = plain_256().with_(model=1)
    for cav, trips in ((big, 7), (small, 5)):
        es, ns, ts = run_static(cav, trips)
        ep, np_, tp = run_plan(cav, trips)
        print("N=%d: E %.2e N %.2e trace %.2e bitwise %s" % (
            cav.N, rel(es, ep), rel(ns, np_), rel(ts, tp), np.array_equal(es, ep) and np.array_equal(ns, np_)))
        assert rel(es, ep) <= 1e-6 and rel(ns, np_) <= 1e-6
        assert rel(ts, tp) <= 1e-6


def test_static_entry_point_rejects_bad_arguments():
    e = torch.zeros((256, 256), dtype=torch.complex64, device="cuda")
    n = torch.zeros((256, 256), dtype=torch.float32, device="cuda")
    ap = lsr.lsr_aperture(1, 1e-4, 10, None)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_roundtrips_static(1000, 1e-6, 1e-6, 1e-3, 0.0, 0.9, ap, 0.2, 100.0, 0.0, 0.0, 0,
                                  e, n, 1, None, None)
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_roundtrips_static(256, 1e-6, 1e-6, 1e-3, 0.0, 1.5, ap, 0.2, 100.0, 0.0, 0.0, 0,
                                  e, n, 1, None, None)
    assert ei.value.code == lsr.LSR_EINVAL
