"""Several thin gain sheets per round trip (the distributed-gain variant of
Sec. 2.2, after Eq. (12)) on the GPU against the FP64 oracle: m sheets, each
with its own inversion, the nonlocal step split into m equal steps, the
mirror and aperture at sheet 0."""
import numpy as np
import pytest

import oracle
from paper_1410_2855_amd.inputs import Cavity, initial_state, oracle_params, sweep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402

TAB, PLAIN, F64 = lsr.LSR_PREC_FP64TAB, lsr.LSR_PREC_PLAIN, lsr.LSR_PREC_FP64


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def sheets(m, N=512, **kw):
    return Cavity(N=N, F=180.0, R=0.88, pump_ratio=3.0, T1=300.0, index=55, slices=m, **kw)


def run_both(cav, prec, trips):
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav, prec=prec)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    p.close()
    eo, no, to = oracle.run(oracle_params(cav), e0, n0, trips)
    return (e.cpu().numpy(), n.cpu().numpy(), tr), (eo, no, to)


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("prec,steps,tol", [(TAB, 50, 1e-5), (PLAIN, 10, 1e-3), (F64, 150, 1e-11)])
def test_sheets_match_oracle(m, prec, steps, tol):
    """The FP32 forms are held to the single-sheet bars at the same number of
    nonlocal steps (transform pairs): 50 steps are 50/m round trips."""
    cav = sheets(m)
    trips = steps // m
    (eg, ng, tg), (eo, no, to) = run_both(cav, prec, trips)
    assert ng.shape == (m, cav.N, cav.N)
    assert rel(eg, eo) <= tol and rel(ng, no) <= tol
    for k in range(m):
        assert rel(ng[k], no[k]) <= tol, k
    assert rel(tg, to) <= max(tol, cav.N ** 2 * 2.3e-16)


@pytest.mark.parametrize("variant", ["filter", "b-exact", "class-a", "focal", "pump-mod"])
@pytest.mark.parametrize("prec", [TAB, PLAIN])
def test_sheets_with_the_other_forms(variant, prec):
    """Sheets combined with the filter (variance delta^2/m per step), the
    alternative local steps, a curved mirror (phase at sheet 0 only) and a
    modulated pump (N0/m times the pattern on every sheet)."""
    cav = sheets(3)
    cav = {"filter": cav.with_(filter_delta=2.5 * cav.dx), "b-exact": cav.with_(model=1),
           "class-a": cav.with_(model=2), "focal": cav.with_(focal=4 * cav.L),
           "pump-mod": cav.with_(mod_amp=0.3, mod_periods=16)}[variant]
    trips, tol = (16, 1e-5) if prec == TAB else (3, 1e-3)   # 48 or 9 nonlocal steps
    (eg, ng, _), (eo, no, _) = run_both(cav, prec, trips)
    assert rel(eg, eo) <= tol and rel(ng, no) <= tol


def test_sheets_one_trip_every_size():
    for N in (256, 384, 768, 1024, 2048, 4096):
        cav = sheets(2, N=N)
        (eg, ng, _), (eo, no, _) = run_both(cav, TAB, 1)
        assert rel(eg, eo) <= 1e-6 and rel(ng, no) <= 1e-6, N


def test_one_sheet_is_the_default_map_bitwise():
    """set_slices(1) after 3 is the single-sheet map, bitwise."""
    cav = sheets(1)
    e0, n0 = initial_state(cav)
    out = []
    for toggle in (False, True):
        p = lsr.Plan(cav)
        if toggle:
            lsr.lsr_plan_set_slices(p.handle, 3)
            lsr.lsr_plan_set_slices(p.handle, 1)
        e, n = p.state(e0, n0)
        p.roundtrips(e, n, 7)
        p.sync()
        out.append((e.cpu(), n.cpu(), p.trace(7)))
        p.close()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


def test_timed_launches_advance_like_roundtrips_and_diag_reads_sheet_zero():
    cav = sheets(3, N=256)
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav)
    e1, n1 = p.state(e0, n0)
    e2, n2 = p.state(e0, n0)
    p.roundtrips(e1, n1, 4)
    row_ms, col_ms = lsr.lsr_time_kernels(p.handle, e2, n2, 4)
    p.sync()
    assert row_ms > 0 and col_ms > 0
    assert torch.equal(e1, e2) and torch.equal(n1, n2)
    d_all = p.diag(e1, n1)
    d_zero = p.diag(e1, n1[0].clone())
    assert d_all["energy"] == d_zero["energy"] and d_all["power_out"] == d_zero["power_out"]
    assert np.array_equal(d_all["radial"], d_zero["radial"])
    p.close()


def test_batches_refuse_several_sheets_and_bad_counts():
    cavs = sweep(2, seed=3, sizes=(512,))
    plans = [lsr.Plan(c) for c in cavs]
    st = [p.state(*initial_state(c)) for p, c in zip(plans, cavs)]
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_plan_set_slices(plans[0].handle, 2)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_roundtrips(b, [s[0] for s in st], [s[1] for s in st], 1)
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    lsr.lsr_batch_destroy(b)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_create([p.handle for p in plans])
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    for bad in (0, -2, lsr.LSR_MAX_SLICES + 1):
        with pytest.raises(lsr.LsrError) as ei:
            lsr.lsr_plan_set_slices(plans[1].handle, bad)
        assert ei.value.code == lsr.LSR_EINVAL
    for p in plans:
        p.close()
