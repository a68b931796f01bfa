"""GPU round-trip map (through the C ABI) against the FP64 oracle.

Tolerance (from the stated parity bar): relative L2 error of E and N at most
1e-5 after 50 round trips for the FP32 field with FP64-built tables; the
FP64 form is held to 1e-11.  One-trip checks run every compiled grid size.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1410_2855_amd.inputs import (Cavity, initial_state, oracle_params, plain_1024,
                                        plain_256, precision_2048, structured_4096)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402

TAB, PLAIN, F64 = lsr.LSR_PREC_FP64TAB, lsr.LSR_PREC_PLAIN, lsr.LSR_PREC_FP64
SIZES = [256, 384, 512, 768, 1024, 2048, 4096]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_run(cav, prec, trips, e0=None, n0=None):
    if e0 is None:
        e0, n0 = initial_state(cav)
    p = lsr.Plan(cav, prec=prec)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    out = e.cpu().numpy(), n.cpu().numpy(), tr
    p.close()
    return out


def oracle_run(cav, trips, e0=None, n0=None):
    if e0 is None:
        e0, n0 = initial_state(cav)
    return oracle.run(oracle_params(cav), e0, n0, trips)


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("prec", [TAB, F64])
def test_one_trip_every_size(N, prec):
    if not lsr.lsr_supported(N, prec):
        pytest.skip("N=%d not compiled for prec %d" % (N, prec))
    cav = Cavity(N=N, F=100.0, R=0.9, pump_ratio=2.0, T1=1000.0, index=N)
    eg, ng, tg = gpu_run(cav, prec, 1)
    eo, no, to = oracle_run(cav, 1)
    # FP64: the sums over N^2 points are added in another order than the
    # oracle's, which allows a relative difference up to about N^2 eps
    tol = 1e-6 if prec == TAB else 1e-11
    tol_tr = 1e-6 if prec == TAB else N * N * 2.3e-16
    print("N=%d prec=%d errE=%.2e errN=%.2e" % (N, prec, rel(eg, eo), rel(ng, no)))
    assert rel(eg, eo) <= tol
    assert rel(ng, no) <= tol
    assert rel(tg, to) <= tol_tr


@pytest.mark.parametrize("N", [256, 384, 512, 768, 1024])
def test_fifty_trips_fp32_tables(N):
    cav = Cavity(N=N, F=200.0, R=0.9, pump_ratio=3.0, T1=800.0, index=7 + N)
    eg, ng, tg = gpu_run(cav, TAB, 50)
    eo, no, to = oracle_run(cav, 50)
    print("N=%d 50 trips errE=%.2e errN=%.2e trace=%.2e" % (N, rel(eg, eo), rel(ng, no), rel(tg, to)))
    assert rel(eg, eo) <= 1e-5
    assert rel(ng, no) <= 1e-5
    assert rel(tg, to) <= 1e-5


@pytest.mark.parametrize("make", [plain_256, plain_1024], ids=["plain_256", "plain_1024"])
def test_workload_fifty_trips(make):
    cav = make()
    eg, ng, tg = gpu_run(cav, TAB, 50)
    eo, no, to = oracle_run(cav, 50)
    assert rel(eg, eo) <= 1e-5 and rel(ng, no) <= 1e-5 and rel(tg, to) <= 1e-5


def test_precision_2048_full_size():
    cav = precision_2048()
    eg, ng, _ = gpu_run(cav, TAB, 3)
    eo, no, _ = oracle_run(cav, 3)
    assert rel(eg, eo) <= 1e-5 and rel(ng, no) <= 1e-5


def test_structured_gain_4096_full_size():
    cav = structured_4096()[3]
    eg, ng, tg = gpu_run(cav, TAB, 1)
    eo, no, to = oracle_run(cav, 1)
    assert rel(eg, eo) <= 1e-5 and rel(ng, no) <= 1e-5 and rel(tg, to) <= 1e-5


def test_fp64_form_fifty_trips():
    cav = Cavity(N=384, F=150.0, R=0.92, pump_ratio=2.5, T1=600.0, index=3)
    eg, ng, tg = gpu_run(cav, F64, 50)
    eo, no, to = oracle_run(cav, 50)
    assert rel(eg, eo) <= 1e-11 and rel(ng, no) <= 1e-11
    assert rel(tg, to) <= cav.N ** 2 * 2.3e-16


@pytest.mark.parametrize("N", [512, 1024])
def test_plain_phase_is_the_weaker_form(N):
    """The FP32-evaluated propagator phase is off where it is large (it reaches
    pi (N/2)^2/(2F) rad at the grid corner); the FP64-built table is not.  One
    trip from white noise, whose spectrum fills the whole grid."""
    cav = Cavity(N=N, F=100.0, R=0.95, pump_ratio=3.0, T1=2000.0, index=1)
    eo, _, _ = oracle_run(cav, 1)
    e_tab, _, _ = gpu_run(cav, TAB, 1)
    e_plain, _, _ = gpu_run(cav, PLAIN, 1)
    print("N=%d 1 trip: plain %.2e, fp64 tables %.2e" % (N, rel(e_plain, eo), rel(e_tab, eo)))
    assert rel(e_tab, eo) <= 1e-6
    assert rel(e_plain, eo) > 10 * rel(e_tab, eo)
    assert rel(e_plain, eo) <= 1e-2


@pytest.mark.parametrize("variant", ["gauss", "none", "focal", "pump_mod", "diverging"])
def test_cavity_variants(variant):
    kw = dict(N=512, F=120.0, R=0.88, pump_ratio=2.2, T1=700.0, index=11)
    if variant == "gauss":
        kw.update(ap_kind=2, ap_radius_frac=0.3)
    elif variant == "none":
        kw.update(ap_kind=0)
    elif variant == "focal":
        kw.update(focal=0.05)
    elif variant == "diverging":
        kw.update(focal=-0.2)
    elif variant == "pump_mod":
        kw.update(mod_amp=0.3, mod_periods=16)
    cav = Cavity(**kw)
    eg, ng, tg = gpu_run(cav, TAB, 10)
    eo, no, to = oracle_run(cav, 10)
    assert rel(eg, eo) <= 1e-5 and rel(ng, no) <= 1e-5 and rel(tg, to) <= 1e-5


def test_mask_aperture_matches_supergaussian():
    cav = Cavity(N=256, F=100.0, R=0.9, pump_ratio=2.0, T1=1000.0, index=5)
    x = (np.arange(cav.N) - cav.N / 2) * cav.dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    mask = np.exp(-((X ** 2 + Y ** 2) / cav.ap_radius ** 2) ** 5)
    mdev = torch.from_numpy(mask.astype(np.float32)).cuda()
    h = lsr.lsr_plan_create(cav.N, cav.dx, cav.lam, cav.L, 0.0, cav.R, ap_kind=lsr.LSR_AP_MASK,
                            ap_mask=mdev, prec=TAB)
    lsr.lsr_plan_set_gain(h, cav.N0, cav.T1)
    e0, n0 = initial_state(cav)
    e = torch.from_numpy(e0).to("cuda", torch.complex64)
    n = torch.from_numpy(n0).to("cuda", torch.float32)
    lsr.lsr_roundtrips(h, e, n, 10)
    lsr.lsr_sync(h)
    lsr.lsr_plan_destroy(h)
    eo, no, _ = oracle_run(cav, 10)
    assert rel(e.cpu().numpy(), eo) <= 1e-5 and rel(n.cpu().numpy(), no) <= 1e-5


def test_zero_trips_is_identity_and_one_trip_works():
    cav = plain_256()
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav)
    e, n = p.state(e0, n0)
    e_ref, n_ref = e.clone(), n.clone()
    p.roundtrips(e, n, 0)
    p.sync()
    assert torch.equal(e, e_ref) and torch.equal(n, n_ref)
    p.close()
    eg, ng, _ = gpu_run(cav, TAB, 1)
    eo, no, _ = oracle_run(cav, 1)
    assert rel(eg, eo) <= 1e-6


def test_split_run_equals_continuous_and_is_deterministic():
    cav = Cavity(N=768, F=250.0, R=0.9, pump_ratio=2.0, T1=900.0, index=2)
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav)
    ea, na = p.state(e0, n0)
    p.roundtrips(ea, na, 17)
    eb, nb = p.state(e0, n0)
    p.roundtrips(eb, nb, 5)
    p.roundtrips(eb, nb, 12)
    ec, nc = p.state(e0, n0)
    p.roundtrips(ec, nc, 17)
    p.sync()
    assert torch.equal(ea, eb) and torch.equal(na, nb)
    assert torch.equal(ea, ec) and torch.equal(na, nc)
    p.close()


def test_trace_records_each_trip_in_order():
    cav = plain_256()
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, 30)
    tr1 = p.trace(30)
    p.roundtrips(e, n, 20)
    tr2 = p.trace(100)
    p.close()
    _, _, to = oracle_run(cav, 50)
    assert tr1.shape == (30, 4) and tr2.shape == (20, 4)
    assert rel(np.vstack([tr1, tr2]), to) <= 1e-5


@pytest.mark.parametrize("N", [512, 4096])
def test_diag_matches_oracle_spectrum_and_sums(N):
    cav = Cavity(N=N, F=150.0 if N == 512 else 1000.0, R=0.9, pump_ratio=2.0, T1=1000.0, index=4)
    e0, n0 = initial_state(cav)
    rng = np.random.default_rng(0)
    n0 = n0 + 0.02 * rng.standard_normal(n0.shape)
    p = lsr.Plan(cav)
    e, n = p.state(e0, n0)
    d = p.diag(e, n)
    p.close()
    radial, dom = oracle.spectrum(oracle_params(cav), e0, n0)
    _, _, to = oracle_run(cav, 1, e0, n0)
    s1, s2, s3, s4 = to[0]
    dx2 = cav.dx ** 2
    assert d["nbins"] == radial.size == oracle.nbins(cav.N)
    assert rel(d["radial"], radial) <= 1e-5
    assert d["dominant_bin"] == dom
    assert abs(d["energy"] - s1 * dx2) <= 1e-6 * s1 * dx2
    assert abs(d["power_out"] - (1 - cav.R) * s3 * dx2) <= 1e-6 * s3 * dx2
    assert abs(d["gain_sum"] - (s3 - s2) * dx2) <= 1e-5 * s3 * dx2
    assert abs(d["inv_sum"] - s4 * dx2) <= 1e-6 * abs(s4) * dx2


def test_nonfinite_state_is_reported():
    cav = plain_256()
    e0, n0 = initial_state(cav)
    e0 = e0.copy()
    e0[17, 33] = np.nan
    p = lsr.Plan(cav)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, 3)
    with pytest.raises(lsr.LsrError) as ei:
        p.sync()
    assert ei.value.code == lsr.LSR_ENONFINITE
    p.sync()   # flag cleared by the report
    p.close()


def test_bad_arguments_on_device():
    cav = plain_256()
    p = lsr.Plan(cav)
    e, n = p.state(*initial_state(cav))
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_roundtrips(p.handle, e, n, -1)
    assert ei.value.code == lsr.LSR_EINVAL
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_roundtrips(p.handle, int(e.data_ptr()) + 8, n, 1)
    assert ei.value.code == lsr.LSR_EINVAL
    p.close()


@pytest.mark.parametrize("N,k", [(256, 1), (256, 2), (256, 3), (2048, 1)])
def test_one_cavity_fft_plans(N, k, tmp_path):
    """The one-cavity FFT plans (256: 8 points per lane; 4 points per lane
    on four or two lines per workgroup; 2048: a wave per line) compute the
    same map: 50 trips (20 at 2048^2)
    against the oracle at the usual bar, 3 trips against the default plan to
    FP32 rounding; a batch holding such a plan runs its group's plan and
    stays bitwise the default one-cavity path; the autotuner picks one of
    them and records it; FP64 plans and other sizes have none."""
    from paper_1410_2855_amd.inputs import Cavity

    cav = Cavity(N=N, F=200.0 if N < 2048 else 1000.0, R=0.9, pump_ratio=2.5, T1=600.0, index=9)
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav)
    lsr.lsr_plan_set_fft_plan(p.handle, k)
    trips = 50 if N < 2048 else 20
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, trips)
    p.sync()
    eo, no, to = oracle.run(oracle_params(cav), e0, n0, trips)
    assert rel(e.cpu().numpy(), eo) <= 1e-5 and rel(n.cpu().numpy(), no) <= 1e-5
    assert rel(p.trace(trips), to) <= 1e-5
    # the diagnostics on this plan's blocks (up to 128 column blocks of partials)
    d = p.diag(e, n)
    radial, dom = oracle.spectrum(oracle_params(cav), e.cpu().numpy().astype(np.complex128),
                                  n.cpu().numpy().astype(np.float64))
    assert rel(d["radial"], radial) <= 1e-5 and d["dominant_bin"] == dom
    q = lsr.Plan(cav)
    e1, n1 = p.state(e0, n0)
    e2, n2 = q.state(e0, n0)
    p.roundtrips(e1, n1, 3)
    q.roundtrips(e2, n2, 3)
    torch.cuda.synchronize()
    assert rel(e1.cpu().numpy(), e2.cpu().numpy()) <= 2e-6
    # a batch runs its group's plan whatever the plan's own
    e3, n3 = p.state(e0, n0)
    b = lsr.lsr_batch_create([p.handle])
    lsr.lsr_batch_roundtrips(b, [e3], [n3], 3)
    torch.cuda.synchronize()
    assert torch.equal(e3, e2) and torch.equal(n3, n2)
    lsr.lsr_batch_destroy(b)
    cache = str(tmp_path / "tune.json")
    lsr.lsr_autotune(q.handle, None, cache)
    import json
    assert json.load(open(cache))["gfx950:plan:%d:1" % N]["shape"] in ((0, 1, 2, 3) if N == 256 else (0, 1))
    f = lsr.Plan(cav, prec=lsr.LSR_PREC_FP64)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_plan_set_fft_plan(f.handle, k)
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    for x in (p, q, f):
        x.close()
    r = lsr.Plan(cav.with_(N=512))
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_plan_set_fft_plan(r.handle, k)
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    r.close()
    r = lsr.Plan(cav)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_plan_set_fft_plan(r.handle, 4)
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    r.close()
