"""Randomised combinations of the map's options on the GPU against the FP64
oracle: grid size, Fresnel number, mirror reflectivity and curvature,
aperture form, mirror roughness, pump level and modulation, relaxation
time, local-step model,
nonlocal step (Fresnel or filter), number of gain sheets, precision form and
one-cavity FFT plan, drawn from one seeded generator.  Each case runs a few round trips and must
match the oracle to the single-cavity bar."""
import math

import numpy as np
import pytest

import oracle
from paper_1410_2855_amd.inputs import Cavity, initial_state, oracle_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402

CASES = 24


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def draw(i):
    r = np.random.default_rng(9000 + i)
    N = int(r.choice([256, 384, 512]))
    cav = Cavity(N=N, F=float(10 ** r.uniform(2, 3)), R=float(r.uniform(0.8, 0.99)),
                 pump_ratio=float(r.uniform(1.2, 4.0)), T1=float(r.uniform(50, 3000)), index=100 + i,
                 ap_kind=int(r.choice([0, 1, 2])), ap_radius_frac=float(r.uniform(0.3, 0.9)))
    if r.random() < 0.3:
        cav = cav.with_(focal=float(r.choice([-1, 1]) * r.uniform(2, 20)) * cav.L)
    if r.random() < 0.3:
        cav = cav.with_(mod_amp=float(r.uniform(0.1, 0.5)), mod_periods=int(r.choice([8, 16, 32])))
    if r.random() < 0.25:
        cav = cav.with_(filter_delta=float(r.uniform(1.0, 4.0)) * cav.dx)
    cav = cav.with_(model=int(r.choice([0, 0, 1, 2])), slices=int(r.choice([1, 1, 2, 3])))
    prec = int(r.choice([lsr.LSR_PREC_FP64TAB, lsr.LSR_PREC_FP64TAB, lsr.LSR_PREC_FP64]))
    trips = int(r.integers(3, 8))
    if r.random() < 0.3:   # drawn after the others, so their values stay as they were
        cav = cav.with_(rough_rms=float(r.uniform(0.2, 2.0)), rough_corr=int(r.integers(1, 6)))
    # the one-cavity FFT plan (256 in the FP32 forms has four), drawn last
    plan = int(r.integers(0, 4))
    if N != 256 or prec == lsr.LSR_PREC_FP64:
        plan = 0
    return cav, prec, trips, plan


@pytest.mark.parametrize("i", range(CASES))
def test_random_cavity_matches_oracle(i):
    cav, prec, trips, plan = draw(i)
    e0, n0 = initial_state(cav)
    # a field strong enough to deplete the inversion within the run
    e0 = e0 * math.sqrt(0.3 / cav.T1) / 1e-3
    p = lsr.Plan(cav, prec=prec)
    if plan:
        lsr.lsr_plan_set_fft_plan(p.handle, plan)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    p.close()
    eo, no, to = oracle.run(oracle_params(cav), e0, n0, trips)
    tol = 1e-11 if prec == lsr.LSR_PREC_FP64 else 5e-6
    case = "N=%d F=%.0f model=%d sheets=%d filter=%s rough=%.2f prec=%d trips=%d fft plan %d" % (
        cav.N, cav.F, cav.model, cav.slices, cav.filter_delta > 0, cav.rough_rms, prec, trips, plan)
    assert rel(e.cpu().numpy(), eo) <= tol, case
    assert rel(n.cpu().numpy(), no) <= tol, case
    assert rel(tr, to) <= max(tol, cav.N ** 2 * 2.3e-16), case


BATCH_CASES = 6


@pytest.mark.parametrize("i", range(BATCH_CASES))
def test_random_batch_is_bitwise_the_one_cavity_path(i):
    """Batches of randomly drawn cavities (the draws above with sizes up to
    2048, one sheet count per batch, the FP64-table form batches take; with
    one sheet, some cavities with a general transfer function), on a random
    engine and graph length, in calls of random lengths: every cavity
    bitwise the one-cavity path over the same trips."""
    r = np.random.default_rng(7000 + i)
    m = int(r.choice([1, 1, 2, 3]))
    cavs = []
    for k in range(int(r.integers(3, 7))):
        cav = draw(100 * i + k)[0]
        cavs.append(cav.with_(slices=m, N=int(r.choice([256, 384, 512, 768, 1024, 2048])), index=300 + k))
    engine = int(r.choice([0, 1, 1, 2]))
    graph_k = int(r.choice([0, 2, 5, 16]))
    calls = [int(x) for x in r.integers(1, 9, size=3)]
    trips = sum(calls)
    # general transfer functions (a random-phase all-pass of gain 0.98), from
    # a generator of their own so that the draws above stay as they were
    rt = np.random.default_rng(7500 + i)
    trans = [rt.random() < 0.4 and m == 1 for _ in cavs]
    tables = [0.98 * np.exp(2j * np.pi * rt.random((c.N, c.N))) if t else None for c, t in zip(cavs, trans)]

    def plan_of(c, t):
        p = lsr.Plan(c)
        if t is not None:
            lsr.lsr_plan_set_transfer(p.handle, t)
        return p

    ref = []
    for c, t in zip(cavs, tables):
        p = plan_of(c, t)
        e, n = p.state(*initial_state(c))
        p.roundtrips(e, n, trips)
        p.sync()
        ref.append((e, n))
        p.close()
    plans = [plan_of(c, t) for c, t in zip(cavs, tables)]
    st = [p.state(*initial_state(c)) for p, c in zip(plans, cavs)]
    Es, Ns = [x[0] for x in st], [x[1] for x in st]
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_configure(b, engine=engine, graph_k=graph_k)
    for k in calls:
        lsr.lsr_batch_roundtrips(b, Es, Ns, k)
    for p in plans:
        p.sync()
    case = "sheets=%d engine=%d graph_k=%d calls=%s sizes=%s models=%s transfer=%s" % (
        m, engine, graph_k, calls, [c.N for c in cavs], [c.model for c in cavs], trans)
    for j in range(len(cavs)):
        assert torch.equal(Es[j], ref[j][0]) and torch.equal(Ns[j], ref[j][1]), "%s cavity %d" % (case, j)
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()
