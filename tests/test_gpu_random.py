"""Randomised combinations of the map's options on the GPU against the FP64
oracle: grid size, Fresnel number, mirror reflectivity and curvature,
aperture form, mirror roughness, pump level and modulation, relaxation
time, local-step model,
nonlocal step (Fresnel or filter), number of gain sheets and precision form,
drawn from one seeded generator.  Each case runs a few round trips and must
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
    if r.random() < 0.3:   # drawn last, so the other options of a case stay as they were
        cav = cav.with_(rough_rms=float(r.uniform(0.2, 2.0)), rough_corr=int(r.integers(1, 6)))
    return cav, prec, trips


@pytest.mark.parametrize("i", range(CASES))
def test_random_cavity_matches_oracle(i):
    cav, prec, trips = draw(i)
    e0, n0 = initial_state(cav)
    # a field strong enough to deplete the inversion within the run
    e0 = e0 * math.sqrt(0.3 / cav.T1) / 1e-3
    p = lsr.Plan(cav, prec=prec)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    p.close()
    eo, no, to = oracle.run(oracle_params(cav), e0, n0, trips)
    tol = 1e-11 if prec == lsr.LSR_PREC_FP64 else 5e-6
    case = "N=%d F=%.0f model=%d sheets=%d filter=%s rough=%.2f prec=%d trips=%d" % (
        cav.N, cav.F, cav.model, cav.slices, cav.filter_delta > 0, cav.rough_rms, prec, trips)
    assert rel(e.cpu().numpy(), eo) <= tol, case
    assert rel(n.cpu().numpy(), no) <= tol, case
    assert rel(tr, to) <= max(tol, cav.N ** 2 * 2.3e-16), case
