"""The real renormalization-group filter (Sec. 2.3, Eq. (18)) in place of the
Fresnel step, on the GPU against the FP64 oracle, and switched on and off
under a running batch."""
import numpy as np
import pytest

import oracle
from paper_1410_2855_amd.inputs import Cavity, initial_state, oracle_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def filtered(N=512, **kw):
    c = Cavity(N=N, F=200.0, R=0.9, pump_ratio=2.5, T1=600.0, index=21, **kw)
    return c.with_(filter_delta=2.5 * c.dx)


@pytest.mark.parametrize("prec,trips,tol", [(lsr.LSR_PREC_FP64TAB, 50, 1e-5), (lsr.LSR_PREC_PLAIN, 20, 1e-5),
                                             (lsr.LSR_PREC_FP64, 50, 1e-11)])
def test_filtered_map_matches_oracle(prec, trips, tol):
    cav = filtered()
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav, prec=prec)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    p.close()
    eo, no, to = oracle.run(oracle_params(cav), e0, n0, trips)
    assert rel(e.cpu().numpy(), eo) <= tol and rel(n.cpu().numpy(), no) <= tol
    assert rel(tr, to) <= max(tol, cav.N ** 2 * 2.3e-16)


@pytest.mark.parametrize("N", [256, 1024, 4096])
def test_filtered_one_trip_other_sizes(N):
    cav = filtered(N)
    e0, n0 = initial_state(cav)
    p = lsr.Plan(cav)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, 1)
    p.sync()
    p.close()
    eo, no, _ = oracle.run(oracle_params(cav), e0, n0, 1)
    assert rel(e.cpu().numpy(), eo) <= 1e-6


def test_switching_the_filter_under_a_batch():
    """Set and clear the filter on one cavity between batch calls: the batch
    must follow, bitwise like the one-cavity path doing the same."""
    cavs = [Cavity(N=512, F=150.0 + 40 * i, R=0.9, pump_ratio=2.0, T1=700.0, index=30 + i) for i in range(3)]
    delta = 3 * cavs[1].dx

    def run(batched):
        plans = [lsr.Plan(c) for c in cavs]
        st = [p.state(*initial_state(c)) for p, c in zip(plans, cavs)]
        Es, Ns = [s[0] for s in st], [s[1] for s in st]
        b = lsr.lsr_batch_create([p.handle for p in plans]) if batched else None

        def go(k):
            if batched:
                lsr.lsr_batch_roundtrips(b, Es, Ns, k)
            else:
                for p, e, n in zip(plans, Es, Ns):
                    p.roundtrips(e, n, k)

        go(5)
        lsr.lsr_plan_set_filter(plans[1].handle, delta)
        go(5)
        lsr.lsr_plan_set_filter(plans[1].handle, 0.0)
        go(5)
        for p in plans:
            p.sync()
        out = [(e.clone(), n.clone()) for e, n in zip(Es, Ns)]
        if b:
            lsr.lsr_batch_destroy(b)
        for p in plans:
            p.close()
        return out

    ref = run(False)
    got = run(True)
    for (e1, n1), (e2, n2) in zip(ref, got):
        assert torch.equal(e1, e2) and torch.equal(n1, n2)


def test_filter_bad_width():
    p = lsr.Plan(filtered(256))
    for bad in (-1e-6, float("nan"), float("inf")):
        with pytest.raises(lsr.LsrError) as ei:
            lsr.lsr_plan_set_filter(p.handle, bad)
        assert ei.value.code == lsr.LSR_EINVAL
    p.close()
