"""Batched path (persistent kernel per round trip, HIP graph of k trips)
against the one-cavity path and the oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1410_2855_amd.inputs import Cavity, initial_state, oracle_params, sweep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1410_2855_amd import lsr  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def make(cavs):
    plans, Es, Ns = [], [], []
    for c in cavs:
        p = lsr.Plan(c)
        e, n = p.state(*initial_state(c))
        plans.append(p)
        Es.append(e)
        Ns.append(n)
    return plans, Es, Ns


def plain_reference(cavs, trips):
    plans, Es, Ns = make(cavs)
    for p, e, n in zip(plans, Es, Ns):
        p.roundtrips(e, n, trips)
    traces = [p.trace(trips) for p in plans]
    for p in plans:
        p.sync()
    out = [(e.clone(), n.clone()) for e, n in zip(Es, Ns)]
    for p in plans:
        p.close()
    return out, traces


def mixed(count, sizes):
    cavs = sweep(count, seed=3, sizes=sizes)
    return cavs


def assert_matches_plain(cfg, Es, Ns, ref):
    """Bitwise the one-cavity path with the default FFT plans; to rounding
    (FP32, a few trips) with an alternative plan."""
    for i in range(len(ref)):
        if cfg["shape"] == 0:
            assert torch.equal(Es[i], ref[i][0]) and torch.equal(Ns[i], ref[i][1]), i
        else:
            assert rel(Es[i].cpu().numpy(), ref[i][0].cpu().numpy()) <= 2e-6, i
            assert rel(Ns[i].cpu().numpy(), ref[i][1].cpu().numpy()) <= 2e-6, i


@pytest.mark.parametrize("sizes,count,trips,k,engine,merge", [
    ((256, 384, 512, 768, 1024), 9, 13, 4, 2, 1),  # one kernel for all sizes, graph + remainder
    ((256, 384, 512, 768, 1024), 9, 13, 4, 1, 0),  # one kernel per size
    ((256, 384, 512, 768, 1024), 5, 6, 2, 0, 1),   # one persistent kernel for all sizes
    ((256, 384, 512, 768, 1024), 5, 6, 2, 0, 0),   # a persistent kernel per size
    ((1024,), 5, 7, 0, 2, 0),                      # single-size group, pipelined, eager
    ((1024,), 5, 7, 3, 1, 0),                      # grouped, not pipelined
    ((1024,), 4, 5, 2, 0, 0),                      # persistent kernel
    ((1024,), 3, 1, 16, 2, 0),                     # one trip: FIRST + LAST only
    ((2048,), 2, 5, 2, 2, 0),
    ((256, 2048), 4, 6, 3, 2, 1),                  # different workgroup sizes: two kernels
    ((256, 2048), 4, 6, 3, 1, 0),
    ((4096, 512), 2, 3, 1, 2, 1),                  # two workgroup sizes: two groups either way
    ((384,), 7, 4, 2, 2, 0),
])
def test_batch_is_bitwise_the_plain_path(sizes, count, trips, k, engine, merge):
    cavs = mixed(count, sizes)
    ref, ref_tr = plain_reference(cavs, trips)
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    cfg = lsr.lsr_batch_configure(b, engine=engine, merge=merge)
    assert cfg["engine"] == engine and cfg["merge"] == merge
    lsr.lsr_batch_set_graph_trips(b, k)
    lsr.lsr_batch_roundtrips(b, Es, Ns, trips)
    for p in plans:
        p.sync()
    for i, (p, e, n) in enumerate(zip(plans, Es, Ns)):
        assert torch.equal(e, ref[i][0]), "cavity %d (N=%d) field" % (i, cavs[i].N)
        assert torch.equal(n, ref[i][1]), "cavity %d (N=%d) inversion" % (i, cavs[i].N)
        assert np.array_equal(p.trace(trips), ref_tr[i])
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_batch_graph_replays_and_repeated_calls_match_eager():
    cavs = mixed(6, (512, 1024))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_set_graph_trips(b, 3)
    for _ in range(3):          # graph replayed several times across calls
        lsr.lsr_batch_roundtrips(b, Es, Ns, 7)
        torch.cuda.synchronize()
    ref, _ = plain_reference(cavs, 21)
    for i in range(len(cavs)):
        assert torch.equal(Es[i], ref[i][0]) and torch.equal(Ns[i], ref[i][1])
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_batch_fifty_trips_against_oracle():
    cavs = mixed(4, (256, 384, 512, 768))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_roundtrips(b, Es, Ns, 50)
    for p in plans:
        p.sync()
    for c, e, n in zip(cavs, Es, Ns):
        eo, no, _ = oracle.run(oracle_params(c), *initial_state(c), 50)
        assert rel(e.cpu().numpy(), eo) <= 1e-5 and rel(n.cpu().numpy(), no) <= 1e-5
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_batch_diag_and_bad_arguments():
    cavs = mixed(2, (256,))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    d = lsr.lsr_batch_diag(b, 1, Es[1], Ns[1], lsr.lsr_plan_nbins(plans[1].handle))
    assert d["energy"] > 0
    with pytest.raises(lsr.LsrError):
        lsr.lsr_batch_roundtrips(b, Es, Ns, -2)
    with pytest.raises(lsr.LsrError):
        lsr.lsr_batch_diag(b, 5, Es[0], Ns[0], 10)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_create([plans[0].handle, plans[0].handle])
    assert ei.value.code == lsr.LSR_EINVAL
    f64 = lsr.Plan(cavs[0], prec=lsr.LSR_PREC_FP64)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_create([f64.handle])
    assert ei.value.code == lsr.LSR_EUNSUPPORTED
    lsr.lsr_batch_destroy(b)
    for p in plans + [f64]:
        p.close()


def test_autotune_writes_cache_and_keeps_results(tmp_path):
    cavs = mixed(3, (512,))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    path = str(tmp_path / "tune.json")
    lsr.lsr_autotune(None, b, path)
    text = open(path).read()
    assert "gfx950:batch:512x3;" in text and '"shape"' in text
    lsr.lsr_batch_roundtrips(b, Es, Ns, 9)
    ref, _ = plain_reference(cavs, 9)
    assert_matches_plain(lsr.lsr_batch_configure(b), Es, Ns, ref)
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_autotune_mixed_sizes_keeps_results(tmp_path):
    """A batch whose grid sizes share a workgroup size: the tuner also times
    the merged kernel and the alternative FFT plans; whatever it picks, the
    results stay those of the one-cavity path (bitwise with default plans)."""
    cavs = mixed(4, (256, 512))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    path = str(tmp_path / "tune.json")
    lsr.lsr_autotune(None, b, path)
    assert '"merge"' in open(path).read()
    cfg = lsr.lsr_batch_configure(b)
    assert cfg["merge"] in (0, 1)
    lsr.lsr_batch_roundtrips(b, Es, Ns, 9)
    ref, _ = plain_reference(cavs, 9)
    assert_matches_plain(cfg, Es, Ns, ref)
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


@pytest.mark.parametrize("chunk,lag", [(8, 128), (16, 512), (1, 0)])
def test_persistent_kernel_with_interleaved_rows_and_columns(chunk, lag):
    """Many cavities, short packer lag and large ticket chunks: column tasks
    start while other cavities' rows still run and often wait on their own
    cavity's rows.  The results must stay bitwise those of the one-cavity
    path."""
    cavs = mixed(48, (512,))
    trips = 6
    ref, ref_tr = plain_reference(cavs, trips)
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_configure(b, engine=0, chunk=chunk, lag=lag, graph_k=0)
    lsr.lsr_batch_roundtrips(b, Es, Ns, trips)
    for p in plans:
        p.sync()
    bad = [i for i in range(len(cavs)) if not (torch.equal(Es[i], ref[i][0]) and torch.equal(Ns[i], ref[i][1]))]
    assert not bad, "cavities differing from the one-cavity path: %s" % bad
    for i, p in enumerate(plans):
        assert np.array_equal(p.trace(trips), ref_tr[i])
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_batch_follows_new_state_buffers_between_calls():
    """The batch keeps per-cavity descriptors (and graphs reading them) on the
    device; a call with other state tensors must act on those tensors."""
    cavs = mixed(4, (512, 1024))
    ref, _ = plain_reference(cavs, 12)
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_set_graph_trips(b, 2)
    lsr.lsr_batch_roundtrips(b, Es, Ns, 6)
    Es2 = [e.clone() for e in Es]
    Ns2 = [n.clone() for n in Ns]
    keep = [(e.clone(), n.clone()) for e, n in zip(Es, Ns)]
    lsr.lsr_batch_roundtrips(b, Es2, Ns2, 6)
    torch.cuda.synchronize()
    for i in range(len(cavs)):
        assert torch.equal(Es2[i], ref[i][0]) and torch.equal(Ns2[i], ref[i][1])
        # the first buffers were left alone by the second call
        assert torch.equal(Es[i], keep[i][0]) and torch.equal(Ns[i], keep[i][1])
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


@pytest.mark.parametrize("N,shape", [(256, 1), (512, 1), (1024, 1), (1024, 2), (2048, 1), (4096, 1)])
@pytest.mark.parametrize("engine", [1, 0, 2])
def test_alternative_fft_plans(N, shape, engine):
    """The batch's alternative FFT plans (another radix order, 8 x 8 tiles, or
    half the lanes per line) compute the same map: 50 trips (4 at 4096^2,
    where the oracle takes seconds per trip) against the FP64 oracle to the
    usual bar, a few trips against the one-cavity path to FP32 rounding, and
    every engine bitwise equal to the grouped one on the same plan."""
    cavs = [c.with_(N=N) for c in sweep(3, seed=11, sizes=(N,))]
    trips = (50 if N < 4096 else 4) if engine == 1 else 6
    results = {}
    for eng in sorted({1, engine}):
        plans, Es, Ns = make(cavs)
        b = lsr.lsr_batch_create([p.handle for p in plans])
        cfg = lsr.lsr_batch_configure(b, engine=eng, shape=shape, graph_k=4)
        assert cfg["shape"] == shape
        lsr.lsr_batch_roundtrips(b, Es, Ns, trips)
        for p in plans:
            p.sync()
        results[eng] = [(e.clone(), n.clone()) for e, n in zip(Es, Ns)]
        tr = [p.trace(trips) for p in plans]
        lsr.lsr_batch_destroy(b)
        for p in plans:
            p.close()
    if engine != 1:
        for (e1, n1), (e2, n2) in zip(results[1], results[engine]):
            assert torch.equal(e1, e2) and torch.equal(n1, n2)
        return
    eo, no, to = oracle.run(oracle_params(cavs[0]), *initial_state(cavs[0]), trips)
    e, n = results[1][0]
    assert rel(e.cpu().numpy(), eo) <= 1e-5 and rel(n.cpu().numpy(), no) <= 1e-5
    assert rel(tr[0], to) <= 1e-5
    ref, _ = plain_reference(cavs, 3)
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    cfg = lsr.lsr_batch_configure(b, engine=1, shape=shape)
    lsr.lsr_batch_roundtrips(b, Es, Ns, 3)
    for p in plans:
        p.sync()
    assert_matches_plain(cfg, Es, Ns, ref)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_configure(b, shape=lsr.LSR_MAX_SHAPES + 1)
    assert ei.value.code == lsr.LSR_EINVAL
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


@pytest.mark.parametrize("engine", [1, 0])
def test_graphs_for_every_call_length(engine):
    """Calls of any length replay graphs (whole-call graphs up to k + 1 trips,
    k-trip graphs plus a remainder graph beyond), prepared or captured on
    first use, several lengths interleaved so the graph cache is reused and
    evicted: bitwise the one-cavity path over the same total trips."""
    cavs = mixed(4, (512, 1024))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_configure(b, engine=engine, graph_k=4)
    lengths = [1, 2, 5, 3, 9, 5, 2, 6, 7, 1, 11, 4, 12, 3, 5]   # > 8 distinct graphs over the run
    lsr.lsr_batch_prepare(b, 5)
    lsr.lsr_batch_prepare(b, 9)
    for n in lengths:
        lsr.lsr_batch_roundtrips(b, Es, Ns, n)
    for p in plans:
        p.sync()
    total = sum(lengths)
    ref, _ = plain_reference(cavs, total)
    for i in range(len(cavs)):
        assert torch.equal(Es[i], ref[i][0]) and torch.equal(Ns[i], ref[i][1]), i
    # the last call's trace is the last `lengths[-1]` trips of the one-cavity run
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_batch_rejects_plans_on_different_streams():
    cavs = mixed(2, (256,))
    plans, Es, Ns = make(cavs)
    other = torch.cuda.Stream()
    lsr.lsr_plan_set_stream(plans[1].handle, other)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_create([p.handle for p in plans])
    assert ei.value.code == lsr.LSR_EINVAL
    lsr.lsr_plan_set_stream(plans[1].handle, torch.cuda.current_stream())
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_roundtrips(b, Es, Ns, 2)
    # a plan rebound after the batch was built is refused on the next call
    lsr.lsr_plan_set_stream(plans[0].handle, other)
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_batch_roundtrips(b, Es, Ns, 2)
    assert ei.value.code == lsr.LSR_EINVAL
    lsr.lsr_plan_set_stream(plans[0].handle, torch.cuda.current_stream())
    lsr.lsr_batch_roundtrips(b, Es, Ns, 2)
    torch.cuda.synchronize()
    ref, _ = plain_reference(cavs, 4)
    for i in range(len(cavs)):
        assert torch.equal(Es[i], ref[i][0]) and torch.equal(Ns[i], ref[i][1]), i
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_persistent_wait_failure_flags_every_cavity():
    """The persistent kernel's bounded wait, forced from the host to give up
    (one row block more than exists, a poll limit of 64): every cavity's
    column tasks are skipped and flagged, the kernels finish, and every plan
    reports LSR_EDEVICE once; afterwards the batch runs correctly again."""
    cavs = mixed(5, (256, 512))
    plans, Es, Ns = make(cavs)
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_configure(b, engine=0, graph_k=0)
    lsr.lsr_batch_test_wait(b, 1, 64)
    lsr.lsr_batch_roundtrips(b, Es, Ns, 3)
    torch.cuda.synchronize()
    for i, p in enumerate(plans):
        with pytest.raises(lsr.LsrError) as ei:
            p.sync()
        assert ei.value.code == lsr.LSR_EDEVICE, i
        p.sync()          # the report cleared the flag
    lsr.lsr_batch_test_wait(b, 0, 0)
    for c, e, n in zip(cavs, Es, Ns):
        e0, n0 = initial_state(c)
        e.copy_(torch.from_numpy(e0).to(e.device, e.dtype))
        n.copy_(torch.from_numpy(n0).to(n.device, n.dtype))
    lsr.lsr_batch_roundtrips(b, Es, Ns, 4)
    for p in plans:
        p.sync()
    ref, ref_tr = plain_reference(cavs, 4)
    for i in range(len(cavs)):
        assert torch.equal(Es[i], ref[i][0]) and torch.equal(Ns[i], ref[i][1]), i
        assert np.array_equal(plans[i].trace(4), ref_tr[i]), i
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


@pytest.mark.parametrize("graph_k", [0, 5, 12])
def test_batch_plan_matches_the_one_cavity_plan_of_256(graph_k):
    """Batch FFT plan 1 of 256 is the one-cavity FFT plan 1 (8 points per
    lane): a batch of one (and of three) on it, eager or replayed from
    graphs, is bitwise the plan path with lsr_plan_set_fft_plan(p, 1)."""
    cavs = [c.with_(N=256) for c in sweep(3, seed=23, sizes=(256,))]
    trips = 11
    ref = []
    for c in cavs:
        p = lsr.Plan(c)
        lsr.lsr_plan_set_fft_plan(p.handle, 1)
        e, n = p.state(*initial_state(c))
        p.roundtrips(e, n, trips)
        p.sync()
        ref.append((e, n))
        p.close()
    for subset in ([0], [0, 1, 2]):
        plans, Es, Ns = make([cavs[i] for i in subset])
        b = lsr.lsr_batch_create([p.handle for p in plans])
        cfg = lsr.lsr_batch_configure(b, engine=1, shape=1, graph_k=graph_k)
        assert cfg["shape"] == 1
        if graph_k:
            lsr.lsr_batch_prepare(b, trips)
        lsr.lsr_batch_roundtrips(b, Es, Ns, trips)
        for p in plans:
            p.sync()
        for j, i in enumerate(subset):
            assert torch.equal(Es[j], ref[i][0]) and torch.equal(Ns[j], ref[i][1]), (subset, i)
        lsr.lsr_batch_destroy(b)
        for p in plans:
            p.close()
