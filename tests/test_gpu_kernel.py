"""A general nonlocal step, the map with kernel K of Eq. (10), given by its
transfer function (lsr_plan_set_transfer), on the GPU against the FP64
oracle, against the exact shift of a point kernel, in batches against the
one-cavity path, and the boundary's refusals."""
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


def kernel_transfer(K, dx):
    """T(f) = dx^2 sum_u K(u) exp(+2 pi i f.u/N) for a kernel sampled at the
    grid offsets u (frequency order)."""
    n = K.shape[0]
    return dx * dx * n * n * np.fft.ifft2(K)


def skewed_kernel(N, dx, total=0.97):
    """A real kernel that is neither symmetric nor isotropic: a Gaussian of
    widths 2 dx (x) and 1 dx (y) centred at (1.5 dx, -0.5 dx), scaled so that
    its integral is `total`."""
    u = np.fft.fftfreq(N) * N * dx
    UX, UY = np.meshgrid(u, u)
    K = np.exp(-((UX - 1.5 * dx) ** 2 / (2 * (2 * dx) ** 2) + (UY + 0.5 * dx) ** 2 / (2 * dx ** 2)))
    return K * (total / (K.sum() * dx * dx))


def cavity(N=256):
    return Cavity(N=N, F=150.0, R=0.9, pump_ratio=2.5, T1=500.0, index=77)


def run_gpu(cav, T, prec, trips):
    p = lsr.Plan(cav, prec=prec)
    lsr.lsr_plan_set_transfer(p.handle, T)
    e, n = p.state(*initial_state(cav))
    p.roundtrips(e, n, trips)
    p.sync()
    tr = p.trace(trips)
    p.close()
    return e.cpu().numpy(), n.cpu().numpy(), tr


@pytest.mark.parametrize("N,prec,trips,tol", [
    (256, lsr.LSR_PREC_FP64TAB, 50, 1e-5), (256, lsr.LSR_PREC_PLAIN, 20, 1e-5),
    (256, lsr.LSR_PREC_FP64, 50, 1e-11), (768, lsr.LSR_PREC_FP64TAB, 20, 1e-5),
    (2048, lsr.LSR_PREC_FP64TAB, 3, 2e-6),
])
def test_general_kernel_map_matches_the_oracle(N, prec, trips, tol):
    cav = cavity(N)
    T = kernel_transfer(skewed_kernel(N, cav.dx), cav.dx)
    eg, ng, tg = run_gpu(cav, T, prec, trips)
    par = oracle_params(cav)
    par.transfer = T
    eo, no, to = oracle.run(par, *initial_state(cav), trips)
    print("N=%d prec=%d, %d trips: E %.2e N %.2e trace %.2e" % (N, prec, trips, rel(eg, eo), rel(ng, no), rel(tg, to)))
    assert rel(eg, eo) <= tol and rel(ng, no) <= tol
    assert rel(tg, to) <= max(tol, N ** 2 * 2.3e-16)


def test_point_kernel_shifts_the_field_exactly():
    """K = one point at offset (3, -2) cells with weight 1/dx^2, no gain, no
    aperture, R = 1: one trip moves the field to E(x + s), on the GPU alone."""
    N = 512
    cav = Cavity(N=N, F=200.0, R=1.0, pump_ratio=0.0, T1=100.0, index=5, ap_kind=0, n0_override=0.0)
    K = np.zeros((N, N))
    K[-2 % N, 3] = 1.0 / (cav.dx * cav.dx)
    e0, n0 = initial_state(cav)
    eg, _, _ = run_gpu(cav, kernel_transfer(K, cav.dx), lsr.LSR_PREC_FP64TAB, 1)
    assert rel(eg, np.roll(e0, (2, -3), axis=(0, 1))) <= 1e-6


def test_transfer_cleared_restores_the_propagator_and_refusals():
    cav = cavity(256)
    e0, n0 = initial_state(cav)
    ref = lsr.Plan(cav)
    er, nr = ref.state(e0, n0)
    ref.roundtrips(er, nr, 4)
    ref.sync()
    p = lsr.Plan(cav)
    lsr.lsr_plan_set_transfer(p.handle, kernel_transfer(skewed_kernel(256, cav.dx), cav.dx))
    # several gain sheets are refused
    other = lsr.Plan(cav.with_(index=78))
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_plan_set_slices(p.handle, 2)
    assert ei.value.code == lsr.LSR_EINVAL
    bad = np.ones((256, 256), np.complex128)
    bad[3, 4] = np.nan
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_plan_set_transfer(p.handle, bad)
    assert ei.value.code == lsr.LSR_EINVAL
    lsr.lsr_plan_set_transfer(p.handle, None)
    e, n = p.state(e0, n0)
    p.roundtrips(e, n, 4)
    p.sync()
    assert torch.equal(e, er) and torch.equal(n, nr)
    for q in (p, other, ref):
        q.close()


@pytest.mark.parametrize("engine,graph_k", [(0, 0), (1, 0), (1, 4), (2, 4)])
def test_batch_with_general_kernels_is_bitwise_the_one_cavity_path(engine, graph_k):
    """Batches holding plans with a general transfer function, beside plans
    of the same size (default and exact-update local steps) and of another
    size, on every engine, with and without graphs: every cavity advances
    bitwise as on the one-cavity path.  Setting the function on another plan
    and clearing it on the first between calls regroups the batch, and the
    cavities still follow the one-cavity path with the same changes."""
    base = cavity(256)
    cavs = [base.with_(index=80), base.with_(index=81), base.with_(index=82, model=1),
            cavity(512).with_(index=83)]
    T = {256: kernel_transfer(skewed_kernel(256, base.dx), base.dx)}
    T[512] = kernel_transfer(skewed_kernel(512, cavs[3].dx, total=0.95), cavs[3].dx)
    first = {0: True, 1: False, 2: False, 3: True}    # which plans carry T in the first calls
    second = {0: False, 1: True, 2: False, 3: True}   # and after the change
    calls1, calls2 = (3, 4), (3,)

    def apply(p, c, on):
        lsr.lsr_plan_set_transfer(p.handle, T[c.N] if on else None)

    ref = []
    for j, c in enumerate(cavs):
        p = lsr.Plan(c)
        apply(p, c, first[j])
        e, n = p.state(*initial_state(c))
        p.roundtrips(e, n, sum(calls1))
        apply(p, c, second[j])
        p.roundtrips(e, n, sum(calls2))
        p.sync()
        ref.append((e, n))
        p.close()
    plans = [lsr.Plan(c) for c in cavs]
    for j, (p, c) in enumerate(zip(plans, cavs)):
        apply(p, c, first[j])
    st = [p.state(*initial_state(c)) for p, c in zip(plans, cavs)]
    Es, Ns = [x[0] for x in st], [x[1] for x in st]
    b = lsr.lsr_batch_create([p.handle for p in plans])
    lsr.lsr_batch_configure(b, engine=engine, graph_k=graph_k)
    for k in calls1:
        lsr.lsr_batch_roundtrips(b, Es, Ns, k)
    for j, (p, c) in enumerate(zip(plans, cavs)):
        if second[j] != first[j]:
            apply(p, c, second[j])
    for k in calls2:
        lsr.lsr_batch_roundtrips(b, Es, Ns, k)
    for p in plans:
        p.sync()
    for j in range(len(cavs)):
        assert torch.equal(Es[j], ref[j][0]) and torch.equal(Ns[j], ref[j][1]), (engine, graph_k, j)
    lsr.lsr_batch_destroy(b)
    for p in plans:
        p.close()


def test_batched_general_kernel_matches_the_oracle():
    """50 batched trips of a cavity with a general transfer function beside
    a default cavity of its size, against the FP64 oracle."""
    cav = cavity(256)
    T = kernel_transfer(skewed_kernel(256, cav.dx), cav.dx)
    p = lsr.Plan(cav)
    lsr.lsr_plan_set_transfer(p.handle, T)
    q = lsr.Plan(cav.with_(index=90))
    (e, n), (e2, n2) = p.state(*initial_state(cav)), q.state(*initial_state(cav.with_(index=90)))
    b = lsr.lsr_batch_create([p.handle, q.handle])
    lsr.lsr_batch_roundtrips(b, [e, e2], [n, n2], 50)
    p.sync()
    tr = p.trace(50)
    lsr.lsr_batch_destroy(b)
    par = oracle_params(cav)
    par.transfer = T
    eo, no, to = oracle.run(par, *initial_state(cav), 50)
    assert rel(e.cpu().numpy(), eo) <= 1e-5 and rel(n.cpu().numpy(), no) <= 1e-5
    assert rel(tr, to) <= 1e-5
    p.close()
    q.close()
