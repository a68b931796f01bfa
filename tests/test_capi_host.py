"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point include/lsr.h declares, and
its host logic (table builders, shape registry, argument validation, batch
packer) must be right without any compute call.
"""
import ctypes
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from paper_1410_2855_amd import lsr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsr.h")


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(lsr.LIB_PATH):
        from paper_1410_2855_amd import build

        build.build(force=False)
    lsr.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsr_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(lsr.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    # and the binding wraps exactly the declared set
    assert sorted(lsr.exported_symbols()) == names


def test_binding_constants_match_the_header():
    text = open(HEADER).read()
    assert int(re.search(r"#define LSR_MAX_SLICES (\d+)", text).group(1)) == lsr.LSR_MAX_SLICES
    assert int(re.search(r"#define LSR_MAX_SHAPES (\d+)", text).group(1)) == lsr.LSR_MAX_SHAPES
    for name in ("LSR_MODEL_B_EULER", "LSR_MODEL_B_EXACT", "LSR_MODEL_CLASS_A", "LSR_PREC_PLAIN",
                 "LSR_PREC_FP64TAB", "LSR_PREC_FP64", "LSR_EINVAL", "LSR_EUNSUPPORTED", "LSR_ENONFINITE"):
        m = re.search(name + r"\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(lsr, name), name


def test_version_and_registry():
    assert "gfx950" in lsr.lsr_version()
    for N in (256, 384, 512, 768, 1024, 2048, 4096):
        assert lsr.lsr_supported(N, lsr.LSR_PREC_FP64TAB)
        assert lsr.lsr_supported(N, lsr.LSR_PREC_PLAIN)
    assert lsr.lsr_supported(4096, lsr.LSR_PREC_FP64)
    assert not lsr.lsr_supported(1000, lsr.LSR_PREC_FP64TAB)
    assert not lsr.lsr_supported(1024, 7)


@pytest.mark.parametrize("N", [256, 384, 512, 768, 1024, 2048, 4096])
def test_fft_shape_factorises_N(N):
    rad, lanes, lines = lsr.lsr_fft_shape(N)
    assert math.prod(rad) == N
    assert N % lanes == 0 and N % lines == 0
    assert all((N // lanes) % r == 0 for r in rad)
    assert lanes * lines <= 1024 and (lanes * lines) % 64 == 0


def _turns_exact(N, dx, lam, L, p):
    q = p if 2 * p < N else p - N
    t = Fraction(lam) * Fraction(L) * q * q / (2 * (Fraction(N) * Fraction(dx)) ** 2)
    return t - math.floor(t)


@pytest.mark.parametrize("F", [100.0, 300.0, 1000.0])
def test_propagator_table_is_fp64_reduced(F):
    """hx(p) = exp(-i pi lambda L fx^2)/N with the phase reduced exactly: the
    table's error is FP32 rounding only, although the phase reaches ~1e3 turns."""
    N, lam, L = 2048, 1.064e-6, 2e-3
    a = math.sqrt(F * lam * L)
    dx = 2 * a / N
    h = lsr.lsr_propagator_table(N, dx, lam, L)
    ps = list(range(0, N, 37)) + [N // 2, N // 2 - 1, N - 1]
    for p in ps:
        f = float(_turns_exact(N, dx, lam, L, p))
        want = complex(math.cos(2 * math.pi * f), -math.sin(2 * math.pi * f)) / N
        assert abs(h[p] - want) <= 1.2e-7 / N
    # the phase reaches (N/2)^2/(8F) turns
    assert (N / 2) ** 2 / (8 * F) > 100


@pytest.mark.parametrize("N", [256, 384, 1024])
def test_twiddle_tables(N):
    rad, _, _ = lsr.lsr_fft_shape(N)
    tab = lsr.lsr_twiddle_table(N, lsr.LSR_PREC_FP64TAB)
    plain = lsr.lsr_twiddle_table(N, lsr.LSR_PREC_PLAIN)
    want = []
    for sign, order in ((-1, rad), (1, rad[::-1])):
        ns = 1
        for R in order:
            if ns > 1:
                seg = [0j] * (ns * R)
                for k in range(ns):
                    for r in range(R):
                        th = 2 * math.pi * r * k / (ns * R)
                        at = (r // 2) * 2 * ns + 2 * k + r % 2 if R % 2 == 0 else r * ns + k
                        seg[at] = complex(math.cos(th), sign * math.sin(th))
                want.extend(seg)
            ns *= R
    want = np.asarray(want)
    assert tab.size == want.size == plain.size
    assert np.max(np.abs(tab - want)) <= 6e-8
    assert np.max(np.abs(plain - want)) <= 1e-6
    assert np.max(np.abs(plain - want)) >= np.max(np.abs(tab - want))


def test_argument_validation_without_a_device():
    bad = [
        dict(N=1000),                      # unsupported size
        dict(dx=0.0), dict(dx=-1.0), dict(lam=0.0), dict(L=-1.0),
        dict(R=0.0), dict(R=1.5), dict(F=float("nan")),
        dict(ap_kind=9), dict(ap_kind=1, ap_radius=0.0), dict(ap_kind=1, ap_order=3),
        dict(ap_kind=3), dict(prec=5),
    ]
    base = dict(N=256, dx=1e-5, lam=1.064e-6, L=2e-3, F=0.0, R=0.9, ap_kind=1, ap_radius=1e-3,
                ap_order=10, prec=lsr.LSR_PREC_FP64TAB)
    for b in bad:
        kw = dict(base)
        kw.update(b)
        with pytest.raises(lsr.LsrError) as ei:
            lsr.lsr_plan_create(**kw)
        want = lsr.LSR_EUNSUPPORTED if b.get("N") == 1000 else lsr.LSR_EINVAL
        assert ei.value.code == want, b
        assert lsr.lsr_last_error()
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_roundtrips(None, None, None, 1)
    assert ei.value.code == lsr.LSR_EINVAL
    with pytest.raises(lsr.LsrError) as ei:
        lsr.lsr_plan_set_roughness(None, np.zeros((4, 4)))
    assert ei.value.code == lsr.LSR_EINVAL


@pytest.mark.parametrize("sizes,lag", [([1024] * 5, -1), ([256, 384, 512, 768, 1024] * 3, 0),
                                       ([256, 4096], 100), ([512], 7)])
def test_pack_tasks_orders_dependencies(sizes, lag):
    t = lsr.lsr_pack_tasks(sizes, lag)
    nrb = []
    for N in sizes:
        _, _, lines = lsr.lsr_fft_shape(N)
        nrb.append(N // lines)
    assert len(t) == 2 * sum(nrb)
    seen_rows = {}
    seen = set()
    for i, (c, kind, blk) in enumerate(t):
        assert 0 <= c < len(sizes) and 0 <= blk < nrb[c]
        assert (c, kind, blk) not in seen
        seen.add((c, kind, blk))
        if kind == 0:
            seen_rows[c] = seen_rows.get(c, 0) + 1
        else:
            assert kind == 1
            assert seen_rows.get(c, 0) == nrb[c], "column task before all rows of its cavity"
    with pytest.raises(lsr.LsrError):
        lsr.lsr_pack_tasks([1000])


def test_missing_library_fails_loudly():
    """No fallback: without liblsr.so the binding raises instead of computing
    anything (fresh interpreter, so nothing is cached)."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_1410_2855_amd import lsr\n"
            "try:\n"
            "    lsr.load('/nonexistent/liblsr.so')\n"
            "except ImportError as e:\n"
            "    print('IMPORT_ERROR', e)\n"
            "    raise SystemExit(3)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 3 and "IMPORT_ERROR" in r.stdout and "not built" in r.stdout
