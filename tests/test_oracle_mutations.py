"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, index or factor,
a transposed operand) in a temporary copy of the oracle's C source and runs
the pins of tests/test_oracle.py against that copy in a fresh interpreter:
at least one pin must fail.  The unmodified copy must pass.  Nothing here
touches the oracle in the repository or the GPU path.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what the mistake is, exact text in oracle/orc.c, its replacement)
MUTATIONS = [
    ("propagator sign", "H[2 * i + 1] = -sin(ph);", "H[2 * i + 1] = sin(ph);"),
    ("propagator phase doubled", "double ph = M_PI * p->lambda * Ls * (fx * fx + fy * fy);",
     "double ph = 2.0 * M_PI * p->lambda * Ls * (fx * fx + fy * fy);"),
    ("unsigned frequency index", "double fy = signed_index(q, N) / (N * p->dx);", "double fy = q / (N * p->dx);"),
    ("grid offset by half a cell", "return ((double)j - 0.5 * (double)p->N) * p->dx;",
     "return ((double)j - 0.5 * (double)p->N + 0.5) * p->dx;"),
    ("twiddle sign", "w[2 * k + 1] = sign * sin(ang);", "w[2 * k + 1] = -sign * sin(ang);"),
    ("mirror amplitude R instead of sqrt(R)", "const double sqR = sqrt(p->R);\n    const double inv_nn",
     "const double sqR = p->R;\n    const double inv_nn"),
    ("depletion without N", "return Nn + (P - Nn) / p->T1 - Nn * I;", "return Nn + (P - Nn) / p->T1 - I;"),
    ("update drops the old inversion", "return Nn + (P - Nn) / p->T1 - Nn * I;", "return (P - Nn) / p->T1 - Nn * I;"),
    ("pump pattern transposed", "double cy = cos(2.0 * M_PI * coord(y, p) / p->mod_period);",
     "double cy = cos(2.0 * M_PI * coord(x, p) / p->mod_period);"),
    ("pump not split over the sheets", "P0[i] = pump(p, y, x) / (double)m;", "P0[i] = pump(p, y, x);"),
    ("sheet step over L instead of L/m", "const double Ls = p->L / (double)m;", "const double Ls = p->L;"),
    ("mirror at the last sheet", "if (k == 0) {\n", "if (k == m - 1) {\n"),
    ("roughness sign", "if (p->rough) ph += p->rough[(size_t)y * p->N + x];",
     "if (p->rough) ph -= p->rough[(size_t)y * p->N + x];"),
    ("roughness transposed", "if (p->rough) ph += p->rough[(size_t)y * p->N + x];",
     "if (p->rough) ph += p->rough[(size_t)x * p->N + y];"),
    ("roughness replaces the curvature", "if (p->rough) ph += p->rough[(size_t)y * p->N + x];",
     "if (p->rough) ph = p->rough[(size_t)y * p->N + x];"),
    ("exact update at the wrong rate", "double rate = 1.0 / p->T1 + I;", "double rate = 1.0 / p->T1;"),
    ("class-A saturation factor", "if (p->model == 2) return exp(0.5 * Nn / (1.0 + p->T1 * I));",
     "if (p->model == 2) return exp(0.5 * Nn / (1.0 + I));"),
    ("aperture sum over A instead of A^2", "s2 += a2 * I;",
     "s2 += sqrt(a2) * I;"),
    ("general kernel conjugated", "H[2 * i + 1] = p->transfer[2 * i + 1];",
     "H[2 * i + 1] = -p->transfer[2 * i + 1];"),
    ("general kernel transposed",
     "H[2 * i] = p->transfer[2 * i];\n                H[2 * i + 1] = p->transfer[2 * i + 1];",
     "H[2 * i] = p->transfer[2 * ((size_t)pp * N + q)];\n"
     "                H[2 * i + 1] = p->transfer[2 * ((size_t)pp * N + q) + 1];"),
    ("pump modulation without the N0 factor", "return p->N0 * (1.0 + p->mod_amp * cx * cy);",
     "return p->N0 + p->mod_amp * cx * cy;"),
    ("pump period from (N - 1) dx",
     "double cx = cos(2.0 * M_PI * coord(x, p) / p->mod_period);\n"
     "    double cy = cos(2.0 * M_PI * coord(y, p) / p->mod_period);",
     "double dd = p->mod_period * (p->N - 1) / p->N;\n"
     "    double cx = cos(2.0 * M_PI * coord(x, p) / dd);\n"
     "    double cy = cos(2.0 * M_PI * coord(y, p) / dd);"),
]


def _copy(tmp, source=None):
    """A minimal tree with the oracle (source optionally replaced), its pins
    and the input generators they import."""
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(tmp, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "*.tmp*", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(tmp, "tests"),
                    ignore=shutil.ignore_patterns("__pycache__", "test_gpu_*", "test_oracle_mutations.py"))
    pkg = os.path.join(tmp, "paper_1410_2855_amd")
    os.makedirs(pkg)
    for f in ("__init__.py", "inputs.py"):
        shutil.copy(os.path.join(ROOT, "paper_1410_2855_amd", f), pkg)
    if source is not None:
        with open(os.path.join(tmp, "oracle", "orc.c"), "w") as fh:
            fh.write(source)


def _pins(tmp):
    return subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle.py", "-q", "-x",
                           "-p", "no:cacheprovider"], cwd=tmp, capture_output=True, text=True, timeout=600)


def test_unmodified_copy_passes(tmp_path):
    _copy(str(tmp_path))
    r = _pins(str(tmp_path))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("label,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_the_mistake(tmp_path, label, old, new):
    with open(os.path.join(ROOT, "oracle", "orc.c")) as fh:
        src = fh.read()
    assert src.count(old) >= 1, "mutation text not found: %s" % label
    _copy(str(tmp_path), src.replace(old, new, 1))
    r = _pins(str(tmp_path))
    assert r.returncode != 0 and "failed" in r.stdout, "%s went unnoticed:\n%s" % (label, r.stdout[-1500:])
