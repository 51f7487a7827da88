"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin suite against that
build in a subprocess: the suite must fail.  The shipped oracle is untouched.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dqz_oracle.c")

MUTATIONS = [
    ("lorenzo sign", "p += (s % 2 == 1) ? v : -v;", "p += (s % 2 == 0) ? v : -v;"),
    ("padding test", "if (kz && (z % g->b[0]) == 0) continue;", "if (kz && (z % g->b[0]) == 1) continue;"),
    ("tie rule", "else take_leaf = (w[next_leaf] <= w[next_int]);", "else take_leaf = (w[next_leaf] < w[next_int]);"),
    ("symbol order", "return x->s < y->s ? -1 : (x->s > y->s ? 1 : 0);", "return x->s > y->s ? -1 : (x->s < y->s ? 1 : 0);"),
    ("canonical index", "c = (c + bl_count[bits - 1]) << 1;", "c = (c + bl_count[bits]) << 1;"),
    ("cap bound", "if (d > -(int32_t)radius && d < (int32_t)radius)", "if (d >= -(int32_t)radius && d < (int32_t)radius)"),
    ("rounding mode", "dq[i] = (int32_t)rintf(t);", "dq[i] = (int32_t)roundf(t);"),
    ("patch bound", "return !(fabs((double)x - (double)xr) <= eb_abs);", "return !(fabs((double)x - (double)xr) <= 2*eb_abs);"),
    ("bit order", "v |= 1u << (31 - (w->nbits & 31));", "v |= 1u << (w->nbits & 31);"),
    ("valrel scale", "e = eb * range;", "e = eb * range * 0.5;"),
    ("code bit order", "for (int i = len - 1; i >= 0; i--) bw_put_bit", "for (int i = 0; i < len; i++) bw_put_bit"),
    ("2-layer sign", "p += ((kz + ky + kx) % 2 == 1) ? c * v : -c * v;", "p += ((kz + ky + kx) % 2 == 0) ? c * v : -c * v;"),
    ("2-layer padding", "if ((uint64_t)kz > z % g->b[0] ||", "if ((uint64_t)kz >= z % g->b[0] ||"),
    ("2-layer binomial", "for (int i = 1; i <= k; i++) c = c * (n - k + i) / i;", "for (int i = 1; i < k; i++) c = c * (n - k + i) / i;"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-shared", "-fPIC", "-o", str(lib),
                    str(mutated), "-lm"], check=True)
    env = dict(os.environ, DQZ_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation '{name}' survived the pins:\n{r.stdout[-2000:]}"
