"""The pins must catch plausible mistakes in the oracle.

Each mutant below is the oracle's C source with one deliberate, plausible mistake (a dropped
term, a wrong sign or index, a transposed operand, a reversed tie-break, a missing wrap). Each is
compiled on the CPU and the `pin`-marked tests are run against it in a separate process; every
mutant must make at least one of them fail. Mistakes are planted only here, in throwaway copies
of the oracle; nothing runs on a GPU.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ht_oracle.c")

MUTANTS = [
    ("sign of A2*x", "float num = s.r2 - ax;", "float num = s.r2 + ax;"),
    ("k = 1/y instead of 1/(2y)", "h->k = 1.0f / twice_y;", "h->k = 1.0f / y;"),
    ("dropped b_min offset", "float d = B - b_min;", "float d = B;"),
    ("half-plane sign", "return (lhs - rhs) >= 0.0f;", "return (rhs - lhs) >= 0.0f;"),
    ("theta (z, r) transposed",
     "s_th += half_plane(th_cs[2 * m], th_cs[2 * m + 1], z, h->r);",
     "s_th += half_plane(th_cs[2 * m], th_cs[2 * m + 1], h->r, z);"),
    ("phi neighbour side swapped",
     "pc[1] = (s_phi & 1) ? (pc[0] + 1) % g->n_phi : (pc[0] - 1 + g->n_phi) % g->n_phi;",
     "pc[1] = (s_phi & 1) ? (pc[0] - 1 + g->n_phi) % g->n_phi : (pc[0] + 1) % g->n_phi;"),
    ("theta neighbour side swapped",
     "int32_t other = (s_th & 1) ? (s_th >> 1) + 1 : (s_th >> 1) - 1;",
     "int32_t other = (s_th & 1) ? (s_th >> 1) - 1 : (s_th >> 1) + 1;"),
    ("lower half-plane phi offset dropped", "    s_phi = g->n_phi;\n", "    s_phi = 0;\n"),
    ("tie-break reversed", "(w == v && nb < c)", "(w == v && nb > c)"),
    ("phi not periodic in peaks", "int64_t pp = (p + dp + n_p) % n_p;",
     "int64_t pp = p + dp; if (pp < 0 || pp >= n_p) continue;"),
    ("theta periodic in peaks", "if (tt < 0 || tt >= n_t || aa < 0",
     "tt = (tt + n_t) % n_t; if (aa < 0"),
    ("A bin edge instead of centre", "(double)(2 * (int64_t)i + 1) * da", "(double)(2 * (int64_t)i) * da"),
    ("threshold strict", "if (v < T) continue;", "if (v <= T) continue;"),
    ("cos/sin swapped in phi table",
     "phi_cs[2 * m] = (float)cos(ang);\n    phi_cs[2 * m + 1] = (float)sin(ang);",
     "phi_cs[2 * m] = (float)sin(ang);\n    phi_cs[2 * m + 1] = (float)cos(ang);"),
    ("last B bin dropped", "if (!(f >= 0.0f && f < nb_f)) continue;",
     "if (!(f >= 0.0f && f < nb_f - 1.0f)) continue;"),
    ("lower B edge open", "if (!(f >= 0.0f && f < nb_f)) continue;",
     "if (!(f > 0.0f && f < nb_f)) continue;"),
    ("A index reversed in the scatter", "M[(slab * n_a + i) * n_b + j] += 1u;",
     "M[(slab * n_a + (n_a - 1 - i)) * n_b + j] += 1u;"),
    ("theta boundary loop off by one", "for (int32_t m = 1; m < 2 * g->n_theta; ++m)\n    s_th",
     "for (int32_t m = 1; m < 2 * g->n_theta - 1; ++m)\n    s_th"),
    ("r2 with a minus", "float r2 = xx + yy;", "float r2 = xx - yy;"),
    ("readout phi not wrapped", "if (phi < 0.0) phi += 2.0 * kPi;", "(void)0;"),
    ("readout B at the bin edge", "((double)b + 0.5) * db", "((double)b) * db"),
    ("sector keeps the widened phi cell", "const int32_t np_cells = g->phi_sectors ? 1 : 2;",
     "const int32_t np_cells = 2;"),
    ("sector peaks compare phi neighbours", "const int dp_max = g->phi_sectors ? 0 : 1;",
     "const int dp_max = 1;"),
    ("sector of the neighbouring half-sector", "pc[0] = s_phi >> 1;",
     "pc[0] = g->phi_sectors ? ((s_phi + 1) >> 1) % g->n_phi : s_phi >> 1;"),
]


def _run_mutant(tmpdir, idx, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: %r" % old
    path_c = os.path.join(tmpdir, "mutant%d.c" % idx)
    path_so = os.path.join(tmpdir, "mutant%d.so" % idx)
    with open(path_c, "w") as fh:
        fh.write(src.replace(old, new))
    from oracle import oracle
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", path_so, path_c, "-lm"])
    env = dict(os.environ, HT_ORACLE_LIB_FOR_MUTANT_TEST=path_so)
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "pin", "-p",
                           "no:cacheprovider", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return proc.returncode, proc.stdout[-800:]


def test_every_mutant_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=6) as pool:
            futs = [pool.submit(_run_mutant, tmp, i, old, new)
                    for i, (_, old, new) in enumerate(MUTANTS)]
            results = [f.result() for f in futs]
    survivors = [MUTANTS[i][0] for i, (rc, _) in enumerate(results) if rc == 0]
    assert not survivors, "mutants not caught by any pin: %s" % survivors
    # a crash is not a catch: each mutant must fail an assertion
    for i, (rc, out) in enumerate(results):
        assert rc == 1, (MUTANTS[i][0], rc, out)
