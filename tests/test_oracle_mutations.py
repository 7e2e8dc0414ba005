"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of oracle/farm_oracle.c (a sign flip, a
dropped term, a transposed operand, a missing self-exclusion, a reversed
tie-break, a wrong constant or derivative), builds it with gcc, and runs the
oracle pin suites (tests/test_oracle_pins.py, tests/test_oracle_mlp_pins.py,
tests/test_oracle_rrf_pins.py) against that build in a child process.  Every
mutant must fail at least one pin; the unmodified oracle passes them in the
main suite.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "farm_oracle.c")

# (name, text in the source, replacement); the text must occur exactly once
MUTATIONS = [
    ("above sign flip", "case P_ABOVE: return logistic(dz / ORACLE_TAU);",
     "case P_ABOVE: return logistic(-dz / ORACLE_TAU);"),
    ("near drops the vertical term", "case P_NEAR: {\n        double d2 = dx * dx + dy * dy + dz * dz;",
     "case P_NEAR: {\n        double d2 = dx * dx + dy * dy;"),
    ("right-of transposed viewer axis", "case P_RIGHT_OF: return logistic((dx * right[0] + dy * right[1])",
     "case P_RIGHT_OF: return logistic((dx * right[1] + dy * right[0])"),
    ("viewing direction reversed", "double depth = dx * -right[1] + dy * right[0];",
     "double depth = dx * right[1] - dy * right[0];"),
    ("inside uses the full extent", "logistic((0.5 * ej[k] - fabs(ci[k] - cj[k]))",
     "logistic((ej[k] - fabs(ci[k] - cj[k]))"),
    ("on swaps top and bottom faces", "(ci[2] - 0.5 * ei[2]) - (cj[2] + 0.5 * ej[2])",
     "(ci[2] + 0.5 * ei[2]) - (cj[2] - 0.5 * ej[2])"),
    ("class factor dropped", "? ORACLE_CLASS_FACTOR : 1.0", "? 1.0 : 1.0"),
    ("cosine not clamped", "return dot > 0.0 ? dot : 0.0;", "return dot;"),
    ("target not excluded as its own anchor", "        if (j == i) continue;\n        double v = a[j]",
     "        double v = a[j]"),
    ("anchor tie-break by larger id", "(v == best && s->id[j] < best_id)", "(v == best && s->id[j] > best_id)"),
    ("rank tie-break by larger id", "(dc == dij && s->id[c] < s->id[i])", "(dc == dij && s->id[c] > s->id[i])"),
    ("farthest target rank off by one", "p == P_CLOSEST ? 1 : m + 1;", "p == P_CLOSEST ? 1 : m;"),
    ("geometric mean without the root", "gbar = pow(prod, 1.0 / (double)cnt);", "gbar = prod;"),
    ("blend floor dropped", "return sem * ((1.0 - ORACLE_W) + ORACLE_W * gbar);", "return sem * (ORACLE_W * gbar);"),
    ("topk tie-break by larger id", "return (id[a] < id[b]) ? -1 : (id[a] > id[b]);",
     "return (id[a] > id[b]) ? -1 : (id[a] < id[b]);"),
    ("between drops the far-side margin", "return logistic(s / ORACLE_TAU) * logistic((L - s) / ORACLE_TAU) *",
     "return logistic(s / ORACLE_TAU) *"),
    ("between's invocation counted twice in the mean", "        if (pred[rr] == P_AND) continue;\n", ""),
    ("hellinger drops the determinant factor",
     "double bc = pow(det3(A), 0.25) * pow(det3(B), 0.25) / sqrt(det3(M)) * exp(-q / 8.0);",
     "double bc = exp(-q / 8.0);"),
    ("hellinger quadratic form scaled by 1/2", "* exp(-q / 8.0);", "* exp(-q / 2.0);"),
    ("hellinger similarity taken as the squared distance", "return 1.0 - sqrt(h2);", "return 1.0 - h2;"),
    ("stored view rotation transposed",
     "xc[r] = view[3 + 3 * r] * w[0] + view[4 + 3 * r] * w[1] + view[5 + 3 * r] * w[2];",
     "xc[r] = view[3 + r] * w[0] + view[6 + r] * w[1] + view[9 + r] * w[2];"),
    ("view gate ignores the field of view",
     "return xc[2] >= ORACLE_VIEW_Z_MIN && fabs(xc[0]) <= ORACLE_VIEW_HALF_W * xc[2] &&",
     "return xc[2] >= ORACLE_VIEW_Z_MIN; return 1 &&"),
    ("left-of compares image coordinates the other way", "case P_LEFT_OF_V: return logistic((ub - ua) / ORACLE_VIEW_TAU_U);",
     "case P_LEFT_OF_V: return logistic((ua - ub) / ORACLE_VIEW_TAU_U);"),
    ("in-front-of on world height instead of camera depth",
     "case P_IN_FRONT_OF_V: return logistic((b[2] - a[2]) / ORACLE_TAU);",
     "case P_IN_FRONT_OF_V: return logistic((cj[2] - ci[2]) / ORACLE_TAU);"),
    ("supplied relation rows read without the query's offset",
     "qs->asim[(size_t)rr * n + j] = g_sim_asim[(size_t)(r0 + rr) * n + j];",
     "qs->asim[(size_t)rr * n + j] = g_sim_asim[(size_t)rr * n + j];"),
    ("gelu derivative drops its second term",
     "return 0.5 * (1.0 + erf(v / sqrt(2.0))) + v * exp(-0.5 * v * v) / sqrt(2.0 * M_PI);",
     "return 0.5 * (1.0 + erf(v / sqrt(2.0)));"),
    ("output-layer gradient uses the pre-activation", "gW3[(size_t)p * h + k] += dy * a2[k];",
     "gW3[(size_t)p * h + k] += dy * z2[k];"),
]


def _run_mutant(tmp, idx, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not unique/found"
    c_path = os.path.join(tmp, f"mutant{idx}.c")
    so_path = os.path.join(tmp, f"mutant{idx}.so")
    with open(c_path, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so_path, c_path, "-lm"])
    env = dict(os.environ, FARM_ORACLE_LIB=so_path, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_mlp_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_rrf_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        futs = [ex.submit(_run_mutant, str(tmp_path), i, *m) for i, m in enumerate(MUTATIONS)]
        results = [f.result() for f in futs]
    survivors = [(name, out) for name, rc, out in results if rc == 0]
    assert not survivors, f"mutants that passed every pin: {[n for n, _ in survivors]}"
    # a mutant must fail a pin (exit 1), not break the test run itself
    broken = [(name, rc, out) for name, rc, out in results if rc != 1]
    assert not broken, broken
