"""Planted mistakes in the oracle, on the CPU: each mutant is a copy of
oracle.c with one plausible error (a dropped term, a wrong sign, bound or
index, a changed tie rule), compiled on its own.  The oracle's pins, run
against it in a child process, must fail; the unchanged source, compiled the
same way, must pass them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MIS2 = ["tests/test_oracle_mis2.py"]
AGG = ["tests/test_oracle_aggregate.py"]
BASIC = ["tests/test_oracle_basic.py"]
ABL = ["tests/test_oracle_ablation.py"]
CGS = ["tests/test_oracle_cgs.py"]
GAL = ["tests/test_oracle_galerkin.py"]
SMO = ["tests/test_oracle_smoothed.py"]

# name: (pin files, text replaced (its first occurrence), replacement)
MUTANTS = {
    "refresh_column_without_v": (MIS2, "uint32_t m = T[v];", "uint32_t m = ORACLE_OUT;"),
    "no_in_to_out": (MIS2, "if (m == ORACLE_IN) m = ORACLE_OUT;", ";"),
    "decide_ignores_out": (MIS2, "if (M[w] == ORACLE_OUT) any_out = 1;", ";"),
    # (M_w < t0 in place of M_w != t0 would be equivalent: v is in N[w], so a
    # neighbour's M is never above T_v unless it is OUT, which decides first)
    "decide_all_equal_as_above": (MIS2, "if (M[w] != t0) all_eq = 0;",
                                  "if (M[w] > t0) all_eq = 0;"),
    "xorshift_star_shift": (MIS2, "x ^= x << 25;", "x ^= x << 24;"),
    "id_bits_bound": (MIS2, "(INT64_C(1) << b) < n + 2", "(INT64_C(1) << b) < n + 1"),
    "phase2_one_neighbour": (AGG, "if (cnt < 2) continue;", "if (cnt < 1) continue;"),
    "phase3_larger_aggregate": (AGG, "(aggsize[a] < aggsize[best] ||",
                                "(aggsize[a] > aggsize[best] ||"),
    "quotient_self_loops": (AGG, "if (a != c) { p[k].a = a; p[k].c = c; k++; }",
                            "{ p[k].a = a; p[k].c = c; k++; }"),
    "basic_join_largest": (BASIC, "if (a >= 0 && (best < 0 || a < best)) best = a;",
                           "if (a >= 0 && (best < 0 || a > best)) best = a;"),
    "xorshift_plain_shift": (ABL, "x ^= x >> 27;\n    return x;\n}\n\n/* Priority",
                             "x ^= x >> 26;\n    return x;\n}\n\n/* Priority"),
    "colouring_skips_zero": (CGS, "while (used[c]) c++;", "while (used[c] || c == 0) c++;"),
    "gauss_seidel_sign": (CGS, "r -= val[e] * x[col[e]];", "r += val[e] * x[col[e]];"),
    "galerkin_without_diagonal": (GAL, "cdiag[a] = cdiag[a] + diag[i];", "(void)diag;"),
    "galerkin_without_inner_couplings": (GAL, "cdiag[a] = cdiag[a] + val[e];", ";"),
    "galerkin_split_sqrt": (GAL, "cval[p] = cval[p] / sqrt((double)size[a] * (double)size[ccol[p]]);",
                            "cval[p] = cval[p] / (sqrt((double)size[a]) * sqrt((double)size[ccol[p]]));"),
    "galerkin_diagonal_scale": (GAL, "cdiag[a] = cdiag[a] / sqrt((double)size[a] * (double)size[a]);",
                                "cdiag[a] = cdiag[a] / sqrt((double)size[a]);"),
    "smoothed_sign": (SMO, "double r = ind - t;", "double r = ind + t;"),
    "smoothed_without_jacobi_scaling": (SMO, "double w = omega / diag[i];", "double w = omega;"),
    "smoothed_without_diagonal": (SMO, "if (agg[i] == a) s = s + diag[i];", ";"),
    "smoothed_ap_without_diagonal": (SMO, "if (pib) acc = acc + diag[i] * *pib;", ";"),
    "smoothed_tentative_scale": (SMO, "P.val[p] = r / sqrt((double)size[a]);",
                                 "P.val[p] = r / (double)size[a];"),
}


def _build(tmp_path, text):
    src = tmp_path / "oracle.c"
    src.write_text(text)
    lib = tmp_path / "liboracle.so"
    subprocess.check_call(["gcc", "-O1", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                           str(src), "-o", str(lib), "-lm"])
    return str(lib)


def _pins(lib, files):
    env = dict(os.environ, MIS2_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + files, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    return r.returncode, r.stdout[-2000:]


def test_unchanged_oracle_passes_the_pins(tmp_path):
    with open(SRC) as f:
        lib = _build(tmp_path, f.read())
    files = sorted({f for v in MUTANTS.values() for f in v[0]})
    rc, out = _pins(lib, files)
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    files, old, new = MUTANTS[name]
    with open(SRC) as f:
        text = f.read()
    assert old in text, name
    lib = _build(tmp_path, text.replace(old, new, 1))
    rc, out = _pins(lib, files)
    assert rc != 0, "%s survived the pins:\n%s" % (name, out)
