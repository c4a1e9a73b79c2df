"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (a dropped
term, a wrong weight, a flipped sign, a product in the wrong order), builds
that copy on the CPU, and runs one pin of tests/test_oracle_pins.py against
it: the pin must fail.  The oracle itself is not modified.
"""

import importlib.util
import os

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_SRC = os.path.join(ROOT, "oracle", "hgmm_oracle.c")
PY_SRC = os.path.join(ROOT, "oracle", "oracle.py")

# (case, file, original text, planted text, pin, pin arguments after the oracle)
MUTATIONS = [
    ("descent score without log|cov|", "c",
     "s_all[k] = log(t->pi[g]) - 0.5 * ld[g] - 0.5 * maha2(Lm, d);",
     "s_all[k] = log(t->pi[g]) - 0.5 * maha2(Lm, d);", "test_descent_one_level_bruteforce", ()),
    # (global weights in the sibling scores would be no mistake: they differ
    # from the sibling weights by the parent's weight, which cancels)
    ("complexity stop with the test reversed", "c",
     "int stop = (t->kappa[chosen] <= lambda_c)", "int stop = (t->kappa[chosen] > lambda_c)",
     "test_descent_greedy_path_and_limits", ()),
    ("moment mass counts points instead of weights", "c",
     "      b[0] += gm;\n      b[1] += gm * q[0];", "      b[0] += 1.0;\n      b[1] += gm * q[0];",
     "test_descent_one_level_bruteforce", ()),
    ("normal equations with the printed sign of Eq. 16", "c",
     "g[u] -= w * a[u] * r;", "g[u] += w * a[u] * r;", "test_exact_recovery_blob_tree", ()),
    ("point-to-plane weight times instead of over lambda", "c",
     "double w = pis / t->lam[3 * j + l];", "double w = pis * t->lam[3 * j + l];",
     "test_normal_equations_inverse_form", ()),
    ("complexity from the largest eigenvalue", "c",
     "t->kappa[g] = t->lam[3 * g + 2] / (", "t->kappa[g] = t->lam[3 * g] / (", "test_tree_invariants", ()),
    ("octant children without the regularisation", "c",
     "o[0] = c[0][0] + eps; o[1] = c[0][1]; o[2] = c[0][2];", "o[0] = c[0][0]; o[1] = c[0][1]; o[2] = c[0][2];",
     "test_octant_init_halfnormal_closed_form", ()),
    ("single-level mixture with sibling weights", "c",
     "cst[j] = log(t->pig[g]) - 0.5 * ld[j];", "cst[j] = log(t->pi[g]) - 0.5 * ld[j];",
     "test_flat_estep_bruteforce", ()),
    ("soft descent without the path product", "c",
     "const double e = pe * exp(s[k] - smax) / den;", "const double e = exp(s[k] - smax) / den;",
     "test_soft_estep_unpruned_leaves_bruteforce", ()),
    ("trajectory composed in the wrong order", "py",
     "R_abs[k] = R_abs[k - 1] @ R_rel[k - 1]", "R_abs[k] = R_rel[k - 1] @ R_abs[k - 1]",
     "test_compose_chain_recovers_absolute_poses", ()),
]


def _mutated_oracle(tmp_path, kind, old, new, *_):
    csrc = open(C_SRC).read()
    pysrc = open(PY_SRC).read()
    text = csrc if kind == "c" else pysrc
    assert text.count(old) >= 1, f"mutation target not found: {old!r}"
    text = text.replace(old, new, 1)
    if kind == "c":
        csrc = text
    else:
        pysrc = text
    c_path = tmp_path / "hgmm_oracle.c"
    c_path.write_text(csrc)
    (tmp_path / "hgmm_oracle.h").write_text(open(C_SRC[:-2] + ".h").read())
    py_path = tmp_path / "oracle_mutant.py"
    py_path.write_text(pysrc)
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{abs(hash((old, new)))}", str(py_path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._SRC = str(c_path)
    mod._LIB_PATH = str(tmp_path / "liboracle_mutant.so")
    mod._lib = None
    mod.build_library(force=True)
    return mod


@pytest.mark.parametrize("case,kind,old,new,pin,args", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, case, kind, old, new, pin, args):
    mod = _mutated_oracle(tmp_path, kind, old, new)
    with pytest.raises(AssertionError):
        getattr(pins, pin)(mod, *args)


def test_unmutated_copy_passes_the_same_pins(tmp_path):
    """The harness itself: an unmodified copy passes every pin used above."""
    mod = _mutated_oracle(tmp_path, "c", "#include", "#include", None, None)
    for name in sorted({m[4] for m in MUTATIONS}):
        getattr(pins, name)(mod)
