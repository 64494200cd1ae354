"""Mutation check of the oracle's pins.

Each case plants one plausible mistake (a dropped +1, a transposed operand, a
wrong sign, a wrong index or array) into a copy of the oracle's source --
``oracle/oracle.c`` through a temporary build, ``oracle/mlp_ref.py`` through a
temporary module -- runs the pins of ``test_oracle.py`` against the copy, and
requires at least one pin to fail.  An unmodified copy, built the same way,
must pass every pin.  The planted mistakes live only in the temporary copies.
"""
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
import test_oracle as P
import test_oracle_deferred as D

HERE = os.path.dirname(os.path.abspath(__file__))

# (function, original text, planted mistake, what the mistake is)
C_MUTANTS = [
    ("or_peel", "level[u] = level[w] + 1;", "level[u] = level[w];",
     "peeling step without its +1"),
    ("or_peel", "pre[fill[col[e]]++] = u;", "pre[fill[col[e]]++] = col[e];",
     "G^T entries hold the target, not the source (wrong operand)"),
    ("or_peel", "pre[fill[col[e]]++] = u;", "pre[fill[u]++] = col[e];",
     "G instead of G^T (transposed operand; may crash the copy)"),
    ("or_peel", "if (cnt[u] == 0 && live[u])", "if (cnt[u] == 1 && live[u])",
     "removal one successor early"),
    ("or_counts", "t6 += fl + 1;", "t6 += fl;", "T6 without the support check"),
    ("or_counts", "out[2] = m + t4s;", "out[2] = m - t4s;", "AC4Trim total with a wrong sign"),
    ("or_counts", "t3 += deg + (int64_t)level[v] - 1;", "t3 += deg + (int64_t)level[v];",
     "AC-3 re-checks of a removed vertex off by one"),
    ("ac3_run", "(dround[w] < rounds)", "(dround[w] <= rounds)",
     "Jacobi round reading this round's removals"),
    ("ac6_dopost", "        checked += 1;\n", "",
     "AC-6 check not counted"),
    ("or_implicit_nbr", "((v << 8) | i)", "((v << 7) | i)", "wrong key of POST(v)[i]"),
    ("or_peel2", "cin[x] -= 1;", "cout[x] -= 1;", "two-sided: successor loss on the wrong counter"),
    ("or_counts2", "t_live += fo + 1 + fi + 1;", "t_live += fo + 1 + fi;",
     "two-sided live checks without the in-side support"),
    ("or_peel_preset", "            live[v] = 0;\n            q[qt++] = v;\n        }",
     "            live[v] = 0;\n        }", "preset removal not propagated"),
    ("or_counts_deferred", "t += fl + rounds;", "t += fl + rounds - 1;",
     "late registration: live vertex without its first check"),
    ("or_counts_deferred", "int64_t k = (int64_t)level[v] - 1 < R ? (int64_t)level[v] - 1 : R;",
     "int64_t k = (int64_t)level[v] < R ? (int64_t)level[v] : R;",
     "late registration: rounds of a removed vertex from its level, not level - 1"),
    ("or_counts_deferred", "const int64_t a = alpha > 1 ? alpha : 1;",
     "const int64_t a = alpha + 1;", "late registration: alpha + 1 rounds as in AC-3"),
    ("or_ac6_deferred", "if (dround[col[cur[v]]] >= rounds) { found = 1; break; }",
     "if (dround[col[cur[v]]] > rounds) { found = 1; break; }",
     "late registration: a round reading its own removals"),
    ("or_ac6_deferred", "if (row_off[v + 1] == row_off[v]) {",
     "if (0) {", "late registration: vertices without successors not removed up front"),
    ("or_ac6_deferred", "for (cur[u] += 1; cur[u] < end; cur[u] += 1) {",
     "for (; cur[u] < end; cur[u] += 1) {",
     "late registration: a handed-back vertex re-checks its old support"),
]

# (original text, planted mistake, what the mistake is) in oracle/mlp_ref.py
PY_MUTANTS = [
    ("np.log1p(indeg[dst].astype(np.float32))", "np.log1p(indeg[src].astype(np.float32))",
     "feature 3 from the source (transposed operand)"),
    ("(lu - lw)", "(lw - lu)", "degree-ratio feature with a wrong sign"),
    ('side="right"', 'side="left"', "edge source off by one list"),
    ('g["W2"] = dz2r.T @ h1', 'g["W2"] = h1.T @ dz2r', "W2 gradient transposed"),
    ('dh1 = dz2r @ P["W2"]', 'dh1 = dz2r @ P["W2"].T', "backward through W2 transposed"),
    ("np.sqrt(v_hat) + eps", "np.sqrt(v_hat + eps)", "Adam epsilon inside the root"),
    ("(1.0 - beta2 ** step)", "(1.0 - beta1 ** step)", "Adam second moment corrected by beta1"),
]


def c_pins(orc, gen):
    return [
        ("worked_example", lambda: P.test_worked_example(orc, gen)),
        ("stepwise_peel", lambda: [P.test_random_small_vs_stepwise_peel(orc, gen, s)
                                   for s in range(4)]),
        ("closed_forms", lambda: P.test_simulations_equal_closed_forms(orc, gen, 0)),
        ("exhaustive3", lambda: P.test_exhaustive_three_vertices_all_algorithms(orc, gen)),
        ("special_cases", lambda: P.test_duplicates_and_self_loops_special_cases(orc, gen)),
        ("config0", lambda: P.test_config0_closed_form(orc, gen)),
        ("implicit", lambda: P.test_implicit_generator_two_implementations(orc, gen)),
        ("two_sided_hand", lambda: P.test_two_sided_hand_examples(orc, gen)),
        ("two_sided_steps", lambda: P.test_two_sided_levels_by_whole_steps(orc, gen, 0)),
        ("two_sided_ac3", lambda: P.test_two_sided_ac3_hand_example(orc, gen)),
        ("preset_exhaustive", lambda: P.test_preset_exhaustive_three_vertices(orc, gen)),
        ("preset_totals", lambda: P.test_preset_totals_by_literal_runs(orc, gen, 0)),
        ("deferred_hand", lambda: [D.test_hand_example(orc, gen, R) for R in (2, 3, 4)]),
        ("deferred_literal",
         lambda: D.test_literal_run_against_closed_form_and_other_algorithms(orc, gen, 3)),
        ("deferred_small", lambda: D.test_no_removal_and_empty(orc, gen)),
    ]


def py_pins(mod, orc):
    return [
        ("features", lambda: P.pin_features_hand_computed(mod, orc.fin64)),
        ("finite_differences", lambda: P.pin_finite_differences(mod)),
        ("logits", lambda: P.pin_logits_hand_computed(mod)),
        ("bf16", lambda: P.pin_bf16_rounding(mod)),
        ("adam_first", lambda: P.pin_adam_first_step(mod)),
        ("adam_two", lambda: P.pin_adam_two_steps_by_hand(mod)),
    ]


def failing(pins):
    out = []
    for name, f in pins:
        try:
            with np.errstate(all="ignore"):
                f()
        except Exception:   # a failed assertion, or an error the mistake causes
            out.append(name)
    return out


def function_span(src, fn):
    """[start, end) of the definition of C function ``fn`` (its body ends at
    the first closing brace in column 0)."""
    m = re.search(r"^[A-Za-z].*\b" + re.escape(fn) + r"\(", src, re.M)
    assert m, fn
    end = src.index("\n}", m.start())
    return m.start(), end


def plant_c(src, fn, old, new):
    a, b = function_span(src, fn)
    body = src[a:b]
    assert body.count(old) == 1, (fn, old)
    return src[:a] + body.replace(old, new) + src[b:]


def run_pins(kind, path):
    """Failed pins of the copy at ``path`` (a built oracle.c, or mlp_ref.py),
    run in a child process: a planted mistake may crash the process, and a
    crash counts as a failed pin."""
    r = subprocess.run([sys.executable, "-c", RUNNER, kind, path], cwd=HERE,
                       capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return [f"crash (exit {r.returncode})"]
    return json.loads(r.stdout.strip().splitlines()[-1])


RUNNER = """
import json, sys
sys.path.insert(0, '..')
import graphgen, oracle
import test_oracle_mutation as M
kind, path = sys.argv[1], sys.argv[2]
if kind == 'c':
    oracle.swap_library(oracle.load(path))
    print(json.dumps(M.failing(M.c_pins(oracle, graphgen))))
else:
    import importlib.util
    spec = importlib.util.spec_from_file_location('mlp_ref_copy', path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    print(json.dumps(M.failing(M.py_pins(mod, oracle))))
"""


def build_c(tmp_path, text, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(text)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(so), str(c)])
    return str(so)


def write_py(tmp_path, text, name):
    path = tmp_path / f"{name}.py"
    path.write_text(text)
    return str(path)


def test_unmodified_copies_pass_every_pin(tmp_path):
    from oracle import mlp_ref
    assert run_pins("c", build_c(tmp_path, open(oracle._SRC).read(), "same")) == []
    assert run_pins("py", write_py(tmp_path, open(mlp_ref.__file__).read(), "same")) == []


@pytest.mark.parametrize("fn,old,new,what", C_MUTANTS, ids=[m[3] for m in C_MUTANTS])
def test_planted_mistake_in_oracle_c_fails_a_pin(tmp_path, fn, old, new, what):
    src = open(oracle._SRC).read()
    failed = run_pins("c", build_c(tmp_path, plant_c(src, fn, old, new), "mutant"))
    assert failed, f"no pin caught: {what}"


@pytest.mark.parametrize("old,new,what", PY_MUTANTS, ids=[m[2] for m in PY_MUTANTS])
def test_planted_mistake_in_mlp_ref_fails_a_pin(tmp_path, old, new, what):
    from oracle import mlp_ref
    src = open(mlp_ref.__file__).read()
    assert src.count(old) == 1, old
    assert run_pins("py", write_py(tmp_path, src.replace(old, new), "mutant")), \
        f"no pin caught: {what}"
