"""Plants plausible mistakes in a copy of the oracle and checks the pins catch each one.

Every mutant is built from a modified copy of oracle/gee_oracle.c in a temporary
directory; the committed oracle is never touched. A mutant survives only if every pin
still passes, which would mean the pins cannot tell that mistake from the definition.
"""

import os
import shutil
import subprocess

import pytest

import pins
from gee_workloads import random_small_graph
from oracle import oracle as orc

SRC = os.path.join(os.path.dirname(orc.__file__), "gee_oracle.c")

# (name, text in the oracle, replacement)
MUTATIONS = [
    ("drop_mirror_entry", "if ((flags & OR_SYMMETRIZE) && s != d) {", "if (0) {"),
    ("self_loop_twice", "if ((flags & OR_SYMMETRIZE) && s != d) {", "if ((flags & OR_SYMMETRIZE)) {"),
    ("drop_diagonal", "if (flags & OR_DIAG) {", "if (0) {"),
    ("diag_value_two", "L->v[L->n] = 1.0;", "L->v[L->n] = 2.0;"),
    ("rescale_row_twice", "L.v[t] * dinv[L.i[t]] * dinvc[L.j[t]]", "L.v[t] * dinv[L.i[t]] * dinv[L.i[t]]"),
    ("rescale_drop_col", "L.v[t] * dinv[L.i[t]] * dinvc[L.j[t]]", "L.v[t] * dinv[L.i[t]]"),
    ("in_out_swapped", "L.v[t] * dinv[L.i[t]] * dinvc[L.j[t]]", "L.v[t] * dinvc[L.i[t]] * dinv[L.j[t]]"),
    ("directed_degrees_ignored", "if (flags & OR_DIRECTED_DEGREES)", "if (0)"),
    ("in_degree_by_row", "degc[L.j[t]] += L.v[t];", "degc[L.i[t]] += L.v[t];"),
    ("in_degree_inverse_not_sqrt", "dinvc[j] = degc[j] > 0.0 ? 1.0 / sqrt(degc[j]) : 0.0;",
     "dinvc[j] = degc[j] > 0.0 ? 1.0 / degc[j] : 0.0;"),
    ("inverse_not_sqrt", "dinv[i] = deg[i] > 0.0 ? 1.0 / sqrt(deg[i]) : 0.0;",
     "dinv[i] = deg[i] > 0.0 ? 1.0 / deg[i] : 0.0;"),
    ("zero_degree_one", "dinv[i] = deg[i] > 0.0 ? 1.0 / sqrt(deg[i]) : 0.0;",
     "dinv[i] = deg[i] > 0.0 ? 1.0 / sqrt(deg[i]) : 1.0;"),
    ("degree_by_column", "        for (int64_t t = 0; t < L.n; ++t)\n            deg[L.i[t]] += L.v[t];\n        for (int64_t t = 0; t < L.n; ++t)\n            degc",
     "        for (int64_t t = 0; t < L.n; ++t)\n            deg[L.j[t]] += L.v[t];\n        for (int64_t t = 0; t < L.n; ++t)\n            degc"),
    ("class_of_row_node", "int32_t k = labels[j];", "int32_t k = labels[i] < 0 ? labels[j] : labels[i];"),
    ("wrong_class_size", "Z[i * K + k] += L.v[t] * (1.0 / (double)nk[k]);",
     "Z[i * K + k] += L.v[t] * (1.0 / (double)(nk[k] + 1));"),
    ("no_class_scale", "Z[i * K + k] += L.v[t] * (1.0 / (double)nk[k]);", "Z[i * K + k] += L.v[t];"),
    ("transposed_scatter", "Z[i * K + k] += L.v[t] * (1.0 / (double)nk[k]);",
     "Z[j * K + (labels[i] < 0 ? k : labels[i])] += L.v[t] * (1.0 / (double)nk[labels[i] < 0 ? k : labels[i]]);"),
    ("cor_l1_norm", "double r = sqrt(ss);", "double r = ss;"),
    ("cor_dropped", "if (flags & OR_CORRELATION) {", "if (0) {"),
    ("unknown_counted", "if (y >= 0)\n            counts[y] += 1;", "if (y >= 0)\n            counts[y] += 1;\n        else\n            counts[0] += 1;"),
    ("drop_last_edge", "for (int64_t e = 0; e < E; ++e) {", "for (int64_t e = 0; e + 1 < E; ++e) {"),
]


def _check_all_pins(lib):
    """Return the names of pins that fail for this library."""
    failed = []
    checks = [(name, lambda n=name: getattr(pins, n)(lib)) for name in pins.ALL_CHEAP_PINS]
    g = random_small_graph(3, N=120, E=700, K=5, weighted=True)
    checks.append(("pin_invariants", lambda: pins.pin_invariants(lib, g)))
    checks.append(("pin_scipy_route", lambda: pins.pin_scipy_route(lib, [
        g.with_options(d, l, c, name=f"m{d}{l}{c}") for d, l, c in pins.FLAG_COMBOS])))
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(name)
        except orc.OracleError:
            failed.append(name + "(error code)")
    return failed


def test_real_oracle_passes_every_pin():
    assert _check_all_pins(orc.load()) == []


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mutant = tmp_path / f"{name}.c"
    mutant.write_text(text.replace(old, new))
    so = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(mutant), "-lm"],
                   check=True)
    failed = _check_all_pins(orc.load(str(so)))
    assert failed, f"mutant {name} survived every pin"
