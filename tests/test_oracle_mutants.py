"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch every one of them. The committed oracle is untouched.

Base-model mutants patch the first occurrence of their anchor (the base
procedure precedes the extended one in the file); extended-model mutants
patch anchors of the extended procedure and are checked by its pins."""
import os

import pytest

from oracle import oracle as O
from tests import oracle_pins as P
from tests import test_oracle_ext as X

MUTANTS = {
    "eq1_strict_tie": ("while (out->n > 0 && out->t[out->n - 1] >= t_r)",
                       "while (out->n > 0 && out->t[out->n - 1] > t_r)"),
    "no_redundant_drop": ("if (v == current) return 0;", ";"),
    "max_not_min_delay": ("if (d < del) del = d;", "if (del == O1_INF || d > del) del = d;"),
    "unchanged_pins_in_min": ("if (!changed[i]) continue; /* no edge on this pin: infinite delay */",
                              ";"),
    "rise_fall_swapped": ("if (out_value == 1) return rise;\n    if (out_value == 0) return fall;",
                          "if (out_value == 1) return fall;\n    if (out_value == 0) return rise;"),
    "x_delay_max": ("return rise < fall ? rise : fall;", "return rise > fall ? rise : fall;"),
    "table1_and_typo": ("    {0, 1, 2, 2},\n    {0, 2, 2, 2},\n    {0, 2, 2, 2},\n};\nstatic const uint8_t TABLE1_OR",
                        "    {0, 1, 1, 2},\n    {0, 2, 2, 2},\n    {0, 2, 2, 2},\n};\nstatic const uint8_t TABLE1_OR"),
    "z_not_read_as_x": ("static uint8_t z_as_x(uint8_t a) { return a == O1_Z ? O1_X : a; }",
                        "static uint8_t z_as_x(uint8_t a) { return a; }"),
    "prev_output_not_updated": ("        previous_output = new_output;\n", "\n"),
    "initial_output_zero": ("uint8_t previous_output = O1_X;", "uint8_t previous_output = 0;"),
    "initial_inputs_zero": ("current_signals[i] = O1_X;", "current_signals[i] = 0;"),
    "deny_only_last": ("while (out->n > 0 && out->t[out->n - 1] >= t_r) out->n--;",
                       "if (out->n > 0 && out->t[out->n - 1] >= t_r) out->n--;"),
    "drop_against_previous_eval": ("uint8_t current = out->n > 0 ? out->v[out->n - 1] : O1_X;",
                                   "uint8_t current = out->n > 1 ? out->v[out->n - 2] : O1_X;"),
    "mux_select_swapped": ("if (s == 0) return d0;\n        if (s == 1) return d1;",
                           "if (s == 0) return d1;\n        if (s == 1) return d0;"),
    "and4_drops_a_pin": ("TABLE1_AND[TABLE1_AND[TABLE1_AND[in[0]][in[1]]][in[2]]][in[3]]",
                         "TABLE1_AND[TABLE1_AND[in[0]][in[1]]][in[2]]"),
}


EXT_MUTANTS = {
    "edge_rise_fall_swapped": (
        "if (new_v == 1 || (old_v == 0 && (new_v == O1_X || new_v == O1_Z))) return 0;\n"
        "    if (new_v == 0 || (old_v == 1 && (new_v == O1_X || new_v == O1_Z))) return 1;",
        "if (new_v == 1 || (old_v == 0 && (new_v == O1_X || new_v == O1_Z))) return 1;\n"
        "    if (new_v == 0 || (old_v == 1 && (new_v == O1_X || new_v == O1_Z))) return 0;"),
    "edge_ignores_old_value": ("edge[i] = edge_of(current_signals[i], in_v[i][j]);",
                               "edge[i] = edge_of(O1_X, in_v[i][j]);"),
    "xz_change_counts_as_rise": ("return 2; /* X <-> Z */", "return 0;"),
    "x_output_uses_only_out0": ("if (out != O1_X && o != out) continue;",
                                "if (o != (out == 1)) continue;"),
    "inf_candidate_kept": ("if (del != O1_INF && add_signal_change(out, new_output, t_earliest + del)) return -1;",
                           "if (add_signal_change(out, new_output, del == O1_INF ? (int64_t)1 << 40 : t_earliest + del)) return -1;"),
    "inf_read_as_zero": ("if (x != O1X_NO_RELATION && x < best) best = x;",
                         "if ((x == O1X_NO_RELATION ? 0 : x) < best) best = x == O1X_NO_RELATION ? 0 : x;"),
    "table_misindexed": ("packed |= current_signals[i] << (2 * i);",
                         "packed |= current_signals[i] << i;"),
}


@pytest.mark.parametrize("name", sorted(EXT_MUTANTS))
def test_extended_mutant_is_caught(name, tmp_path):
    src = open(O.SRC).read()
    a, b = EXT_MUTANTS[name]
    assert src.count(a) == 1, f"mutation anchor for {name} not unique"
    path = tmp_path / "o1_mut.c"
    path.write_text(src.replace(a, b))
    lib = O.build(force=True, src=str(path), out=str(tmp_path / f"libo1_{name}.so"))
    assert X.check_ext(lib), f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(O.SRC).read()
    a, b = MUTANTS[name]
    assert src.count(a) >= 1, f"mutation anchor for {name} missing"
    path = tmp_path / "o1_mut.c"
    path.write_text(src.replace(a, b, 1))
    lib = O.build(force=True, src=str(path), out=str(tmp_path / f"libo1_{name}.so"))
    fails = []
    for check in P.FAST_CHECKS:
        fails += check(lib)
        if fails:
            break
    if not fails:
        fails = P.check_bruteforce_o3(lib, cases_per_type=60, seed=5)
    assert fails, f"no pin caught mutant {name}"
