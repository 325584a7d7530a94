"""Planted mistakes in the oracle must fail its pins (CPU only).

Each case copies oracle/escg_oracle.c to a temporary directory, plants one
plausible mistake in the copy (a wrong sign, index, operand, branch order or
dropped term), builds it, and runs the pins that should catch it in a child
pytest with ESCG_ORACLE_SRC pointing at the copy.  The case passes only if
those pins fail.  The real oracle source is never modified.  A control run
builds an unmodified copy the same way and expects the pins to pass, so a
failure of a mutant is due to its mistake, not to the copy or the build.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "escg_oracle.c")

KAT = "tests/test_oracle_philox.py::test_philox_known_answers"
WORKED = "tests/test_oracle_rule.py::test_paper_worked_transitions"
FIGURE = "tests/test_oracle_rule.py::test_rpsls_matrix_matches_paper_figure"
TRUTH = "tests/test_oracle_rule.py::test_pair_rule_truth_table"
MUTUAL = ("tests/test_oracle_rule.py::"
          "test_pair_rule_mutual_dominance_selected_cell_wins")
THRESH = ("tests/test_oracle_rule.py::"
          "test_thresholds_are_floor_of_exact_probabilities")
INIT = "tests/test_oracle_rule.py::test_init_is_uniform_over_species_and_empty"
CONSERVE = ("tests/test_oracle_invariants.py::"
            "test_counts_conserve_sites_and_values_stay_in_range")
PERMUTE = "tests/test_oracle_invariants.py::test_exchange_only_permutes_sites"
UNTIL = "tests/test_oracle_invariants.py::test_run_until_agrees_with_plain_run"
L2_RSU = "tests/test_oracle_chain.py::test_L2_rsu_matches_exact_chain"
L3_RSU = "tests/test_oracle_chain.py::test_L3_rsu_matches_exact_chain"
L2_MCS = ("tests/test_oracle_chain.py::"
          "test_L2_block_schedule_mcs_equals_four_rsu_steps")
L4_PASS = "tests/test_oracle_chain.py::test_L4_one_pass_matches_exact_block_law"
L3_MOORE = "tests/test_oracle_chain.py::test_L3_moore_rsu_matches_exact_chain"
L4_MOORE = ("tests/test_oracle_chain.py::"
            "test_L4_moore_one_pass_matches_exact_block_law")
L2_PROB_RSU = ("tests/test_oracle_chain.py::"
               "test_L2_probabilistic_rsu_matches_exact_chain")
L4_PROB = ("tests/test_oracle_chain.py::"
           "test_L4_probabilistic_one_pass_matches_exact_block_law")
RNG_INIT = "tests/test_rng_artefacts.py::test_init_has_no_spatial_correlation"

# (name, text in escg_oracle.c, planted replacement, pins that must fail)
MUTANTS = [
    # Philox (Salmon et al., SC'11): multiplier on the wrong lane, key
    # schedule missing its second Weyl increment
    ("philox_multiplier_swapped",
     "uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;",
     "uint64_t p0 = (uint64_t)PHILOX_M1 * (uint64_t)x0;", [KAT]),
    ("philox_key_not_bumped",
     "        k1 += PHILOX_W1;\n", "", [KAT]),
    # circulant dominance matrix transposed (circulant-matrix equation)
    ("circulant_transposed",
     "((j - i + S) % S)", "((i - j + S) % S)", [FIGURE]),
    # Dominance Check reading the matrix with row and column swapped
    ("dominance_index_transposed",
     "D[(uint32_t)(species - 1) * S + (uint32_t)(neighbour - 1)]",
     "D[(uint32_t)(neighbour - 1) * S + (uint32_t)(species - 1)]", [WORKED]),
    # interaction without the reverse test (only the cell can win)
    ("reverse_dominance_missing",
     "            else if (dominates(neighbour, species, S, D))\n"
     "                *cell = 0;\n", "", [TRUTH]),
    # neighbour's win tested before the selected cell's
    ("neighbour_win_tested_first",
     "            if (dominates(species, neighbour, S, D))\n"
     "                *nbr = 0;\n"
     "            else if (dominates(neighbour, species, S, D))\n"
     "                *cell = 0;\n",
     "            if (dominates(neighbour, species, S, D))\n"
     "                *cell = 0;\n"
     "            else if (dominates(species, neighbour, S, D))\n"
     "                *nbr = 0;\n", [MUTUAL]),
    # migration copies instead of swapping
    ("exchange_copies",
     "        *cell = neighbour;\n        *nbr = species;\n",
     "        *cell = neighbour;\n", [TRUTH, PERMUTE]),
    # reproduction writes the wrong site
    ("reproduction_wrong_site",
     "        if (neighbour == 0)\n            *nbr = species;",
     "        if (neighbour == 0)\n            *cell = neighbour;", [TRUTH]),
    # first threshold from the selection rate instead of the exchange rate
    ("thresholds_rates_swapped",
     "*T1 = (uint32_t)floor(ldexp(ex / tot, 24));",
     "*T1 = (uint32_t)floor(ldexp(sel / tot, 24));", [THRESH]),
    # roulette order of the block schedule swapped
    ("o2_roulette_order_swapped",
     "    if (u24 < T1)\n        return ACT_EXCHANGE;\n"
     "    if (u24 < T2)\n        return ACT_SELECTION;",
     "    if (u24 < T1)\n        return ACT_SELECTION;\n"
     "    if (u24 < T2)\n        return ACT_EXCHANGE;", [L2_MCS, L4_PASS]),
    # initial lattice never empty (species 1..S only)
    ("init_never_empty",
     "(uint64_t)(S + 1u)) >> 32);", "(uint64_t)S) >> 32) + 1u;", [INIT]),
    # initial lattice: one draw shared by sites four columns apart (a
    # spatial artefact of the kind the paper's Metal generator showed)
    ("init_draws_shared_between_sites",
     "draw(seed, (uint32_t)(n >> 2), 0u, TAG_INIT << 8",
     "draw(seed, (uint32_t)(n >> 3), 0u, TAG_INIT << 8", [RNG_INIT]),
    # counts drop the last species
    ("counts_drop_last_species",
     "if (grid[n] <= S)", "if (grid[n] < S)", [CONSERVE]),
    # block pass: vertical edge (A,C) replaced by a horizontal one
    ("o2_wrong_neighbour_axis",
     "            case 2: first = A; second = C; break;",
     "            case 2: first = A; second = B; break;", [L4_PASS]),
    # block pass: row offset of the Margolus shift dropped
    ("o2_missing_row_offset",
     "uint32_t r0 = 2 * by + oy, r1", "uint32_t r0 = 2 * by, r1", [L4_PASS]),
    # block pass: both offset coordinates from the same bit
    ("o2_offset_bits_shared",
     "uint32_t ox = woff & 1u, oy = (woff >> 1) & 1u;",
     "uint32_t ox = woff & 1u, oy = woff & 1u;", [L4_PASS]),
    # block pass: orientation bit ignored (first site always selected)
    ("o2_orientation_ignored",
     "            if (orient) {", "            if (0 && orient) {",
     [L4_PASS]),
    # random-sequential step: "down" neighbour taken as "up"
    ("o1_down_is_up",
     "    case 1: nr = down; break;", "    case 1: nr = up; break;",
     [L3_RSU]),
    # random-sequential roulette: interaction band starts at 0
    ("o1_roulette_band",
     "    else if (r < ex + sel)", "    else if (r < sel)", [L2_RSU]),
    # Moore block pass: diagonal (A,D) given one slot instead of two
    ("moore_diagonal_single_slot",
     "            case 4: case 6: first = A; second = Dd; break;",
     "            case 4: first = A; second = Dd; break;", [L4_MOORE]),
    # Moore random-sequential step: up-right taken as up-left
    ("moore_o1_wrong_diagonal",
     "    case 5: nr = up; nc = right; break;",
     "    case 5: nr = up; nc = left; break;", [L3_MOORE]),
    # probabilistic dominance, block schedule: the neighbour's try not
    # conditioned on the cell's failure
    ("prob_o2_second_try_unconditioned",
     "(double)(R - A)", "(double)R", [L4_PROB]),
    # probabilistic dominance, random-sequential step: the same mistake
    ("prob_o1_second_try_unconditioned",
     "f < pxy + pyx * (1.0 - pxy)", "f < pxy + pyx", [L2_PROB_RSU]),
    # monoculture stop tested as "no species left"
    ("monoculture_off_by_one",
     "return mode == 0 ? extinct > 0 : alive <= 1;",
     "return mode == 0 ? extinct > 0 : alive < 1;", [UNTIL]),
]


def _run_pins(tmp_path, text: str, pins):
    src = tmp_path / "escg_oracle.c"
    src.write_text(text)
    env = dict(os.environ, ESCG_ORACLE_SRC=str(src))
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p",
           "no:cacheprovider", "-m", "not gpu", *pins]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=600)


def _source() -> str:
    with open(SRC) as f:
        return f.read()


def test_unmodified_copy_passes_the_pins(tmp_path):
    r = _run_pins(tmp_path, _source(), [KAT, WORKED, TRUTH, L2_RSU])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("name,orig,planted,pins", MUTANTS,
                         ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, orig, planted, pins):
    text = _source()
    assert text.count(orig) == 1, f"{name}: text to mutate not found once"
    r = _run_pins(tmp_path, text.replace(orig, planted), pins)
    # pytest exit code 1 = tests ran and some failed (2..5 would be an
    # interrupted run, an internal or usage error, or no tests collected)
    assert r.returncode == 1, (
        f"{name}: pins {pins} did not fail (exit {r.returncode})\n"
        + r.stdout[-2000:] + r.stderr[-2000:])
    assert " failed" in r.stdout
