"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of oracle.c -- a dropped
factor, a wrong sign, a double-counted bond, a reordered table, a wrong
index -- compiles it, points the oracle wrapper at the broken copy, and
requires that one of the pins fails.  The real oracle passes every pin (the
other test files), so a pin that still passed here would be blind to that
class of mistake.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests import test_oracle_maps as maps
from tests import test_oracle_mu as mu_pins
from tests import test_oracle_model as model
from tests import test_oracle_stats as stats

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")


def _pin_4x4():
    stats.test_structured_chain_4x4_matches_exact_enumeration(0.125, 1.0)


def _pin_3x3():
    stats.test_general_mode_3x3_matches_exact_enumeration(1, 1.5)


def _pin_pair_delta():
    model.test_pair_delta_equals_full_energy_difference(4)


def _pin_threshold():
    model.test_threshold_always_for_downhill_and_monotone_uphill()


def _pin_sets():
    model.test_pair_sets_follow_the_paper_listing()


def _pin_schedule():
    model.test_schedule_covers_each_site_once_and_pairs_never_interact(8)


def _pin_init():
    model.test_init_has_exact_counts(32, 0.1)


def _pin_philox():
    from tests import test_oracle_rng as rng

    rng.test_philox_matches_rocrand_on_grid()


def _pin_observables():
    model.test_observables_of_known_configurations()


def _pin_charge_target():
    for L, n, Q, Nc in [(32, 0.1, 102, 256), (4, 0.0625, 0, 4), (128, 0.30, 4916, 4916)]:
        model.test_charge_target(L, n, Q, Nc)


def _pin_map_structure():
    for L in (8, 10, 16):
        maps.test_map_pairs_never_interact(L)


def _pin_map_adjacency():
    maps.test_map_first_site_uniform_and_partner_may_be_adjacent()


def _pin_nn_map_structure():
    for L in (8, 10, 16):
        maps.test_nn_map_pairs_are_adjacent_and_never_interact(L)


def _pin_grand_canonical():
    mu_pins.test_fixed_mu_samples_the_grand_canonical_ensemble(0.3, 1.0)


def _pin_controller():
    mu_pins.test_controller_holds_the_charge_on_average()


def _pin_energy():
    model.test_energy_of_known_configurations(0.25, 0.75, 1.5)


def _pin_map_chain():
    maps.test_map_mode_matches_exact_enumeration(4, 2, 1.0)


MUTANTS = [
    ("J/4 coefficient of eq. (3) dropped", "double dE = Delta * nD + V * nV + 0.25 * J * nJ;",
     "double dE = Delta * nD + V * nV + J * nJ;", _pin_4x4),
    ("bond a-b counted twice for adjacent pairs", "if (nb[k] == a) continue;", ";", _pin_pair_delta),
    ("Boltzmann factor sign flipped", "exp(-dE / T)", "exp(dE / T)", _pin_threshold),
    ("acceptance test inverted", "(u_acc < thr)", "(u_acc > thr)", _pin_4x4),
    ("q = 0 set reordered", "{0, 1}, {1, 0}}", "{1, 0}, {0, 1}}", _pin_sets),
    ("q = 0 choice over 4 of the 6 configurations", "uint32_t kq = (q == 0) ? 6u : 4u;", "uint32_t kq = 4u;",
     _pin_4x4),
    ("vertical displacement made even", "Dy[p] = (int32_t)((1 + 2 * (int64_t)k) % L);",
     "Dy[p] = (int32_t)((2 * (int64_t)k) % L);", _pin_schedule),
    ("init charges swapped", "(k < n_plus ? 2 : 3)", "(k < n_plus ? 3 : 2)", _pin_init),
    ("Philox key increment wrong", "#define PHILOX_W1 0xBB67AE85u", "#define PHILOX_W1 0xBB67AE86u", _pin_philox),
    ("staggered sign dropped", "o[5] += sgn * SIG_OF[c];", "o[5] += SIG_OF[c];", _pin_observables),
    ("charge-target ties rounded up", "Q = (dhi < dlo) ? hi : lo;", "Q = (dhi <= dlo) ? hi : lo;",
     _pin_charge_target),
    ("general-mode partner may equal the first site", "uint32_t b = bp + (bp >= a ? 1u : 0u);",
     "uint32_t b = bp;", _pin_3x3),
    ("map: neighbours of the partner not marked", "for (int h = 0; h < 2; ++h) {\n            int64_t nb[4];",
     "for (int h = 0; h < 1; ++h) {\n            int64_t nb[4];", _pin_map_structure),
    ("map: only three neighbours marked", "for (int d = 0; d < 4; ++d) marked[nb[d]] = 1;",
     "for (int d = 0; d < 3; ++d) marked[nb[d]] = 1;", _pin_map_structure),
    ("map: a drawn site is not checked for a mark", "if (!marked[cand]) {", "if (1) {", _pin_map_structure),
    ("map: N/11 pairs instead of N/10", "int64_t n = (int64_t)L * L / 10;", "int64_t n = (int64_t)L * L / 11;",
     _pin_map_structure),
    ("map: partner drawn only among sites not adjacent to the first", "site[h] = cand;\n                    break;",
     "site[h] = cand;\n                    if (h == 0) { int64_t q[4]; neighbours(L, cand, q); "
     "for (int d = 0; d < 4; ++d) marked[q[d]] = 1; }\n                    break;", _pin_map_adjacency),
    ("nearest-neighbour map: neighbours of the partner not marked", "neighbours(L, h ? b : a, q);",
     "neighbours(L, a, q);", _pin_nn_map_structure),
    ("nearest-neighbour map: partner not checked for a mark", "if (marked[b]) continue;", ";", _pin_nn_map_structure),
    ("penalty term sign flipped", "0.25 * J * nJ - mu * dS;", "0.25 * J * nJ + mu * dS;", _pin_grand_canonical),
    ("penalty controller pushes the wrong way", "*mu = *mu + kappa * (double)(Q - sumS) / (double)N;",
     "*mu = *mu + kappa * (double)(sumS - Q) / (double)N;", _pin_controller),
    ("penalty mode: neighbour spins ignored", "sG += SIG_OF[codes[nb[d]]];", ";", _pin_grand_canonical),
    ("energy: J term without the 1/4 of eq. (3)",
     "return Delta * (double)obs[1] + V * (double)obs[2] + 0.25 * J * (double)obs[3];",
     "return Delta * (double)obs[1] + V * (double)obs[2] + J * (double)obs[3];", _pin_energy),
    ("energy: charge-bond term with the wrong sign",
     "return Delta * (double)obs[1] + V * (double)obs[2] + 0.25 * J * (double)obs[3];",
     "return Delta * (double)obs[1] - V * (double)obs[2] + 0.25 * J * (double)obs[3];", _pin_energy),
    ("map step: a pair's configuration drawn with the acceptance word", "pairs[2 * i + 1], w[h], w[h + 1],",
     "pairs[2 * i + 1], w[h + 1], w[h + 1],", _pin_map_chain),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, pin):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mutant.c")
        so = os.path.join(d, "libmutant.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", *oracle.GCC_FLAGS, "-o", so, c, "-lm"])
        oracle.use_library(so)
        try:
            with pytest.raises(AssertionError):
                pin()
        finally:
            oracle.use_library(None)
    # the real oracle still passes the same pin
    pin()
