"""The oracle's pins must catch plausible mistakes (the paper's own check of
this kind: a regression test sensitive to a 1 % change of G, Sec. 10.10).

Each mutation is compiled from the oracle source with -DORC_MUTATION=k (CPU
only) and the named pin must fail on it.
"""
import os

import pytest

import oracle
from tests import test_oracle_keys as K
from tests import test_oracle_isolated as ISO
from tests import test_oracle_kernels as KN
from tests import test_oracle_pm as PM
from tests import test_oracle_relative as REL
from tests import test_oracle_softening_mixed as MS
from tests import test_oracle_tree as TR
from tests import test_oracle_walk as WK

MUTATIONS = {
    1: ("G x 1.01", [lambda o: WK.test_plummer_shells_closed_form(o),
                     lambda o: KN.test_two_body_closed_form(o)]),
    2: ("no 1.2 L box rule", [lambda o: WK.test_box_rule_opens_own_node(o)]),
    3: ("short-range factor without its Gaussian term",
        [lambda o: KN.test_short_range_factor_identity(o)]),
    4: ("wrong sign of the periodic wrap",
        [lambda o: WK.test_open_all_equals_truncated_direct_periodic(o)]),
    5: ("centre of mass not divided by the mass", [lambda o: TR.test_moments(o)]),
    6: ("FFT twiddle of the wrong sign", [lambda o: PM.test_fft_bruteforce_8(o)]),
    7: ("four-point difference with a wrong coefficient",
        [lambda o: PM.test_single_mode_solve(o, (3, 2, 5))]),
    8: ("Hilbert key without its Gray-code correction",
        [lambda o: K.test_key_bijection_adjacency_nesting(o, 3)]),
    9: ("geometric criterion with theta instead of theta^2",
        [lambda o: WK.test_plummer_config_accuracy(o)]),
    10: ("CIC weights swapped", [lambda o: PM.test_cic_mass_and_linear(o)]),
    11: ("isolated Green's function sampled at unsigned mesh offsets",
         [lambda o: ISO.test_isolated_solve_is_open_convolution(o)]),
    12: ("pair softening from the target alone",
         [lambda o: MS.test_open_all_equals_direct_mixed(o, False)]),
    13: ("no opening of nodes with larger softening",
         [lambda o: MS.test_softening_node_rule(o)]),
    14: ("relative criterion without the node's G m",
         [lambda o: REL.test_relative_threshold_exact(o),
          lambda o: REL.test_relative_unit_scaling_invariance(o, False),
          lambda o: REL.test_relative_unit_scaling_invariance(o, True)]),
    15: ("relative criterion with L in place of L^2",
         [lambda o: REL.test_relative_threshold_exact(o)]),
    16: ("relative criterion without |a_old|",
         [lambda o: REL.test_relative_threshold_exact(o),
          lambda o: REL.test_relative_unit_scaling_invariance(o, False)]),
    17: ("relative criterion with d^2 in place of d^4",
         [lambda o: REL.test_relative_threshold_exact(o)]),
}


@pytest.fixture(scope="module")
def mutdir(tmp_path_factory):
    return tmp_path_factory.mktemp("mut")


@pytest.mark.parametrize("k", sorted(MUTATIONS))
def test_mutation_is_caught(k, mutdir):
    path = os.path.join(mutdir, f"liboracle_m{k}.so")
    oracle.build(path, mutation=k)
    saved = oracle._lib
    oracle._lib = oracle.Lib(path)
    try:
        for pin in MUTATIONS[k][1]:
            with pytest.raises(AssertionError):
                pin(oracle)
    finally:
        oracle._lib = saved
