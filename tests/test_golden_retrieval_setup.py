"""The retrieval set-up the paper prints (tests/golden/retrieval_setup.json,
each entry with its citation) against the parameter layout, the oracle's
parameter count and the synthetic parameter draws."""
import json
import os

import numpy as np

import oracle.params as op
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "retrieval_setup.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_temperature_and_total_parameter_counts():
    g = golden()
    for K, q in g["temperature_parameters"]["element_configs"]:
        lay = wl.c2_param_layout(K, q, with_eps=True)
        assert lay.n_elements * lay.order + 1 == g["temperature_parameters"]["count"]
        assert op.n_theta(lay) == g["free_chemistry_parameter_count"]["free"]


def test_free_mixing_ratios_and_the_sodium_tie():
    g = golden()
    lay = wl.c2_param_layout(3, 2, with_eps=True)
    assert lay.n_free == len(g["free_mixing_ratios"]["species"])
    # the eighth table species takes the last free ratio times a fixed factor
    assert lay.species_src[-1] == lay.species_src[-2]
    assert lay.species_factor[-1] == wl.SOLAR_NA_K
    assert list(lay.species_src[:-1]) == list(range(lay.n_free))


def test_draws_stay_inside_the_paper_priors():
    pri = golden()["priors"]
    lay = wl.c2_param_layout(3, 2, with_eps=True)
    th = wl.draw_theta(lay, 2000, seed=9)
    NT = lay.n_elements * lay.order + 1
    cols = {"log_g": th[:, 0], "f": th[:, 1], "T1_K": th[:, 3], "b_i": th[:, 4:4 + NT - 1],
            "x_i": th[:, 4 + NT - 1:4 + NT - 1 + lay.n_free]}
    for name, v in cols.items():
        kind, lo, hi = pri[name]
        assert kind in ("uniform", "log-uniform")
        assert np.all(v >= lo) and np.all(v <= hi), name


def test_paper_angle_count_is_a_compiled_tier():
    # the paper's two upward angles fall in the kernels' small angle tier
    # (up to 3), which the parity tests run at every count
    assert golden()["angles_upward"]["count"] <= 3
