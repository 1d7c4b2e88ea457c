"""Checks against numbers the paper prints (tests/golden/paper_numbers.json)."""
import json
import os

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_vortex_input_reading_matches_printed_minimum_pressure():
    # The printed vortex formula with mu = 5.389489439 gives a negative centre
    # pressure; with the 1/(2 pi) factors the centre pressure is the printed 5.3e-12.
    prob = I.vortex(8, mu=GOLD["vortex_mu"]["value"])
    w = prob.prim(np.array([0.0]), np.array([0.0]), 0.0)
    g = GOLD["vortex_central_pressure"]
    assert w[7][0] == pytest.approx(g["value"], rel=g["rel_tol"])


def test_simpson_rule_reproduces_printed_nodes_and_weights():
    # The Simpson weights are the 3-point Newton-Cotes weights: integrate 1, x^2, x^4 exactly... up to degree 3.
    x = np.array(GOLD["simpson_nodes"]["value"])
    w = np.array(GOLD["simpson_weights"]["value"])
    for k in range(4):
        exact = ((0.5) ** (k + 1) - (-0.5) ** (k + 1)) / (k + 1)
        assert np.dot(w, x ** k) == pytest.approx(exact, abs=1e-15)


def test_newton_iterations_on_a_limiter_active_run(oracle):
    p = I.random_shock(20, 17, seed=1, bc=I.OUTFLOW)
    u = I.sample(p)
    c = oracle.Counters()
    for _ in range(6):
        u, _ = oracle.step(p, u, counters=c)
    assert c.n_newton > 0
    assert c.newton_iters_max <= GOLD["newton_iterations_max"]["value"] + 1
