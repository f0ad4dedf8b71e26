"""Warm start of the outer step in the oracle: the first step size comes from
the previous outer step's h_next (the step it would have taken next)
instead of the starting-step algorithm; everything after the start is the
same integrator."""
import math

import numpy as np

import oracle as oracle_pkg
from paper_2501_00011_amd import synth


def _decay():
    return synth.mechanism_from_lists(2, [([0], [(1, 1.0)], 1.0, 0.0, 0)])


def test_h_next_is_the_step_before_the_landing_cut(oracle_mod):
    """A -> B, k = 1, from (1, 1), rtol 0, atol 100: the start gives h = 1
    (worked by hand in the controller pins); with dt = 1.5 the first step
    ends at t = 1 and the second, still of size 1, is cut to 0.5 to land on
    dt: h_last = 0.5, h_next = 1."""
    o = oracle_mod.Oracle(_decay())
    _, st, stats = o.solve(np.array([[1.0]]), np.array([[1.0], [1.0]]), 1.5,
                           oracle_mod.default_opts(rtol=0.0, atol=100.0))
    assert st[0] == 0 and stats["steps"][0] == 2
    assert abs(stats["h_last"][0] - 0.5) <= 1e-14 and abs(stats["h_next"][0] - 1.0) <= 1e-14


def test_warm_start_with_the_cold_first_step_reproduces_the_cold_solve(oracle_mod):
    """Given the very step size the starting-step algorithm chose, a warm
    start takes the same steps bit for bit (one f evaluation fewer: the
    algorithm's probe at y0 + h0 f0)."""
    m, c, dt = synth.workload("small10", 4)
    o = oracle_mod.Oracle(m)
    k = o.rate_constants(c.T, c.jscale)
    for i in range(4):
        y, s, st, tape = o.solve_taped(k[:, i], c.y0[:, i], dt)
        h0 = tape.values()[2]  # the start entry: type, order, first h
        yw, sw, stw, tw = o.solve_taped(k[:, i], c.y0[:, i], dt, oracle_mod.default_opts(warm_start=1), h_warm=h0)
        assert s == 0 and sw == 0
        assert np.array_equal(y, yw)
        assert np.array_equal(tape.values(), tw.values())
        assert stw["f_evals"] == st["f_evals"] - 1 and stw["steps"] == st["steps"]


def test_warm_started_consecutive_steps_follow_the_closed_form(oracle_mod):
    """Three consecutive 60 s steps of A -> B (k = 0.02 s^-1), each warm
    started from the previous one's h_next: exp(-k t) within the step bar,
    with fewer steps than starting afresh every time."""
    o = oracle_mod.Oracle(_decay())
    k = np.array([[0.02, 0.05]])
    y = np.array([[1.0, 2.0], [0.0, 0.5]])
    total = y.sum(axis=0)
    opts_w = oracle_mod.default_opts(rtol=1e-8, atol=1e-14, warm_start=1)
    opts_c = oracle_mod.default_opts(rtol=1e-8, atol=1e-14)
    yw, yc, h = y.copy(), y.copy(), None
    steps_w = steps_c = 0
    for n in range(1, 4):
        yw, sw, stw = o.solve(k, yw, 60.0, opts_w if h is not None else opts_c, h_warm=h)
        h = stw["h_next"]
        yc, sc, stc = o.solve(k, yc, 60.0, opts_c)
        assert np.all(sw == 0) and np.all(sc == 0)
        exact = y[0] * np.exp(-k[0] * 60.0 * n)
        for yy in (yw, yc):
            assert np.all(np.abs(yy[0] - exact) <= 1e-6 * exact + 1e-12)
            assert np.all(np.abs(yy.sum(axis=0) - total) <= 1e-12 * total)
        if n > 1:
            steps_w += int(stw["steps"].sum())
            steps_c += int(stc["steps"].sum())
    assert steps_w < steps_c


def test_nonpositive_h_next_falls_back_to_the_starting_step(oracle_mod):
    m, c, dt = synth.workload("small10", 3)
    o = oracle_mod.Oracle(m)
    k = o.rate_constants(c.T, c.jscale)
    y0, s0, st0 = o.solve(k, c.y0, dt)
    for bad in (0.0, -1.0, math.nan, math.inf):
        y1, s1, st1 = o.solve(k, c.y0, dt, oracle_pkg.default_opts(warm_start=1), h_warm=np.full(3, bad))
        assert np.array_equal(y0, y1) and np.array_equal(s0, s1)
        assert np.array_equal(st0["steps"], st1["steps"])
