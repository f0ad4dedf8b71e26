"""Pins of the oracle's BDF step-size controller: the starting step
(Hairer, Norsett & Wanner I, Sec. II.4, order 1), the factor after a failed
error test, and the order and step-size selection (Shampine & Reichelt 1997,
Sec. 2.3) against hand-worked values on constructed inputs, plus the first
controller decisions of a whole solve on a problem small enough to follow by
hand."""
import json
import math
import os

import numpy as np
import pytest

import oracle as oracle_pkg
from paper_2501_00011_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handworked_controller.json")


def _golden():
    return json.load(open(GOLDEN))


def check_controller(lib_path):
    """Every hand-worked controller case; returns the names of the cases that differ."""
    g = _golden()
    c = oracle_pkg.Controller(lib_path)
    bad = []
    for case in g["start_h0"]:
        h0 = c.start_h0(case["y0"], case["f0"], case["w"], case["dt"])
        if not abs(h0 - case["expect"]) <= 1e-14 * case["expect"]:
            bad.append(case["name"])
    for case in g["start_h"]:
        h = c.start_h(case["f0"], case["f1"], case["w"], case["h0"], case["dt"])
        if not abs(h - case["expect"]) <= 1e-14 * case["expect"]:
            bad.append(case["name"])
    for case in g["reject_factor"]:
        fac = c.reject_factor(case["err"], case["order"], case["safety"], case["fac_min"])
        if not abs(fac - case["expect"]) <= 1e-14 * case["expect"]:
            bad.append(case["name"])
    for case in g["select_order"]:
        fac, k = c.select_order(np.array(case["D"]), case["w"], case["order"], case["max_order"], case["err"])
        if k != case["expect_order"] or not abs(fac - case["expect"]) <= 1e-14 * case["expect"]:
            bad.append(case["name"])
    return bad


def first_decisions(lib_path):
    """A -> B with k = 1 s^-1 from (1, 1), rtol 0, atol 100 (all weights
    0.01), worked by hand.  Start: d0 = d1 = 0.01, h0 = 0.01; y1 = (0.99,
    1.01), f1 - f0 = (0.01, -0.01), d2 = 0.01; h1 = sqrt(0.01 / 0.01) = 1 =
    100 h0, so h = 1.  Two backward-Euler steps of h = 1 halve A: z = (0.5,
    1.5), then (0.25, 1.75), with c = h / gamma_1 = 1; the Newton corrections
    are d = (0.5, -0.5) and (0.25, -0.25), so err = 0.005 / 2 = 0.0025, then
    0.00125, and D_3 = (-0.25, 0.25) gives e(k+1) = 0.0025 / 3.  After these
    two equal steps, r(k) = 0.00125^(-1/2) = 28.3 beats r(k+1) =
    (0.0025/3)^(-1/3) = 10.6: the order stays 1 and the factor 0.9 * 28.3 is
    cut to fac_max = 10.  Returns the first four tape entries as
    (type, order, value, payload)."""
    m = synth.mechanism_from_lists(2, [([0], [(1, 1.0)], 1.0, 0.0, 0)])
    o = oracle_pkg.Oracle(m, lib_path=lib_path)
    _, s, _, tape = o.solve_taped(np.array([1.0]), np.array([1.0, 1.0]), 1000.0,
                                  oracle_pkg.default_opts(rtol=0.0, atol=100.0))
    v = tape.values()
    out, p = [], 0
    while p < len(v) and len(out) < 4:
        t = int(v[p])
        n = 2 if t == 2 else 0
        out.append((t, int(v[p + 1]), float(v[p + 2]), v[p + 3:p + 3 + n].copy()))
        p += 3 + n
    return s, out


def first_decisions_ok(lib_path):
    s, e = first_decisions(lib_path)
    if s != 0 or len(e) < 4:
        return False
    want = [(0, 0, 1.0, []), (2, 1, 1.0, [0.5, 1.5]), (2, 1, 1.0, [0.25, 1.75]), (1, 1, 10.0, [])]
    for (t, k, x, z), (wt, wk, wx, wz) in zip(e, want):
        if t != wt or k != wk or not abs(x - wx) <= 1e-12 * wx:
            return False
        if len(z) != len(wz) or np.any(np.abs(np.array(z) - np.array(wz, dtype=float)) > 1e-13):
            return False
    return True


def test_controller_against_handworked_cases(oracle_mod):
    assert check_controller(oracle_mod.LIB_PATH) == []


def test_first_controller_decisions_of_a_solve(oracle_mod):
    s, e = first_decisions(oracle_mod.LIB_PATH)
    assert s == 0
    assert [x[:2] for x in e] == [(0, 0), (2, 1), (2, 1), (1, 1)], e
    assert first_decisions_ok(oracle_mod.LIB_PATH), e


def test_golden_closed_forms_evaluate_to_the_stored_values():
    """The irrational entries of the golden file are the closed forms written
    in their derivations; re-evaluating those forms guards against a typo in
    the stored decimals."""
    g = _golden()
    by_name = {c["name"]: c["expect"] for sec in ("start_h", "reject_factor", "select_order") for c in g[sec]}
    assert by_name["T1 curvature bound"] == pytest.approx(0.1 * 2 ** 0.25, rel=1e-15)
    assert by_name["T6 weights"] == pytest.approx(math.sqrt(0.02 / math.sqrt(0.025)), rel=1e-15)
    assert by_name["T8 d1 largest"] == pytest.approx(math.sqrt(0.2 * math.sqrt(2)), rel=1e-15)
    assert by_name["R4 barely failed"] == pytest.approx(0.9 * 1.0000001 ** (-1 / 6), rel=1e-15)
    assert by_name["O6 two components with weights"] == pytest.approx(0.9 * math.sqrt(20), rel=1e-15)


def test_multicell_shares_the_controller(oracle_mod):
    """One cell as a Multi-cells system takes exactly the per-cell solve's
    controller decisions (same step and rejection counts, same result)."""
    m, c, dt = synth.workload("small10")
    o = oracle_mod.Oracle(m)
    k = o.rate_constants(c.T[:1], c.jscale[:1])
    y1, s1, st1 = o.solve(k, c.y0[:, :1], dt)
    ym, sm, stm = o.solve_multicell(k, c.y0[:, :1], dt)
    assert s1[0] == 0 and sm == 0
    assert (st1["steps"][0], st1["rejects"][0]) == (stm["steps"], stm["rejects"])
    assert np.array_equal(y1, ym)
