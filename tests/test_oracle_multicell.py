"""The oracle's Multi-cells solve (Section 3: every cell's data grouped into
one structure and solved as one system) against the single-system oracle.

Reading: one ODE system of N*C unknowns, one shared step size and order, the
WRMS norms over all N*C components.  Pins: with one cell it is the per-cell
solve bit for bit; with C cells it is the per-cell solve of the explicitly
concatenated mechanism (C copies, species offset c*N) bit for bit; on the
paper's test mechanism it meets the closed form; and its step count does not
grow with the number of cells (Section 5 reports about the same iteration
count for any number of cells, against a linear growth for One-cell)."""
import math

import numpy as np
import pytest

from paper_2501_00011_amd import synth

T_END = 60.0


def _concatenate(m, C):
    """C copies of mechanism m, copy c's species at c*N + i, reactions copy by copy."""
    N = m.n_species
    rx = []
    for c in range(C):
        for j in range(m.n_reactions):
            reac = [int(s) + c * N for s in m.reac_idx[m.reac_ptr[j]:m.reac_ptr[j + 1]]]
            prod = [(int(s) + c * N, float(yl)) for s, yl in
                    zip(m.prod_idx[m.prod_ptr[j]:m.prod_ptr[j + 1]], m.prod_yield[m.prod_ptr[j]:m.prod_ptr[j + 1]])]
            rx.append((reac, prod, float(m.A[j]), float(m.theta[j]), int(m.rxn_type[j])))
    return synth.mechanism_from_lists(N * C, rx)


def _fields_equal(a, b):
    for f in ("steps", "rejects", "newton_fails", "newton_iters", "f_evals", "jac_evals", "lu_count", "order"):
        assert a[f] == b[f], f
    assert a["h_last"] == b["h_last"]


@pytest.mark.parametrize("mech_fn,seed", [(synth.mech_small_thermal, 5), (synth.mech_medium, 6)])
def test_one_cell_is_the_per_cell_solve(oracle_mod, mech_fn, seed):
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = synth.make_cells(m, 3, seed=seed)
    k = o.rate_constants(c.T, c.jscale)
    dt = 60.0
    y_ref, s_ref, st_ref = o.solve(k, c.y0, dt)
    for i in range(3):
        y, s, st = o.solve_multicell(k[:, i:i + 1], c.y0[:, i:i + 1], dt)
        assert s == s_ref[i] == 0
        np.testing.assert_array_equal(y[:, 0], y_ref[:, i])
        _fields_equal(st, st_ref[i])


@pytest.mark.parametrize("mech_fn,C", [(synth.mech_small_thermal, 6), (synth.mech_small, 4)])
def test_cells_are_the_concatenated_system(oracle_mod, mech_fn, C):
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = synth.make_cells(m, C, seed=11)
    k = o.rate_constants(c.T, c.jscale)
    y, s, st = o.solve_multicell(k, c.y0, 60.0)
    big = _concatenate(m, C)
    ob = oracle_mod.Oracle(big)
    yb, sb, stb = ob.solve(k.T.reshape(-1, 1), c.y0.T.reshape(-1, 1), 60.0)
    assert s == 0 and sb[0] == 0
    np.testing.assert_array_equal(y.T.reshape(-1), yb[:, 0])
    _fields_equal(st, stb[0])


def _paper_cells(C):
    """Section 4's mechanism and initial values over C concatenated cells."""
    m = synth.mechanism_from_lists(3, [([0], [(1, 1.0)], 0.05, 0.0, 0), ([0], [(2, 1.0)], 0.02, 0.0, 0)])
    base = np.array([1.0, 0.0, 0.0])
    flat = np.concatenate([base + 0.1 * (c * 3 + np.arange(3) + 1) for c in range(C)])
    return m, flat.reshape(C, 3).T.copy()


def test_paper_mechanism_closed_form(oracle_mod):
    m, y0 = _paper_cells(9)
    o = oracle_mod.Oracle(m)
    k = o.rate_constants(np.full(9, 298.0), np.ones(9))
    y, s, _ = o.solve_multicell(k, y0, T_END, oracle_mod.default_opts(rtol=1e-8, atol=1e-14))
    assert s == 0
    ks = 0.07
    A = y0[0] * math.exp(-ks * T_END)
    exact = np.stack([A, y0[1] + 0.05 / ks * (y0[0] - A), y0[2] + 0.02 / ks * (y0[0] - A)])
    assert np.all(np.abs(y - exact) <= 1e-6 * np.abs(exact) + 1e2 * 1e-14)


def test_iterations_independent_of_cell_count(oracle_mod):
    """Multi-cells: about the same number of steps and f evaluations for 1
    and for 1,000 cells; One-cell: the per-cell counts add up."""
    opts = oracle_mod.default_opts(rtol=1e-8, atol=1e-14)
    counts = {}
    for C in (1, 10, 100, 1000):
        m, y0 = _paper_cells(C)
        o = oracle_mod.Oracle(m)
        k = o.rate_constants(np.full(C, 298.0), np.ones(C))
        _, s, st = o.solve_multicell(k, y0, T_END, opts)
        _, s1, st1 = o.solve(k, y0, T_END, opts)
        assert s == 0 and np.all(s1 == 0)
        counts[C] = (int(st["f_evals"]), int(st1["f_evals"].sum()))
    multi = [v[0] for v in counts.values()]
    assert max(multi) <= 1.5 * counts[1][0], counts
    assert counts[1000][1] >= 500 * counts[1][1], counts
