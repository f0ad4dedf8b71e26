"""The solver's compiled tables, run on the host by the library's emulator
(mcc_debug_emulate_cell), against the oracle: f at a state, and the solution
of the Newton system (I - c J) x = b from the sparse level-scheduled LU and
the two triangular sweeps.  The emulator also counts schedule violations
(offsets out of range, same-level read/write hazards), which must be zero."""
import numpy as np
import pytest

from paper_2501_00011_amd import mcchem, synth


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_small, synth.mech_medium,
                                     synth.mech_large])
@pytest.mark.parametrize("c", [1e-9, 1e-3, 10.0])
def test_emulated_solver_phases_match_oracle(oracle_mod, mech_fn, c):
    m = mech_fn()
    h = mcchem.Mechanism(m, device=-1)
    o = oracle_mod.Oracle(m)
    cells = synth.make_cells(m, 3, seed=31)
    k = o.rate_constants(cells.T, cells.jscale)
    f_ref, fs = o.deriv(k, cells.y0)
    J_ref, _ = o.jac(k, cells.y0)
    rng = np.random.default_rng(5)
    for cell in range(3):
        b = rng.normal(size=m.n_species) * cells.y0[:, cell]
        f, x, viol = h.emulate_cell(k[:, cell], cells.y0[:, cell], c, b)
        assert viol == 0
        assert np.all(np.abs(f - f_ref[:, cell]) <= 1e-12 * fs[:, cell])
        M = np.eye(m.n_species) - c * J_ref[cell]
        x_ref = np.linalg.solve(M, b)
        # backward-stable solves: the residual is at roundoff of |M||x|
        resid = np.abs(M @ x - b)
        scale = np.abs(M) @ np.abs(x) + np.abs(b)
        assert np.all(resid <= 1e-12 * scale), (resid / scale).max()
        cond = np.linalg.cond(M)
        assert np.max(np.abs(x - x_ref)) <= 1e-13 * cond * np.max(np.abs(x_ref))


@pytest.mark.parametrize("tail", [0, 32, 48, 64])
def test_emulated_solver_every_dense_tail(oracle_mod, tail):
    """The 72-species mechanism compiled with every dense-tail size (the
    autotuner's choices): f and the Newton solve from the tables, with the
    compact state layout each size implies."""
    m = synth.mech_medium()
    h = mcchem.Mechanism(m, device=-1, dense_tail=tail)
    assert h.schedule_info()["dense_tail"] == tail
    o = oracle_mod.Oracle(m)
    cells = synth.make_cells(m, 2, seed=37)
    k = o.rate_constants(cells.T, cells.jscale)
    f_ref, fs = o.deriv(k, cells.y0)
    J_ref, _ = o.jac(k, cells.y0)
    rng = np.random.default_rng(tail)
    for cell in range(2):
        b = rng.normal(size=m.n_species) * cells.y0[:, cell]
        f, x, viol = h.emulate_cell(k[:, cell], cells.y0[:, cell], 1e-3, b)
        assert viol == 0
        assert np.all(np.abs(f - f_ref[:, cell]) <= 1e-12 * fs[:, cell])
        M = np.eye(m.n_species) - 1e-3 * J_ref[cell]
        resid = np.abs(M @ x - b)
        assert np.all(resid <= 1e-12 * (np.abs(M) @ np.abs(x) + np.abs(b)))


def test_emulator_handles_tiny_mechanisms():
    for rx in ([([0], [(1, 1.0)], 0.5, 0.0, 0)],
               [([0, 0, 0], [(1, 1.0)], 0.25, 0.0, 0)],
               [([0, 1], [(2, 1.0)], 1.0, 0.0, 0), ([2], [(0, 1.0), (1, 1.0)], 0.1, 0.0, 0)]):
        n = 1 + max(max(r[0]) for r in rx)
        n = max(n, 1 + max(p[0] for r in rx for p in r[1]))
        m = synth.mechanism_from_lists(n, rx)
        h = mcchem.Mechanism(m, device=-1)
        y = np.linspace(1.0, 2.0, n)
        f, x, viol = h.emulate_cell(np.array([r[2] for r in rx]), y, 0.1, np.ones(n))
        assert viol == 0
        assert np.all(np.isfinite(x))


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_small, synth.mech_medium,
                                     synth.mech_large])
def test_emulated_fj_tables_match_oracle(oracle_mod, mech_fn):
    m = mech_fn()
    h = mcchem.Mechanism(m, device=-1)
    o = oracle_mod.Oracle(m)
    cells = synth.make_cells(m, 3, seed=37)
    k = o.rate_constants(cells.T, cells.jscale)
    f_ref, fs = o.deriv(k, cells.y0)
    J_ref, Js = o.jac(k, cells.y0)
    rp, ci = h.jac_pattern()
    rows = np.repeat(np.arange(m.n_species), np.diff(rp))
    for cell in range(3):
        f, J, viol = h.emulate_fj(k[:, cell], cells.y0[:, cell])
        assert viol == 0
        assert np.all(np.abs(f - f_ref[:, cell]) <= 1e-12 * fs[:, cell])
        assert np.all(np.abs(J - J_ref[cell][rows, ci]) <= 1e-12 * Js[cell][rows, ci])


def test_fj_tables_split_wide_units():
    """A species changed by more reactions than one chunk holds is split into
    parts that accumulate into the same output."""
    n = 60
    rx = [([i], [(0, 1.0)], 1e-3 * (i + 1), 0.0, 0) for i in range(1, n)]
    m = synth.mechanism_from_lists(n, rx)
    h = mcchem.Mechanism(m, device=-1)
    k = np.array([r[2] for r in rx])
    y = np.linspace(1.0, 2.0, n)
    f, J, viol = h.emulate_fj(k, y)
    assert viol == 0
    assert f[0] == pytest.approx(float(np.sum(k * y[1:])), rel=1e-14)
    np.testing.assert_allclose(f[1:], -k * y[1:], rtol=1e-15)


def test_fj_tables_wide_item():
    """A species formed by 130 reactions: its f row spans many chunks of one
    work item, the later ones adding to what the first wrote."""
    n = 140
    rx = [([i, i + 1], [(0, 1.0)], 1e-3 * (1 + i % 7), 0.0, 0) for i in range(1, 131)]
    m = synth.mechanism_from_lists(n, rx)
    h = mcchem.Mechanism(m, device=-1)
    k = np.array([r[2] for r in rx])
    y = np.linspace(1.0, 2.0, n)
    f, J, viol = h.emulate_fj(k, y)
    assert viol == 0
    r = k * y[1:131] * y[2:132]
    assert f[0] == pytest.approx(float(np.sum(r)), rel=1e-14)


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_medium])
def test_generated_fj_kernel_compiles(mech_fn):
    """The mechanism-specialised f/J and VJP kernels are generated from the
    compiled tables and compile for gfx950 with hipRTC (no GPU needed)."""
    m = mech_fn()
    h = mcchem.Mechanism(m, device=-1)
    src = h.fj_source()
    # one switch case per work item; every output row stored exactly once
    n_items = src.count("    case ")
    assert n_items >= 2
    rp, _ = h.jac_pattern()
    for i in range(m.n_species):
        assert src.count(f"st_out(&F[{i} * ld], acc);") == 1
        assert src.count(f"st_out(&GY[{i} * ld], g{i});") == 1
    for e in range(int(rp[-1])):
        assert src.count(f"st_out(&G[{e} * ld], acc);") == 1
    for j in range(m.n_reactions):
        assert src.count(f"st_out(&GK[{j} * ld], ") == 1
    assert h.compile_fj("gfx950") > 0


def test_fj_kernel_kind_validation():
    h = mcchem.Mechanism(synth.mech_small(), device=-1)
    h.set_fj_kernel(mcchem.Mechanism.FJ_TABLES)
    h.set_fj_kernel(mcchem.Mechanism.FJ_GENERATED)
    with pytest.raises(mcchem.MccError):
        h.set_fj_kernel(7)


def test_dense_tail_configuration():
    """The caller may fix the dense-tail size; every admissible choice gives
    tables that solve the Newton system correctly; invalid choices fail."""
    m = synth.mech_medium()
    for M in (0, 32, 48, 64):
        h = mcchem.Mechanism(m, device=-1, dense_tail=M)
        assert h.schedule_info()["dense_tail"] == M
        rng = np.random.default_rng(M)
        y = synth.make_cells(m, 1, seed=9).y0[:, 0]
        k = rng.uniform(1e-3, 1.0, m.n_reactions)
        b = rng.normal(size=m.n_species)
        f, x, viol = h.emulate_cell(k, y, 1e-3, b)
        assert viol == 0 and np.all(np.isfinite(x))
    for bad in (16, 200):
        with pytest.raises(mcchem.MccError, match="status 1"):
            mcchem.Mechanism(m, device=-1, dense_tail=bad)
    with pytest.raises(mcchem.MccError):
        mcchem.Mechanism(synth.mech_small(), device=-1, dense_tail=32)


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_medium, synth.mech_large])
@pytest.mark.parametrize("c", [1e-6, 10.0])
def test_transposed_tables_solve_the_adjoint_system(oracle_mod, mech_fn, c):
    """The reverse-mode tables (the solver compiled for I - c J^T: transposed
    pattern, its own ordering and schedule) solve (I - c J)^T x = b."""
    m = mech_fn()
    h = mcchem.Mechanism(m, device=-1)
    o = oracle_mod.Oracle(m)
    cells = synth.make_cells(m, 2, seed=41)
    k = o.rate_constants(cells.T, cells.jscale)
    J_ref, _ = o.jac(k, cells.y0)
    rng = np.random.default_rng(8)
    for cell in range(2):
        b = rng.normal(size=m.n_species)
        _, x, viol = h.emulate_cell(k[:, cell], cells.y0[:, cell], c, b, transposed=True)
        assert viol == 0
        Mt = (np.eye(m.n_species) - c * J_ref[cell]).T
        resid = np.abs(Mt @ x - b)
        assert np.all(resid <= 1e-12 * (np.abs(Mt) @ np.abs(x) + np.abs(b)))
