"""The C ABI library (no GPU needed): it loads, exports every symbol include/mcc.h
declares, and its host logic (validation, compiled sizes, the Jacobian
pattern) behaves as documented.  No compute entry point is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2501_00011_amd import mcchem, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcc.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mcc_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mcc_mech_create", "mcc_cells_create", "mcc_cells_bind", "mcc_calc_deriv",
                 "mcc_calc_jac", "mcc_solve_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = mcchem.library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_version():
    o = mcchem.default_opts()
    assert (o.rtol, o.atol, o.eta_newton, o.safety) == (1e-8, 1.0, 0.03, 0.9)
    assert (o.fac_min, o.fac_max, o.fac_newton_fail, o.h_min_rel) == (0.2, 10.0, 0.5, 1e-30)
    assert (o.max_order, o.max_newton, o.max_steps) == (5, 4, 100000)
    assert b"gfx950" in mcchem.library().mcc_version()


def _expected_pattern(m):
    """Column s of row i is structurally nonzero iff some reaction has s as a
    reactant and i as a participant; the diagonal is always present."""
    N = m.n_species
    P = np.eye(N, dtype=bool)
    for j in range(m.n_reactions):
        reac = m.reac_idx[m.reac_ptr[j]:m.reac_ptr[j + 1]]
        part = np.concatenate([reac, m.prod_idx[m.prod_ptr[j]:m.prod_ptr[j + 1]]])
        for s in reac:
            P[part, s] = True
    return P


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_medium, synth.mech_large])
def test_host_compile_pattern_and_sizes(mech_fn):
    m = mech_fn()
    h = mcchem.Mechanism(m, device=-1)
    assert (h.n_species, h.n_reactions) == (m.n_species, m.n_reactions)
    rp, ci = h.jac_pattern()
    P = np.zeros((m.n_species, m.n_species), dtype=bool)
    for i in range(m.n_species):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)  # sorted, unique
        P[i, cols] = True
    np.testing.assert_array_equal(P, _expected_pattern(m))
    assert h.nnz == P.sum()
    # fill-in never removes entries and never exceeds the dense matrix
    assert h.nnz <= h.lu_nnz <= m.n_species ** 2
    # one cell of the solver fits in the 160 KiB local data share of a CU
    assert h.solver_lds_bytes <= 160 * 1024
    h.close()


def test_jacobian_pattern_of_oracle_is_inside_compiled_pattern(oracle_mod):
    m = synth.mech_medium()
    h = mcchem.Mechanism(m, device=-1)
    rp, ci = h.jac_pattern()
    o = oracle_mod.Oracle(m)
    c = synth.make_cells(m, 2, seed=3)
    J, _ = o.jac(o.rate_constants(c.T, c.jscale), c.y0)
    inside = np.zeros_like(J[0], dtype=bool)
    for i in range(m.n_species):
        inside[i, ci[rp[i]:rp[i + 1]]] = True
    assert np.all(J[:, ~inside] == 0.0)


def _bad(m, **changes):
    import copy
    b = copy.deepcopy(m)
    for k, v in changes.items():
        setattr(b, k, v)
    return b


@pytest.mark.parametrize("case", ["species_range", "arity0", "arity4", "nan_A", "neg_A", "bad_type",
                                  "nan_yield", "zero_species"])
def test_validation_rejects(case):
    m = synth.mechanism_from_lists(4, [([0, 1], [(2, 1.0)], 1e-12, 100.0, 0),
                                       ([3], [(0, 0.5), (1, 0.5)], 1e-3, 0.0, 1)])
    if case == "species_range":
        b = _bad(m, reac_idx=np.array([0, 7, 3], dtype=np.int32))
    elif case == "arity0":
        b = _bad(m, reac_ptr=np.array([0, 0, 3], dtype=np.int32), reac_idx=np.array([0, 1, 3], dtype=np.int32))
    elif case == "arity4":
        b = synth.mechanism_from_lists(5, [([0, 1, 2, 3], [(4, 1.0)], 1e-12, 0.0, 0)])
    elif case == "nan_A":
        b = _bad(m, A=np.array([np.nan, 1e-3]))
    elif case == "neg_A":
        b = _bad(m, A=np.array([-1.0, 1e-3]))
    elif case == "bad_type":
        b = _bad(m, rxn_type=np.array([0, 7], dtype=np.int32))
    elif case == "nan_yield":
        b = _bad(m, prod_yield=np.array([1.0, np.inf, 0.5]))
    else:
        b = _bad(m, n_species=0)
    with pytest.raises(mcchem.MccError, match="status 2"):
        mcchem.Mechanism(b, device=-1)


def test_host_only_mechanism_refuses_cells():
    h = mcchem.Mechanism(synth.mech_small_thermal(), device=-1)
    with pytest.raises(mcchem.MccError, match="status 5"):
        mcchem.Cells(h, 4)
    with pytest.raises(mcchem.MccError, match="status 1"):
        mcchem.Cells.__new__(mcchem.Cells).__init__(h, 5, 3)  # ld < n_cells


def test_mechanism_without_reactions_compiles():
    m = synth.mechanism_from_lists(3, [])
    h = mcchem.Mechanism(m, device=-1)
    assert h.nnz == 3 and h.lu_nnz == 3


def test_null_arguments_are_rejected():
    lib = mcchem.library()
    assert lib.mcc_mech_create(None, 0, None) == 1
    assert lib.mcc_solver_opts_default(None) == 1
    assert lib.mcc_mech_info(None, None, None, None, None, None) == 1
    assert lib.mcc_mech_destroy(None) == 0
    assert lib.mcc_cells_destroy(None) == 0
    assert lib.mcc_solve_step(None, None, 1.0, None, None, None, None) == 1
    assert ctypes.string_at(lib.mcc_last_error()) != b""


def test_reverse_mode_entry_points_reject_null_handles():
    """The taping solver and the reverse-mode call validate their arguments
    before touching a device."""
    lib = mcchem.library()
    assert lib.mcc_adjoint_step(None, None, None, None, 0, None, None, 0, None, None) == 1
    assert b"cells is null" in lib.mcc_last_error()
    assert lib.mcc_solve_step_taped(None, None, 60.0, None, None, None, None, None, 4, None) == 1
    assert b"cells is null" in lib.mcc_last_error()
    assert lib.mcc_replay_step(None, None, None, None, 0, None, 50, 1e-15, None, None) == 1
    assert b"cells is null" in lib.mcc_last_error()
    assert lib.mcc_cells_set_schedule(None, None) == 1
    assert b"cells is null" in lib.mcc_last_error()
    assert lib.mcc_cells_schedule_from_stats(None, None, None) == 1
    assert b"cells is null" in lib.mcc_last_error()
