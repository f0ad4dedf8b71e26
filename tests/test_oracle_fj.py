"""Pins of the oracle's rate constants, f and J against things other than itself.

- hand-worked values of tiny mechanisms (tests/golden/handworked_fj.json),
  derived by hand from the tendency equations of Section 2 (Background);
- J against central finite differences of f;
- Euler homogeneity: a mass-action rate of order p is homogeneous of degree p
  in y, so sum_s J_is y_s = sum_p p f^(p)_i, where f^(p) is f of the
  sub-mechanism holding only the order-p reactions;
- atom balance: the generated mechanisms conserve two elements, so
  a_e^T f = 0 and a_e^T J = 0 for every state;
- the first-order special case: J is constant and f = J y.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2501_00011_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handworked_fj.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _mech_from_case(case):
    rx = [(r["reac"], [tuple(p) for p in r["prod"]], r["k"], 0.0, 0) for r in case["reactions"]]
    return synth.mechanism_from_lists(case["n_species"], rx, name=case["name"])


@pytest.mark.parametrize("idx", range(len(_golden()["cases"])))
def test_handworked_f_and_J(oracle_mod, idx):
    case = _golden()["cases"][idx]
    m = _mech_from_case(case)
    o = oracle_mod.Oracle(m)
    k = np.array([[r["k"]] for r in case["reactions"]])  # A = k, theta = 0 -> use k directly
    y = np.array(case["y"], dtype=np.float64)[:, None]
    f, _ = o.deriv(k, y)
    J, _ = o.jac(k, y)
    np.testing.assert_allclose(f[:, 0], case["f"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(J[0], np.array(case["J"]), rtol=1e-15, atol=0)


def test_handworked_rate_constants(oracle_mod):
    g = _golden()["rate_constants"]
    th, ph = g["thermal"], g["photolysis"]
    m = synth.mechanism_from_lists(2, [([0], [(1, 1.0)], th["A"], th["theta"], 0),
                                       ([0], [(1, 1.0)], ph["J"], 0.0, 1)])
    o = oracle_mod.Oracle(m)
    k = o.rate_constants(np.array([th["T"]]), np.array([ph["s"]]))
    assert k[0, 0] == pytest.approx(th["k"], rel=4e-16)
    assert k[1, 0] == pytest.approx(ph["k"], rel=0, abs=0)


def test_rate_constant_temperature_ratio(oracle_mod):
    """k(T1)/k(T2) = exp(theta (1/T2 - 1/T1)); theta = 0 gives k = A at any T."""
    m = synth.mech_medium()
    o = oracle_mod.Oracle(m)
    T = np.array([220.0, 310.0])
    k = o.rate_constants(T, np.array([0.3, 0.3]))
    thermal = m.rxn_type == 0
    ratio = k[thermal, 0] / k[thermal, 1]
    expect = np.exp(m.theta[thermal] * (1 / 310.0 - 1 / 220.0))
    np.testing.assert_allclose(ratio, expect, rtol=1e-13)
    photo = m.rxn_type == 1
    np.testing.assert_array_equal(k[photo, 0], m.A[photo] * 0.3)


def _states(mech, n_cells, seed):
    c = synth.make_cells(mech, n_cells, seed=seed)
    return c


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_medium])
def test_J_against_central_differences(oracle_mod, mech_fn):
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = _states(m, 3, seed=7)
    k = o.rate_constants(c.T, c.jscale)
    J, Js = o.jac(k, c.y0)
    _, fs = o.deriv(k, c.y0)
    N = m.n_species
    for cell in range(3):
        y = c.y0[:, cell:cell + 1]
        kk = k[:, cell:cell + 1]
        Jfd = np.zeros((N, N))
        hs = 1e-6 * np.abs(y[:, 0])
        for s in range(N):
            yp, ym = y.copy(), y.copy()
            yp[s] += hs[s]
            ym[s] -= hs[s]
            Jfd[:, s] = (o.deriv(kk, yp)[0][:, 0] - o.deriv(kk, ym)[0][:, 0]) / (2 * hs[s])
        # Truncation: central differences are exact for terms linear in y_s and
        # O(h^2) ~ 1e-12 relative for quadratic and cubic terms.  Rounding: the
        # difference of two f values of size <= fscale_i costs ~eps*fscale_i/h.
        err = np.abs(J[cell] - Jfd)
        tol = 1e-6 * Js[cell] + 1e-14 * fs[:, cell][:, None] / hs[None, :]
        assert np.all(err <= tol), (err / tol).max()
        # and the pattern: J is exactly zero where no reaction couples i and s
        assert np.all(Jfd[J[cell] == 0.0] == 0.0)


def _submech(m, order):
    keep = np.nonzero(m.arity() == order)[0]
    rx = []
    for j in keep:
        reac = m.reac_idx[m.reac_ptr[j]:m.reac_ptr[j + 1]].tolist()
        prod = list(zip(m.prod_idx[m.prod_ptr[j]:m.prod_ptr[j + 1]].tolist(),
                        m.prod_yield[m.prod_ptr[j]:m.prod_ptr[j + 1]].tolist()))
        rx.append((reac, prod, m.A[j], m.theta[j], m.rxn_type[j]))
    return synth.mechanism_from_lists(m.n_species, rx), keep


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_medium, synth.mech_large])
def test_euler_homogeneity(oracle_mod, mech_fn):
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = _states(m, 4, seed=11)
    k = o.rate_constants(c.T, c.jscale)
    J, Js = o.jac(k, c.y0)
    Jy = np.einsum("cis,sc->ic", J, c.y0)
    rhs = np.zeros_like(Jy)
    bound = np.zeros_like(Jy)
    for p in (1, 2, 3):
        sub, keep = _submech(m, p)
        if sub.n_reactions == 0:
            continue
        fp, sp = oracle_mod.Oracle(sub).deriv(k[keep], c.y0)
        rhs += p * fp
        bound += p * sp
    err = np.abs(Jy - rhs)
    assert np.all(err <= 1e-12 * bound + 1e-300), (err / bound).max()


@pytest.mark.parametrize("mech_fn", [synth.mech_small_thermal, synth.mech_medium, synth.mech_large])
def test_atom_balance(oracle_mod, mech_fn):
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = _states(m, 5, seed=13)
    k = o.rate_constants(c.T, c.jscale)
    f, fs = o.deriv(k, c.y0)
    J, Js = o.jac(k, c.y0)
    a = m.composition.astype(np.float64)  # [N, 2]
    for e in range(a.shape[1]):
        af = a[:, e] @ f
        assert np.all(np.abs(af) <= 1e-12 * (a[:, e] @ fs)), np.abs(af).max()
        aJ = np.einsum("i,cis->cs", a[:, e], J)
        aJs = np.einsum("i,cis->cs", a[:, e], Js)
        assert np.all(np.abs(aJ) <= 1e-12 * aJs + 1e-300)


def test_first_order_linear_case(oracle_mod):
    m = synth.mech_medium()
    sub, keep = _submech(m, 1)
    o = oracle_mod.Oracle(sub)
    c = _states(m, 3, seed=17)
    k = oracle_mod.Oracle(m).rate_constants(c.T, c.jscale)[keep]
    J1, _ = o.jac(k, c.y0)
    J2, _ = o.jac(k, 3.0 * c.y0 + 1.0)
    np.testing.assert_array_equal(J1, J2)
    f, fs = o.deriv(k, c.y0)
    np.testing.assert_allclose(np.einsum("cis,sc->ic", J1, c.y0), f, rtol=0, atol=1e-13 * fs.max())


def test_scale_matches_contributions(oracle_mod):
    """The f scale is a sum of absolute contributions, so |f| <= scale and the
    scale equals |f| for species with contributions of one sign only."""
    m = synth.mech_medium()
    o = oracle_mod.Oracle(m)
    c = _states(m, 4, seed=19)
    k = o.rate_constants(c.T, c.jscale)
    f, fs = o.deriv(k, c.y0)
    assert np.all(np.abs(f) <= fs * (1 + 1e-15))
    # a species that is never a product only loses mass: f = -scale
    produced = set(m.prod_idx.tolist())
    only_lost = [i for i in range(m.n_species) if i not in produced]
    for i in only_lost:
        np.testing.assert_allclose(f[i], -fs[i], rtol=1e-15)
    assert math.isfinite(float(fs.sum()))


# ---- vector-Jacobian products (reverse mode) ---------------------------------

def test_vjp_handworked(oracle_mod):
    """gy = J^T v with the hand-derived J of every golden case; for a single
    reaction d(v.f)/d ln k = v.f (f is proportional to k)."""
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    for case in gold["cases"]:
        m = _mech_from_case(case)
        o = oracle_mod.Oracle(m)
        N = m.n_species
        y = np.array(case["y"], dtype=np.float64)[:, None]
        k = np.array([r["k"] for r in case["reactions"]], dtype=np.float64)[:, None]
        v = (1.0 + np.arange(N, dtype=np.float64))[:, None] * np.array([1.0, -0.5, 0.25] * N)[:N, None]
        gy, gk = o.vjp(k, y, v)
        J = np.array(case["J"], dtype=np.float64)
        np.testing.assert_allclose(gy[:, 0], J.T @ v[:, 0], rtol=1e-14, atol=1e-14)
        if len(case["reactions"]) == 1:
            f = np.array(case["f"], dtype=np.float64)
            assert gk[0, 0] == pytest.approx(float(v[:, 0] @ f), rel=1e-14)


@pytest.mark.parametrize("mech_fn", [synth.mech_small, synth.mech_medium])
def test_vjp_rate_constants_linear_and_euler(oracle_mod, mech_fn):
    """f is linear in each k_j: d(v.f)/d ln k_j = v.(f(k + k_j e_j) - f(k));
    and sum_j d(v.f)/d ln k_j = v.f (f is homogeneous of degree 1 in k)."""
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = synth.make_cells(m, 2, seed=77)
    k = o.rate_constants(c.T, c.jscale)
    rng = np.random.default_rng(3)
    v = rng.normal(size=c.y0.shape)
    gy, gk = o.vjp(k, c.y0, v)
    f0, fs = o.deriv(k, c.y0)
    vf = np.sum(v * f0, axis=0)
    scale = np.sum(np.abs(v) * fs, axis=0)
    assert np.all(np.abs(gk.sum(axis=0) - vf) <= 1e-12 * scale)
    for j in rng.choice(m.n_reactions, 12, replace=False):
        k2 = k.copy()
        k2[j] *= 2.0
        f2, _ = o.deriv(k2, c.y0)
        ref = np.sum(v * (f2 - f0), axis=0)
        assert np.all(np.abs(gk[j] - ref) <= 1e-12 * scale)


@pytest.mark.parametrize("mech_fn", [synth.mech_small, synth.mech_medium])
def test_vjp_state_central_differences(oracle_mod, mech_fn):
    """v.(f(y + e u) - f(y - e u)) / 2e = gy.u up to the cubic term of f."""
    m = mech_fn()
    o = oracle_mod.Oracle(m)
    c = synth.make_cells(m, 2, seed=78)
    k = o.rate_constants(c.T, c.jscale)
    rng = np.random.default_rng(4)
    v = rng.normal(size=c.y0.shape)
    gy, _ = o.vjp(k, c.y0, v)
    for _ in range(4):
        u = rng.normal(size=c.y0.shape) * c.y0
        e = 1e-4
        fp, _ = o.deriv(k, c.y0 + e * u)
        fm, fs = o.deriv(k, c.y0 - e * u)
        fd = np.sum(v * (fp - fm), axis=0) / (2 * e)
        an = np.sum(gy * u, axis=0)
        scale = np.sum(np.abs(v) * fs, axis=0)
        assert np.all(np.abs(fd - an) <= 1e-6 * scale), (fd, an, scale)
