"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bars
- rate constants: |dk| <= 8 eps |k| (exp differs by at most a few ulp);
- f and J: |d| <= 1e-12 * S, S = sum of absolute contributions (oracle scale);
- one outer step: |dy| <= 1e-6 |y_oracle| + 1e2 atol (rtol 1e-8, atol 1).
The oracle and the library share no code; the seeded generator feeds both.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2501_00011_amd import mcchem, synth  # noqa: E402

import tape_format  # noqa: E402

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _padded(a, ld, fill=np.nan):
    out = np.full((a.shape[0], ld), fill)
    out[:, :a.shape[1]] = a
    return out


class Batch:
    """One mechanism + cells on the GPU and the oracle beside it."""

    def __init__(self, dev, mech, cells, ld=None, oracle_mod=None, dense_tail=-1):
        self.m, self.c = mech, cells
        self.C = cells.n_cells
        self.ld = ld or self.C
        self.dev = dev
        self.h = mcchem.Mechanism(mech, dense_tail=dense_tail)
        self.cells = mcchem.Cells(self.h, self.C, self.ld)
        self.T = _t(cells.T, dev)
        self.P = _t(cells.P, dev)
        self.s = _t(cells.jscale, dev)
        self.cells.bind(self.T, self.P, self.s)
        self.o = oracle_mod.Oracle(mech) if oracle_mod else None

    def k_gpu(self):
        torch.cuda.synchronize()
        return self.cells.rate_constants().cpu().numpy()[:, :self.C]

    def y_dev(self, y=None):
        y = self.c.y0 if y is None else y
        return _t(_padded(y, self.ld), self.dev)


@pytest.mark.parametrize("name,n", [("small10", 10), ("medium10k", 777)])
def test_rate_constants(dev, oracle_mod, name, n):
    m, c, _ = synth.workload(name, n)
    b = Batch(dev, m, c, ld=n + 3, oracle_mod=oracle_mod)
    k_ref = b.o.rate_constants(c.T, c.jscale)
    k = b.k_gpu()
    assert np.all(np.abs(k - k_ref) <= 8 * EPS * np.abs(k_ref))


def _check_fj(b, f, J, y):
    k_ref = b.o.rate_constants(b.c.T, b.c.jscale)
    f_ref, fs = b.o.deriv(k_ref, y)
    J_ref, Js = b.o.jac(k_ref, y)
    assert np.all(np.abs(f - f_ref) <= 1e-12 * fs), np.max(np.abs(f - f_ref) / np.maximum(fs, 1e-300))
    rp, ci = b.h.jac_pattern()
    rows = np.repeat(np.arange(b.m.n_species), np.diff(rp))
    Jr = J_ref[:, rows, ci].T   # [nnz][C]
    Jsr = Js[:, rows, ci].T
    assert np.all(np.abs(J - Jr) <= 1e-12 * Jsr), np.max(np.abs(J - Jr) / np.maximum(Jsr, 1e-300))
    # the oracle's J has no entries outside the compiled pattern
    mask = np.ones((b.m.n_species, b.m.n_species), dtype=bool)
    mask[rows, ci] = False
    assert np.all(J_ref[:, mask] == 0.0)


KINDS = [mcchem.Mechanism.FJ_GENERATED, mcchem.Mechanism.FJ_TABLES]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("name,n,ld", [("small10", 10, 10), ("small10", 10, 67),
                                       ("medium10k", 777, 800), ("medium10k", 1, 1)])
def test_deriv_and_jac_parity(dev, oracle_mod, name, n, ld, kind):
    m, c, _ = synth.workload(name, n)
    b = Batch(dev, m, c, ld=ld, oracle_mod=oracle_mod)
    b.h.set_fj_kernel(kind)
    y = b.y_dev()
    f = torch.full((m.n_species, ld), 7.0, dtype=torch.float64, device=dev)
    J = torch.full((b.h.nnz, ld), 7.0, dtype=torch.float64, device=dev)
    b.cells.deriv(y, f)
    b.cells.jac(y, J)
    f2, J2 = b.cells.deriv_jac(y)
    torch.cuda.synchronize()
    fn, Jn = f.cpu().numpy(), J.cpu().numpy()
    # padding columns are never written
    assert np.all(fn[:, n:] == 7.0) and np.all(Jn[:, n:] == 7.0)
    _check_fj(b, fn[:, :n], Jn[:, :n], c.y0)
    # the fused call computes the same values bit for bit
    np.testing.assert_array_equal(f2.cpu().numpy()[:, :n], fn[:, :n])
    np.testing.assert_array_equal(J2.cpu().numpy()[:, :n], Jn[:, :n])


@pytest.mark.parametrize("kind", KINDS)
def test_large_mechanism_fj_parity(dev, oracle_mod, kind):
    m = synth.mech_large()
    c = synth.make_cells(m, 300, seed=4242)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    b.h.set_fj_kernel(kind)
    f, J = b.cells.deriv_jac(b.y_dev())
    torch.cuda.synchronize()
    _check_fj(b, f.cpu().numpy(), J.cpu().numpy(), c.y0)


@pytest.mark.parametrize("kind", KINDS)
def test_full_size_fj_sampled_and_homogeneity(dev, oracle_mod, kind):
    """10,000 cells in the benchmark's launch: sampled cells against the
    oracle, every cell against Euler's identity sum_s J_is y_s = sum_j ord_j nu_ij r_j."""
    m, c, _ = synth.workload("medium10k")
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    b.h.set_fj_kernel(kind)
    f, J = b.cells.deriv_jac(b.y_dev())
    torch.cuda.synchronize()
    fn, Jn = f.cpu().numpy(), J.cpu().numpy()
    rng = np.random.default_rng(99)
    sel = np.sort(rng.choice(c.n_cells, 48, replace=False))
    sub = synth.Cells(T=c.T[sel], P=c.P[sel], jscale=c.jscale[sel], y0=c.y0[:, sel])
    bs = Batch.__new__(Batch)
    bs.m, bs.c, bs.h, bs.o = m, sub, b.h, b.o
    _check_fj(bs, fn[:, sel], Jn[:, sel], sub.y0)
    # identity at every cell, with the orders taken from the mechanism
    rp, ci = b.h.jac_pattern()
    rows = np.repeat(np.arange(m.n_species), np.diff(rp))
    Jy = np.zeros_like(fn)
    np.add.at(Jy, rows, Jn * c.y0[ci])
    k = b.k_gpu()
    rhs = np.zeros_like(fn)
    bound = np.zeros_like(fn)
    for j in range(m.n_reactions):
        reac = m.reac_idx[m.reac_ptr[j]:m.reac_ptr[j + 1]]
        r = k[j] * np.prod(c.y0[reac], axis=0)
        order = len(reac)
        for s in reac:
            rhs[s] -= order * r
            bound[s] += order * abs(r)
        for s, yl in zip(m.prod_idx[m.prod_ptr[j]:m.prod_ptr[j + 1]], m.prod_yield[m.prod_ptr[j]:m.prod_ptr[j + 1]]):
            rhs[s] += order * yl * r
            bound[s] += order * abs(yl * r)
    assert np.all(np.abs(Jy - rhs) <= 1e-12 * bound)


@pytest.mark.parametrize("ld_pad", [0, 1])
def test_streaming_fj_and_vjp_at_200k_cells(dev, oracle_mod, ld_pad):
    """200,000 cells, where the inputs exceed the memory-side cache and the
    f/J launch runs each work item over 128 consecutive tiles at once: every
    output written (prefilled with NaN), Euler's identity at every cell,
    sampled cells (first and last tiles among them) against the oracle for
    f/J and for the VJP.  ld_pad 1: odd leading dimension, the one-cell
    kernel everywhere."""
    m, c, _ = synth.workload("medium200k")
    ld = c.n_cells + ld_pad
    b = Batch(dev, m, c, ld=ld, oracle_mod=oracle_mod)
    y = b.y_dev()
    f = torch.full((m.n_species, ld), float("nan"), dtype=torch.float64, device=dev)
    J = torch.full((b.h.nnz, ld), float("nan"), dtype=torch.float64, device=dev)
    b.cells.deriv_jac(y, f, J)
    rng = np.random.default_rng(2024)
    v = rng.normal(size=c.y0.shape)
    gy = torch.full_like(f, float("nan"))
    gk = torch.full((m.n_reactions, ld), float("nan"), dtype=torch.float64, device=dev)
    b.cells.vjp(y, _t(_padded(v, ld), dev), gy, gk)
    torch.cuda.synchronize()
    C = c.n_cells
    fn = f.cpu().numpy()[:, :C]
    gyn, gkn = gy.cpu().numpy()[:, :C], gk.cpu().numpy()[:, :C]
    assert np.isfinite(fn).all() and np.isfinite(gyn).all() and np.isfinite(gkn).all()
    sel = np.unique(np.concatenate([np.arange(130), np.arange(C - 130, C), rng.choice(C, 60, replace=False)]))
    Jn_sel = J[:, torch.from_numpy(sel).to(dev)].cpu().numpy()
    sub = synth.Cells(T=c.T[sel], P=c.P[sel], jscale=c.jscale[sel], y0=c.y0[:, sel])
    bs = Batch.__new__(Batch)
    bs.m, bs.c, bs.h, bs.o = m, sub, b.h, b.o
    _check_fj(bs, fn[:, sel], Jn_sel, sub.y0)
    k = b.o.rate_constants(sub.T, sub.jscale)
    gy_ref, gk_ref = b.o.vjp(k, sub.y0, v[:, sel])
    _, Js = b.o.jac(k, sub.y0)
    by, bk = _vjp_bounds(m, k, sub.y0, v[:, sel], Js)
    assert np.all(np.abs(gyn[:, sel] - gy_ref) <= 1e-12 * by)
    assert np.all(np.abs(gkn[:, sel] - gk_ref) <= 1e-12 * bk)
    # Euler's identity at every cell, J copied over in blocks of cells
    rp, ci = b.h.jac_pattern()
    rows = np.repeat(np.arange(m.n_species), np.diff(rp))
    kg = b.k_gpu()
    for c0 in range(0, C, 50000):
        c1 = min(C, c0 + 50000)
        Jn = J[:, c0:c1].cpu().numpy()
        assert np.isfinite(Jn).all()
        y0 = c.y0[:, c0:c1]
        Jy = np.zeros((m.n_species, c1 - c0))
        np.add.at(Jy, rows, Jn * y0[ci])
        rhs = np.zeros_like(Jy)
        bound = np.zeros_like(Jy)
        for j in range(m.n_reactions):
            reac = m.reac_idx[m.reac_ptr[j]:m.reac_ptr[j + 1]]
            r = kg[j, c0:c1] * np.prod(y0[reac], axis=0)
            order = len(reac)
            for s in reac:
                rhs[s] -= order * r
                bound[s] += order * abs(r)
            for s, yl in zip(m.prod_idx[m.prod_ptr[j]:m.prod_ptr[j + 1]],
                             m.prod_yield[m.prod_ptr[j]:m.prod_ptr[j + 1]]):
                rhs[s] += order * yl * r
                bound[s] += order * abs(yl * r)
        assert np.all(np.abs(Jy - rhs) <= 1e-12 * bound)


def _solve_parity(b, dt, opts_kw=None, y0=None):
    opts_kw = opts_kw or {}
    y0 = b.c.y0 if y0 is None else y0
    y = b.y_dev(y0)
    st, stats = b.cells.step(y, dt, mcchem.default_opts(**opts_kw))
    torch.cuda.synchronize()
    yg = y.cpu().numpy()[:, :b.C]
    sg = st.cpu().numpy()
    statg = mcchem.stats_numpy(stats)
    k_ref = b.o.rate_constants(b.c.T, b.c.jscale)
    import oracle as orc
    yo, so, stato = b.o.solve(k_ref, y0, dt, orc.default_opts(**opts_kw))
    return yg, sg, statg, yo, so, stato


def _within(yg, yo, atol):
    err = np.abs(yg - yo)
    tol = 1e-6 * np.abs(yo) + 1e2 * atol
    return float(np.max(err / tol))


# every dense-tail size the solver is built with for the 72-species mechanism
# (the benchmark times the size the autotuner picks, usually 32)
@pytest.mark.parametrize("name,n,tail", [("small10", 10, -1), ("medium10k", 96, 0), ("medium10k", 96, 32),
                                         ("medium10k", 96, 48), ("medium10k", 96, 64)])
def test_solve_step_parity(dev, oracle_mod, name, n, tail):
    m, c, dt = synth.workload(name, n)
    b = Batch(dev, m, c, ld=n + 5, oracle_mod=oracle_mod, dense_tail=tail)
    yg, sg, statg, yo, so, stato = _solve_parity(b, dt)
    assert np.all(so == 0) and np.all(sg == 0), (so, sg)
    worst = _within(yg, yo, 1.0)
    same = np.mean((statg["steps"] == stato["steps"]) & (statg["rejects"] == stato["rejects"]))
    print(f"{name}: worst {worst:.3g} of the bar, identical step sequences in {same:.0%} of cells")
    assert worst <= 1.0
    assert np.all(statg["lu_count"] == statg["jac_evals"])
    assert np.all(np.abs(statg["steps"] - stato["steps"]) <= 0.1 * stato["steps"] + 5)


@pytest.mark.parametrize("tail", [32, 48])
def test_solve_full_size_sampled(dev, oracle_mod, tail):
    """All 10,000 cells in one launch as the benchmark times it: the
    dense-tail size fixed, the cells scheduled longest first by a first
    step's counters; 32 sampled cells of the second step against the oracle
    (a cell's result does not depend on the batch or the schedule)."""
    m, c, dt = synth.workload("medium10k")
    b = Batch(dev, m, c, oracle_mod=oracle_mod, dense_tail=tail)
    assert b.h.schedule_info()["dense_tail"] == tail
    y = b.y_dev()
    _, stats0 = b.cells.step(y, dt)
    order = b.cells.balance(stats0)
    assert not np.array_equal(order, np.arange(c.n_cells))
    y = b.y_dev()
    st, stats = b.cells.step(y, dt)
    torch.cuda.synchronize()
    sg = st.cpu().numpy()
    assert np.all(sg == 0), np.bincount(sg)
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(c.n_cells, 32, replace=False))
    k_ref = b.o.rate_constants(c.T[sel], c.jscale[sel])
    yo, so, _ = b.o.solve(k_ref, c.y0[:, sel], dt)
    assert np.all(so == 0)
    assert _within(y.cpu().numpy()[:, sel], yo, 1.0) <= 1.0
    # atom conservation at every cell
    a = m.composition.astype(np.float64)
    before, after = a.T @ c.y0, a.T @ y.cpu().numpy()
    assert np.all(np.abs(after - before) <= 1e-10 * before)
    b.cells.set_schedule(None)


def test_paper_test_mechanism_on_gpu(dev, oracle_mod):
    """Section 4's mechanism (A gives B and C by two Arrhenius reactions, A = 1,
    B = C = 0 plus 0.1 per flattened concentration index) against its closed form."""
    m = synth.mechanism_from_lists(3, [([0], [(1, 1.0)], 0.05, 0.0, 0), ([0], [(2, 1.0)], 0.02, 0.0, 0)])
    n = 100
    y0 = (np.array([1.0, 0.0, 0.0])[None, :] + 0.1 * (np.arange(3 * n).reshape(n, 3) + 1)).T.copy()
    cells = synth.Cells(T=np.full(n, 298.0), P=np.full(n, 1013.25), jscale=np.ones(n), y0=y0)
    b = Batch(dev, m, cells, oracle_mod=oracle_mod)
    y = b.y_dev()
    st, _ = b.cells.step(y, 60.0, mcchem.default_opts(atol=1e-14))
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    A = y0[0] * math.exp(-0.07 * 60.0)
    exact = np.stack([A, y0[1] + 0.05 / 0.07 * (y0[0] - A), y0[2] + 0.02 / 0.07 * (y0[0] - A)])
    assert _within(y.cpu().numpy(), exact, 1e-14) <= 1.0


def test_large_mechanism_solve_parity(dev, oracle_mod):
    m = synth.mech_large()
    c = synth.make_cells(m, 6, seed=515)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    yg, sg, _, yo, so, _ = _solve_parity(b, 60.0)
    assert np.all(so == 0) and np.all(sg == 0)
    assert _within(yg, yo, 1.0) <= 1.0


def test_status_codes_match_oracle(dev, oracle_mod):
    m, c, dt = synth.workload("small10")
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    _, sg, statg, _, so, stato = _solve_parity(b, dt, {"max_steps": 1})
    assert np.all(sg == 1) and np.all(so == 1)
    _, sg, statg, _, so, stato = _solve_parity(b, dt, {"max_newton": 1, "h_min_rel": 1e-12})
    assert np.all(sg == 2) and np.all(so == 2)
    np.testing.assert_array_equal(statg["newton_fails"], stato["newton_fails"])
    y0 = c.y0.copy()
    y0[4, 3] = np.nan
    yg, sg, _, _, so, _ = _solve_parity(b, dt, None, y0)
    assert sg[3] == 4 and so[3] == 4
    assert np.all(np.delete(sg, 3) == 0)


def test_empty_batch_and_determinism(dev, oracle_mod):
    m, c, dt = synth.workload("small10")
    h = mcchem.Mechanism(m)
    empty = mcchem.Cells(h, 0, 0)
    T0 = torch.empty(0, dtype=torch.float64, device=dev)
    empty.bind(T0)
    y0 = torch.empty((m.n_species, 0), dtype=torch.float64, device=dev)
    empty.deriv(y0)
    empty.step(y0, dt)
    empty.sync()
    # same inputs twice -> identical bits; permuted cells -> permuted results
    b = Batch(dev, m, c)
    y1, y2 = b.y_dev(), b.y_dev()
    b.cells.step(y1, dt)
    b.cells.step(y2, dt)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    perm = np.array([9, 3, 0, 5])
    sub = synth.Cells(T=c.T[perm], P=c.P[perm], jscale=c.jscale[perm], y0=c.y0[:, perm])
    bp = Batch(dev, m, sub)
    yp = bp.y_dev()
    bp.cells.step(yp, dt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(yp.cpu().numpy(), y1.cpu().numpy()[:, perm])


def test_errors_before_bind_and_bad_args(dev):
    m, c, dt = synth.workload("small10")
    h = mcchem.Mechanism(m)
    cells = mcchem.Cells(h, c.n_cells)
    y = torch.from_numpy(c.y0).to(dev)
    with pytest.raises(mcchem.MccError, match="status 5"):
        cells.deriv(y)
    cells.bind(torch.from_numpy(c.T).to(dev))
    with pytest.raises(mcchem.MccError, match="status 1"):
        cells.step(y, -1.0)
    with pytest.raises(mcchem.MccError, match="status 1"):
        cells.step(y, dt, mcchem.default_opts(max_order=6))
    with pytest.raises(mcchem.MccError, match="status 1"):
        cells.step(y, dt, mcchem.default_opts(steps_per_launch=-1))
    with pytest.raises(mcchem.MccError, match="status 5"):
        h.close()  # a batch is still alive
    cells.close()
    h.close()


def test_fj_split_unit_accumulates(dev, oracle_mod):
    """One species changed by 59 reactions: its f row and J rows span two
    chunks of the f/J kernel, the second adding to what the first wrote."""
    n = 60
    rx = [([i], [(0, 1.0)], 1e-3 * (i + 1), 0.0, 0) for i in range(1, n)]
    rx.append(([0, 1], [(2, 0.5), (3, 0.5)], 1e-2, 0.0, 0))
    m = synth.mechanism_from_lists(n, rx)
    cells = synth.Cells(T=np.full(130, 280.0), P=np.full(130, 1000.0), jscale=np.ones(130),
                        y0=np.random.default_rng(3).uniform(0.5, 2.0, size=(n, 130)))
    b = Batch(dev, m, cells, oracle_mod=oracle_mod)
    f, J = b.cells.deriv_jac(b.y_dev())
    torch.cuda.synchronize()
    _check_fj(b, f.cpu().numpy(), J.cpu().numpy(), cells.y0)


@pytest.mark.parametrize("kind", [mcchem.Mechanism.FJ_GENERATED, mcchem.Mechanism.FJ_TABLES])
def test_fj_wide_species(dev, oracle_mod, kind):
    """A species formed by 130 bimolecular reactions: its f row spans many
    chunks of one work item, the later ones adding to what the first wrote."""
    n = 140
    rx = [([i, i + 1], [(0, 1.0)], 1e-12 * (1 + i % 7), 0.0, 0) for i in range(1, 131)]
    rx.append(([0], [(139, 1.0)], 1e-3, 0.0, 0))
    m = synth.mechanism_from_lists(n, rx)
    C = 100
    rng = np.random.default_rng(8)
    cells = synth.Cells(T=np.full(C, 280.0), P=np.full(C, 1000.0), jscale=np.ones(C),
                        y0=rng.uniform(1e8, 1e9, size=(n, C)))
    b = Batch(dev, m, cells, ld=C + 28, oracle_mod=oracle_mod)
    b.h.set_fj_kernel(kind)
    f, J = b.cells.deriv_jac(b.y_dev())
    torch.cuda.synchronize()
    _check_fj(b, f.cpu().numpy()[:, :C], J.cpu().numpy()[:, :C], cells.y0)


def _step_all(b, dt, **kw):
    y = b.y_dev()
    st, stats = b.cells.step(y, dt, mcchem.default_opts(**kw))
    torch.cuda.synchronize()
    return y.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("K", [1, 7])
def test_per_launch_form_is_bit_identical(dev, K):
    """The per-launch form (state in HBM between launches, at most K accepted
    steps per launch) computes exactly what the one-launch form computes."""
    m, c, dt = synth.workload("medium10k", 200)
    b = Batch(dev, m, c, ld=203)
    y0, s0, t0 = _step_all(b, dt)
    y1, s1, t1 = _step_all(b, dt, steps_per_launch=K)
    assert np.all(s0 == 0)
    np.testing.assert_array_equal(s1, s0)
    np.testing.assert_array_equal(y1, y0)
    np.testing.assert_array_equal(t1, t0)
    # a second outer step on the same handle starts every cell afresh
    y2, s2, t2 = _step_all(b, dt, steps_per_launch=K)
    np.testing.assert_array_equal(y2, y0)
    np.testing.assert_array_equal(t2, t0)


def test_per_launch_form_status_codes(dev):
    m, c, dt = synth.workload("small10")
    b = Batch(dev, m, c)
    for kw in ({"max_steps": 1}, {"max_steps": 40}, {"max_newton": 1, "h_min_rel": 1e-12}):
        y0, s0, t0 = _step_all(b, dt, **kw)
        y1, s1, t1 = _step_all(b, dt, steps_per_launch=3, **kw)
        np.testing.assert_array_equal(s1, s0)
        np.testing.assert_array_equal(y1, y0)
        np.testing.assert_array_equal(t1, t0)


def test_mixed_mechanisms_graph_replay(dev, oracle_mod):
    """Three mechanisms (20, 72, 150 species), each batch on its own stream,
    one outer step of all of them captured into one graph and replayed:
    every replay equals the eager steps bit for bit, with eager work and
    synchronisations between replays; sampled cells match the oracle."""
    groups, owner, dt = synth.mixed_workload(900)
    streams = [torch.cuda.Stream(device=dev) for _ in groups]
    batches, ys, yeager, st = [], [], [], []
    for (m, c), s in zip(groups, streams):
        b = Batch(dev, m, c, oracle_mod=oracle_mod)
        batches.append(b)
        ys.append(b.y_dev())
        yeager.append(b.y_dev())
        st.append(torch.empty(c.n_cells, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    # eager reference: three consecutive outer steps
    ref = []
    for _ in range(3):
        for b, y, s_ in zip(batches, yeager, st):
            b.cells.step(y, dt, status=s_, want_stats=False)
        torch.cuda.synchronize()
        ref.append([y.clone() for y in yeager])
    # capture one outer step of every batch, each on its own stream
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cap):
        for b, y, s_, side in zip(batches, ys, st, streams):
            side.wait_stream(cap)
            b.cells.step(y, dt, status=s_, want_stats=False, stream=side)
            cap.wait_stream(side)
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=dev).sum().item()  # unrelated eager work between replays
        for y, yr in zip(ys, ref[r]):
            assert torch.equal(y, yr), f"replay {r}"
    # the first eager step against the oracle on a few cells of every mechanism
    import oracle as orc
    for b, yr in zip(batches, ref[0]):
        sel = np.arange(0, b.C, max(1, b.C // 6))
        k = b.o.rate_constants(b.c.T[sel], b.c.jscale[sel])
        yo, so, _ = b.o.solve(k, b.c.y0[:, sel], dt, orc.default_opts())
        assert np.all(so == 0)
        assert _within(yr.cpu().numpy()[:, sel], yo, 1.0) <= 1.0


def _vjp_bounds(m, k, y, v, Js):
    """Scales of the two products: sum_i |v_i| |J|_is and r_j sum_i |nu_ij v_i|."""
    by = np.einsum("ic,cis->sc", np.abs(v), Js)
    bk = np.zeros((m.n_reactions, y.shape[1]))
    for j in range(m.n_reactions):
        reac = m.reac_idx[m.reac_ptr[j]:m.reac_ptr[j + 1]]
        r = k[j] * np.prod(y[reac], axis=0)
        w = np.zeros(y.shape[1])
        for s in reac:
            w += np.abs(v[s])
        for s, yl in zip(m.prod_idx[m.prod_ptr[j]:m.prod_ptr[j + 1]], m.prod_yield[m.prod_ptr[j]:m.prod_ptr[j + 1]]):
            w += np.abs(yl * v[s])
        bk[j] = np.abs(r) * w
    return by, bk


@pytest.mark.parametrize("name,n,ld", [("small10", 10, 13), ("medium10k", 333, 333)])
def test_vjp_parity(dev, oracle_mod, name, n, ld):
    m, c, _ = synth.workload(name, n)
    b = Batch(dev, m, c, ld=ld, oracle_mod=oracle_mod)
    rng = np.random.default_rng(12)
    v = rng.normal(size=c.y0.shape)
    gy, gk = b.cells.vjp(b.y_dev(), _t(_padded(v, ld), dev))
    gy_only, _ = b.cells.vjp(b.y_dev(), _t(_padded(v, ld), dev), want_glnk=False)
    torch.cuda.synchronize()
    gy, gk = gy.cpu().numpy()[:, :n], gk.cpu().numpy()[:, :n]
    k = b.o.rate_constants(c.T, c.jscale)
    gy_ref, gk_ref = b.o.vjp(k, c.y0, v)
    _, Js = b.o.jac(k, c.y0)
    by, bk = _vjp_bounds(m, k, c.y0, v, Js)
    assert np.all(np.abs(gy - gy_ref) <= 1e-12 * by)
    assert np.all(np.abs(gk - gk_ref) <= 1e-12 * bk)
    np.testing.assert_array_equal(gy_only.cpu().numpy()[:, :n], gy)


def test_vjp_large_mechanism(dev, oracle_mod):
    m = synth.mech_large()
    c = synth.make_cells(m, 130, seed=4243)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    v = np.random.default_rng(13).normal(size=c.y0.shape)
    gy, gk = b.cells.vjp(b.y_dev(), _t(v, dev))
    torch.cuda.synchronize()
    k = b.o.rate_constants(c.T, c.jscale)
    gy_ref, gk_ref = b.o.vjp(k, c.y0, v)
    _, Js = b.o.jac(k, c.y0)
    by, bk = _vjp_bounds(m, k, c.y0, v, Js)
    assert np.all(np.abs(gy.cpu().numpy() - gy_ref) <= 1e-12 * by)
    assert np.all(np.abs(gk.cpu().numpy() - gk_ref) <= 1e-12 * bk)


def test_autograd_deriv(dev, oracle_mod):
    """torch autograd through f(y, ln k): gradients of sum(w * f) equal the
    oracle's vector-Jacobian products."""
    from paper_2501_00011_amd import autograd as mag
    m, c, _ = synth.workload("medium10k", 200)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    k = b.o.rate_constants(c.T, c.jscale)
    y = _t(c.y0, dev).requires_grad_(True)
    lnk = _t(np.log(k), dev).requires_grad_(True)
    w = np.random.default_rng(14).normal(size=c.y0.shape)
    f = mag.deriv(b.cells, y, lnk)
    (f * _t(w, dev)).sum().backward()
    f_ref, fs = b.o.deriv(k, c.y0)
    gy_ref, gk_ref = b.o.vjp(k, c.y0, w)
    _, Js = b.o.jac(k, c.y0)
    by, bk = _vjp_bounds(m, k, c.y0, w, Js)
    # k = exp(ln k) in torch: one rounding of exp on each side
    assert np.all(np.abs(f.detach().cpu().numpy() - f_ref) <= 1e-11 * fs)
    assert np.all(np.abs(y.grad.cpu().numpy() - gy_ref) <= 1e-11 * by)
    assert np.all(np.abs(lnk.grad.cpu().numpy() - gk_ref) <= 1e-11 * bk)


# ---- the paper's Multi-cells mode -------------------------------------------

def _multicell(b, dt, opts_kw=None, atol=None):
    import oracle as orc
    kw = dict(opts_kw or {})
    if atol is not None:
        kw["atol"] = atol
    y = b.y_dev()
    st, stats = b.cells.step_multicell(y, dt, mcchem.default_opts(**kw))
    torch.cuda.synchronize()
    k = b.o.rate_constants(b.c.T, b.c.jscale)
    yo, so, sto = b.o.solve_multicell(k, b.c.y0, dt, orc.default_opts(**kw))
    return y.cpu().numpy()[:, :b.C], st.cpu().numpy(), mcchem.stats_numpy(stats), yo, so, sto


@pytest.mark.parametrize("C", [1, 37, 1000])
def test_multicell_paper_mechanism(dev, oracle_mod, C):
    m, c, dt = synth.workload("paper_test", C)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    yg, sg, stg, yo, so, sto = _multicell(b, dt, atol=1e-14)
    assert so == 0 and np.all(sg == 0)
    assert _within(yg, yo, 1e-14) <= 1.0
    # one shared step sequence: every cell reports the system's counters
    assert np.all(stg["steps"] == stg["steps"][0]) and abs(int(stg["steps"][0]) - int(sto["steps"])) <= 2
    ks = 0.07
    A = c.y0[0] * math.exp(-ks * dt)
    exact = np.stack([A, c.y0[1] + 0.05 / ks * (c.y0[0] - A), c.y0[2] + 0.02 / ks * (c.y0[0] - A)])
    assert _within(yg, exact, 1e-14) <= 1.0


@pytest.mark.parametrize("name,n", [("small10", 10), ("medium10k", 64)])
def test_multicell_parity(dev, oracle_mod, name, n):
    m, c, dt = synth.workload(name, n)
    b = Batch(dev, m, c, ld=n + 3, oracle_mod=oracle_mod)
    yg, sg, stg, yo, so, sto = _multicell(b, dt)
    assert so == 0 and np.all(sg == 0)
    assert _within(yg, yo, 1.0) <= 1.0
    assert abs(int(stg["steps"][0]) - int(sto["steps"])) <= 0.05 * int(sto["steps"]) + 2


def test_multicell_one_cell_is_per_cell_and_deterministic(dev):
    m, c, dt = synth.workload("medium10k", 1)
    b = Batch(dev, m, c)
    y1, y2, y3 = b.y_dev(), b.y_dev(), b.y_dev()
    b.cells.step(y1, dt)
    b.cells.step_multicell(y2, dt)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    m, c, dt = synth.workload("small10")
    b = Batch(dev, m, c)
    y1, y2 = b.y_dev(), b.y_dev()
    b.cells.step_multicell(y1, dt)
    b.cells.step_multicell(y2, dt)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_multicell_limits(dev):
    m, c, dt = synth.workload("paper_test", 1)
    h = mcchem.Mechanism(m)
    big = mcchem.Cells(h, 300000)
    big.bind(torch.full((300000,), 298.0, dtype=torch.float64, device=dev))
    y = torch.ones((3, 300000), dtype=torch.float64, device=dev)
    with pytest.raises(mcchem.MccError, match="at most"):
        big.step_multicell(y, dt)
    with pytest.raises(mcchem.MccError, match="steps_per_launch"):
        big.step_multicell(y, dt, mcchem.default_opts(steps_per_launch=2))


# ---- ablation: the paper's Derivative kernel -------------------------------

@pytest.mark.parametrize("inverted", [False, True])
def test_paper_deriv_kernel(dev, oracle_mod, inverted):
    """The paper's one-thread-per-reaction kernel with atomic adds, on its
    concatenated cell-major layout, computes f (to rounding: the atomic adds
    sum in any order)."""
    m, c, _ = synth.workload("medium10k", 500)
    o = oracle_mod.Oracle(m)
    k = o.rate_constants(c.T, c.jscale)
    h = mcchem.Mechanism(m)
    f = h.paper_deriv(_t(c.y0.T, dev), _t(k.T, dev), inverted=inverted)
    torch.cuda.synchronize()
    f_ref, fs = o.deriv(k, c.y0)
    assert np.all(np.abs(f.cpu().numpy().T - f_ref) <= 1e-12 * fs)


def test_autotune_solver(dev, oracle_mod):
    """The autotuner times every admissible dense-tail size, register budget
    and cell schedule and returns the fastest; the tuned mechanism meets the
    solver's parity bar."""
    m, c, dt = synth.workload("medium10k", 600)
    h, times, choice = mcchem.autotune_solver(m, c, dt, reps=1)
    tails = {int(k.split("/")[0]) for k in times}
    waves = {int(k.split("/")[1]) for k in times}
    scheds = {k.split("/")[2] for k in times}
    assert tails == {0, 32, 48, 64} and waves == {1, 2} and scheds == {"identity", "longest", "zigzag"}
    assert all(t > 0 for t in times.values())
    best = min(times, key=times.get)
    assert f"{choice[0]}/{choice[1]}/{choice[2]}" == best
    info = h.schedule_info()
    assert (info["dense_tail"], info["waves_per_simd"]) == (choice[0], choice[1])
    sub = synth.Cells(T=c.T[:40], P=c.P[:40], jscale=c.jscale[:40], y0=c.y0[:, :40])
    b = Batch.__new__(Batch)
    b.m, b.c, b.C, b.ld, b.dev, b.h = m, sub, 40, 40, dev, h
    b.cells = mcchem.Cells(h, 40)
    b.T, b.P, b.s = _t(sub.T, dev), _t(sub.P, dev), _t(sub.jscale, dev)
    b.cells.bind(b.T, b.P, b.s)
    b.o = oracle_mod.Oracle(m)
    yg, sg, _, yo, so, _ = _solve_parity(b, dt)
    assert np.all(sg == 0) and np.all(so == 0)
    assert _within(yg, yo, 1.0) <= 1.0


@pytest.mark.parametrize("n,ld", [(333, 334), (334, 334), (1, 2)])
def test_vjp_pair_and_remainder(dev, oracle_mod, n, ld):
    """Even leading dimension: the two-cell kernel over whole pairs, the
    one-cell kernel for an odd last cell."""
    m, c, _ = synth.workload("medium10k", n)
    b = Batch(dev, m, c, ld=ld, oracle_mod=oracle_mod)
    v = np.random.default_rng(15).normal(size=c.y0.shape)
    gy, gk = b.cells.vjp(b.y_dev(), _t(_padded(v, ld), dev))
    f, J = b.cells.deriv_jac(b.y_dev())
    torch.cuda.synchronize()
    k = b.o.rate_constants(c.T, c.jscale)
    gy_ref, gk_ref = b.o.vjp(k, c.y0, v)
    _, Js = b.o.jac(k, c.y0)
    by, bk = _vjp_bounds(m, k, c.y0, v, Js)
    assert np.all(np.abs(gy.cpu().numpy()[:, :n] - gy_ref) <= 1e-12 * by)
    assert np.all(np.abs(gk.cpu().numpy()[:, :n] - gk_ref) <= 1e-12 * bk)
    _check_fj(b, f.cpu().numpy()[:, :n], J.cpu().numpy()[:, :n], c.y0)


def _elementwise(got, ref):
    """Worst element-wise ratio to the reverse-mode bar |d| <= 1e-8 |ref| +
    1e-13 max|ref| (the second term only matters for entries some thirteen
    orders below the cell's largest, where the discrete adjoint's
    cancellations leave no relative accuracy)."""
    bar = 1e-8 * np.abs(ref) + 1e-13 * np.abs(ref).max()
    return float(np.max(np.abs(got - ref) / bar))


@pytest.mark.parametrize("name,n,ld", [("small10", 10, 13), ("medium10k", 40, 41)])
def test_adjoint_step_parity(dev, oracle_mod, name, n, ld):
    """Reverse mode of one outer step against the oracle's discrete adjoint,
    both walking the same replayed (converged) step tapes."""
    m, c, dt = synth.workload(name, n)
    b = Batch(dev, m, c, ld=ld, oracle_mod=oracle_mod)
    N, R = m.n_species, m.n_reactions
    k = b.o.rate_constants(c.T, c.jscale)
    rng = np.random.default_rng(21)
    W = np.zeros((N, n))
    lam_ref, g_ref, tapes = np.zeros((N, n)), np.zeros((R, n)), []
    for i in range(n):
        y, s, _, tape = b.o.solve_taped(k[:, i], c.y0[:, i], dt)
        assert s == 0
        _, rt = b.o.replay(k[:, i], c.y0[:, i], tape)
        W[:, i] = rng.normal(size=N) / np.maximum(np.abs(y), 1.0)
        lam_ref[:, i], g_ref[:, i] = b.o.adjoint(k[:, i], c.y0[:, i], rt, W[:, i])
        tapes.append(tape_format.to_device(rt.values(), N))
    buf, lens = tape_format.pack(tapes)
    lam = _t(_padded(W, ld, 0.0), dev)
    glnk, st = b.cells.adjoint_step(b.y_dev(), _t(buf, dev), _t(lens, dev), lam)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == mcchem.CELL_OK)
    lam_g = lam.cpu().numpy()[:, :n]
    g_g = glnk.cpu().numpy()[:, :n]
    el = max(_elementwise(lam_g[:, i], lam_ref[:, i]) for i in range(n))
    eg = max(_elementwise(g_g[:, i], g_ref[:, i]) for i in range(n))
    print(f"{name}: worst element-wise ratio to the bar, dL/dy0 {el:.3g}, dL/dlnk {eg:.3g}")
    assert el <= 1.0 and eg <= 1.0


def test_adjoint_step_accumulate_and_bad_tapes(dev, oracle_mod):
    m, c, dt = synth.workload("small10", 4)
    b = Batch(dev, m, c, ld=4, oracle_mod=oracle_mod)
    N, R = m.n_species, m.n_reactions
    k = b.o.rate_constants(c.T, c.jscale)
    tapes = []
    for i in range(4):
        _, s, _, tape = b.o.solve_taped(k[:, i], c.y0[:, i], dt)
        _, rt = b.o.replay(k[:, i], c.y0[:, i], tape)
        tapes.append(tape_format.to_device(rt.values(), N))
    buf, lens = tape_format.pack(tapes)
    W = np.ones((N, 4))
    lam = _t(W, dev)
    g1, st = b.cells.adjoint_step(b.y_dev(), _t(buf, dev), _t(lens, dev), lam)
    lam1 = lam.clone()
    lam2 = _t(W, dev)
    g2 = torch.ones((R, 4), dtype=torch.float64, device=dev)
    b.cells.adjoint_step(b.y_dev(), _t(buf, dev), _t(lens, dev), lam2, glnk=g2, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(lam1, lam2) and torch.equal(g2, g1 + 1.0)
    # cell 0: empty tape (lam unchanged, no k sensitivity); cell 1: length
    # beyond the stride; cell 2: an entry of order 0; cell 3: no start
    bad = buf.copy()
    blen = lens.copy()
    blen[0] = 0
    blen[1] = buf.shape[1] + 1
    assert int(bad[2, lens[2] - 1]) in (1, 2)  # the last entry is a step or a re-sampling
    bad[2, lens[2] - 3] = 0.0  # ... of order 0
    S = tape_format.SCALARS
    bad[3, 0:lens[3] - S] = bad[3, S:lens[3]]  # drop the start entry
    blen[3] = lens[3] - S
    lam = _t(W, dev)
    g, st = b.cells.adjoint_step(b.y_dev(), _t(bad, dev), _t(blen, dev), lam)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert list(st) == [mcchem.CELL_OK, mcchem.CELL_BAD_TAPE, mcchem.CELL_BAD_TAPE, mcchem.CELL_BAD_TAPE]
    lam, g = lam.cpu().numpy(), g.cpu().numpy()
    assert np.all(lam[:, 0] == 1.0) and np.all(g[:, 0] == 0.0)
    assert np.all(np.isnan(lam[:, 1:])) and np.all(np.isnan(g[:, 1:]))


@pytest.mark.parametrize("name,n,K,tail", [("small10", 10, 0, -1), ("medium10k", 48, 0, 0), ("medium10k", 48, 0, 32),
                                           ("medium10k", 48, 0, 48), ("medium10k", 48, 0, 64),
                                           ("medium10k", 48, 5, 32)])
def test_taped_solve_and_gpu_adjoint(dev, oracle_mod, name, n, K, tail):
    """The taping solver gives the same y as the plain one (bit for bit); its
    tapes hold the steps the stats count; the oracle's adjoint on those tapes
    agrees with the GPU reverse mode (same states z) element by element, and,
    after the oracle replays each tape to convergence, to the Newton
    tolerance.  Every dense-tail size of the reverse-mode kernels."""
    m, c, dt = synth.workload(name, n)
    b = Batch(dev, m, c, ld=n + 1, oracle_mod=oracle_mod, dense_tail=tail)
    N = m.n_species
    opts = mcchem.default_opts(steps_per_launch=K)
    y_plain = b.y_dev()
    st_plain, stats_plain = b.cells.step(y_plain, dt, opts)
    y0 = b.y_dev()
    y = y0.clone()
    sp = mcchem.stats_numpy(stats_plain)
    attempts = sp["steps"] + sp["rejects"] + sp["newton_fails"]
    stride = int((4 + 8 * attempts + N * sp["steps"]).max())  # the documented bound
    tape = torch.full((n, stride), float("nan"), dtype=torch.float64, device=dev)
    tlen = torch.empty(n, dtype=torch.int64, device=dev)
    stats = torch.empty_like(stats_plain)
    st, _ = b.cells.step_taped(y, dt, tape, tlen, opts, stats=stats)
    torch.cuda.synchronize()
    assert np.all(tlen.cpu().numpy() >= 0)
    assert torch.equal(y[:, :n], y_plain[:, :n]) and torch.equal(st, st_plain) and torch.equal(stats, stats_plain)
    assert np.all(st.cpu().numpy() == 0)
    stn = mcchem.stats_numpy(stats)
    tv, tl = tape.cpu().numpy(), tlen.cpu().numpy()
    k = b.o.rate_constants(c.T, c.jscale)
    rng = np.random.default_rng(5)
    W = rng.normal(size=(N, n)) / np.maximum(np.abs(y.cpu().numpy()[:, :n]), 1.0)
    lam = _t(_padded(W, n + 1, 0.0), dev)
    glnk, ast = b.cells.adjoint_step(y0, tape, tlen, lam)
    torch.cuda.synchronize()
    assert np.all(ast.cpu().numpy() == 0)
    lam_g, g_g = lam.cpu().numpy()[:, :n], glnk.cpu().numpy()[:, :n]
    worst_same, worst_replay = 0.0, 0.0
    for i in range(n):
        ov = tape_format.to_oracle(tv[i, :tl[i]], N)
        assert tape_format.count_steps(ov, N) == stn["steps"][i]  # a step entry per accepted step
        t = oracle_mod.Tape.from_values(b.o.lib, ov)
        lr, gr = b.o.adjoint(k[:, i], c.y0[:, i], t, W[:, i])
        worst_same = max(worst_same, _elementwise(lam_g[:, i], lr), _elementwise(g_g[:, i], gr))
        _, rt = b.o.replay(k[:, i], c.y0[:, i], t)
        lr2, gr2 = b.o.adjoint(k[:, i], c.y0[:, i], rt, W[:, i])
        worst_replay = max(worst_replay, np.abs(lam_g[:, i] - lr2).max() / np.abs(lr2).max(),
                           np.abs(g_g[:, i] - gr2).max() / np.abs(gr2).max())
    print(f"{name} K={K} tail={tail}: worst element-wise ratio to the bar, same tape {worst_same:.3g}; "
          f"worst relative difference after the oracle's replay {worst_replay:.3g}")
    assert worst_same <= 1.0
    assert worst_replay <= 1e-4


def test_taped_solve_overflow_marks_tape(dev, oracle_mod):
    m, c, dt = synth.workload("small10", 3)
    b = Batch(dev, m, c)
    y = b.y_dev()
    tape = torch.zeros((3, 20), dtype=torch.float64, device=dev)
    tlen = torch.zeros(3, dtype=torch.int64, device=dev)
    st, _ = b.cells.step_taped(y, dt, tape, tlen)
    y_plain = b.y_dev()
    b.cells.step(y_plain, dt)
    torch.cuda.synchronize()
    assert torch.equal(y, y_plain) and np.all(st.cpu().numpy() == 0)
    assert np.all(tlen.cpu().numpy() == -1)
    lam = torch.ones_like(y)
    _, ast = b.cells.adjoint_step(b.y_dev(), tape, tlen, lam)
    torch.cuda.synchronize()
    assert np.all(ast.cpu().numpy() == mcchem.CELL_BAD_TAPE)


def test_autograd_solve_step(dev, oracle_mod):
    """torch autograd through one outer step (taped forward, reverse-mode
    backward in the library) against the oracle's adjoint of the same tapes,
    for the log loss of the adjoint workload summed over cells."""
    from paper_2501_00011_amd import autograd
    m, c, dt = synth.workload("medium10k", 16)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    N = m.n_species
    k_gpu = b.cells.rate_constants().clone()
    lnk = torch.log(k_gpu).requires_grad_(True)
    y0 = b.y_dev().requires_grad_(True)
    y = autograd.solve_step(b.cells, y0, lnk, dt, tape_stride=50)  # forces the regrow path
    atol = 1.0
    target = torch.from_numpy(c.y0).to(dev) * 0.5 + 10.0
    loss = ((torch.log(y + atol) - torch.log(target + atol)) ** 2).sum()
    loss.backward()
    gl = lnk.grad.cpu().numpy()
    gy = y0.grad.cpu().numpy()
    # the oracle on the tapes the forward pass recorded (the Function keeps them)
    yd = y.detach().cpu().numpy()
    W = 2 * (np.log(yd + atol) - np.log(target.cpu().numpy() + atol)) / (yd + atol)
    k = k_gpu.cpu().numpy()
    tape = torch.empty((16, 4 + 2000 * (N + 8)), dtype=torch.float64, device=dev)
    tlen = torch.empty(16, dtype=torch.int64, device=dev)
    yy = b.y_dev()
    b.cells.step_taped(yy, dt, tape, tlen)
    torch.cuda.synchronize()
    assert torch.equal(yy, y.detach())
    tv, tl = tape.cpu().numpy(), tlen.cpu().numpy()
    for i in range(16):
        t = oracle_mod.Tape.from_values(b.o.lib, tape_format.to_oracle(tv[i, :tl[i]], N))
        lr, gr = b.o.adjoint(k[:, i], c.y0[:, i], t, W[:, i])
        assert np.abs(gy[:, i] - lr).max() <= 1e-9 * np.abs(lr).max()
        assert np.abs(gl[:, i] - gr).max() <= 1e-9 * np.abs(gr).max()


def test_autograd_integrate_checkpointed(dev, oracle_mod):
    """Three 60 s outer steps through autograd.integrate (checkpoints forward,
    tapes recomputed backward) against the oracle's adjoint chained over the
    same step tapes, for the log loss of the adjoint workload; the gradient
    with respect to log A is the sum over cells."""
    from paper_2501_00011_amd import autograd
    m, c, _ = synth.workload("medium10k", 8)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    N, n_out, dt = m.n_species, 3, 60.0
    k_gpu = b.cells.rate_constants().clone()
    lnk = torch.log(k_gpu).requires_grad_(True)
    y0 = b.y_dev().requires_grad_(True)
    y = autograd.integrate(b.cells, y0, lnk, dt, n_out)
    target = torch.from_numpy(c.y0).to(dev) * 0.7 + 5.0
    loss = ((torch.log(y + 1.0) - torch.log(target + 1.0)) ** 2).sum()
    loss.backward()
    gl, gy = lnk.grad.cpu().numpy(), y0.grad.cpu().numpy()
    # the same outer steps again, each with its tape, for the oracle
    yd = y.detach().cpu().numpy()
    W = 2 * (np.log(yd + 1.0) - np.log(target.cpu().numpy() + 1.0)) / (yd + 1.0)
    k = b.cells.rate_constants().cpu().numpy()
    ys, tapes = [], []
    yy = b.y_dev()
    for _ in range(n_out):
        ys.append(yy.cpu().numpy())
        tape = torch.empty((8, 4 + 3000 * (N + 8)), dtype=torch.float64, device=dev)
        tlen = torch.empty(8, dtype=torch.int64, device=dev)
        b.cells.step_taped(yy, dt, tape, tlen)
        torch.cuda.synchronize()
        tapes.append((tape.cpu().numpy(), tlen.cpu().numpy()))
    assert np.array_equal(yy.cpu().numpy(), yd)
    for i in range(8):
        lam, g = W[:, i].copy(), np.zeros(m.n_reactions)
        for s in reversed(range(n_out)):
            tv, tl = tapes[s]
            t = oracle_mod.Tape.from_values(b.o.lib, tape_format.to_oracle(tv[i, :tl[i]], N))
            lam, gs = b.o.adjoint(k[:, i], ys[s][:, i], t, lam)
            g += gs
        assert np.abs(gy[:, i] - lam).max() <= 1e-9 * np.abs(lam).max()
        assert np.abs(gl[:, i] - g).max() <= 1e-9 * np.abs(g).max()
    gA = gl.sum(axis=1)  # d L / d log A_j: every cell's k_j scales with A_j
    assert np.all(np.isfinite(gA)) and np.abs(gA).max() > 0


def test_gradient_full_size_sampled(dev, oracle_mod):
    """The log-loss gradient of 10 x 60 s for all 10,000 cells (as the
    gradient benchmark runs it); three sampled cells re-solved alone give
    the same states, and the oracle's adjoint chained over their tapes gives
    the same per-cell gradients."""
    from paper_2501_00011_amd import autograd
    m, c, dt = synth.workload("adjoint10k", None)
    C, N, R, n_out = c.n_cells, m.n_species, m.n_reactions, 10
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    k = b.cells.rate_constants().clone()
    y0 = b.y_dev()
    with torch.no_grad():
        pert = torch.from_numpy(np.random.default_rng(5005).normal(0.0, 0.1, R)).to(dev)
        target = autograd.integrate(b.cells, y0, torch.log(k) + pert[:, None], dt, n_out)
    lnk = torch.log(k).requires_grad_(True)
    y0g = y0.clone().requires_grad_(True)
    y = autograd.integrate(b.cells, y0g, lnk, dt, n_out)
    loss = ((torch.log(y + 1.0) - torch.log(target + 1.0)) ** 2).sum()
    loss.backward()
    sel = np.array([0, C // 2 + 1, C - 1])
    yd, td = y.detach().cpu().numpy()[:, sel], target.cpu().numpy()[:, sel]
    W = 2 * (np.log(yd + 1.0) - np.log(td + 1.0)) / (yd + 1.0)
    gl, gy = lnk.grad.cpu().numpy()[:, sel], y0g.grad.cpu().numpy()[:, sel]
    sub = synth.Cells(T=c.T[sel], P=c.P[sel], jscale=c.jscale[sel], y0=c.y0[:, sel])
    bs = Batch(dev, m, sub)
    bs.cells.set_rate_constants(torch.exp(torch.log(k[:, sel].contiguous())))
    kk = bs.cells.rate_constants().cpu().numpy()
    yy = bs.y_dev()
    ys, tapes = [], []
    for _ in range(n_out):
        ys.append(yy.cpu().numpy())
        tape = torch.empty((3, 4 + 3000 * (N + 8)), dtype=torch.float64, device=dev)
        tlen = torch.empty(3, dtype=torch.int64, device=dev)
        bs.cells.step_taped(yy, dt, tape, tlen)
        torch.cuda.synchronize()
        tapes.append((tape.cpu().numpy(), tlen.cpu().numpy()))
    assert np.array_equal(yy.cpu().numpy(), yd)  # a cell's solve does not depend on its batch
    for i in range(3):
        lam, g = W[:, i].copy(), np.zeros(R)
        for s in reversed(range(n_out)):
            tv, tl = tapes[s]
            t = oracle_mod.Tape.from_values(b.o.lib, tape_format.to_oracle(tv[i, :tl[i]], N))
            lam, gs = b.o.adjoint(kk[:, i], ys[s][:, i], t, lam)
            g += gs
        assert np.abs(gy[:, i] - lam).max() <= 1e-9 * np.abs(lam).max()
        assert np.abs(gl[:, i] - g).max() <= 1e-9 * np.abs(g).max()


@pytest.mark.parametrize("name,n", [("small10", 10), ("medium10k", 24)])
def test_replay_step_parity(dev, oracle_mod, name, n):
    """The GPU replay of GPU-recorded tapes against the oracle's replay of
    the same tapes (both solve every step to convergence), and against the
    forward solve it replays (to the forward's Newton tolerance)."""
    m, c, dt = synth.workload(name, n)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    N = m.n_species
    y0 = b.y_dev()
    y = y0.clone()
    tape = torch.empty((n, 4 + 2000 * (N + 8)), dtype=torch.float64, device=dev)
    tlen = torch.empty(n, dtype=torch.int64, device=dev)
    st, _ = b.cells.step_taped(y, dt, tape, tlen)
    yr, rst = b.cells.replay_step(y0, tape, tlen)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0) and np.all(rst.cpu().numpy() == 0)
    yr, yf = yr.cpu().numpy(), y.cpu().numpy()
    assert np.all(np.abs(yr - yf) <= 1e-6 * np.abs(yf) + 1e2)  # the step bar
    k = b.cells.rate_constants().cpu().numpy()
    tv, tl = tape.cpu().numpy(), tlen.cpu().numpy()
    worst = 0.0
    for i in range(n):
        t = oracle_mod.Tape.from_values(b.o.lib, tape_format.to_oracle(tv[i, :tl[i]], N))
        yo, _ = b.o.replay(k[:, i], c.y0[:, i], t)
        worst = max(worst, float(np.max(np.abs(yr[:, i] - yo) / (np.abs(yo) + 1.0))))
    print(f"{name}: GPU replay vs oracle replay, worst relative difference {worst:.3g}")
    assert worst <= 1e-10


def test_replay_rejects_bad_tapes(dev):
    m, c, dt = synth.workload("small10", 3)
    b = Batch(dev, m, c)
    N = m.n_species
    y0 = b.y_dev()
    y = y0.clone()
    tape = torch.empty((3, 4 + 2000 * (N + 8)), dtype=torch.float64, device=dev)
    tlen = torch.empty(3, dtype=torch.int64, device=dev)
    b.cells.step_taped(y, dt, tape, tlen)
    torch.cuda.synchronize()
    bad_len = tlen.clone()
    bad_len[0] = 0                  # empty: y = y0
    bad_len[1] = tape.shape[1] + 4  # beyond the stride
    bad_len[2] = tlen[2] - 1        # the last entry cut short
    yr, rst = b.cells.replay_step(y0, tape, bad_len)
    torch.cuda.synchronize()
    assert rst.cpu().tolist() == [mcchem.CELL_OK, mcchem.CELL_BAD_TAPE, mcchem.CELL_BAD_TAPE]
    assert torch.equal(yr[:, 0], y0[:, 0]) and torch.isnan(yr[:, 1:]).all()


def test_gradient_against_central_differences_of_the_replay(dev):
    """d L / d log A for 64 cells over 10 x 60 s (the adjoint workload's log
    loss and perturbed target) against central differences, h = 1e-6, of
    the frozen step sequences replayed on the GPU, for six parameters, and
    d L / d y0 along one direction."""
    from paper_2501_00011_amd import autograd
    m, c, dt = synth.workload("adjoint10k", 64)
    C, N, R, n_out, eps = 64, m.n_species, m.n_reactions, 10, 1e-6
    b = Batch(dev, m, c)
    k = b.cells.rate_constants().clone()
    y0 = b.y_dev()
    with torch.no_grad():
        pert = torch.from_numpy(np.random.default_rng(5005).normal(0.0, 0.1, R)).to(dev)
        target = autograd.integrate(b.cells, y0, torch.log(k) + pert[:, None], dt, n_out)
    lnk = torch.log(k).requires_grad_(True)
    y = autograd.integrate(b.cells, y0, lnk, dt, n_out)
    loss = ((torch.log(y + 1.0) - torch.log(target + 1.0)) ** 2).sum()
    loss.backward()
    gA = lnk.grad.sum(dim=1).cpu().numpy()
    # the forward's tapes, then the loss of the replayed chain at perturbed log A
    b.cells.set_rate_constants(k)
    tapes, yy = [], y0.clone()
    for _ in range(n_out):
        tape = torch.empty((C, 4 + 3000 * (N + 8)), dtype=torch.float64, device=dev)
        tlen = torch.empty(C, dtype=torch.int64, device=dev)
        b.cells.step_taped(yy, dt, tape, tlen)
        tapes.append((tape, tlen))

    def replayed_loss(j, sign, y_start=None):
        kp = k.clone()
        if j is not None:
            kp[j] *= math.exp(sign * eps)
        b.cells.set_rate_constants(kp)
        ys = y0 if y_start is None else y_start
        for tape, tlen in tapes:
            ys, st = b.cells.replay_step(ys, tape, tlen)
            assert int((st != 0).sum()) == 0
        return float(((torch.log(ys + 1.0) - torch.log(target + 1.0)) ** 2).sum())

    sel = list(np.argsort(-np.abs(gA))[:3]) + list(np.random.default_rng(3).choice(R, 3, replace=False))
    for j in sel:
        fd = (replayed_loss(j, 1) - replayed_loss(j, -1)) / (2 * eps)
        print(f"log A_{j}: adjoint {gA[j]:.9g}, central difference {fd:.9g}")
        assert abs(fd - gA[j]) <= 1e-5 * abs(gA[j]) + 1e-7 * float(loss.detach()), (j, fd, gA[j])
    # d L / d y0 along a direction u (relative perturbations of every cell's state)
    u = torch.from_numpy(np.random.default_rng(4).normal(size=tuple(y0.shape))).to(dev) * y0
    y0g = y0.clone().requires_grad_(True)
    lnk2 = torch.log(k)
    yy2 = autograd.integrate(b.cells, y0g, lnk2, dt, n_out)
    ((torch.log(yy2 + 1.0) - torch.log(target + 1.0)) ** 2).sum().backward()
    adj = float((y0g.grad * u).sum())
    fd = (replayed_loss(None, 0, y0 + eps * u) - replayed_loss(None, 0, y0 - eps * u)) / (2 * eps)
    print(f"d L / d y0 along u: adjoint {adj:.9g}, central difference {fd:.9g}")
    assert abs(fd - adj) <= 1e-5 * abs(adj) + 1e-7 * float(loss.detach())
    b.cells.set_rate_constants(k)


@pytest.mark.parametrize("K", [0, 3])
def test_cell_schedule_leaves_results_unchanged(dev, K):
    """Any cell schedule (here longest first by the previous step's
    attempts, and a random one) gives every cell the same bits, in one
    launch and in the per-launch form, and the same step tapes and
    reverse-mode results."""
    m, c, dt = synth.workload("medium10k", 300)
    b = Batch(dev, m, c)
    N = m.n_species
    opts = mcchem.default_opts(steps_per_launch=K)
    y0 = b.y_dev()

    def run():
        y = y0.clone()
        st, stats = b.cells.step(y, dt, opts)
        tape = torch.empty((300, 4 + 1500 * (N + 8)), dtype=torch.float64, device=dev)
        tlen = torch.empty(300, dtype=torch.int64, device=dev)
        yt = y0.clone()
        b.cells.step_taped(yt, dt, tape, tlen, opts)
        lam = torch.ones_like(y0)
        glnk, ast = b.cells.adjoint_step(y0, tape, tlen, lam)
        torch.cuda.synchronize()
        return y, st, stats, tape, tlen, lam, glnk

    ref = run()
    order = b.cells.balance(ref[2])
    assert sorted(order.tolist()) == list(range(300))
    att = mcchem.stats_numpy(ref[2])
    attempts = (att["steps"] + att["rejects"] + att["newton_fails"]).astype(np.int64)
    assert np.all(np.diff(attempts[order]) <= 0)  # longest first
    assert np.array_equal(order, np.argsort(-attempts, kind="stable"))  # ties keep the cell order
    for sched in (order, np.random.default_rng(1).permutation(300).astype(np.int32)):
        b.cells.set_schedule(sched)
        got = run()
        for x, y in zip(ref, got):
            if x.dtype == torch.float64 and x.dim() == 2 and x.shape[0] == 300:  # tapes: up to each length
                for i in range(300):
                    assert torch.equal(x[i, :int(ref[4][i])], y[i, :int(ref[4][i])])
            else:
                assert torch.equal(x, y)
    b.cells.set_schedule(None)
    assert torch.equal(run()[0], ref[0])


def test_register_budget_and_zigzag_leave_results_unchanged(dev):
    """The solver built for one wavefront per SIMD, and the zigzag cell
    schedule, give every cell the bits of the default build and order."""
    m, c, dt = synth.workload("medium10k", 300)
    ref = Batch(dev, m, c, dense_tail=32)
    y_ref = ref.y_dev()
    _, st_ref = ref.cells.step(y_ref, dt)
    one = Batch.__new__(Batch)
    one.m, one.c, one.C, one.ld, one.dev = m, c, 300, 300, dev
    one.h = mcchem.Mechanism(m, dense_tail=32, waves_per_simd=1)
    assert one.h.schedule_info()["waves_per_simd"] == 1 and ref.h.schedule_info()["waves_per_simd"] == 2
    one.cells = mcchem.Cells(one.h, 300)
    one.cells.bind(ref.T, ref.P, ref.s)
    order = one.cells.balance(st_ref, "zigzag")
    att = mcchem.stats_numpy(st_ref)
    a = (att["steps"] + att["rejects"] + att["newton_fails"]).astype(np.int64)
    lf = np.argsort(-a, kind="stable")
    assert order[0] == lf[0] and order[1] == lf[-1] and order[2] == lf[1] and sorted(order) == list(range(300))
    y = one.y_dev()
    _, st = one.cells.step(y, dt)
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref) and torch.equal(st, st_ref)
    with pytest.raises(mcchem.MccError, match="wavefronts"):
        mcchem.Mechanism(synth.mech_large(), waves_per_simd=2)


def test_cell_schedule_rejects_non_permutations(dev):
    m, c, _ = synth.workload("small10", 4)
    b = Batch(dev, m, c)
    for bad in ([0, 1, 2, 2], [0, 1, 2, 4], [-1, 0, 1, 2]):
        with pytest.raises(mcchem.MccError, match="permutation"):
            b.cells.set_schedule(np.array(bad, dtype=np.int32))
    with pytest.raises(mcchem.MccError):
        b.cells.set_schedule(np.arange(3, dtype=np.int32))


def test_reverse_mode_large_mechanism(dev, oracle_mod):
    """The 150-species mechanism (three register slots, 64-row dense tail):
    taped solve equal to the plain one, reverse pass and replay against the
    oracle's adjoint and replay of the same tapes."""
    m = synth.mech_large()
    n, dt = 6, 60.0
    c = synth.make_cells(m, n, seed=516)
    b = Batch(dev, m, c, oracle_mod=oracle_mod)
    N = m.n_species
    info = b.h.schedule_info()
    assert info["dense_tail"] == 64
    y0 = b.y_dev()
    y_plain = y0.clone()
    st_plain, stats = b.cells.step(y_plain, dt)
    sn = mcchem.stats_numpy(stats)
    stride = int((4 + 8 * (sn["steps"] + sn["rejects"] + sn["newton_fails"]) + N * sn["steps"]).max())
    tape = torch.empty((n, stride), dtype=torch.float64, device=dev)
    tlen = torch.empty(n, dtype=torch.int64, device=dev)
    y = y0.clone()
    st, _ = b.cells.step_taped(y, dt, tape, tlen)
    torch.cuda.synchronize()
    assert torch.equal(y, y_plain) and np.all(st.cpu().numpy() == 0) and np.all(tlen.cpu().numpy() > 0)
    rng = np.random.default_rng(17)
    yd = y.cpu().numpy()
    W = rng.normal(size=(N, n)) / np.maximum(np.abs(yd), 1.0)
    lam = _t(W, dev)
    glnk, ast = b.cells.adjoint_step(y0, tape, tlen, lam)
    yr, rst = b.cells.replay_step(y0, tape, tlen)
    torch.cuda.synchronize()
    assert np.all(ast.cpu().numpy() == 0) and np.all(rst.cpu().numpy() == 0)
    lam_g, g_g, yr = lam.cpu().numpy(), glnk.cpu().numpy(), yr.cpu().numpy()
    k = b.cells.rate_constants().cpu().numpy()
    tv, tl = tape.cpu().numpy(), tlen.cpu().numpy()
    for i in range(n):
        t = oracle_mod.Tape.from_values(b.o.lib, tape_format.to_oracle(tv[i, :tl[i]], N))
        lr, gr = b.o.adjoint(k[:, i], c.y0[:, i], t, W[:, i])
        assert np.abs(lam_g[:, i] - lr).max() <= 1e-9 * np.abs(lr).max()
        assert np.abs(g_g[:, i] - gr).max() <= 1e-9 * np.abs(gr).max()
        yo, _ = b.o.replay(k[:, i], c.y0[:, i], t)
        assert np.abs(yr[:, i] - yo).max() <= 1e-10 * (np.abs(yo).max() + 1.0)


# ---- the 200,000-cell workload: stiffness spread over the photolysis scale ----

def test_medium200k_sampled_both_forms(dev, oracle_mod):
    """200,000 cells with the photolysis scale log-uniform on [1e-3, 1] (step
    counts spread across cells), 32-row dense tail: one launch and the
    per-launch form (at most 8 accepted steps per launch) give the same bits;
    64 cells spread over the photolysis-scale range against the oracle."""
    m, c, dt = synth.workload("medium200k")
    b = Batch(dev, m, c, oracle_mod=oracle_mod, dense_tail=32)
    y1 = b.y_dev()
    s1, t1 = b.cells.step(y1, dt)
    y2 = b.y_dev()
    s2, t2 = b.cells.step(y2, dt, mcchem.default_opts(steps_per_launch=8))
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(s1, s2) and torch.equal(t1, t2)
    assert int((s1 != 0).sum()) == 0
    sn = mcchem.stats_numpy(t1)
    print(f"medium200k: steps per cell 1st/50th/99th percentile {np.percentile(sn['steps'], [1, 50, 99])}")
    order = np.argsort(c.jscale)
    sel = np.sort(order[np.linspace(0, c.n_cells - 1, 64).astype(int)])
    k = b.o.rate_constants(c.T[sel], c.jscale[sel])
    yo, so, sto = b.o.solve(k, c.y0[:, sel], dt)
    assert np.all(so == 0)
    worst = _within(y1.cpu().numpy()[:, sel], yo, 1.0)
    same = np.mean((sn["steps"][sel] == sto["steps"]) & (sn["rejects"][sel] == sto["rejects"]))
    print(f"medium200k: worst {worst:.3g} of the bar over jscale {c.jscale[sel].min():.2g}..{c.jscale[sel].max():.2g}, "
          f"identical step sequences in {same:.0%} of cells")
    assert worst <= 1.0


# ---- warm start -------------------------------------------------------------

def _stats_with_h_next(h, dev):
    st = np.zeros(len(h), dtype=mcchem.STATS_DTYPE)
    st["h_next"] = h
    return torch.from_numpy(st.view(np.uint8).reshape(len(h), -1).copy()).to(dev)


def test_warm_start_parity(dev, oracle_mod):
    """A warm-started outer step (first step size from the stats record)
    against the oracle given the same first step sizes (seeded, log-uniform
    on [1e-4, 10] s), then a cold step followed by a warm one on each side."""
    import oracle as orc
    m, c, dt = synth.workload("medium10k", 64)
    b = Batch(dev, m, c, oracle_mod=oracle_mod, dense_tail=32)
    k = b.o.rate_constants(c.T, c.jscale)
    hw = 10.0 ** np.random.default_rng(31).uniform(-4.0, 1.0, 64)
    y = b.y_dev()
    stats = _stats_with_h_next(hw, dev)
    st, _ = b.cells.step(y, dt, mcchem.default_opts(warm_start=1), stats=stats)
    torch.cuda.synchronize()
    yo, so, sto = b.o.solve(k, c.y0, dt, orc.default_opts(warm_start=1), h_warm=hw)
    assert np.all(st.cpu().numpy() == 0) and np.all(so == 0)
    assert _within(y.cpu().numpy(), yo, 1.0) <= 1.0
    # cold then warm, each side from its own first step
    y = b.y_dev()
    _, stats = b.cells.step(y, dt)
    cold = mcchem.stats_numpy(stats)["steps"].copy()
    st2, stats2 = b.cells.step(y, dt, mcchem.default_opts(warm_start=1), stats=stats)
    torch.cuda.synchronize()
    y1o, _, st1o = b.o.solve(k, c.y0, dt)
    y2o, s2o, st2o = b.o.solve(k, y1o, dt, orc.default_opts(warm_start=1), h_warm=st1o["h_next"])
    sg = mcchem.stats_numpy(stats2)
    assert np.all(st2.cpu().numpy() == 0) and np.all(s2o == 0)
    assert _within(y.cpu().numpy(), y2o, 1.0) <= 1.0
    print(f"warm start: second step {sg['steps'].mean():.0f} steps per cell (first, cold: {cold.mean():.0f})")
    with pytest.raises(mcchem.MccError, match="stats"):
        b.cells.step(b.y_dev(), dt, mcchem.default_opts(warm_start=1), want_stats=False)
    with pytest.raises(mcchem.MccError, match="warm_start"):
        b.cells.step_multicell(b.y_dev(), dt, mcchem.default_opts(warm_start=1))


# ---- mixed batch: a captured window of ten outer steps ----------------------

def test_mixed_mechanisms_ten_step_graph_window(dev, oracle_mod):
    """Three mechanisms (20, 72, 150 species) on their own streams, ten
    consecutive 60 s outer steps of all of them captured into one graph:
    one replay equals ten eager steps bit for bit (and a second replay the
    next ten); sampled cells after ten steps match the oracle's ten chained
    steps."""
    import oracle as orc
    groups, owner, dt = synth.mixed_workload(600)
    streams = [torch.cuda.Stream(device=dev) for _ in groups]
    batches, ys, ye, st = [], [], [], []
    for (m, c), s in zip(groups, streams):
        b = Batch(dev, m, c, oracle_mod=oracle_mod)
        batches.append(b)
        ys.append(b.y_dev())
        ye.append(b.y_dev())
        st.append(torch.empty(c.n_cells, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    ref = []
    for w in range(2):
        for _ in range(10):
            for b, y, s_ in zip(batches, ye, st):
                b.cells.step(y, dt, status=s_, want_stats=False)
        torch.cuda.synchronize()
        ref.append([y.clone() for y in ye])
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cap):
        for _ in range(10):
            for b, y, s_, side in zip(batches, ys, st, streams):
                side.wait_stream(cap)
                b.cells.step(y, dt, status=s_, want_stats=False, stream=side)
                cap.wait_stream(side)
    for w in range(2):
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=dev).sum().item()  # unrelated eager work between replays
        for y, yr in zip(ys, ref[w]):
            assert torch.equal(y, yr), f"window {w}"
    for b, yr in zip(batches, ref[0]):
        sel = np.arange(0, b.C, max(1, b.C // 4))
        k = b.o.rate_constants(b.c.T[sel], b.c.jscale[sel])
        yo = b.c.y0[:, sel]
        for _ in range(10):
            yo, so, _ = b.o.solve(k, yo, dt, orc.default_opts())
            assert np.all(so == 0)
        worst = _within(yr.cpu().numpy()[:, sel], yo, 1.0)
        print(f"{b.m.n_species} species: ten chained steps, worst {worst:.3g} of the bar")
        assert worst <= 1.0


# ---- the adjoint workload in full: every log A against central differences --

def test_gradient_all_parameters_against_central_differences(dev):
    """d L / d log A for all 156 reactions (64 cells, 10 x 60 s, the adjoint
    workload's log loss and perturbed target) against central differences,
    h = 1e-6, of the frozen step sequences replayed on the GPU.  The 2 x 156
    perturbed replays run as batches of replicated cells, each copy of the
    64 cells with its own rate constants and the forward's step tapes."""
    from paper_2501_00011_amd import autograd
    m, c, dt = synth.workload("adjoint10k", 64)
    C, N, R, n_out, eps = 64, m.n_species, m.n_reactions, 10, 1e-6
    b = Batch(dev, m, c)
    k = b.cells.rate_constants().clone()
    y0 = b.y_dev()
    with torch.no_grad():
        pert = torch.from_numpy(np.random.default_rng(5005).normal(0.0, 0.1, R)).to(dev)
        target = autograd.integrate(b.cells, y0, torch.log(k) + pert[:, None], dt, n_out)
    lnk = torch.log(k).requires_grad_(True)
    y = autograd.integrate(b.cells, y0, lnk, dt, n_out)
    loss = ((torch.log(y + 1.0) - torch.log(target + 1.0)) ** 2).sum()
    loss.backward()
    gA = lnk.grad.sum(dim=1).cpu().numpy()
    b.cells.set_rate_constants(k)
    tapes, yy = [], y0.clone()
    for _ in range(n_out):
        tape = torch.empty((C, 4 + 3000 * (N + 8)), dtype=torch.float64, device=dev)
        tlen = torch.empty(C, dtype=torch.int64, device=dev)
        st, _ = b.cells.step_taped(yy, dt, tape, tlen)
        assert int((st != 0).sum()) == 0 and int(tlen.min()) > 0
        width = int(tlen.max())
        tapes.append((tape[:, :width].contiguous(), tlen))
    per = 26  # parameters per batch: 2 x 26 copies of the 64 cells
    fd = np.zeros(R)
    h = mcchem.Mechanism(m)
    for j0 in range(0, R, per):
        js = list(range(j0, min(R, j0 + per)))
        P = 2 * len(js)
        cells = mcchem.Cells(h, P * C)
        kp = k.repeat(1, P)  # copy q of the cells at columns q C .. q C + C - 1
        for q, j in enumerate(js):
            kp[j, (2 * q) * C:(2 * q + 1) * C] *= math.exp(eps)
            kp[j, (2 * q + 1) * C:(2 * q + 2) * C] *= math.exp(-eps)
        cells.set_rate_constants(kp.contiguous())
        ys = y0.repeat(1, P).contiguous()
        for tape, tlen in tapes:
            ys, rst = cells.replay_step(ys, tape.repeat(P, 1).contiguous(), tlen.repeat(P).contiguous())
            assert int((rst != 0).sum()) == 0
        lc = ((torch.log(ys + 1.0) - torch.log(target.repeat(1, P) + 1.0)) ** 2).reshape(N, P, C).sum(dim=(0, 2))
        lc = lc.cpu().numpy()
        for q, j in enumerate(js):
            fd[j] = (lc[2 * q] - lc[2 * q + 1]) / (2 * eps)
        cells.close()
    bar = 1e-5 * np.abs(gA) + 1e-7 * float(loss.detach())
    ratio = np.abs(fd - gA) / bar
    print(f"all {R} log A: worst ratio to the bar {ratio.max():.3g} (parameter {int(ratio.argmax())}); "
          f"largest |dL/dlogA| {np.abs(gA).max():.3g}, loss {float(loss.detach()):.4g}")
    assert np.all(ratio <= 1.0)
