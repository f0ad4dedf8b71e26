"""Seeded synthetic inputs: mechanisms and cell states.

This module is the single source of inputs for the oracle, the tests and the
benchmark.  It builds mechanisms and initial states only; it evaluates no rate,
tendency, Jacobian or integrator step.

Mechanism (general reaction of Section 2, "Background"):
    c_1 y_1 + ... + c_m y_m  ->  c_{m+1} y_{m+1} + ... + c_n y_n
Reactants carry integer coefficients (a repeated index is a multiplicity);
products carry floating-point yields, matching the split the paper makes between
integer reaction parameters (indices, stoichiometric coefficients) and
floating-point ones (conversion factors, rate parameters).

The paper's own workloads (a CB05 mechanism, MONARCH fields and a 3-species
test mechanism with unstated Arrhenius parameters) are not available, so these
generators stand in for them: random gas-phase mass-action mechanisms with
first-order (thermal or photolysis), bimolecular and termolecular reactions.
Every reaction conserves two synthetic "elements": each species has an integer
composition vector in {0..4}^2 and product yields are solved so that atoms
balance, which gives conservation laws that any correct f and J obey.

State is a number density in molecule cm^-3: n = x * M with
M = 100 * P[hPa] / (k_B * T) * 1e-6 (air number density).
Per-cell arrays are laid out [entity][ld] with the cell index fastest.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

K_BOLTZMANN = 1.380649e-23  # J/K (exact SI value)
# Reference air number density (molecule cm^-3).  Termolecular pre-factors are
# drawn on the same log-uniform range as bimolecular ones and then divided by
# this, which puts them on the physical scale of a bimolecular rate times 1/M.
M_REF = 2.46e19

RXN_THERMAL = 0
RXN_PHOTOLYSIS = 1


@dataclasses.dataclass
class Mechanism:
    n_species: int
    n_reactions: int
    rxn_type: np.ndarray    # int32 [R]: 0 thermal Arrhenius, 1 photolysis
    reac_ptr: np.ndarray    # int32 [R+1] CSR over reactants
    reac_idx: np.ndarray    # int32 [nreac]; a repeated index is a multiplicity
    prod_ptr: np.ndarray    # int32 [R+1] CSR over products
    prod_idx: np.ndarray    # int32 [nprod]
    prod_yield: np.ndarray  # float64 [nprod]
    A: np.ndarray           # float64 [R]: Arrhenius pre-factor, or J-rate for photolysis
    theta: np.ndarray       # float64 [R]: Ea/R in K (0 for photolysis)
    composition: np.ndarray | None = None  # int32 [N, n_elements], None if not atom-balanced
    name: str = ""

    def arity(self) -> np.ndarray:
        return np.diff(self.reac_ptr).astype(np.int32)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.rxn_type, self.reac_ptr, self.reac_idx, self.prod_ptr,
                  self.prod_idx, self.prod_yield, self.A, self.theta):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


@dataclasses.dataclass
class Cells:
    T: np.ndarray       # float64 [C] temperature, K
    P: np.ndarray       # float64 [C] pressure, hPa
    jscale: np.ndarray  # float64 [C] photolysis scale factor
    y0: np.ndarray      # float64 [N, C] number densities, molecule cm^-3

    @property
    def n_cells(self) -> int:
        return int(self.T.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.T, self.P, self.jscale, self.y0):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def split_counts(total: int, percents) -> list[int]:
    """Largest-remainder split of `total` by integer percentages (sum 100).

    Integer arithmetic only, ties to the earlier entry, so 156 reactions at
    30/60/10 give 47/94/15 (a float split would round to 47/93/16).
    """
    percents = [int(p) for p in percents]
    if sum(percents) != 100:
        raise ValueError("percentages must sum to 100")
    base = [p * total // 100 for p in percents]
    rem = [p * total % 100 for p in percents]
    left = total - sum(base)
    order = sorted(range(len(percents)), key=lambda i: (-rem[i], i))
    for i in order[:left]:
        base[i] += 1
    return base


def make_mechanism(n_species: int, n_reactions: int, percents=(30, 60, 10),
                   first_order: str = "photolysis", seed: int | None = None,
                   max_draws: int = 10000, termolecular_per_M: bool = True) -> Mechanism:
    """Random atom-balanced mass-action mechanism.

    percents: share of first-order, bimolecular and termolecular reactions.
    first_order: "photolysis" (k = J * s_cell) or "thermal" (Arrhenius).
    Reactants are distinct species; each reaction has two distinct products
    that are not reactants, with yields in [0.05, 5] solving the 2x2 atom
    balance exactly (up to rounding).  Product pairs are drawn until one fits;
    after 100 misfits the reactant set itself is redrawn.
    Thermal pre-factors are log-uniform on [1e-14, 1e-10]; with
    termolecular_per_M the termolecular ones are then divided by M_REF.
    """
    if seed is None:
        seed = n_species
    if first_order not in ("photolysis", "thermal"):
        raise ValueError(first_order)
    if n_species < 5:
        raise ValueError("need at least 5 species (3 reactants + 2 products)")
    rng = np.random.default_rng(seed)
    comp = rng.integers(0, 5, size=(n_species, 2))
    for i in range(n_species):
        while comp[i, 0] == 0 and comp[i, 1] == 0:
            comp[i] = rng.integers(0, 5, size=2)
    n1, n2, n3 = split_counts(n_reactions, percents)
    arity = np.array([1] * n1 + [2] * n2 + [3] * n3, dtype=np.int32)
    rng.shuffle(arity)

    reac_idx, prod_idx, prod_yield = [], [], []
    reac_ptr, prod_ptr = [0], [0]
    for j in range(n_reactions):
        for attempt in range(max_draws):
            if attempt % 100 == 0:
                # a reactant set whose atoms no product pair balances is redrawn
                reac = rng.choice(n_species, size=int(arity[j]), replace=False)
                need = comp[reac].sum(axis=0).astype(np.float64)
                others = np.setdiff1d(np.arange(n_species), reac)
            p = rng.choice(others, size=2, replace=False)
            a = comp[p].T.astype(np.float64)  # columns = product compositions
            det = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
            if det == 0:
                continue
            if np.linalg.cond(a) > 50.0:
                continue
            yl = np.linalg.solve(a, need)
            if np.all(yl >= 0.05) and np.all(yl <= 5.0):
                break
        else:
            raise RuntimeError(f"reaction {j}: no balanced product pair in {max_draws} draws")
        reac_idx.extend(int(s) for s in reac)
        prod_idx.extend(int(s) for s in p)
        prod_yield.extend(float(v) for v in yl)
        reac_ptr.append(len(reac_idx))
        prod_ptr.append(len(prod_idx))

    log10A = rng.uniform(-14.0, -10.0, size=n_reactions)
    theta = rng.uniform(0.0, 2000.0, size=n_reactions)
    jrate = rng.uniform(0.0, 1e-2, size=n_reactions)
    rtype = np.zeros(n_reactions, dtype=np.int32)
    A = 10.0 ** log10A
    if termolecular_per_M:
        A[arity == 3] /= M_REF
    if first_order == "photolysis":
        photo = arity == 1
        rtype[photo] = RXN_PHOTOLYSIS
        A[photo] = jrate[photo]
        theta[photo] = 0.0
    return Mechanism(
        n_species=n_species, n_reactions=n_reactions, rxn_type=rtype,
        reac_ptr=np.array(reac_ptr, dtype=np.int32), reac_idx=np.array(reac_idx, dtype=np.int32),
        prod_ptr=np.array(prod_ptr, dtype=np.int32), prod_idx=np.array(prod_idx, dtype=np.int32),
        prod_yield=np.array(prod_yield, dtype=np.float64), A=A.astype(np.float64),
        theta=theta.astype(np.float64), composition=comp.astype(np.int32),
        name=f"synthetic N{n_species}/R{n_reactions} {first_order} {percents} seed {seed}")


def mechanism_from_lists(n_species, reactions, composition=None, name="") -> Mechanism:
    """Build a Mechanism from a list of
    (reactants: list[int], products: list[(int, yield)], A, theta, kind) tuples,
    kind 0 thermal / 1 photolysis.  Used for hand-written test mechanisms."""
    reac_ptr, reac_idx, prod_ptr, prod_idx, prod_yield = [0], [], [0], [], []
    A, theta, rtype = [], [], []
    for reac, prods, a, th, kind in reactions:
        reac_idx.extend(int(s) for s in reac)
        for s, yl in prods:
            prod_idx.append(int(s))
            prod_yield.append(float(yl))
        reac_ptr.append(len(reac_idx))
        prod_ptr.append(len(prod_idx))
        A.append(float(a))
        theta.append(float(th))
        rtype.append(int(kind))
    return Mechanism(
        n_species=int(n_species), n_reactions=len(reactions),
        rxn_type=np.array(rtype, dtype=np.int32),
        reac_ptr=np.array(reac_ptr, dtype=np.int32), reac_idx=np.array(reac_idx, dtype=np.int32),
        prod_ptr=np.array(prod_ptr, dtype=np.int32), prod_idx=np.array(prod_idx, dtype=np.int32),
        prod_yield=np.array(prod_yield, dtype=np.float64),
        A=np.array(A, dtype=np.float64), theta=np.array(theta, dtype=np.float64),
        composition=None if composition is None else np.asarray(composition, dtype=np.int32),
        name=name)


def air_number_density(T, P_hPa):
    """M = P / (k_B T) in molecule cm^-3 (P in hPa, T in K)."""
    return 100.0 * np.asarray(P_hPa, dtype=np.float64) / (K_BOLTZMANN * np.asarray(T, dtype=np.float64)) * 1e-6


def make_cells(mech: Mechanism, n_cells: int, seed: int, T_range=(220.0, 310.0),
               P_range=(100.0, 1013.0), P_fixed: float | None = None,
               jscale_log10_range: tuple | None = None,
               x_log10_range=(-12.0, -6.0)) -> Cells:
    """Random per-cell environment and initial number densities.

    Draw order (fixed): T, P, photolysis scale, mixing ratios.
    """
    rng = np.random.default_rng(seed)
    T = rng.uniform(T_range[0], T_range[1], size=n_cells)
    if P_fixed is not None:
        P = np.full(n_cells, float(P_fixed))
    else:
        P = rng.uniform(P_range[0], P_range[1], size=n_cells)
    if jscale_log10_range is None:
        s = np.ones(n_cells)
    else:
        s = 10.0 ** rng.uniform(jscale_log10_range[0], jscale_log10_range[1], size=n_cells)
    x = 10.0 ** rng.uniform(x_log10_range[0], x_log10_range[1], size=(mech.n_species, n_cells))
    y0 = x * air_number_density(T, P)[None, :]
    return Cells(T=T, P=P, jscale=s, y0=np.ascontiguousarray(y0))


# ---------------------------------------------------------------------------
# The workloads: five configurations of increasing size.
# ---------------------------------------------------------------------------

def mech_small_thermal() -> Mechanism:
    """20 species, 30 reactions: 40% first-order thermal, 50% bi-, 10% termolecular."""
    return make_mechanism(20, 30, (40, 50, 10), first_order="thermal", seed=20)


def mech_small() -> Mechanism:
    """20 species, 30 reactions at the 30/60/10 photolysis mix (mixed-batch member)."""
    return make_mechanism(20, 30, (30, 60, 10), first_order="photolysis", seed=21)


def mech_medium() -> Mechanism:
    """72 species, 156 reactions: 30% photolysis, 60% bi-, 10% termolecular."""
    return make_mechanism(72, 156, (30, 60, 10), first_order="photolysis", seed=72)


def mech_large() -> Mechanism:
    """150 species, 350 reactions at the 30/60/10 photolysis mix."""
    return make_mechanism(150, 350, (30, 60, 10), first_order="photolysis", seed=150)


def workload(name: str, n_cells: int | None = None):
    """Return (mechanism, cells, dt) for a named workload.

    small10   : 20/30 thermal mechanism, 10 cells, T 250-310 K, P 1013.25 hPa, one 60 s step
    medium10k : 72/156 mechanism, 10,000 cells, T 220-310 K, P 100-1013 hPa, one 180 s step
    medium200k: as medium10k with 200,000 cells and photolysis scale log-uniform 1e-3..1
    adjoint10k: as medium10k, 60 s steps (ten of them for the adjoint workload)
    paper_test: Section 4's 3-species mechanism, 1,000 cells with index offsets, one 60 s step
    """
    if name == "small10":
        m = mech_small_thermal()
        c = make_cells(m, n_cells or 10, seed=1001, T_range=(250.0, 310.0), P_fixed=1013.25)
        return m, c, 60.0
    if name == "medium10k":
        m = mech_medium()
        c = make_cells(m, n_cells or 10000, seed=1002)
        return m, c, 180.0
    if name == "medium200k":
        m = mech_medium()
        c = make_cells(m, n_cells or 200000, seed=1003, jscale_log10_range=(-3.0, 0.0))
        return m, c, 180.0
    if name == "paper_test":
        # Section 4's mechanism: A gives B and C through two Arrhenius
        # reactions (theta = 0; A = 0.05 and 0.02 s^-1, parameters the paper
        # does not print); A = 1, B = C = 0 plus 0.1 * (flattened index + 1)
        # over the concatenated cells; T, P and parameters equal in all cells
        C = n_cells or 1000
        m = mechanism_from_lists(3, [([0], [(1, 1.0)], 0.05, 0.0, RXN_THERMAL),
                                     ([0], [(2, 1.0)], 0.02, 0.0, RXN_THERMAL)])
        flat = np.concatenate([np.array([1.0, 0.0, 0.0]) + 0.1 * (c * 3 + np.arange(3) + 1) for c in range(C)])
        c = Cells(T=np.full(C, 298.0), P=np.full(C, 1013.25), jscale=np.ones(C), y0=flat.reshape(C, 3).T.copy())
        return m, c, 60.0
    if name == "adjoint10k":
        m = mech_medium()
        c = make_cells(m, n_cells or 10000, seed=1005)
        return m, c, 60.0
    raise KeyError(name)


def mixed_workload(n_cells: int = 100000):
    """The mixed batch: 20/30, 72/156 and 150/350 mechanisms with 30% / 50% /
    20% of n_cells, randomly interleaved (seed 1004), 60 s steps.

    Returns (groups, owner, dt): groups is a list of (mechanism, cells) with
    the cells of each mechanism in their interleaved order, and owner[g] the
    global indices of group g's cells in the interleaved batch."""
    mechs = [mech_small(), mech_medium(), mech_large()]
    counts = split_counts(n_cells, [30, 50, 20])
    rng = np.random.default_rng(1004)
    label = rng.permutation(np.repeat(np.arange(3), counts))
    groups, owner = [], []
    for g, m in enumerate(mechs):
        idx = np.flatnonzero(label == g)
        groups.append((m, make_cells(m, len(idx), seed=1004 + 10 * (g + 1))))
        owner.append(idx)
    return groups, owner, 60.0
