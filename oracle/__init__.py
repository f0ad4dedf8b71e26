"""CPU oracle for the multi-cell chemistry path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never does, and this package
imports nothing from it: the two share no code.  Inputs come from the seeded
generators as plain numpy arrays.

The arithmetic lives in oracle.c (plain C, double precision, one cell at a
time); this module only marshals numpy arrays through ctypes.  See oracle.c
for what is computed and which passages of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MCC_ORACLE_LIB: another build of the same source (e.g. one with sanitizers)
LIB_PATH = os.environ.get("MCC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

STATUS = {0: "OK", 1: "TOO_MUCH_WORK", 2: "CONV_FAIL", 3: "ERR_FAIL", 4: "NONFINITE", 5: "SINGULAR"}


def build(src: str = SRC_PATH, out: str = LIB_PATH, extra_flags=()) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", *extra_flags,
           "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Mech(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("rxn_type", ctypes.c_void_p), ("reac_ptr", ctypes.c_void_p),
                ("reac_idx", ctypes.c_void_p), ("prod_ptr", ctypes.c_void_p),
                ("prod_idx", ctypes.c_void_p), ("prod_yield", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("theta", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("eta_newton", ctypes.c_double), ("safety", ctypes.c_double),
                ("fac_min", ctypes.c_double), ("fac_max", ctypes.c_double),
                ("fac_newton_fail", ctypes.c_double), ("h_min_rel", ctypes.c_double),
                ("max_order", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("warm_start", ctypes.c_int32)]


STATS_DTYPE = np.dtype([("steps", np.int32), ("rejects", np.int32), ("newton_fails", np.int32),
                        ("newton_iters", np.int32), ("f_evals", np.int32), ("jac_evals", np.int32),
                        ("lu_count", np.int32), ("order", np.int32),
                        ("h_last", np.float64), ("y_min", np.float64), ("h_next", np.float64)])


def default_opts(rtol=1e-8, atol=1.0, **kw) -> Opts:
    """Solver constants: rtol 1e-8; atol 1 molecule cm^-3 (use ~1e-14 for O(1) tests)."""
    o = Opts(rtol=rtol, atol=atol, eta_newton=0.03, safety=0.9, fac_min=0.2, fac_max=10.0,
             fac_newton_fail=0.5, h_min_rel=1e-30, max_order=5, max_newton=4, max_steps=100000, warm_start=0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Tape:
    """An owned step tape of the oracle (freed with the object)."""

    def __init__(self, lib):
        self.lib = lib
        self.h = lib.orc_tape_new()

    def __len__(self):
        return int(self.lib.orc_tape_size(self.h))

    @classmethod
    def from_values(cls, lib, values):
        """A tape holding the given entries (recorded elsewhere)."""
        t = cls(lib)
        v = np.ascontiguousarray(values, dtype=np.float64)
        lib.orc_tape_assign(t.h, v.ctypes.data, len(v))
        return t

    def values(self):
        """A copy of the entries: type, order, value, then for a step the N
        state values."""
        n = len(self)
        if n == 0:
            return np.zeros(0)
        ptr = ctypes.cast(self.lib.orc_tape_data(self.h), ctypes.POINTER(ctypes.c_double))
        return np.ctypeslib.as_array(ptr, shape=(n,)).copy()

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_tape_free(self.h)
            self.h = None


class Oracle:
    """ctypes view of liboracle.so bound to one mechanism."""

    def __init__(self, mech, lib_path: str = LIB_PATH):
        if not os.path.exists(lib_path):
            build(out=lib_path)
        self.lib = ctypes.CDLL(lib_path)
        self.mech = mech
        self._keep = [np.ascontiguousarray(a, dtype=dt) for a, dt in (
            (mech.rxn_type, np.int32), (mech.reac_ptr, np.int32), (mech.reac_idx, np.int32),
            (mech.prod_ptr, np.int32), (mech.prod_idx, np.int32), (mech.prod_yield, np.float64),
            (mech.A, np.float64), (mech.theta, np.float64))]
        p = [a.ctypes.data for a in self._keep]
        self._m = _Mech(mech.n_species, mech.n_reactions, *p)
        i64, vp, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        L = self.lib
        L.orc_rate_constants.argtypes = [vp, i64, vp, vp, vp]
        L.orc_deriv.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_jac.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_vjp.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.orc_solve_multicell.argtypes = [vp, i64, vp, vp, dbl, vp, vp]
        L.orc_tape_new.restype = vp
        L.orc_tape_free.argtypes = [vp]
        L.orc_tape_size.argtypes = [vp]
        L.orc_tape_size.restype = i64
        L.orc_tape_data.argtypes = [vp]
        L.orc_tape_data.restype = vp
        L.orc_tape_assign.argtypes = [vp, vp, i64]
        L.orc_tape_assign.restype = None
        L.orc_cell_solve_taped.argtypes = [vp, vp, vp, dbl, vp, vp, vp]
        L.orc_cell_solve_taped.restype = ctypes.c_int
        L.orc_cell_replay.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_cell_replay.restype = ctypes.c_int
        L.orc_cell_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_solve_multicell.restype = ctypes.c_int
        L.orc_solve.argtypes = [vp, i64, vp, vp, dbl, vp, vp, vp, ctypes.c_int]
        L.orc_solve.restype = ctypes.c_int
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_rescale_differences.argtypes = [ctypes.c_int32, vp, ctypes.c_int32, dbl]
        L.orc_dense_solve.argtypes = [ctypes.c_int32, vp, vp]
        L.orc_dense_solve.restype = ctypes.c_int

    @property
    def N(self):
        return self.mech.n_species

    @property
    def R(self):
        return self.mech.n_reactions

    def _mp(self):
        return ctypes.addressof(self._m)

    def rate_constants(self, T, jscale) -> np.ndarray:
        T = np.ascontiguousarray(T, dtype=np.float64)
        s = np.ascontiguousarray(jscale, dtype=np.float64)
        C = T.shape[0]
        k = np.empty((self.R, C))
        self.lib.orc_rate_constants(self._mp(), C, T.ctypes.data, s.ctypes.data, k.ctypes.data)
        return k

    def deriv(self, k, y):
        """f and its absolute-value scale, both [N][C]."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        C = y.shape[1]
        f = np.empty((self.N, C))
        s = np.empty((self.N, C))
        self.lib.orc_deriv(self._mp(), C, k.ctypes.data, y.ctypes.data, f.ctypes.data, s.ctypes.data)
        return f, s

    def jac(self, k, y):
        """Dense J and its scale, both [C][N][N] (row = f index, column = y index)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        C = y.shape[1]
        J = np.empty((C, self.N, self.N))
        s = np.empty((C, self.N, self.N))
        self.lib.orc_jac(self._mp(), C, k.ctypes.data, y.ctypes.data, J.ctypes.data, s.ctypes.data)
        return J, s

    def vjp(self, k, y, v):
        """gy = J^T v [N][C] and glnk = d(v.f)/d ln k [R][C] (f is linear in k)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        C = y.shape[1]
        gy = np.empty((self.N, C))
        gk = np.empty((self.R, C))
        self.lib.orc_vjp(self._mp(), C, k.ctypes.data, y.ctypes.data, v.ctypes.data, gy.ctypes.data,
                         gk.ctypes.data)
        return gy, gk

    def solve(self, k, y0, dt, opts: Opts | None = None, n_threads: int = 0, h_warm=None):
        """One outer BDF step of length dt for every cell.  h_warm [C]: the
        first step sizes of a warm start (with opts.warm_start = 1).

        Returns (y [N][C], status [C] int32, stats structured array [C])."""
        if opts is None:
            opts = default_opts()
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.array(y0, dtype=np.float64, order="C", copy=True)
        C = y.shape[1]
        status = np.empty(C, dtype=np.int32)
        stats = np.zeros(C, dtype=STATS_DTYPE)
        if h_warm is not None:
            stats["h_next"] = np.asarray(h_warm, dtype=np.float64)
        self.lib.orc_solve(self._mp(), C, k.ctypes.data, y.ctypes.data, float(dt),
                           ctypes.addressof(opts), status.ctypes.data, stats.ctypes.data,
                           int(n_threads))
        return y, status, stats

    def solve_multicell(self, k, y0, dt, opts: Opts | None = None):
        """Multi-cells: all cells as one system (shared h and order, norms over
        all cells).  Returns (y, status, stats) with one status and one stats
        record for the whole system."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.array(y0, dtype=np.float64, order="C", copy=True)
        C = y.shape[1]
        stats = np.zeros(1, dtype=STATS_DTYPE)
        o = opts or default_opts()
        s = self.lib.orc_solve_multicell(self._mp(), C, k.ctypes.data, y.ctypes.data, float(dt),
                                         ctypes.addressof(o), stats.ctypes.data)
        return y, int(s), stats[0]

    # -- reverse mode through one outer step of one cell --------------------
    def solve_taped(self, k_cell, y0_cell, dt, opts: Opts | None = None, h_warm: float = 0.0):
        """One outer step of one cell (k [R], y0 [N]) recording its step
        tape (h_warm: the first step size of a warm start, with
        opts.warm_start = 1).  Returns (y, status, stats, tape)."""
        k = np.ascontiguousarray(k_cell, dtype=np.float64)
        y = np.array(y0_cell, dtype=np.float64, copy=True)
        st = np.zeros(1, dtype=STATS_DTYPE)
        st["h_next"] = h_warm
        tape = Tape(self.lib)
        o = opts or default_opts()
        s = self.lib.orc_cell_solve_taped(self._mp(), k.ctypes.data, y.ctypes.data, float(dt), ctypes.addressof(o),
                                          st.ctypes.data, tape.h)
        return y, int(s), st[0], tape

    def replay(self, k_cell, y0_cell, tape):
        """The tape's frozen step sequence run again with these k and y0
        (implicit steps solved to convergence).  Returns (y, replay tape)."""
        k = np.ascontiguousarray(k_cell, dtype=np.float64)
        y0 = np.ascontiguousarray(y0_cell, dtype=np.float64)
        y = np.empty_like(y0)
        out = Tape(self.lib)
        if self.lib.orc_cell_replay(self._mp(), k.ctypes.data, y0.ctypes.data, tape.h, y.ctypes.data, out.h):
            raise RuntimeError("replay: a Newton matrix is singular")
        return y, out

    def adjoint(self, k_cell, y0_cell, replay_tape, lam_y):
        """Discrete adjoint of a replayed tape: (dL/dy0 [N], dL/d ln k [R])
        for dL/dy(dt) = lam_y."""
        k = np.ascontiguousarray(k_cell, dtype=np.float64)
        y0 = np.ascontiguousarray(y0_cell, dtype=np.float64)
        lam = np.array(lam_y, dtype=np.float64, copy=True)
        g = np.empty(self.R)
        self.lib.orc_cell_adjoint(self._mp(), k.ctypes.data, y0.ctypes.data, replay_tape.h, lam.ctypes.data,
                                  g.ctypes.data)
        return lam, g

    def rescale_differences(self, D, order, rho):
        """Backward differences D [order+1][N] re-sampled at spacing rho*h."""
        D = np.array(D, dtype=np.float64, order="C", copy=True)
        self.lib.orc_rescale_differences(D.shape[1], D.ctypes.data, int(order), float(rho))
        return D

    def dense_solve(self, a, b):
        """x with a x = b by Gaussian elimination with partial pivoting (None if singular)."""
        a = np.array(a, dtype=np.float64, order="C", copy=True)
        x = np.array(b, dtype=np.float64, order="C", copy=True)
        if self.lib.orc_dense_solve(a.shape[0], a.ctypes.data, x.ctypes.data):
            return None
        return x

    def max_threads(self) -> int:
        return int(self.lib.orc_max_threads())


class Controller:
    """ctypes view of the oracle's step-size controller (no mechanism): the
    starting step's two stages, the factor after a failed error test and the
    order and step-size selection, exactly as both the per-cell and the
    Multi-cells solves call them."""

    def __init__(self, lib_path: str = LIB_PATH):
        if not os.path.exists(lib_path):
            build(out=lib_path)
        self.lib = L = ctypes.CDLL(lib_path)
        vp, dbl, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32
        L.orc_start_h0.argtypes = [i32, vp, vp, vp, dbl]
        L.orc_start_h0.restype = dbl
        L.orc_start_h.argtypes = [i32, vp, vp, vp, dbl, dbl]
        L.orc_start_h.restype = dbl
        L.orc_reject_factor.argtypes = [dbl, i32, dbl, dbl]
        L.orc_reject_factor.restype = dbl
        L.orc_select_order.argtypes = [i32, vp, vp, i32, i32, dbl, dbl, dbl, vp]
        L.orc_select_order.restype = dbl

    @staticmethod
    def _vec(v):
        return np.ascontiguousarray(v, dtype=np.float64)

    def start_h0(self, y0, f0, w, dt) -> float:
        y0, f0, w = self._vec(y0), self._vec(f0), self._vec(w)
        return float(self.lib.orc_start_h0(len(y0), y0.ctypes.data, f0.ctypes.data, w.ctypes.data, float(dt)))

    def start_h(self, f0, f1, w, h0, dt) -> float:
        f0, f1, w = self._vec(f0), self._vec(f1), self._vec(w)
        return float(self.lib.orc_start_h(len(f0), f0.ctypes.data, f1.ctypes.data, w.ctypes.data, float(h0),
                                          float(dt)))

    def reject_factor(self, err_norm, order, safety=0.9, fac_min=0.2) -> float:
        return float(self.lib.orc_reject_factor(float(err_norm), int(order), float(safety), float(fac_min)))

    def select_order(self, D, w, order, max_order, err_norm, safety=0.9, fac_max=10.0):
        """D: difference table [order+3][n].  Returns (factor, new order)."""
        D, w = self._vec(D), self._vec(w)
        assert D.ndim == 2 and D.shape[0] >= order + 3 and D.shape[1] == len(w)
        k = ctypes.c_int32(0)
        fac = self.lib.orc_select_order(D.shape[1], D.ctypes.data, w.ctypes.data, int(order), int(max_order),
                                        float(err_norm), float(safety), float(fac_max), ctypes.byref(k))
        return float(fac), int(k.value)
