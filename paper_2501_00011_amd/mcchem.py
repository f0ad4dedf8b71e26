"""Thin Python binding of libmcchem (include/mcc.h) over PyTorch device tensors.

Argument marshalling only: every rate constant, f, J and solver step is
computed by the HIP kernels in libmcchem.so.  There is no CPU fallback; if the
library is missing or no GPU is present, construction raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcchem.so")

CELL_STATUS = {0: "OK", 1: "TOO_MUCH_WORK", 2: "CONV_FAIL", 3: "ERR_FAIL", 4: "NONFINITE", 5: "SINGULAR",
               6: "BAD_TAPE"}
CELL_OK, CELL_SINGULAR, CELL_BAD_TAPE = 0, 5, 6

STATS_DTYPE = np.dtype([("steps", np.int32), ("rejects", np.int32), ("newton_fails", np.int32),
                        ("newton_iters", np.int32), ("f_evals", np.int32), ("jac_evals", np.int32),
                        ("lu_count", np.int32), ("order", np.int32),
                        ("h_last", np.float64), ("y_min", np.float64), ("h_next", np.float64)])
assert STATS_DTYPE.itemsize == 56


class MccError(RuntimeError):
    pass


class SolverOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("eta_newton", ctypes.c_double),
                ("safety", ctypes.c_double), ("fac_min", ctypes.c_double), ("fac_max", ctypes.c_double),
                ("fac_newton_fail", ctypes.c_double), ("h_min_rel", ctypes.c_double),
                ("max_order", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32),
                ("warm_start", ctypes.c_int32)]


class _MechDesc(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("rxn_type", ctypes.c_void_p), ("reac_ptr", ctypes.c_void_p),
                ("reac_idx", ctypes.c_void_p), ("prod_ptr", ctypes.c_void_p),
                ("prod_idx", ctypes.c_void_p), ("prod_yield", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("theta", ctypes.c_void_p)]


_lib = None


def library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmcchem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime then satisfies the library's libamdhip64.so.7
    # dependency, so tensors and kernels share one runtime.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise MccError(f"{path} is missing: build it with `python -m paper_2501_00011_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pi32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "mcc_last_error": ([], ctypes.c_char_p),
        "mcc_version": ([], ctypes.c_char_p),
        "mcc_solver_opts_default": ([vp], ctypes.c_int),
        "mcc_mech_create": ([vp, ctypes.c_int, vp], ctypes.c_int),
        "mcc_mech_create_ex": ([vp, ctypes.c_int, vp, vp], ctypes.c_int),
        "mcc_mech_config_default": ([vp], ctypes.c_int),
        "mcc_mech_info": ([vp, pi32, pi32, pi32, pi32, pi32], ctypes.c_int),
        "mcc_mech_jac_pattern": ([vp, vp, vp], ctypes.c_int),
        "mcc_mech_op_counts": ([vp, vp], ctypes.c_int),
        "mcc_debug_emulate_cell": ([vp, vp, vp, dbl, vp, vp, vp, vp], ctypes.c_int),
        "mcc_debug_schedule_info": ([vp, vp], ctypes.c_int),
        "mcc_debug_emulate_fj": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mcc_debug_emulate_vjp": ([vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mcc_debug_emulate_cell_adjoint": ([vp, vp, vp, dbl, vp, vp, vp, vp], ctypes.c_int),
        "mcc_mech_set_fj_kernel": ([vp, ctypes.c_int32], ctypes.c_int),
        "mcc_calc_vjp": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mcc_adjoint_step": ([vp, vp, vp, vp, i64, vp, vp, i32, vp, vp], ctypes.c_int),
        "mcc_solve_step_taped": ([vp, vp, dbl, vp, vp, vp, vp, vp, i64, vp], ctypes.c_int),
        "mcc_replay_step": ([vp, vp, vp, vp, i64, vp, i32, dbl, vp, vp], ctypes.c_int),
        "mcc_cells_set_schedule": ([vp, vp], ctypes.c_int),
        "mcc_cells_schedule_from_stats": ([vp, vp, vp], ctypes.c_int),
        "mcc_cells_schedule_from_stats_ex": ([vp, vp, i32, vp], ctypes.c_int),
        "mcc_solve_step_multicell": ([vp, vp, dbl, vp, vp, vp, vp], ctypes.c_int),
        "mcc_solve_step_multicell_noalloc": ([vp, vp, dbl, vp, vp, vp, vp], ctypes.c_int),
        "mcc_ablation_paper_deriv": ([vp, i64, vp, vp, vp, i32, vp], ctypes.c_int),
        "mcc_cells_set_rate_constants": ([vp, vp, vp], ctypes.c_int),
        "mcc_debug_fj_source": ([vp, vp, i64, vp], ctypes.c_int),
        "mcc_debug_compile_fj": ([vp, ctypes.c_char_p, vp], ctypes.c_int),
        "mcc_mech_destroy": ([vp], ctypes.c_int),
        "mcc_cells_create": ([vp, i64, i64, vp], ctypes.c_int),
        "mcc_cells_bind": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "mcc_cells_rate_constants": ([vp, vp], ctypes.c_int),
        "mcc_calc_deriv": ([vp, vp, vp, vp], ctypes.c_int),
        "mcc_calc_jac": ([vp, vp, vp, vp], ctypes.c_int),
        "mcc_calc_deriv_jac": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "mcc_solve_step": ([vp, vp, dbl, vp, vp, vp, vp], ctypes.c_int),
        "mcc_sync": ([vp], ctypes.c_int),
        "mcc_cells_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _ = i32
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        msg = library().mcc_last_error().decode()
        raise MccError(f"mcc status {status}: {msg}")


def default_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    _check(library().mcc_solver_opts_default(ctypes.addressof(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, what, dtype=None, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise MccError(f"{what} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise MccError(f"{what} must have dtype {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise MccError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise MccError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Mechanism:
    """A compiled mechanism resident on one GPU (mcc_mech_create)."""

    def __init__(self, mech, device: int = 0, dense_tail: int = -1, waves_per_simd: int = 0):
        L = library()
        self.source = mech
        arrays = [np.ascontiguousarray(a, dtype=dt) for a, dt in (
            (mech.rxn_type, np.int32), (mech.reac_ptr, np.int32), (mech.reac_idx, np.int32),
            (mech.prod_ptr, np.int32), (mech.prod_idx, np.int32), (mech.prod_yield, np.float64),
            (mech.A, np.float64), (mech.theta, np.float64))]
        desc = _MechDesc(int(mech.n_species), int(mech.n_reactions), *[a.ctypes.data for a in arrays])
        h = ctypes.c_void_p()
        cfg = (ctypes.c_int32 * 8)()
        _check(L.mcc_mech_config_default(ctypes.addressof(cfg)))
        cfg[0] = int(dense_tail)
        cfg[1] = int(waves_per_simd)
        _check(L.mcc_mech_create_ex(ctypes.addressof(desc), int(device), ctypes.addressof(cfg), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        n, r, nnz, lu, lds = (ctypes.c_int32() for _ in range(5))
        _check(L.mcc_mech_info(h, ctypes.byref(n), ctypes.byref(r), ctypes.byref(nnz),
                               ctypes.byref(lu), ctypes.byref(lds)))
        self.n_species, self.n_reactions = n.value, r.value
        self.nnz, self.lu_nnz, self.solver_lds_bytes = nnz.value, lu.value, lds.value

    def op_counts(self) -> dict:
        """Algorithmic flops and HBM bytes per cell (mcc_mech_op_counts)."""
        buf = (ctypes.c_int64 * 8)()
        _check(library().mcc_mech_op_counts(self._h, ctypes.addressof(buf)))
        names = ["deriv_flops", "newton_matrix_flops", "lu_flops", "solve_flops",
                 "fj_bytes", "f_bytes", "j_bytes"]
        return dict(zip(names, list(buf)[:7]))

    def emulate_cell(self, k, y, c, b, transposed: bool = False):
        """Host emulation of the solver phases for one cell (testing aid):
        returns (f, x = (I - c J)^-1 b, violations), or with transposed the
        solve with (I - c J)^T by the reverse-mode tables."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        f = np.zeros(self.n_species)
        x = np.zeros(self.n_species)
        v = ctypes.c_int32()
        fn = library().mcc_debug_emulate_cell_adjoint if transposed else library().mcc_debug_emulate_cell
        _check(fn(self._h, k.ctypes.data, y.ctypes.data, float(c), b.ctypes.data, f.ctypes.data, x.ctypes.data,
                  ctypes.byref(v)))
        return f, x, v.value

    def emulate_fj(self, k, y):
        """Host emulation of the f/J kernel's tables for one cell (testing
        aid): returns (f, J nonzeros in CSR order, violations)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(self.n_species)
        J = np.zeros(max(self.nnz, 1))
        v = ctypes.c_int32()
        _check(library().mcc_debug_emulate_fj(self._h, k.ctypes.data, y.ctypes.data, f.ctypes.data,
                                              J.ctypes.data, ctypes.byref(v)))
        return f, J[:self.nnz], v.value

    def emulate_vjp(self, k, y, v):
        """Host emulation of the generated VJP kernel's work items for one
        cell (testing aid): returns (gy = J^T v, glnk = d(v.f)/d ln k,
        violations)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        gy = np.zeros(self.n_species)
        glnk = np.zeros(max(self.n_reactions, 1))
        n = ctypes.c_int32()
        _check(library().mcc_debug_emulate_vjp(self._h, k.ctypes.data, y.ctypes.data, v.ctypes.data, gy.ctypes.data,
                                               glnk.ctypes.data, ctypes.byref(n)))
        return gy, glnk[:self.n_reactions], n.value

    FJ_GENERATED, FJ_TABLES = 0, 1

    def set_fj_kernel(self, kind: int):
        """Choose the f/J kernel: FJ_GENERATED (default) or FJ_TABLES."""
        _check(library().mcc_mech_set_fj_kernel(self._h, int(kind)))

    def fj_source(self) -> str:
        """The generated f/J kernel source (testing aid)."""
        n = ctypes.c_int64()
        _check(library().mcc_debug_fj_source(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(library().mcc_debug_fj_source(self._h, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def compile_fj(self, arch: str = "gfx950") -> int:
        """Compile the generated f/J kernel with hipRTC (no GPU needed); code bytes."""
        n = ctypes.c_int64()
        _check(library().mcc_debug_compile_fj(self._h, arch.encode(), ctypes.byref(n)))
        return n.value

    def paper_deriv(self, y_cm, k_cm, f_cm=None, inverted=False, stream=None):
        """Ablation: the paper's Derivative kernel on cell-major arrays
        y [C][N], k [C][R] -> f [C][N] (device float64)."""
        import torch
        C = y_cm.shape[0]
        if f_cm is None:
            f_cm = torch.empty_like(y_cm)
        _check(library().mcc_ablation_paper_deriv(
            self._h, C, _dptr(y_cm, "y", torch.float64, (C, self.n_species)),
            _dptr(k_cm, "k", torch.float64, (C, self.n_reactions)),
            _dptr(f_cm, "f", torch.float64, (C, self.n_species)), int(bool(inverted)), _stream_ptr(stream)))
        return f_cm

    def schedule_info(self) -> dict:
        """Sizes of the solver schedule (testing aid)."""
        buf = (ctypes.c_int64 * 16)()
        _check(library().mcc_debug_schedule_info(self._h, ctypes.addressof(buf)))
        v = list(buf)
        return {"lu_blocks": v[0], "lu_levels": v[1], "nm_blocks": v[2], "fg_blocks": v[3:7],
                "dense_tail": v[7], "waves_per_simd": v[8]}

    def jac_pattern(self):
        rp = np.zeros(self.n_species + 1, dtype=np.int32)
        ci = np.zeros(max(self.nnz, 1), dtype=np.int32)
        _check(library().mcc_mech_jac_pattern(self._h, rp.ctypes.data, ci.ctypes.data))
        return rp, ci[:self.nnz]

    def close(self):
        if getattr(self, "_h", None):
            _check(library().mcc_mech_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                library().mcc_mech_destroy(self._h)
        except Exception:
            pass


class Cells:
    """A batch of cells of one mechanism (mcc_cells_create); arrays are
    float64 device tensors laid out [entity][ld], cell index fastest."""

    def __init__(self, mech: Mechanism, n_cells: int, ld: int | None = None):
        self.mech = mech
        self.n_cells = int(n_cells)
        self.ld = int(ld) if ld is not None else self.n_cells
        h = ctypes.c_void_p()
        _check(library().mcc_cells_create(mech._h, self.n_cells, self.ld, ctypes.byref(h)))
        self._h = h

    def bind(self, T, P=None, jscale=None, stream=None):
        import torch
        f64 = torch.float64
        shape = (self.n_cells,)
        tp = _dptr(T, "T", f64, shape)
        pp = _dptr(P, "P", f64, shape) if P is not None else None
        sp = _dptr(jscale, "jscale", f64, shape) if jscale is not None else None
        _check(library().mcc_cells_bind(self._h, tp, pp, sp, _stream_ptr(stream)))

    def rate_constants(self):
        """Copy of the rate constants [R][ld] as a device tensor."""
        import torch
        k = ctypes.c_void_p()
        _check(library().mcc_cells_rate_constants(self._h, ctypes.byref(k)))
        out = torch.empty((self.mech.n_reactions, self.ld), dtype=torch.float64,
                          device=f"cuda:{self.mech.device}")
        if out.numel():
            import ctypes as _c
            torch.cuda.synchronize()
            hip = _hip_runtime()
            _check_hip(hip.hipMemcpy(_c.c_void_p(out.data_ptr()), k, out.numel() * 8, 3))
        return out

    def _yshape(self):
        return (self.mech.n_species, self.ld)

    def deriv(self, y, f=None, stream=None):
        import torch
        if f is None:
            f = torch.empty(self._yshape(), dtype=torch.float64, device=y.device)
        _check(library().mcc_calc_deriv(self._h, _dptr(y, "y", torch.float64, self._yshape()),
                                        _dptr(f, "f", torch.float64, self._yshape()), _stream_ptr(stream)))
        return f

    def jac(self, y, jac=None, stream=None):
        import torch
        shape = (self.mech.nnz, self.ld)
        if jac is None:
            jac = torch.empty(shape, dtype=torch.float64, device=y.device)
        _check(library().mcc_calc_jac(self._h, _dptr(y, "y", torch.float64, self._yshape()),
                                      _dptr(jac, "jac", torch.float64, shape), _stream_ptr(stream)))
        return jac

    def deriv_jac(self, y, f=None, jac=None, stream=None):
        import torch
        shape = (self.mech.nnz, self.ld)
        if f is None:
            f = torch.empty(self._yshape(), dtype=torch.float64, device=y.device)
        if jac is None:
            jac = torch.empty(shape, dtype=torch.float64, device=y.device)
        _check(library().mcc_calc_deriv_jac(self._h, _dptr(y, "y", torch.float64, self._yshape()),
                                            _dptr(f, "f", torch.float64, self._yshape()),
                                            _dptr(jac, "jac", torch.float64, shape), _stream_ptr(stream)))
        return f, jac

    def vjp(self, y, v, gy=None, glnk=None, want_gy=True, want_glnk=True, stream=None):
        """gy = J^T v [N][ld] and glnk = d(v.f)/d ln k [R][ld] at y."""
        import torch
        if want_gy and gy is None:
            gy = torch.empty(self._yshape(), dtype=torch.float64, device=y.device)
        if want_glnk and glnk is None:
            glnk = torch.empty((self.mech.n_reactions, self.ld), dtype=torch.float64, device=y.device)
        _check(library().mcc_calc_vjp(
            self._h, _dptr(y, "y", torch.float64, self._yshape()), _dptr(v, "v", torch.float64, self._yshape()),
            _dptr(gy, "gy", torch.float64, self._yshape()) if gy is not None else None,
            _dptr(glnk, "glnk", torch.float64, (self.mech.n_reactions, self.ld)) if glnk is not None else None,
            _stream_ptr(stream)))
        return gy, glnk

    def adjoint_step(self, y0, tape, tape_len, lam, glnk=None, accumulate=False, status=None, stream=None):
        """Reverse mode of one outer step: lam (dL/dy(dt), [N][ld]) is
        overwritten with dL/dy0; dL/d ln k [R][ld] is written to (or, with
        accumulate, added to) glnk.  tape: device float64 [n_cells][stride]
        in the entry format of mcc_adjoint_step, tape_len: int64 [n_cells].
        Returns (glnk, status)."""
        import torch
        if glnk is None:
            glnk = torch.zeros((self.mech.n_reactions, self.ld), dtype=torch.float64, device=lam.device)
        if status is None:
            status = torch.empty(self.n_cells, dtype=torch.int32, device=lam.device)
        if tape.dim() != 2 or tape.shape[0] != self.n_cells:
            raise ValueError(f"tape must be [n_cells={self.n_cells}][stride]")
        stride = int(tape.shape[1])
        _check(library().mcc_adjoint_step(
            self._h, _dptr(y0, "y0", torch.float64, self._yshape()),
            _dptr(tape, "tape", torch.float64, (self.n_cells, stride)),
            _dptr(tape_len, "tape_len", torch.int64, (self.n_cells,)), stride,
            _dptr(lam, "lam", torch.float64, self._yshape()),
            _dptr(glnk, "glnk", torch.float64, (self.mech.n_reactions, self.ld)), 1 if accumulate else 0,
            _dptr(status, "status", torch.int32, (self.n_cells,)), _stream_ptr(stream)))
        return glnk, status

    def replay_step(self, y0, tape, tape_len, y=None, max_newton=50, tol=1e-15, status=None, stream=None):
        """The tapes' frozen step sequences run again from y0 with the
        current rate constants (Newton to convergence at every step).
        Returns (y, status)."""
        import torch
        if y is None:
            y = torch.empty_like(y0)
        if status is None:
            status = torch.empty(self.n_cells, dtype=torch.int32, device=y0.device)
        if tape.dim() != 2 or tape.shape[0] != self.n_cells:
            raise ValueError(f"tape must be [n_cells={self.n_cells}][stride]")
        stride = int(tape.shape[1])
        _check(library().mcc_replay_step(
            self._h, _dptr(y0, "y0", torch.float64, self._yshape()),
            _dptr(tape, "tape", torch.float64, (self.n_cells, stride)),
            _dptr(tape_len, "tape_len", torch.int64, (self.n_cells,)), stride,
            _dptr(y, "y", torch.float64, self._yshape()), int(max_newton), float(tol),
            _dptr(status, "status", torch.int32, (self.n_cells,)), _stream_ptr(stream)))
        return y, status

    def set_schedule(self, order=None):
        """Workgroup i of the per-cell solver kernels integrates cell
        order[i] (host int32 permutation of the cells); None: the identity."""
        if order is None:
            _check(library().mcc_cells_set_schedule(self._h, None))
            return
        o = np.ascontiguousarray(order, dtype=np.int32)
        if o.shape != (self.n_cells,):
            raise MccError(f"order must have shape ({self.n_cells},)")
        _check(library().mcc_cells_set_schedule(self._h, o.ctypes.data))

    SCHEDULES = {"longest": 0, "zigzag": 1}

    def balance(self, stats, kind: str = "longest"):
        """Schedule the cells by their step attempts in stats (device
        counters of a previous outer step; mcc_cells_schedule_from_stats_ex):
        "longest" first, or "zigzag" (longest, shortest, second longest, ...).
        Returns the order."""
        import torch
        order = np.empty(self.n_cells, dtype=np.int32)
        _check(library().mcc_cells_schedule_from_stats_ex(
            self._h, _dptr(stats, "stats", torch.uint8, (self.n_cells, STATS_DTYPE.itemsize)),
            self.SCHEDULES[kind], order.ctypes.data))
        return order

    def set_rate_constants(self, k, stream=None):
        """Use caller rate constants k [R][ld] (device float64) instead of bind()'s."""
        import torch
        _check(library().mcc_cells_set_rate_constants(
            self._h, _dptr(k, "k", torch.float64, (self.mech.n_reactions, self.ld)), _stream_ptr(stream)))

    def step(self, y, dt, opts: SolverOpts | None = None, status=None, stats=None, want_stats=True,
             stream=None):
        """One outer step of length dt in place on y.  Returns (status, stats)
        device tensors: int32 [n_cells] and uint8 [n_cells, 56] (see stats_numpy).
        With opts.warm_start, stats must be the previous step's counters."""
        import torch
        if status is None:
            status = torch.empty(self.n_cells, dtype=torch.int32, device=y.device)
        if want_stats and stats is None:
            stats = torch.empty((self.n_cells, STATS_DTYPE.itemsize), dtype=torch.uint8, device=y.device)
        op = ctypes.addressof(opts) if opts is not None else None
        sp = _dptr(stats, "stats", torch.uint8, (self.n_cells, STATS_DTYPE.itemsize)) if stats is not None else None
        _check(library().mcc_solve_step(self._h, _dptr(y, "y", torch.float64, self._yshape()), float(dt), op,
                                        _dptr(status, "status", torch.int32, (self.n_cells,)), sp,
                                        _stream_ptr(stream)))
        return status, stats

    def step_taped(self, y, dt, tape, tape_len, opts: SolverOpts | None = None, status=None, stats=None,
                   stream=None):
        """step() recording each cell's step tape for adjoint_step: tape
        float64 [n_cells][stride], tape_len int64 [n_cells] (-1: did not fit)."""
        import torch
        if status is None:
            status = torch.empty(self.n_cells, dtype=torch.int32, device=y.device)
        if tape.dim() != 2 or tape.shape[0] != self.n_cells:
            raise ValueError(f"tape must be [n_cells={self.n_cells}][stride]")
        stride = int(tape.shape[1])
        op = ctypes.addressof(opts) if opts is not None else None
        sp = _dptr(stats, "stats", torch.uint8, (self.n_cells, STATS_DTYPE.itemsize)) if stats is not None else None
        _check(library().mcc_solve_step_taped(
            self._h, _dptr(y, "y", torch.float64, self._yshape()), float(dt), op,
            _dptr(status, "status", torch.int32, (self.n_cells,)), sp,
            _dptr(tape, "tape", torch.float64, (self.n_cells, stride)),
            _dptr(tape_len, "tape_len", torch.int64, (self.n_cells,)), stride, _stream_ptr(stream)))
        return status, stats

    def step_multicell(self, y, dt, opts: SolverOpts | None = None, status=None, stats=None, stream=None,
                       noalloc: bool = False):
        """The Multi-cells outer step: all cells as one system (shared h and
        order).  noalloc: the entry point that allocates nothing (static
        reduction slots shared by every call on the device)."""
        import torch
        if status is None:
            status = torch.empty(self.n_cells, dtype=torch.int32, device=y.device)
        if stats is None:
            stats = torch.empty((self.n_cells, STATS_DTYPE.itemsize), dtype=torch.uint8, device=y.device)
        op = ctypes.addressof(opts) if opts is not None else None
        fn = library().mcc_solve_step_multicell_noalloc if noalloc else library().mcc_solve_step_multicell
        _check(fn(
            self._h, _dptr(y, "y", torch.float64, self._yshape()), float(dt), op,
            _dptr(status, "status", torch.int32, (self.n_cells,)),
            _dptr(stats, "stats", torch.uint8, (self.n_cells, STATS_DTYPE.itemsize)), _stream_ptr(stream)))
        return status, stats

    def sync(self):
        _check(library().mcc_sync(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _check(library().mcc_cells_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                library().mcc_cells_destroy(self._h)
        except Exception:
            pass


def stats_numpy(stats) -> np.ndarray:
    """Device stats buffer -> structured numpy array (fields of mcc_cell_stats)."""
    raw = stats.cpu().numpy()
    return raw.reshape(-1).view(STATS_DTYPE)


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        library()
        _hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime already loaded with torch
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def _check_hip(e):
    if e != 0:
        raise MccError(f"hipMemcpy failed with {e}")


def autotune_solver(mech, cells, dt: float, opts: SolverOpts | None = None, device: int = 0,
                    candidates=(0, 32, 48, 64), waves=(0, 1), schedules=("identity", "longest", "zigzag"),
                    reps: int = 2):
    """Pick the solver build and the cell schedule for `mech` by measurement.
    Every admissible combination of dense-tail size (`candidates`) and
    register budget (`waves`: 0 the library's choice, 1 one wavefront per
    SIMD) is compiled; for each, one outer step of the sample `cells` (a
    synth.Cells) runs untimed to produce per-cell counters, then one timed
    step per schedule (`schedules`: the identity, longest first by those
    counters, zigzag) with HIP events, best of `reps`.  The choices change
    how many cells a compute unit holds and in which order the dispatcher
    starts them, so the sample should fill the device several times over
    (several thousand cells).  Returns (Mechanism of the fastest build,
    {"tail/waves/schedule": ms}, the fastest (tail, waves, schedule))."""
    import torch
    dev = torch.device(f"cuda:{device}")
    T = torch.from_numpy(np.ascontiguousarray(cells.T)).to(dev)
    P = torch.from_numpy(np.ascontiguousarray(cells.P)).to(dev)
    s = torch.from_numpy(np.ascontiguousarray(cells.jscale)).to(dev)
    y0 = torch.from_numpy(np.ascontiguousarray(cells.y0)).to(dev)
    times, best = {}, None
    for m_tail in candidates:
        if m_tail > mech.n_species:
            continue
        for w in waves:
            try:
                h = Mechanism(mech, device=device, dense_tail=m_tail, waves_per_simd=w)
            except MccError:
                continue  # this choice does not fit the solver's register slots or LDS, or has no build
            w_eff = h.schedule_info()["waves_per_simd"]
            if any(k[0] == m_tail and k[1] == w_eff for k in times):
                h.close()
                continue  # the same build as the library's choice
            c = Cells(h, cells.n_cells)
            c.bind(T, P, s)
            y = y0.clone()
            _, stats = c.step(y, dt, opts)  # untimed: the counters the schedules are made from
            torch.cuda.synchronize()
            for sched in schedules:
                if sched == "identity":
                    c.set_schedule(None)
                else:
                    c.balance(stats, sched)
                ts = []
                for _ in range(reps):
                    y.copy_(y0)
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    c.step(y, dt, opts)
                    b.record()
                    torch.cuda.synchronize()
                    ts.append(a.elapsed_time(b))
                times[(m_tail, w_eff, sched)] = min(ts)
            c.close()
            fastest = min((k for k in times if k[0] == m_tail and k[1] == w_eff), key=times.get)
            if best is None or times[fastest] < times[best[0]]:
                if best is not None:
                    best[1].close()
                best = (fastest, h)
            else:
                h.close()
    if best is None:
        raise MccError("no solver build compiles for this mechanism")
    return best[1], {f"{k[0]}/{k[1]}/{k[2]}": v for k, v in times.items()}, best[0]
