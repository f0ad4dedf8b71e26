"""Benchmark: one step = the whole hot path over one batch of synthetic cells.

Step (all on cuda:0, inputs resident in HBM):
  1. rate constants from T, P and the photolysis scale (mcc_cells_bind),
  2. fused f and sparse J at the initial state (mcc_calc_deriv_jac),
  3. one 180 s BDF outer step of every cell (mcc_solve_step), restarted from
     the same initial state each step (a device-to-device copy).
Workload: 72 species / 156 reactions (47 photolysis, 94 bimolecular,
15 termolecular), 10,000 cells, T 220-310 K, P 100-1013 hPa, FP64.

Prints one JSON line: cell-timesteps/s with a roofline object for the
dominant kernel (the BDF solver, FP64 ALU-bound) and for the f+J kernel
(HBM-bound), and the CPU oracle timed on a bounded sample of the same cells.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
# vector-issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one 64-wide instruction per SIMD every 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wavefront-instructions/s


SOLVE_SOURCES = ["paper_2501_00011_amd/csrc/kernels_solve.hip", "paper_2501_00011_amd/csrc/mcc_internal.hpp",
                 "paper_2501_00011_amd/csrc/mech_compile.cpp"]
FJ_SOURCES = ["paper_2501_00011_amd/csrc/fj_codegen.cpp", "paper_2501_00011_amd/csrc/mcc_internal.hpp",
              "paper_2501_00011_amd/csrc/mech_compile.cpp", "paper_2501_00011_amd/csrc/api.hip"]
FJ_KERNEL = "mcc_fj_generated2"  # the two-cell variant (even leading dimension)
VJP_KERNEL = "mcc_vjp_generated2"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_medium10k.txt")


def measured_counter(kernel, sources, key="traffic_bytes"):
    """A per-launch figure measured with rocprofv3 counters for this workload
    (HBM bytes, or the solver's vector instructions), or None when the
    kernel's sources changed since the measurement."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec.get(key) if h.hexdigest()[:16] == rec["source_sha256_16"] else None


def measured_traffic(kernel, sources, n_cells=10000):
    """HBM bytes per launch of a generated kernel, measured at 10,000 cells
    (key: the kernel's name) or at another size (key: name@cells)."""
    return measured_counter(kernel if n_cells == 10000 else f"{kernel}@{n_cells}", sources, "traffic_bytes")


def solver_counter(key, n_cells, dense_tail):
    """A counter figure of the solver launch, only for the configuration it
    was measured in (10,000 cells, the recorded dense-tail size)."""
    if n_cells != 10000 or measured_counter("bdf_kernel", SOLVE_SOURCES, "dense_tail") != dense_tail:
        return None
    return measured_counter("bdf_kernel", SOLVE_SOURCES, key)


def issue_roofline(launch_s, n_cells, dense_tail):
    """The solver launch against the vector-issue peak: its vector
    instructions (SQ_INSTS_VALU, measured for this workload with the
    scheduled build) per launch time, or None when not measured for the
    current sources or this configuration."""
    insts = solver_counter("valu_instructions", n_cells, dense_tail)
    if insts is None:
        return None
    achieved = insts / launch_s
    return {"achieved": achieved, "peak": VALU_ISSUE_PEAK, "unit": "wavefront-instructions/s",
            "frac": achieved / VALU_ISSUE_PEAK, "instructions_per_launch": insts}


def per_launch_state(sn, K, n_species, mech):
    """HBM bytes the per-launch form moves for the solver state in one outer
    step: a cell takes part in about L = ceil(steps / K) launches, writes
    its state (backward differences [8][NS x 64] and 16 scalars, doubles)
    at the end of all but the last and reads it at the start of all but the
    first.  None for one launch."""
    if K <= 0:
        return None
    import numpy as np
    ns = len([b for b in mech.schedule_info()["fg_blocks"] if b > 0]) or 1
    state_bytes = 8 * (8 * ns * 64 + 16)
    launches = np.ceil(sn["steps"].astype(np.float64) / K)
    return {"state_bytes_per_cell": state_bytes, "launches_max": int(launches.max()),
            "bytes_per_outer_step": float(2 * state_bytes * np.maximum(launches - 1, 0).sum())}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium10k")
    ap.add_argument("--cells", type=int, default=None, help="override the number of cells")
    ap.add_argument("--fj-reps", type=int, default=100, help="extra timed f+J launches for its roofline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target wall time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--steps-per-launch", type=int, default=0,
                    help="0: each outer step in one launch (default); K > 0: the per-launch form, at most K "
                         "accepted BDF steps per launch with the solver state in HBM between launches")
    ap.add_argument("--multicell", action="store_true",
                    help="the paper's Multi-cells mode: all cells one system with a shared step size "
                         "(the batch must fit on the device at once)")
    ap.add_argument("--dense-tail", type=int, default=None,
                    help="compile the solver with this dense-tail size (0, 32, 48, 64) instead of autotuning")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the compiler's dense-tail choice instead of timing each choice on the first "
                         "8,192 cells (untimed, before the warm-up)")
    ap.add_argument("--ablation", action="store_true",
                    help="time the paper's Derivative kernel (thread per reaction, atomic adds; record and "
                         "inverted reaction data; with and without per-call host-device copies) beside "
                         "this library's f kernel, and exit")
    ap.add_argument("--adjoint", action="store_true",
                    help="reverse mode of the outer step: taped forward solve + adjoint kernel (one JSON line "
                         "with their times beside the plain solve)")
    ap.add_argument("--gradient", action="store_true",
                    help="gradient of the log loss with respect to log A over 10 x 60 s outer steps "
                         "(checkpointed forward + reverse mode; one JSON line)")
    ap.add_argument("--fd-params", type=int, default=4,
                    help="with --gradient: parameters checked against central differences (h = 1e-6) of the "
                         "frozen step sequences replayed on the GPU")
    ap.add_argument("--window", type=int, default=10,
                    help="mixed100k: consecutive outer steps captured in the replayed graph")
    ap.add_argument("--consecutive", type=int, default=5,
                    help="after the timed steps, this many consecutive outer steps with y advancing and the "
                         "cells scheduled longest first by the previous step's counters, cold and warm started "
                         "(reported beside the headline; 0: skip)")
    ap.add_argument("--no-balance", action="store_true",
                    help="keep the identity cell schedule (no longest-first ordering from the previous step)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three device-to-device copies of 1 GiB (the reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    return ap.parse_args()


def calibrate_copy():
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 3}))


def cpu_baseline(m, c, dt, target_s, y_gpu=None, atol=1.0):
    """The oracle as it stands, on all host threads it is given, on a bounded
    sample of the same cells; cell-timesteps/s.  With y_gpu (the timed
    step's output, [N][C] host array) the oracle's results for the sampled
    cells are also compared with it: the parity of what was timed."""
    import numpy as np
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    o = oracle.Oracle(m)
    threads = o.max_threads()
    # one untimed warm-up round, then consecutive chunks until the target time
    chunk = max(1, 4 * threads)
    warm = min(c.n_cells, threads)
    sel = np.arange(warm)
    o.solve(o.rate_constants(c.T[sel], c.jscale[sel]), c.y0[:, sel], dt)
    start, n, wall, failed = warm, 0, 0.0, 0
    worst, compared = 0.0, 0
    while wall < target_s and start < c.n_cells:
        sel = np.arange(start, min(c.n_cells, start + chunk))
        k = o.rate_constants(c.T[sel], c.jscale[sel])
        t0 = time.perf_counter()
        yo, st, _ = o.solve(k, c.y0[:, sel], dt)
        wall += time.perf_counter() - t0
        failed += int((st != 0).sum())
        n += len(sel)
        start += len(sel)
        if y_gpu is not None:
            ok = st == 0
            err = np.abs(y_gpu[:, sel][:, ok] - yo[:, ok]) / (1e-6 * np.abs(yo[:, ok]) + 1e2 * atol)
            worst = max(worst, float(err.max()) if err.size else 0.0)
            compared += int(ok.sum())
    # the same oracle on one thread (the paper's single-thread baseline), a
    # shorter sample of the next cells
    n1, wall1 = 0, 0.0
    while wall1 < target_s / 4 and start < c.n_cells:
        sel = np.arange(start, min(c.n_cells, start + 4))
        k = o.rate_constants(c.T[sel], c.jscale[sel])
        t0 = time.perf_counter()
        o.solve(k, c.y0[:, sel], dt, n_threads=1)
        wall1 += time.perf_counter() - t0
        n1 += len(sel)
        start += len(sel)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    out = {"value": n / wall, "unit": "cell-timesteps/s", "cores": threads, "kind": "oracle",
           "sample": f"cells {warm}..{warm + n - 1} of {c.n_cells}, one {dt:g} s step each, "
                     f"{wall:.1f} s wall on {threads} OpenMP threads ({failed} failed)",
           "host_cpu": model,
           "value_1_thread": n1 / wall1 if wall1 > 0 else None,
           "sample_1_thread": f"the next {n1} cells, {wall1:.1f} s wall on one thread"}
    if y_gpu is not None:
        out["parity"] = {"cells": compared, "worst_ratio_to_bar": worst, "pass": bool(worst <= 1.0 and compared > 0),
                         "bar": "|y_gpu - y_oracle| <= 1e-6 |y_oracle| + 1e2 atol, the timed step's output, "
                                "cells of the oracle sample",
                         "oracle_accuracy": "the oracle itself agrees with scipy Radau (rtol 1e-12) to 5e-6 "
                                            "relative + 1e2 atol on sampled cells of the nonlinear workloads, "
                                            "to 1e-6 on every closed form"}
    return out


def bench_mixed(args):
    """Mixed batch of three mechanisms (20, 72 and 150 species; 30/50/20% of
    100,000 cells): a window of --window consecutive 60 s outer steps of
    every batch (y advancing), each batch on its own stream, captured into
    one HIP graph that starts by restoring y0; one timed step = one replay
    of the window."""
    import numpy as np
    import torch

    from paper_2501_00011_amd import mcchem, synth
    groups, owner, dt = synth.mixed_workload(args.cells or 100000)
    W = max(1, args.window)
    dev = torch.device("cuda:0")
    opts = mcchem.default_opts()
    streams = [torch.cuda.Stream(device=dev) for _ in groups]
    runs = []
    for (m, c), side in zip(groups, streams):
        mech = mcchem.Mechanism(m, device=0)
        cells = mcchem.Cells(mech, c.n_cells)
        cells.bind(torch.from_numpy(c.T).to(dev), torch.from_numpy(c.P).to(dev),
                   torch.from_numpy(c.jscale).to(dev))
        y0 = torch.from_numpy(c.y0).to(dev)
        runs.append({"m": m, "c": c, "mech": mech, "cells": cells, "y0": y0, "y": y0.clone(), "side": side,
                     "status": [torch.empty(c.n_cells, dtype=torch.int32, device=dev) for _ in range(W)],
                     "stats": [torch.empty((c.n_cells, mcchem.STATS_DTYPE.itemsize), dtype=torch.uint8, device=dev)
                               for _ in range(W)]})
    torch.cuda.synchronize()
    # one eager outer step per batch; its counters schedule each batch's
    # cells longest first (the schedule is read by the captured launches)
    for r in runs:
        r["cells"].step(r["y"], dt, opts, r["status"][0], r["stats"][0])
        r["cells"].balance(r["stats"][0])
        r["y"].copy_(r["y0"])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cap):
        for r in runs:
            r["side"].wait_stream(cap)
            with torch.cuda.stream(r["side"]):
                r["y"].copy_(r["y0"])  # a copy kernel: every replay starts from y0
            for k in range(W):
                r["cells"].step(r["y"], dt, opts, r["status"][k], r["stats"][k], stream=r["side"])
            cap.wait_stream(r["side"])
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    flops, failed, gpu_s = 0.0, 0, 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev[0].record()
        g.replay()
        ev[1].record()
        torch.cuda.synchronize()
        gpu_s += ev[0].elapsed_time(ev[1]) / 1e3
        for r in runs:  # the window's work from the stats of this replay (host reads lie between replays)
            oc = r["mech"].op_counts()
            for k in range(W):
                sn = mcchem.stats_numpy(r["stats"][k])
                flops += float(np.sum(sn["f_evals"].astype(np.int64) * oc["deriv_flops"]
                                      + sn["jac_evals"].astype(np.int64) * oc["newton_matrix_flops"]
                                      + sn["lu_count"].astype(np.int64) * oc["lu_flops"]
                                      + sn["newton_iters"].astype(np.int64) * oc["solve_flops"]))
                failed += int((r["status"][k].cpu().numpy() != 0).sum())
    wall = time.perf_counter() - t0
    C = sum(r["c"].n_cells for r in runs)
    tf = flops / gpu_s / 1e12
    result = {
        "metric": "cell-timesteps/s (FP64, 1e-6 rel vs oracle); mixed mechanisms, graph replay",
        "value": C * W * args.steps / wall, "unit": "cell-timesteps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"mixed batch of {C} cells: "
                               + ", ".join(f"{r['c'].n_cells} x {r['m'].n_species}/{r['m'].n_reactions}"
                                           for r in runs)
                               + f", a window of {W} consecutive {dt:g} s BDF steps per replay of a captured "
                                 f"graph (3 streams); one timed step = one replay",
                   "cells": C, "dt_s": dt, "window": W, "rtol": opts.rtol, "atol": opts.atol,
                   "cell_schedule": "per batch, longest first by the counters of an eager first step"},
        "roofline": {"kernel": "bdf_kernel x 3 mechanisms (solve_step)", "bound": "alu", "achieved": tf,
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP64_VALU_PEAK_TFLOPS,
                     "traffic": None, "replay_ms": gpu_s / args.steps * 1e3, "flops_per_replay": flops / args.steps},
        "solver": {"failed_cells": failed},
    }
    print(json.dumps(result), flush=True)


def bench_ablation(args):
    """f for every cell of the workload, four ways, each the median of
    --fj-reps launches timed with events on one stream."""
    import numpy as np
    import torch

    from paper_2501_00011_amd import mcchem, synth
    m, c, dt = synth.workload(args.workload, args.cells)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mech = mcchem.Mechanism(m, device=0)  # f only: the solver's dense tail plays no part
    C = c.n_cells
    cells = mcchem.Cells(mech, C)
    cells.bind(torch.from_numpy(c.T).to(dev), torch.from_numpy(c.P).to(dev), torch.from_numpy(c.jscale).to(dev))
    y = torch.from_numpy(c.y0).to(dev)
    f = torch.empty_like(y)
    k_cm = cells.rate_constants().t().contiguous()          # [C][R], the paper's layout
    y_cm = y.t().contiguous()
    f_cm = torch.empty_like(y_cm)
    y_host = y_cm.cpu().pin_memory()
    f_host = torch.empty_like(y_cm, device="cpu").pin_memory()

    def timed(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(args.fj_reps, 1)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            ts.append((a, b))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ts])) * 1e3  # us

    def paper_with_copies():
        y_cm.copy_(y_host, non_blocking=True)
        mech.paper_deriv(y_cm, k_cm, f_cm, inverted=True, stream=stream)
        f_host.copy_(f_cm, non_blocking=True)

    res = {
        "ours_generated_f_us": timed(lambda: cells.deriv(y, f, stream=stream)),
        "paper_records_us": timed(lambda: mech.paper_deriv(y_cm, k_cm, f_cm, inverted=False, stream=stream)),
        "paper_inverted_us": timed(lambda: mech.paper_deriv(y_cm, k_cm, f_cm, inverted=True, stream=stream)),
        "paper_inverted_with_copies_us": timed(paper_with_copies),
    }
    torch.cuda.synchronize()
    fb = mech.op_counts()["f_bytes"] * C
    out = {"metric": "f evaluation time (us, median)", "workload": f"{m.n_species} species / {m.n_reactions} "
           f"reactions, {C} cells", "f_bytes_algorithmic": fb, **{k: round(v, 2) for k, v in res.items()},
           "inversion_speedup": res["paper_records_us"] / res["paper_inverted_us"],
           "copy_share_of_paper_call": 1.0 - res["paper_inverted_us"] / res["paper_inverted_with_copies_us"],
           "ours_vs_paper_inverted": res["paper_inverted_us"] / res["ours_generated_f_us"],
           "ours_f_GBps": fb / res["ours_generated_f_us"] / 1e3}
    print(json.dumps(out), flush=True)


def _solver_mechanism(args, m, c, dt):
    """The mechanism compiled with --dense-tail, or with the tail size the
    autotuner measures fastest on (up to) the first 8,192 cells."""
    from paper_2501_00011_amd import mcchem, synth
    if args.dense_tail is not None:
        return mcchem.Mechanism(m, device=0, dense_tail=args.dense_tail)
    if not args.autotune:
        return mcchem.Mechanism(m, device=0)
    n = min(8192, c.n_cells)
    sample = synth.Cells(T=c.T[:n], P=c.P[:n], jscale=c.jscale[:n], y0=c.y0[:, :n])
    # the reverse-mode kernels are built for tails of 0, 32 and 48 rows (and
    # for the library's register budget only)
    mech, _, _ = mcchem.autotune_solver(m, sample, dt, mcchem.default_opts(), candidates=(0, 32, 48), waves=(0,),
                                        schedules=("longest",))
    return mech


def bench_adjoint(args):
    """Forward outer step with its step tape, then the reverse pass
    (mcc_adjoint_step) for dL/dy0 and dL/d ln k, each timed with events on
    the launch stream; the plain forward step beside them."""
    import numpy as np
    import torch

    from paper_2501_00011_amd import mcchem, synth
    m, c, dt = synth.workload(args.workload, args.cells)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mech = _solver_mechanism(args, m, c, dt)
    C, N, R = c.n_cells, m.n_species, m.n_reactions
    cells = mcchem.Cells(mech, C)
    cells.bind(torch.from_numpy(c.T).to(dev), torch.from_numpy(c.P).to(dev), torch.from_numpy(c.jscale).to(dev))
    y0 = torch.from_numpy(c.y0).to(dev)
    y = torch.empty_like(y0)
    status = torch.empty(C, dtype=torch.int32, device=dev)
    stats = torch.empty((C, mcchem.STATS_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    opts = mcchem.default_opts()
    y.copy_(y0)
    cells.step(y, dt, opts, status, stats, stream=stream)
    cells.balance(stats)  # the cells longest first, for all three launches
    sn = mcchem.stats_numpy(stats)
    attempts = sn["steps"] + sn["rejects"] + sn["newton_fails"]
    stride = int((4 + 8 * attempts + N * sn["steps"]).max())
    tape = torch.empty((C, stride), dtype=torch.float64, device=dev)
    tlen = torch.empty(C, dtype=torch.int64, device=dev)
    lam = torch.empty_like(y0)
    w = torch.ones_like(y0)
    glnk = torch.empty((R, C), dtype=torch.float64, device=dev)
    ast = torch.empty(C, dtype=torch.int32, device=dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            ts.append((a, b))
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ts]))  # ms

    def plain():
        y.copy_(y0)
        cells.step(y, dt, opts, status, stats, stream=stream)

    def taped():
        y.copy_(y0)
        cells.step_taped(y, dt, tape, tlen, opts, status, stats, stream=stream)

    def reverse():
        lam.copy_(w)
        cells.adjoint_step(y0, tape, tlen, lam, glnk, status=ast, stream=stream)

    reps = max(args.steps, 1)
    t_plain = timed(plain, reps)
    t_taped = timed(taped, reps)
    t_rev = timed(reverse, reps)
    tl = tlen.cpu().numpy()
    ok = int(((ast.cpu().numpy() == 0) & (status.cpu().numpy() == 0)).sum())
    oc = mech.op_counts()
    steps = sn["steps"].astype(np.int64)
    # reverse pass per accepted step: Newton matrix, factorisation, one
    # solve, the rates twice (Jacobian partials and rates) -- counted as
    # the forward kernel's per-operation flops
    rev_flops = float(np.sum(steps * (oc["newton_matrix_flops"] + oc["lu_flops"] + oc["solve_flops"]
                                      + oc["deriv_flops"])))
    out = {"metric": "reverse mode of one outer step (ms per launch, mean)",
           "workload": f"{N} species / {R} reactions, {C} cells, one {dt:g} s BDF step",
           "dense_tail": mech.schedule_info()["dense_tail"], "cell_schedule": "longest first",
           "plain_forward_ms": round(t_plain, 3), "taped_forward_ms": round(t_taped, 3),
           "reverse_ms": round(t_rev, 3), "taping_overhead": t_taped / t_plain - 1.0,
           "reverse_over_forward": t_rev / t_plain,
           "forward_plus_reverse_cell_steps_per_s": C / ((t_taped + t_rev) / 1e3),
           "tape_bytes_mean_per_cell": float(tl.mean() * 8), "tape_stride": stride,
           "cells_ok": ok, "steps_mean": float(steps.mean()),
           "reverse_tflops": rev_flops / (t_rev / 1e3) / 1e12}
    if not args.no_cpu:
        import oracle
        o = oracle.Oracle(m)
        k = o.rate_constants(c.T, c.jscale)
        t0 = time.perf_counter()
        n = 0
        while n < C and (n < 2 or time.perf_counter() - t0 < args.cpu_seconds):
            _, _, _, tp = o.solve_taped(k[:, n], c.y0[:, n], dt)
            o.adjoint(k[:, n], c.y0[:, n], tp, np.ones(N))
            n += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / el, "unit": "cells/s (taped forward + adjoint)", "cores": 1,
                               "kind": "oracle", "sample": f"first {n} cells, one thread"}
        out["gpu_cells_per_s"] = C / ((t_taped + t_rev) / 1e3)
    print(json.dumps(out), flush=True)


def bench_gradient(args):
    """d L / d log A for L = sum over cells and species of
    (ln(y + atol) - ln(y_target + atol))^2 after 10 outer steps of 60 s, the
    target being the forward result with log A perturbed by N(0, 0.1^2)
    (seed 5005): forward with checkpoints, then the reverse sweep (each
    outer step re-run with its tape and reversed), timed on the GPU."""
    import numpy as np
    import torch

    from paper_2501_00011_amd import autograd, mcchem, synth
    m, c, dt = synth.workload("adjoint10k" if args.workload == "medium10k" else args.workload, args.cells)
    n_out = 10
    dev = torch.device("cuda:0")
    mech = _solver_mechanism(args, m, c, dt)
    C, N, R = c.n_cells, m.n_species, m.n_reactions
    cells = mcchem.Cells(mech, C)
    cells.bind(torch.from_numpy(c.T).to(dev), torch.from_numpy(c.P).to(dev), torch.from_numpy(c.jscale).to(dev))
    k = cells.rate_constants().clone()
    y0 = torch.from_numpy(c.y0).to(dev)
    _, first = cells.step(y0.clone(), dt)
    cells.balance(first)  # the cells longest first by their first outer step
    atol = mcchem.default_opts().atol
    with torch.no_grad():
        pert = torch.from_numpy(np.random.default_rng(5005).normal(0.0, 0.1, R)).to(dev)
        target = autograd.integrate(cells, y0, torch.log(k) + pert[:, None], dt, n_out)

    def run():
        lnk = torch.log(k).requires_grad_(True)
        y = autograd.integrate(cells, y0, lnk, dt, n_out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = ((torch.log(y + atol) - torch.log(target + atol)) ** 2).sum()
        loss.backward()
        gA = lnk.grad.sum(dim=1)
        torch.cuda.synchronize()
        return time.perf_counter() - t1, gA, float(loss.detach())

    for _ in range(args.warmup):
        run()
    ts = []
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        t_bwd, gA, loss = run()
        ts.append((time.perf_counter() - t0, t_bwd))
    tot = float(np.mean([a for a, _ in ts]))
    bwd = float(np.mean([b for _, b in ts]))
    out = {"metric": "gradient of the log loss wrt log A, 10 x 60 s forward + reverse (s per gradient)",
           "dense_tail": mech.schedule_info()["dense_tail"], "cell_schedule": "longest first by the first step",
           "workload": f"{N} species / {R} reactions, {C} cells, 10 outer steps of {dt:g} s",
           "value": tot, "unit": "s", "higher_is_better": False,
           "forward_s": tot - bwd, "reverse_s": bwd, "reverse_over_forward": bwd / (tot - bwd),
           "cell_gradients_per_s": C / tot, "loss": loss,
           "grad_logA_norm": float(gA.norm()), "grad_logA_first4": [float(v) for v in gA[:4]]}
    if args.fd_params > 0:
        # the forward's step tapes, one buffer per outer step, then the loss
        # of the replayed chain at log A_j +- h for the largest components
        cells.set_rate_constants(k)
        tapes, yy, stats = [], y0.clone(), None
        for _ in range(n_out):
            probe = yy.clone()
            _, stats = cells.step(probe, dt, stats=stats)
            tape = torch.empty((C, autograd._tape_bound(stats, N)), dtype=torch.float64, device=dev)
            tlen = torch.empty(C, dtype=torch.int64, device=dev)
            cells.step_taped(yy, dt, tape, tlen)
            tapes.append((tape, tlen))
        eps = 1e-6

        def replayed_loss(j, sign):
            kp = k.clone()
            kp[j] *= float(np.exp(sign * eps))
            cells.set_rate_constants(kp)
            ys = y0
            for tape, tlen in tapes:
                ys, st = cells.replay_step(ys, tape, tlen)
            bad = int((st != 0).sum())
            return float(((torch.log(ys + atol) - torch.log(target + atol)) ** 2).sum()), bad

        g = gA.cpu().numpy()
        sel = [int(j) for j in np.argsort(-np.abs(g))[:args.fd_params]]
        rel, failed = [], 0
        t0 = time.perf_counter()
        for j in sel:
            (lp, bp), (lm, bm) = replayed_loss(j, 1), replayed_loss(j, -1)
            failed += bp + bm
            rel.append(abs((lp - lm) / (2 * eps) - g[j]) / abs(g[j]))
        t_fd = time.perf_counter() - t0
        cells.set_rate_constants(k)
        out["fd_check"] = {"params": sel, "h": eps, "max_rel_diff": max(rel), "replay_failed_cells": failed,
                           "replayed_chains": 2 * len(sel), "s_per_chain": t_fd / (2 * len(sel))}
    if not args.no_cpu:
        import oracle
        o = oracle.Oracle(m)
        kc = o.rate_constants(c.T, c.jscale)
        t0 = time.perf_counter()
        n = 0
        while n < C and (n < 1 or time.perf_counter() - t0 < args.cpu_seconds):
            y, tapes = c.y0[:, n].copy(), []
            for _ in range(n_out):
                ys = y.copy()
                y, _, _, tp = o.solve_taped(kc[:, n], ys, dt)
                tapes.append((ys, tp))
            lam = np.ones(N)
            for ys, tp in reversed(tapes):
                lam, _ = o.adjoint(kc[:, n], ys, tp, lam)
            n += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / el, "unit": "cell gradients/s (10 x 60 s forward + adjoint)",
                               "cores": 1, "kind": "oracle", "sample": f"first {n} cells, one thread"}
    print(json.dumps(out), flush=True)


def consecutive_steps(cells, y0, T, P, s, dt, args, stream):
    """Consecutive outer steps as an application runs them: y advances from
    step to step, and before each step the cells are scheduled longest first
    by the previous step's counters (a prediction, not the step being timed);
    once starting every step afresh, once warm started from the previous
    step's step size.  Wall time per step, schedule upload included."""
    import torch

    from paper_2501_00011_amd import mcchem
    out = {}
    n = args.consecutive
    for warm in (0, 1):
        y = y0.clone()
        cells.set_schedule(None)
        _, stats = cells.step(y, dt, stream=stream)  # the first step, cold: sets the counters
        torch.cuda.synchronize()
        opts = mcchem.default_opts(warm_start=warm)
        steps = []
        t0 = time.perf_counter()
        for _ in range(n):
            cells.balance(stats)
            st, stats = cells.step(y, dt, opts, stats=stats, stream=stream)
            steps.append(stats.clone())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sn = [mcchem.stats_numpy(x) for x in steps]
        out["warm" if warm else "cold"] = {
            "value": cells.n_cells * n / wall, "ms_per_step": wall / n * 1e3,
            "steps_mean": float(sum(x["steps"].mean() for x in sn) / n),
            "failed_cells": int((st != 0).sum())}
    cells.set_schedule(None)
    out["note"] = (f"{n} consecutive {dt:g} s outer steps after a first cold one, y advancing, cells ordered "
                   "longest first by the previous step's attempts; warm: first step size from the previous "
                   "step (opts.warm_start)")
    return out


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the cells of this workload are independent, so one GPU's "
              "share is what it measures (sharding is by contiguous cell ranges); use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.ablation:
        bench_ablation(args)
        return
    if args.workload == "mixed100k":
        bench_mixed(args)
        return
    if args.adjoint:
        bench_adjoint(args)
        return
    if args.gradient:
        bench_gradient(args)
        return
    import numpy as np
    import torch

    from paper_2501_00011_amd import mcchem, synth

    m, c, dt = synth.workload(args.workload, args.cells)
    dev = torch.device("cuda:0")
    tuned, choice = None, None
    schedule = "longest"
    if args.dense_tail is not None:
        mech = mcchem.Mechanism(m, device=0, dense_tail=args.dense_tail)
    elif args.autotune and not args.multicell:  # Multi-cells is built for fewer tail sizes
        n = min(8192, c.n_cells)
        sample = synth.Cells(T=c.T[:n], P=c.P[:n], jscale=c.jscale[:n], y0=c.y0[:, :n])
        mech, tuned, choice = mcchem.autotune_solver(m, sample, dt, mcchem.default_opts())
        schedule = choice[2]
    else:
        mech = mcchem.Mechanism(m, device=0)
    C = c.n_cells
    cells = mcchem.Cells(mech, C)
    T = torch.from_numpy(c.T).to(dev)
    P = torch.from_numpy(c.P).to(dev)
    s = torch.from_numpy(c.jscale).to(dev)
    y0 = torch.from_numpy(c.y0).to(dev)
    y = torch.empty_like(y0)
    f = torch.empty_like(y0)
    J = torch.empty((mech.nnz, C), dtype=torch.float64, device=dev)
    status = torch.empty(C, dtype=torch.int32, device=dev)
    stats = torch.empty((C, mcchem.STATS_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    opts = mcchem.default_opts(steps_per_launch=args.steps_per_launch)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        cells.bind(T, P, s, stream=stream)
        cells.deriv_jac(y0, f, J, stream=stream)
        y.copy_(y0)
        if ev is not None:
            ev[0].record(stream)
        if args.multicell:
            cells.step_multicell(y, dt, opts, status, stats, stream=stream)
        else:
            cells.step(y, dt, opts, status, stats, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # cell schedule: the solver takes the cells longest first by the step
    # attempts they needed in the previous outer step (its counters); the
    # identity schedule's solve time is reported beside it
    unbalanced_ms = None
    if not args.multicell and not args.no_balance:
        ev0 = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        step(ev0)
        torch.cuda.synchronize()
        unbalanced_ms = ev0[0].elapsed_time(ev0[1])
        if schedule != "identity":
            cells.balance(stats, schedule)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    solve_ms = [a.elapsed_time(b) for a, b in evs]

    st = status.cpu().numpy()
    sn = mcchem.stats_numpy(stats)
    oc = mech.op_counts()
    flops = float(np.sum(sn["f_evals"].astype(np.int64) * oc["deriv_flops"]
                         + sn["jac_evals"].astype(np.int64) * oc["newton_matrix_flops"]
                         + sn["lu_count"].astype(np.int64) * oc["lu_flops"]
                         + sn["newton_iters"].astype(np.int64) * oc["solve_flops"]))
    solve_s = float(np.mean(solve_ms)) / 1e3
    achieved_tf = flops / solve_s / 1e12

    # f+J and VJP rooflines: each kernel's average launch duration, from 20
    # back-to-back launches captured in a HIP graph (host launch gaps, about
    # 9 us per call through the Python binding, would otherwise pad the
    # short launches) and replayed 5 times between two events on the launch
    # stream; eager back-to-back launches beside them for reference
    v = torch.ones_like(y0)
    gy = torch.empty_like(y0)
    glnk = torch.empty((m.n_reactions, C), dtype=torch.float64, device=dev)

    def per_launch(fn, n_graph=20, replays=5):
        for _ in range(10):
            fn(stream)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record(stream)
        for _ in range(max(args.fj_reps, 1)):
            fn(stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        eager = ev[0].elapsed_time(ev[1]) / 1e3 / max(args.fj_reps, 1)
        graph = None
        try:
            cap = torch.cuda.Stream(device=dev)
            cap.wait_stream(stream)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                for _ in range(n_graph):
                    fn(cap)
            g.replay()
            torch.cuda.synchronize()
            ge = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            with torch.cuda.stream(stream):  # replays go to the current stream
                ge[0].record(stream)
                for _ in range(replays):
                    g.replay()
                ge[1].record(stream)
            torch.cuda.synchronize()
            graph = ge[0].elapsed_time(ge[1]) / 1e3 / (n_graph * replays)
        except RuntimeError as e:  # capture refused: reported, the eager figure used
            print(f"graph capture failed: {e}", file=sys.stderr)
        return (graph if graph is not None else eager), eager, graph

    fj_s, fj_eager_s, fj_graph_s = per_launch(lambda s_: cells.deriv_jac(y0, f, J, stream=s_))
    fj_gbs = oc["fj_bytes"] * C / fj_s / 1e9
    # reverse mode: J^T v and d(v.f)/d ln k in one launch
    vj_s, vj_eager_s, vj_graph_s = per_launch(lambda s_: cells.vjp(y0, v, gy, glnk, stream=s_))
    vj_bytes = 8 * (3 * m.n_species + 2 * m.n_reactions)  # read y, v, k; write gy, glnk
    vj_gbs = vj_bytes * C / vj_s / 1e9

    # counter figures were taken for one scheduled launch per outer step
    plain = args.steps_per_launch == 0 and not args.multicell and unbalanced_ms is not None
    tail_measured = mech.schedule_info()["dense_tail"] if plain else None
    result = {
        "metric": "cell-timesteps/s (FP64, 1e-6 rel vs oracle); f+J evals/s as % HBM peak",
        "value": C * args.steps / wall,
        "unit": "cell-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{m.n_species} species / {m.n_reactions} reactions, {C} cells, "
                               f"one {dt:g} s BDF step + rate constants + fused f/J per step; termolecular "
                               f"pre-factors on the scaled reading (log-uniform 1e-14..1e-10 divided by "
                               f"M_ref = {synth.M_REF:g} cm^-3)",
                   "cells": C, "species": m.n_species, "reactions": m.n_reactions, "dt_s": dt,
                   "rtol": opts.rtol, "atol": opts.atol, "steps_per_launch": args.steps_per_launch,
                   "step_control": "multi-cells (shared)" if args.multicell else "per cell",
                   "dense_tail": mech.schedule_info()["dense_tail"],
                   "waves_per_simd": mech.schedule_info()["waves_per_simd"],
                   "cell_schedule": "identity" if unbalanced_ms is None or schedule == "identity" else
                   f"{schedule} by the previous outer step's attempts",
                   "solve_ms_identity_schedule": unbalanced_ms,
                   "autotune_ms": {k: round(v, 2) for k, v in tuned.items()} if tuned else None,
                   "autotune_note": "keys: dense tail / wavefronts per SIMD / cell schedule; one outer step of "
                                    "the first 8,192 cells" if tuned else None},
        "roofline": {"kernel": "bdf_kernel (solve_step)", "bound": "alu", "achieved": achieved_tf,
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_VALU_PEAK_TFLOPS,
                     "traffic": solver_counter("traffic_bytes", C, tail_measured),
                     "launch_ms": solve_s * 1e3, "flops_per_launch": flops,
                     "issue": issue_roofline(solve_s, C, tail_measured)},
        "fj_roofline": {"kernel": FJ_KERNEL + " (calc_deriv_jac, generated for this mechanism)", "bound": "hbm",
                        "achieved": fj_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fj_gbs / HBM_PEAK_GBS,
                        "traffic": measured_traffic(FJ_KERNEL, FJ_SOURCES, C),
                        "launch_us": fj_s * 1e6, "bytes_per_cell": oc["fj_bytes"],
                        "launch_us_eager": fj_eager_s * 1e6,
                        "timing": "20 launches in a HIP graph" if fj_graph_s is not None else "eager"},
        "vjp_roofline": {"kernel": VJP_KERNEL + " (calc_vjp: J^T v and d(v.f)/d ln k)", "bound": "hbm",
                         "achieved": vj_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": vj_gbs / HBM_PEAK_GBS,
                         "traffic": measured_traffic(VJP_KERNEL, FJ_SOURCES, C),
                         "launch_us": vj_s * 1e6, "bytes_per_cell": vj_bytes,
                         "launch_us_eager": vj_eager_s * 1e6,
                         "timing": "20 launches in a HIP graph" if vj_graph_s is not None else "eager"},
        "per_launch_state": per_launch_state(sn, args.steps_per_launch, m.n_species, mech),
        "solver": {"failed_cells": int((st != 0).sum()),
                   "steps_mean": float(sn["steps"].mean()), "steps_max": int(sn["steps"].max()),
                   "steps_percentiles": {str(q): float(np.percentile(sn["steps"], q)) for q in (1, 10, 50, 90, 99)},
                   "attempts_mean": float((sn["steps"] + sn["rejects"] + sn["newton_fails"]).mean()),
                   "newton_per_attempt": float(sn["newton_iters"].sum() / max(sn["lu_count"].sum(), 1))},
    }
    if args.consecutive > 0 and not args.multicell:
        result["consecutive_steps"] = consecutive_steps(cells, y0, T, P, s, dt, args, stream)
    failed_parity = False
    if not args.no_cpu:
        cb = cpu_baseline(m, c, dt, args.cpu_seconds, y_gpu=y.cpu().numpy(), atol=opts.atol)
        result["parity"] = cb.pop("parity")
        failed_parity = not result["parity"]["pass"]
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)
    if failed_parity:
        print(f"bench: the timed output differs from the oracle ({result['parity']})", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
