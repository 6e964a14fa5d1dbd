"""Benchmark: FP64 FMG solve throughput on one MI355X.

Default workload: two interacting streamers plus Poisson background
ionisation on an octree of base 64^3 + 7 refinement levels (effective
8192^3, ~1.2e8 leaf cells, 11 levels), the largest single-GPU configuration.

One step = one mg_fmg_solve: the FMG pass plus V(2,2) cycles until the
relative residual is below 1e-8, residual checks included (tree creation and
right-hand-side upload excluded).  value = leaf cells solved per second over
the K timed steps; each step is also timed on its own (the solve returns
after its last residual check has been read back), and the median and the
minimum are reported.

Prints one JSON line with the solve throughput, the solve-level roofline
(the byte model of the FMG solve against the 8 TB/s HBM peak) with the
dominant kernel beside it (red-black Gauss-Seidel half-sweep on the level
that moves the most bytes, timed with HIP events on the library's stream),
the mixed-precision and learned solves on the same workload, the oracle's
CPU throughput, and each GPU result's distance from the oracle's solution.
The time-step, mesh-adaptation and fluid legs run on the smaller static
streamer tree (base 64^3 + 4 levels) as secondary keys.

--copy-probe BYTES adds one device-to-device copy of that many bytes (a plain
copy kernel of known size, used to calibrate rocprofv3 traffic counters).
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BETA_FP64 = 127.0          # bytes per stored cell per V(2,2) visit (per-sweep model)
NORM_BYTES = 16.0          # bytes per leaf cell per residual check
METRIC = ("cells/s per FMG solve to rel. residual 1e-8 (FP64 vs mixed vs learned); HBM GB/s")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gsrb_finest_traffic_{}.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1708_08434_amd", "csrc", "kernels.hip")


def log(*a):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print("bench:", *a, file=sys.stderr, flush=True)


def model_bytes(level_counts, n_leaf, k):
    """Per-sweep byte model of an FMG solve with k V-cycles after the FMG pass."""
    cum, s = [], 0
    for c in level_counts:
        s += 512 * c
        cum.append(s)
    fmg = sum(BETA_FP64 * cum[l] for l in range(1, len(cum)))
    return fmg + k * BETA_FP64 * cum[-1] + (k + 1) * NORM_BYTES * n_leaf


def gsrb_kernel_name(v):
    """The Gauss-Seidel kernel of launch variant v (include/mg.h)."""
    if v < 6:
        return f"k_gsrb<C,double,{(1, 2, 4)[v >> 1]}> (red-black Gauss-Seidel half-sweep)"
    if v < 8:
        return "k_gsrb_sweep<double> (fused red-black Gauss-Seidel sweep)"
    if v < 10:
        return "k_gsrb_oct<C,double> (red-black Gauss-Seidel half-sweep over sibling octets)"
    return (f"k_gsrb_pipe<C,double> (red-black Gauss-Seidel half-sweep, at most "
            f"{2048 if v < 12 else 4096} persistent workgroups)")


def traffic_per_launch(workload, level, variant):
    """HBM bytes per launch of the Gauss-Seidel kernel on the given level of
    this workload in this launch variant, from the committed rocprofv3 counter
    summary, or None if there is none or the kernel source has changed since
    the counters were taken."""
    path = TRAFFIC_FILE.format(workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if rec.get("kernel_sha256") != src or rec.get("level") != level:
        return None
    v = rec.get("variants", {}).get(str(variant))
    return v["bytes_per_launch"] if v else None


def traffic_probe(w, reps=8):
    """Launches to count HBM traffic under rocprofv3 --pmc: on the level of
    the tree with the most boxes (the finest level of a single streamer),
    `reps` smoothing calls of 2 sweeps with each Gauss-Seidel launch variant
    in turn (that level's schedule entry), each variant's launches preceded by a 1 KiB copy-kernel launch of variant + 1
    blocks that marks where they start; then the 2 GiB copy kernel whose
    counters calibrate FETCH_SIZE and WRITE_SIZE.  No autotuning (the other
    levels keep the default variant, and only the finest level runs)."""
    import numpy as np
    import torch
    from paper_1708_08434_amd import mg as M
    g = M.Tree.from_workload(w, device="cuda:0")
    g.set_rhs_from(w)
    g.fmg_solve()
    levels = np.bincount(g.index(M.MG_IDX_LEVEL).reshape(-1))
    fin = int(np.argmax(levels))
    sched = [3] * g.nlev
    mark = torch.zeros(2, 1024 // 8, dtype=torch.float64, device="cuda:0")
    out = {}
    for v in range(M.MG_GSRB_VARIANTS):
        sched[fin - 1] = v
        M.mg_set_schedule(g.h, M.MG_FP64, sched)
        torch.cuda.synchronize()
        M.mg_stream_copy(mark[1].data_ptr(), mark[0].data_ptr(), 1024, v + 1, g.stream.cuda_stream)
        for _ in range(reps):
            M.mg_step(g.h, M.MG_OP_SMOOTH, fin, 2)
        torch.cuda.synchronize()
        out[v] = {"smooth_calls": reps, "sweeps_per_call": 2}
        print(f"traffic probe: variant {v} done", flush=True)
    nbytes = 2 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        M.mg_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, 0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": {"workload": w.name, "level": fin,
                                        "boxes": int(levels[fin]), "variants": out,
                                        "copy_bytes": nbytes,
                                        "kernel_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()}}),
          flush=True)


def solve_traffic_probe(w, schedule=None, fusion=None):
    """Launches to count the HBM traffic of one FP64 FMG solve under
    rocprofv3 --pmc: a warm-up solve (graphs recorded), then a 1 KiB
    copy-kernel launch of 1 block, one FP64 solve, a 1 KiB copy of 2 blocks
    (the markers that bracket the solve's dispatches), then the 2 GiB copy
    kernel whose counters calibrate FETCH_SIZE and WRITE_SIZE."""
    import torch
    from paper_1708_08434_amd import mg as M
    g = M.Tree.from_workload(w, device="cuda:0")
    if fusion is not None:
        M.mg_set_fusion(g.h, fusion)
    if schedule:
        parts = parse_schedule(schedule, g.nlev, M.MG_GSRB_VARIANTS)
        M.mg_set_schedule(g.h, M.MG_FP64, parts[0])
    g.set_rhs_from(w)
    st = g.fmg_solve()
    mark = torch.zeros(2, 1024 // 8, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    M.mg_stream_copy(mark[1].data_ptr(), mark[0].data_ptr(), 1024, 1, g.stream.cuda_stream)
    st = g.fmg_solve()
    M.mg_stream_copy(mark[1].data_ptr(), mark[0].data_ptr(), 1024, 2, g.stream.cuda_stream)
    torch.cuda.synchronize()
    nbytes = 2 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    M.mg_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, 0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ls = list(g.info.level_start[:g.nlev + 1])
    counts = [ls[i + 1] - ls[i] for i in range(g.nlev)]
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read() + open(DRIVER_SRC, "rb").read()).hexdigest()
    print(json.dumps({"solve_traffic_probe": {
        "workload": w.name, "vcycles_after_fmg": st["n_vcycles"], "copy_bytes": nbytes,
        "model_bytes": model_bytes(counts, int(g.info.n_leaf_cells), st["n_vcycles"]),
        "source_sha256": sha}}), flush=True)


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def leaf_rel_l2(x, ref, leaf):
    """Relative L2 distance of x from ref over the leaf cells."""
    import numpy as np
    return float(np.linalg.norm((x - ref)[leaf]) / np.linalg.norm(ref[leaf]))


def cpu_baseline(w, rhs, order, gpu_cycles, results, small=None, budget_s=20.0):
    """The oracle (the plain FP64 CPU multigrid of the same algorithm) on the
    host cores, on the same tree and right-hand side.

    Timed: FP64 FMG solves to a relative residual of 1e-8 on all host threads
    (at least one; up to five while under budget_s), and one FMG solve of the
    smaller workload `small` on one thread and on all
    threads.  Untimed: V-cycles from the oracle's 1e-8 solution until 1e-12,
    the converged reference against which every GPU result in `results`
    (name -> potential in natural layout, canonical order) is stated as a
    relative L2 distance over the leaf cells, beside its distance from the
    oracle's own 1e-8 solution."""
    import numpy as np
    import oracle as O
    O.build(force=False)
    threads = O.set_threads(0)
    t = O.OracleTree.from_workload(w)
    assert np.array_equal(t.index(O.IDX_ORDER), order), "oracle and library orders differ"
    t.set_field(O.RHS, rhs)
    times, cyc = [], None
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        st = t.fmg_solve(tol=1e-8)
        times.append(time.perf_counter() - t0)
        cyc = st["n_vcycles"]
        el = time.perf_counter() - t_start
        if len(times) >= 5 or el + times[-1] > budget_s:
            break
    med = statistics.median(times)
    log(f"oracle: {len(times)} solve(s), median {med:.2f} s")
    leaf = t.leaf_mask()
    phi8 = t.get_field(O.PHI)
    st12 = t.vcycles(0, tol=1e-12)
    ref = t.get_field(O.PHI)
    log(f"oracle reference: {st12['n_vcycles']} more V-cycles, rel {st12['rel']:.2e}")
    del t
    acc = {"reference": f"oracle FP64 solve continued to rel. residual {st12['rel']:.2e} "
                        f"({cyc} + {st12['n_vcycles']} V-cycles)",
           "oracle_1e-8_vs_reference": leaf_rel_l2(phi8, ref, leaf)}
    for name, phi in results.items():
        acc[name] = {"rel_l2_vs_reference": leaf_rel_l2(phi, ref, leaf),
                     "rel_l2_vs_oracle_1e-8": leaf_rel_l2(phi, phi8, leaf)}
    del phi8, ref
    out = {"value": w.n_leaf / med, "unit": "cells/s", "cores": threads, "kind": "oracle",
           "sample": f"full workload, {len(times)} FP64 FMG solve(s) to 1e-8 on {threads} threads "
                     f"({cyc} V-cycles, GPU {gpu_cycles}), median {med:.3f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if small is not None:
        ws = small
        ts = O.OracleTree.from_workload(ws)
        ts.set_rhs_from(ws)
        t0 = time.perf_counter()
        ts.fmg_solve(tol=1e-8)
        t_all = time.perf_counter() - t0
        O.set_threads(1)
        try:
            t0 = time.perf_counter()
            ts.fmg_solve(tol=1e-8)
            t_one = time.perf_counter() - t0
        finally:
            O.set_threads(threads)
        out["one_thread"] = {"workload": ws.name, "n_leaf": ws.n_leaf,
                             "value": ws.n_leaf / t_one, "unit": "cells/s",
                             "all_threads_value": ws.n_leaf / t_all,
                             "sample": f"one FP64 FMG solve to 1e-8 of {ws.name}: "
                                       f"{t_one:.2f} s on 1 thread, {t_all:.3f} s on {threads}"}
    return out, acc


NN_FLOP_PER_CELL = 2 * 27 * (16 + 16 * 16 + 16)  # the three convolutions, multiply-adds x 2
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA


def copy_bandwidth(nbytes=2 << 30, reps=10):
    """Achievable streaming bandwidth: the library's 16-byte-vector copy
    kernel (mg_stream_copy) timed with HIP events on torch's stream; bytes
    read plus bytes written per second, best over a few grid sizes."""
    import torch
    from paper_1708_08434_amd import mg as M
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    best = None
    for blocks in (0, 2048, 4096):
        for _ in range(2):
            M.mg_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, blocks, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            M.mg_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, blocks, stream)
        e1.record()
        torch.cuda.synchronize()
        gbps = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
        if best is None or gbps > best[0]:
            best = (gbps, blocks)
    assert torch.equal(dst[:1024], src[:1024])
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": best[0], "bytes": nbytes, "grid": best[1] or "4 per CU",
            "kernel": "mg_stream_copy (16-byte vector loads and stores, grid-stride)"}


def learned_leg(g, args, k_plain, value_plain):
    """Train the correction network on seeded streamer trees that are not the
    benchmark problem, then time the learned solve on the benchmark tree and
    the network's forward kernel on all of its leaf boxes."""
    import numpy as np
    import torch
    from paper_1708_08434_amd import mg as M
    from paper_1708_08434_amd import nn as NN
    from workloads import forest

    # training problems: 8 streamer trees of the seeded forest generator
    tw = forest(n_trees=8)
    tt = M.Tree.from_workload(tw, device="cuda:0")
    tt.set_rhs_from(tw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, tgt = NN.training_pairs(tt, states=(0, 1, 2))
    rng = np.random.default_rng(1000)
    p0 = np.concatenate([rng.standard_normal(432) * np.sqrt(2.0 / 27), np.zeros(16),
                         rng.standard_normal(6912) * np.sqrt(2.0 / 432), np.zeros(16),
                         rng.standard_normal(432) * np.sqrt(1.0 / 432), np.zeros(1)])
    net = NN.Net(p0.astype(np.float32), device="cuda:0")
    losses = NN.train(net, x, tgt, steps=args.train_steps, batch=1024, lr=1e-3, seed=1,
                      log_every=max(1, args.train_steps - 1))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del tt
    L = NN.Learned(g)
    for _ in range(max(1, args.warmup)):
        res = L.solve(net)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_s = []
    for _ in range(args.steps):
        t_run = time.perf_counter()
        res = L.solve(net)  # returns after its last residual check is read back
        run_s.append(time.perf_counter() - t_run)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    phi = g.get_field(M.MG_FIELD_PHI)
    n_leaf = int(g.info.n_leaf_cells)
    # the per-level placement: a learned step on each level's leaf boxes after
    # that level's up-sweeps (its cycles launch kernel by kernel)
    for _ in range(max(1, args.warmup)):
        resl = L.solve(net, learned_placement=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    run_l = []
    for _ in range(args.steps):
        t_run = time.perf_counter()
        resl = L.solve(net, learned_placement=1)
        run_l.append(time.perf_counter() - t_run)
    torch.cuda.synchronize()
    el_l = time.perf_counter() - t2
    phi_levels = g.get_field(M.MG_FIELD_PHI)
    per_level = {"placement": "a learned step on each level's leaf boxes after its up-sweeps",
                 "value": n_leaf * args.steps / el_l, "unit": "cells/s",
                 "ms_per_step": 1e3 * el_l / args.steps, "runs": run_stats(run_l, n_leaf),
                 "vcycles": resl["n_vcycles"], "accepted_cycles": resl["accepted"],
                 "fallback_cycle": resl["fallback_cycle"], "learned_ms_per_step": resl["t_learned_ms"],
                 "final_rel_res": resl["rel"], "hist": [float(v) for v in resl["hist"]],
                 "vs_plain_fp64": (n_leaf * args.steps / el_l) / value_plain}
    # forward kernel on every leaf box of the benchmark tree, HIP events on
    # the stream it is launched on (torch's current stream)
    xin, _ = L.inputs()
    nbox = int(xin.shape[0])
    y = torch.empty((nbox, 512), dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        NN.mg_nn_forward(net.h, nbox, xin.data_ptr(), y.data_ptr())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        NN.mg_nn_forward(net.h, nbox, xin.data_ptr(), y.data_ptr())
    e1.record()
    torch.cuda.synchronize()
    launch_s = e0.elapsed_time(e1) / 1e3 / reps
    tflops = NN_FLOP_PER_CELL * 512 * nbox / launch_s / 1e12
    return phi, phi_levels, {"placement": "a learned step after every V-cycle that does not stop the solve",
            "value": n_leaf * args.steps / el, "unit": "cells/s", "ms_per_step": 1e3 * el / args.steps,
            "runs": run_stats(run_s, n_leaf), "hist": [float(v) for v in res["hist"]],
            "per_level": per_level,
            "vcycles": res["n_vcycles"], "vcycles_plain_fp64": k_plain,
            "accepted_steps": res["accepted"], "fallback_cycle": res["fallback_cycle"],
            "learned_ms_per_step": res["t_learned_ms"], "final_rel_res": res["rel"],
            "vs_plain_fp64": (n_leaf * args.steps / el) / value_plain,
            "train": {"problems": "8 seeded streamer trees (base 32^3 + <=5 levels), not the "
                                  "benchmark tree", "pairs": int(x.shape[0]),
                      "adam_steps": args.train_steps, "batch": 1024, "lr": 1e-3,
                      "loss_first_last": [losses[0][1], losses[-1][1]], "seconds": train_s},
            "nn_forward": {"bound": "mfma", "kernel": "k_nn_fwd (BF16 MFMA implicit GEMM)",
                           "boxes": nbox, "avg_launch_us": launch_s * 1e6,
                           "flop_per_cell": NN_FLOP_PER_CELL, "achieved": tflops,
                           "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": tflops / BF16_PEAK_TFLOPS}}


EFIELD_BYTES_PER_BOX = 8 * (512 + 3 * 9 * 64 + 512)  # read phi; write face components and |E|


def time_step_leg(g, args):
    """The solver as a time-stepped streamer run uses it (paper sections
    2.1.2 and 2.4): after the initial FMG solve, every field solve sets the
    new right-hand side, runs two V-cycles warm-started from the previous
    potential (mg_vcycle) and forms the electric field on every box
    (mg_efield); a time step holds two field solves.  The right-hand sides are
    the benchmark streamer with its head moved down by dz per field solve, on
    the same tree, generated beforehand and resident in HBM."""
    import numpy as np
    import torch
    from paper_1708_08434_amd import mg as M
    from workloads import c2_head_sequence
    nsolve = 2 * args.ts_steps
    dz = 2.5e-5  # 1 um of the paper's 40 mm domain per field solve
    lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
    seq = c2_head_sequence(lv, ij, nsolve + 3, dz)
    rhs = [torch.from_numpy(seq[s]).to("cuda:0") for s in range(nsolve + 3)]
    del seq
    face = torch.empty((g.n, 3, 9, 8, 8), dtype=torch.float64, device="cuda:0")
    norm = torch.empty((g.n, 8, 8, 8), dtype=torch.float64, device="cuda:0")
    # the time step's field solves: two V-cycles with no statistics (no
    # residual norm, no host wait: mg_vcycle with stats NULL); the residuals
    # before and after each solve come from an untimed replay with a check
    # around every cycle, which must end on the same phi bits
    opts = g.opts()
    M.mg_field_set(g.h, M.MG_FIELD_RHS, rhs[0].data_ptr())
    g.fmg_solve()

    def field_solve(s, stats):
        M.mg_field_set(g.h, M.MG_FIELD_RHS, rhs[s].data_ptr())
        st = M.mg_vcycle(g.h, opts, 2, stats=stats)
        M.mg_efield(g.h, face.data_ptr(), norm.data_ptr())
        return st
    for s in (1, 2):  # warm-up (records the V-cycle graphs)
        field_solve(s, False)
    phi_start = g.get_field(M.MG_FIELD_PHI)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(3, nsolve + 3):
        field_solve(s, False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phi_end = g.get_field(M.MG_FIELD_PHI)
    g.set_field(M.MG_FIELD_PHI, phi_start)
    rel0, rel2 = [], []
    for s in range(3, nsolve + 3):
        st = field_solve(s, True)
        rel0.append(st.rel_hist[0])
        rel2.append(st.rel_res)
    replay_same = bool(np.array_equal(phi_end, g.get_field(M.MG_FIELD_PHI)))
    # the field kernel alone, HIP events on the tree's stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(g.stream):
        e0.record()
        for _ in range(10):
            M.mg_efield(g.h, face.data_ptr(), norm.data_ptr())
        e1.record()
    torch.cuda.synchronize()
    ef_s = e0.elapsed_time(e1) / 1e3 / 10
    n_leaf = int(g.info.n_leaf_cells)
    gbps = EFIELD_BYTES_PER_BOX * g.n / ef_s / 1e9
    return {"field_solves_per_s": nsolve / el, "ms_per_field_solve": 1e3 * el / nsolve,
            "ms_per_time_step": 2e3 * el / nsolve, "vcycles_per_s": 2 * nsolve / el,
            "leaf_cells_per_s": n_leaf * nsolve / el, "field_solves": nsolve,
            "head_shift_per_solve": dz,
            "rel_res_before_max": max(rel0), "rel_res_after_2_vcycles_max": max(rel2),
            "checks": "none in the timed solves (no statistics requested); the residuals from "
                      "an untimed replay with a check around every cycle",
            "replay_same_phi": replay_same,
            "efield": {"kernel": "k_efield (face components + cell strength, all boxes)",
                       "boxes": g.n, "avg_launch_us": ef_s * 1e6,
                       "bytes_per_box": EFIELD_BYTES_PER_BOX, "achieved": gbps,
                       "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS}}


def regrid_leg(w, args, sched64):
    """Mesh adaptation as the streamer moves (paper section 2.5).  The
    benchmark tree is refined geometrically around the channel, more finely
    than its charge asks for, so it is first adapted to the charge (an
    untimed regrid step with c3 = 0.1 of the largest leaf-box score: leaf
    cells whose |b| h^2 exceeds 10% of the leaf peak keep or get the finest
    level).  Then the head
    moves down 2.5e-4 (10 um of the paper's 40 mm domain, a quarter of a
    finest cell) per field solve, each field solve runs two warm-started
    V-cycles, and every 2nd solve is preceded by a timed regrid step: GPU
    refinement scores reduced on the GPU to the criterion's per-box values
    (mg_refine_near), the host plan from those, the new tree (create + bind, with the
    benchmark tree's autotuned schedule) and the transfer of phi
    (mg_transfer).  The charge of each mesh is generated on the host and is
    not timed."""
    import torch
    from paper_1708_08434_amd import mg as M
    from workloads import c2_head_sequence
    dz, every, z0, deref = 2.5e-4, 2, 0.62, 0.125

    def tree(lv, ij, tr, split=None):
        t = M.Tree(lv, ij, tr, w.lo, w.length, w.bc_type, w.bc_val, bind=False)
        if split is not None:
            split.append(time.perf_counter())
        t.bind("cuda:0")
        if int(t.nlev) == len(sched64):
            M.mg_set_schedule(t.h, M.MG_FP64, sched64)
        return t

    def charge(t, s):
        lv, ij = t.index(M.MG_IDX_LEVEL), t.index(M.MG_IDX_IJK)
        t.set_field(M.MG_FIELD_RHS, c2_head_sequence(lv, ij, 1, dz, z_head=z0 - s * dz)[0])

    g0 = M.Tree.from_workload(w, device="cuda:0")
    charge(g0, 0)
    sc = g0.refine_scores()
    leaf = g0.leaf_mask()
    c3, max_level = 0.1 * float(sc[leaf, 13].max()), g0.nlev
    g = tree(*M.mg_regrid_plan(g0.h, sc, c3, deref, max_level))
    bench_boxes, adapted_boxes = g0.n, g.n
    del g0
    charge(g, 0)
    g.fmg_solve()
    opts = g.opts()
    regrids, vtimes, rel_after = [], [], []
    for s in range(1, args.regrid_steps + 1):
        fresh = s % every == 0
        if fresh:
            charge(g, s)  # the current charge on the current mesh
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            near = g.refine_near()
            t1 = time.perf_counter()
            plan = M.mg_regrid_plan_near(g.h, near, c3, deref, max_level)
            t2 = time.perf_counter()
            split = []
            g2 = tree(*plan, split=split)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            M.mg_transfer(g.h, g2.h)
            t4 = time.perf_counter()
            regrids.append({"solve": s, "boxes_before": g.n, "boxes_after": g2.n,
                            "leaf_cells_after": int(g2.info.n_leaf_cells),
                            "ms": {"scores": 1e3 * (t1 - t0), "plan": 1e3 * (t2 - t1),
                                   "create_bind": 1e3 * (t3 - t2), "create": 1e3 * (split[0] - t2),
                                   "bind": 1e3 * (t3 - split[0]), "transfer": 1e3 * (t4 - t3),
                                   "total": 1e3 * (t4 - t0)}})
            del g
            g = g2
        charge(g, s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.mg_vcycle(g.h, opts, 2, stats=False)  # no statistics: no residual norm, no host wait
        torch.cuda.synchronize()
        vtimes.append((1e3 * (time.perf_counter() - t0), fresh))
        rel_after.append(M.mg_residual(g.h)["rel"])  # untimed
    steady = [t for t, fresh in vtimes if not fresh]
    return {"c3": c3, "deref_factor": deref, "boxes_benchmark_tree": bench_boxes,
            "boxes_adapted": adapted_boxes, "head_shift_per_solve": dz, "regrid_every": every,
            "field_solves": len(vtimes), "regrids": regrids,
            "ms_regrid_median": statistics.median(r["ms"]["total"] for r in regrids) if regrids else None,
            "ms_2_vcycles_median": statistics.median(steady) if steady else None,
            "ms_2_vcycles_first_on_new_tree": [t for t, fresh in vtimes if fresh],
            "rel_res_after_2_vcycles_max": max(rel_after)}


FLUID_BYTES_PER_LEAF_BOX = 8 * (4 * 512 + 1728 + 512 + 3 * 512)


def fluid_leg(args, sched64):
    """The fluid model's time step (paper sections 2.2-2.4) on the benchmark tree in
    the paper's SI setup ((40 mm)^3, 80 kV): electron and ion densities of a
    perturbed 1e19 m^-3 blob at the streamer head over a 1e15 m^-3
    background, synthetic transport table (1000 entries up to 35 MV/m).
    Each step is the explicit trapezoidal rule with two warm-started
    V-cycles per field solve (mg_fluid_step); the step size follows the
    limits of the previous step.  The stage alone (restriction, refinement
    boundaries, update, bound) is timed with HIP events."""
    import numpy as np
    import torch
    from paper_1708_08434_amd import mg as M
    from workloads import paper_setup, synthetic_n2_table, EMAX
    w = paper_setup()
    g = M.Tree.from_workload(w, device="cuda:0")
    if int(g.nlev) == len(sched64):
        M.mg_set_schedule(g.h, M.MG_FP64, sched64)
    lv = g.index(M.MG_IDX_LEVEL).astype(np.float64)
    ij = g.index(M.MG_IDX_IJK).astype(np.float64)
    L = w.length
    h = L / (8.0 * 2.0 ** (lv - 1))
    c = (np.arange(8) + 0.5)
    x = (8 * ij[:, 0, None, None, None] + c[None, None, None, :]) * h[:, None, None, None]
    y = (8 * ij[:, 1, None, None, None] + c[None, None, :, None]) * h[:, None, None, None]
    z = (8 * ij[:, 2, None, None, None] + c[None, :, None, None]) * h[:, None, None, None]
    rng = np.random.default_rng(21)
    blob = 1e19 * np.exp(-((x - 0.5 * L) ** 2 + (y - 0.5 * L) ** 2 + (z - 0.62 * L) ** 2) / (0.03 * L) ** 2)
    ne = 1e15 + blob * (1.0 + 0.3 * rng.random(blob.shape))
    ni = 1e15 + 0.8 * blob
    g.set_field(M.MG_FIELD_RHS, -1.602176634e-19 * (ni - ne) / 8.8541878128e-12)
    g.fmg_solve()
    g.fluid_bind(synthetic_n2_table(), EMAX)
    Ne = torch.from_numpy(ne).to("cuda:0")
    Ni = torch.from_numpy(ni).to("cuda:0")
    del x, y, z, blob, ne, ni
    dt = 1e-12
    for _ in range(2):
        dt = M.mg_fluid_step(g.h, Ne.data_ptr(), Ni.data_ptr(), dt, 2)
    torch.cuda.synchronize()
    dts = []
    t0 = time.perf_counter()
    for _ in range(args.fluid_steps):
        dts.append(dt)
        dt = M.mg_fluid_step(g.h, Ne.data_ptr(), Ni.data_ptr(), dt, 2)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # one stage alone, on the tree's stream
    face, norm = g.efield(to_numpy=False)
    Oe, Oi = torch.empty_like(Ne), torch.empty_like(Ni)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    with torch.cuda.stream(g.stream):
        e0.record()
        for _ in range(reps):
            M.mg_fluid_stage(g.h, face.data_ptr(), norm.data_ptr(), Ne.data_ptr(), Ni.data_ptr(),
                             Ne.data_ptr(), Ni.data_ptr(), dt, 0.0, 1.0, Oe.data_ptr(), Oi.data_ptr(),
                             want_limit=False)
        e1.record()
    torch.cuda.synchronize()
    st_s = e0.elapsed_time(e1) / 1e3 / reps
    nleaf_box = int(g.info.n_leaf_cells) // 512
    gbps = FLUID_BYTES_PER_LEAF_BOX * nleaf_box / st_s / 1e9
    n_leaf = int(g.info.n_leaf_cells)
    return {"workload": "paper_setup_40mm (benchmark tree, SI units), perturbed head blob",
            "steps": args.fluid_steps, "ms_per_step": 1e3 * el / args.fluid_steps,
            "leaf_cells_per_s": n_leaf * args.fluid_steps / el,
            "dt_first": dts[0], "dt_last": dt, "n_e_max": float(Ne.max()),
            "stage": {"kernels": "k_fluid_restrict, k_fluid_cf, k_fluid_update, k_fluid_min",
                      "avg_us": st_s * 1e6, "leaf_boxes": nleaf_box,
                      "bytes_per_leaf_box": FLUID_BYTES_PER_LEAF_BOX, "achieved": gbps,
                      "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS}}


def parse_schedule(text, nlev, nvariants):
    """--schedule text: the FP64 list of launch variants per level, optionally
    '/' and the FP32 list; each list has nlev entries in 0..nvariants-1."""
    try:
        parts = [[int(v) for v in p.split(",")] for p in text.split("/")]
    except ValueError:
        parts = None
    if (not parts or len(parts) > 2
            or any(len(p) != nlev or not all(0 <= v < nvariants for v in p) for p in parts)):
        raise SystemExit(f"--schedule: one or two lists of {nlev} variants in 0..{nvariants - 1}, "
                         f"separated by '/', got {text!r}")
    return parts


def run_stats(run_s, n_leaf):
    """Median, minimum and maximum of individually timed solves."""
    med = statistics.median(run_s)
    return {"n": len(run_s), "median_ms": 1e3 * med, "min_ms": 1e3 * min(run_s),
            "max_ms": 1e3 * max(run_s), "median_cells_per_s": n_leaf / med,
            "best_cells_per_s": n_leaf / min(run_s)}


SOLVE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solve_traffic_{}.json")
DRIVER_SRC = os.path.join(ROOT, "paper_1708_08434_amd", "csrc", "mg_api.hip")


def solve_traffic(workload):
    """HBM bytes per FP64 FMG solve of this workload from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE summed over one
    solve's dispatches, scaled by the copy kernel's reading), or None if
    there is none or the kernels or the driver changed since."""
    path = SOLVE_TRAFFIC_FILE.format(workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read() + open(DRIVER_SRC, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("bytes_per_solve")


WORKLOAD_TEXT = {
    "uniform": " uniform 64^3 grid (levels 1-4 of 8^3 boxes, no refinement)",
    "streamer": " static streamer octree (base 64^3 + 4 refinement levels)",
    "forest": " forest of 128 uneven streamer trees (base 32^3 + <=5 levels)",
    "branched": " branched streamer octree (base 64^3 + 6 refinement levels)",
    "two_streamers": " two streamers + Poisson background (base 64^3 + 7 refinement levels)",
    "paper_setup": " streamer octree in SI units: (40 mm)^3, 80 kV top, grounded bottom, "
                   "Neumann sides"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed FMG solves (each also timed on its own: median and minimum)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction leg")
    ap.add_argument("--train-steps", type=int, default=300, help="Adam steps of the learned leg")
    ap.add_argument("--regrid-steps", type=int, default=16,
                    help="field solves of the regrid leg (a regrid every 2nd); 0 skips it")
    ap.add_argument("--ts-steps", type=int, default=8,
                    help="time steps (2 warm-started field solves each) of the time-stepping leg; "
                         "0 skips it")
    ap.add_argument("--copy-probe", type=int, default=0, help="bytes of a calibration copy")
    ap.add_argument("--fluid-steps", type=int, default=10,
                    help="time steps of the fluid leg (paper setup, SI units); 0 skips it")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only the launches that rocprofv3 --pmc counts for the traffic summary")
    ap.add_argument("--solve-traffic-probe", action="store_true",
                    help="only the launches that rocprofv3 --pmc counts for the traffic of one FP64 solve")
    ap.add_argument("--schedule", default=None,
                    help="fixed Gauss-Seidel launch variant per level instead of the autotuner: "
                         "FP64 list, optionally '/' and the FP32 list, e.g. 3,7,7,1,7,7,1,11/3,1,7,1,7,7,1,9 "
                         "(reproduces a tuned run's launches, e.g. under a profiler)")
    ap.add_argument("--fusion", type=int, default=None,
                    help="mg_set_fusion flags for the solves (default: all fused sequences)")
    ap.add_argument("--workload", default="two_streamers",
                    choices=["uniform", "streamer", "forest", "branched", "two_streamers", "paper_setup"],
                    help="two_streamers: base 64^3 + 7 levels, 1.2e8 cells (default); uniform: 64^3 "
                         "cells, no refinement; streamer: "
                         "base 64^3 + 4 levels, 4.8e6 cells; forest: 128 uneven trees, 7.1e7 "
                         "cells; branched: base 64^3 + 6 levels, 2.9e7 cells; paper_setup: the "
                         "streamer tree in the paper's SI setup (40 mm, 80 kV, Neumann sides)")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.exit("bench.py: measures one GPU only; the solver has no multi-GPU path "
                 "(sharding across GPUs is a design, not code).  Use --gpus 1.")
    rank = int(os.environ.get("RANK", "0"))

    import numpy as np
    import torch
    from paper_1708_08434_amd import mg as M
    from workloads import c1, c2, c3, c5, forest, paper_setup

    from paper_1708_08434_amd import autotune

    gen = {"uniform": c1, "streamer": c2, "forest": forest, "branched": c3, "two_streamers": c5,
           "paper_setup": paper_setup}
    w = gen[args.workload]()
    if args.traffic_probe:
        traffic_probe(w)
        return
    if args.solve_traffic_probe:
        solve_traffic_probe(w, args.schedule, args.fusion)
        return
    g = M.Tree.from_workload(w, device="cuda:0")
    if args.fusion is not None:
        M.mg_set_fusion(g.h, args.fusion)
    order = g.index(M.MG_IDX_ORDER)
    rhs = w.rhs(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK), g.index(M.MG_IDX_TREE))
    g.set_field(M.MG_FIELD_RHS, rhs)
    torch.cuda.synchronize()
    log(f"{w.name}, {g.n} boxes, {int(g.info.n_leaf_cells)} leaf cells")
    if args.schedule:
        parts = parse_schedule(args.schedule, g.nlev, M.MG_GSRB_VARIANTS)
        sched64 = parts[0]
        M.mg_set_schedule(g.h, M.MG_FP64, sched64)
        if len(parts) > 1:
            sched32 = parts[1]
            M.mg_set_schedule(g.h, M.MG_MIXED, sched32)
        else:
            sched32, _ = autotune.tune(g, M.MG_MIXED)
    else:
        sched64, _ = autotune.tune(g, M.MG_FP64)
        sched32, _ = autotune.tune(g, M.MG_MIXED)
    log("schedules", sched64, sched32)
    for _ in range(args.warmup):
        g.fmg_solve()
    # timed region 1: the solve as shipped (recorded graphs replayed); every
    # solve returns after its last residual check has been read back, so it
    # is also timed on its own
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, run_s = None, []
    for _ in range(args.steps):
        t_run = time.perf_counter()
        stats = g.fmg_solve()
        run_s.append(time.perf_counter() - t_run)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    results = {"fp64": g.get_field(M.MG_FIELD_PHI)}
    # timed region 2: the same solves with HIP-event probes around the
    # Gauss-Seidel half-sweeps on the library's stream (kernel-by-kernel
    # launches, since events inside replayed graphs carry no usable times)
    M.mg_timing_read(g.h)
    M.mg_timing_enable(g.h, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g.fmg_solve()
    torch.cuda.synchronize()
    elapsed_probe = time.perf_counter() - t1
    M.mg_timing_enable(g.h, False)
    kt = M.mg_timing_read(g.h)
    n_leaf = int(g.info.n_leaf_cells)
    log("fp64 solves done")
    mixed = None
    if not args.no_mixed:
        for _ in range(args.warmup):
            g.fmg_solve(precision=M.MG_MIXED)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        mrun = []
        for _ in range(args.steps):
            t_run = time.perf_counter()
            ms_stats = g.fmg_solve(precision=M.MG_MIXED)
            mrun.append(time.perf_counter() - t_run)
        torch.cuda.synchronize()
        el_m = time.perf_counter() - t2
        results["mixed"] = g.get_field(M.MG_FIELD_PHI)
        mixed = {"value": n_leaf * args.steps / el_m, "unit": "cells/s",
                 "ms_per_step": 1e3 * el_m / args.steps, "runs": run_stats(mrun, n_leaf),
                 "refinement_steps": ms_stats["n_vcycles"], "final_rel_res": ms_stats["rel"],
                 "launches": {"start_and_fmg": ms_stats["launches_fmg"],
                              "per_refinement_step": ms_stats["launches_cycle"]}}
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ls = list(g.info.level_start[:g.nlev + 1])
    counts = [ls[i + 1] - ls[i] for i in range(g.nlev)]
    ms = 1e3 * elapsed / args.steps
    value = n_leaf * args.steps / elapsed
    k = stats["n_vcycles"]
    learned = None
    if not args.no_learned:
        log("learned leg")
        results["learned"], results["learned_per_level"], learned = learned_leg(g, args, k, value)
    copy = copy_bandwidth()
    mb = model_bytes(counts, n_leaf, k)
    # the level whose half-sweeps move the most bytes (the finest level of a
    # single streamer tree; a middle level of the forest)
    fin = max(range(g.nlev), key=lambda l: kt["level_bytes"][l])
    per_launch_s = kt["level_ms"][fin] / 1e3 / max(kt["level_launches"][fin], 1)
    bytes_per_launch = kt["level_bytes"][fin] / max(kt["level_launches"][fin], 1)
    achieved = bytes_per_launch / per_launch_s / 1e9
    all_us = kt["total_ms"] * 1e3 / max(kt["launches"], 1)
    tr = traffic_per_launch(w.name, fin + 1, sched64[fin])
    model_gbps = mb / (ms / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name + WORKLOAD_TEXT[args.workload],
                   "n_trees": int(g.info.n_trees),
                   "n_leaf": n_leaf, "n_boxes": g.n, "levels": g.nlev, "rel_tol": 1e-8,
                   "vcycles_after_fmg": k, "final_rel_res": stats["rel"], "precision": "fp64",
                   "launches": {"fmg_with_check": stats["launches_fmg"],
                                "per_vcycle_with_check": stats["launches_cycle"],
                                "per_solve": stats["launches_fmg"] + k * stats["launches_cycle"]},
                   "smoothing": "V(2,2) red-black Gauss-Seidel",
                   "fusion": M.MG_FUSE_ALL if args.fusion is None else args.fusion,
                   "gsrb_schedule": {"fp64": sched64, "fp32": sched32}},
        "runs": run_stats(run_s, n_leaf),
        "hist": [float(v) for v in stats["hist"]],
        # solve level: the per-sweep byte model of the FMG solve (127 B per
        # stored cell per V(2,2) visit, FMG summed over the top levels, 16 B
        # per leaf cell per residual check) over the solve time
        "roofline": {"bound": "hbm", "scope": "FP64 FMG solve (all kernels), per-sweep byte model",
                     "achieved": model_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": model_gbps / HBM_PEAK_GBPS, "traffic": solve_traffic(w.name),
                     "alg_bytes_per_solve": mb,
                     "copy_GBps": copy["GBps"], "frac_of_copy": model_gbps / copy["GBps"]},
        "dominant_kernel": {
            "bound": "hbm",
            "kernel": gsrb_kernel_name(sched64[fin])
                      + f", level {fin + 1} ({counts[fin]} boxes, the most bytes), "
                        f"schedule variant {sched64[fin]}",
            "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "copy_GBps": copy["GBps"], "frac_of_copy": achieved / copy["GBps"],
            "traffic": tr,
            "launches": kt["level_launches"][fin], "avg_launch_us": per_launch_s * 1e6,
            "alg_bytes_per_launch": bytes_per_launch,
            "all_levels": {"launches": kt["launches"], "avg_launch_us": all_us,
                           "GBps": kt["alg_bytes"] / (kt["total_ms"] / 1e3) / 1e9},
            "probe_region_ms_per_step": 1e3 * elapsed_probe / args.steps},
        "model": {"bytes_per_solve": mb, "GBps": model_gbps,
                  "roofline_cells_per_s": HBM_PEAK_GBPS * 1e9 * n_leaf / mb,
                  "frac": value / (HBM_PEAK_GBPS * 1e9 * n_leaf / mb),
                  "frac_of_copy": value / (copy["GBps"] * 1e9 * n_leaf / mb)},
        "copy_probe": copy,
    }
    if mixed is not None:
        mixed["vs_fp64"] = mixed["value"] / value
        out["mixed"] = mixed
    if learned is not None:
        out["learned"] = learned
    if args.workload == "paper_setup":
        g.fmg_solve()
        _, en = g.efield()
        leaf = g.leaf_mask()
        out["field"] = {"background_V_per_m": w.meta["e0"], "max_E_V_per_m": float(en[leaf].max()),
                        "max_E_over_background": float(en[leaf].max() / w.meta["e0"]),
                        "n_head_per_m3": w.meta["n_head"]}
    del g
    torch.cuda.empty_cache()
    # secondary legs on the static streamer tree (base 64^3 + 4 levels)
    w2 = g2 = None
    if args.ts_steps > 0 or args.regrid_steps > 0 or args.fluid_steps > 0 or not args.no_cpu:
        w2 = w if args.workload == "streamer" else c2()
    if args.ts_steps > 0 or args.regrid_steps > 0 or args.fluid_steps > 0:
        g2 = M.Tree.from_workload(w2, device="cuda:0")
        g2.set_rhs_from(w2)
        if args.workload == "streamer":
            s2 = sched64
            M.mg_set_schedule(g2.h, M.MG_FP64, s2)
        else:
            s2, _ = autotune.tune(g2, M.MG_FP64)
        g2.fmg_solve()
        sec = {"workload": w2.name + WORKLOAD_TEXT["streamer"], "n_leaf": w2.n_leaf}
        log("secondary legs on", w2.name)
        if args.ts_steps > 0:
            out["time_step"] = dict(sec, **time_step_leg(g2, args))
        if args.regrid_steps > 0:
            out["regrid"] = dict(sec, **regrid_leg(w2, args, s2))
        if args.fluid_steps > 0:
            out["fluid"] = fluid_leg(args, s2)
        del g2
        torch.cuda.empty_cache()
    if rank == 0 and not args.no_cpu:
        small = w2 if (w2 is not None and w2 is not w) else None
        log("cpu baseline")
        base, acc = cpu_baseline(w, rhs, order, k, results, small=small)
        out["cpu_baseline"] = base
        out["accuracy"] = acc
        for name, key in (("mixed", "mixed"), ("learned", "learned")):
            if key in out and name in acc:
                out[key]["rel_l2_vs_oracle_reference"] = acc[name]["rel_l2_vs_reference"]
        if "learned" in out and "learned_per_level" in acc:
            out["learned"]["per_level"]["rel_l2_vs_oracle_reference"] = \
                acc["learned_per_level"]["rel_l2_vs_reference"]
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
