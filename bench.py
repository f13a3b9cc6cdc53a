"""Benchmark of the ADMoM NTF hot path on one MI355X.

A step is one outer ADMoM iteration (three mode updates: MTTKRP, Gram
Hadamard product, FP64 Cholesky, fused inner sweep) over a synthetic planted
tensor resident in HBM.  Default workload: 1000 x 800 x 600 tensor of F = 64
Exponential(1) planted factors at 30 dB SNR, 10 inner iterations, in the
mixed-precision arm (BF16 MTTKRP with FP32 accumulation, FP32 Gram, FP64
Cholesky/solves); the FP32 arm is timed beside it.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c1|c5|s1|n4] [--no-ttt]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: dims, F, factor distribution, SNR dB, clip, inner iterations, arms
    "c1": dict(dims=(40, 40, 40), F=5, dist="uniform", snr=20.0, clip=True, T=5, config=1,
               arms=("fp64",)),
    "c2": dict(dims=(400, 400, 400), F=20, dist="uniform", snr=20.0, clip=False, T=10, config=2,
               arms=("fp32", "mixed")),
    "c3": dict(dims=(1000, 800, 600), F=64, dist="exponential", snr=30.0, clip=False, T=10,
               config=3, arms=("mixed", "fp32")),
    # sparse: dims, solver rank F, about nnz distinct non-zeros drawn with a skewed
    # (power-law-like) slice distribution, values from a rank-`planted` model
    "s1": dict(dims=(12092, 9184, 28818), F=32, nnz=76_000_000, planted=8, skew=2.0, T=10, config=6,
               arms=("fp32",)),
    # order N: a dense four-way tensor (Appendix A)
    "n4": dict(dims=(120, 110, 100, 90), F=32, dist="uniform", snr=20.0, T=10, config=7, arms=("fp32",)),
    # batched: n tensors, every mode uniform on [lo, hi], F uniform on 5..40
    "c5": dict(n=256, lo=50, hi=500, ranks=tuple(range(5, 41)), dist="uniform", snr=20.0,
               clip=False, T=10, config=5, arms=("mixed",)),
}

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The MTTKRP kernels whose HBM traffic the committed counter runs measured
# live in these sources; a change to them voids the stored traffic figures.
MTTKRP_SOURCES = ("mttkrp.hip", "ntf_device.h")


def src_hash(files=None):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1409_2383_amd", "csrc")
    for f in sorted(files or os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def make_solver(ntf, torch, Xd, H0, arm, T, dev, warm_hidden=0, H=None, U=None, workspace=None):
    prec = {"fp32": ntf.PREC_F32, "mixed": ntf.PREC_BF16_MIXED, "fp64": ntf.PREC_F64}[arm]
    fdt = torch.float64 if arm == "fp64" else torch.float32
    if H is None:
        H = [torch.from_numpy(h).to(dev, dtype=fdt) for h in H0]
    X = Xd.to(fdt) if Xd.dtype != fdt else Xd
    return ntf.NtfAdmm(X, H, U=U, workspace=workspace,
                       opts=ntf.AdmmOptions(inner_iters=T, precision=prec,
                                            warm_hidden=warm_hidden)), H


def time_steps(torch, solver, steps, warmup):
    for _ in range(warmup):
        solver.step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        solver.step()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_passes(torch, solver, reps):
    """Average duration of each MTTKRP kernel launched on its own (HIP events
    on the stream the library launches on: torch's current stream)."""
    s = torch.cuda.current_stream()
    out = {}
    for name, which in (("pass1", 0), ("mode2", 1), ("pass3", 2)):
        solver.launch_pass(which)          # warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            solver.launch_pass(which)
        e1.record(s)
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps   # ms
    return out


def blas_info():
    """BLAS library numpy uses and its thread count, and the host cores this
    process may run on."""
    info = {"affinity_cores": len(os.sched_getaffinity(0)), "blas": None, "blas_threads": None}
    try:
        from threadpoolctl import threadpool_info
        for lib in threadpool_info():
            if lib.get("user_api") == "blas":
                info["blas"] = f"{lib.get('internal_api')} {lib.get('version')}"
                info["blas_threads"] = int(lib.get("num_threads", 1))
                break
    except Exception:
        pass
    return info


def cpu_baseline(X, H0, T, sample_slabs, min_seconds=10.0, max_iters=5):
    """The FP64 oracle (as it stands) on the host: outer iterations over the
    first `sample_slabs` mode-1 slabs of the same tensor (all of them by
    default), repeated until `min_seconds` have passed, scaled to the full
    tensor by the slab ratio (MTTKRP work is linear in I)."""
    from oracle import ntf_oracle as orc
    bi = blas_info()
    I = X.shape[0]
    S = min(I, sample_slabs) if sample_slabs > 0 else I
    Xs = np.ascontiguousarray(X[:S], dtype=np.float64)
    st = orc.init_state([H0[0][:S].astype(np.float64), H0[1].astype(np.float64),
                         H0[2].astype(np.float64)])
    opts = orc.Opts(inner_iters=T)
    n = 0
    t0 = time.perf_counter()
    while True:
        orc.outer_step(Xs, st, opts)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or n >= max_iters:
            break
    per_iter = dt / n * I / S
    where = f"all {I}" if S == I else f"the first {S} of {I}"
    return {"value": 1.0 / per_iter, "unit": "outer_iters/s",
            "cores": bi["blas_threads"] or bi["affinity_cores"], "kind": "oracle",
            "sample": f"{n} outer iteration(s) (T={T}) of the FP64 oracle on {where} mode-1 slabs "
                      f"of the same tensor ({dt:.1f} s)" + ("" if S == I else f", scaled by {I}/{S}"),
            "seconds_measured": dt, "blas": bi["blas"], "affinity_cores": bi["affinity_cores"]}


def copy_calibration(torch, dev, mib, reps=3):
    """Launches a plain elementwise copy-type kernel (negation: reads and writes
    exactly `mib` MiB each) so that hardware byte counters taken in the same
    run can be scaled against a known transfer."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {reps} x neg over {mib} MiB")
    del src, dst


def load_rfe_star(workload):
    """RFE* of the workload from the FP64 oracle's converged run, stored by
    tests/golden/make_golden.py (None if that file is absent)."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_rfe_star.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    return {"rfe_star": g["rfe_star"],
            "source": f"FP64 oracle run to {g['stop']} ({g['outer_iters']} outer iterations; "
                      f"tests/golden/{os.path.basename(path)})",
            "exact_iters": g.get("exact_iters_to_rel_1e-4")}


def time_to_target(torch, ntf, Xd, H0, T, arms, dev, star, max_outer=400, tol=1e-4, warm=None):
    """Time for each arm to reach (RFE - RFE*)/RFE* <= tol.  The clock
    (HIP events on the stream the library launches on) covers the arm's
    set-up on the device (BF16 copies of X, graph capture, which happen in
    the first step) and every outer iteration up to the first whose RFE meets
    the target; the RFE is evaluated after every iteration, outside the
    clock.  `warm` maps an arm name to a warm-start network (an ntf.Mlp-like
    argument for set_warmstart) and its one-off cost in ms."""
    rfe_star = star["rfe_star"]
    res = {"rfe_star": rfe_star, "rfe_star_source": star["source"], "target_rel": tol,
           "check_every": 1}
    s = torch.cuda.current_stream()
    # untimed: a few steps of every arm first, so the clock does not include the
    # GPU coming out of an idle state (the host-side CPU baseline may run before);
    # this also gives each arm's workspace size, allocated before its clock starts
    ws_bytes = {}
    for arm in arms:
        base = "mixed" if arm.startswith("mixed") else arm
        solver, H = make_solver(ntf, torch, Xd, H0, base, T, dev,
                                warm_hidden=(warm[arm]["hidden"] if warm and arm in warm else 0))
        ws_bytes[arm] = solver.workspace.numel()
        for _ in range(5):
            solver.step()
        torch.cuda.synchronize()
        solver.close()
        del solver, H
    for arm in arms:
        base = "mixed" if arm.startswith("mixed") else arm
        # device memory (workspace, factors, duals) is allocated before the clock
        # starts; the clock covers the set-up work on the device (bfloat16 copies,
        # norms, Grams, the graph capture in the first step) and the iterations
        fdt = torch.float64 if base == "fp64" else torch.float32
        Hb = [torch.from_numpy(h).to(dev, dtype=fdt) for h in H0]
        Ub = [torch.zeros_like(h) for h in Hb]
        wsb = torch.empty(ws_bytes[arm], dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        # (untimed: about 5 ms of device work queued right before the clock
        # starts, so the arm's set-up does not start on a GPU that went idle
        # during the host-side allocations; one run had its first ten steps
        # at twice the usual time without it)
        spin = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        for _ in range(80):
            spin.mul_(1.0000001)
        del spin
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        solver, H = make_solver(ntf, torch, Xd, H0, base, T, dev,
                                warm_hidden=(warm[arm]["hidden"] if warm and arm in warm else 0),
                                H=Hb, U=Ub, workspace=wsb)
        extra_ms = 0.0
        if warm and arm in warm:
            warm[arm]["attach"](solver)
            extra_ms = warm[arm].get("setup_ms", 0.0)
        solver.step()
        e1.record(s)
        torch.cuda.synchronize()
        init_ms = e0.elapsed_time(e1) + extra_ms
        total_ms, it = init_ms, 1
        r = solver.fit()
        hit = (it, total_ms, r) if (r - rfe_star) / rfe_star <= tol else None
        trace = [(it, total_ms, r)]
        while hit is None and it < max_outer:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            solver.step()
            e1.record(s)
            torch.cuda.synchronize()
            total_ms += e0.elapsed_time(e1)
            it += 1
            r = solver.fit()
            trace.append((it, total_ms, r))
            if (r - rfe_star) / rfe_star <= tol:
                hit = (it, total_ms, r)
        taken = None
        if warm and arm in warm:
            # (untimed, after the run) rows the judge started from the network in one more step
            taken = [int(v) for v in solver.step(stats=True)["warm_taken"]]
        res[arm] = {"reached": hit is not None, "outer_iters": hit[0] if hit else None,
                    "ms": hit[1] if hit else None, "init_and_first_step_ms": init_ms,
                    "rfe": r, "rel_to_star": (r - rfe_star) / rfe_star,
                    "rel_before": ((trace[-2][2] - rfe_star) / rfe_star) if len(trace) > 1 else None,
                    "trace_every_10": [t for t in trace if t[0] % 10 == 0 or t[0] == 1]}
        if taken is not None:
            res[arm]["warm_rows_taken_next_step"] = taken
        log(f"[bench] ttt {arm}: " + (f"{hit[0]} outer iterations, {hit[1]:.1f} ms" if hit else
                                       f"not reached in {max_outer} (rel {(r - rfe_star) / rfe_star:.2e})"))
        solver.close()
        del solver, H, Hb, Ub, wsb
    return res


def warm_arm(torch, ntf, log):
    """The F = 64 warm-start network for the mixed arm, trained by the
    library's kernels on pairs from small planted tensors of the same kind."""
    import ctypes
    from paper_1409_2383_amd import _lib, warmstart as ws
    t0 = time.perf_counter()
    net = ws.train_rank64(log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    st = net.struct(True)

    def attach(solver):
        _lib.check(_lib.lib().ntf_admm_set_warmstart(solver._ctx, ctypes.byref(st)),
                   "set_warmstart", solver._ctx)
    return {"mixed+mlp": {"hidden": net.hidden, "attach": attach, "setup_ms": 0.0,
                          "net": net}}, train_s


PASS_KERNELS = {"pass1": "k_pass1", "mode2": "k_mode2", "pass3": "k_pass3"}


def _counter_means(path):
    import collections
    import csv
    agg = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def write_traffic(fetch_csv, write_csv, calib_mib, workload, arm, pass_bytes, cmd):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch) into HBM bytes per launch of each MTTKRP kernel.  Each counter is
    scaled by what it reads for the copy-calibration kernel, which reads and
    writes exactly `calib_mib` MiB per launch."""
    fetch, write = _counter_means(fetch_csv), _counter_means(write_csv)

    def find(tab, needle, counter):
        hits = [(v, k[0]) for k, v in tab.items() if needle in k[0] and k[1] == counter]
        if len(hits) != 1:
            raise SystemExit(f"expected one kernel matching {needle!r} for {counter}, got {len(hits)}")
        return hits[0][0][0], hits[0][1]
    kib = calib_mib * 1024.0
    f_cal, _ = find(fetch, "neg_kernel", "FETCH_SIZE")
    w_cal, _ = find(write, "neg_kernel", "WRITE_SIZE")
    f_scale, w_scale = f_cal / kib, w_cal / kib
    tag = src_hash(MTTKRP_SOURCES)
    lines = [f"# HBM traffic per launch, {workload} {arm} arm", "",
             "Commands (run from the repository root, NTF_NO_GRAPH=1):", "",
             "    " + cmd.replace("COUNTER", "FETCH_SIZE").replace("OUT", "pmc_fetch"),
             "    " + cmd.replace("COUNTER", "WRITE_SIZE").replace("OUT", "pmc_write"), "",
             f"Copy calibration (elementwise negation, {calib_mib} MiB read + {calib_mib} MiB "
             f"written per launch): FETCH_SIZE reads {f_cal:.0f} KiB (scale {f_scale:.4f}), "
             f"WRITE_SIZE reads {w_cal:.0f} KiB (scale {w_scale:.4f}).", "",
             "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | algorithmic bytes "
             "| traffic / algorithmic |", "|---|---|---|---|---|---|"]
    out = {}
    for name, needle in PASS_KERNELS.items():
        fk, full = find(fetch, needle, "FETCH_SIZE")
        wk, _ = find(write, needle, "WRITE_SIZE")
        nbytes = fk * 1024.0 / f_scale + wk * 1024.0 / w_scale
        out[name] = {"kernel": full, "fetch_kib": fk, "write_kib": wk, "bytes_per_launch": nbytes,
                     "algorithmic_bytes": pass_bytes[name], "src_hash": tag,
                     "fetch_scale": f_scale, "write_scale": w_scale}
        lines.append(f"| {name} (`{full[:48]}`) | {fk:.0f} | {wk:.0f} | {nbytes / 1e9:.4f} GB | "
                     f"{pass_bytes[name] / 1e9:.4f} GB | {nbytes / pass_bytes[name]:.3f} |")
        with open(os.path.join(ROOT, "profiles", f"traffic_{workload}_{arm}_{name}.json"), "w") as fh:
            json.dump(out[name], fh, indent=1)
    lines += ["", f"Source hash of the kernels measured: `{tag}`.", ""]
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}_{arm}.md"), "w") as fh:
        fh.write("\n".join(lines))
    return out


MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F32",
                 "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def write_mfma(pmc_csv, workload, arm, pass_ms, pass_flops, cmd):
    """Turns a rocprofv3 --pmc run of MFMA_COUNTERS into per-launch MFMA work of
    each MTTKRP kernel: flops = MOPS x 512 (rocprofv3's MfmaFlops* definition),
    busy fraction = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs)
    (its MfmaUtil), achieved TFLOP/s = counted flops / the kernel's average time
    from the same workload's timing run.  GRBM_GUI_ACTIVE comes summed over the
    eight XCDs in the per-dispatch CSV (about 8 x 2.2 GHz x the kernel time), so
    the busy fraction divides it by 8 (the counter's per-XCD maximum in
    MfmaUtil's definition)."""
    tab = _counter_means(pmc_csv)
    peak = {"mixed": 2500.0, "fp32": 157.3}[arm]
    dtype = {"mixed": "BF16", "fp32": "F32"}[arm]
    lines = [f"# MFMA work per launch, {workload} {arm} arm", "",
             "Command (run from the repository root, NTF_NO_GRAPH=1):", "", "    " + cmd, "",
             f"Dense {dtype} MFMA peak of MI355X: {peak} TFLOP/s.  Counted flops are what the",
             "MFMA instructions issued (padding and, in mixed pass 3, both bfloat16 terms",
             "included); algorithmic flops are 2 IJK F per MTTKRP (mixed pass 3: two terms).", "",
             "| kernel | MOPS (x512 flops) | counted GFLOP | algorithmic GFLOP | avg ms | achieved TFLOP/s "
             "| frac of peak | MFMA busy fraction (counters) |", "|---|---|---|---|---|---|---|---|"]
    out = {}
    for name, needle in PASS_KERNELS.items():
        if name == "mode2":
            continue
        vals = {c: [v for k, v in tab.items() if needle in k[0] and k[1] == c] for c in MFMA_COUNTERS}
        if any(len(v) != 1 for v in vals.values()):
            raise SystemExit(f"expected one kernel matching {needle!r}: {vals}")
        mops = vals[f"SQ_INSTS_VALU_MFMA_MOPS_{dtype}"][0][0]
        busy = vals["SQ_VALU_MFMA_BUSY_CYCLES"][0][0] / (vals["GRBM_GUI_ACTIVE"][0][0] / 8.0 * 1024.0)
        flops = mops * 512.0
        tf = flops / (pass_ms[name] * 1e-3) / 1e12
        out[name] = {"mops": mops, "flops": flops, "algorithmic_flops": pass_flops[name],
                     "avg_ms": pass_ms[name], "tflops": tf, "frac": tf / peak, "busy": busy}
        lines.append(f"| {name} | {mops:.4g} | {flops / 1e9:.1f} | {pass_flops[name] / 1e9:.1f} | "
                     f"{pass_ms[name]:.4f} | {tf:.1f} | {tf / peak:.3f} | {busy:.3f} |")
    lines += ["", f"Source hash of the kernels measured: `{src_hash(MTTKRP_SOURCES)}`.", ""]
    with open(os.path.join(ROOT, "profiles", f"mfma_{workload}_{arm}.md"), "w") as fh:
        fh.write("\n".join(lines))
    return out


def write_kernel_stats(stats_csv, workload, arm, cmd):
    """Short text summary of a rocprofv3 --kernel-trace --stats run."""
    import csv
    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    lines = [f"# Kernel time, {workload} {arm} arm", "", "Command (from /tmp, TMPDIR=/tmp):", "",
             "    " + cmd, "", "| kernel | calls | average us | min us | max us | share % |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:64]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    lines += ["", f"Source hash of the kernels measured: `{src_hash()}`.", ""]
    with open(os.path.join(ROOT, "profiles", f"kernels_{workload}_{arm}.md"), "w") as fh:
        fh.write("\n".join(lines))


def summarize(args):
    wl = WORKLOADS[args.workload]
    arm = args.arm or wl["arms"][0]
    if args.write_kernel_stats:
        # the traced run's own flags: pass the same --steps/--warmup/--pass-reps here
        cmd = (f"rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- python3 "
               f"<repo>/bench.py --workload {args.workload} --steps {args.steps} --warmup {args.warmup} "
               f"--pass-reps {args.pass_reps} --no-cpu-baseline"
               + ("" if args.workload in ("s1", "n4") else
                  (f" --arm {args.arm}" if args.arm else " --single-arm")))
        write_kernel_stats(args.write_kernel_stats, args.workload, arm, cmd)
    if args.write_mfma:
        csv_path, timing_json = args.write_mfma
        with open(timing_json) as fh:
            tj = json.loads(fh.read().strip().splitlines()[-1])
        pass_ms = tj["arms"][arm]["pass_ms"]
        I, J, K = wl["dims"]
        F = wl["F"]
        alg = 2.0 * I * J * K * F
        pass_flops = {"pass1": alg, "pass3": alg * (2 if arm == "mixed" else 1)}
        cmd = (f"timeout -s KILL 180 rocprofv3 --pmc {' '.join(MFMA_COUNTERS)} --output-format csv "
               f"-d gpurun_out/pmc_mfma_{arm} -o run -- python3 bench.py --workload {args.workload} "
               f"--steps 2 --warmup 1 --pass-reps 3 --no-cpu-baseline --no-ttt --arm {arm}")
        write_mfma(csv_path, args.workload, arm, pass_ms, pass_flops, cmd)
    if args.write_traffic:
        import paper_1409_2383_amd as ntf
        if args.copy_calib_mib <= 0:
            raise SystemExit("--write-traffic needs --copy-calib-mib (the size the runs used)")
        prec = {"fp32": ntf.PREC_F32, "mixed": ntf.PREC_BF16_MIXED, "fp64": ntf.PREC_F64}[arm]
        nb = ntf.pass_bytes(wl["dims"], wl["F"], prec, 8 if arm == "fp64" else 4)
        cmd = (f"timeout -s KILL 180 rocprofv3 --pmc COUNTER --output-format csv -d gpurun_out/OUT "
               f"-o run -- python3 bench.py --workload {args.workload} --steps 2 --warmup 1 "
               f"--pass-reps 3 --no-cpu-baseline --single-arm --copy-calib-mib {args.copy_calib_mib}")
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.copy_calib_mib,
                      args.workload, arm, nb, cmd)


def _gen_tensor(args):
    import ntf_synth
    dims, F, seed, snr = args
    pt = ntf_synth.planted(dims, F, seed, snr_db=snr, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    return pt.X, H0


def bench_batched(args):
    """Batched workload: many planted tensors of uneven shapes factorised
    together (one persistent kernel per outer iteration).  value = problem
    outer iterations per second over the whole batch."""
    import concurrent.futures as cf
    import torch
    import ntf_synth
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    n = args.batch_n or wl["n"]
    base = ntf_synth.config_seed(wl["config"])
    shapes = ntf_synth.batch_shapes(n, base, wl["lo"], wl["hi"], wl["ranks"])
    jobs = [(dims, F, ntf_synth.config_seed(wl["config"], t), wl["snr"]) for t, (dims, F) in enumerate(shapes)]
    log(f"[bench] generating {n} tensors (modes {wl['lo']}..{wl['hi']}, F 5..40)")
    t0 = time.perf_counter()
    Xs, Hs = [], []
    # threads of this process (numpy releases the GIL in its matrix products
    # and bulk random draws): a profiled run then holds one process only
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(workers) as pool:
        for t, (X, H0) in enumerate(pool.map(_gen_tensor, jobs)):
            Xs.append(torch.from_numpy(X).to(dev))
            Hs.append([torch.from_numpy(h).to(dev) for h in H0])
            if (t + 1) % 64 == 0:
                log(f"[bench] {t + 1}/{n} tensors on the device ({time.perf_counter() - t0:.0f} s)")
    T = wl["T"]
    opts = ntf.AdmmOptions(inner_iters=T, precision=ntf.PREC_BF16_MIXED)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b = ntf.NtfBatch(Xs, Hs, opts=opts)
    init_s = time.perf_counter() - t1
    tiles = None
    if not args.no_tune:
        t1 = time.perf_counter()
        tiles = b.autotune(reps=2)
        log(f"[bench] autotuned {len(tiles)} buckets in {time.perf_counter() - t1:.1f} s")
    info = b.info()
    log(f"[bench] batch ready: {info}")
    s = torch.cuda.current_stream()
    b.step(args.warmup)
    b.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    b.step(args.steps)
    e1.record(s)
    flags = b.sync()
    ms = e0.elapsed_time(e1) / args.steps
    # pass-only launches of the whole batch (the persistent kernel with one kind)
    pass_ms = {}
    for name, kind in (("pass1", b.KIND_PASS1), ("mode2", b.KIND_MODE2), ("pass3", b.KIND_PASS3)):
        b.launch_kind(kind)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(args.pass_reps):
            b.launch_kind(kind)
        e1.record(s)
        torch.cuda.synchronize()
        pass_ms[name] = e0.elapsed_time(e1) / args.pass_reps
    nbytes = {"pass1": info["x_bytes"] + info["t_bytes"], "mode2": info["t_bytes"],
              "pass3": info["x_bytes"]}
    gbs = {k: nbytes[k] / (pass_ms[k] * 1e-3) / 1e9 for k in pass_ms}
    prof = b.profile()          # one more outer iteration, instrumented per item kind
    fits = b.fit()
    dom = max(("pass1", "pass3"), key=lambda k: pass_ms[k])
    # algorithmic bytes of one MTTKRP of every problem: one read of each BF16 tensor copy
    ach = info["x_bytes"] / (pass_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": f"k_batch ({dom} items only)",
                "algorithmic_bytes_per_launch": info["x_bytes"],
                "kernel_bytes_per_launch": nbytes[dom], "avg_launch_ms": pass_ms[dom]}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batched(jobs, T, shapes)
    b.close()
    line = {
        "metric": "NTF outer iters/s + MTTKRP GB/s (% HBM peak), mixed vs FP32 at rel fit 1e-4",
        "value": n * 1e3 / ms, "unit": "problem_outer_iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"batch of {n} planted tensors, modes uniform {wl['lo']}-{wl['hi']}, "
                               f"F uniform 5-40, {wl['snr']:.0f} dB, T={T}, BF16 MTTKRP",
                   "n_tensors": n, "inner_iters": T},
        "roofline": roofline, "cpu_baseline": cpu,
        "batch": {"init_s": init_s, "info": info, "tiles": tiles, "pass_ms": pass_ms, "pass_gbs": gbs,
                  "flags": flags, "rfe_after": {"min": float(fits.min()), "median": float(np.median(fits)),
                                                "max": float(fits.max())},
                  "outer_iters_done": args.warmup + args.steps + 1,
                  "profile_one_iteration": prof},
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_batched(jobs, T, shapes, min_seconds=10.0):
    """The FP64 oracle on the host: one outer iteration per tensor over the
    first tensors of the batch (regenerated from their seeds) until
    min_seconds of oracle time have passed, scaled to the whole batch by
    MTTKRP work (sum of I J K F)."""
    from oracle import ntf_oracle as orc
    bi = blas_info()
    cores = bi['blas_threads'] or bi['affinity_cores']
    work = [d[0] * d[1] * d[2] * F for d, F in shapes]
    done, used, dt = 0.0, 0, 0.0
    for job in jobs:
        X, H0 = _gen_tensor(job)
        X64 = X.astype(np.float64)
        st = orc.init_state([h.astype(np.float64) for h in H0])
        t0 = time.perf_counter()
        orc.outer_step(X64, st, orc.Opts(inner_iters=T))
        dt += time.perf_counter() - t0
        done += work[used]
        used += 1
        if dt >= min_seconds:
            break
    per_batch_iter = dt * sum(work) / done
    return {"value": len(shapes) / per_batch_iter, "unit": "problem_outer_iters/s", "cores": cores,
            "kind": "oracle", "blas": bi["blas"], "affinity_cores": bi["affinity_cores"],
            "sample": f"1 outer iteration (T={T}) of the FP64 oracle on each of the first {used} tensors "
                      f"({dt:.1f} s), scaled to all {len(shapes)} by sum(I J K F)",
            "seconds_measured": dt}


def cpu_baseline_sparse(T, H0, Topt, sample_nnz, min_seconds=10.0):
    """The FP64 oracle on the host: outer iterations on the first
    `sample_nnz` non-zeros (the order is random), with the MTTKRP share
    scaled to all non-zeros (its cost is linear in nnz; the rest is not)."""
    from oracle import ntf_oracle as orc
    bi = blas_info()
    cores = bi['blas_threads'] or bi['affinity_cores']
    n = T.idx.shape[0]
    S = min(n, sample_nnz)
    sub = orc.SparseTensor(idx=T.idx[:S], val=T.val[:S], dims=T.dims)
    st = orc.init_state([h.astype(np.float64) for h in H0])
    opts = orc.Opts(inner_iters=Topt)
    t_outer, t_mk, iters = 0.0, 0.0, 0
    while t_outer < min_seconds and iters < 5:
        t0 = time.perf_counter()
        orc.outer_step(sub, st, opts)
        t_outer += time.perf_counter() - t0
        t0 = time.perf_counter()
        for m in range(3):
            orc.mttkrp_sparse(sub, st.H, m)
        t_mk += time.perf_counter() - t0
        iters += 1
    per_iter = (t_outer + t_mk * (n / S - 1.0)) / iters
    return {"value": 1.0 / per_iter, "unit": "outer_iters/s", "cores": cores, "kind": "oracle", "blas": bi["blas"],
            "affinity_cores": bi["affinity_cores"],
            "sample": f"{iters} outer iteration(s) (T={Topt}) of the FP64 oracle on the first {S} of "
                      f"{n} non-zeros ({t_outer:.1f} s), its three MTTKRPs (timed again, "
                      f"{t_mk / iters:.2f} s per iteration) scaled by {n}/{S}",
            "seconds_measured": t_outer + t_mk}


def bench_sparse(args):
    """Sparse workload: one outer iteration is three sparse MTTKRPs (one per
    mode, from the sorted copies) plus the dense per-mode work."""
    import torch
    import ntf_synth
    import paper_1409_2383_amd as ntf
    from oracle import ntf_oracle as orc
    ntf.library_path()
    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    dims, F, T = wl["dims"], wl["F"], wl["T"]
    seed = ntf_synth.config_seed(wl["config"])
    log(f"[bench] generating sparse {dims} nnz~{wl['nnz']} seed {seed}")
    t0 = time.perf_counter()
    s = ntf_synth.sparse_planted(dims, wl["planted"], wl["nnz"], seed, skew=wl["skew"], dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    nnz = int(s.idx.shape[0])
    log(f"[bench] {nnz} non-zeros ready in {time.perf_counter() - t0:.1f} s")
    idx = torch.from_numpy(s.idx).to(dev)
    val = torch.from_numpy(s.val).to(dev)
    H = [torch.from_numpy(h).to(dev) for h in H0]
    t0 = time.perf_counter()
    solver = ntf.NtfAdmmSparse(idx, val, dims, H, opts=ntf.AdmmOptions(inner_iters=T, precision=ntf.PREC_F32))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    del idx, val
    ms, wall = time_steps(torch, solver, args.steps, args.warmup)
    st = torch.cuda.current_stream()
    passes = {}
    for m, name in enumerate(("mode1", "mode2", "mode3")):
        solver.launch_pass(m)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.pass_reps):
            solver.launch_pass(m)
        e1.record(st)
        torch.cuda.synchronize()
        passes[name] = e0.elapsed_time(e1) / args.pass_reps
    nbytes = solver.plan_info()
    rfe = solver.fit()
    solver.close()
    log(f"[bench] sparse: {ms:.3f} ms/step, MTTKRP {passes}, set-up {setup_s:.2f} s, RFE {rfe:.4f}")
    dom = max(passes, key=lambda k: passes[k])
    achieved = nbytes[dom] / (passes[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": f"sparse MTTKRP {dom}",
                "algorithmic_bytes_per_launch": nbytes[dom], "avg_launch_ms": passes[dom]}
    cpu = None
    if not args.no_cpu_baseline:
        Tor = orc.SparseTensor(idx=s.idx, val=s.val.astype(np.float64), dims=tuple(dims))
        log("[bench] CPU oracle baseline on a sample of the non-zeros")
        cpu = cpu_baseline_sparse(Tor, H0, T, 3_000_000)
    line = {
        "metric": "NTF outer iters/s, sparse tensor",
        "value": 1e3 / ms, "unit": "outer_iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} sparse, {nnz} non-zeros (skew {wl['skew']}), "
                               f"F={F}, T={T} inner iters, fp32",
                   "dims": list(dims), "nnz": nnz, "F": F, "inner_iters": T},
        "roofline": roofline, "cpu_baseline": cpu,
        "mttkrp_ms": passes, "mttkrp_bytes": nbytes,
        "mttkrp_gbs": {k: nbytes[k] / (passes[k] * 1e-3) / 1e9 for k in passes},
        "setup_s": setup_s, "rfe": rfe,
    }
    print(json.dumps(line), flush=True)


def bench_nway(args):
    """Order-N workload: one outer iteration updates the N factors, each
    MTTKRP a pass over X on a three-way view of it."""
    import torch
    import ntf_synth
    import paper_1409_2383_amd as ntf
    from oracle import ntf_oracle as orc
    ntf.library_path()
    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    dims, F, T = wl["dims"], wl["F"], wl["T"]
    N = len(dims)
    seed = ntf_synth.config_seed(wl["config"])
    log(f"[bench] generating {dims} F={F} ({wl['snr']} dB) seed {seed}")
    t0 = time.perf_counter()
    X, _, _ = ntf_synth.planted_nway(dims, F, seed, dist=wl["dist"], snr_db=wl["snr"], dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    log(f"[bench] data ready in {time.perf_counter() - t0:.1f} s")
    Xd = torch.from_numpy(X).to(dev)
    H = [torch.from_numpy(h).to(dev) for h in H0]
    solver = ntf.NtfNway(Xd, H, opts=ntf.AdmmOptions(inner_iters=T, precision=ntf.PREC_F32))
    ms, wall = time_steps(torch, solver, args.steps, args.warmup)
    st = torch.cuda.current_stream()
    passes = {}
    Ws = [torch.empty((d, F), dtype=torch.float64, device=dev) for d in dims]
    import ctypes
    from paper_1409_2383_amd import _lib
    L = _lib.lib()
    for m in range(N):
        L.ntf_nway_mttkrp(solver._ctx, m, ctypes.c_void_p(Ws[m].data_ptr()))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.pass_reps):
            L.ntf_nway_mttkrp(solver._ctx, m, ctypes.c_void_p(Ws[m].data_ptr()))
        e1.record(st)
        torch.cuda.synchronize()
        passes[f"mode{m + 1}"] = e0.elapsed_time(e1) / args.pass_reps
    rfe = solver.fit()
    solver.close()
    log(f"[bench] {N}-way: {ms:.3f} ms/step, MTTKRP {passes}, RFE {rfe:.4f}")
    # one pass over X per mode (the folded factors and W are small beside it).
    # Inside an outer iteration the middle modes go in pairs (2, 3), (4, 5), ...
    # (1-based) while the pair's reduction grid fits: the second mode of a pair
    # takes T from the first one's pass and runs no pass of its own, so its
    # stand-alone time above (a full pass) is not part of the step.
    xbytes = int(np.prod(dims)) * 4
    second = {n + 1 for n in range(1, N - 2, 2) if -(-int(np.prod(dims[:n])) // 4) <= 65535}
    in_step = [f"mode{m + 1}" for m in range(N) if m not in second]
    dom = max(in_step, key=lambda k: passes[k])
    achieved = xbytes / (passes[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": f"MTTKRP {dom}",
                "algorithmic_bytes_per_launch": xbytes, "avg_launch_ms": passes[dom],
                "passes_in_step": in_step}
    cpu = None
    if not args.no_cpu_baseline:
        S = max(1, dims[0] // 8)
        log(f"[bench] CPU oracle baseline on {S} of {dims[0]} mode-1 slabs")
        Xs = np.ascontiguousarray(X[:S], dtype=np.float64)
        sto = orc.init_state([H0[0][:S].astype(np.float64)] + [h.astype(np.float64) for h in H0[1:]])
        n_it, t_cpu = 0, 0.0
        while t_cpu < 10.0 and n_it < 5:
            t0 = time.perf_counter()
            orc.outer_step(Xs, sto, orc.Opts(inner_iters=T))
            t_cpu += time.perf_counter() - t0
            n_it += 1
        bi = blas_info()
        cores = bi['blas_threads'] or bi['affinity_cores']
        per_iter = t_cpu / n_it * dims[0] / S
        cpu = {"value": 1.0 / per_iter, "unit": "outer_iters/s", "cores": cores, "kind": "oracle", "blas": bi["blas"],
            "affinity_cores": bi["affinity_cores"],
               "sample": f"{n_it} outer iteration(s) (T={T}) of the FP64 oracle on the first {S} of "
                         f"{dims[0]} mode-1 slabs ({t_cpu:.1f} s), scaled by {dims[0]}/{S}",
               "seconds_measured": t_cpu}
    line = {
        "metric": "NTF outer iters/s, order-N dense tensor",
        "value": 1e3 / ms, "unit": "outer_iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} dense {N}-way, F={F} planted U[0,1] factors, "
                               f"{wl['snr']:.0f} dB, T={T} inner iters, fp32",
                   "dims": list(dims), "F": F, "inner_iters": T},
        "roofline": roofline, "cpu_baseline": cpu, "mttkrp_ms": passes,
        "mttkrp_gbs": {k: xbytes / (v * 1e-3) / 1e9 for k, v in passes.items()}, "rfe": rfe,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--pass-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-slabs", type=int, default=0, help="0 = all slabs")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also launch a known-size copy kernel (for byte-counter scaling)")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time to rel fit 1e-4")
    ap.add_argument("--ttt-warm", action="store_true",
                    help="also time the mixed arm with the learned warm start (trains the F = 64 "
                         "network first; its training time is reported, not counted)")
    ap.add_argument("--single-arm", action="store_true")
    ap.add_argument("--arm", default="", help="run this arm only (e.g. fp32, mixed)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs into profiles/ and exit")
    ap.add_argument("--write-mfma", nargs=2, metavar=("PMC_CSV", "TIMING_JSON"),
                    help="summarise a rocprofv3 --pmc run of the MFMA counters into profiles/ and exit "
                         "(kernel times from a bench.py line of the same arm)")
    ap.add_argument("--write-kernel-stats", metavar="STATS_CSV",
                    help="summarise a rocprofv3 --kernel-trace --stats run into profiles/ and exit")
    ap.add_argument("--batch-n", type=int, default=0, help="batched workload: number of tensors")
    ap.add_argument("--no-tune", action="store_true", help="batched workload: skip the autotuner")
    args = ap.parse_args()
    if args.write_traffic or args.write_kernel_stats or args.write_mfma:
        summarize(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the design notes say how "
              "the path would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5":
        bench_batched(args)
        return
    if args.workload == "s1":
        bench_sparse(args)
        return
    if args.workload == "n4":
        bench_nway(args)
        return
    import torch
    import ntf_synth
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    dims, F, T = wl["dims"], wl["F"], wl["T"]
    seed = ntf_synth.config_seed(wl["config"])
    log(f"[bench] generating {dims} F={F} ({wl['dist']}, {wl['snr']} dB) seed {seed}")
    t0 = time.perf_counter()
    x_dt = np.float64 if wl["arms"][0] == "fp64" else np.float32
    pt = ntf_synth.planted(dims, F, seed, dist=wl["dist"], snr_db=wl["snr"], clip=wl["clip"],
                           dtype=x_dt)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float64)
    Xd = torch.from_numpy(pt.X).to(dev)
    log(f"[bench] data ready in {time.perf_counter() - t0:.1f} s")

    arms = wl["arms"][:1] if args.single_arm else wl["arms"]
    if args.arm:
        if args.arm not in wl["arms"]:
            raise SystemExit(f"arm {args.arm} not in {wl['arms']}")
        arms = (args.arm,)
    results = {}
    for arm in arms:
        solver, H = make_solver(ntf, torch, Xd, H0, arm, T, dev)
        ms, wall = time_steps(torch, solver, args.steps, args.warmup)
        passes = time_passes(torch, solver, args.pass_reps)
        nbytes = solver.plan_info()
        results[arm] = {"ms_per_step": ms, "wall_s": wall, "outer_iters_per_s": 1e3 / ms,
                        "pass_ms": passes, "pass_bytes": nbytes,
                        "pass_gbs": {k: nbytes[k] / (passes[k] * 1e-3) / 1e9 for k in passes}}
        log(f"[bench] {arm}: {ms:.3f} ms/step, passes {passes}")
        solver.close()
        del solver, H
        torch.cuda.empty_cache()

    if args.copy_calib_mib > 0:
        copy_calibration(torch, dev, args.copy_calib_mib)

    head = arms[0]
    r = results[head]
    dom = max(("pass1", "pass3"), key=lambda k: r["pass_ms"][k])
    # Algorithmic bytes of one MTTKRP of the method: one read of the tensor in
    # the arm's storage type, IJK s (the Khatri-Rao factors are L2-resident).
    # Pass 1 is the mode-1 MTTKRP; it also writes the I x J x F intermediate
    # that the mode-2 MTTKRP reads instead of X (counted in kernel_bytes only).
    x_es = 8 if head == "fp64" else (2 if head == "mixed" else 4)
    method_bytes = int(np.prod(dims)) * x_es
    achieved = method_bytes / (r["pass_ms"][dom] * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{head}_{dom}.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("src_hash") == src_hash(MTTKRP_SOURCES):
            traffic = tj.get("bytes_per_launch")
    per_step = 3 * method_bytes / (r["ms_per_step"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                "algorithmic_bytes_per_launch": method_bytes,
                "algorithmic_bytes": "IJK s: one read of the tensor copy the arm streams",
                "kernel_bytes_per_launch": r["pass_bytes"][dom],
                "avg_launch_ms": r["pass_ms"][dom],
                "per_step": {"bytes": 3 * method_bytes, "ms": r["ms_per_step"], "GB/s": per_step,
                             "frac": per_step / HBM_PEAK_GBS,
                             "note": "three MTTKRPs of IJK s each per outer iteration over the "
                                     "whole step time"}}

    cpu = None
    if not args.no_cpu_baseline:
        slabs = args.cpu_sample_slabs
        log(f"[bench] CPU oracle baseline on {slabs or 'all'} slabs")
        cpu = cpu_baseline(pt.X, H0, T, slabs)

    ttt = None
    if not args.no_ttt and args.workload == "c3" and not args.single_arm and not args.arm:
        star = load_rfe_star(args.workload)
        if star is None:
            log("[bench] no stored oracle RFE*: time to target skipped")
        else:
            arms_t, warm = ("mixed", "fp32"), None
            if args.ttt_warm:
                warm, train_s = warm_arm(torch, ntf, log)
                arms_t = ("mixed", "mixed+mlp", "fp32")
            log("[bench] time to rel fit 1e-4")
            ttt = time_to_target(torch, ntf, Xd, H0, T, arms_t, dev, star, warm=warm)
            if warm:
                ttt["mixed+mlp"]["network"] = {"F": 64, "hidden": 256, "train_s": train_s,
                                               "note": "trained once on 64 small planted tensors "
                                                       "(not counted in the time)"}

    dtype = {"mixed": "bf16", "fp32": "f32", "fp64": "f64"}[head]
    line = {
        "metric": "NTF outer iters/s + MTTKRP GB/s (% HBM peak), mixed vs FP32 at rel fit 1e-4",
        "value": r["outer_iters_per_s"], "unit": "outer_iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} dense, F={F} planted {wl['dist']} "
                               f"factors, {wl['snr']:.0f} dB, T={T} inner iters, {head} arm",
                   "dims": list(dims), "F": F, "inner_iters": T, "arm": head},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "arms": results,
    }
    if ttt is not None:
        line["time_to_rel_fit_1e-4"] = ttt
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
