"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Every value here comes from ``oracle/ntf_oracle.py`` run on inputs from
``ntf_synth`` (the same seeded arrays the GPU tests and the benchmark build);
nothing is read from the GPU path.  Each output file records the command that
wrote it.

    python tests/golden/make_golden.py c2       # 400^3, F = 20, FP32 data, 200 outer iterations
    python tests/golden/make_golden.py c3       # 1000 x 800 x 600, F = 64: converged RFE*
    python tests/golden/make_golden.py c5       # 16 tensors of the 256-tensor batch
    python tests/golden/make_golden.py c5mixed  # the same with the batch's bf16 operand rounding
    python tests/golden/make_golden.py mixed    # 80 x 70 x 60, F = 12: exact and bf16-operand runs

The c3 run needs ~12 GB of host memory and some tens of minutes; the others
minutes.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import ntf_synth  # noqa: E402
from oracle import ntf_oracle as orc  # noqa: E402


def _write(name, obj):
    obj["written_by"] = "python tests/golden/make_golden.py " + " ".join(sys.argv[1:])
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        json.dump(obj, fh, indent=1)
    print(f"wrote {path}", flush=True)


def _xnorm2(X):
    x = np.asarray(X, dtype=np.float64).ravel()
    return float(np.dot(x, x))


def golden_c2(args):
    """Config 2: 400^3 FP32 tensor of F = 20 U[0,1] planted factors, 20 dB,
    T = 10, rho = tr(G)/F, 200 outer iterations from the float32 start the
    GPU's FP32 arm takes.  Stores the RFE along the run (expanded form every
    10 iterations) and the RFE by definition after 200."""
    dims, F, T, outer = (400, 400, 400), 20, 10, args.outer or 200
    seed = ntf_synth.config_seed(2)
    pt = ntf_synth.planted(dims, F, seed, snr_db=20.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    X = pt.X.astype(np.float64)
    xn2 = _xnorm2(X)
    st = orc.init_state([h.astype(np.float64) for h in H0])
    opts = orc.Opts(inner_iters=T)
    trace = []
    t0 = time.perf_counter()
    for k in range(1, outer + 1):
        orc.outer_step(X, st, opts)
        if k % 10 == 0 or k in (1, 2, 5):
            r = orc.rfe_expanded(X, st.H, xn2)
            trace.append([k, r])
            print(f"c2 outer {k}: RFE {r:.12f} ({time.perf_counter() - t0:.0f} s)", flush=True)
    rfe_final = orc.rfe(X, st.H)
    _write("c2_fp32_400cubed.json", {
        "workload": "400x400x400 FP32 tensor, F=20 planted U[0,1] factors, 20 dB, T=10, rho=tr(G)/F",
        "seed": seed, "outer_iters": outer, "rfe_final": rfe_final, "rfe_trace": trace,
        "rho_final": list(st.rho),
        "factor_norms": [float(np.linalg.norm(h)) for h in st.H],
    })


def golden_c3(args):
    """Config 3: 1000 x 800 x 600 FP32 tensor of F = 64 Exponential(1)
    planted factors, 30 dB, T = 10; the exact FP64 method from the start the
    benchmark's arms take, run until |dRFE|/RFE < 1e-9 between consecutive
    outer iterations (cap 3000).  RFE* is its final RFE; the trace gives the
    exact method's own iterations to (RFE - RFE*)/RFE* <= 1e-4."""
    dims, F, T = (1000, 800, 600), 64, 10
    seed = ntf_synth.config_seed(3)
    pt = ntf_synth.planted(dims, F, seed, dist="exponential", snr_db=30.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float64)
    X = pt.X.astype(np.float64)
    del pt
    xn2 = _xnorm2(X)
    st = orc.init_state(H0)
    opts = orc.Opts(inner_iters=T)
    trace = []
    prev = None
    cap = args.outer or 3000
    t0 = time.perf_counter()
    k = 0
    while k < cap:
        orc.outer_step(X, st, opts)
        k += 1
        r = orc.rfe_expanded(X, st.H, xn2)
        trace.append([k, r])
        print(f"c3 outer {k}: RFE {r:.12f} ({time.perf_counter() - t0:.0f} s)", flush=True)
        if prev is not None and abs(prev - r) < 1e-9 * r:
            break
        prev = r
    rfe_star = trace[-1][1]
    first = next((it for it, r in trace if (r - rfe_star) / rfe_star <= 1e-4), None)
    _write("c3_rfe_star.json", {
        "workload": "1000x800x600 FP32 tensor, F=64 planted Exponential(1) factors, 30 dB, T=10, "
                    "rho=tr(G)/F, FP64 oracle from the benchmark's start",
        "seed": seed, "rfe_star": rfe_star, "outer_iters": k,
        "stop": "|dRFE|/RFE < 1e-9 between consecutive outer iterations",
        "exact_iters_to_rel_1e-4": first, "rfe_trace": trace,
    })


def c5_subset():
    """The first 16 tensors of the 256-tensor batch (modes uniform on
    50..500, F uniform on 5..40, U[0,1] factors, 20 dB): shapes, ranks, seeds."""
    shapes = ntf_synth.batch_shapes(256, ntf_synth.config_seed(5), 50, 500, tuple(range(5, 41)))
    return [(t, dims, F, ntf_synth.config_seed(5, t)) for t, (dims, F) in enumerate(shapes[:16])]


def golden_c5(args):
    """Batched workload: each of the 16 tensors run by the exact FP64 method
    (T = 10, rho = tr(G)/F) from the float32 start the batch takes; RFE every
    10 outer iterations up to `outer`."""
    outer = args.outer or 300
    out = []
    for t, dims, F, seed in c5_subset():
        pt = ntf_synth.planted(dims, F, seed, snr_db=20.0, dtype=np.float32)
        H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
        X = pt.X.astype(np.float64)
        del pt
        xn2 = _xnorm2(X)
        st = orc.init_state([h.astype(np.float64) for h in H0])
        opts = orc.Opts(inner_iters=10)
        trace = []
        t0 = time.perf_counter()
        for k in range(1, outer + 1):
            orc.outer_step(X, st, opts)
            if k % 10 == 0:
                trace.append([k, orc.rfe_expanded(X, st.H, xn2)])
        print(f"c5 tensor {t} {dims} F={F}: RFE {trace[-1][1]:.9f} after {outer} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        out.append({"tensor": t, "dims": list(dims), "F": F, "seed": seed, "rfe_trace": trace})
        _write("c5_subset16.json", {
            "workload": "first 16 tensors of the 256-tensor batch (modes U{50..500}, F U{5..40}, "
                        "U[0,1] factors, 20 dB), FP32 data and start, exact FP64 method, T=10, "
                        "rho=tr(G)/F",
            "outer_iters": outer, "tensors": out})


def golden_c5_mixed(args):
    """The same 16 tensors, the same start and T, but the MTTKRPs with the
    batched path's operand rounding (per-slab bf16 X, bf16 C for modes 1-2,
    B as two bf16 terms for mode 3; exact accumulation, FP64 otherwise)."""
    outer = args.outer or 300
    out = []
    for t, dims, F, seed in c5_subset():
        pt = ntf_synth.planted(dims, F, seed, snr_db=20.0, dtype=np.float32)
        H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
        X = pt.X.astype(np.float64)
        xn2 = _xnorm2(X)
        st = orc.init_state([h.astype(np.float64) for h in H0])
        opts = orc.Opts(inner_iters=10, mttkrp_operands="bf16_split")
        trace = []
        t0 = time.perf_counter()
        for k in range(1, outer + 1):
            orc.outer_step(pt.X, st, opts)
            if k % 10 == 0:
                trace.append([k, orc.rfe_expanded(X, st.H, xn2)])
        print(f"c5 mixed tensor {t} {dims} F={F}: RFE {trace[-1][1]:.9f} after {outer} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        out.append({"tensor": t, "dims": list(dims), "F": F, "seed": seed, "rfe_trace": trace})
        del pt, X
        _write("c5_subset16_mixed.json", {
            "workload": "first 16 tensors of the 256-tensor batch (modes U{50..500}, F U{5..40}, "
                        "U[0,1] factors, 20 dB), FP32 data and start, FP64 method with the batched "
                        "path's bf16 operand rounding of the MTTKRPs, T=10, rho=tr(G)/F",
            "outer_iters": outer, "tensors": out})


def golden_mixed(args):
    """80 x 70 x 60, F = 12 Exponential(1) planted factors, 30 dB, T = 10:
    the exact method and the same method with the bfloat16 operand rounding
    of the mixed-precision recipe (per-slab bf16 X, bf16 C for modes 1-2,
    split bf16 B for mode 3), both FP64 otherwise, from the float32 start.
    RFE every 10 outer iterations up to `outer`."""
    dims, F, T, outer = (80, 70, 60), 12, 10, args.outer or 400
    seed = 9001
    pt = ntf_synth.planted(dims, F, seed, dist="exponential", snr_db=30.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    X = pt.X.astype(np.float64)
    res = {}
    for name, operands in (("exact", "exact"), ("bf16_split", "bf16_split")):
        st = orc.init_state([h.astype(np.float64) for h in H0])
        opts = orc.Opts(inner_iters=T, mttkrp_operands=operands)
        trace = []
        Xin = pt.X if operands != "exact" else X
        for k in range(1, outer + 1):
            orc.outer_step(Xin, st, opts)
            if k % 10 == 0:
                trace.append([k, orc.rfe(X, st.H)])
        res[name] = trace
        print(f"mixed {name}: RFE {trace[-1][1]:.12f} after {outer}", flush=True)
    _write("mixed_80x70x60.json", {
        "workload": "80x70x60 FP32 tensor, F=12 planted Exponential(1) factors, 30 dB, T=10, "
                    "rho=tr(G)/F, seed 9001",
        "seed": seed, "outer_iters": outer, "rfe_trace": res,
    })


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c2", "c3", "c5", "c5mixed", "mixed"])
    ap.add_argument("--outer", type=int, default=0)
    args = ap.parse_args()
    {"c2": golden_c2, "c3": golden_c3, "c5": golden_c5, "c5mixed": golden_c5_mixed,
     "mixed": golden_mixed}[args.which](args)


if __name__ == "__main__":
    main()
