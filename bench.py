#!/usr/bin/env python3
"""Benchmark: certified top-k Katz ranking on one MI355X.

Workload: R-MAT scale 22 (2^22 nodes, edge factor 16, a,b,c,d = .57,.19,.19,.05,
symmetrised, deduplicated, self-loops dropped, seeded relabelling; seed 1),
CSR with int32 offsets, alpha = 1/(1 + deg_max), top-k = 1000, eps = 1e-6.

One step is one katz_rank_static call: binning, every iteration (walk step,
selection, converged()) until the ranking is certified, and the output writes,
on device-resident inputs.  The FP32-SpMV form (FP64 bounds and margins) is the
headline value; the plain FP64 form is timed the same way beside it.

value = GTEPS = r * nnz / t_step / 1e9 with nnz the directed CSR entries (each
undirected edge counted twice, as traversed).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SCALE, EDGE_FACTOR, SEED, K, EPS = 22, 16, 1, 1000, 1e-6


def algorithmic_bytes_per_walk_step(n, nnz, precision):
    """Compulsory HBM bytes of one walk step (iteration r >= 2): every column
    index once (4 B per arc) and, per node, the int32 row offset (4 B), the
    previous walk entry (4 B FP32 / 8 B FP64), the new walk entry (4 / 8 B), the
    read-modify-write of c (16 B), and for FP32 the margin accumulator (8 B)."""
    per_node = 4 + 4 + 4 + 16 + 8 if precision == "fp32" else 4 + 8 + 8 + 16
    return 4 * nnz + per_node * n


def time_form(katz, torch, rp_t, col_t, precision, steps, warmup, flags=0):
    for _ in range(warmup):
        res = katz.rank_static(rp_t, col_t, K, eps=EPS, precision=precision, flags=flags)
    torch.cuda.synchronize()
    katz.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = katz.rank_static(rp_t, col_t, K, eps=EPS, precision=precision, flags=flags)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = katz.timing_read()
    katz.timing_enable(False)
    return res, (t1 - t0) / steps, tm


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthgraph as sg
    import paper_1807_03847_amd.katz as katz

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {args.copy_mib} MiB read + {args.copy_mib} MiB written", flush=True)
        del src, dst

    t = time.perf_counter()
    rp, col = sg.rmat(SCALE, EDGE_FACTOR, 0.57, 0.19, 0.19, seed=SEED)
    n, nnz = len(rp) - 1, int(rp[-1])
    dmax = int(np.max(np.diff(rp)))
    print(f"[bench] graph generated: n={n} nnz={nnz} dmax={dmax} ({time.perf_counter() - t:.1f}s)", flush=True)
    rp_t = torch.from_numpy(rp.astype(np.int32)).cuda()
    col_t = torch.from_numpy(col).cuda()
    torch.cuda.synchronize()

    forms = {}
    for precision in ("fp32", "fp64"):
        res, sec, tm = time_form(katz, torch, rp_t, col_t, precision, args.steps, args.warmup)
        walk_avg_ms = tm["walk_step_ms"] / max(tm["walk_step_launches"], 1)
        forms[precision] = dict(res=res, sec=sec, tm=tm, walk_avg_ms=walk_avg_ms,
                                gteps=res.iterations * nnz / sec / 1e9)
        print(f"[bench] {precision}: r={res.iterations} status={res.status} {sec * 1e3:.3f} ms/step "
              f"walk_step {walk_avg_ms * 1e3:.1f} us", flush=True)

    # The same FP32 run without the internal renumbering, for context.
    res_nr, sec_nr, tm_nr = time_form(katz, torch, rp_t, col_t, "fp32", max(1, args.steps // 2), 1,
                                      flags=katz.FLAG_NO_REORDER)
    print(f"[bench] fp32 caller order: {sec_nr * 1e3:.3f} ms/step", flush=True)

    f32, f64 = forms["fp32"], forms["fp64"]
    bytes_step = algorithmic_bytes_per_walk_step(n, nnz, "fp32")
    achieved = bytes_step / (f32["walk_avg_ms"] * 1e-3) / 1e9

    out = {
        "metric": "certified top-k Katz ranking: GTEPS and % HBM peak, FP32-SpMV vs FP64, 1 GPU",
        "value": round(f32["gteps"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["sec"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "rmat22_top1000_eps1e-6",
            "graph": "R-MAT scale 22, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, "
                     "deduplicated, no self-loops, seeded relabel, seed 1",
            "n": n, "nnz_directed": nnz, "deg_max": dmax, "k": K, "eps": EPS,
            "alpha": "1/(1+deg_max)", "row_ptr": "int32",
            "form": "FP32 walk vector and row sums; FP64 c, bounds and rounding margin",
        },
        "iterations": f32["res"].iterations,
        "status": f32["res"].status,
        "fp64": {
            "gteps": round(f64["gteps"], 3),
            "ms_per_step": round(f64["sec"] * 1e3, 4),
            "iterations": f64["res"].iterations,
            "status": f64["res"].status,
            "walk_step_avg_us": round(f64["walk_avg_ms"] * 1e3, 2),
            "walk_step_hbm_gbs": round(algorithmic_bytes_per_walk_step(n, nnz, "fp64")
                                       / (f64["walk_avg_ms"] * 1e-3) / 1e9, 1),
        },
        "speedup_fp32_vs_fp64": round(f64["sec"] / f32["sec"], 3),
        "phase_ms_per_step_fp32": {
            key: round(f32["tm"][key] / max(f32["tm"]["calls"], 1), 4)
            for key in ("prep_ms", "walk_first_ms", "walk_step_ms", "select_ms", "result_ms", "call_ms")
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "walk_step<fp32>",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": bytes_step,
            "avg_launch_us": round(f32["walk_avg_ms"] * 1e3, 2),
            "launches_timed": f32["tm"]["walk_step_launches"],
        },
    }

    out["fp32_caller_order"] = {
        "ms_per_step": round(sec_nr * 1e3, 4),
        "walk_step_avg_us": round(tm_nr["walk_step_ms"] / max(tm_nr["walk_step_launches"], 1) * 1e3, 2),
        "same_result": bool(torch.equal(res_nr.topk, f32["res"].topk) and torch.equal(res_nr.lower, f32["res"].lower)),
    }
    same = bool(torch.equal(f32["res"].topk, f64["res"].topk))
    out["fp32_fp64_same_topk"] = same

    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        orc = oracle.rank_static(rp, col, None, K, EPS)
        sec = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": round(orc.iterations * nnz / sec / 1e9, 5),
            "unit": "GTEPS",
            "cores": 1,
            "kind": "oracle",
            "sample": "one full certified FP64 run of the same workload (numpy/scipy, single thread), "
                      f"{sec:.1f} s, r={orc.iterations}",
        }
        g32 = f32["res"]
        lo32 = g32.lower.cpu().numpy()
        idx = g32.topk.cpu().numpy()
        rel = np.abs(lo32 - orc.lower_all[idx]) / orc.lower_all[idx]
        out["fp32_max_rel_err_vs_oracle"] = float(rel.max())
        out["topk_equal_oracle"] = {
            "fp32": bool(np.array_equal(idx, orc.topk)),
            "fp64": bool(np.array_equal(f64["res"].topk.cpu().numpy(), orc.topk)),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
