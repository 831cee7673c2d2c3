#!/usr/bin/env python3
"""Benchmark: certified top-k Katz ranking on one MI355X.

Default workload (the headline line): R-MAT scale 27 (2^27 nodes, edge factor
16, a,b,c,d = .57,.19,.19,.05, symmetrised, deduplicated, self-loops dropped,
seeded relabelling; seed 3), CSR with int64 row offsets (about 4.3e9 directed
entries), alpha = 1/(1 + deg_max), top-k = 100, eps = 1e-6.  The same
measurement on R-MAT scale 22 (seed 1, int32 offsets, top-1000) is reported
beside it under "rmat22".  The graphs are generated on the device.

One step is one katz_rank_static call: binning, every iteration (walk step,
selection, converged()) until the ranking is certified, and the output writes,
on device-resident inputs.  The FP32-SpMV form (FP64 bounds and margins) is the
headline value; the plain FP64 form is timed the same way beside it.

value = GTEPS = r * nnz / t_step / 1e9 with nnz the directed CSR entries (each
undirected edge counted twice, as traversed).

CPU baseline: the C++/OpenMP FP64 oracle's full certified run on every host
core (it also checks that both forms return the oracle's top-k), plus a
single-thread walk over a leading row range.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
EDGE_FACTOR, EPS = 16, 1e-6
WORKLOADS = {
    27: dict(scale=27, seed=3, k=100, rp64=True, name="rmat27_top100_eps1e-6"),
    22: dict(scale=22, seed=1, k=1000, rp64=False, name="rmat22_top1000_eps1e-6"),
}


def algorithmic_bytes_per_walk_step(n, nnz, precision, rp64):
    """Compulsory HBM bytes of one walk step (iteration r >= 2): every column
    index once (4 B per arc) and, per node, the row offset (4 B int32 / 8 B
    int64), the previous walk entry (4 B FP32 / 8 B FP64), the new walk entry
    (4 / 8 B), the read-modify-write of c (16 B), and for FP32 the margin
    accumulator (8 B)."""
    off = 8 if rp64 else 4
    per_node = off + (4 + 4 + 16 + 8 if precision == "fp32" else 8 + 8 + 16)
    return 4 * nnz + per_node * n


def counters_path(scale):
    return os.path.join(ROOT, "profiles", f"walk_step_rmat{scale}_counters.json")


def measured_traffic(scale, tuning_arg):
    """HBM bytes per walk_step launch from the committed FETCH_SIZE / WRITE_SIZE
    record of this workload (scaled by the copy calibration stored with it), or
    None when the kernel sources or the launch tuning differ from the ones
    measured."""
    import hashlib
    path = counters_path(scale)
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None, "no counter record"
    for src, digest in rec["sources_sha256"].items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None, f"kernel source changed since the counters were taken ({src})"
    other = rec.get("by_tuning", {})
    if rec["tuning"] == tuning_arg:
        traffic = rec["traffic_bytes_per_launch"]
    elif tuning_arg in other:
        traffic = other[tuning_arg]
    else:
        return None, f"counters taken at tunings {[rec['tuning']] + sorted(other)}, timed at {tuning_arg}"
    return traffic, ("FETCH_SIZE x%.2f + WRITE_SIZE x%.2f per launch at tuning %s, from %s" % (
        rec["calibration"]["fetch_scale"], rec["calibration"]["write_scale"], tuning_arg,
        os.path.relpath(path, ROOT)))


def time_form(katz, torch, rp_t, col_t, k, precision, steps, warmup, flags=0):
    for _ in range(warmup):
        res = katz.rank_static(rp_t, col_t, k, eps=EPS, precision=precision, flags=flags)
    torch.cuda.synchronize()
    katz.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = katz.rank_static(rp_t, col_t, k, eps=EPS, precision=precision, flags=flags)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = katz.timing_read()
    katz.timing_enable(False)
    return res, (t1 - t0) / steps, tm


def tuning_arg(t):
    """HUB_BYTES:BLOCKS_PER_CU:WALK_GROUPS[:B0,...,B5] (the row-length classes
    only when they are not the defaults)."""
    arg = f"{t['hub_bytes']}:{t['blocks_per_cu']}:{t['walk_groups']}"
    if any(t.get("bin_bounds", [0])):
        arg += ":" + ",".join(str(v) for v in t["bin_bounds"])
    return arg


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_static(args, katz, sg, torch, np, wl):
    """Times both forms on one R-MAT workload; returns (line fields, graph tensors)."""
    scale, k, rp64 = wl["scale"], wl["k"], wl["rp64"]
    t = time.perf_counter()
    rp_t, col_t = sg.rmat_device(scale, EDGE_FACTOR, 0.57, 0.19, 0.19, seed=wl["seed"])
    if not rp64:
        rp_t = rp_t.to(torch.int32)
    torch.cuda.synchronize()
    n, nnz = rp_t.numel() - 1, col_t.numel()
    dmax = int((rp_t[1:] - rp_t[:-1]).max().item())
    print(f"[bench] rmat{scale} generated on the device: n={n} nnz={nnz} dmax={dmax} "
          f"({time.perf_counter() - t:.1f}s)", flush=True)

    tunings, forms = {}, {}
    for precision in ("fp32", "fp64"):
        if args.tuning == "auto":
            tunings[precision] = katz.autotune(rp_t, col_t, k, eps=EPS, precision=precision)
        else:
            parts = args.tuning.split(":")
            katz.tuning_set(int(parts[0]), int(parts[1]), walk_groups=int(parts[2]) if len(parts) > 2 else 0,
                            bin_bounds=[int(v) for v in parts[3].split(",")] if len(parts) > 3 else None)
            tunings[precision] = katz.tuning_get()
        print(f"[bench] rmat{scale} {precision} tuning {tunings[precision]}", flush=True)
        res, sec, tm = time_form(katz, torch, rp_t, col_t, k, precision, args.steps, args.warmup)
        # Plain walk steps that did work: r - 2 per call (steps 3..r; step 2 is
        # fused with the renumbering and timed on its own).  The host enqueues
        # one more walk launch before it reads the stop flag; that launch
        # returns at once and is not a walk step.
        walk_avg_ms = tm["walk_step_ms"] / max(tm["calls"] * (res.iterations - 2), 1)
        renum_avg_ms = tm["renumber_step_ms"] / max(tm["renumber_step_launches"], 1)
        forms[precision] = dict(res=res, sec=sec, tm=tm, walk_avg_ms=walk_avg_ms, renum_avg_ms=renum_avg_ms,
                                gteps=res.iterations * nnz / sec / 1e9)
        print(f"[bench] rmat{scale} {precision}: r={res.iterations} status={res.status} {sec * 1e3:.3f} ms/step "
              f"walk_step {walk_avg_ms * 1e3:.1f} us, renumbering step {renum_avg_ms * 1e3:.1f} us", flush=True)

    # The same FP32 run without the internal renumbering, for context.
    katz.tuning_set(**tunings["fp32"])
    res_nr, sec_nr, tm_nr = time_form(katz, torch, rp_t, col_t, k, "fp32", max(1, args.steps // 5), 1,
                                      flags=katz.FLAG_NO_REORDER)
    print(f"[bench] rmat{scale} fp32 caller order: {sec_nr * 1e3:.3f} ms/step", flush=True)

    f32, f64 = forms["fp32"], forms["fp64"]
    bytes_step = algorithmic_bytes_per_walk_step(n, nnz, "fp32", rp64)
    achieved = bytes_step / (f32["walk_avg_ms"] * 1e-3) / 1e9
    tuning = {p: dict(t, arg=tuning_arg(t)) for p, t in tunings.items()}
    traffic, traffic_note = measured_traffic(scale, tuning["fp32"]["arg"])
    out = {
        "value": round(f32["gteps"], 3),
        "ms_per_step": round(f32["sec"] * 1e3, 4),
        "config": {
            "workload": wl["name"],
            "graph": f"R-MAT scale {scale}, edge factor {EDGE_FACTOR}, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, "
                     f"deduplicated, no self-loops, seeded relabel, seed {wl['seed']}",
            "n": n, "nnz_directed": nnz, "deg_max": dmax, "k": k, "eps": EPS,
            "alpha": "1/(1+deg_max)", "row_ptr": "int64" if rp64 else "int32",
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
            "renumber_step_avg_us": round(f64["renum_avg_ms"] * 1e3, 2),
            "walk_step_hbm_gbs": round(algorithmic_bytes_per_walk_step(n, nnz, "fp64", rp64)
                                       / (f64["walk_avg_ms"] * 1e-3) / 1e9, 1),
        },
        "speedup_fp32_vs_fp64": round(f64["sec"] / f32["sec"], 3),
        "walk_step_gteps_fp32": round(nnz / (f32["walk_avg_ms"] * 1e-3) / 1e9, 2),
        "phase_ms_per_step_fp32": {
            key: round(f32["tm"][key] / max(f32["tm"]["calls"], 1), 4)
            for key in ("prep_ms", "walk_first_ms", "renumber_step_ms", "walk_step_ms", "select_ms", "result_ms",
                        "call_ms")
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "walk_step_grouped<fp32>" if tunings["fp32"].get("walk_groups") == 4 else "walk_step<fp32>",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_note": traffic_note,
            "bytes_per_launch": bytes_step,
            "avg_launch_us": round(f32["walk_avg_ms"] * 1e3, 2),
            "walk_steps_timed": f32["tm"]["calls"] * (f32["res"].iterations - 2),
            "launches_timed": f32["tm"]["walk_step_launches"],
            "renumber_step_avg_us": round(f32["renum_avg_ms"] * 1e3, 2),
        },
        "fp32_caller_order": {
            "ms_per_step": round(sec_nr * 1e3, 4),
            "walk_step_avg_us": round(tm_nr["walk_step_ms"] / max(tm_nr["calls"] * (res_nr.iterations - 1), 1)
                                      * 1e3, 2),
            "same_result": bool(torch.equal(res_nr.topk, f32["res"].topk)
                                and torch.equal(res_nr.lower, f32["res"].lower)),
        },
        "fp32_fp64_same_topk": bool(torch.equal(f32["res"].topk, f64["res"].topk)),
        "tuning": tuning,
    }
    return out, (rp_t, col_t, f32["res"], f64["res"], dmax)


def oracle_leg(args, np, torch, rp_t, col_t, k, r32, r64, dmax):
    """CPU baseline: the C++/OpenMP FP64 oracle's full certified run on every
    host core (about ten seconds at R-MAT 27), which also checks the top-k of
    both forms, plus a single-thread walk over a leading row range."""
    from oracle import cpp as ocpp
    t = time.perf_counter()
    rp = rp_t.to(torch.int64).cpu().numpy()
    col = col_t.cpu().numpy()
    n, nnz = rp.size - 1, int(rp[-1])
    print(f"[bench] graph copied to the host ({time.perf_counter() - t:.1f}s)", flush=True)
    cores = ocpp.max_threads()
    t = time.perf_counter()
    orc = ocpp.rank_static(rp, col, None, k, EPS, full=False, threads=cores)
    sec = time.perf_counter() - t
    # One thread: the walk over a leading row range of about 1/32 of the arcs.
    hi = int(np.searchsorted(rp, nnz // 32))
    x = np.ones(n)
    t = time.perf_counter()
    ocpp.walk_rows(rp, col, 1.0 / (1 + dmax), 0, hi, x, threads=1)
    sec_st = time.perf_counter() - t
    del x
    out = {"cpu_baseline": {
        "value": round(orc.iterations * nnz / sec / 1e9, 5),
        "unit": "GTEPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"one full certified run of the C++ FP64 oracle (Algorithm 1, top-{k}, eps={EPS}) on the whole "
                  f"graph with {cores} OpenMP threads: {sec:.2f} s, r={orc.iterations}",
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "single_thread_walk_gteps": round(int(rp[hi]) / sec_st / 1e9, 5),
        "single_thread_sample": f"walk step of rows 0..{hi - 1} ({int(rp[hi])} arcs), one thread, {sec_st:.2f} s",
    }}
    ids32, ids64 = r32.topk.cpu().numpy(), r64.topk.cpu().numpy()
    same32 = bool(np.array_equal(ids32, orc.topk))
    out["topk_equal_oracle"] = {"fp32": same32, "fp64": bool(np.array_equal(ids64, orc.topk)),
                                "oracle_iterations": orc.iterations, "oracle_status": orc.status}
    if same32:
        lo32 = r32.lower.cpu().numpy()
        out["fp32_max_rel_err_vs_oracle"] = float(np.max(np.abs(lo32 - orc.lower) / orc.lower))
    print(f"[bench] cpu baseline {out['cpu_baseline']} parity {out['topk_equal_oracle']}", flush=True)
    return out


def bench_extras(args, katz, sg, torch, np):
    """The other stopping criteria of Section 3.1 (ranking with k = n, score,
    pair), inbound Katz on a directed graph (Section 2.1) and the comparison
    methods (Foster's heuristic, CG on Eq. (la)), on R-MAT graphs of 2^scale
    nodes.  Each form: the mean of `steps` device calls after `warmup`, the
    walk step's rate from the device timers against its algorithmic bytes, and
    the oracle's time for one call on the same graph beside it."""
    import oracle
    from oracle.katz import PAIR, RANKING, SCORE, TOPK
    scale = args.extras_scale
    eps = 1e-6
    rp, col = sg.rmat(scale, EDGE_FACTOR, 0.57, 0.19, 0.19, seed=5)
    drp, dcol = sg.rmat_directed(scale, EDGE_FACTOR, seed=6)
    n, nnz = len(rp) - 1, int(rp[-1])
    dev = lambda a, b: (torch.from_numpy(np.asarray(a, np.int64)).cuda(), torch.from_numpy(np.asarray(b, np.int32)).cuda())
    g_und, g_dir = dev(rp, col), dev(drp, dcol)
    alpha = 1.0 / (1 + int(np.max(np.diff(rp))))
    out = {}

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        katz.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        tm = katz.timing_read()
        katz.timing_enable(False)
        return res, ms, tm

    def walk_rate(tm, nn, mm, precision):
        if tm["walk_step_launches"] == 0:
            return {}
        us = tm["walk_step_ms"] * 1e3 / tm["walk_step_launches"]
        gbs = algorithmic_bytes_per_walk_step(nn, mm, precision, True) / us / 1e3
        return {"walk_step_avg_us": round(us, 1), "walk_step_gbs": round(gbs, 1), "walk_step_frac": round(gbs / 8000.0, 4)}

    def oracle_time(fn):
        t0 = time.perf_counter()
        r = fn()
        return r, round(time.perf_counter() - t0, 3)

    forms = [("ranking", dict(criterion="ranking")), ("score", dict(criterion="score")),
             ("topk1000", dict(criterion="topk"))]
    for name, kw in forms:
        k = n if name != "topk1000" else 1000
        res, ms, tm = timed(lambda: katz.rank_static(*g_und, k, alpha=alpha, eps=eps, precision="fp32", **kw))
        crit = {"ranking": RANKING, "score": SCORE, "topk1000": TOPK}[name]
        orc, ot = oracle_time(lambda: oracle.rank_static(rp, col, alpha, 1000, eps, criterion=crit))
        ids = res.topk.cpu().numpy()[:100]
        out[name] = {"ms": round(ms, 3), "iterations": res.iterations, "status": res.status,
                     "separated_fraction": None if res.separated_fraction != res.separated_fraction
                     else round(res.separated_fraction, 6),
                     "oracle_s": ot, "oracle_iterations": orc.iterations, "oracle_status": orc.status,
                     "first100_equal_oracle": bool(np.array_equal(ids, np.asarray(orc.topk)[:100]))}
        out[name].update(walk_rate(tm, n, nnz, "fp32"))
    top2 = [int(v) for v in katz.rank_static(*g_und, 2, alpha=alpha, eps=eps, precision="fp32").topk.cpu()]
    res, ms, tm = timed(lambda: katz.rank_static(*g_und, 2, alpha=alpha, eps=eps, precision="fp32", criterion="pair",
                                                 pair=(top2[0], top2[1])))
    orc, ot = oracle_time(lambda: oracle.rank_static(rp, col, alpha, 2, eps, criterion=PAIR,
                                                     pair=(top2[0], top2[1])))
    out["pair"] = {"ms": round(ms, 3), "pair": top2, "iterations": res.iterations, "status": res.status,
                   "oracle_s": ot, "oracle_iterations": orc.iterations, "oracle_status": orc.status,
                   "order_equal_oracle": bool(np.array_equal(res.topk.cpu().numpy(), np.asarray(orc.topk)))}
    out["pair"].update(walk_rate(tm, n, nnz, "fp32"))
    trp, tcol = oracle.reverse_graph(drp, dcol)
    dalpha = 1.0 / (1 + int(np.max(np.diff(trp))))
    res, ms, tm = timed(lambda: katz.rank_static(*g_dir, 1000, alpha=dalpha, eps=eps, precision="fp32",
                                                 undirected=False, flags=katz.FLAG_INBOUND))
    orc, ot = oracle_time(lambda: oracle.rank_static(trp, tcol, dalpha, 1000, eps, undirected=False))
    out["inbound_topk1000"] = {"ms": round(ms, 3), "nnz": int(drp[-1]), "iterations": res.iterations,
                               "status": res.status, "oracle_s": ot, "oracle_iterations": orc.iterations,
                               "topk_equal_oracle": bool(np.array_equal(res.topk.cpu().numpy(), np.asarray(orc.topk)))}
    out["inbound_topk1000"].update(walk_rate(tm, n, int(drp[-1]), "fp32"))
    for method, ofn in (("foster", lambda: oracle.foster(rp, col, alpha, tol=1e-9)),
                        ("cg", lambda: oracle.conjugate_gradient(rp, col, alpha, tol=1e-12))):
        tol = 1e-9 if method == "foster" else 1e-12
        (sc, info, st), ms, tm = timed(lambda: katz.solve(*g_und, method, tol, alpha=alpha))
        o, ot = oracle_time(ofn)
        oscore = np.asarray(o.scores)
        rel = float(np.max(np.abs(sc.cpu().numpy() - oscore) / np.maximum(np.abs(oscore), 1e-300)))
        out[method] = {"ms": round(ms, 3), "tol": tol, "iterations": info.get("iterations"), "status": st,
                       "oracle_s": ot, "oracle_iterations": o.iterations, "max_rel_diff_oracle": rel}
    line = {"metric": "other criteria, inbound Katz and comparison methods: ms per call, 1 GPU",
            "value": out["ranking"]["ms"], "unit": "ms per ranking call (k = n)", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out["ranking"]["ms"], "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"rmat{scale}_extras", "n": n, "nnz_directed": nnz, "eps": eps,
                       "alpha": "1/(1+deg_max)", "oracle": "numpy/scipy oracle, one call on the same graph"},
            "forms": out}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--workload", default="static",
                    choices=["static", "static27", "static22", "batched", "serving", "extras"],
                    help="static: R-MAT 27 (the headline line) with R-MAT 22 beside it; static27 / static22: "
                         "one of them alone; batched: 256 Barabasi-Albert graphs; serving: update batches "
                         "against R-MAT 24")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests per load point")
    ap.add_argument("--graphs", type=int, default=256, help="batched: number of graphs")
    ap.add_argument("--serving-scale", type=int, default=24, help="serving: R-MAT scale of the resident graph")
    ap.add_argument("--extras-scale", type=int, default=22, help="extras: R-MAT scale of the graphs")
    ap.add_argument("--serving-precision", default="fp64", choices=["fp64", "fp32"],
                    help="serving: form of the resident state (FP32: scaled walk history, Section 3.3 margin)")
    ap.add_argument("--batched-max-log2n", type=int, default=18, help="batched: n is log-uniform in [2^10, 2^this]")
    ap.add_argument("--tuning", default="auto",
                    help="walk launch shape: 'auto' (katz_autotune per precision before timing), "
                         "or HUB_BYTES:BLOCKS_PER_CU[:WALK_GROUPS[:B0,B1,B2,B3,B4,B5]] for both precisions "
                         "(B: the row-length classes of the binning)")
    ap.add_argument("--tuning-sweep", action="store_true",
                    help="batched: also time every autotuner candidate and report them")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(a graph, its bins and its walk vectors live on one device)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthgraph as sg
    import paper_1807_03847_amd.katz as katz

    if args.workload == "batched":
        return bench_batched(args, katz, sg, torch, np)
    if args.workload == "serving":
        return bench_serving(args, katz, sg, torch, np)
    if args.workload == "extras":
        return bench_extras(args, katz, sg, torch, np)

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {args.copy_mib} MiB read + {args.copy_mib} MiB written", flush=True)
        del src, dst

    head = WORKLOADS[22 if args.workload == "static22" else 27]
    fields, (rp_t, col_t, r32, r64, dmax) = run_static(args, katz, sg, torch, np, head)
    out = {
        "metric": "certified top-k Katz ranking: GTEPS and % HBM peak, FP32-SpMV vs FP64, 1 GPU",
        "value": fields.pop("value"),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fields.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
    }
    out.update(fields)
    if not args.no_cpu_baseline:
        out.update(oracle_leg(args, np, torch, rp_t, col_t, head["k"], r32, r64, dmax))
    del rp_t, col_t, r32, r64
    torch.cuda.empty_cache()
    if args.workload == "static":
        extra, _ = run_static(args, katz, sg, torch, np, WORKLOADS[22])
        out["rmat22"] = extra
    print(json.dumps(out), flush=True)


def bench_batched(args, katz, sg, torch, np):
    """256 Barabasi-Albert graphs, n log-uniform in [2^10, 2^18], m in 4..32 new
    edges per node, alpha_g = f_g / (1 + d_max,g) with f_g in (0, 1], k_g in
    [10, 500], eps_g = 1e-6 f_g (seeds 1..256); one katz_rank_static call with
    count = 256, FP32 walk vector with FP64 bounds."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(2026)
    specs = []
    for gidx in range(args.graphs):
        n = int(round(2 ** rng.uniform(10, args.batched_max_log2n)))
        m = int(rng.integers(4, 33))
        specs.append((n, m, gidx + 1, float(rng.uniform(1e-3, 1.0)), int(rng.integers(10, 501))))
    t = time.perf_counter()
    with ThreadPoolExecutor(16) as ex:
        csrs = list(ex.map(lambda sp: sg.barabasi_albert(sp[0], sp[1], sp[2]), specs))
    nnz = sum(int(rp[-1]) for rp, _ in csrs)
    ntot = sum(len(rp) - 1 for rp, _ in csrs)
    print(f"[bench] batched graphs generated: {len(csrs)} graphs, n={ntot} nnz={nnz} "
          f"({time.perf_counter() - t:.1f}s)", flush=True)
    graphs = [(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), True) for rp, col in csrs]
    params = []
    for (rp, col), (n, m, seed, f, k) in zip(csrs, specs):
        params.append(dict(k=min(k, n), alpha=f / (1 + int(np.max(np.diff(rp)))), eps=1e-6 * f, precision="fp32"))
    torch.cuda.synchronize()
    tuning = katz.autotune_batch(graphs, params)
    print(f"[bench] batched tuning {tuning}", flush=True)
    for _ in range(args.warmup):
        res = katz.rank_static_batch(graphs, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = katz.rank_static_batch(graphs, params)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    traversed = sum(r.iterations * int(rp[-1]) for r, (rp, _) in zip(res, csrs))
    out = {
        "metric": f"batched certified top-k Katz ranking: GTEPS over {len(csrs)} graphs, one call, 1 GPU",
        "value": round(traversed / sec / 1e9, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ba{len(csrs)}_batched", "graphs": len(csrs), "n_total": ntot, "nnz_total": nnz,
                   "iterations_max": max(r.iterations for r in res),
                   "iterations_min": min(r.iterations for r in res)},
        "status_counts": {str(st): sum(1 for r in res if r.status == st) for st in sorted({r.status for r in res})},
        "tuning": tuning,
    }
    if args.tuning_sweep:
        sweep = []
        for bbpc, tile, xcd in [(0, 1, 0), (0, 1, 1), (4, 4, 0), (4, 4, 1), (16, 4, 0), (16, 4, 1), (16, 8, 0),
                                (16, 8, 1), (32, 8, 1)]:
            katz.tuning_set(**dict(tuning, batch_blocks_per_cu=bbpc, batch_tile=tile, batch_xcd=xcd))
            katz.rank_static_batch(graphs, params)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(2):
                r2 = katz.rank_static_batch(graphs, params)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) / 2 * 1e3
            same = all(bool(torch.equal(a.topk, b.topk) and torch.equal(a.lower, b.lower)) for a, b in zip(r2, res))
            sweep.append({"batch_blocks_per_cu": bbpc, "batch_tile": tile, "batch_xcd": xcd,
                          "ms_per_step": round(ms, 3), "same_result": same})
            print(f"[bench] batched sweep {bbpc}:{tile}:{xcd} {ms:.3f} ms same={same}", flush=True)
        out["tuning_sweep"] = sweep
        katz.tuning_set(**tuning)
    print(json.dumps(out), flush=True)


def serving_requests(rp, col, n, count, rng, np, sg, scale, seed):
    """Update batches of size round(10^U(0,4)): 70% insertions whose endpoints
    are drawn from the graph's own R-MAT distribution (same quadrant recursion
    and relabelling as the graph, a separate counter stream), rejecting
    self-loops, existing edges and repeats; 30% deletions of original edges
    (each at most once, uniform)."""
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    keys = src * n + col
    und = np.nonzero(src < col)[0]
    order = rng.permutation(und.size)
    taken = 0
    inserted = set()
    pool = np.empty((0, 2), dtype=np.int64)   # R-MAT endpoint pairs, drawn a million at a time
    drawn = 0
    out = []
    for _ in range(count):
        size = max(1, int(round(10 ** rng.uniform(0, 4))))
        n_del = int(round(0.3 * size))
        n_ins = size - n_del
        di = und[order[taken:taken + n_del]]
        taken += n_del
        dels = np.stack([src[di], col[di].astype(np.int64)], 1)
        ins = []
        while len(ins) < n_ins:
            want = 2 * (n_ins - len(ins)) + 8
            if pool.shape[0] < want:
                pool = np.concatenate([pool, sg.rmat_pairs(scale, 1 << 20, seed=seed, stream=11, first=drawn)])
                drawn += 1 << 20
            pairs, pool = pool[:want], pool[want:]
            lo, hi = np.minimum(pairs[:, 0], pairs[:, 1]), np.maximum(pairs[:, 0], pairs[:, 1])
            cand = lo * n + hi
            pos = np.searchsorted(keys, cand)
            present = (pos < keys.size) & (keys[np.minimum(pos, keys.size - 1)] == cand)
            for x, y, pr in zip(lo.tolist(), hi.tolist(), present.tolist()):
                if x != y and not pr and (x, y) not in inserted:
                    inserted.add((x, y))
                    ins.append((x, y))
                    if len(ins) == n_ins:
                        break
        out.append((np.array(ins, dtype=np.int64).reshape(-1, 2), dels))
    return out


def bench_serving(args, katz, sg, torch, np):
    """R-MAT scale 24 (seed 2) resident on the device; alpha = 1/(1 + d_max + 1e5),
    degree cap d_max + 1e5, k = 100, eps = 1e-6; update batches arrive as a
    Poisson process at a fraction of the measured saturation rate."""
    import threading
    t = time.perf_counter()
    rp, col = sg.rmat(args.serving_scale, 16, 0.57, 0.19, 0.19, seed=2)
    n = len(rp) - 1
    dmax = int(np.max(np.diff(rp)))
    H = 100000
    print(f"[bench] serving graph: n={n} nnz={int(rp[-1])} dmax={dmax} ({time.perf_counter() - t:.1f}s)", flush=True)
    rng = np.random.default_rng(24)
    total = args.requests * 3
    reqs = serving_requests(rp, col, n, total, rng, np, sg, args.serving_scale, 2)
    print(f"[bench] {total} requests generated, {sum(len(a) + len(b) for a, b in reqs)} edge updates", flush=True)
    rp_t, col_t = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    # The launch shape of the state's whole-graph walks (creation, dense
    # re-walk levels, resumed iterations): the autotuner's choice for a
    # static FP64 ranking of the resident graph.
    prec = args.serving_precision
    tuning = katz.autotune(rp_t, col_t, 100, eps=1e-6, precision=prec)
    print(f"[bench] serving tuning {tuning}", flush=True)
    sv = katz.Server(slots=4)
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    gid, _ = sv.add_graph(rp_t, col_t, 100, alpha=1.0 / (1 + dmax + H), eps=1e-6, degree_cap=dmax + H,
                          precision=prec)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t_create) * 1e3
    print(f"[bench] state created (checks, slack CSR, renumbering, first certified ranking) in {create_ms:.1f} ms",
          flush=True)
    # Saturation: the first block of requests submitted at once.
    block = reqs[:args.requests]
    t0 = time.perf_counter()
    tick = [sv.submit(gid, a, b) for a, b in block]
    svc = [sv.wait(tk)[2] for tk in tick]
    sat = len(block) / (time.perf_counter() - t0)
    print(f"[bench] saturation {sat:.1f} req/s", flush=True)
    points = []
    for frac, chunk in ((0.5, reqs[args.requests:2 * args.requests]), (0.8, reqs[2 * args.requests:])):
        lam = frac * sat
        gaps = rng.exponential(1.0 / lam, len(chunk))
        tickets = []

        def submitter():
            t_next = time.perf_counter()
            for (a, b), gap in zip(chunk, gaps):
                t_next += gap
                delay = t_next - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets.append(sv.submit(gid, a, b))

        t0 = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        lat = []
        i = 0
        while i < len(chunk):
            if i < len(tickets):
                lat.append(sv.wait(tickets[i])[1])
                i += 1
            else:
                time.sleep(0.0005)
        th.join()
        wall = time.perf_counter() - t0
        edges = sum(len(a) + len(b) for a, b in chunk)
        points.append({"load": frac, "arrival_rate": round(lam, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                       "p99_ms": round(float(np.percentile(lat, 99)), 3), "requests_per_s": round(len(chunk) / wall, 2),
                       "edge_updates_per_s": round(edges / wall, 1)})
        print(f"[bench] load {frac}: {points[-1]}", flush=True)
    sv.close()
    out = {
        "metric": "serving dynamic updates: p50/p99 latency and throughput, 1 GPU",
        "value": points[0]["p50_ms"], "unit": "ms p50 latency at 50% load", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0, "ms_per_step": round(float(np.mean(svc)), 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"rmat{args.serving_scale}_serving", "form": prec, "n": n, "nnz_directed": int(rp[-1]), "k": 100, "eps": 1e-6,
                   "batch": "round(10^U(0,4)) edges, 70% insertions", "slots": 4},
        "saturation_requests_per_s": round(sat, 2), "load_points": points, "tuning": tuning,
        "state_create_ms": round(create_ms, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
