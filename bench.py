"""Benchmark: apply points/s (forward + adjoint) of the skeletonization FMM on
3D Laplace, N = 2^20 points uniform in the unit cube, leaf <= 128, ID tolerance
1e-7, on one MI355X.

A step is one forward apply u = Atilde q followed by one adjoint apply
w = Atilde^H v (the whole GPU sweep each: gather, upward pass, near field,
downward pass, output), inputs resident in HBM.  value = N * nrhs / (time of
one step).  The run also reports each path's error against the float64 dense
sum on 2,048 random targets, the near-field kernel's arithmetic roofline (HIP
events around that pass, on the apply's stream), the transfer passes' HBM
rate, and the CPU oracle timed on a bounded sample of the same workload.

It also times the eight-geometry, 64-RHS float32 batch (one captured hipGraph
holding a batched forward and a batched adjoint sweep) and reports it beside
the float64 single-RHS rate of the 1M cube.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only f32|f64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Vector ALU peaks (published): float32 157.3 TFLOP/s = 256 CUs x 4 SIMDs x 32 lanes
# x 2.4 GHz x 2 flops -- a plain (non-packed) float32 multiply-add issues in two
# cycles per wave of 64 -- and float64 78.6 TFLOP/s (four cycles per wave).  Each
# path is priced against the peak of its evaluation type.
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# Issue cycles per wave instruction (64 lanes) used for the instruction-mix bound of
# the float32 pair kernel: float64 add / multiply-add and the float64 -> float32
# conversion 4, float32 multiply-add 2, reciprocal square root 16.  The cheapest
# evaluation of a symmetric pair (expanded |d|^2: one float64 add and three float64
# multiply-adds; one conversion; one reciprocal square root; two float32
# multiply-adds) therefore costs 40 cycles per wave of 64 pairs.
CLOCK_GHZ = 2.4
SIMDS = 1024
MIX_CYCLES_PER_64_SYM_PAIRS = {"f32": 4 * 4 + 4 + 16 + 2 * 2}
PEAK_HBM_GBS = 8000.0
# algorithmic flops of one 3D Laplace pair in k_near: 3 subtractions, |d|^2
# (3 mul + 2 add), one reciprocal square root, one multiply-add into u; a skeleton
# pair adds one multiply-add into uhat.  A symmetric pair item serves both orders:
# the same evaluation plus a second multiply-add (into the source side), and two
# uhat multiply-adds for a skeleton pair.
FLOPS_PER_PAIR = 11
FLOPS_PER_SKEL_PAIR = 2
FLOPS_PER_SYM_PAIR = 13
FLOPS_PER_SYM_SKEL_PAIR = 4
# HBM bytes per near-field launch from rocprofv3 FETCH_SIZE + WRITE_SIZE runs of this
# workload (scaled by a plain 512 MiB copy: x2.000 fetch, x1.000 write), per
# targets-per-lane variant, valid only for the kernel and kernel source they were
# measured on (first 16 hex digits of the source's sha256).
NEAR_TRAFFIC = {"f32": {"kernel": "k_near_sym", "kernels_sha256": "542e57b9110cce95",
                        "bytes_by_tpl": {
                          1: 6.4410e+09 + 2.0518e+09,
                          2: 3.9893e+09 + 1.5460e+09,
                          3: 2.8289e+09 + 1.0113e+09,
                          4: 1.9410e+09 + 7.4405e+08}}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work to sample")
    ap.add_argument("--profile-only", action="store_true", help="skip accuracy checks and baseline")
    ap.add_argument("--only", choices=["f32", "f64"], default=None, help="time one path only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the eight-geometry, 64-RHS float32 batched measurement")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched measurement and print its object (for profiling)")
    return ap.parse_args()


def pair_counts(P) -> np.ndarray:
    """Kernel evaluations the oracle's apply does per target box (all pairs it visits)."""
    nb = P["n_boxes"]
    n = np.diff(P["idx_ptr"])
    k = np.maximum(P["rank"], 0)
    top = P["top_level"]
    lev = P["level"]
    cnt = np.zeros(nb, dtype=np.float64)
    tops = np.nonzero(lev == top)[0]
    ntop = n[tops].sum()
    for b in range(nb):
        if lev[b] < top:
            continue
        c = 0.0
        if lev[b] == top:
            c += n[b] * ntop
        else:
            cl = P["coll_idx"][P["coll_ptr"][b]:P["coll_ptr"][b + 1]]
            c += n[b] * n[cl].sum() + k[b] * k[cl].sum()
            co = P["coarse_idx"][P["coarse_ptr"][b]:P["coarse_ptr"][b + 1]]
            c += (n[b] + k[b]) * n[co].sum()
        if P["is_leaf"][b]:
            fi = P["fine_idx"][P["fine_ptr"][b]:P["fine_ptr"][b + 1]]
            c += n[b] * (n[fi] + k[fi]).sum()
        cnt[b] = c
    return cnt


def cpu_baseline(P, q, v, budget_s: float, nrhs: int = 1):
    """Time the oracle's float64 apply (O2) of the same skeleton operators on the
    host cores: the full forward apply, then the full adjoint apply when both fit
    the budget.  A forward apply longer than the budget is instead timed on a
    random sample of target boxes (upward and downward passes in full) and
    scaled by the pair counts, with the adjoint taken equal to it."""
    import oracle

    n = P["points"].shape[0]
    cores = oracle.num_threads()
    cnt = pair_counts(P)
    total = cnt.sum()
    rng = np.random.default_rng(77)
    mask0 = np.zeros(P["n_boxes"], dtype=np.uint8)
    t0 = time.perf_counter()
    oracle.apply(P, q, box_mask=mask0)
    t_base = time.perf_counter() - t0
    frac = 5e-2
    mask = (rng.random(P["n_boxes"]) < frac).astype(np.uint8)
    t0 = time.perf_counter()
    oracle.apply(P, q, box_mask=mask)
    t_cal = max(time.perf_counter() - t0 - t_base, 1e-3)
    est_full = t_base + t_cal * total / max(cnt[mask == 1].sum(), 1.0)
    if est_full <= budget_s:
        t0 = time.perf_counter()
        oracle.apply(P, q)
        t_f = time.perf_counter() - t0
        if 2 * t_f <= 1.5 * budget_s:
            t0 = time.perf_counter()
            oracle.apply(P, v, adjoint=True)
            t_a = time.perf_counter() - t0
            return {"value": n * nrhs / (t_f + t_a), "unit": "points/s", "cores": cores, "kind": "oracle",
                    "sample": (f"CPU float64 apply (oracle O2) of the same skeleton operators, whole workload: "
                               f"forward {t_f:.1f}s + adjoint {t_a:.1f}s")}
        return {"value": n * nrhs / (2 * t_f), "unit": "points/s", "cores": cores, "kind": "oracle",
                "sample": (f"CPU float64 apply (oracle O2) of the same skeleton operators: full forward "
                           f"{t_f:.1f}s, adjoint taken equal")}
    frac = min(1.0, budget_s * (total / max(est_full - t_base, 1e-3)) / total)
    mask = (rng.random(P["n_boxes"]) < frac).astype(np.uint8)
    t0 = time.perf_counter()
    oracle.apply(P, q, box_mask=mask)
    t_s = time.perf_counter() - t0
    sampled = cnt[mask == 1].sum()
    t_full = t_base + (t_s - t_base) * total / max(sampled, 1.0)
    return {
        "value": n * nrhs / (2.0 * t_full),
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"CPU float64 apply (oracle O2) of the same skeleton operators; translations for "
                   f"{int(mask.sum())} of {P['n_boxes']} target boxes ({100 * sampled / total:.2f}% of "
                   f"{total:.3e} pair evaluations) in {t_s:.1f}s, upward/downward passes in full "
                   f"({t_base:.1f}s); forward+adjoint time extrapolated as 2 x {t_full:.1f}s"),
    }


def batched_run(steps: int, warmup: int):
    """Eight 3D Laplace geometries (65,536 .. 2,097,152 points, cube / ellipsoid,
    tol 1e-6, leaf 128), 64 float32 right-hand sides each: one captured hipGraph
    holds a batched forward sweep and a batched adjoint sweep; value = total
    points x RHS per second of that step."""
    import torch

    import workloads
    import paper_2310_16668_amd as sk

    wls = workloads.batch_workloads()
    t0 = time.perf_counter()
    ops = [sk.build(w.points(), "laplace", tol=w.tol, leaf_size=w.leaf_size) for w in wls]
    t_build = time.perf_counter() - t0
    batch = sk.Batch(ops)
    dev = torch.device("cuda:0")
    q = [torch.from_numpy(w.charges()).to(dev, torch.float32) for w in wls]
    v = [torch.from_numpy(w.weights()).to(dev, torch.float32) for w in wls]
    batch.apply(q)
    batch.apply(v, adjoint=True)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.apply(q)
        batch.apply(v, adjoint=True)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    n_total = sum(w.n for w in wls)
    return {"value": n_total * 64 / (ms * 1e-3), "unit": "points x RHS/s (fwd+adjoint)", "ms_per_step": ms,
            "n_total": n_total, "sizes": [w.n for w in wls], "nrhs": 64, "dtype": "f32", "graph": True,
            "build_s": t_build}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: --gpus must be 1 (the apply does not shard across GPUs)"}))
        return 2
    if args.batched_only:
        print(json.dumps({"batched": batched_run(args.steps, args.warmup)}))
        return 0
    import torch

    import workloads
    import paper_2310_16668_amd as sk

    w = workloads.LAPLACE3D_1M
    x = w.points()
    q_h = w.charges()
    v_h = w.weights()
    log(f"[bench] building {w.name}: N={w.n} leaf={w.leaf_size} tol={w.tol}")
    t0 = time.perf_counter()
    op = sk.build(x, "laplace", tol=w.tol, leaf_size=w.leaf_size)
    t_build = time.perf_counter() - t0
    st = op.stats()
    log(f"[bench] build {t_build:.1f}s levels={st['max_level']} k_max={st['k_max']} "
        f"pairs={st['pairs_near']:.3e} skel_pairs={st['pairs_skel']:.3e}")

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    results = {}
    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calibrate_copy} MiB done")
        del a, b
    paths = [("f64", torch.float64), ("f32", torch.float32)]
    if args.only:
        paths = [p for p in paths if p[0] == args.only]
    tuned = {}
    for dt_name, tdt in paths:
        op.prepare(1, tdt)
        if not args.no_autotune:
            tuned[dt_name] = op.autotune(tdt)
            log(f"[bench] {dt_name} autotune {tuned[dt_name]}")
        q = torch.from_numpy(q_h).to(dev, tdt)
        v = torch.from_numpy(v_h).to(dev, tdt)
        for _ in range(args.warmup):
            op.apply(q)
            op.apply_adjoint(v)
        # the timed region: K steps; the library records HIP events around each
        # pass on the apply's stream (the per-kernel durations of the roofline)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        op.timing(True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            u = op.apply(q)
            wv = op.apply_adjoint(v)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / args.steps
        passes = op.timing_read()
        op.timing(False)
        res = {"ms_per_step": ms_step, "passes_ms_per_sweep": {k: passes[k] / passes["sweeps"] for k in sk.PASSES}}
        if not args.profile_only:
            import oracle
            tg = w.targets()
            u1 = oracle.direct(x, q_h, targets=tg)
            uu = u.double().cpu().numpy()
            res["relerr_vs_direct"] = float(np.linalg.norm(uu[tg] - u1) / np.linalg.norm(u1))
            ww = wv.double().cpu().numpy()
            w1 = oracle.direct(x, v_h, targets=tg)   # Laplace: A^H = A
            res["relerr_adjoint_vs_direct"] = float(np.linalg.norm(ww[tg] - w1) / np.linalg.norm(w1))
        results[dt_name] = res
        log(f"[bench] {dt_name}: {ms_step:.3f} ms/step {res}")

    # headline: the requested path, else the fastest path within 1e-6 of the dense sum
    if args.only:
        chosen = args.only
    else:
        ok = [k for k, v in results.items() if v.get("relerr_vs_direct", 0.0) <= 1e-6
              and v.get("relerr_adjoint_vs_direct", 0.0) <= 1e-6]
        chosen = min(ok or list(results), key=lambda k: results[k]["ms_per_step"])
    r = results[chosen]
    pm = r["passes_ms_per_sweep"]
    # pair counts at the headline path's targets per lane (the diagonal tiles depend on it)
    if chosen in tuned:
        op.set_targets_per_lane(tuned[chosen]["targets_per_lane"])
    st = op.stats()
    # pairs left to k_near after symmetric pairing (each paired evaluation covers two)
    pairs_ns = st["pairs_near"] - 2 * st["pairs_sym"] - st["pairs_tile"]
    skel_ns = st["pairs_skel"] - 2 * st["pairs_sym_skel"] - st["pairs_tile_skel"]
    # per near-field kernel: (ms per launch, algorithmic flops per launch)
    kernels = {
        "k_near": (pm["near_field"], FLOPS_PER_PAIR * pairs_ns + FLOPS_PER_SKEL_PAIR * skel_ns),
        "k_near_sym": (pm["near_pairs"], FLOPS_PER_SYM_PAIR * st["pairs_sym"]
                       + FLOPS_PER_SYM_SKEL_PAIR * st["pairs_sym_skel"]
                       + FLOPS_PER_PAIR * st["pairs_tile"] + FLOPS_PER_SKEL_PAIR * st["pairs_tile_skel"]),
    }
    dom = max(kernels, key=lambda k: kernels[k][0])
    near_ms, flops = kernels[dom]
    achieved = flops / (near_ms * 1e-3) / 1e12
    import hashlib
    src = os.path.join(ROOT, "paper_2310_16668_amd", "csrc", "device", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    tr = NEAR_TRAFFIC.get(chosen)
    tpl = tuned.get(chosen, {}).get("targets_per_lane")
    traffic = (tr["bytes_by_tpl"].get(tpl) if tr and tr["kernels_sha256"] == digest and tr.get("kernel") == dom
               else None)
    # the same launch against its instruction mix: every evaluation (a symmetric pair,
    # or a one-direction tile pair) priced at the cheapest symmetric-pair cost
    issue_bound = None
    if dom == "k_near_sym" and chosen in MIX_CYCLES_PER_64_SYM_PAIRS:
        evals = st["pairs_sym"] + st["pairs_tile"]
        ideal_ms = evals / 64 * MIX_CYCLES_PER_64_SYM_PAIRS[chosen] / SIMDS / (CLOCK_GHZ * 1e9) * 1e3
        issue_bound = {"cycles_per_64_pairs_ideal": MIX_CYCLES_PER_64_SYM_PAIRS[chosen],
                       "cycles_per_64_pairs_achieved": near_ms * 1e-3 * CLOCK_GHZ * 1e9 * SIMDS / (evals / 64),
                       "ideal_ms": ideal_ms, "frac": ideal_ms / near_ms}
    sT = 8 if chosen == "f64" else 4
    # upward and downward each read every T once, plus their vectors (n and k entries)
    t_bytes = st["m_proj_elems"] * sT
    vec_bytes = st["n_entries"] * sT * 4
    trans_ms = r["passes_ms_per_sweep"]["upward"] + r["passes_ms_per_sweep"]["downward"]
    out = {
        "metric": "apply points/s (fwd+adjoint), 3D Laplace N=1M @1e-6 rel err; % HBM/VALU roofline",
        "value": w.n / (r["ms_per_step"] * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": chosen,
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": 3, "kernel": "laplace", "leaf_size": w.leaf_size,
                   "tol": w.tol, "nrhs": 1, "step": "forward apply + adjoint apply"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[chosen], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[chosen], "traffic": traffic,
                     "issue_bound": issue_bound,
                     "kernel": dom, "ms_per_launch": near_ms,
                     "sym_pairs_per_launch": st["pairs_sym"], "sym_skel_pairs_per_launch": st["pairs_sym_skel"],
                     "tile_pairs_per_launch": st["pairs_tile"], "tile_skel_pairs_per_launch": st["pairs_tile_skel"],
                     "segment_pairs_per_launch": pairs_ns, "segment_skel_pairs_per_launch": skel_ns,
                     "near_kernels": {k: {"ms": v[0], "tflops": v[1] / (v[0] * 1e-3) / 1e12 if v[0] > 0 else None}
                                      for k, v in kernels.items()},
                     "near_reduce_ms": pm["near_reduce"]},
        "transfer_passes": {"bound": "hbm", "bytes_per_sweep": 2 * (t_bytes + vec_bytes),
                            "ms_per_sweep": trans_ms,
                            "achieved_GBs": 2 * (t_bytes + vec_bytes) / (trans_ms * 1e-3) / 1e9,
                            "peak_GBs": PEAK_HBM_GBS},
        "paths": results,
        "autotune": tuned,
        "build_s": t_build,
    }
    if not args.no_batched and not args.profile_only:
        log("[bench] eight-geometry batched run")
        bt = batched_run(args.steps, args.warmup)
        if "f64" in results:
            # the float64 single-RHS apply (fwd + adjoint) of the 1M cube, for comparison
            f64_rate = w.n / (results["f64"]["ms_per_step"] * 1e-3)
            bt["f64_single_rhs_points_per_s"] = f64_rate
            bt["ratio_to_f64_single_rhs"] = bt["value"] / f64_rate
        out["batched"] = bt
        log(f"[bench] batched: {bt}")
    if not args.no_cpu_baseline and not args.profile_only:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(op.export(), q_h, v_h, args.cpu_budget)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
