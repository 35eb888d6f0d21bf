"""Benchmark: apply points/s (forward + adjoint) of the skeletonization FMM on
3D Laplace, N = 2^20 points uniform in the unit cube, leaf <= 128, ID tolerance
1e-7, on one MI355X.

A step is one forward apply u = Atilde q followed by one adjoint apply
w = Atilde^H v (the whole GPU sweep each: gather, upward pass, near field,
downward pass, output), inputs resident in HBM.  value = N * nrhs / (time of
one step).  The timed region holds the K steps only; per-kernel durations (the
roofline) come from a second, separate run of the same steps with the
library's HIP events around every pass on the apply's stream.

Beside the headline the run reports, each with its error against the float64
dense sum on random targets (relative l2 and max|e| / max|u|):
  * both precision paths of the 1M cube (float64, float32);
  * the float32 apply of 64 right-hand sides on the same 1M operator (the
    matrix-core path), against the float64 single-RHS apply at that accuracy;
  * the 4M-point ellipsoid (float32, compensated leaf sums);
  * the 1M-point Helmholtz cube (complex64 with float64 leaf sums, forward and
    conjugated adjoint);
  * the eight-geometry, 64-RHS float32 batch (one captured hipGraph holding a
    batched forward and a batched adjoint sweep);
  * the CPU oracle timed on a bounded sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only f32|f64]
       [--headline-only] [--batched-only]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
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
# Dense float32 matrix-core peak (published), for the many-RHS kernels.
PEAK_MFMA_F32_TFLOPS = 157.3
# Issue cycles per wave instruction (64 lanes) used for the instruction-mix bound of
# the float32 pair kernel, measured on MI355X with loop kernels of independent
# instructions (8 chains per lane, 8 waves per SIMD): float64 add / multiply-add
# and the float64 -> float32 conversion 4, float32 multiply-add 2, reciprocal
# square root 8 (it does not overlap the other VALU work of its SIMD).  The
# cheapest evaluation of a symmetric pair (expanded |d|^2: one float64 add and
# three float64 multiply-adds; one conversion; one reciprocal square root; two
# float32 multiply-adds per column) therefore costs 32 cycles per wave of 64 pairs
# with one column and 36 with the two columns of the fused forward + adjoint sweep.
CLOCK_GHZ = 2.4
SIMDS = 1024
MIX_CYCLES_PER_64_SYM_PAIRS = {"f32": 4 * 4 + 4 + 8 + 2 * 2,
                               "f32_fused": 4 * 4 + 4 + 8 + 4 * 2}
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
# One 3D Helmholtz pair: 3 subtractions, |d|^2 (5), reciprocal square root with one
# Newton step (5), r and kappa r (2), sincos (1), the kernel's real and imaginary
# parts (2), one complex multiply-add into u (8); a skeleton pair adds a complex
# multiply-add into uhat (8).  Transcendentals count one flop each.
FLOPS_PER_HELM_PAIR = 26
FLOPS_PER_HELM_SKEL_PAIR = 8
# a paired Helmholtz evaluation serves both directions: the evaluation (18) and two
# complex multiply-adds (16); a skeleton pair adds two more (16)
FLOPS_PER_HELM_SYM_PAIR = 34
FLOPS_PER_HELM_SYM_SKEL_PAIR = 16
# HBM bytes per near-field launch from rocprofv3 FETCH_SIZE + WRITE_SIZE runs of this
# workload (scaled by a plain 512 MiB copy: x2.000 fetch, x1.000 write), per
# targets-per-lane variant, valid only for the kernel and kernel source they were
# measured on (first 16 hex digits of the sha256 of the pair kernel's section of
# kernels.hip, pair_kernel_digest).
NEAR_TRAFFIC = {
    "f32": {"kernel": "k_near_sym", "kernels_sha256": "3c712fe22d9617b0",
            "bytes_by_tpl": {1: 1.0774e+10 + 2.0505e+09, 2: 6.0437e+09 + 1.2162e+09, 3: 4.6171e+09 + 9.4871e+08, 4: 3.2840e+09 + 7.4526e+08}},
    "f32_fused": {"kernel": "k_near_sym", "kernels_sha256": "3c712fe22d9617b0",
                  "bytes_by_tpl": {1: 1.4166e+10 + 4.0731e+09, 2: 7.5355e+09 + 2.4531e+09, 3: 5.6397e+09 + 1.9096e+09, 4: 3.9151e+09 + 1.4802e+09}},
    "f64": {"kernel": "k_near_sym", "kernels_sha256": "3c712fe22d9617b0",
            "bytes_by_tpl": {1: 1.1541e+10 + 2.0484e+09, 2: 6.3858e+09 + 1.2125e+09, 3: 4.8105e+09 + 9.4521e+08, 4: 3.3710e+09 + 7.4385e+08}},
}


PAIR_KERNEL_BEGIN = "// symmetric near field (real kernels, one right-hand side)"
PAIR_KERNEL_END = "// many right-hand sides on the matrix cores (real kernels, float32 policy)"


def pair_kernel_digest() -> str:
    """sha256 (16 hex digits) of the pair kernel's section of kernels.hip (k_near_sym and
    k_sym_reduce, between the two section banners)."""
    import hashlib
    src = os.path.join(ROOT, "paper_2310_16668_amd", "csrc", "device", "kernels.hip")
    text = open(src, encoding="utf-8").read()
    i, j = text.index(PAIR_KERNEL_BEGIN), text.index(PAIR_KERNEL_END)
    return hashlib.sha256(text[i:j].encode()).hexdigest()[:16]


def near_traffic(path: str, kernel: str, tpl):
    """HBM bytes per launch carried in NEAR_TRAFFIC, or None when they were taken on
    another kernel, another launch shape or another source of the pair kernel."""
    tr = NEAR_TRAFFIC.get(path)
    if not tr or tr.get("kernel") != kernel or tr["kernels_sha256"] != pair_kernel_digest():
        return None
    return tr["bytes_by_tpl"].get(tpl)


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
    ap.add_argument("--only", choices=["f32", "f64", "f32_fused"], default=None, help="time one path only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the 1M cube only (no 64-RHS, ellipsoid, Helmholtz or batched legs)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the eight-geometry, 64-RHS float32 batched measurement")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched measurement and print its object (for profiling)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# measurement helpers
# ---------------------------------------------------------------------------
def errors(u, ref) -> dict:
    """relative l2 and max|e| / max|u| (the paper's measure) of u against ref."""
    u, ref = np.asarray(u), np.asarray(ref)
    return {"rel_l2": float(np.linalg.norm(u - ref) / np.linalg.norm(ref)),
            "max_rel": float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))}


def clocks() -> dict | None:
    """Current shader and memory clocks of GPU 0 as rocm-smi reports them (None if it cannot)."""
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        d = json.loads(r.stdout)
        card = d[sorted(d)[0]]
        out = {}
        for k, v in card.items():
            kl = k.lower()
            if "sclk" in kl and "sclk" not in out:
                out["sclk"] = v
            if "mclk" in kl and "mclk" not in out:
                out["mclk"] = v
        return out or None
    except Exception:
        return None


def timed_steps(step, steps: int, warmup: int) -> float:
    """ms per step over `steps` calls of step() between device synchronisations
    (after `warmup` untimed calls)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def pass_times(obj, step, steps: int) -> dict:
    """ms per sweep of every pass, from the library's HIP events over `steps`
    further calls of step() (a separate run from the timed region)."""
    import torch
    obj.timing(True)
    torch.cuda.synchronize()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = obj.timing_read()
    obj.timing(False)
    n = max(t.pop("sweeps"), 1)
    return {k: v / n for k, v in t.items()}


def near_kernels(st: dict, pm: dict, helm: bool = False, columns: int = 1) -> dict:
    """(ms per launch, algorithmic flops per launch) of the near-field kernels;
    columns = 2 for the fused forward + adjoint sweep (each kernel value serves
    two columns: the evaluation once, the multiply-adds twice)."""
    pairs_ns = st["pairs_near"] - 2 * st["pairs_sym"] - st["pairs_tile"]
    skel_ns = st["pairs_skel"] - 2 * st["pairs_sym_skel"] - st["pairs_tile_skel"]
    if columns == 2:
        ev = FLOPS_PER_PAIR - 2   # the evaluation without its multiply-add
        return {
            "k_near": (pm["near_field"], (ev + 4) * pairs_ns + 2 * FLOPS_PER_SKEL_PAIR * skel_ns),
            "k_near_sym": (pm["near_pairs"], (ev + 8) * st["pairs_sym"] + 2 * FLOPS_PER_SYM_SKEL_PAIR * st["pairs_sym_skel"]
                           + (ev + 4) * st["pairs_tile"] + 2 * FLOPS_PER_SKEL_PAIR * st["pairs_tile_skel"]),
        }
    if helm:
        return {"k_near": (pm["near_field"], FLOPS_PER_HELM_PAIR * pairs_ns + FLOPS_PER_HELM_SKEL_PAIR * skel_ns),
                "k_near_sym_c": (pm["near_pairs"], FLOPS_PER_HELM_SYM_PAIR * st["pairs_sym"]
                                 + FLOPS_PER_HELM_SYM_SKEL_PAIR * st["pairs_sym_skel"])}
    return {
        "k_near": (pm["near_field"], FLOPS_PER_PAIR * pairs_ns + FLOPS_PER_SKEL_PAIR * skel_ns),
        "k_near_sym": (pm["near_pairs"], FLOPS_PER_SYM_PAIR * st["pairs_sym"]
                       + FLOPS_PER_SYM_SKEL_PAIR * st["pairs_sym_skel"]
                       + FLOPS_PER_PAIR * st["pairs_tile"] + FLOPS_PER_SKEL_PAIR * st["pairs_tile_skel"]),
    }


def transfer_figures(st: dict, pm: dict, s_bytes: int, width: int = 1, mfma: bool = False) -> dict:
    """HBM (and, on the matrix cores, MFMA) rate of the upward + downward passes: each
    reads every T once (sum k (n - k) entries) and the vectors of its entries
    (width reals per entry)."""
    t_bytes = st["m_proj_elems"] * s_bytes
    vec_bytes = st["n_entries"] * s_bytes * 4 * width
    ms = pm["upward"] + pm["downward"]
    out = {"bound": "mfma" if mfma else "hbm", "bytes_per_sweep": 2 * (t_bytes + vec_bytes),
           "ms_per_sweep": ms, "achieved_GBs": 2 * (t_bytes + vec_bytes) / (ms * 1e-3) / 1e9,
           "peak_GBs": PEAK_HBM_GBS}
    out["hbm_frac"] = out["achieved_GBs"] / PEAK_HBM_GBS
    if mfma:
        flops = 2 * 2 * st["m_proj_elems"] * width
        out["flops_per_sweep"] = flops
        out["achieved_TFLOPs"] = flops / (ms * 1e-3) / 1e12
        out["peak_TFLOPs"] = PEAK_MFMA_F32_TFLOPS
        out["mfma_frac"] = out["achieved_TFLOPs"] / PEAK_MFMA_F32_TFLOPS
    return out


def mfma_near_figures(st: dict, pm: dict, nrhs: int) -> dict:
    """Matrix-core rate of the many-RHS near field: 2 flops per (pair evaluation, column)."""
    ms = pm["near_field"]
    flops = 2 * st["pairs_near"] * nrhs
    out = {"bound": "mfma", "ms_per_sweep": ms, "mfma_flops_per_sweep": flops,
           "achieved_TFLOPs": flops / (ms * 1e-3) / 1e12, "peak_TFLOPs": PEAK_MFMA_F32_TFLOPS}
    out["frac"] = out["achieved_TFLOPs"] / PEAK_MFMA_F32_TFLOPS
    return out


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
    """The oracle's float64 apply (O2) of the same skeleton operators on the host
    cores, on a bounded sample: the translations of a random sample of target
    boxes (sized so one sampled apply takes about a tenth of the budget) with the
    upward and downward passes in full; one warm-up run, then the median of
    three, scaled to the whole workload by the pair counts.  The oracle samples
    the forward apply only (its adjoint visits the same pairs), so a step
    (forward + adjoint) is taken as twice the forward."""
    import oracle

    n = P["points"].shape[0]
    cores = oracle.num_threads()
    cnt = pair_counts(P)
    total = cnt.sum()
    rng = np.random.default_rng(77)
    # calibration: the passes alone, then a 2% sample
    mask0 = np.zeros(P["n_boxes"], dtype=np.uint8)
    t0 = time.perf_counter()
    oracle.apply(P, q, box_mask=mask0)
    t_base = time.perf_counter() - t0
    mask = (rng.random(P["n_boxes"]) < 0.02).astype(np.uint8)
    t0 = time.perf_counter()
    oracle.apply(P, q, box_mask=mask)
    t_cal = max(time.perf_counter() - t0 - t_base, 1e-3)
    per_pair = t_cal / max(cnt[mask == 1].sum(), 1.0)
    target = max(budget_s / 10 - t_base, 0.2)
    frac = min(1.0, target / max(per_pair * total, 1e-9))
    mask = (rng.random(P["n_boxes"]) < frac).astype(np.uint8)
    sampled = cnt[mask == 1].sum()
    runs = []
    for rep in range(4):
        t0 = time.perf_counter()
        oracle.apply(P, q, box_mask=mask)
        if rep > 0:
            runs.append(time.perf_counter() - t0)
    t_s = sorted(runs)[1]
    t_fwd = t_base + (t_s - t_base) * total / max(sampled, 1.0)
    return {
        "value": n * nrhs / (2.0 * t_fwd),
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"CPU float64 apply (oracle O2) of the same skeleton operators; translations for "
                   f"{int(mask.sum())} of {P['n_boxes']} target boxes ({100 * sampled / total:.2f}% of "
                   f"{total:.3e} pair evaluations), upward/downward passes in full ({t_base:.2f}s); 1 warm-up "
                   f"then the median of 3 runs ({t_s:.2f}s), scaled by pair counts to a {t_fwd:.1f}s forward "
                   f"apply; forward + adjoint taken as twice that"),
    }


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------
def f32_differences_leg(op, w, x, q_h, v_h, steps, warmup, fused_ms, build_s):
    """skelfmm_apply_fwd_adj on an operator built with f32_differences: step time,
    pair-kernel time, errors against the dense sum, items on the float32 form."""
    import torch

    import oracle
    dev = torch.device("cuda:0")
    op.prepare(1, torch.float32)
    tuned = op.autotune_fwd_adj()
    q = torch.from_numpy(q_h).to(dev, torch.float32)
    v = torch.from_numpy(v_h).to(dev, torch.float32)
    holder = {}

    def step():
        holder["u"], holder["w"] = op.apply_fwd_adj(q, v)

    ms = timed_steps(step, steps, warmup)
    pm = pass_times(op, step, steps)
    tg = w.targets()
    qr = q_h.astype(np.float32).astype(np.float64)
    vr = v_h.astype(np.float32).astype(np.float64)
    e = errors(holder["u"].double().cpu().numpy()[tg], oracle.direct(x, qr, targets=tg))
    ea = errors(holder["w"].double().cpu().numpy()[tg], oracle.direct(x, vr, targets=tg))
    st = op.stats()
    return {"value": w.n / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "ratio_to_headline_fused_ms": ms / fused_ms,
            "autotune": tuned, "near_pairs_ms": pm["near_pairs"], "passes_ms_per_sweep": pm,
            "relerr_vs_direct": e["rel_l2"], "maxrel_vs_direct": e["max_rel"],
            "relerr_adjoint_vs_direct": ea["rel_l2"], "maxrel_adjoint_vs_direct": ea["max_rel"],
            "sym_items": st["n_sym_tasks"], "f32diff_items": st["n_sym_f32diff"],
            "expanded_items": st["n_sym_expanded"], "build_s": build_s}


def many_rhs_same_operator(op, w, x, steps, warmup, f64_rate):
    """64 float32 right-hand sides on the 1M cube's operator (matrix-core near field
    and transfers): forward + adjoint points x RHS/s against the float64 single-RHS
    rate of the same operator, errors against the dense sum on 4 columns at 2,048
    targets."""
    import torch

    import oracle
    nrhs = 64
    dev = torch.device("cuda:0")
    Qh = w.charges(nrhs)
    Vh = w.weights(nrhs)
    Q = torch.from_numpy(Qh).to(dev, torch.float32)
    V = torch.from_numpy(Vh).to(dev, torch.float32)
    op.prepare(nrhs, torch.float32)
    xfer = op.autotune_transfers(nrhs)
    holder = {}

    def step():
        holder["u"] = op.apply(Q)
        holder["w"] = op.apply_adjoint(V)

    ms = timed_steps(step, steps, warmup)
    pm = pass_times(op, step, max(3, steps // 2))
    st = op.stats()
    rate = w.n * nrhs / (ms * 1e-3)
    res = {"value": rate, "unit": "points x RHS/s (fwd+adjoint)", "ms_per_step": ms, "nrhs": nrhs, "dtype": "f32",
           "transfer_shape": xfer, "passes_ms_per_sweep": pm, "f64_single_rhs_points_per_s": f64_rate,
           "ratio_to_f64_single_rhs": rate / f64_rate,
           "roofline": {"transfers": transfer_figures(st, pm, 4, nrhs, mfma=True),
                        "near_field": mfma_near_figures(st, pm, nrhs)}}
    tg = w.targets()
    cols = [0, 21, 42, 63]
    U = holder["u"].double().cpu().numpy()
    W = holder["w"].double().cpu().numpy()
    Qr = Qh.astype(np.float32).astype(np.float64)
    Vr = Vh.astype(np.float32).astype(np.float64)
    ref_u = np.stack([oracle.direct(x, np.ascontiguousarray(Qr[:, c]), targets=tg) for c in cols], axis=1)
    ref_w = np.stack([oracle.direct(x, np.ascontiguousarray(Vr[:, c]), targets=tg) for c in cols], axis=1)
    res["error_vs_direct"] = errors(U[np.ix_(tg, cols)], ref_u)
    res["adjoint_error_vs_direct"] = errors(W[np.ix_(tg, cols)], ref_w)
    return res


def single_leg(name, op, q_h, v_h, x, kind, kappa, tdt, targets, steps, warmup, helm=False):
    """One operator, one RHS: forward + adjoint timed, per-pass figures, errors vs O1."""
    import torch

    import oracle
    dev = torch.device("cuda:0")
    op.prepare(1, tdt)
    tuned = op.autotune(tdt)
    q = torch.from_numpy(q_h).to(dev, tdt)
    v = torch.from_numpy(v_h).to(dev, tdt)
    holder = {}

    def step():
        holder["u"] = op.apply(q)
        holder["w"] = op.apply_adjoint(v)

    ms = timed_steps(step, steps, warmup)
    pm = pass_times(op, step, max(3, steps // 2))
    st = op.stats()
    ker = near_kernels(st, pm, helm)
    dom = max(ker, key=lambda k: ker[k][0])
    f64_eval = tdt in (torch.float64, torch.complex128) or helm
    peak = PEAK_TFLOPS["f64" if f64_eval else "f32"]
    n = x.shape[0]
    s_bytes = 8 if tdt in (torch.float64, torch.complex128) else 4
    res = {"value": n / (ms * 1e-3), "unit": "points/s (fwd+adjoint)", "ms_per_step": ms, "autotune": tuned,
           "passes_ms_per_sweep": pm,
           "roofline": {"bound": "alu", "kernel": dom, "ms_per_launch": ker[dom][0],
                        "achieved": ker[dom][1] / (ker[dom][0] * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                        "pair_evaluations_per_launch": st["pairs_near"] - st["pairs_sym"]},
           "transfers": transfer_figures(st, pm, s_bytes, 2 if helm else 1)}
    res["roofline"]["frac"] = res["roofline"]["achieved"] / peak
    up = np.complex128 if helm else np.float64
    u = holder["u"].cpu().numpy().astype(up)
    wv = holder["w"].cpu().numpy().astype(up)
    cast = {torch.float32: np.float32, torch.complex64: np.complex64}.get(tdt)
    qr = q_h.astype(cast).astype(q_h.dtype) if cast else q_h
    vr = v_h.astype(cast).astype(v_h.dtype) if cast else v_h
    res["error_vs_direct"] = errors(u[targets], oracle.direct(x, qr, kind, kappa, targets=targets))
    # A^H v = conj(A conj v) for the complex-symmetric kernel (A for Laplace)
    ref_w = (np.conj(oracle.direct(x, np.conj(vr), kind, kappa, targets=targets)) if helm
             else oracle.direct(x, vr, kind, kappa, targets=targets))
    res["adjoint_error_vs_direct"] = errors(wv[targets], ref_w)
    log(f"[bench] {name}: {ms:.3f} ms/step err {res['error_vs_direct']} adj {res['adjoint_error_vs_direct']}")
    return res


def batched_run(steps: int, warmup: int, check: bool = True):
    """Eight 3D Laplace geometries (65,536 .. 2,097,152 points, cube / ellipsoid,
    tol 1e-6, leaf 128), 64 float32 right-hand sides each: one captured hipGraph
    holds a batched forward sweep and a batched adjoint sweep; value = total
    points x RHS per second of that step.  Per-pass figures come from separate
    eager batched sweeps with the library's events; the adjoint sweep's output
    (the gradient A^T w of L = sum(w u)) and the forward are checked against the
    dense sum on 4 columns at 256 targets per geometry."""
    import torch

    import oracle
    import workloads
    import paper_2310_16668_amd as sk

    wls = workloads.batch_workloads()
    t0 = time.perf_counter()
    xs = [w.points() for w in wls]
    ops = [sk.build(x, "laplace", tol=w.tol, leaf_size=w.leaf_size) for x, w in zip(xs, wls)]
    t_build = time.perf_counter() - t0
    batch = sk.Batch(ops)
    dev = torch.device("cuda:0")
    q_h = [w.charges() for w in wls]
    v_h = [w.weights() for w in wls]
    q = [torch.from_numpy(a).to(dev, torch.float32) for a in q_h]
    v = [torch.from_numpy(a).to(dev, torch.float32) for a in v_h]
    xfer = batch.autotune_transfers(64)
    log(f"[bench] batched transfer shapes (ms per up + down pass pair): {xfer}")
    outs = {}

    def eager():
        outs["u"] = batch.apply(q)
        outs["w"] = batch.apply(v, adjoint=True)

    eager()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gu = batch.apply(q)
        gw = batch.apply(v, adjoint=True)
    ms = timed_steps(graph.replay, steps, warmup)
    pm = pass_times(batch, eager, max(3, steps // 2))
    n_total = sum(w.n for w in wls)
    sts = [o.stats() for o in ops]
    st = {k: sum(s[k] for s in sts) for k in ("m_proj_elems", "n_entries", "pairs_near", "pairs_skel")}
    res = {"value": n_total * 64 / (ms * 1e-3), "unit": "points x RHS/s (fwd+adjoint)", "ms_per_step": ms,
           "n_total": n_total, "sizes": [w.n for w in wls], "nrhs": 64, "dtype": "f32", "graph": True,
           "build_s": t_build, "transfer_shape": xfer, "passes_ms_per_sweep": pm,
           "roofline": {"transfers": transfer_figures(st, pm, 4, 64, mfma=True),
                        "near_field": mfma_near_figures(st, pm, 64)}}
    if check:
        graph.replay()
        torch.cuda.synchronize()
        e_u, e_w = [], []
        cols = [0, 21, 42, 63]
        for g, w in enumerate(wls):
            tg = w.targets(256)
            qr = q_h[g].astype(np.float32).astype(np.float64)
            vr = v_h[g].astype(np.float32).astype(np.float64)
            U = gu[g].double().cpu().numpy()[np.ix_(tg, cols)]
            W = gw[g].double().cpu().numpy()[np.ix_(tg, cols)]
            ru = np.stack([oracle.direct(xs[g], np.ascontiguousarray(qr[:, c]), targets=tg) for c in cols], axis=1)
            rw = np.stack([oracle.direct(xs[g], np.ascontiguousarray(vr[:, c]), targets=tg) for c in cols], axis=1)
            e_u.append(errors(U, ru))
            e_w.append(errors(W, rw))
        res["error_vs_direct"] = {"rel_l2_max_over_geometries": max(e["rel_l2"] for e in e_u),
                                  "max_rel_max_over_geometries": max(e["max_rel"] for e in e_u)}
        res["gradient_error_vs_dense_ATw"] = {"rel_l2_max_over_geometries": max(e["rel_l2"] for e in e_w),
                                              "max_rel_max_over_geometries": max(e["max_rel"] for e in e_w)}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: --gpus must be 1 (the apply does not shard across GPUs)"}))
        return 2
    if args.batched_only:
        print(json.dumps({"batched": batched_run(args.steps, args.warmup, check=False)}))
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
    # f64 / f32: skelfmm_apply then skelfmm_apply_adjoint, two sweeps per step;
    # f32_fused: skelfmm_apply_fwd_adj, both in one sweep of two columns
    paths = [("f64", torch.float64), ("f32", torch.float32), ("f32_fused", torch.float32)]
    if args.only:
        paths = [p for p in paths if p[0] == args.only]
    tuned = {}
    # rocm-smi is a separate program: not started under a profiler (--profile-only)
    clk = {"before": clocks()} if not args.profile_only else {}
    for dt_name, tdt in paths:
        fused = dt_name == "f32_fused"
        op.prepare(1, tdt)
        if not args.no_autotune:
            tuned[dt_name] = op.autotune_fwd_adj() if fused else op.autotune(tdt)
            log(f"[bench] {dt_name} autotune {tuned[dt_name]}")
        q = torch.from_numpy(q_h).to(dev, tdt)
        v = torch.from_numpy(v_h).to(dev, tdt)
        holder = {}

        def step():
            if fused:
                holder["u"], holder["w"] = op.apply_fwd_adj(q, v)
            else:
                holder["u"] = op.apply(q)
                holder["w"] = op.apply_adjoint(v)

        # the timed region: K steps and nothing else
        ms_step = timed_steps(step, args.steps, args.warmup)
        if not args.profile_only:
            clk["after_" + dt_name] = clocks()
        # per-pass durations: a separate run of the same steps with HIP events
        pm = pass_times(op, step, args.steps)
        res = {"ms_per_step": ms_step, "passes_ms_per_sweep": pm}
        if not args.profile_only:
            import oracle
            tg = w.targets()
            cast = np.float32 if tdt == torch.float32 else np.float64
            qr = q_h.astype(cast).astype(np.float64)
            vr = v_h.astype(cast).astype(np.float64)
            e = errors(holder["u"].double().cpu().numpy()[tg], oracle.direct(x, qr, targets=tg))
            ea = errors(holder["w"].double().cpu().numpy()[tg], oracle.direct(x, vr, targets=tg))  # A^H = A
            res["relerr_vs_direct"], res["maxrel_vs_direct"] = e["rel_l2"], e["max_rel"]
            res["relerr_adjoint_vs_direct"], res["maxrel_adjoint_vs_direct"] = ea["rel_l2"], ea["max_rel"]
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
    fused = chosen == "f32_fused"
    base = chosen.split("_")[0]   # the arithmetic type
    # pair counts at the headline path's targets per lane (the diagonal tiles depend on it)
    if chosen in tuned:
        op.set_targets_per_lane(tuned[chosen]["targets_per_lane"])
    st = op.stats()
    kernels = near_kernels(st, pm, columns=2 if fused else 1)
    dom = max(kernels, key=lambda k: kernels[k][0])
    near_ms, flops = kernels[dom]
    achieved = flops / (near_ms * 1e-3) / 1e12
    tpl = tuned.get(chosen, {}).get("targets_per_lane")
    traffic = near_traffic(chosen, dom, tpl)
    # the same launch against its instruction mix: every evaluation (a symmetric pair,
    # or a one-direction tile pair) priced at the cheapest symmetric-pair cost
    issue_bound = None
    if dom == "k_near_sym" and chosen in MIX_CYCLES_PER_64_SYM_PAIRS:
        evals = st["pairs_sym"] + st["pairs_tile"]
        ideal_ms = evals / 64 * MIX_CYCLES_PER_64_SYM_PAIRS[chosen] / SIMDS / (CLOCK_GHZ * 1e9) * 1e3
        issue_bound = {"cycles_per_64_pairs_ideal": MIX_CYCLES_PER_64_SYM_PAIRS[chosen],
                       "cycles_per_64_pairs_achieved": near_ms * 1e-3 * CLOCK_GHZ * 1e9 * SIMDS / (evals / 64),
                       "ideal_ms": ideal_ms, "frac": ideal_ms / near_ms}
    pairs_ns = st["pairs_near"] - 2 * st["pairs_sym"] - st["pairs_tile"]
    skel_ns = st["pairs_skel"] - 2 * st["pairs_sym_skel"] - st["pairs_tile_skel"]
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
        "dtype": base,
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": 3, "kernel": "laplace", "leaf_size": w.leaf_size,
                   "tol": w.tol, "nrhs": 1,
                   "step": ("forward apply of q + adjoint apply of v in one two-column sweep (skelfmm_apply_fwd_adj)"
                            if fused else "forward apply + adjoint apply")},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[base], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[base], "traffic": traffic,
                     "issue_bound": issue_bound,
                     "kernel": dom, "ms_per_launch": near_ms,
                     "sym_pairs_per_launch": st["pairs_sym"], "sym_skel_pairs_per_launch": st["pairs_sym_skel"],
                     "tile_pairs_per_launch": st["pairs_tile"], "tile_skel_pairs_per_launch": st["pairs_tile_skel"],
                     "segment_pairs_per_launch": pairs_ns, "segment_skel_pairs_per_launch": skel_ns,
                     "near_kernels": {k: {"ms": v[0], "tflops": v[1] / (v[0] * 1e-3) / 1e12 if v[0] > 0 else None}
                                      for k, v in kernels.items()},
                     "near_reduce_ms": pm["near_reduce"]},
        "transfer_passes": transfer_figures(st, pm, 8 if chosen == "f64" else 4, width=2 if fused else 1),
        "paths": results,
        "autotune": tuned,
        "clocks": clk,
        "build_s": t_build,
    }
    f64_rate = w.n / (results["f64"]["ms_per_step"] * 1e-3) if "f64" in results else None
    if f64_rate:
        # the float32 step against the plain float64 forward + adjoint applies on this GPU
        out["ratio_to_f64_fwd_adj"] = out["value"] / f64_rate
    legs = not (args.headline_only or args.profile_only)
    if legs and f64_rate:
        log("[bench] 64 float32 RHS on the same operator")
        out["many_rhs_same_operator"] = many_rhs_same_operator(op, w, x, args.steps, args.warmup, f64_rate)
        log(f"[bench] many RHS: {out['many_rhs_same_operator']}")
    if legs and "f32_fused" in results:
        # the same cube built with f32_differences: the pair items whose reach is at
        # most 1024 x their smallest spacing form |d|^2 from float32 differences (an
        # option with a looser bound per kernel value, so not a headline candidate)
        log("[bench] fused float32 step with f32_differences")
        t0 = time.perf_counter()
        opf = sk.build(x, "laplace", tol=w.tol, leaf_size=w.leaf_size, f32_differences=True)
        tb = time.perf_counter() - t0
        out["f32_differences_fused"] = f32_differences_leg(opf, w, x, q_h, v_h, args.steps, args.warmup,
                                                           results["f32_fused"]["ms_per_step"], tb)
        log(f"[bench] f32 differences: {out['f32_differences_fused']}")
        del opf
    if legs:
        we = workloads.LAPLACE3D_ELLIPSOID_4M
        log(f"[bench] building {we.name}")
        xe = we.points()
        t0 = time.perf_counter()
        ope = sk.build(xe, "laplace", tol=we.tol, leaf_size=we.leaf_size, compensated_leaf=True)
        tb = time.perf_counter() - t0
        leg = single_leg(we.name, ope, we.charges(), we.weights(), xe, "laplace", 0.0, torch.float32,
                         we.targets(), args.steps, args.warmup)
        leg.update({"config": {"workload": we.name, "n": we.n, "tol": we.tol, "leaf_size": we.leaf_size,
                               "dtype": "f32", "compensated_leaf": True}, "build_s": tb})
        out["ellipsoid_4m"] = leg
        del ope
        wh = workloads.HELMHOLTZ3D_1M
        log(f"[bench] building {wh.name}")
        xh = wh.points()
        t0 = time.perf_counter()
        oph = sk.build(xh, "helmholtz", tol=wh.tol, leaf_size=wh.leaf_size, kappa=wh.kappa, f64_leaf=True)
        tb = time.perf_counter() - t0
        vh = workloads.charges(wh.n, 1, 1300 + wh.number, complex_=True)
        leg = single_leg(wh.name, oph, wh.charges(), vh, xh, "helmholtz", wh.kappa, torch.complex64, wh.targets(),
                         args.steps, args.warmup, helm=True)
        leg.update({"config": {"workload": wh.name, "n": wh.n, "tol": wh.tol, "leaf_size": wh.leaf_size,
                               "kappa": wh.kappa, "dtype": "c64", "f64_leaf": True}, "build_s": tb})
        out["helmholtz_1m"] = leg
        del oph
    if legs and not args.no_batched:
        log("[bench] eight-geometry batched run")
        bt = batched_run(args.steps, args.warmup)
        if f64_rate:
            bt["f64_single_rhs_points_per_s_1m_cube"] = f64_rate
        out["batched"] = bt
        log(f"[bench] batched: {bt}")
    if not args.no_cpu_baseline and not args.profile_only:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(op.export(), q_h, v_h, args.cpu_budget)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
