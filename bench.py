"""Benchmark of the short-range particle-particle force on one MI355X.

One step is one stream-kick-stream subcycle of the differentiable rollout on
the 256^3 NFW-clustered workload, forward and reverse: stream, checkpoint,
force (binning, work list, pair kernel), kick, stream; then the reverse
pass at the checkpoint: adjoint stream, kick adjoint, VJP (re-binning, work
list, VJP pair kernel), adjoint streams.  Every pair inside r_cut is thus
evaluated twice per step, once by each pair kernel.

Prints one JSON line: value = pair interactions per second (forward +
adjoint, in-cut-off pairs) for the whole step, with the roofline of the
dominant pair kernel against the FP32 vector peak and the float64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "short-range pair interactions/s (fwd & adjoint) + % FP32 VALU peak, 1 GPU"
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector, 256 CU x 2.4 GHz x 256 FLOP/clk
FLOP_FWD = 30                     # counted FLOP per evaluated forward pair
FLOP_VJP = 61                     # counted FLOP per evaluated adjoint pair
WORKLOADS = {
    "cfg1": "32^3 = 32768 particles, uniform + Gaussian displacements (0.3 cell), "
            "periodic unit box, r_cut = 3/128, eps = 1e-5, 42^3 chaining cells, seed 1",
    "cfg4": "cfg2 positions (128^3 = 2.1M, Plummer-clustered) with cotangents "
            "g ~ N(0, 1) float32 for the VJP, seed 4",
    "cfg3": "256^3 = 16.8M particles, 20000 NFW halos (70%, masses log-uniform over "
            "4 decades, c 4-15) + uniform background, periodic unit box, "
            "r_cut = 3/256, eps = 2.5e-6, 85^3 chaining cells, seed 3",
    "cfg3s": "cfg3 with its ten most massive halos moved into one 2x2x2-cell block "
             "(load-balance stress: one chaining cell holds ~26000 particles), seed 3",
    "cfg2": "128^3 = 2.1M particles, 2000 Plummer halos (60%) + uniform, periodic, "
            "r_cut = 3/128, eps = 1e-5, 42^3 chaining cells, seed 2",
    "cfg5": "one GPU's share of a 512^3 periodic parent: 134.2M particles in 160000 "
            "NFW halos (70%) + uniform, plus the periodic images within 3 cells of "
            "each face (particle overloading), open box of side 1 + 6/512, "
            "r_cut = 3/512, eps = 6.25e-7, seed 5",
}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pair_kernels_cfg3_counters.md")
KERNEL_SOURCES = ("pair.hip", "common.h", "worklist.hip")


def kernel_source_hash() -> str:
    """sha256 over the code of the pair kernels, of the work list that orders
    their items and of the shared definitions they use (common.h up to its
    launch-wrapper declarations); line comments and blank lines removed.  It
    ties counter readings to the code they were taken on."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1211_4864_amd", "csrc", name)) as f:
            text = f.read()
        if name == "common.h":
            text = text.split("// ---- launch wrappers", 1)[0]
        lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.split("\n"))
        h.update("\n".join(line for line in lines if line.strip()).encode())
    return h.hexdigest()


def _counter_block():
    """The JSON block of the committed rocprofv3 counter summary, or None when
    the summary is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            text = f.read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if data.get("source_sha256") != kernel_source_hash():
        return None
    return data


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by what the same counters read
    for a device copy of known size), or None when the summary is missing or
    was taken on other kernel sources."""
    data = _counter_block()
    k = None if data is None else data.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def measured_counters(kernel: str, launch_ms: float):
    """VALU busy, VALU lane utilisation, LDS bank-conflict share, resident
    waves per SIMD and HBM rate of `kernel` from the committed counter summary
    (the HBM rate divides its bytes per launch by this run's launch time), or
    None under the same conditions as `measured_traffic`."""
    data = _counter_block()
    k = None if data is None else data.get("kernels", {}).get(kernel)
    if k is None:
        return None
    out = {key: k.get(key) for key in ("valu_busy", "valu_lane_utilisation",
                                       "lds_bank_conflict_frac", "waves_per_simd")}
    b = k.get("hbm_bytes_per_launch")
    out["hbm_tb_per_s"] = None if b is None else round(b / (launch_ms * 1e-3) / 1e12, 3)
    return out


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline_full(w, g, repeats=3):
    """The float64 oracle over every target: forward and VJP each timed
    `repeats` times (median).  Pair interactions per second over the two
    passes (in-cut-off pairs, fwd + adjoint), and each pass on its own."""
    import oracle
    tf, tv = [], []
    pairs = 0
    for r in range(repeats):
        t0 = time.perf_counter()
        _, _, cnt = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
        tf.append(time.perf_counter() - t0)
        log(f"[bench] cpu oracle forward {r + 1}/{repeats}: {tf[-1]:.2f} s")
        t0 = time.perf_counter()
        oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, g)
        tv.append(time.perf_counter() - t0)
        log(f"[bench] cpu oracle VJP {r + 1}/{repeats}: {tv[-1]:.2f} s")
        pairs = int(cnt.sum())
    mf, mv = float(np.median(tf)), float(np.median(tv))
    return {"value": 2.0 * pairs / (mf + mv), "unit": "pair interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "fwd_interactions_per_s": pairs / mf, "adj_interactions_per_s": pairs / mv,
            "sample": f"all {w.n} targets, float64 forward ({mf:.2f} s) and VJP "
                      f"({mv:.2f} s), median of {repeats} runs each, {pairs} in-cut-off "
                      f"pairs"}


def cpu_baseline(w, sample_seconds: float, g):
    """The float64 oracle on a random sample of targets: forward and VJP.
    Returns pair interactions per second (in-cut-off pairs, fwd + adjoint),
    the rate the whole workload would run at (extrapolated from the
    sample)."""
    import oracle
    rng = np.random.default_rng(11)
    k = 500
    t_used = 0.0
    pairs = 0
    elapsed = 0.0
    while True:
        idx = np.sort(rng.choice(w.n, k, replace=False))
        t0 = time.perf_counter()
        _, _, cnt = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, targets=idx)
        oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, g, targets=idx)
        dt = time.perf_counter() - t0
        t_used += dt
        if dt > 0.25 * sample_seconds or t_used > sample_seconds or k >= w.n:
            pairs = int(cnt.sum())
            elapsed = dt
            break
        k = min(w.n, int(k * max(2.0, 0.3 * sample_seconds / max(dt, 1e-3))))
    return {"value": 2.0 * pairs / elapsed, "unit": "pair interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{k} random targets of the same workload (all their sources), "
                      f"float64 forward + VJP, {pairs} in-cut-off pairs each, "
                      f"{elapsed:.2f} s; the rate is extrapolated to the whole "
                      f"workload"}


def accuracy(w, acc, gradp, g):
    """Per-particle floored relative error against the float64 oracle on a
    random sample of 2000 targets."""
    import oracle
    idx = np.sort(np.random.default_rng(12).choice(w.n, min(2000, w.n), replace=False))
    ref, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, targets=idx)
    e = oracle.rel_err_floored(acc[idx], ref, an)
    raw = np.linalg.norm(acc[idx] - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    gref, bn, amb, pm = oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, g,
                                         targets=idx, cut_band=1e-6, pair_floor=True)
    clean = amb == 0.0     # f' jumps at r_cut: pairs on the cut are excluded
    ge = oracle.rel_err_floored(gradp[idx][clean], gref[clean], bn[clean])
    gp = oracle.rel_err_floored(gradp[idx][clean], gref[clean], pm[clean])
    return {"sample": int(idx.size), "force_max_err": float(e.max()),
            "force_raw_rel_median": float(np.median(raw)),
            "force_raw_rel_p99": float(np.quantile(raw, 0.99)),
            "force_count_above_1e-5": int((e > 1e-5).sum()),
            "vjp_max_err": float(ge.max()),
            "vjp_max_err_pair_floor": float(gp.max()),
            "vjp_count_above_1e-4_pair_floor": int((gp > 1e-4).sum()),
            "vjp_particles_with_pairs_on_cut": int((~clean).sum()),
            "metric": "|x - x*| / max(|x*|, 0.1 F): F = summed Newtonian pair "
                      "magnitude (forces); for the VJP, F = summed magnitude of the "
                      "Newtonian and polynomial parts of the pair terms (vjp_max_err) "
                      "or of the pair terms themselves, sum (|f| + 2|f'| s)|w| "
                      "(vjp_max_err_pair_floor)"}


def measured_peak(hsr):
    """Float32 VALU peak measured on this GPU at the clock it sustains under
    a VALU load: the best FMA probe rate over 1, 2, 4 and 8 waves per SIMD
    (2 FLOP per lane operation), with the shader clock and the shader cycles
    between two instructions of one wave, for an FMA, a reciprocal square
    root and the forward pair term's mix (1 rsq per 18 FMA)."""
    sweep = {w: hsr.valu_probe(hsr.PROBE_FMA, w) for w in (1, 2, 4, 8)}
    fmac = hsr.valu_probe(hsr.PROBE_FMAC, 8)
    best = max(sweep, key=lambda w: sweep[w]["lane_ops_per_s"])
    top = max(sweep[best]["lane_ops_per_s"], fmac["lane_ops_per_s"])
    rsq = hsr.valu_probe(hsr.PROBE_RSQ, 8)
    mix = hsr.valu_probe(hsr.PROBE_PAIR_MIX, 8)
    fma8 = sweep[8]
    simds = 1024.0
    clk = fma8["clock_ghz"] * 1e9
    return {"fma_tflops": round(2.0 * top / 1e12, 3),
            "best_waves_per_simd": best,
            "fma_tflops_by_waves": {w: round(2.0 * r["lane_ops_per_s"] / 1e12, 3)
                                    for w, r in sweep.items()},
            "fmac_tflops_8_waves": round(2.0 * fmac["lane_ops_per_s"] / 1e12, 3),
            "clock_ghz": round(fma8["clock_ghz"], 4),
            # SIMD cycles per wave64 instruction, from the aggregate rates
            "simd_cycles_per_fma": round(simds * 64 * clk / top, 3),
            "simd_cycles_per_rsq": round(simds * 64 * clk / rsq["lane_ops_per_s"], 3),
            "simd_cycles_per_mix_instr": round(simds * 64 * clk / mix["lane_ops_per_s"], 3),
            "probe": "16 independent float32 chains per lane, one-wave workgroups, "
                     "5 launches; packed float32 disabled"}


def unequal_mass_leg(hsr, torch, w, pos, g_np, inside, launches=2):
    """Both pair kernels on the same positions with masses spread over a
    decade (m_i = 10^U(-0.5, 0.5) / N): the general path, which multiplies
    every pair term by its mass and forms w = m_k g_j - m_j g_k from two
    products, as the counted 30 / 61 FLOP per pair assume."""
    dev = pos.device
    rng = np.random.default_rng(77)
    m = (10.0 ** rng.uniform(-0.5, 0.5, w.n) / w.n).astype(np.float32)
    mass = torch.from_numpy(m).to(dev)
    ga = torch.from_numpy(g_np).to(dev)
    box, rc, eps, poly = w.box, w.r_cut, w.eps, w.poly
    acc = hsr.force(pos, mass, box, rc, eps, poly)
    gp = hsr.force_vjp(pos, mass, box, rc, eps, poly, ga)
    torch.cuda.synchronize()
    hsr.timing_enable(True)
    for _ in range(launches):
        hsr.force(pos, mass, box, rc, eps, poly, out=acc)
        hsr.force_vjp(pos, mass, box, rc, eps, poly, ga, out=gp)
    torch.cuda.synchronize()
    n_f, ms_f = hsr.timing_read(hsr.TIMER_FORCE)
    n_v, ms_v = hsr.timing_read(hsr.TIMER_VJP)
    hsr.timing_enable(False)
    f_ms, v_ms = ms_f / max(n_f, 1), ms_v / max(n_v, 1)
    fwd = FLOP_FWD * inside / (f_ms * 1e-3) / 1e12
    vjp = FLOP_VJP * inside / (v_ms * 1e-3) / 1e12
    return {"force_pair_ms": round(f_ms, 4), "vjp_pair_ms": round(v_ms, 4),
            "fwd_tflops": round(fwd, 3), "vjp_tflops": round(vjp, 3),
            "fwd_pct_fp32_peak": round(100 * fwd / FP32_PEAK_TFLOPS, 2),
            "vjp_pct_fp32_peak": round(100 * vjp / FP32_PEAK_TFLOPS, 2),
            "masses": "10^U(-0.5, 0.5) / N, seed 77"}


def rcb_leg(hsr, torch, w, pos, mass, g_np, inside, leaf_max, launches=2):
    """The same forward and VJP with the RCB fat leaves (centre-of-mass
    bisection inside the chaining cells) as the work items: pair-kernel
    times, the tree build, and their roofline beside the chaining mesh's."""
    dev = pos.device
    ga = torch.from_numpy(g_np).to(dev)
    box, rc, eps, poly = w.box, w.r_cut, w.eps, w.poly
    acc = hsr.force_rcb(pos, mass, box, rc, eps, poly, leaf_max)
    gp = hsr.force_vjp_rcb(pos, mass, box, rc, eps, poly, ga, leaf_max)
    torch.cuda.synchronize()
    hsr.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(launches):
        hsr.force_rcb(pos, mass, box, rc, eps, poly, leaf_max, out=acc)
        hsr.force_vjp_rcb(pos, mass, box, rc, eps, poly, ga, leaf_max, out=gp)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / launches
    n_f, ms_f = hsr.timing_read(hsr.TIMER_FORCE)
    n_v, ms_v = hsr.timing_read(hsr.TIMER_VJP)
    n_r, ms_r = hsr.timing_read(hsr.TIMER_RCB)
    n_b, ms_b = hsr.timing_read(hsr.TIMER_BIN)
    n_w, ms_w = hsr.timing_read(hsr.TIMER_WORKLIST)
    hsr.timing_enable(False)
    f_ms, v_ms = ms_f / max(n_f, 1), ms_v / max(n_v, 1)
    fwd = FLOP_FWD * inside / (f_ms * 1e-3) / 1e12
    vjp = FLOP_VJP * inside / (v_ms * 1e-3) / 1e12
    _, _, _, ls = hsr.rcb_bin(pos, mass, box, rc, leaf_max)
    return {"leaf_max": leaf_max, "leaves": int(ls.numel() - 1),
            "force_pair_ms": round(f_ms, 4), "vjp_pair_ms": round(v_ms, 4),
            "rcb_tree_ms": round(ms_r / max(n_r, 1), 4),
            "bin_ms": round(ms_b / max(n_b, 1), 4),
            "worklist_ms": round(ms_w / max(n_w, 1), 4),
            "force_plus_vjp_wall_ms": round(1e3 * wall, 3),
            "fwd_tflops": round(fwd, 3), "vjp_tflops": round(vjp, 3),
            "fwd_pct_fp32_peak": round(100 * fwd / FP32_PEAK_TFLOPS, 2),
            "vjp_pct_fp32_peak": round(100 * vjp / FP32_PEAK_TFLOPS, 2)}


PM_GRID = {"cfg1": 128, "cfg2": 128, "cfg4": 128, "cfg3": 256, "cfg3s": 256, "cfg5": 512}


def pm_leg(hsr, torch, w, pos, mass, ng, launches=3):
    """The long-range PM solve (Sec. II) on the workload's own PM grid (the
    grid whose 3 cells are r_cut): time per solve and its HBM rate against
    the algorithmic bytes of its passes: per grid cell 144 B (clearing the
    fixed-point grid 8; forward z pass 16, y pass 16; the fused x pass reads
    8 and writes two grids 16; inverse y and z passes over two grids 32
    each; interpolation reads two grids 16), per particle 172 B (mass
    maximum 4; cell keys 32; three radix passes 60; deposit 36;
    interpolation 40).  Atomic traffic is not counted."""
    if w.box <= 0:
        return None
    acc = hsr.pm_accel(pos, mass, w.box, ng)
    torch.cuda.synchronize()
    hsr.timing_enable(True)
    for _ in range(launches):
        hsr.pm_accel(pos, mass, w.box, ng, out=acc)
    torch.cuda.synchronize()
    n_p, ms_p = hsr.timing_read(hsr.TIMER_PM)
    hsr.timing_enable(False)
    ms = ms_p / max(n_p, 1)
    algo = 144.0 * ng ** 3 + 172.0 * w.n
    return {"ng": ng, "ms_per_solve": round(ms, 4),
            "algorithmic_bytes": algo,
            "roofline": {"bound": "hbm", "achieved": round(algo / (ms * 1e-3) / 1e9, 1),
                         "peak": 8000.0, "unit": "GB/s",
                         "frac": round(algo / (ms * 1e-3) / 8e12, 4)}}


def full_step_leg(hsr, torch, w, pos, mass, ng, n_c=5, steps=2):
    """One full split-operator step (Eq. 6: PM half kick, n_c short-range
    subcycles, PM half kick) on the workload, with the grid-force polynomial
    of the workload."""
    if w.box <= 0:
        return None
    x = pos.clone()
    v = torch.zeros_like(x)
    acc = torch.empty((w.n, 3), dtype=torch.float32, device=pos.device)
    dt = 1e-4
    hsr.full_step(x, v, mass, w.box, ng, w.r_cut, w.eps, w.poly, dt, n_c, scratch=acc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.copy_(pos)
        v.zero_()
        hsr.full_step(x, v, mass, w.box, ng, w.r_cut, w.eps, w.poly, dt, n_c, scratch=acc)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return {"n_c": n_c, "ng": ng, "ms_per_step": round(ms, 3)}


def plain_comparison(hsr, torch, w, pos, mass, g_np, inside, f_ms, v_ms,
                     with_accuracy, launches=2):
    """The plain float32 kernels (one thread per target, sources read from
    global memory, no LDS staging, no culling; the same float32 pair formula
    with the polynomial in the t basis; per-target sums in float64) on the
    same input: time per launch, interactions/s and accuracy on the same
    sample."""
    dev = pos.device
    box, rc, eps, poly = w.box, w.r_cut, w.eps, w.poly
    ga = torch.from_numpy(g_np).to(dev)
    acc = hsr.force_plain(pos, mass, box, rc, eps, poly)
    gp = hsr.force_vjp_plain(pos, mass, box, rc, eps, poly, ga)
    torch.cuda.synchronize()
    hsr.timing_enable(True)
    for _ in range(launches):
        hsr.force_plain(pos, mass, box, rc, eps, poly, out=acc)
        hsr.force_vjp_plain(pos, mass, box, rc, eps, poly, ga, out=gp)
    torch.cuda.synchronize()
    n_f, ms_f = hsr.timing_read(hsr.TIMER_FORCE_PLAIN)
    n_v, ms_v = hsr.timing_read(hsr.TIMER_VJP_PLAIN)
    hsr.timing_enable(False)
    pf, pv = ms_f / max(n_f, 1), ms_v / max(n_v, 1)
    out = {"force_ms": round(pf, 4), "vjp_ms": round(pv, 4),
           "fwd_interactions_per_s": inside / (pf * 1e-3),
           "adj_interactions_per_s": inside / (pv * 1e-3),
           "speedup_fwd": round(pf / f_ms, 3), "speedup_adj": round(pv / v_ms, 3)}
    if with_accuracy:
        a = accuracy(w, acc.cpu().numpy().astype(np.float64), gp.cpu().numpy(),
                     g_np.astype(np.float64))
        out["force_max_err"] = a["force_max_err"]
        out["vjp_max_err"] = a["vjp_max_err"]
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle over every target (median of 3) instead "
                         "of a sample; for the small workloads cfg1, cfg2, cfg4")
    ap.add_argument("--no-unequal", action="store_true",
                    help="skip the unequal-mass leg")
    ap.add_argument("--no-pm", action="store_true",
                    help="skip the long-range PM and full-step legs")
    ap.add_argument("--rcb", type=int, nargs="*", default=[64],
                    help="leaf sizes of the RCB fat-leaf legs (none: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain float32 comparison kernels")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the float32 VALU rate probes (measured peak)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--rollout", type=int, default=1,
                    help="SKS subcycles per step; above 1 the step is the "
                         "differentiable rollout (autograd, checkpointed) forward "
                         "and backward")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the short-range force is rank-local; see the sharding notes)",
              file=sys.stderr)
        return 2

    import torch
    import paper_1211_4864_amd as hsr
    from workloads import make_config, cotangent

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = make_config(args.workload)
    g_np = cotangent(w.n, 4)
    log(f"[bench] generated {args.workload} n={w.n} in {time.perf_counter() - t0:.1f}s")

    pos = torch.from_numpy(w.pos).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    gx = torch.from_numpy(g_np.astype(np.float64)).to(dev)
    n = w.n
    box, rc, eps, poly = w.box, w.r_cut, w.eps, w.poly

    cand, inside = hsr.count_pairs(pos, box, rc, eps)
    acc0 = hsr.force(pos, mass, box, rc, eps, poly)
    a_rms = float(torch.sqrt((acc0.double() ** 2).sum(1).mean()))
    h = math.sqrt(0.01 * w.cell / a_rms)
    log(f"[bench] pairs: candidates {cand:.4e}, inside r_cut {inside:.4e}; h = {h:.3e}")

    if not args.no_accuracy:
        gpu_g = hsr.force_vjp(pos, mass, box, rc, eps, poly,
                              torch.from_numpy(g_np).to(dev))
        acc_info = accuracy(w, acc0.cpu().numpy().astype(np.float64),
                            gpu_g.cpu().numpy(), g_np.astype(np.float64))
        log(f"[bench] accuracy {acc_info}")
    else:
        acc_info = None

    n_c = max(1, args.rollout)
    x = pos.clone()
    v = torch.zeros_like(x)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    ga = torch.empty_like(acc)
    gv = torch.zeros_like(x)
    gtmp = torch.empty_like(x)
    cp = torch.empty_like(x)

    def step():
        # every step starts from the generated state (positions as drawn,
        # zero velocities), so each timed force and VJP sees the workload
        # exactly as counted above
        x.copy_(pos)
        v.zero_()
        # forward subcycle with its checkpoint
        hsr.stream(x, v, 0.5 * h, box)
        cp.copy_(x)
        hsr.force(x, mass, box, rc, eps, poly, out=acc)
        token = hsr.binning_token()
        hsr.kick(v, acc, h)
        hsr.stream(x, v, 0.5 * h, box)
        # reverse subcycle at the checkpoint, loss = sum gx . x_final; the
        # VJP at the checkpoint reuses the forward's binning of it
        gxx = gx.clone()
        gv.zero_()
        hsr.stream(gv, gxx, 0.5 * h, 0.0)
        hsr.kick_adjoint(gv, h, out=ga)
        hsr.force_vjp(cp, mass, box, rc, eps, poly, ga, out=gtmp, binned=token)
        hsr.stream(gxx, gtmp, 1.0, 0.0)
        hsr.stream(gv, gxx, 0.5 * h, 0.0)

    if n_c > 1:
        x0 = pos.clone().requires_grad_(True)
        v0 = torch.zeros_like(pos).requires_grad_(True)

        def step():  # noqa: F811  (the rollout step)
            x0.grad = None
            v0.grad = None
            xf, _ = hsr.rollout_sks(x0, v0, mass, box, rc, eps, poly, h, n_c)
            (gx * xf).sum().backward()

        # in-cut-off pairs at each subcycle's force position (untimed)
        xs, vs = pos.clone(), torch.zeros_like(pos)
        cps = []
        hsr.sks_forward(xs, vs, mass, box, rc, eps, poly, h, n_c, cps)
        counts = [hsr.count_pairs(c, box, rc, eps) for c in cps]
        cand = sum(c[0] for c in counts) / n_c
        inside_per_force = [c[1] for c in counts]
        inside = sum(inside_per_force) / n_c
        del xs, vs, cps
        log(f"[bench] rollout of {n_c} subcycles: mean in-cut-off pairs per force "
            f"{inside:.4e}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")
    hsr.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    n_f, ms_f = hsr.timing_read(hsr.TIMER_FORCE)
    n_v, ms_v = hsr.timing_read(hsr.TIMER_VJP)
    n_b, ms_b = hsr.timing_read(hsr.TIMER_BIN)
    n_w, ms_w = hsr.timing_read(hsr.TIMER_WORKLIST)
    hsr.timing_enable(False)
    log(f"[bench] timed {args.steps} steps in {t_total:.3f}s")

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    peak = None
    if not args.no_probe:
        peak = measured_peak(hsr)
        log(f"[bench] measured VALU peak {peak}")

    ms_step = 1e3 * t_total / args.steps
    value = 2.0 * n_c * inside / (t_total / args.steps)
    f_ms = ms_f / max(n_f, 1)
    v_ms = ms_v / max(n_v, 1)
    fwd_tflops = FLOP_FWD * inside / (f_ms * 1e-3) / 1e12
    vjp_tflops = FLOP_VJP * inside / (v_ms * 1e-3) / 1e12
    if v_ms >= f_ms:
        dom = ("vjp pair kernel (k_pair_vjp)", vjp_tflops, FLOP_VJP, v_ms, "k_pair_vjp")
    else:
        dom = ("forward pair kernel (k_pair_force)", fwd_tflops, FLOP_FWD, f_ms,
               "k_pair_force")
    roof = {"bound": "alu", "kernel": dom[0], "achieved": round(dom[1], 3),
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(dom[1] / FP32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(dom[4]),
            "flop_per_pair": dom[2], "pairs_per_launch": inside,
            "avg_launch_ms": round(dom[3], 4)}
    if peak is not None:
        roof["peak_measured"] = peak["fma_tflops"]
        roof["frac_measured"] = round(dom[1] / peak["fma_tflops"], 4)

    plain = None
    if not args.no_plain:
        plain = plain_comparison(hsr, torch, w, pos, mass, g_np, inside, f_ms, v_ms,
                                 not args.no_accuracy)
        log(f"[bench] plain float32 kernels {plain}")

    rcb = []
    for leaf_max in args.rcb:
        rcb.append(rcb_leg(hsr, torch, w, pos, mass, g_np, inside, leaf_max))
        log(f"[bench] rcb fat leaves {rcb[-1]}")

    pm = None
    full = None
    if not args.no_pm and w.box > 0:
        ng = PM_GRID[args.workload]
        pm = pm_leg(hsr, torch, w, pos, mass, ng)
        log(f"[bench] long-range PM {pm}")
        full = full_step_leg(hsr, torch, w, pos, mass, ng)
        log(f"[bench] full step {full}")

    unequal = None
    if not args.no_unequal:
        unequal = unequal_mass_leg(hsr, torch, w, pos, g_np, inside)
        log(f"[bench] unequal masses {unequal}")

    cpu = None
    if not args.no_cpu_baseline:
        if args.cpu_full:
            cpu = cpu_baseline_full(w, g_np.astype(np.float64))
        else:
            cpu = cpu_baseline(w, args.cpu_seconds, g_np.astype(np.float64))
        log(f"[bench] cpu baseline {cpu}")

    out = {
        "metric": METRIC, "value": value, "unit": "pair interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "n": n, "pairs_inside_rcut": inside,
                   "candidate_pairs": cand,
                   "step": ("one SKS subcycle forward + reverse (force + VJP)"
                            if n_c == 1 else
                            f"differentiable rollout of {n_c} SKS subcycles "
                            f"(autograd, position checkpoints) forward + backward")},
        "roofline": roof,
        "peak_probe": peak,
        "counters": {"k_pair_force": measured_counters("k_pair_force", f_ms),
                     "k_pair_vjp": measured_counters("k_pair_vjp", v_ms)},
        "cpu_baseline": cpu,
        "kernels": {
            "force_pair_ms": round(f_ms, 4), "vjp_pair_ms": round(v_ms, 4),
            "bin_ms": round(ms_b / max(n_b, 1), 4),
            "worklist_ms": round(ms_w / max(n_w, 1), 4),
            "bin_and_gather_ms_per_step": round(ms_b / args.steps, 4),
            "binnings_per_step": round(n_w / args.steps, 3),
            "fwd_interactions_per_s": inside / (f_ms * 1e-3),
            "adj_interactions_per_s": inside / (v_ms * 1e-3),
            "fwd_tflops": round(fwd_tflops, 3), "vjp_tflops": round(vjp_tflops, 3),
            "fwd_pct_fp32_peak": round(100 * fwd_tflops / FP32_PEAK_TFLOPS, 2),
            "vjp_pct_fp32_peak": round(100 * vjp_tflops / FP32_PEAK_TFLOPS, 2),
            # executed rate: counted FLOP x every evaluated candidate pair
            "fwd_executed_tflops": round(FLOP_FWD * cand / (f_ms * 1e-3) / 1e12, 3),
            "vjp_executed_tflops": round(FLOP_VJP * cand / (v_ms * 1e-3) / 1e12, 3),
            "useful_fraction": round(inside / cand, 4),
            "peak_device_memory_gb": round(torch.cuda.max_memory_allocated(dev) / 1e9, 3),
        },
        "unequal_masses": unequal,
        "rcb_fat_leaves": rcb,
        "pm_long_range": pm,
        "full_step": full,
        "accuracy": acc_info,
        "plain_fp32": plain,
        "context": "paper: 13.94 PFlops at 69.2% of peak on 1,572,864 BG/Q cores "
                   "(whole code); force kernel ~80% of BG/Q peak",
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
