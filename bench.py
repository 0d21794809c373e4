#!/usr/bin/env python3
"""Matrix-profile join benchmark on one MI355X.

Default workload (the largest single-GPU self-join): an n = 2^20 float32
random walk with 8 planted motif pairs and 4 planted discords, window
m = 256, exclusion zone 64.  One step is the whole hot path of one join:
window statistics, FP64 diagonal seeds, the FP32 diagonal sweep (reseeded
every 4096 rows), the packed-key merge, the FP64 finalize of P from I, and
the FP64 recheck of the 8 best motif pairs and 4 discords.  The input is
resident in HBM before timing starts.

Printed: one JSON line with cells/s (admissible pairs per second), the
sweep kernel's VALU roofline fraction (timed live with HIP events on the
launch stream), the FP64 GPU path's rate and the FP32-vs-FP64 agreement,
and the FP64 CPU oracle timed on sampled rows of the same workload.  The
default run adds one record per further workload under "workloads" (the
plain FP64 self-join n=4096, the ECG-like AB-join, the ragged batch of 512
series, the differentiable batch of 64 series): each timed as the median of
at least 5 event-timed steps after 3 warm-ups, with its sweep's roofline
fraction, its tolerance check and its own timed CPU-oracle baseline.

Usage: python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-workloads]
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

METRIC = "matrix-profile cells/sec (FP32-mixed vs FP64) at stated max |ΔP| vs FP64 oracle"

# VALU roofline of the sweep from MI355X's published rates: 256 CUs at
# 2.4 GHz; FP32 vector 157.3 TFLOP/s = 128 FP32 lanes per CU per clock, FP64
# vector 78.6 TFLOP/s = 64 lanes; other VALU instructions (integer minima)
# 64 lanes (4 SIMDs x 16).  A cell costs 6 algorithmic operations: 2 FMA
# (cross product), MUL + FMA (key) in the sweep's precision, and a row and
# a column minimum (integer compares of packed keys).
CU_CLOCKS = 256 * 2.4e9
PEAK_LANE_OPS = CU_CLOCKS * 64               # 3.93e13: one 64-lane instruction per CU per clock
OPS_PER_CELL = 6
PEAK_CELLS = {"f32": CU_CLOCKS / (4 / 128 + 2 / 64),   # 9.83e12 cells/s (FP32-mixed sweep)
              "f64": CU_CLOCKS / (4 / 64 + 2 / 64)}    # 6.55e12 cells/s (FP64 sweep)
PEAK_NOTE = ("published MI355X rates: 4 FP ops per cell at the FP32 (157.3 TFLOP/s: 128 lanes/CU/clock) or FP64 "
             "(78.6: 64 lanes) vector rate plus 2 integer minima at 64 lanes/CU/clock, 256 CUs at 2.4 GHz")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """The host the CPU baseline ran on: CPU model and the cores this
    process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0))}


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the FP32 sweep
    kernel built here is not the one the counters were taken on (compared by
    the SHA-256 of its gfx950 assembly, which the build writes next to the
    library)."""
    rec = os.path.join(ROOT, "profiles", "k_sweep_f32_traffic.json")
    built = os.path.join(ROOT, "paper_1904_12626_amd", "libmpx.sweep.sha256")
    try:
        with open(rec) as f:
            r = json.load(f)
        with open(built) as f:
            h = f.read().strip()
    except OSError:
        return None
    return r["traffic_bytes_per_launch"] if h and r.get("sweep_isa_sha256") == h else None


def valu_ceiling(log):
    """Issue rates the device sustains for the sweep's instruction classes
    and per-cell mixes (bench_valu.hip, built next to the library objects),
    or None when the probe is missing or fails."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1904_12626_amd", "_build", "bench_valu")
    if not os.path.exists(exe):
        return None
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        if r.returncode != 0:
            log(f"[bench] VALU probe failed: {r.stderr.strip()[:200]}")
            return None
        return json.loads(r.stdout)
    except (OSError, ValueError, subprocess.TimeoutExpired) as e:
        log(f"[bench] VALU probe failed: {e}")
        return None


# VALU instructions per cell of the sweeps' loops as compiled (the mixes the
# probe replays): FP32, 24 cells per row pair at 12 slots: 48 v_fmac + 24
# v_fma + 24 v_mul + 24 v_and_or + 21 v_min3 + 4 v_min + 8 DPP + 8 lane
# writes = 161; FP64, 8 cells per row: 24 FMA + 8 MUL + 8 v_and_or + 16
# v_min_f64 + 10 DPP + 8 moves = 74
MIX_F32_PER_CELL = 161 / 24
MIX_F64_PER_CELL = 74 / 8


def ceilings(vc, sweep32_cells_s, sweep64_ms, cells):
    """The sweep's rate against three ceilings: the nominal 6 operations per
    cell at one 64-lane VALU instruction per CU-clock (2.4 GHz); the issue
    rate the probe measured for the loop's own instruction mix; and the
    probe's FMA rate for the 4 floating-point operations per cell alone
    (the bound if every other instruction were free)."""
    out = {"probe": {k: {"lane_instructions_per_s": v["lane_instructions_per_s"],
                         "wave_instructions_per_cu_clock": v["wave_instructions_per_cu_clock"],
                         "core_clock_mhz": v["core_clock_mhz"]}
                     for k, v in vc.items() if isinstance(v, dict)}}
    nominal = PEAK_LANE_OPS / OPS_PER_CELL
    mix32 = vc["fp32_sweep_mix"]["lane_instructions_per_s"] / MIX_F32_PER_CELL
    fp32 = vc["v_fmac_f32"]["lane_instructions_per_s"] / 4
    out["fp32"] = {"published_rates_cells_per_s": PEAK_CELLS["f32"],
                   "frac_published_rates": sweep32_cells_s / PEAK_CELLS["f32"],
                   "one_instruction_per_cu_clock_cells_per_s": nominal, "frac_one_instruction": sweep32_cells_s / nominal,
                   "measured_mix_cells_per_s": mix32, "frac_measured_mix": sweep32_cells_s / mix32,
                   "measured_fma_only_cells_per_s": fp32, "frac_measured_fma_only": sweep32_cells_s / fp32}
    w4 = vc.get("fp32_sweep_mix_4_waves_per_simd")
    if w4:
        # the same mix at the sweep's own occupancy (4 waves per SIMD)
        mix32_w4 = w4["lane_instructions_per_s"] / MIX_F32_PER_CELL
        out["fp32"]["measured_mix_4_waves_cells_per_s"] = mix32_w4
        out["fp32"]["frac_measured_mix_4_waves"] = sweep32_cells_s / mix32_w4
    if sweep64_ms:
        s64 = cells / (sweep64_ms / 1e3)
        mix64 = vc["fp64_sweep_mix"]["lane_instructions_per_s"] / MIX_F64_PER_CELL
        fp64 = vc["v_fma_f64"]["lane_instructions_per_s"] / 4
        out["fp64"] = {"published_rates_cells_per_s": PEAK_CELLS["f64"],
                       "frac_published_rates": s64 / PEAK_CELLS["f64"],
                       "measured_mix_cells_per_s": mix64, "frac_measured_mix": s64 / mix64,
                       "measured_fma_only_cells_per_s": fp64, "frac_measured_fma_only": s64 / fp64}
    return out


def workload(name: str, n_override=None):
    import workloads as W
    if name == "selfjoin_large":
        n = n_override or (1 << 20)
        pw = W.planted_walk(n, 256, 2)
        return dict(kind="self", T=pw.T, m=256, ez=64, planted=pw,
                    desc=f"self-join, float32 random walk n={n} with 8 planted motif pairs and 4 discords, "
                         f"m=256, ez=64")
    if name == "anytime":
        n = n_override or (1 << 20)
        pw = W.planted_walk(n, 256, 2)
        return dict(kind="anytime", T=pw.T, m=256, ez=64, planted=pw,
                    desc=f"anytime self-join: a random 5% of the diagonal-offset chunks of the float32 random walk "
                         f"n={n} with 8 planted motif pairs and 4 discords, m=256, ez=64")
    if name == "left_right":
        n = n_override or (1 << 20)
        pw = W.planted_walk(n, 256, 2)
        return dict(kind="lr", T=pw.T, m=256, ez=64, planted=pw,
                    desc=f"left/right profiles of the float32 random walk n={n} with 8 planted motif pairs and 4 "
                         f"discords, m=256, ez=64, then the corrected arc curve with 2 boundaries and the chains")
    if name == "stream":
        n = n_override or (1 << 20)
        pw = W.planted_walk(n, 256, 2)
        return dict(kind="stream", T=pw.T, m=256, ez=64,
                    desc=f"incremental self-join: the profile of the first {n - 8192} samples of the float32 planted "
                         f"walk (n={n}, m=256, ez=64), then the last 8192 samples appended 512 at a time")
    if name in ("md_simple", "md_multi"):
        n = n_override or (1 << 18)
        rng = np.random.default_rng(7)
        T = np.cumsum(rng.standard_normal((3, n)), axis=1).astype(np.float32)
        mode = "simple" if name == "md_simple" else "multi"
        what = ("SiMPle self-join (raw Euclidean distance summed over the dimensions)" if mode == "simple"
                else "multidimensional profiles (k = 1..3 of the sorted per-dimension z-normalised distances)")
        return dict(kind="md", T=T, m=128, ez=32, mode=mode,
                    desc=f"{what}, 3-dimensional float32 random walk n={n}, m=128, ez=32")
    if name == "selfjoin_small":
        T, m, ez = W.selfjoin_small()
        return dict(kind="self", T=T, m=m, ez=ez, planted=None,
                    desc="self-join, float64 random walk n=4096, m=64, ez=16")
    if name == "abjoin_ecg":
        n = n_override or (1 << 19)
        return dict(kind="ab", A=W.ecg_like(n, 31), B=W.ecg_like(n, 32), m=128,
                    desc=f"AB-join, two float32 ECG-like series n={n}, m=128")
    if name == "batch_ragged":
        rb = W.batch_ragged(n_override or 512)
        return dict(kind="batch", rb=rb, m=None,
                    desc=f"{len(rb.series)} float32 random walks, lengths U{{2048..65536}}, m in {{32,64,128}}, "
                         "ez=m/4, one launch sequence replayed from a captured graph")
    if name == "diff_batch":
        T, m, ez = W.diff_batch(64, n_override or 16384)
        return dict(kind="diff", T=T, m=m, ez=ez,
                    desc=f"differentiable profile: {T.shape[0]} float32 random walks n={T.shape[1]}, m={m}, ez={ez}; "
                         "forward + backward of L = sum(P)")
    raise SystemExit(f"unknown workload {name}")


def ev_steps(fn, steps, warmup):
    """Run `fn` `warmup` times, then `steps` times with a pair of events on
    the current stream around each; returns (last output, median ms, all ms)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    out = None
    for a, b in ev:
        a.record()
        out = fn()
        b.record()
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    return out, float(np.median(ms)), ms


def lib_sweep_ms(fn, reps):
    """Mean duration of the library's sweep kernel and of its whole launch
    sequence per call (HIP events the library records on its stream)."""
    import torch
    import paper_1904_12626_amd as mpx
    torch.cuda.synchronize()
    mpx.timing_query()
    mpx.timing_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    mpx.timing_enable(False)
    sw, tot, calls = mpx.timing_query()
    return sw / max(1, calls), tot / max(1, calls)


def roofline_of(cells, sweep_ms, kernel, prec="f32"):
    ach = cells * OPS_PER_CELL / (sweep_ms / 1e3) / 1e12
    peak = PEAK_CELLS[prec] * OPS_PER_CELL / 1e12
    return {"bound": "alu", "kernel": kernel, "ops_per_cell": OPS_PER_CELL, "sweep_ms_per_launch": sweep_ms,
            "achieved": ach, "peak": peak, "unit": "TOP/s", "frac": ach / peak, "peak_model": PEAK_NOTE,
            "frac_one_instruction_per_cu_clock": ach / (PEAK_LANE_OPS / 1e12)}


def admissible(I, l, ez):
    """Indices in range and outside the exclusion zone (self-join)."""
    i = np.arange(I.size)
    return bool(np.all((I >= 0) & (I < l) & (np.abs(I - i) > ez)))


def rec_selfjoin_f64(steps, warmup, dev):
    """Plain FP64 self-join of a float64 random walk, n = 4096, m = 64,
    ez = 16: the FP64 sweep, P float64, checked against the full oracle."""
    import torch
    import paper_1904_12626_amd as mpx
    import workloads as W
    T, m, ez = W.selfjoin_small()
    n = T.size
    l = n - m + 1
    Tg = torch.from_numpy(T).to(dev)
    cells = mpx.selfjoin_cells(n, m, ez)
    step = lambda: mpx.selfjoin(Tg, m, ez, precision="f64")  # noqa: E731
    (P, I), med, _ = ev_steps(step, steps, warmup)
    sweep_ms, _ = lib_sweep_ms(step, steps)
    Pg, Ig = P.cpu().numpy(), I.cpu().numpy()
    tol = 1e-3 * np.sqrt(m)
    rec = {"workload": f"plain FP64 self-join, float64 random walk n={n}, m={m}, ez={ez}; FP64 sweep, P float64",
           "cells": cells, "dtype": "f64", "steps": steps, "warmup": warmup, "ms_per_step_median": med,
           "cells_per_s": cells / (med / 1e3), "roofline": roofline_of(cells, sweep_ms, "k_sweep<double>", "f64")}
    from oracle import cimpl   # CPU baseline leg: the full oracle, timed
    t0 = time.perf_counter()
    Po, Io = cimpl.selfjoin(T, m, ez)
    dt = time.perf_counter() - t0
    rec["cpu_baseline"] = {"value": cells / dt, "unit": "cells/s", "cores": cimpl.max_threads(), "kind": "oracle",
                           "sample": f"the whole join ({l} rows, {cells} pairs), each O(m) in FP64, {dt:.2f} s"}
    dP = float(np.max(np.abs(Pg - Po)))
    rec["check"] = {"against": "oracle, every row", "max_abs_dP": dP, "tolerance": tol,
                    "index_agreement": float(np.mean(Ig == Io)), "indices_admissible": admissible(Ig, l, ez),
                    "pass": bool(dP <= tol and admissible(Ig, l, ez))}
    return rec


def rec_abjoin(steps, warmup, dev):
    """AB-join of two float32 ECG-like series n = 2^19, m = 128: FP32 sweep
    and the FP64 GPU path, both directions; the oracle on 256 rows of each."""
    import torch
    import paper_1904_12626_amd as mpx
    import workloads as W
    A, Bh, m = W.abjoin_ecg()
    Ag, Bg = torch.from_numpy(A).to(dev), torch.from_numpy(Bh).to(dev)
    cells = mpx.abjoin_cells(A.size, Bh.size, m)
    lA, lB = A.size - m + 1, Bh.size - m + 1
    step32 = lambda: mpx.abjoin(Ag, Bg, m, precision="f32")  # noqa: E731
    step64 = lambda: mpx.abjoin(Ag, Bg, m, precision="f64")  # noqa: E731
    o32, med32, _ = ev_steps(step32, steps, warmup)
    sw32, _ = lib_sweep_ms(step32, max(5, steps // 2))
    o64, med64, _ = ev_steps(step64, steps, warmup)
    sw64, _ = lib_sweep_ms(step64, 5)
    tol = 1e-3 * np.sqrt(m)
    P32 = np.concatenate([o32[0].double().cpu().numpy(), o32[2].double().cpu().numpy()])
    I32 = np.concatenate([o32[1].cpu().numpy(), o32[3].cpu().numpy()])
    P64 = np.concatenate([o64[0].double().cpu().numpy(), o64[2].double().cpu().numpy()])
    I64 = np.concatenate([o64[1].cpu().numpy(), o64[3].cpu().numpy()])
    dP = float(np.max(np.abs(P32 - P64)))
    rec = {"workload": f"AB-join, two float32 ECG-like series n={A.size}, m={m}; P_ab, I_ab, P_ba, I_ba; "
                       "FP32 sweep with FP64 stats and seeds, FP64 finalize",
           "cells": cells, "dtype": "f32", "steps": steps, "warmup": warmup, "ms_per_step_median": med32,
           "cells_per_s": cells / (med32 / 1e3), "roofline": roofline_of(cells, sw32, "k_sweep<float>"),
           "fp64_path": {"ms_per_step_median": med64, "cells_per_s": cells / (med64 / 1e3),
                         "sweep_ms_per_launch": sw64, "speedup_f32_over_f64": med64 / med32,
                         "max_abs_dP_f32_vs_f64": dP, "index_agreement_f32_vs_f64": float(np.mean(I32 == I64))}}
    from oracle import cimpl
    rng = np.random.default_rng(0)
    ra = np.sort(rng.choice(lA, 256, replace=False))
    rb = np.sort(rng.choice(lB, 256, replace=False))
    A64, B64 = A.astype(np.float64), Bh.astype(np.float64)
    t0 = time.perf_counter()
    Pa, Ia = cimpl.abjoin_rows(A64, B64, m, ra)
    Pb, Ib = cimpl.abjoin_rows(B64, A64, m, rb)
    dt = time.perf_counter() - t0
    pairs = int(ra.size * lB + rb.size * lA)
    rec["cpu_baseline"] = {"value": pairs / dt, "unit": "cells/s", "cores": cimpl.max_threads(), "kind": "oracle",
                           "sample": f"{ra.size} rows of P_ab and {rb.size} rows of P_ba, {pairs} pairs, each O(m) "
                                     f"in FP64, {dt:.1f} s"}
    d32 = max(float(np.max(np.abs(P32[:lA][ra] - Pa))), float(np.max(np.abs(P32[lA:][rb] - Pb))))
    d64 = max(float(np.max(np.abs(P64[:lA][ra] - Pa))), float(np.max(np.abs(P64[lA:][rb] - Pb))))
    agree = float(np.mean(np.concatenate([I32[:lA][ra] == Ia, I32[lA:][rb] == Ib])))
    rec["check"] = {"against": "oracle on 256 + 256 sampled rows; FP64 GPU path on every row",
                    "max_abs_dP_f32_vs_oracle": d32, "max_abs_dP_f64_vs_oracle": d64,
                    "index_agreement_f32_vs_oracle": agree, "max_abs_dP_f32_vs_f64": dP, "tolerance": tol,
                    "min_P_ab_equals_min_P_ba": bool(abs(P32[:lA].min() - P32[lA:].min()) <= tol),
                    "pass": bool(max(d32, dP) <= tol)}
    return rec


def rec_batch(steps, warmup, dev, log):
    """512 ragged float32 random walks in one launch sequence, tile shape
    from the autotuner, replayed from a captured graph."""
    import torch
    import paper_1904_12626_amd as mpx
    from paper_1904_12626_amd import autotune as AT
    import workloads as W
    rb = W.batch_ragged()
    Tc, off = rb.concat()
    Tg = torch.from_numpy(Tc).to(dev)
    lengths = [s.size for s in rb.series]
    choice, entry = AT.tune_batch(Tg, lengths, rb.m, rb.ez, force=True, log=log, return_entry=True)
    plans = {}

    def plan_for(prec, slots=0, rows=0):
        k = (prec, slots, rows)
        if k not in plans:
            plans[k] = mpx.BatchPlan(lengths, rb.m, rb.ez, dtype=torch.float32, device=dev, precision=prec,
                                     tile_slots=slots, reseed_rows=rows)
        return plans[k]

    def replay_ms(plan):
        Pg = torch.empty(plan.profile_length, dtype=torch.float32, device=dev)
        Ig = torch.empty(plan.profile_length, dtype=torch.int64, device=dev)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.run(Tg, Pg, Ig)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run(Tg, Pg, Ig)
        _, med, _ = ev_steps(graph.replay, steps, warmup)
        return Pg, Ig, med

    tuned = plan_for("f32", choice["tile_slots"], choice["reseed_rows"])
    cells = tuned.cells
    Pe, Ie = tuned.run(Tg)
    Pr, Ir, med = replay_ms(tuned)
    same = bool(torch.equal(Pr, Pe) and torch.equal(Ir, Ie))
    sweep_ms, _ = lib_sweep_ms(lambda: tuned.run(Tg), 5)
    _, _, med_default = replay_ms(plan_for("f32"))
    P64, I64 = plan_for("f64").run(Tg)
    Pg, Ig = Pr.double().cpu().numpy(), Ir.cpu().numpy()
    P64, I64 = P64.double().cpu().numpy(), I64.cpu().numpy()
    ratio, agree = [], []
    for s, (a, b) in enumerate(zip(tuned.p_off[:-1], tuned.p_off[1:])):
        tol = 1e-3 * np.sqrt(rb.m[s])
        ratio.append(float(np.max(np.abs(Pg[a:b] - P64[a:b]))) / tol)
        agree.append(np.mean(Ig[a:b] == I64[a:b]))
    rec = {"workload": f"{len(lengths)} float32 random walks, lengths U{{2048..65536}}, m in {{32,64,128}}, ez=m/4; "
                       "one launch sequence replayed from a captured graph; FP32 sweep, FP64 finalize",
           "cells": cells, "dtype": "f32", "steps": steps, "warmup": warmup, "ms_per_step_median": med,
           "cells_per_s": cells / (med / 1e3), "roofline": roofline_of(cells, sweep_ms, "k_sweep<float>"),
           "graph_replay_equals_eager": same, "ms_per_step_median_library_defaults": med_default,
           "autotune": {"space": entry["space"], "choice": choice, "budget": entry["budget"],
                        "trials": [{k: t[k] for k in ("tile_slots", "reseed_rows", "sweep_ms", "within_budget")
                                    if k in t} for t in entry["trials"]]}}
    from oracle import cimpl
    order = np.argsort(lengths, kind="stable")
    short = [int(s) for s in order[:8]]
    rng = np.random.default_rng(0)
    rest = [int(s) for s in rng.choice(order[8:], 8, replace=False)]
    t0 = time.perf_counter()
    res, pairs = [], 0
    for s in short:
        T64 = rb.series[s].astype(np.float64)
        Po, Io = cimpl.selfjoin(T64, rb.m[s], rb.ez[s])
        res.append((s, np.arange(Po.size), Po, Io))
        pairs += mpx.selfjoin_cells(T64.size, rb.m[s], rb.ez[s])
    for s in rest:
        T64 = rb.series[s].astype(np.float64)
        l = T64.size - rb.m[s] + 1
        rows = np.sort(rng.choice(l, 32, replace=False))
        Po, Io = cimpl.selfjoin_rows(T64, rb.m[s], rb.ez[s], rows)
        res.append((s, rows, Po, Io))
        pairs += int(sum(l - (min(l - 1, r + rb.ez[s]) - max(0, r - rb.ez[s]) + 1) for r in rows))
    dt = time.perf_counter() - t0
    rec["cpu_baseline"] = {"value": pairs / dt, "unit": "cells/s", "cores": cimpl.max_threads(), "kind": "oracle",
                           "sample": f"the whole joins of the 8 shortest series and 32 random rows of 8 other "
                                     f"series, {pairs} pairs, each O(m) in FP64, {dt:.1f} s"}
    worst, iok = 0.0, []
    for s, rows, Po, Io in res:
        a = tuned.p_off[s]
        worst = max(worst, float(np.max(np.abs(Pg[a + rows] - Po))) / (1e-3 * np.sqrt(rb.m[s])))
        iok.append(np.mean(Ig[a + rows] == Io))
    rec["check"] = {"against": "oracle on 16 series (8 whole, 8 sampled); FP64 GPU batch on every series",
                    "max_abs_dP_over_tolerance_vs_oracle": worst,
                    "index_agreement_vs_oracle": float(np.mean(iok)),
                    "max_abs_dP_over_tolerance_vs_f64": float(max(ratio)),
                    "index_agreement_vs_f64": float(np.mean(agree)),
                    "tolerance": "1e-3 sqrt(m_s) per series",
                    "pass": bool(worst <= 1.0 and max(ratio) <= 1.0 and same)}
    return rec


def rec_diff(steps, warmup, dev, log):
    """Differentiable profile of 64 float32 random walks n = 16384, m = 100:
    forward + backward of L = sum(P) replayed from one captured graph, tile
    shape from the autotuner; the FP64 reference gradient timed on the host."""
    import torch
    import paper_1904_12626_amd as mpx
    from paper_1904_12626_amd import autotune as AT
    import workloads as W
    T, m, ez = W.diff_batch()
    Bn, n = T.shape
    Tg = torch.from_numpy(T).to(dev)
    flat = Tg.reshape(-1)
    choice, entry = AT.tune_batch(flat, [n] * Bn, [m] * Bn, [ez] * Bn, force=True, log=log, return_entry=True)
    plan = mpx.BatchPlan([n] * Bn, [m] * Bn, [ez] * Bn, dtype=torch.float32, device=dev,
                         tile_slots=choice["tile_slots"], reseed_rows=choice["reseed_rows"])
    cells = plan.cells
    ones = torch.ones(Bn, n - m + 1, dtype=torch.float32, device=dev)
    xs = Tg.clone().requires_grad_(True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mpx.MatrixProfileFn.apply(xs, plan)[0].backward(ones)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager_grad = xs.grad.clone()
    xs.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        Pg, Ig = mpx.MatrixProfileFn.apply(xs, plan)
        Pg.backward(ones)
    _, med, _ = ev_steps(graph.replay, steps, warmup)
    same = bool(torch.equal(xs.grad, eager_grad))
    sweep_ms, fwd_ms = lib_sweep_ms(lambda: plan.run(flat), 5)
    Pf, If = plan.run(flat)
    gP = torch.ones(plan.profile_length, dtype=torch.float32, device=dev)
    # the step's backward (autograd reuses the forward's window statistics
    # and distances), and the standalone one that recomputes them
    _, bwd_ms, _ = ev_steps(lambda: plan.backward_after_forward(flat, If, Pf, gP), steps, warmup)
    _, bwd_full_ms, _ = ev_steps(lambda: plan.backward(flat, If, gP), steps, warmup)
    rec = {"workload": f"differentiable profile: {Bn} float32 random walks n={n}, m={m}, ez={ez}; forward + "
                       "backward of L = sum(P) replayed as one captured graph",
           "cells": cells, "dtype": "f32", "steps": steps, "warmup": warmup, "ms_per_step_median": med,
           "cells_per_s": cells / (med / 1e3), "roofline": roofline_of(cells, sweep_ms, "k_sweep<float>"),
           "forward_ms": fwd_ms, "backward_ms_median": bwd_ms, "backward_recomputing_ms_median": bwd_full_ms,
           "graph_replay_equals_eager": same,
           "note": "cells_per_s counts forward cells per second of forward+backward steps",
           "autotune": {"space": entry["space"], "choice": choice, "budget": entry["budget"],
                        "trials": [{k: t[k] for k in ("tile_slots", "reseed_rows", "sweep_ms", "within_budget")
                                    if k in t} for t in entry["trials"]]}}
    g = xs.grad.double().cpu().numpy()
    Ih = Ig.cpu().numpy()
    P64, _ = mpx.BatchPlan([n] * Bn, [m] * Bn, [ez] * Bn, dtype=torch.float32, device=dev,
                           precision="f64").run(flat)
    dP = float(np.max(np.abs(Pg.detach().double().cpu().numpy().reshape(-1) - P64.double().cpu().numpy())))
    from oracle import mp_oracle as O
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(Bn, 4, replace=False))
    T64 = T.astype(np.float64)
    t0 = time.perf_counter()
    refs = [O.reference_gradient(T64[b], m, Ih[b], np.ones(Ih.shape[1])) for b in sel]
    dt = time.perf_counter() - t0
    rel = max(float(np.max(np.abs(g[b] - r)) / np.max(np.abs(r))) for b, r in zip(sel, refs))
    rows = int(sel.size * Ih.shape[1])
    rec["cpu_baseline"] = {"value": rows / dt, "unit": "rows/s", "cores": 1, "kind": "oracle",
                           "sample": f"FP64 reference gradient (closed form through each row's argmin pair, numpy) "
                                     f"of {sel.size} of the {Bn} series, {rows} rows, {dt:.1f} s; the GPU backward "
                                     f"does {Bn * Ih.shape[1]} rows in {bwd_ms:.3f} ms"}
    rec["check"] = {"against": "FP64 reference gradient on 4 series; FP64 GPU forward on every row",
                    "max_rel_grad_err": rel, "grad_tolerance": 1e-4, "max_abs_dP_f32_vs_f64": dP,
                    "tolerance": 1e-3 * np.sqrt(m), "pass": bool(rel <= 1e-4 and dP <= 1e-3 * np.sqrt(m) and same)}
    return rec


def extra_workloads(steps, warmup, dev, log):
    out = {}
    for name, fn in (("selfjoin_f64_n4096_m64", lambda: rec_selfjoin_f64(steps, warmup, dev)),
                     ("abjoin_ecg_2x2p19_m128", lambda: rec_abjoin(steps, warmup, dev)),
                     ("batch_ragged_512", lambda: rec_batch(steps, warmup, dev, log)),
                     ("diff_batch_64x16384_m100", lambda: rec_diff(steps, warmup, dev, log))):
        t0 = time.perf_counter()
        try:
            out[name] = fn()
            r = out[name]
            log(f"[bench] {name}: {r['ms_per_step_median']:.3f} ms/step, {r['cells_per_s']:.3e} cells/s, "
                f"roofline {r['roofline']['frac']:.3f}, check pass={r['check']['pass']} "
                f"({time.perf_counter() - t0:.1f} s)")
        except Exception as e:  # keep the headline line even if one record fails
            out[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {name}: FAILED {type(e).__name__}: {e}")
    return out


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="selfjoin_large",
                    choices=["selfjoin_large", "selfjoin_small", "abjoin_ecg", "batch_ragged", "diff_batch",
                             "anytime", "left_right", "md_simple", "md_multi", "stream"])
    ap.add_argument("--fraction", type=float, default=0.05, help="anytime workload: fraction of chunks timed")
    ap.add_argument("--n", type=int, default=None, help="override the series length")
    ap.add_argument("--slots", type=int, default=0, help="diagonals per lane (0 = automatic)")
    ap.add_argument("--reseed", type=int, default=0, help="rows per tile / reseed interval (0 = automatic)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path comparison")
    ap.add_argument("--autotune", action="store_true",
                    help="pick tile slots and reseed rows with the autotuner before timing (search logged)")
    ap.add_argument("--cpu-rows", type=int, default=600,
                    help="random oracle rows timed for the CPU baseline, about 10-30 s of host work on the default "
                         "workload (0 = skip)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="default workload only: skip the records of the other workloads")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-traffic reference "
                         "for hardware byte counters)")
    return ap.parse_args()


def copy_calibration(mib, dev):
    """One plain device copy of `mib` MiB: a known-traffic reference for the
    hardware byte counters of a profiled run."""
    import torch
    nb = mib << 20
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {nb} bytes read, {nb} bytes written")


def setup(wl, args, dev):
    """The inputs of a workload on the device, its cell count and `step`, one
    pass of its hot path in a given precision ("f32" or "f64")."""
    import types
    import torch
    import paper_1904_12626_amd as mpx
    w = types.SimpleNamespace(kind=wl["kind"], m=wl["m"], plans={})
    m, slots, reseed = wl["m"], args.slots, args.reseed
    if w.kind in ("self", "anytime", "lr", "stream", "md", "diff"):
        w.T, w.ez = wl["T"], wl["ez"]
        w.Tg = torch.from_numpy(w.T).to(dev)
    if w.kind == "self":
        w.n = w.T.size
        w.cells = mpx.selfjoin_cells(w.n, m, w.ez)
        km, kd = (8, 4) if wl["planted"] is not None else (3, 1)

        def step(precision):
            P, I = mpx.selfjoin(w.Tg, m, w.ez, precision=precision, tile_slots=args.slots, reseed_rows=args.reseed)
            idx, dist = mpx.recheck(w.Tg, m, P, I, km, kd)
            return P, I, idx, dist
    elif w.kind == "anytime":
        w.n = w.T.size
        w.nchunk, w.cwidth = mpx.selfjoin_chunks(w.n, m, w.ez, tile_slots=slots)
        order = mpx.anytime_order(w.nchunk, 0)

        def anytime_plan(frac, precision="f32"):
            k = min(w.nchunk, max(1, int(np.ceil(frac * w.nchunk))))
            if (k, precision) not in w.plans:
                w.plans[(k, precision)] = mpx.SelfJoinPlan(w.n, m, w.ez, dtype=torch.float32, device=dev,
                                                           chunks=order[:k], precision=precision,
                                                           tile_slots=slots, reseed_rows=reseed)
            return w.plans[(k, precision)]
        w.anytime_plan = anytime_plan
        w.cells = anytime_plan(args.fraction).cells

        def step(precision):
            P, I = anytime_plan(args.fraction, precision).run(w.Tg)
            idx, dist = mpx.recheck(w.Tg, m, P, I, 8, 4)
            return P, I, idx, dist
    elif w.kind == "lr":
        w.n = w.T.size
        l = w.n - m + 1

        def step(precision):
            if precision not in w.plans:
                w.plans[precision] = mpx.SelfJoinPlan(w.n, m, w.ez, dtype=torch.float32, device=dev, sides="lr",
                                                      precision=precision, tile_slots=slots, reseed_rows=reseed)
            P, I = w.plans[precision].run(w.Tg)
            cac, seg = mpx.fluss(I[:l], m, k=2)
            ch = mpx.chains(I[l:2 * l], I[2 * l:])
            return P, I, cac, seg, ch
        w.cells = mpx.selfjoin_cells(w.n, m, w.ez)
    elif w.kind == "stream":
        w.n = w.T.size
        n0 = w.n - 8192
        l0 = n0 - m + 1
        # pairs scored by the appends: every new window against its admissible earlier windows
        w.cells = sum(max(0, i - w.ez) for i in range(l0, w.n - m + 1))
        w.state = {}

        def step(precision):
            st = mpx.SelfJoinStream(w.Tg[:n0], m, w.ez, n_max=w.n)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for b in range(n0, w.n, 512):
                st.append(w.Tg[b:b + 512])
            torch.cuda.synchronize()
            w.state["append_ms"] = (time.perf_counter() - t0) * 1e3
            w.state["last"] = st
            return st.P, st.I
    elif w.kind == "md":
        w.n = w.T.shape[1]
        w.cells = mpx.selfjoin_cells(w.n, m, w.ez)

        def step(precision):
            return mpx.mdjoin(w.Tg, m, w.ez, mode=wl["mode"])
    elif w.kind == "ab":
        w.Ag, w.Bg = torch.from_numpy(wl["A"]).to(dev), torch.from_numpy(wl["B"]).to(dev)
        w.cells = mpx.abjoin_cells(wl["A"].size, wl["B"].size, m)

        def step(precision):
            return mpx.abjoin(w.Ag, w.Bg, m, precision=precision, tile_slots=args.slots, reseed_rows=args.reseed)
    elif w.kind == "batch":
        rb = wl["rb"]
        Tc, _ = rb.concat()
        w.Tg = torch.from_numpy(Tc).to(dev)

        def plan_for(precision):
            if precision not in w.plans:
                w.plans[precision] = mpx.BatchPlan([s.size for s in rb.series], rb.m, rb.ez, dtype=torch.float32,
                                                   device=dev, precision=precision, tile_slots=args.slots,
                                                   reseed_rows=args.reseed)
            return w.plans[precision]
        w.plan_for = plan_for
        w.cells = plan_for("f32").cells

        def step(precision):
            return plan_for(precision).run(w.Tg)
    else:  # "diff": forward + backward of L = sum(P) through the autograd function
        B, n = w.T.shape
        w.cells = B * mpx.selfjoin_cells(n, m, w.ez)

        def step(precision):
            if precision not in w.plans:
                w.plans[precision] = mpx.BatchPlan([n] * B, [m] * B, [w.ez] * B, dtype=torch.float32, device=dev,
                                                   precision=precision, tile_slots=args.slots,
                                                   reseed_rows=args.reseed)
            x = w.Tg.clone().requires_grad_(True)
            P, I = mpx.MatrixProfileFn.apply(x, w.plans[precision])
            P.sum().backward()
            return P, I, x.grad
    w.step = step
    return w


def autotune(w, wl, args):
    """Replace the tile shape of args by the autotuner's choice for this job
    (self-joins, AB-joins and batches; the search is logged)."""
    from paper_1904_12626_amd import autotune as AT
    if w.kind == "self":
        ch = AT.tune_selfjoin(w.Tg, w.m, w.ez, log=log)
    elif w.kind == "ab":
        ch = AT.tune_abjoin(w.Ag, w.Bg, w.m, log=log)
    else:
        rb = wl["rb"]
        ch = AT.tune_batch(w.Tg, [s.size for s in rb.series], rb.m, rb.ez, log=log)
    args.slots, args.reseed = ch["tile_slots"], ch["reseed_rows"]
    if w.kind == "batch":
        w.plans.clear()


def timed(step, precision, steps, warmup):
    """`warmup` untimed steps, then `steps` steps between two synchronisations.
    Returns the last output, wall-clock ms per step, the median of the steps'
    event-timed ms, and the library's mean sweep and launch-sequence ms."""
    import torch
    import paper_1904_12626_amd as mpx
    for _ in range(warmup):
        step(precision)
    torch.cuda.synchronize()
    mpx.timing_query()                      # drop earlier records
    mpx.timing_enable(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        out = step(precision)
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mpx.timing_enable(False)
    sweep_ms, total_ms, calls = mpx.timing_query()
    med = float(np.median([a.elapsed_time(b) for a, b in ev]))
    return out, (t1 - t0) * 1e3 / steps, med, sweep_ms / max(calls, 1), total_ms / max(calls, 1)


def run_stream(w, wl, args):
    """The streaming workload: 8192 windows appended to the n = 2^20 profile
    in batches of 512 samples; the timed unit is the appends."""
    for _ in range(args.warmup):
        w.step("f64")
    times = []
    for _ in range(args.steps):
        w.step("f64")
        times.append(w.state["append_ms"])
    ms = float(np.median(times))
    st = w.state["last"]
    m, cells = w.m, w.cells
    l = w.n - m + 1
    result = {
        "metric": METRIC, "value": cells / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"] + "; FP64 state, new windows in batches of up to 63",
                   "cells": cells, "windows_appended": 8192, "appended_windows_per_s": 8192 / (ms / 1e3)},
        # a batch of up to 63 new windows reads each column's terms once, so the scored pairs
        # cost FP64 arithmetic: 2 FMA (cross product), MUL + FMA + MAX (key), the column
        # compare and the row minimum = 7 operations
        "roofline": {"bound": "alu", "achieved": cells * 7 / (ms / 1e3) / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "TOP/s", "frac": cells * 7 / (ms / 1e3) / 1e12 / (PEAK_LANE_OPS / 1e12),
                     "traffic": None, "kernel": "k_stream_batch", "ops_per_cell": 7,
                     "note": "per batch of up to 63 windows: ~13 us reading and writing the state of every "
                             "earlier window, then ~0.66 us per window"},
    }
    if args.cpu_rows > 0:
        from oracle import cimpl
        rng = np.random.default_rng(0)
        rows = np.sort(rng.choice(l, 64, replace=False))
        T64 = w.T.astype(np.float64)
        t0 = time.perf_counter()
        Po, Io = cimpl.selfjoin_rows(T64, m, w.ez, rows)
        dt = time.perf_counter() - t0
        pairs = int(sum(l - (min(l - 1, r + w.ez) - max(0, r - w.ez) + 1) for r in rows))
        Pg = st.P.double().cpu().numpy()[rows]
        result["cpu_baseline"] = {"value": pairs / dt, "unit": "cells/s", "cores": cimpl.max_threads(),
                                  "kind": "oracle",
                                  "sample": f"{rows.size} full rows of the grown series' self-join, {pairs} pairs, "
                                            f"{dt:.1f} s",
                                  "host": host_cpu()}
        result["oracle_check"] = {"rows": int(rows.size), "max_abs_dP_vs_oracle": float(np.max(np.abs(Pg - Po)))}
    return result


def fp32_result(w, wl, args, ms32, med32, sweep32):
    """The line of the FP32 run: whole-step rate and the sweep's roofline."""
    cells = w.cells
    achieved = cells * OPS_PER_CELL / (sweep32 / 1e3) / 1e12
    peak32 = PEAK_CELLS["f32"] * OPS_PER_CELL / 1e12
    default = (w.kind == "self" and args.n is None and not args.slots and not args.reseed
               and args.workload == "selfjoin_large")
    return {
        "metric": METRIC,
        "value": cells / (ms32 / 1e3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "ms_per_step_median": med32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"] + "; FP32 sweep with FP64 stats and seeds, FP64 finalize and recheck",
                   "cells": cells, "tile_slots": args.slots or "auto", "reseed_rows": args.reseed or "auto"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak32, "unit": "TOP/s",
                     "frac": achieved / peak32, "peak_model": PEAK_NOTE,
                     "frac_one_instruction_per_cu_clock": achieved / (PEAK_LANE_OPS / 1e12),
                     "traffic": measured_traffic() if default else None,
                     "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE of the FP32 sweep on this workload "
                                       "(copy-calibrated), profiles/k_sweep_f32_traffic.json; reported only "
                                       "while the built sweep's gfx950 assembly hash equals the counted one, "
                                       "else null",
                     "kernel": "k_sweep<float>", "ops_per_cell": OPS_PER_CELL,
                     "sweep_ms_per_launch": sweep32, "sweep_cells_per_s": cells / (sweep32 / 1e3)},
    }


def replay_graph(capture, outputs_match, result, ms32, args):
    """Capture `capture()` (already run once eagerly, on a side stream) as
    one graph, time its replays and record them in `result` as the step."""
    import torch
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        capture()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    msg = (time.perf_counter() - t0) * 1e3 / args.steps
    same = outputs_match()
    log(f"[bench] graph replay: {msg:.2f} ms/step (eager {ms32:.2f}); replay equals eager: {same}")
    result["eager_ms_per_step"] = ms32
    result["ms_per_step"] = msg
    result["value"] = result["config"]["cells"] / (msg / 1e3)
    result["graph_replay_equals_eager"] = same


def eager_on_side_stream(fn):
    """Run `fn` once on a side stream (the warm-up torch's graph capture
    asks for) and wait for it."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()


def post_batch(w, wl, args, result, out32, ms32, dev):
    """The batch replayed from one captured graph is the timed step."""
    import torch
    plan = w.plan_for("f32")
    Pg = torch.empty(plan.profile_length, dtype=torch.float32, device=dev)
    Ig = torch.empty(plan.profile_length, dtype=torch.int64, device=dev)
    eager_on_side_stream(lambda: plan.run(w.Tg, Pg, Ig))
    replay_graph(lambda: plan.run(w.Tg, Pg, Ig),
                 lambda: bool(torch.equal(Pg, out32[0]) and torch.equal(Ig, out32[1])), result, ms32, args)
    result["config"]["series"] = len(wl["rb"].series)


def post_diff(w, args, result, out32, ms32):
    """The same forward + backward step captured once and replayed: dL/dP = 1
    comes from a static ones tensor (torch's multi-block sum would put a
    memset into the graph), outputs and gradient are static."""
    import torch
    import paper_1904_12626_amd as mpx
    plan = w.plans["f32"]
    ones = torch.ones_like(out32[0])
    xs = w.Tg.clone().requires_grad_(True)
    eager_on_side_stream(lambda: mpx.MatrixProfileFn.apply(xs, plan)[0].backward(ones))
    xs.grad = None
    out = {}

    def capture():
        out["P"], out["I"] = mpx.MatrixProfileFn.apply(xs, plan)
        out["P"].backward(ones)
    replay_graph(capture, lambda: bool(torch.equal(out["P"], out32[0]) and torch.equal(out["I"], out32[1])
                                       and torch.equal(xs.grad, out32[2])), result, ms32, args)
    result["config"]["note"] = ("value counts forward cells per second of forward+backward steps, "
                                "replayed as one captured graph")


def post_md(w, wl, result, sweep32):
    """Multidimensional joins: their own algorithmic VALU operations per cell."""
    D = wl["T"].shape[0]
    ops = 5 * D + 2 if wl["mode"] == "simple" else 6 * D + D * (D - 1) + 4 * D
    ach = w.cells * ops / (sweep32 / 1e3) / 1e12
    result["dtype"] = "f64"
    result["config"]["workload"] = wl["desc"] + "; FP64 cross products, 32-bit candidate keys, FP64 recompute of P"
    result["config"]["dims"] = D
    result["roofline"].update({"achieved": ach, "frac": ach / (PEAK_LANE_OPS / 1e12), "kernel": "k_md_sweep",
                               "ops_per_cell": ops, "traffic": None})


def post_lr(result, out32):
    ch = out32[4]
    result["config"]["longest_chain"] = len(ch["best"])
    result["config"]["chains_min3"] = ch["count"]
    result["config"]["boundaries"] = [int(v) for v in out32[3].cpu().tolist()]


def post_anytime(w, wl, args, result):
    """Convergence of the best-so-far profile towards the exact one as more
    chunks (in one fixed random order) are included."""
    import torch
    import paper_1904_12626_amd as mpx
    m, n = w.m, w.n
    tol = 1e-3 * np.sqrt(m)
    Pfull, _ = w.anytime_plan(1.0).run(w.Tg)
    Pfull = Pfull.double().cpu().numpy()
    planted = wl["planted"].motif_pairs
    conv = []
    for frac in (0.01, 0.02, 0.05, 0.1, 0.25, 0.5, 1.0):
        plan = w.anytime_plan(frac)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, I = plan.run(w.Tg)
        idx, _ = mpx.recheck(w.Tg, m, P, I, 8, 0)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        Ph = P.double().cpu().numpy()
        fin = np.isfinite(Pfull)
        found = [tuple(sorted(p)) for p in idx.cpu().numpy()[:16].reshape(8, 2)]
        hits = sum(any(abs(a - x) <= m // 8 and abs(b - y) <= m // 8 for x, y in found) for a, b in planted)
        conv.append({"fraction_of_chunks": plan.cells / mpx.selfjoin_cells(n, m, w.ez), "chunks": len(plan.chunks),
                     "ms": ms, "rows_within_tol_of_exact": float(np.mean(np.abs(Ph[fin] - Pfull[fin]) <= tol)),
                     "mean_excess_over_exact": float(np.mean(Ph[fin] - Pfull[fin])),
                     "planted_pairs_in_top8_motifs": int(hits)})
        log(f"[bench] anytime {conv[-1]}")
    result["convergence"] = conv
    result["config"]["chunk_width"] = w.cwidth
    result["config"]["chunks_total"] = w.nchunk
    result["config"]["chunks_timed"] = len(w.anytime_plan(args.fraction).chunks)


def fp64_leg(w, args, result, out32, ms32):
    """The FP64 GPU path of a self-join or AB-join: 3 warm-ups, then the
    median of at least 5 event-timed steps, and the FP32 path's agreement
    with it.  Returns its last output."""
    import paper_1904_12626_amd as mpx
    m, cells = w.m, w.cells
    out64, ms64, _ = ev_steps(lambda: w.step("f64"), max(5, min(args.steps, 8)), 3)
    sweep64, _ = lib_sweep_ms(lambda: w.step("f64"), 3)
    log(f"[bench] f64: {ms64:.2f} ms/step (median), sweep {sweep64:.2f} ms")
    P32, I32 = out32[0].double().cpu().numpy(), out32[1].cpu().numpy()
    P64, I64 = out64[0].double().cpu().numpy(), out64[1].cpu().numpy()
    if w.kind == "ab":   # both directions
        P32 = np.concatenate([P32, out32[2].double().cpu().numpy()])
        I32 = np.concatenate([I32, out32[3].cpu().numpy()])
        P64 = np.concatenate([P64, out64[2].double().cpu().numpy()])
        I64 = np.concatenate([I64, out64[3].cpu().numpy()])
    fin = np.isfinite(P64)
    raw = None
    if w.kind == "self":
        Praw, _ = mpx.selfjoin(w.Tg, m, w.ez, precision="f32", fp64_finalize=False)
        raw = float(np.max(np.abs(Praw.double().cpu().numpy()[fin] - P64[fin])))
    result["fp64_path"] = {
        "value": cells / (ms64 / 1e3), "ms_per_step": ms64, "sweep_ms_per_launch": sweep64,
        "speedup_f32_over_f64": ms64 / ms32, "steps": max(5, min(args.steps, 8)), "warmup": 3,
        "timing": "median of event-timed steps",
        "max_abs_dP_f32_vs_f64": float(np.max(np.abs(P32[fin] - P64[fin]))),
        "max_abs_dP_f32_raw_vs_f64": raw,
        "index_agreement_f32_vs_f64": float(np.mean(I32 == I64)),
        "tolerance": 1e-3 * np.sqrt(m),
        "roofline": roofline_of(cells, sweep64, "k_sweep<double>", "f64"),
    }
    return out64


def cpu_leg_self(w, wl, args, result, out32, out64):
    """The oracle on sampled full rows of the same self-join (random rows plus
    the planted ones), timed, and the GPU rows checked against it."""
    from oracle import cimpl
    m, ez, n = w.m, w.ez, w.n
    rng = np.random.default_rng(0)
    l = n - m + 1
    rows = list(rng.choice(l, args.cpu_rows, replace=False))
    if wl["planted"] is not None:
        for a, b in wl["planted"].motif_pairs:
            rows += [a, b]
        rows += list(wl["planted"].discords)
    rows = np.array(sorted(set(int(r) for r in rows)), dtype=np.int64)
    T64 = w.T.astype(np.float64)
    threads = cimpl.max_threads()
    t0 = time.perf_counter()
    Po, Io = cimpl.selfjoin_rows(T64, m, ez, rows)
    dt = time.perf_counter() - t0
    pairs = int(sum(l - (min(l - 1, r + ez) - max(0, r - ez) + 1) for r in rows))
    P32 = out32[0].double().cpu().numpy()[rows]
    I32 = out32[1].cpu().numpy()[rows]
    result["cpu_baseline"] = {
        "value": pairs / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
        "sample": f"{rows.size} full rows of the same self-join ({args.cpu_rows} random + the planted motif "
                  f"members and discords), {pairs} pairs, each O(m) in FP64, {dt:.1f} s",
    }
    tol = 1e-3 * np.sqrt(m)
    dP = float(np.max(np.abs(P32 - Po)))
    result["oracle_check"] = {
        "rows": int(rows.size),
        "max_abs_dP_f32_vs_oracle": dP,
        "index_agreement": float(np.mean(I32 == Io)),
        "tolerance": tol,
    }
    ok = dP <= tol
    if out64 is not None:
        P64r = out64[0].double().cpu().numpy()[rows]
        result["oracle_check"]["max_abs_dP_f64_vs_oracle"] = float(np.max(np.abs(P64r - Po)))
        ok = ok and result["fp64_path"]["max_abs_dP_f32_vs_f64"] <= tol
    result["oracle_check"]["pass"] = bool(ok)


def cpu_leg_anytime(w, args, result, out32):
    """The oracle restricted to the timed chunk set, on sampled rows."""
    from oracle import cimpl
    m, ez, n = w.m, w.ez, w.n
    plan = w.anytime_plan(args.fraction)
    l = n - m + 1
    allowed = np.zeros(l, dtype=bool)
    for c in plan.chunks:
        allowed[ez + 1 + c * w.cwidth:min(ez + (c + 1) * w.cwidth, l - 1) + 1] = True
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(l, args.cpu_rows, replace=False)).astype(np.int64)
    T64 = w.T.astype(np.float64)
    t0 = time.perf_counter()
    Po, Io = cimpl.selfjoin_rows_restricted(T64, m, ez, rows, allowed)
    dt = time.perf_counter() - t0
    ks = np.nonzero(allowed)[0]
    pairs = int(sum(np.count_nonzero(r - ks >= 0) + np.count_nonzero(r + ks < l) for r in rows))
    result["cpu_baseline"] = {
        "value": pairs / dt, "unit": "cells/s", "cores": cimpl.max_threads(), "kind": "oracle",
        "sample": f"{rows.size} random rows of the same chunk-restricted self-join, {pairs} pairs, "
                  f"each O(m) in FP64, {dt:.1f} s"}
    result["oracle_check"] = {
        "rows": int(rows.size),
        "max_abs_dP_f32_vs_oracle": float(np.max(np.abs(out32[0].double().cpu().numpy()[rows] - Po))),
        "index_agreement": float(np.mean(out32[1].cpu().numpy()[rows] == Io)),
    }


def cpu_leg_md(w, wl, args, result, out32):
    """The numpy oracle of the multidimensional join on a few sampled rows."""
    from oracle import mp_oracle as O
    m, ez = w.m, w.ez
    T64 = wl["T"].astype(np.float64)
    D, n = T64.shape
    l = n - m + 1
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(l, max(4, args.cpu_rows // 16), replace=False))
    t0 = time.perf_counter()
    if wl["mode"] == "simple":
        Po, Io = O.simple_join(T64, m, ez, rows=rows)
        Po, Io = Po[rows], Io[rows]
        Pg = out32[0].double().cpu().numpy()[rows]
    else:
        Po, Io = O.mstomp(T64, m, ez, rows=rows)
        Po, Io = Po[:, rows], Io[:, rows]
        Pg = out32[0].double().cpu().numpy()[:, rows]
    dt = time.perf_counter() - t0
    pairs = int(sum(l - (min(l - 1, r + ez) - max(0, r - ez) + 1) for r in rows))
    result["cpu_baseline"] = {
        "value": pairs / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
        "sample": f"{rows.size} full rows of the same join (numpy, {D} dimensions), {pairs} pairs, {dt:.1f} s"}
    result["oracle_check"] = {"rows": int(rows.size),
                              "max_rel_dP_vs_oracle": float(np.max(np.abs(Pg - Po) / np.maximum(1.0, Po)))}


def cpu_leg_ab(w, wl, args, result, out32):
    """The oracle on sampled rows of both directions of the AB-join."""
    from oracle import cimpl
    m = w.m
    rng = np.random.default_rng(0)
    A64, B64 = wl["A"].astype(np.float64), wl["B"].astype(np.float64)
    lA, lB = A64.size - m + 1, B64.size - m + 1
    ra = np.sort(rng.choice(lA, args.cpu_rows // 2, replace=False))
    rb_ = np.sort(rng.choice(lB, args.cpu_rows // 2, replace=False))
    t0 = time.perf_counter()
    Pa, Ia = cimpl.abjoin_rows(A64, B64, m, ra)
    Pb, Ib = cimpl.abjoin_rows(B64, A64, m, rb_)
    dt = time.perf_counter() - t0
    pairs = int(ra.size * lB + rb_.size * lA)
    result["cpu_baseline"] = {
        "value": pairs / dt, "unit": "cells/s", "cores": cimpl.max_threads(), "kind": "oracle",
        "sample": f"{ra.size} rows of P_ab and {rb_.size} rows of P_ba, {pairs} pairs, each O(m) in FP64, "
                  f"{dt:.1f} s"}
    result["oracle_check"] = {
        "rows": int(ra.size + rb_.size),
        "max_abs_dP_f32_vs_oracle": float(max(np.max(np.abs(out32[0].double().cpu().numpy()[ra] - Pa)),
                                              np.max(np.abs(out32[2].double().cpu().numpy()[rb_] - Pb)))),
    }


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); the self-join would shard by diagonal ranges with one min-reduction "
              "of the packed keys (see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.copy_calib_mib > 0:
        copy_calibration(args.copy_calib_mib, dev)
    wl = workload(args.workload, args.n)
    w = setup(wl, args, dev)
    if args.autotune and w.kind in ("self", "ab", "batch"):
        autotune(w, wl, args)
    log(f"[bench] workload: {wl['desc']}; cells={w.cells}")
    if w.kind == "stream":
        print(json.dumps(run_stream(w, wl, args)), flush=True)
        return

    out32, ms32, med32, sweep32, tot32 = timed(w.step, "f32", args.steps, args.warmup)
    log(f"[bench] f32: {ms32:.2f} ms/step, sweep {sweep32:.2f} ms, launch sequence {tot32:.2f} ms")
    result = fp32_result(w, wl, args, ms32, med32, sweep32)
    if w.kind == "batch":
        post_batch(w, wl, args, result, out32, ms32, dev)
    elif w.kind == "diff":
        post_diff(w, args, result, out32, ms32)
    elif w.kind == "md":
        post_md(w, wl, result, sweep32)
    elif w.kind == "lr":
        post_lr(result, out32)
    elif w.kind == "anytime":
        post_anytime(w, wl, args, result)

    out64 = None
    if not args.no_fp64 and w.kind in ("self", "ab"):
        out64 = fp64_leg(w, args, result, out32, ms32)
    if args.cpu_rows > 0:
        if w.kind == "self":
            cpu_leg_self(w, wl, args, result, out32, out64)
        elif w.kind == "anytime":
            cpu_leg_anytime(w, args, result, out32)
        elif w.kind == "md":
            cpu_leg_md(w, wl, args, result, out32)
        elif w.kind == "ab":
            cpu_leg_ab(w, wl, args, result, out32)
    if "cpu_baseline" in result:
        result["cpu_baseline"]["host"] = host_cpu()
    if (args.workload == "selfjoin_large" and not args.no_workloads and args.n is None and not args.slots
            and not args.reseed and not args.autotune):
        vc = valu_ceiling(log)
        if vc is not None:
            result["roofline"]["ceilings"] = ceilings(vc, result["roofline"]["sweep_cells_per_s"],
                                                      result.get("fp64_path", {}).get("sweep_ms_per_launch"),
                                                      w.cells)
        result["workloads"] = extra_workloads(max(5, min(args.steps, 20)), 3, dev, log)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
