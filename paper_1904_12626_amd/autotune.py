"""Autotuner for the sweep's tile shape.

Two knobs set the sweep's work decomposition: the diagonals per lane
(`tile_slots`: 8, 12 or 16 — more slots amortise the per-row register
shifts over more cells but cost registers and occupancy) and the tile height
(`reseed_rows`: rows per tile, which is also the interval at which the FP32
sweep restarts each diagonal from an FP64 seed — taller tiles mean fewer
seeds but more FP32 drift).  The tuner times every candidate on the job it
is given (HIP events around the sweep kernel) and gates it on accuracy
against the FP64 sweep in two ways, each within `budget` x 1e-3 sqrt(m):
  * the raw profile (P taken from the FP32 keys themselves, no FP64
    finalize), which measures the drift the tile height allows;
  * the index: P recomputed in FP64 at the candidate's own I may exceed the
    FP64 sweep's P by at most that much (a worse neighbour chosen because of
    drift shows here even when the finalize hides the drift in P).
The fastest admissible candidate is cached per (device, dtype, precision,
window bucket, size bucket) in a JSON file (MPX_AUTOTUNE_CACHE, default
~/.cache/mpx/autotune.json).  Every decision is logged with its search
space, timings and accuracy.
"""

from __future__ import annotations

import json
import math
import os
import time

import torch

from . import _binding as B

SLOTS = (8, 12, 16)
ROWS = (512, 1024, 2048, 4096, 8192)


def _cache_path():
    return os.environ.get("MPX_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mpx",
                                                             "autotune.json"))


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    p = _cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _key(kind, dtype, precision, m, cells):
    prop = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(prop, "gcnArchName", prop.name)
    mb = 1 << max(0, int(math.log2(max(1, m))))
    cb = int(round(math.log2(max(1, cells))))
    return f"{arch}|cu{prop.multi_processor_count}|{kind}|{dtype}|{precision}|m{mb}|c2^{cb}"


def _time_sweep(fn, reps):
    torch.cuda.synchronize()
    B.timing_query()
    B.timing_enable(True)
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    B.timing_enable(False)
    sweep_ms, total_ms, calls = B.timing_query()
    return out, sweep_ms / max(1, calls), total_ms / max(1, calls)


def tune(kind, run, cells, m, dtype, precision="f32", budget=0.5, reps=2, force=False, log=print,
         return_entry=False):
    """Generic search.  `run(slots, rows, fp64_finalize, precision)` launches
    the job and returns its profile tensor P; returns the chosen
    {'tile_slots', 'reseed_rows'} (with `return_entry`, also the logged
    search: space, trials, budget)."""
    key = _key(kind, str(dtype).replace("torch.", ""), precision, m, cells)
    cache = _load_cache()
    if key in cache and not force:
        entry = cache[key]
        return (entry["choice"], entry) if return_entry else entry["choice"]
    tol = 1e-3 * math.sqrt(m)
    ref = run(8, 0, True, "f64").double().clone() if precision == "f32" else None
    fin = torch.isfinite(ref) if ref is not None else None
    trials = []
    slots_space = SLOTS if precision == "f32" else (8,)
    for slots in slots_space:
        for rows in ROWS:
            try:
                _time_sweep(lambda: run(slots, rows, False, precision), 1)
                P, sweep_ms, _ = _time_sweep(lambda: run(slots, rows, False, precision), reps)
                drift = idx_loss = 0.0
                if ref is not None:
                    drift = float((P.double() - ref)[fin].abs().max())
                    Pf = run(slots, rows, True, precision).double()
                    idx_loss = float((Pf - ref)[fin].max())
            except B.MPError as e:
                trials.append({"tile_slots": slots, "reseed_rows": rows, "error": str(e)})
                continue
            ok = drift <= budget * tol and idx_loss <= budget * tol
            trials.append({"tile_slots": slots, "reseed_rows": rows, "sweep_ms": round(sweep_ms, 4),
                           "raw_max_abs_dP_vs_f64": drift, "index_excess_vs_f64": idx_loss,
                           "within_budget": ok})
    good = [t for t in trials if t.get("within_budget")]
    if not good:
        choice = {"tile_slots": 8, "reseed_rows": 1024}
    else:
        best = min(good, key=lambda t: t["sweep_ms"])
        choice = {"tile_slots": best["tile_slots"], "reseed_rows": best["reseed_rows"]}
    entry = {"choice": choice, "space": {"tile_slots": list(slots_space), "reseed_rows": list(ROWS)},
             "trials": trials, "budget": budget * tol, "cells": cells,
             "time": time.strftime("%Y-%m-%d %H:%M:%S")}
    cache[key] = entry
    _save_cache(cache)
    if log:
        log(f"[autotune] {key}: search slots={list(slots_space)} x rows={list(ROWS)}, budget {budget * tol:.3g}; "
            f"chose {choice}")
        for t in trials:
            log(f"[autotune]   {t}")
    return (choice, entry) if return_entry else choice


def tune_selfjoin(T: torch.Tensor, m: int, ez: int, precision="f32", **kw):
    def run(slots, rows, fin, prec):
        return B.selfjoin(T, m, ez, precision=prec, tile_slots=slots, reseed_rows=rows, fp64_finalize=fin)[0]
    return tune("self", run, B.selfjoin_cells(T.numel(), m, ez), m, T.dtype, precision, **kw)


def tune_abjoin(A: torch.Tensor, Bs: torch.Tensor, m: int, precision="f32", **kw):
    def run(slots, rows, fin, prec):
        Pab, _, Pba, _ = B.abjoin(A, Bs, m, precision=prec, tile_slots=slots, reseed_rows=rows, fp64_finalize=fin)
        return torch.cat([Pab, Pba])
    return tune("ab", run, B.abjoin_cells(A.numel(), Bs.numel(), m), m, A.dtype, precision, **kw)


def tune_batch(T_cat: torch.Tensor, lengths, windows, zones, precision="f32", **kw):
    held = {}

    def run(slots, rows, fin, prec):
        k = (slots, rows, fin, prec)
        if k not in held:            # keep one plan (and its workspace) at a time
            held.clear()
            held[k] = B.BatchPlan(lengths, windows, zones, dtype=T_cat.dtype, device=T_cat.device, precision=prec,
                                  tile_slots=slots, reseed_rows=rows, fp64_finalize=fin)
        return held[k].run(T_cat)[0]
    probe = B.BatchPlan(lengths, windows, zones, dtype=T_cat.dtype, device=T_cat.device)
    cells, mmax = probe.cells, max(windows)
    del probe
    return tune("batch", run, cells, mmax, T_cat.dtype, precision, **kw)
