"""Schedule autotuner.

For one packed matrix, level and batch size it measures candidate schedules
on the device -- baby steps n1, fold radix, rotation direction (which fixes
the fold span) -- and the key-switch / baby-step kernel tiles, and keeps the
fastest.  Every candidate computes the same product (the schedules differ
only in rotation bookkeeping and are each replayed bit-exactly by the
oracle), so the choice is purely a timing decision.  Results are stored per
workload shape in ``tuned.json`` next to this file and looked up by
``tuned_schedule``.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import encoding, planner

TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def shape_key(N: int, L: int, level: int, rows: int, cols: int, batch: int) -> str:
    return f"N{N}_L{L}_level{level}_{rows}x{cols}_batch{batch}"


@dataclass
class Schedule:
    n1: int
    radix: int
    sign: int
    ks_tile: int = 4
    baby_tile: int = 4
    baby_share: int = 8
    ntt_col_w: int = 16
    ntt_blk_w: int = 4
    baby_mfma: int = 8
    baby_fold: int = 8


def library_revision() -> str:
    """sha256 over the library's sources (HIP files, device header, C header):
    a tuning record measured on other code says so."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(here, "csrc", "*"))) + [
        os.path.join(os.path.dirname(here), "include", "helrm.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def candidate_schedules(rows: int, cols: int, n: int, n1s=(4, 8, 16, 32, 64), radices=(4, 8, 16),
                        signs=(-1, 1)) -> List[Schedule]:
    m = planner.next_pow2(rows)
    out = []
    for sign in signs:
        for n1 in n1s:
            if n1 > m or n1 > 64:
                continue
            for r in radices:
                out.append(Schedule(n1, r, sign))
    return out


def tuned_schedule(N: int, L: int, level: int, rows: int, cols: int, batch: int,
                   path: str = TUNED_PATH) -> Optional[Schedule]:
    try:
        with open(path) as f:
            db = json.load(f)
    except OSError:
        return None
    rec = db.get(shape_key(N, L, level, rows, cols, batch))
    if rec is None:
        return None
    b = rec["best"]
    return Schedule(b["n1"], b["radix"], b["sign"], b["ks_tile"], b["baby_tile"], b.get("baby_share", 8),
                    b.get("ntt_col_w", 16), b.get("ntt_blk_w", 4), b.get("baby_mfma", 8), b.get("baby_fold", 8))


def tune(prm, tables, level: int, batch: int, key_draws_fn, enc_draws_fn,
         schedules: Optional[Sequence[Schedule]] = None, tiles: Iterable[int] = (2, 4),
         shares: Iterable[int] = (4, 8), steps: int = 10, warmup: int = 2, log=None) -> Dict:
    """Measure every schedule (and its kernel knobs when batch > 1) and return
    {"best": {...}, "results": [...]}.  key_draws_fn(galois) and
    enc_draws_fn() supply the randomness."""
    import torch

    from .binding import Context
    from .client import Client

    ctx = Context(prm.log_n, prm.q, prm.p, prm.alpha)
    M = planner.packed_matrix(tables)
    rows, cols = M.shape
    if schedules is None:
        schedules = candidate_schedules(rows, cols, prm.n)
    specs = []
    steps_union = set()
    for sc in schedules:
        spec = planner.make_plan(M, prm.N, level, float(prm.q[level]), sc.n1, sc.radix, sc.sign)
        specs.append((sc, spec))
        steps_union.update(spec.rotation_steps())
    gals = sorted({planner.galois(s, prm.N) for s in steps_union})
    client = Client(ctx, prm)
    client.keygen(key_draws_fn(gals), gals)
    idx = [[0 for _ in tables] for _ in range(batch)]
    cts = []
    for q in idx:
        m = encoding.encode(planner.packed_selector(tables, q), prm.delta, prm.N)
        cts.append(client.encrypt(m, level, enc_draws_fn()))
    sel = torch.stack(cts).contiguous()
    out = torch.zeros(batch, 2, level, prm.N, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    results = []
    for sc, spec in specs:
        plan = ctx.helrm_plan_create(level, spec.m, spec.n1, spec.n2, spec.radix, spec.diag, spec.coeffs,
                                     spec.sign, spec.span)
        folded = False
        if batch >= 8 and spec.n2 >= 2 and prm.n_digits(level) <= 3:
            plan.helrm_plan_fold_keys()
            folded = True
        ctx.helrm_reserve(plan, batch, stream)
        # (ks_tile, baby_tile, baby_share, baby_mfma, baby_fold)
        if batch == 1:
            knobs = [(4, 4, 8, 0, 0)]
        elif spec.n2 == 1:   # one giant output: the per-thread baby-step tile matters
            knobs = [(a, b, 8, 0, 0) for a in tiles for b in tiles]
        else:                # several giant outputs: the workgroup-shared kernel's width, or the matrix cores
            knobs = [(a, 4, c, 0, 0) for a in tiles for c in shares]
            if batch >= 8:
                knobs += [(a, 4, 8, 8, 0) for a in tiles]
                if folded:
                    knobs += [(a, 4, 8, 8, 8) for a in tiles]
        for kt, bt, sh, mf, fo in knobs:
            ctx.helrm_set_tuning("ks_tile", kt)
            ctx.helrm_set_tuning("baby_tile", bt)
            ctx.helrm_set_tuning("baby_share", sh)
            ctx.helrm_set_tuning("baby_mfma", mf)
            ctx.helrm_set_tuning("baby_fold", fo)
            for _ in range(warmup):
                ctx.helrm_lookup_packed(plan, sel, batch, out, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                ctx.helrm_lookup_packed(plan, sel, batch, out, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            rec = {"n1": sc.n1, "radix": sc.radix, "sign": sc.sign, "span": spec.span, "ks_tile": kt,
                   "baby_tile": bt, "baby_share": sh, "baby_mfma": mf, "baby_fold": fo, "ms_per_batch": ms,
                   "lookups_per_s": batch * len(tables) / (ms / 1e3), "keys": len(spec.rotation_steps())}
            results.append(rec)
            if log:
                log(rec)
        plan.close()
    best = dict(min(results, key=lambda r: r["ms_per_batch"]))
    # NTT workgroup shapes for the chosen schedule
    sc = Schedule(best["n1"], best["radix"], best["sign"])
    spec = next(sp for s_, sp in specs if (s_.n1, s_.radix, s_.sign) == (sc.n1, sc.radix, sc.sign))
    plan = ctx.helrm_plan_create(level, spec.m, spec.n1, spec.n2, spec.radix, spec.diag, spec.coeffs, spec.sign,
                                 spec.span)
    if best["baby_fold"]:
        plan.helrm_plan_fold_keys()
    for knob in ("ks_tile", "baby_tile", "baby_share", "baby_mfma", "baby_fold"):
        ctx.helrm_set_tuning(knob, best[knob])
    best_ntt = None
    for wc, wb in ((16, 4), (16, 8), (8, 4)):
        ctx.helrm_set_tuning("ntt_col_w", wc)
        ctx.helrm_set_tuning("ntt_blk_w", wb)
        for _ in range(warmup):
            ctx.helrm_lookup_packed(plan, sel, batch, out, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            ctx.helrm_lookup_packed(plan, sel, batch, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        if log:
            log({"ntt_col_w": wc, "ntt_blk_w": wb, "ms_per_batch": ms})
        if best_ntt is None or ms < best_ntt[2]:
            best_ntt = (wc, wb, ms)
    plan.close()
    best["ntt_col_w"], best["ntt_blk_w"] = best_ntt[0], best_ntt[1]
    ctx.close()
    return {"key": shape_key(prm.N, prm.L, level, rows, cols, batch), "best": best, "results": results,
            "when": time.strftime("%Y-%m-%d %H:%M:%S"), "revision": library_revision()}


def record(result: Dict, path: str = TUNED_PATH) -> None:
    try:
        with open(path) as f:
            db = json.load(f)
    except OSError:
        db = {}
    db[result["key"]] = {"best": result["best"], "when": result["when"], "revision": result.get("revision"),
                         "candidates": len(result["results"])}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
