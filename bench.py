#!/usr/bin/env python3
"""Benchmark: encrypted packed embedding lookups on one MI355X.

Workloads (seeded synthetic data of the paper's shapes):
  w2  N = 2^16, 24 ciphertext primes (60 + 23 x 40 bits), dnum = 3 with 8
      special 60-bit primes; one 65,536-row x 16 table stored as two 256 x 16
      digit tables (base 256, values U[-0.05, 0.05]); selector at level 23.
  w3  same parameters; 26 tables with log-uniform row counts in [4, 1e7]
      (~3.4e7 rows), 16-dim, base 256 (tables of at most 256 rows stay
      uncompressed), all packed block-diagonally into one selector ciphertext
      per query; batch of 64 queries.
  w6  same parameters; the lookup shape of the paper's comparison with prior
      work (Table I): d = 768 rows from 32 digit tables of 16 x 768 (512
      selector slots), selector at level 1.
  w7  the w3 tables with the threshold rule of Table II: tables of at most
      --threshold rows stay uncompressed, so the packed selector spans several
      ciphertexts (50,000: 3 ciphertexts; 500,000: 20), selector at level 4.
Other modes: --serve (continuous-batching request loop on the w3 tables: one
packed plan for all 26, or --group-size tables per plan), --dlrm (batched
end-to-end small DLRM).
A step is one helrm_lookup_packed call over one batch of selector ciphertexts
already resident in HBM; a lookup is one (query, table) embedding row.

The schedule (n1, fold radix, rotation direction, kernel tiles) comes from the
autotuner's record for this workload shape when there is one
(paper_2506_18150_amd/tuned.json), else the defaults below; --autotune
re-measures it first.  After the timed region the same steps run again with
per-kernel HIP-event timing in the library: the dominant kernel's algorithmic
bytes over its measured time give the roofline entry.  The CPU oracle is then
timed on one lookup of the same workload (cpu_baseline).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Optional

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = ["ntt_fwd_col", "ntt_fwd_blk", "ntt_inv_blk", "ntt_inv_col", "conv", "ks_acc", "baby_mac", "sub_mul",
           "baby_mfma", "baby_fold"]
BABY_CLASSES = ("baby_mac", "baby_mfma", "baby_fold")
KERNEL_SYMBOL = {
    "ntt_fwd_col": "ntt_pass_kernel<4, true, true>", "ntt_fwd_blk": "ntt_pass_kernel<4, true, false>",
    "ntt_inv_blk": "ntt_pass_kernel<4, false, false>", "ntt_inv_col": "ntt_pass_kernel<4, false, true>",
    "conv": "conv_kernel", "ks_acc": "ks_acc_kernel", "baby_mac": "baby_mac_kernel", "sub_mul": "sub_mul_kernel",
    "baby_mfma": "baby_mfma_kernel", "baby_fold": "fold_entries_kernel + baby_fold_kernel",
}
DEFAULTS = {"w2": dict(n1=16, radix=8, sign=-1, batch=1, level=23),
            "w3": dict(n1=64, radix=8, sign=-1, batch=64, level=23),
            "w6": dict(n1=32, radix=2, sign=-1, batch=1, level=1),
            "w7": dict(n1=64, radix=8, sign=-1, batch=1, level=4)}
PMC_DIR = "profiles"   # *_pmc.json: FETCH_SIZE / WRITE_SIZE records, one per kernel and workload


def kernel_source(path: str, name: str) -> str:
    """Text of the kernel `name` in `path`: from its template line to the
    brace that closes its body."""
    with open(os.path.join(ROOT, path)) as f:
        text = f.read()
    at = text.index(f" void {name}(")
    start = text.rfind("\ntemplate", 0, at)
    start = at if start < 0 or "}" in text[start:at] else start
    depth, i = 0, text.index("{", at)
    while True:
        depth += {"{": 1, "}": -1}.get(text[i], 0)
        if depth == 0:
            return text[start:i + 1]
        i += 1


def kernel_hash(rec) -> str:
    """sha256 over the kernel's own text (each kernel's, for a record of a
    kernel class) plus the shared device header."""
    import hashlib
    h = hashlib.sha256()
    for name in rec.get("kernels", [rec["kernel"]]):
        h.update(kernel_source(rec["kernel_file"], name).encode())
    for p in rec["headers"]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(symbol: str, config: dict):
    """HBM bytes per launch of kernel `symbol` from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (scaled by the copy-kernel calibration) for this
    exact workload configuration, or None when there is no such record or the
    kernel (or the device header it uses) changed since the counters were
    taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, PMC_DIR, "*_pmc.json"))):
        try:
            with open(path) as f:
                rec = json.load(f)
            if rec.get("kernel") != symbol or rec.get("config") != config:
                continue
            if kernel_hash(rec) != rec["source_sha256"]:
                return None
        except (OSError, KeyError, ValueError):
            continue
        return rec["traffic_bytes_per_launch"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="w2", choices=["w2", "w3", "w6", "w7"])
    ap.add_argument("--threshold", type=int, default=50000,
                    help="w7: tables of at most this many rows stay uncompressed (selector slots grow)")
    ap.add_argument("--level", type=int, default=None, help="selector level (default 23; 1 for w6)")
    ap.add_argument("--d", type=int, default=768, help="w6: embedding width (rows of the lookup; Table I: 768)")
    ap.add_argument("--vocab", type=int, default=0,
                    help="w6: a token-embedding table of this many rows (base-256 digits) instead of the Table I shape")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--n1", type=int, default=None)
    ap.add_argument("--radix", type=int, default=None)
    ap.add_argument("--sign", type=int, default=None, choices=[1, -1],
                    help="direction of the diagonal rotations; -1 lets the fold stop at the occupied window")
    ap.add_argument("--ks-tile", type=int, default=None)
    ap.add_argument("--baby-tile", type=int, default=None)
    ap.add_argument("--baby-share", type=int, default=None)
    ap.add_argument("--ntt-col-w", type=int, default=None, help="NTT column-pass width (8, 16; 0 = by size)")
    ap.add_argument("--ntt-blk-w", type=int, default=None, help="NTT block-pass width (4, 8; 0 = by size)")
    ap.add_argument("--ntt-small-limbs", type=int, default=None)
    ap.add_argument("--knob", action="append", default=[], metavar="NAME=VALUE",
                    help="any other library tuning knob (repeatable), e.g. conv_wgs=0")
    ap.add_argument("--autotune", action="store_true", help="measure candidate schedules first")
    ap.add_argument("--autotune-out", default=None, help="write the tuning record to this file")
    ap.add_argument("--graph", action="store_true", help="replay one captured HIP graph per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", default="0,1",
                    help="host threads of the oracle timings (0 = all; the first is cpu_baseline)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-fold", action="store_true",
                    help="do not fold the keys into plans of several giant steps (batched matrix-core product)")
    ap.add_argument("--no-extras", action="store_true",
                    help="w2 only: skip the level sweep, the batched w3 leg and the served leg")
    ap.add_argument("--batched", type=int, default=8,
                    help="also time this batch size on the same plan and keys (0 to skip)")
    ap.add_argument("--serve", action="store_true",
                    help="run the request loop (the 26 tables, Poisson arrivals) instead of the step loop")
    ap.add_argument("--rates", default="50,100,200,400", help="arrival rates (requests/s) for --serve")
    ap.add_argument("--requests", type=int, default=200, help="requests per rate for --serve")
    ap.add_argument("--group-size", type=int, default=26,
                    help="--serve: tables per packed plan (26: one plan and one ciphertext per request)")
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--streams", type=int, default=2)
    ap.add_argument("--dlrm", action="store_true",
                    help="encrypted small DLRM (8 tables of 2-200 rows, 13 dense features, bottom 13-64-16, "
                         "top 144-32-1, square activation) on a batch of requests")
    ap.add_argument("--dlrm-level", type=int, default=8, help="input level of the DLRM pass (7 levels used)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the run, copy a 1 GiB buffer 3 times (reference kernel for HBM counters)")
    return ap.parse_args()


def make_tables(workload: str, synth, planner, threshold: int = 256, d: int = 768, vocab: int = 0):
    """Seeded synthetic tables.  w2: one 65,536-row table as two base-256
    digit tables.  w3: 26 tables with log-uniform row counts (the first seed
    whose total lies in [3.0e7, 3.8e7]).  w6: the Table I shape (32 base-16
    digit tables of 16 x d), or with `vocab` a token-embedding table of that
    many rows as base-256 digit tables of 256 x d (50,257 rows: 2 digits, 512
    selector slots)."""
    g = synth.rng(0)
    if workload == "w2":
        parts = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(2)]
        return [planner.Table(rows=65536, d=16, base=256, parts=parts)]
    if workload == "w6" and vocab:
        nd = planner.n_digits(vocab, 256)
        parts = [synth.uniform_table(g, 256, d, -0.05, 0.05) for _ in range(nd)]
        return [planner.Table(rows=vocab, d=d, base=256, parts=parts)]
    if workload == "w6":
        parts = [synth.uniform_table(g, 16, d, -0.05, 0.05) for _ in range(32)]
        return [planner.Table(rows=16 ** 32, d=d, base=16, parts=parts)]
    _, counts = synth.criteo_like_row_counts()
    tables = []
    limit = threshold if workload == "w7" else 256
    for k in counts:
        if k <= limit:
            tables.append(planner.Table(rows=k, d=16, full=synth.uniform_table(g, k, 16, -0.05, 0.05)))
        else:
            nd = planner.n_digits(k, 256)
            parts = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(nd)]
            tables.append(planner.Table(rows=k, d=16, base=256, parts=parts))
    return tables


def cpu_baseline(workload: str, level: int, n1: int, radix: int, sign: int, threads=(0,), d: int = 768,
                 vocab: int = 0):
    """The CPU oracle on one selector ciphertext of the same workload (keys,
    plan encoding and encryption untimed), once per entry of `threads` (0 =
    every host thread OpenMP sees)."""
    import numpy as np

    import synth
    from oracle import oracle as O

    O.build()
    prm = O.config2_params()
    g = synth.rng(0)
    if workload == "w2":
        C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(2)]
        tables = [O.TableSpec(rows=65536, d=16, base=256, C=C)]
    elif workload == "w6" and vocab:
        C = [synth.uniform_table(g, 256, d, -0.05, 0.05) for _ in range(O.num_digits(vocab, 256))]
        tables = [O.TableSpec(rows=vocab, d=d, base=256, C=C)]
    elif workload == "w6":
        C = [synth.uniform_table(g, 16, d, -0.05, 0.05) for _ in range(32)]
        tables = [O.TableSpec(rows=16 ** 32, d=d, base=16, C=C)]
    else:
        _, counts = synth.criteo_like_row_counts()
        tables = []
        for k in counts:
            if k <= 256:
                tables.append(O.TableSpec(rows=k, d=16, E=synth.uniform_table(g, k, 16, -0.05, 0.05)))
            else:
                C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(O.num_digits(k, 256))]
                tables.append(O.TableSpec(rows=k, d=16, base=256, C=C))
    plan = O.make_plan(prm, O.pack_tables(tables), level, n1, radix, sign)
    gals = [O.galois_for_step(k, prm) for k in plan.rotation_steps()]
    print(f"cpu baseline: oracle keys for {len(gals)} rotations", file=sys.stderr, flush=True)
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals))
    qg = synth.rng(1)
    idx = synth.indices(qg, [t.rows for t in tables])
    ct = O.encrypt(prm, keys, O.encode(O.pack_selector(tables, idx), prm.delta, prm), level,
                   synth.enc_draws(qg, prm.N))
    print("cpu baseline: oracle plan residues", file=sys.stderr, flush=True)
    pts = O.plan_residues(prm, plan)
    rows = sum(t.d for t in tables)
    ref = np.concatenate([t.lookup(i) for t, i in zip(tables, idx)])
    from threadpoolctl import threadpool_limits
    res = []
    all_cores = O.max_threads()
    for nt in threads:
        nt = all_cores if nt == 0 else nt
        O.set_threads(nt)
        print(f"cpu baseline: oracle lookup on {nt} thread(s)", file=sys.stderr, flush=True)
        with threadpool_limits(limits=nt):
            t0 = time.perf_counter()
            out = O.lookup(prm, keys, plan, ct, pts)
            dt = time.perf_counter() - t0
        got = O.decode(O.decrypt(prm, keys, out), prm.delta, prm)[:rows].real
        err = float(np.max(np.abs(got - ref)))
        res.append({"value": len(tables) / dt, "unit": "lookups/s", "cores": nt, "kind": "oracle",
                    "sample": f"1 selector ciphertext ({len(tables)} lookups) of the same workload (level {level}, "
                              f"n1={n1}, radix {radix}, sign {sign}) on {nt} thread(s); {dt:.2f} s; decrypted max "
                              f"error {err:.1e}; keygen/encoding untimed"})
    O.set_threads(all_cores)
    return res


def sect8d_bytes(prm, level: int, spec, batch: int) -> dict:
    """Algorithmic HBM bytes per step of the two key-switching kernel classes,
    counted per unit as the scope table does (limb = 8 N bytes; at level l
    with pqn = l + 1 + K limbs and b' digits): a hoisted rotation reads its key
    (2 b' pqn limbs, once per batch) and its ciphertext's digits (b' pqn
    limbs); a plaintext diagonal is pqn limbs, read once per batch; each giant
    output or key-switch result is 2 pqn limbs written per ciphertext.  The
    fused baby-step kernel never writes R_b, so no per-rotation output is
    counted there.  Every word counts 8 bytes, including the halves the kernels
    regenerate from seeds or stream as 40-bit words."""
    limb = 8 * prm.N
    pqn = level + 1 + prm.K
    beta = -(-(level + 1) // prm.alpha)
    key = 2 * beta * pqn * limb
    dig = beta * pqn * limb
    out = 2 * pqn * limb
    babies = sorted({k % spec.n1 for k in spec.diag})
    giants = sorted({k // spec.n1 for k in spec.diag})
    nrot = sum(1 for b in babies if b)
    baby = nrot * (key + batch * dig) + len(spec.diag) * pqn * limb + batch * len(giants) * out
    ks = 0
    ng = sum(1 for g in giants if g)
    if ng:
        ks += ng * (key + batch * dig) + batch * out
    for _, r in spec.stages:
        ks += (r - 1) * (key + batch * dig) + batch * out
    return {"baby_mac": float(baby), "ks_acc": float(ks)}


def kernel_table(ctx, run, steps: int):
    """Per kernel class, over `steps` calls of run() with the library's event
    timing on: ms per step, launches, average launch, and the rates of the
    bytes and modular products the library counts for those launches."""
    import torch
    ctx.helrm_timing_enable(True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    kt = {k: ctx.helrm_timing_read(k) for k in KERNELS}
    ctx.helrm_timing_enable(False)
    table = {}
    for k, v in kt.items():
        if v["launches"] == 0:
            continue
        table[k] = {"ms_per_step": v["ms"] / steps, "launches_per_step": v["launches"] / steps,
                    "avg_us": 1e3 * v["ms"] / v["launches"], "GB/s": v["bytes"] / (v["ms"] * 1e6),
                    "Gmodmul/s": v["ops"] / (v["ms"] * 1e6), "bytes_per_launch": v["bytes"] / v["launches"]}
    return table, kt


def alu_peaks(ctx, prm) -> dict:
    """ALU ceilings measured by the library's calibration kernels on this GPU:
    butterflies/s of the NTT arithmetic on a 60-bit prime (integer Shoup
    butterflies) and on a 40-bit prime (fp64 exact products), and 32x32->64
    integer multiply-adds per second."""
    from paper_2506_18150_amd.binding import HELRM_CAL_BUTTERFLY, HELRM_CAL_FMA_F64, HELRM_CAL_MAD_U64
    q_wide = 0                                  # q_0: 60 bits
    q_small = 1                                 # q_1: 40 bits
    return {"butterfly_60bit_per_s": ctx.helrm_calibrate_alu(HELRM_CAL_BUTTERFLY, q_wide),
            "butterfly_40bit_per_s": ctx.helrm_calibrate_alu(HELRM_CAL_BUTTERFLY, q_small),
            "mad_u64_u32_per_s": ctx.helrm_calibrate_alu(HELRM_CAL_MAD_U64),
            "fma_f64_per_s": ctx.helrm_calibrate_alu(HELRM_CAL_FMA_F64)}


def level_sweep(prm, tables, levels, n1: int, radix: int, sign: int, key_fn, steps: int) -> dict:
    """Lookups/s at batch 1 (plain path) with the selector at other levels."""
    import numpy as np
    import torch

    import synth
    from paper_2506_18150_amd.session import LookupSession
    res = {}
    for lv in levels:
        sess = LookupSession(prm, tables, lv, n1, radix, key_fn, sign=sign)
        qg = synth.rng(1)
        idx = [synth.indices(qg, [t.rows for t in tables])]
        sel = sess.encrypt(idx, [synth.enc_draws(qg, prm.N)])
        out = sess.new_output(1)
        stream = torch.cuda.current_stream()
        sess.ctx.helrm_reserve(sess.plan, 1, stream)
        for _ in range(3):
            sess.lookup(sel, out, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            sess.lookup(sel, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        err = float(np.max(np.abs(sess.decrypt_rows(out)[0] - sess.cleartext(idx[0]))))
        res[str(lv)] = {"lookups_per_s": len(tables) / (ms / 1e3), "ms_per_lookup": ms, "max_abs_err": err}
        del sel, out
        sess.ctx.close()
    return res


def w3_batched(prm, batch: int, steps: int) -> dict:
    """The batching workload (26 tables in one selector ciphertext per query,
    level 23): batch `batch` replayed from a graph captured by the C ABI
    (helrm_batch_graph_create) against the plain path (one ciphertext per
    call, eager launches) with the same plan and keys."""
    import numpy as np
    import torch

    import synth
    from paper_2506_18150_amd import autotune, planner
    from paper_2506_18150_amd.session import LookupSession
    tables = make_tables("w3", synth, planner)
    M = planner.packed_matrix(tables)
    dflt = DEFAULTS["w3"]
    sc = autotune.tuned_schedule(prm.N, prm.L, 23, M.shape[0], M.shape[1], batch) or \
        autotune.Schedule(dflt["n1"], dflt["radix"], dflt["sign"])
    key_fn = lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals)
    t0 = time.time()
    sess = LookupSession(prm, tables, 23, sc.n1, sc.radix, key_fn, sign=sc.sign, fold=True)
    setup_s = time.time() - t0
    qg = synth.rng(5)
    idx = [synth.indices(qg, [t.rows for t in tables]) for _ in range(batch)]
    sel = sess.encrypt(idx, [synth.enc_draws(qg, prm.N) for _ in range(batch)])
    stream = torch.cuda.current_stream()
    # plain: one ciphertext per call, default knobs, eager launches
    out1 = sess.new_output(1)
    sel1 = sel[:1].contiguous()
    sess.ctx.helrm_reserve(sess.plan, 1, stream)
    for _ in range(2):
        sess.lookup(sel1, out1, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_plain = max(3, steps)
    e0.record(stream)
    for _ in range(n_plain):
        sess.lookup(sel1, out1, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / n_plain
    # batched: the tuned knobs for this batch, one captured graph per call
    for k in ("ks_tile", "baby_tile", "baby_share", "ntt_col_w", "ntt_blk_w", "baby_mfma", "baby_fold"):
        sess.ctx.helrm_set_tuning(k, getattr(sc, k))
    out = sess.new_output(batch)
    g = sess.ctx.helrm_batch_graph_create([sess.plan], sel, batch, out)
    g.replay(stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        g.replay(stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    ms = ev[0].elapsed_time(ev[-1]) / steps
    rows = sess.decrypt_rows(out)
    err = max(float(np.max(np.abs(rows[b] - sess.cleartext(idx[b])))) for b in range(batch))
    rows1 = sess.decrypt_rows(out1)
    err1 = float(np.max(np.abs(rows1[0] - sess.cleartext(idx[0]))))
    g.close()
    spec = sess.spec
    # the same batch once eagerly with every launch timed: the dominant class
    # against HBM, in the scope table's bytes and in the bytes it streams
    sess.ctx.helrm_reserve(sess.plan, batch, stream)
    table, _ = kernel_table(sess.ctx, lambda: sess.lookup(sel, out, stream), 1)
    dom = max(table, key=lambda k: table[k]["ms_per_step"])
    alg = sect8d_bytes(prm, 23, spec, batch)
    ak = "baby_mac" if dom in BABY_CLASSES else dom
    roof = {"kernel": KERNEL_SYMBOL[dom], "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "ms_per_call": table[dom]["ms_per_step"], "moved_GBps": table[dom]["GB/s"],
            "moved_bytes_per_call": table[dom]["bytes_per_launch"] * table[dom]["launches_per_step"]}
    if ak in alg:
        roof.update(achieved=alg[ak] / (table[dom]["ms_per_step"] * 1e6), algorithmic_bytes_per_call=alg[ak])
        roof["frac"] = roof["achieved"] / HBM_PEAK_GBS
    traffic = measured_traffic(KERNEL_SYMBOL[dom], dict(workload="w3", level=23, radix=spec.radix, n1=spec.n1,
                                                        batch=batch, sign=spec.sign))
    roof["traffic"] = traffic
    roof["traffic_frac"] = (traffic / (table[dom]["ms_per_step"] * 1e6) / HBM_PEAK_GBS) if traffic else None
    n_hoisted = sum(1 for b in sorted({k % spec.n1 for k in spec.diag}) if b)
    n_full = sum(1 for g_ in sorted({k // spec.n1 for k in spec.diag}) if g_) + sum(r - 1 for _, r in spec.stages)
    lk = len(tables)
    res = {
        "workload": f"w3: 26 tables (~3.4e7 rows) packed {M.shape[0]}x{M.shape[1]} in one selector ciphertext per "
                    f"query, level 23, m={spec.m}, n1={spec.n1}, n2={spec.n2}, fold radix {spec.radix}, sign "
                    f"{spec.sign}",
        "batch": batch,
        "batched": {"lookups_per_s": batch * lk / (ms / 1e3), "ms_per_call": ms,
                    "p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99)),
                    "graph": "helrm_batch_graph_create/replay", "steps": steps,
                    "knobs": {k: getattr(sc, k) for k in ("ks_tile", "baby_tile", "baby_share", "ntt_col_w",
                                                          "ntt_blk_w", "baby_mfma", "baby_fold")},
                    "key_switches_per_s": {"hoisted": n_hoisted * batch / (ms / 1e3),
                                           "full": n_full * batch / (ms / 1e3)},
                    "max_abs_err": err,
                    "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in table.items()},
                    "roofline": roof},
        "plain": {"lookups_per_s": lk / (plain_ms / 1e3), "ms_per_call": plain_ms, "steps": n_plain,
                  "max_abs_err": err1},
        "setup_s": round(setup_s, 2),
        "folded_plan_bytes": sess.folded_bytes,
    }
    res["batched_vs_plain"] = res["batched"]["lookups_per_s"] / res["plain"]["lookups_per_s"]
    del sel, out, out1, sel1
    sess.ctx.close()
    torch.cuda.synchronize()
    return res


def serving_run(level: int, rates, requests: int, group_size: int = 26, n1: Optional[int] = None, radix: int = 8,
                sign: int = -1, streams: int = 2, max_batch: int = 16, seed: int = 12, knobs=(),
                fold: bool = True) -> dict:
    """The request loop on the 26-table set: tables in fixed groups of
    group_size (26: one plan for the whole set, one ciphertext per request),
    one selector ciphertext per touched group, Poisson arrivals, each request
    touching r ~ U{1..26} distinct tables.  Selector ciphertexts wait in
    pinned host memory (a pool per group, encrypted before the run: cost is
    data-oblivious) and are copied in and out by the loop.  Compared with the
    plain per-request path: one stream, one ciphertext per call.  fold: keys
    folded into the plans of several giant steps (batches of 8 and more).
    n1 (baby steps) defaults to 64 for the one plan of all 26 tables (the
    batching workload's tuned value) and 16 for the smaller group plans."""
    import torch

    import synth
    from paper_2506_18150_amd import params, planner
    from paper_2506_18150_amd.serving import GpuExecutor, RealClock, Request, Server, Unit
    from paper_2506_18150_amd.session import GroupedDeployment

    prm = params.n16()
    tables = make_tables("w3", synth, planner)
    if n1 is None:
        n1 = 64 if group_size >= len(tables) else 16
    t0 = time.time()
    dep = GroupedDeployment(prm, tables, group_size, level, n1, radix,
                            lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals), sign=sign,
                            fold=fold and max_batch >= 8)
    for name, v in knobs:
        dep.ctx.helrm_set_tuning(name, v)
    print(f"serve: {len(dep.groups)} group plan(s) at level {level}, {dep.folded_plans} folded, "
          f"{time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    eg = synth.rng(11)
    pool = []
    for g, grp in enumerate(dep.groups):
        cts = []
        for _ in range(4):
            touched = {t: int(eg.integers(0, tables[t].rows)) for t in grp}
            cts.append(dep.encrypt_group(g, touched, synth.enc_draws(eg, prm.N)).cpu().pin_memory())
        pool.append(cts)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    total = torch.cuda.get_device_properties(0).total_memory
    static = dep.key_bytes + dep.plan_bytes + dep.folded_bytes
    # warm-up: every group at every batch size the served mode can form, so
    # that no first launch of a kernel falls inside a measured span
    wx = GpuExecutor(dep.ctx, dep.plans, level, prm.N, n_streams=1, max_batch=max_batch, static_bytes=static)
    for g in range(len(dep.groups)):
        for b in range(1, max_batch + 1):
            wx.launch(0, g, [Unit(None, g, pool[g][k % len(pool[g])], 0.0) for k in range(b)])
    torch.cuda.synchronize()
    wx.close()
    del wx
    out = {"rates": []}
    rg = synth.rng(seed)
    for rate in rates:
        arr = synth.poisson_arrivals(rg, rate, requests)
        specs = []
        for i in range(requests):
            r = int(rg.integers(1, len(tables) + 1))
            ts = rg.choice(len(tables), size=r, replace=False)
            groups = sorted({dep.group_of(int(t)) for t in ts})
            specs.append((float(arr[i]), r, [(g, pool[g][int(rg.integers(0, len(pool[g])))]) for g in groups]))
        row = {"rate": rate}
        for mode, ns, mb, mix in (("served", streams, max_batch, False), ("served_mixed", streams, max_batch, True),
                                  ("plain", 1, 1, False)):
            print(f"serve: rate {rate}, {mode}", file=sys.stderr, flush=True)
            ex = GpuExecutor(dep.ctx, dep.plans, level, prm.N, n_streams=ns, max_batch=mb, static_bytes=static)
            srv = Server(ex, RealClock(), len(dep.groups), hbm_budget=int(total * 0.9), max_batch=mb,
                         admit_timeout=30.0, mix_groups=mix)
            reqs = [Request(rid=i, arrival=a, units=u) for i, (a, _, u) in enumerate(specs)]
            rep = srv.run(reqs)
            looked = sum(specs[r.rid][1] for r in srv.completed)
            rep["lookups_per_s"] = looked / rep["span_s"] if rep["span_s"] > 0 else 0.0
            row[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in rep.items()}
            ex.close()
            del ex, srv
            torch.cuda.synchronize()
        for mode in ("served", "served_mixed"):
            row[mode + "_vs_plain"] = (row[mode]["lookups_per_s"] / row["plain"]["lookups_per_s"]
                                       if row["plain"]["lookups_per_s"] else None)
        out["rates"].append(row)
    out.update(setup_s=round(setup_s, 1), groups=len(dep.groups), level=level, group_size=group_size,
               requests=requests, n1=min(n1, max(sp.m for sp in dep.specs)), radix=radix, sign=sign,
               folded_plans=dep.folded_plans,
               resident_bytes={"keys": dep.key_bytes, "plans": dep.plan_bytes, "folded": dep.folded_bytes},
               what=(f"w5: 26 tables (w3 set) in {len(dep.groups)} groups of {group_size}, selectors at level "
                     f"{level}, Poisson arrivals, {requests} requests per rate, r ~ U{{1..26}} tables per request, "
                     f"one selector ciphertext per touched group; "
                     f"served: {streams} streams, batches of up to {max_batch} units of one group; served_mixed: the "
                     f"same with units of any groups in one launch (helrm_lookup_batch); plain: 1 stream, 1 "
                     f"ciphertext per call; latency = arrival to result on the host"))
    dep.ctx.close()
    return out


def serve_bench(args):
    """--serve: the request loop at several arrival rates (one JSON line)."""
    out = serving_run(args.level, [float(x) for x in args.rates.split(",")], args.requests, args.group_size,
                      args.n1, args.radix or 8, args.sign or -1, args.streams, args.max_batch,
                      knobs=tuple((kv.split("=")[0], int(kv.split("=")[1])) for kv in args.knob),
                      fold=not args.no_fold)
    best = max(out["rates"], key=lambda r: r["served"]["lookups_per_s"])
    res = {
        "metric": "served encrypted lookups/s",
        "value": best["served"]["lookups_per_s"],
        "unit": "lookups/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": out["what"], "level": args.level, "group_size": args.group_size},
        "latency_ms": {"p50": best["served"]["p50_ms"], "p99": best["served"]["p99_ms"]},
        "serving": out,
        "setup_s": out["setup_s"],
        "resident_bytes": out["resident_bytes"],
    }
    print(json.dumps(res))


def dlrm_bench(args):
    """Batched end-to-end small DLRM: one selector ciphertext per request
    (dense features and one-hots), the whole forward pass on the GPU per
    batch, logits decrypted and compared with the fp64 model."""
    import numpy as np
    import torch

    import synth
    from paper_2506_18150_amd import dlrm, params

    prm = params.n16()
    d = synth.small_dlrm_draws(0)
    w = dlrm.DLRMWeights(tables=d.tables, bottom=list(d.bottom), top=list(d.top), n_dense=d.n_dense)
    t0 = time.time()
    sess = dlrm.DLRMSession(prm, w, args.dlrm_level,
                            lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals, relin=True),
                            n1=args.n1 or 32, radix=args.radix or 8, sign=args.sign or -1)
    setup_s = time.time() - t0
    B = args.batch or 128
    g = synth.rng(3)
    dense = [synth.dense_features(g, d.n_dense) for _ in range(B)]
    idx = [synth.indices(g, d.table_rows) for _ in range(B)]
    sel = sess.encrypt(dense, idx, [synth.enc_draws(g, prm.N) for _ in range(B)])
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        out = sess.forward(sel, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for k in range(args.steps):
        out = sess.forward(sel, stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    logits = sess.decrypt_logits(out)
    err = float(max(abs(logits[k] - w.cleartext(dense[k], idx[k])[0]) for k in range(B)))
    res = {"metric": "encrypted DLRM inferences/s", "value": B / (ms / 1e3), "unit": "inferences/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"small DLRM: 8 tables of {min(d.table_rows)}-{max(d.table_rows)} rows x 16, 13 dense "
                                  f"features, bottom 13-64-16, top 144-32-1, square activation; N=2^16, input at level "
                                  f"{args.dlrm_level}; batch {B} requests per call",
                      "batch": B, "level": args.dlrm_level},
           "lookups_per_s": len(d.tables) * B / (ms / 1e3),
           "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
           "max_abs_err": err, "setup_s": round(setup_s, 1)}
    if not args.no_kernel_timing:
        sess.ctx.helrm_timing_enable(True)
        for _ in range(max(1, args.steps // 2)):
            sess.forward(sel, stream)
        torch.cuda.synchronize()
        n = max(1, args.steps // 2)
        table = {}
        for k in KERNELS:
            v = sess.ctx.helrm_timing_read(k)
            if v["launches"]:
                table[k] = {"ms_per_step": v["ms"] / n, "avg_us": 1e3 * v["ms"] / v["launches"],
                            "GB/s": v["bytes"] / (v["ms"] * 1e6), "bytes_per_launch": v["bytes"] / v["launches"]}
        sess.ctx.helrm_timing_enable(False)
        dom = max(table, key=lambda k: table[k]["ms_per_step"])
        symbol = dict(KERNEL_SYMBOL)
        symbol["baby_mac"] = "baby_mac_kernel|baby_mac_shared_kernel"
        res["roofline"] = {"kernel": symbol[dom], "bound": "hbm", "achieved": table[dom]["GB/s"], "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": table[dom]["GB/s"] / HBM_PEAK_GBS, "traffic": None}
        res["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in table.items()}
    print(json.dumps(res))


def hbm_copy_rate(gib: int = 2, reps: int = 5) -> dict:
    """Achievable HBM rate of a plain streaming copy on this GPU (a device-to-
    device tensor copy, read + write), as context for the 8 TB/s peak."""
    import torch
    a = torch.ones(gib << 27, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * a.numel() * 8
    del a, b
    return {"GB/s": moved / (ms * 1e6), "bytes_per_copy": moved, "frac_of_peak": moved / (ms * 1e6) / HBM_PEAK_GBS,
            "what": "device-to-device tensor copy, bytes read + written"}


def main():
    args = parse()
    if args.level is None:
        args.level = DEFAULTS[args.workload]["level"] if not (args.serve or args.dlrm) else 23
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: run with --gpus 1 (multi-GPU is not built)"}))
        sys.exit(2)
    if args.serve:
        return serve_bench(args)
    if args.dlrm:
        return dlrm_bench(args)
    import numpy as np
    import torch

    import synth
    from paper_2506_18150_amd import autotune, params, planner
    from paper_2506_18150_amd.session import LookupSession

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prm = params.n16()
    tables = make_tables(args.workload, synth, planner, args.threshold, args.d, args.vocab)
    M = planner.packed_matrix(tables)
    dflt = DEFAULTS[args.workload]
    B = args.batch or dflt["batch"]
    key_fn = lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals)
    tune_rec = None
    if args.autotune:
        eg = synth.rng(7)
        cands = None
        if args.workload == "w3":
            cands = [autotune.Schedule(n1, r, -1) for n1 in (32, 64) for r in (4, 8)]
        tune_rec = autotune.tune(prm, tables, args.level, B, key_fn, lambda: synth.enc_draws(eg, prm.N),
                                 schedules=cands, log=lambda r: print(json.dumps(r), file=sys.stderr, flush=True))
        if args.autotune_out:
            autotune.record(tune_rec, args.autotune_out)
    sched = autotune.tuned_schedule(prm.N, prm.L, args.level, M.shape[0], M.shape[1], B)
    if tune_rec is not None:
        b = tune_rec["best"]
        sched = autotune.Schedule(b["n1"], b["radix"], b["sign"], b["ks_tile"], b["baby_tile"], b["baby_share"],
                                  b["ntt_col_w"], b["ntt_blk_w"], b.get("baby_mfma", 8), b.get("baby_fold", 8))
    if sched is None:
        sched = autotune.Schedule(dflt["n1"], dflt["radix"], dflt["sign"])
    n1 = args.n1 or sched.n1
    radix = args.radix or sched.radix
    sign = args.sign or sched.sign
    t0 = time.time()
    sess = LookupSession(prm, tables, args.level, n1, radix, key_fn, sign=sign,
                         fold=not args.no_fold and max(B, args.batched or 0) >= 8)
    sess.ctx.helrm_set_tuning("ks_tile", args.ks_tile or sched.ks_tile)
    sess.ctx.helrm_set_tuning("baby_tile", args.baby_tile or sched.baby_tile)
    share = args.baby_share or sched.baby_share
    sess.ctx.helrm_set_tuning("baby_share", share)
    sess.ctx.helrm_set_tuning("baby_mfma", sched.baby_mfma)
    sess.ctx.helrm_set_tuning("baby_fold", sched.baby_fold)
    for knob, v in (("ntt_col_w", args.ntt_col_w if args.ntt_col_w is not None else sched.ntt_col_w),
                    ("ntt_blk_w", args.ntt_blk_w if args.ntt_blk_w is not None else sched.ntt_blk_w),
                    ("ntt_small_limbs", args.ntt_small_limbs)):
        if v is not None:
            sess.ctx.helrm_set_tuning(knob, v)
    extra_knobs = tuple((kv.split("=")[0], int(kv.split("=")[1])) for kv in args.knob)
    for name, v in extra_knobs:
        sess.ctx.helrm_set_tuning(name, v)
    setup_s = time.time() - t0
    qg = synth.rng(1)
    idx = [synth.indices(qg, [t.rows for t in tables]) for _ in range(B)]
    draws = lambda g_, nb: [synth.enc_draws(g_, prm.N) if sess.n_in == 1 else
                            [synth.enc_draws(g_, prm.N) for _ in range(sess.n_in)] for _ in range(nb)]
    sel = sess.encrypt(idx, draws(qg, B))
    out = sess.new_output(B)
    stream = torch.cuda.current_stream()
    sess.ctx.helrm_reserve(sess.plan, B, stream)
    for _ in range(args.warmup):
        sess.lookup(sel, out, stream)
    torch.cuda.synchronize()
    step = lambda: sess.lookup(sel, out, stream)
    if args.graph:
        cap = torch.cuda.Stream()
        sess.ctx.helrm_reserve(sess.plan, B, cap)
        cap.wait_stream(stream)
        with torch.cuda.stream(cap):
            sess.lookup(sel, out, cap)
        stream.wait_stream(cap)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=cap):
            sess.lookup(sel, out, cap)
        graph.replay()
        torch.cuda.synchronize()
        step = graph.replay
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for k in range(args.steps):
        step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    ms_per_step = ev[0].elapsed_time(ev[-1]) / args.steps
    rows = sess.decrypt_rows(out)
    err = max(float(np.max(np.abs(rows[b] - sess.cleartext(idx[b])))) for b in range(B))
    lookups_per_step = B * len(tables)
    value = lookups_per_step / (ms_per_step / 1e3)

    spec = sess.spec
    n_hoisted = sum(1 for b in sorted({k % spec.n1 for k in spec.diag}) if b)
    n_full = sum(1 for g in sorted({k // spec.n1 for k in spec.diag}) if g) + sum(r - 1 for _, r in spec.stages)
    cts_per_s = B / (ms_per_step / 1e3)
    res = {
        "metric": "encrypted lookups/s",
        "value": value,
        "unit": "lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N=2^16, L=23, dnum=3, K=8; {len(tables)} table(s), packed "
                               f"{M.shape[0]}x{M.shape[1]}"
                               + (f" in {sess.n_in} selector ciphertexts" if sess.n_in > 1 else "")
                               + (f" (a {args.vocab}-token embedding table, d={args.d}, base-256 digits)"
                                  if args.workload == "w6" and args.vocab else "")
                               + f"; selector at level {args.level}; n1={n1}, fold radix "
                               f"{radix}, rotation sign {sign} (fold span {spec.span}); batch {B} ciphertext(s) per "
                               f"call" + (", HIP graph replay" if args.graph else ""),
                   "name": args.workload, "level": args.level, "batch": B, "tables": len(tables), "n1": n1,
                   "radix": radix, "sign": sign, "fold_span": spec.span, "graph": args.graph,
                   "ks_tile": args.ks_tile or sched.ks_tile, "baby_tile": args.baby_tile or sched.baby_tile,
                   "baby_share": share, "baby_mfma": sched.baby_mfma, "baby_fold": sched.baby_fold,
                   "folded_plan_bytes": sess.folded_bytes},
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "key_switches_per_s": {"hoisted": n_hoisted * cts_per_s, "full": n_full * cts_per_s,
                               "per_ciphertext": {"hoisted": n_hoisted, "full": n_full}},
        "max_abs_err": err,
        "setup_s": round(setup_s, 2),
    }
    if tune_rec is not None:
        res["autotune"] = {"best": tune_rec["best"], "candidates": len(tune_rec["results"])}

    if args.batched and args.batched != B:
        Bb = args.batched
        bg = synth.rng(2)
        bidx = [synth.indices(bg, [t.rows for t in tables]) for _ in range(Bb)]
        bsel = sess.encrypt(bidx, draws(bg, Bb))
        bout = sess.new_output(Bb)
        sess.ctx.helrm_reserve(sess.plan, Bb, stream)
        bs = autotune.tuned_schedule(prm.N, prm.L, args.level, M.shape[0], M.shape[1], Bb)
        bb_knobs = []
        if bs is not None and (bs.n1, bs.radix, bs.sign) == (n1, radix, sign):
            bb_knobs = [("ks_tile", bs.ks_tile), ("baby_tile", bs.baby_tile), ("baby_share", bs.baby_share),
                        ("baby_mfma", bs.baby_mfma), ("baby_fold", bs.baby_fold)]
        for knob, v in bb_knobs + list(extra_knobs):
            sess.ctx.helrm_set_tuning(knob, v)
        for _ in range(2):
            sess.lookup(bsel, bout, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nb = max(3, args.steps // 4)
        e0.record(stream)
        for _ in range(nb):
            sess.lookup(bsel, bout, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1) / nb
        brows = sess.decrypt_rows(bout)
        berr = max(float(np.max(np.abs(brows[b] - sess.cleartext(bidx[b])))) for b in range(Bb))
        restore_knobs = (("ks_tile", args.ks_tile or sched.ks_tile), ("baby_tile", args.baby_tile or sched.baby_tile),
                         ("baby_share", share), ("baby_mfma", sched.baby_mfma), ("baby_fold", sched.baby_fold))
        for knob, v in restore_knobs + extra_knobs:
            sess.ctx.helrm_set_tuning(knob, v)
        res["batched"] = {"batch": Bb, "steps": nb, "ms_per_step": bms,
                          "lookups_per_s": Bb * len(tables) / (bms / 1e3), "max_abs_err": berr,
                          "vs_plain": (Bb * len(tables) / (bms / 1e3)) / value}
        if not args.no_kernel_timing:
            # the same batch once more, eagerly, with every launch timed
            for knob, v in bb_knobs + list(extra_knobs):
                sess.ctx.helrm_set_tuning(knob, v)
            bt, _ = kernel_table(sess.ctx, lambda: sess.lookup(bsel, bout, stream), 1)
            res["batched"]["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in bt.items()}
            for knob, v in restore_knobs + extra_knobs:
                sess.ctx.helrm_set_tuning(knob, v)
        del bsel, bout

    if not args.no_kernel_timing:
        table, kt = kernel_table(sess.ctx, lambda: sess.lookup(sel, out, stream), args.steps)
        dom = max(table, key=lambda k: table[k]["ms_per_step"])
        symbol = dict(KERNEL_SYMBOL)
        if B >= 2 and spec.n2 >= 2 and share >= 2:
            symbol["baby_mac"] = "baby_mac_shared_kernel"
        pmc_cfg = dict(workload=args.workload, level=args.level, radix=radix, n1=n1, batch=B, sign=sign)
        alg = sect8d_bytes(prm, args.level, spec, B) if sess.n_in == 1 else {}

        def hbm_entry(k):
            d = table[k]
            traffic = measured_traffic(symbol[k], pmc_cfg)
            ent = {"kernel": symbol[k], "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                   "avg_us": d["avg_us"], "launches_per_step": d["launches_per_step"]}
            ak = "baby_mac" if k in BABY_CLASSES else k
            if ak in alg:
                ach = alg[ak] / (d["ms_per_step"] * 1e6)
                ent.update(achieved=ach, frac=ach / HBM_PEAK_GBS,
                           algorithmic_bytes_per_launch=alg[ak] / d["launches_per_step"])
            else:
                ent.update(achieved=d["GB/s"], frac=d["GB/s"] / HBM_PEAK_GBS,
                           algorithmic_bytes_per_launch=d["bytes_per_launch"])
            ent["moved_bytes_per_launch"] = d["bytes_per_launch"]
            ent["moved_GBps"] = d["GB/s"]
            ent["traffic"] = traffic
            ent["traffic_frac"] = (traffic / (d["avg_us"] * 1e3) / HBM_PEAK_GBS) if traffic else None
            return ent

        res["roofline"] = hbm_entry(dom) if dom in BABY_CLASSES + ("ks_acc",) else {
            "kernel": symbol[dom], "bound": "alu", "note": "see roofline_ntt / roofline_conv"}
        if "ks_acc" in table:
            res["roofline_keyswitch"] = hbm_entry("ks_acc")
        peaks = alu_peaks(sess.ctx, prm)
        # butterflies of the lookup's transforms: 60-bit limbs take the integer
        # policy, 40-bit limbs the fp64 one; the launches cover the PQ basis
        # (q_0 and the K special primes wide, q_1..q_l small)
        f_wide = (1 + prm.K) / (args.level + 1 + prm.K)
        bfly_peak = 1.0 / (f_wide / peaks["butterfly_60bit_per_s"] + (1 - f_wide) / peaks["butterfly_40bit_per_s"])
        ntt_cls = [k for k in ("ntt_fwd_col", "ntt_fwd_blk", "ntt_inv_blk", "ntt_inv_col") if k in kt]
        ntt_ops = sum(kt[k]["ops"] for k in ntt_cls)
        ntt_ms = sum(kt[k]["ms"] for k in ntt_cls)
        if ntt_ms > 0:
            ach = ntt_ops / (ntt_ms * 1e-3)
            res["roofline_ntt"] = {"kernel": "ntt_pass_kernel", "bound": "alu", "unit": "Gbutterfly/s",
                                   "achieved": ach / 1e9, "peak": bfly_peak / 1e9, "frac": ach / bfly_peak,
                                   "peak_from": "helrm_calibrate_alu butterflies on a 60-bit and a 40-bit prime, "
                                                f"weighted {f_wide:.3f} / {1 - f_wide:.3f} by the PQ basis",
                                   "ms_per_step": ntt_ms / args.steps}
        if "conv" in kt and kt["conv"]["ms"] > 0:
            ach = kt["conv"]["ops"] / (kt["conv"]["ms"] * 1e-3)
            pk = peaks["mad_u64_u32_per_s"] / 4
            res["roofline_conv"] = {"kernel": "conv_kernel", "bound": "alu", "unit": "Gmodmul/s",
                                    "achieved": ach / 1e9, "peak": pk / 1e9, "frac": ach / pk,
                                    "peak_from": "helrm_calibrate_alu 32x32->64 multiply-adds / 4 per product "
                                                 "(30-bit halves)", "ms_per_step": kt["conv"]["ms"] / args.steps}
        res["alu_calibration"] = peaks
        limb_ntts = (kt["ntt_fwd_col"]["ops"] + kt["ntt_inv_blk"]["ops"]) / ((prm.N // 2) * 8) / args.steps
        res["ntts_per_s"] = limb_ntts * (1e3 / ms_per_step)
        res["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in table.items()}
        res["hbm_copy"] = hbm_copy_rate()

    if args.calibrate_copy:
        a = torch.zeros(1 << 27, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = 1 << 30

    default_run = args.workload == "w2" and not args.no_extras
    if default_run:
        sess.ctx.close()
        del sel, out
        torch.cuda.synchronize()
        res["level_sweep"] = level_sweep(prm, tables, [4, 1], n1, radix, sign, key_fn, max(10, args.steps))
        res["level_sweep"]["23"] = {"lookups_per_s": value, "ms_per_lookup": ms_per_step, "max_abs_err": err}
        res["batched_w3"] = w3_batched(prm, 64, 3)
        srv = serving_run(23, [400.0], 240)
        row = srv["rates"][0]
        keep = ("lookups_per_s", "p50_ms", "p99_ms", "mean_batch", "completed", "rejected", "span_s")
        res["served"] = {"rate_per_s": row["rate"], "requests": srv["requests"],
                         **{m: {k: row[m].get(k) for k in keep} for m in ("served", "served_mixed", "plain")},
                         "served_vs_plain": row["served_vs_plain"],
                         "served_mixed_vs_plain": row["served_mixed_vs_plain"], "what": srv["what"]}
    if not args.no_cpu_baseline and args.workload != "w7":
        cb = cpu_baseline(args.workload, args.level, n1, radix, sign,
                          threads=tuple(int(x) for x in args.cpu_threads.split(",")), d=args.d, vocab=args.vocab)
        res["cpu_baseline"] = cb[0]
        if len(cb) > 1:
            res["cpu_baseline_" + ("single_thread" if cb[1]["cores"] == 1 else "threads_%d" % cb[1]["cores"])] = cb[1]
    print(json.dumps(res))


if __name__ == "__main__":
    main()
