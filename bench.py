#!/usr/bin/env python3
"""Benchmark: encrypted packed embedding lookups on one MI355X.

Default workload ("w2"): N = 2^16, 24 ciphertext primes (60 + 23 x 40 bits),
dnum = 3 with 8 special 60-bit primes; one 65,536-row x 16 table stored as two
256 x 16 digit tables (base 256, values U[-0.05, 0.05]); one selector
ciphertext per call at level 23; double-hoisted BSGS (n1 = 16 baby steps)
with a fold of the given radix, then rescale.  A step is one
helrm_lookup_packed call over one batch of selector ciphertexts already
resident in HBM.  Inputs are seeded synthetic data of the paper's shapes.

After the timed region the same steps run again with per-kernel HIP-event
timing enabled in the library; the dominant kernel's algorithmic bytes over
its measured time give the roofline entry.  The CPU oracle is then timed on
one lookup of the same workload (cpu_baseline).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = ["ntt_fwd_col", "ntt_fwd_blk", "ntt_inv_blk", "ntt_inv_col", "conv", "ks_acc", "baby_mac", "sub_mul"]
KERNEL_SYMBOL = {
    "ntt_fwd_col": "ntt_pass_kernel<4, true, true>", "ntt_fwd_blk": "ntt_pass_kernel<4, true, false>",
    "ntt_inv_blk": "ntt_pass_kernel<4, false, false>", "ntt_inv_col": "ntt_pass_kernel<4, false, true>",
    "conv": "conv_kernel", "ks_acc": "ks_acc_kernel", "baby_mac": "baby_mac_kernel", "sub_mul": "sub_mul_kernel",
}


PMC_PROFILES = {"ks_acc": "profiles/ks_acc_kernel_w2_level23_radix8_pmc.json"}


def measured_traffic(kernel: str, level: int, radix: int, n1: int, batch: int, sign: int):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE counter
    runs (scaled by the copy-kernel calibration), or None when there is no
    such record for this kernel and workload or the kernel source changed
    since the counters were taken."""
    import hashlib
    path = PMC_PROFILES.get(kernel)
    if not path or (level, radix, n1, batch, sign) != (23, 8, 16, 1, 1):
        return None
    try:
        with open(os.path.join(ROOT, path)) as f:
            rec = json.load(f)
        src = b"".join(open(os.path.join(ROOT, p), "rb").read() for p in rec["source_files"])
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=23)
    ap.add_argument("--n1", type=int, default=16)
    ap.add_argument("--radix", type=int, default=8)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--sign", type=int, default=-1, choices=[1, -1],
                    help="direction of the diagonal rotations; -1 lets the fold stop at the occupied window")
    ap.add_argument("--graph", action="store_true", help="replay one captured HIP graph per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the run, copy a 1 GiB buffer 3 times (reference kernel for HBM counters)")
    return ap.parse_args()


def w2_tables(synth, planner):
    g = synth.rng(0)
    parts = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(2)]
    return [planner.Table(rows=65536, d=16, base=256, parts=parts)]


def cpu_baseline(level: int, n1: int, radix: int, sign: int):
    """The CPU oracle on one lookup of the same workload (keys, plan encoding
    and encryption untimed)."""
    import numpy as np

    import synth
    from oracle import oracle as O

    O.build()
    prm = O.config2_params()
    g = synth.rng(0)
    C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(2)]
    t = O.TableSpec(rows=65536, d=16, base=256, C=C)
    plan = O.make_plan(prm, O.pack_tables([t]), level, n1, radix, sign)
    gals = [O.galois_for_step(k, prm) for k in plan.rotation_steps()]
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals))
    qg = synth.rng(1)
    idx = synth.indices(qg, [t.rows])
    ct = O.encrypt(prm, keys, O.encode(O.pack_selector([t], idx), prm.delta, prm), level,
                   synth.enc_draws(qg, prm.N))
    pts = O.plan_residues(prm, plan)
    t0 = time.perf_counter()
    out = O.lookup(prm, keys, plan, ct, pts)
    dt = time.perf_counter() - t0
    got = O.decode(O.decrypt(prm, keys, out), prm.delta, prm)[:16].real
    err = float(np.max(np.abs(got - t.lookup(idx[0]))))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / dt, "unit": "lookups/s", "cores": cores, "kind": "oracle",
            "sample": f"1 lookup of the same workload (level {level}, n1={n1}, radix {radix}, sign {sign}); "
                      f"{dt:.2f} s; decrypted max error {err:.1e}; keygen/encoding untimed"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: run with --gpus 1 (multi-GPU is not built)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2506_18150_amd import params, planner
    from paper_2506_18150_amd.session import LookupSession

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prm = params.n16()
    tables = w2_tables(synth, planner)
    t0 = time.time()
    sess = LookupSession(prm, tables, args.level, args.n1, args.radix,
                         lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals), sign=args.sign)
    setup_s = time.time() - t0
    B = args.batch
    qg = synth.rng(1)
    idx = [synth.indices(qg, [t.rows for t in tables]) for _ in range(B)]
    sel = sess.encrypt(idx, [synth.enc_draws(qg, prm.N) for _ in range(B)])
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

    # key switches per lookup: hoisted (baby steps) and full (giant steps + fold)
    spec = sess.spec
    n_hoisted = sum(1 for b in sorted({k % spec.n1 for k in spec.diag}) if b)
    n_full = sum(1 for g in sorted({k // spec.n1 for k in spec.diag}) if g) + sum(r - 1 for _, r in spec.stages)
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
        "config": {"workload": f"w2: N=2^16, L=23, dnum=3, K=8; 1 table 65536x16 as 2 base-256 digit tables; "
                               f"selector at level {args.level}; n1={args.n1}, fold radix {args.radix}, "
                               f"rotation sign {args.sign} (fold span {sess.spec.span}); "
                               f"batch {B} ciphertext(s) per call" + (", HIP graph replay" if args.graph else ""),
                   "level": args.level, "batch": B, "n1": args.n1, "radix": args.radix, "sign": args.sign,
                   "fold_span": sess.spec.span, "graph": args.graph},
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "key_switches_per_s": {"hoisted": n_hoisted * value, "full": n_full * value,
                               "per_lookup": {"hoisted": n_hoisted, "full": n_full}},
        "max_abs_err": err,
        "setup_s": round(setup_s, 2),
    }

    if not args.no_kernel_timing:
        sess.ctx.helrm_timing_enable(True)
        for _ in range(args.steps):
            sess.lookup(sel, out, stream)
        torch.cuda.synchronize()
        kt = {k: sess.ctx.helrm_timing_read(k) for k in KERNELS}
        sess.ctx.helrm_timing_enable(False)
        table = {}
        for k, v in kt.items():
            if v["launches"] == 0:
                continue
            table[k] = {"ms_per_step": v["ms"] / args.steps, "launches_per_step": v["launches"] / args.steps,
                        "avg_us": 1e3 * v["ms"] / v["launches"], "GB/s": v["bytes"] / (v["ms"] * 1e6),
                        "Gmodmul/s": v["ops"] / (v["ms"] * 1e6), "bytes_per_launch": v["bytes"] / v["launches"]}
        dom = max(table, key=lambda k: table[k]["ms_per_step"])
        d = table[dom]
        res["roofline"] = {"kernel": KERNEL_SYMBOL[dom], "bound": "hbm", "achieved": d["GB/s"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["GB/s"] / HBM_PEAK_GBS,
                           "traffic": measured_traffic(dom, args.level, args.radix, args.n1, B, args.sign),
                           "avg_us": d["avg_us"], "algorithmic_bytes_per_launch": d["bytes_per_launch"]}
        ks = table.get("ks_acc")
        if ks:
            res["roofline_keyswitch"] = {"kernel": KERNEL_SYMBOL["ks_acc"], "bound": "hbm",
                                         "achieved": ks["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": ks["GB/s"] / HBM_PEAK_GBS, "avg_us": ks["avg_us"]}
        limb_ntts = (kt["ntt_fwd_col"]["ops"] + kt["ntt_inv_blk"]["ops"]) / ((prm.N // 2) * 8) / args.steps
        res["ntts_per_s"] = limb_ntts * (1e3 / ms_per_step)
        res["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in table.items()}

    if args.calibrate_copy:
        a = torch.zeros(1 << 27, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = 1 << 30

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.level, args.n1, args.radix, args.sign)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
