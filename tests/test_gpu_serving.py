"""The request loop on the GPU: requests of different table counts arriving
together are batched across requests on two streams, and every result is
bit-identical to the same ciphertext processed alone, and decrypts to the
cleartext rows."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_the_mix():
    import torch
    from paper_2506_18150_amd import params, planner
    from paper_2506_18150_amd.serving import GpuExecutor, RealClock, Request, Server
    from paper_2506_18150_amd.session import GroupedDeployment
    from tests.gpu_helpers import say

    prm = params.n16()
    g = synth.rng(3)
    tables = []
    for k in (70000, 200, 5000, 12, 300000, 90):
        if k <= 256:
            tables.append(planner.Table(rows=k, d=16, full=synth.uniform_table(g, k, 16, -0.05, 0.05)))
        else:
            parts = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(planner.n_digits(k, 256))]
            tables.append(planner.Table(rows=k, d=16, base=256, parts=parts))
    level = 1
    say("serving: deployment of 6 tables in 3 groups at level 1")
    dep = GroupedDeployment(prm, tables, 2, level, 16, 8,
                            lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals))
    rg = synth.rng(4)
    reqs, touched_of = [], {}
    for rid in range(12):
        r = int(rg.integers(1, len(tables) + 1))
        ts = sorted(rg.choice(len(tables), size=r, replace=False).tolist())
        touched = {t: int(rg.integers(0, tables[t].rows)) for t in ts}
        groups = sorted({dep.group_of(t) for t in ts})
        units = []
        for gg in groups:
            ct = dep.encrypt_group(gg, touched, synth.enc_draws(rg, prm.N)).cpu().pin_memory()
            units.append((gg, ct))
        reqs.append(Request(rid=rid, arrival=0.0005 * rid, units=units))
        touched_of[rid] = touched
    torch.cuda.synchronize()
    ex = GpuExecutor(dep.ctx, dep.plans, level, prm.N, n_streams=2, max_batch=4)
    srv = Server(ex, RealClock(), len(dep.groups), hbm_budget=200 << 30, max_batch=4)
    say("serving: 12 requests through the loop")
    rep = srv.run(reqs)
    assert rep["completed"] == 12 and rep["rejected"] == 0
    assert max(srv.batch_sizes) > 1
    out = torch.zeros(1, 2, level, prm.N, dtype=torch.int64, device="cuda")
    say("serving: each unit alone")
    for r in reqs:
        for gg, ct in r.units:
            dep.ctx.helrm_lookup_packed(dep.plans[gg], ct.cuda()[None].contiguous(), 1, out)
            torch.cuda.synchronize()
            alone = out.cpu().reshape(-1)
            assert torch.equal(alone, r.results[gg].reshape(-1)), f"request {r.rid} group {gg}"
            got = dep.decrypt_group(gg, r.results[gg].cuda())
            want = dep.cleartext_group(gg, touched_of[r.rid])
            assert np.max(np.abs(got - want)) < 1e-4
    say("serving: executor closed (workspaces released); a new one with mixed groups serves the requests again")
    ex.close()
    ex2 = GpuExecutor(dep.ctx, dep.plans, level, prm.N, n_streams=2, max_batch=4)
    srv2 = Server(ex2, RealClock(), len(dep.groups), hbm_budget=200 << 30, max_batch=4, mix_groups=True)
    # fresh requests with the original relative arrival times (a run turns
    # each request's arrival into an absolute clock time)
    reqs2 = [Request(rid=r.rid, arrival=0.0005 * r.rid, units=r.units) for r in reqs]
    rep2 = srv2.run(reqs2)
    assert rep2["completed"] == 12
    for r, r2 in zip(reqs, reqs2):
        for gg, _ in r.units:
            assert torch.equal(r2.results[gg].reshape(-1), r.results[gg].reshape(-1)), f"request {r.rid} group {gg}"
    ex2.close()


def test_one_plan_for_all_tables_folded():
    """One packed plan for every table (one selector ciphertext per request)
    with its keys folded: 20 requests arriving together are served in batches
    of up to 12, so the matrix-core folded product runs, and every result is
    bit-identical to the same ciphertext processed alone (batch 1, VALU
    kernels) and decrypts to the cleartext rows."""
    import torch
    from paper_2506_18150_amd import params, planner
    from paper_2506_18150_amd.serving import GpuExecutor, RealClock, Request, Server
    from paper_2506_18150_amd.session import GroupedDeployment
    from tests.gpu_helpers import say

    prm = params.n16()
    g = synth.rng(5)
    tables = []
    for k in (70000, 200, 5000, 12, 300000, 90):
        if k <= 256:
            tables.append(planner.Table(rows=k, d=16, full=synth.uniform_table(g, k, 16, -0.05, 0.05)))
        else:
            parts = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(planner.n_digits(k, 256))]
            tables.append(planner.Table(rows=k, d=16, base=256, parts=parts))
    level = 1
    say("serving: one folded plan for 6 tables at level 1")
    dep = GroupedDeployment(prm, tables, len(tables), level, 16, 8,
                            lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals), fold=True)
    assert len(dep.groups) == 1 and dep.specs[0].n2 >= 2 and dep.folded_plans == 1
    rg = synth.rng(6)
    reqs, touched_of = [], {}
    for rid in range(20):
        r = int(rg.integers(1, len(tables) + 1))
        ts = sorted(rg.choice(len(tables), size=r, replace=False).tolist())
        touched = {t: int(rg.integers(0, tables[t].rows)) for t in ts}
        ct = dep.encrypt_group(0, touched, synth.enc_draws(rg, prm.N)).cpu().pin_memory()
        reqs.append(Request(rid=rid, arrival=0.0, units=[(0, ct)]))
        touched_of[rid] = touched
    torch.cuda.synchronize()
    ex = GpuExecutor(dep.ctx, dep.plans, level, prm.N, n_streams=2, max_batch=12)
    srv = Server(ex, RealClock(), 1, hbm_budget=200 << 30, max_batch=12)
    say("serving: 20 requests through the loop")
    rep = srv.run(reqs)
    assert rep["completed"] == 20 and rep["rejected"] == 0
    assert max(srv.batch_sizes) >= 8
    out = torch.zeros(1, 2, level, prm.N, dtype=torch.int64, device="cuda")
    say("serving: each request alone")
    for r in reqs:
        ct = r.units[0][1]
        dep.ctx.helrm_lookup_packed(dep.plans[0], ct.cuda()[None].contiguous(), 1, out)
        torch.cuda.synchronize()
        assert torch.equal(out.cpu().reshape(-1), r.results[0].reshape(-1)), f"request {r.rid}"
        got = dep.decrypt_group(0, r.results[0].cuda())
        want = dep.cleartext_group(0, touched_of[r.rid])
        assert np.max(np.abs(got - want)) < 1e-4
    ex.close()
    dep.ctx.close()
