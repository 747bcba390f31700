"""Batched fitness (one persistent launch per phase, HIP-graph replay) and the
autotuner, checked against the plain per-population path through the C ABI."""
import os

import numpy as np
import pytest

import oracle
from paper_2103_07512_amd import popgen as pg

import _parity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_07512_amd import tgp
    assert torch.cuda.is_available()
    return tgp, tgp.Context(0), torch


def small_c4(seed, n):
    """A reduced copy of the 64-population workload: same recipe, smaller sizes."""
    rng = pg.Rng(seed)
    out = []
    for p in range(n):
        size = 5 + rng.below(60)
        d_max = 3 + rng.below(8)
        if rng.below(6) == 0:
            shape = (9, 10, 11)
        else:
            shape = (rng.below(70) + 1, rng.below(90) + 1)
        pop = pg.ramped_half_and_half(size, 2, d_max, seed * 100 + p, pg.F18, len(shape))
        out.append((pop, shape, pg.TargetSpec(3, seed * 100 + 50 + p, pg.F18, len(shape), 1)))
    return out


def make_jobs(env, work, loss=0):
    tgp, ctx, torch = env
    jobs, keep = [], []
    for pop, shape, spec in work:
        dom = tgp.Domain(ctx, shape)
        dag = tgp.build_dag(ctx, pop)
        _, target = pg.pick_target(spec, oracle.target_renderer(shape))
        t = torch.from_numpy(target).to("cuda:0")
        out = torch.full((pop.n_individuals,), -1.0, dtype=torch.float64, device="cuda:0")
        jobs.append((dag, dom, t, loss, out))
    return jobs


def plain(env, jobs):
    tgp, ctx, torch = env
    res = []
    for dag, dom, t, loss, _ in jobs:
        o = torch.empty(dag.n_individuals, dtype=torch.float64, device="cuda:0")
        tgp.fitness(ctx, dag, dom, t, loss, o)
        res.append(o)
    torch.cuda.synchronize()
    return [r.cpu().numpy() for r in res]


def same(a, b, rtol):
    a, b = np.asarray(a), np.asarray(b)
    assert np.array_equal(np.isinf(a), np.isinf(b))
    f = np.isfinite(a)
    np.testing.assert_allclose(a[f], b[f], rtol=rtol, atol=0)


def test_batch_equals_plain_bitwise(env):
    tgp, ctx, torch = env
    work = small_c4(3, 12)
    say("batch of", len(work), "jobs, 1 tile per item")
    jobs = make_jobs(env, work)
    ctx.set_tuning(4, 1)
    try:
        want = plain(env, jobs)
        b = tgp.Batch(ctx, use_graph=True)
        b.run(jobs)
        torch.cuda.synchronize()
        for (dag, _, _, _, out), w in zip(jobs, want):
            got = out.cpu().numpy()
            assert np.array_equal(got.view(np.uint64), w.view(np.uint64))
        st = b.stats()
        say(st)
        assert st["captures"] == 1 and st["jobs"] == 12
    finally:
        ctx.set_tuning(0, 0)


def test_batch_plans_fresh_dags(env):
    """A batch of fresh DAGs plans them all at once (host threads, one
    constant-folding round trip for the whole batch); plain calls on the same
    DAGs afterwards reuse or redo those plans and give bitwise the same
    fitness.  One DAG is listed twice, on two domain sizes."""
    tgp, ctx, torch = env
    work = small_c4(13, 10)
    jobs = make_jobs(env, work)
    pop0, shape0, spec0 = work[0]
    shape2 = (3, 4) if len(shape0) == 2 else (2, 3, 4)
    dom2 = tgp.Domain(ctx, shape2)
    _, target2 = pg.pick_target(pg.TargetSpec(3, 1313, pg.F18, len(shape2), 1),
                                oracle.target_renderer(shape2))
    out2 = torch.full((pop0.n_individuals,), -1.0, dtype=torch.float64, device="cuda:0")
    jobs.append((jobs[0][0], dom2, torch.from_numpy(target2).to("cuda:0"), 0, out2))
    folded = sum(1 for p, _, _ in work for t in p.tokens if t["op"] == 1)
    say("batch of", len(jobs), "fresh jobs;", folded, "constant tokens")
    ctx.set_tuning(4, 1)
    try:
        b = tgp.Batch(ctx, use_graph=True)
        b.run(jobs)
        torch.cuda.synchronize()
        got = [o.cpu().numpy().copy() for *_, o in jobs]
        want = plain(env, jobs)
        for g, w in zip(got, want):
            assert np.array_equal(g.view(np.uint64), w.view(np.uint64))
    finally:
        ctx.set_tuning(0, 0)


def test_batch_graph_replay_with_new_jobs(env):
    tgp, ctx, torch = env
    b = tgp.Batch(ctx, use_graph=True)
    big = make_jobs(env, small_c4(5, 10))
    small = make_jobs(env, small_c4(7, 4))
    say("replay: 10 jobs then 4 jobs then 10 again")
    b.run(big)
    b.run(small)
    b.run(big)
    torch.cuda.synchronize()
    st = b.stats()
    assert st["captures"] == 1 and st["replays"] == 3, st
    for jobs in (big, small):
        want = plain(env, jobs)
        for (dag, _, _, _, out), w in zip(jobs, want):
            same(out.cpu().numpy(), w, 1e-6)


def test_batch_without_graph_and_mse(env):
    tgp, ctx, torch = env
    jobs = make_jobs(env, small_c4(9, 6), loss=1)
    b = tgp.Batch(ctx, use_graph=False)
    b.run(jobs)
    torch.cuda.synchronize()
    assert b.stats()["captures"] == 0
    want = plain(env, jobs)
    for (dag, _, _, _, out), w in zip(jobs, want):
        same(out.cpu().numpy(), w, 1e-6)


def test_fitness_batch_against_oracle(env):
    """One batch job checked directly against the oracle's FP64 fitness."""
    tgp, ctx, torch = env
    work = small_c4(11, 3)
    jobs = make_jobs(env, work)
    tgp.fitness_batch(ctx, jobs)
    torch.cuda.synchronize()
    for (pop, shape, spec), (dag, dom, t, loss, out) in zip(work, jobs):
        _, target = pg.pick_target(spec, oracle.target_renderer(shape))
        v64, v32, st, eb = oracle.evaluate(pop.tokens, pop.offsets, shape, bound=True)
        vals = torch.empty(pop.n_roots, dom.cases, dtype=torch.float32, device="cuda:0")
        tgp.evaluate(ctx, dag, dom, vals)
        vals = vals.cpu().numpy()
        _parity.check_cases(vals, v64, v32, st, eb, f"batch job {shape}")
        r = _parity.check_fitness(out.cpu().numpy(), vals, v64, st, eb, target, pop.n_individuals, 1, "rmse",
                                  f"batch job {shape}")
        say(shape, r)


def test_batch_lds_stack(env):
    """Batched steps with the LDS stack agree with the register form."""
    tgp, ctx, torch = env
    jobs = make_jobs(env, small_c4(17, 6))
    want = plain(env, jobs)
    try:
        ctx.set_stack(True)
        b = tgp.Batch(ctx, use_graph=True)
        b.run(jobs)
        torch.cuda.synchronize()
        st = b.stats()
        assert st["cases_per_lane"] == 2
        for (dag, _, _, _, out), w in zip(jobs, want):
            same(out.cpu().numpy(), w, 1e-6)
    finally:
        ctx.set_stack(False)


def test_autotune_and_cache(env, tmp_path):
    tgp, ctx, torch = env
    jobs = make_jobs(env, small_c4(13, 5))
    path = str(tmp_path / "tune.jsonl")
    say("autotune")
    r1 = tgp.autotune(ctx, jobs, path)
    say(r1)
    assert r1["cases_per_lane"] in (2, 4) and r1["tiles_cap"] in (4, 8, 16, 32)
    assert r1["from_cache"] == 0 and r1["candidates"] == 12 and r1["stack_lds"] in (0, 1)
    r2 = tgp.autotune(ctx, jobs, path)
    assert r2["from_cache"] == 1 and (r2["cases_per_lane"], r2["tiles_cap"], r2["stack_lds"]) == \
        (r1["cases_per_lane"], r1["tiles_cap"], r1["stack_lds"])
    assert os.path.getsize(path) > 0
    # results under the tuned shape still match the plain path within the fitness tolerance
    tgp.fitness_batch(ctx, jobs)
    torch.cuda.synchronize()
    ctx.set_tuning(0, 0)
    ctx.set_stack(False)
    want = plain(env, jobs)
    for (dag, _, _, _, out), w in zip(jobs, want):
        same(out.cpu().numpy(), w, 1e-6)
