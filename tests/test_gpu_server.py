"""The serving form (tgp_server_*): continuous batching of many requests,
admission against the subtree-cache budget and reuse of resident subtrees,
checked through the C ABI against the plain per-population path and the
oracle."""
import threading

import numpy as np
import pytest

import oracle
from paper_2103_07512_amd import popgen as pg

from _parity import check_fitness

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_07512_amd import tgp
    assert torch.cuda.is_available()
    return tgp, tgp.Context(0), torch


class Work:
    """One request: a population, its domain and target on the device."""

    def __init__(self, env, pop, shape, spec, loss=0):
        tgp, ctx, torch = env
        self.pop, self.shape, self.loss = pop, shape, loss
        self.dom = tgp.Domain(ctx, shape)
        _, tgt = pg.pick_target(spec, oracle.target_renderer(shape))
        self.target_host = tgt
        self.target = torch.from_numpy(np.ascontiguousarray(tgt)).to("cuda:0")

    def values(self, env):
        """Per-case values of the plain evaluate path (the same device
        operator code the served fitness runs)."""
        tgp, ctx, torch = env
        dag = tgp.build_dag(ctx, self.pop)
        v = torch.empty(self.pop.n_roots, self.dom.cases, dtype=torch.float32, device="cuda:0")
        tgp.evaluate(ctx, dag, self.dom, v)
        torch.cuda.synchronize()
        return v.cpu().numpy()

    def plain(self, env):
        tgp, ctx, torch = env
        dag = tgp.build_dag(ctx, self.pop)
        o = torch.empty(self.pop.n_individuals, dtype=torch.float64, device="cuda:0")
        tgp.fitness(ctx, dag, self.dom, self.target, self.loss, o)
        torch.cuda.synchronize()
        return o.cpu().numpy()


def mixed_work(env, seed):
    """Requests of uneven sizes, domain shapes, channels and losses."""
    out = []
    specs = [(40, 2, 6, (64, 64), 1, 0), (120, 2, 8, (256, 256), 1, 0), (30, 3, 7, (20, 30, 40), 1, 0),
             (60, 2, 9, (512, 512), 1, 0), (25, 2, 6, (128, 96), 3, 1), (200, 2, 10, (32, 32), 1, 0)]
    # the last one uses the interpreter with the bitwise operators and warp
    funcs = [pg.F18] * 5 + [pg.F18 + ("or", "xor", "and", "warp")]
    for i, (n, dmin, dmax, shape, ch, loss) in enumerate(specs):
        pop = pg.ramped_half_and_half(n, dmin, dmax, seed * 10 + i, funcs[i], len(shape), n_channels=ch)
        spec = pg.TargetSpec(4, seed * 10 + 5 + i, pg.F18, len(shape), ch)
        out.append(Work(env, pop, shape, spec, loss))
    return out


def bits(a):
    return np.asarray(a, np.float64).view(np.uint64)


def close(a, b, rtol=1e-6):
    a, b = np.asarray(a), np.asarray(b)
    assert np.array_equal(np.isinf(a), np.isinf(b))
    f = np.isfinite(a)
    np.testing.assert_allclose(a[f], b[f], rtol=rtol, atol=0)


def serve_alone(env, works, slab_work, budget=1 << 30):
    tgp, ctx, torch = env
    res = []
    for w in works:
        srv = tgp.Server(ctx, budget, 4)
        srv.set_slab_work(slab_work)
        t = srv.submit(0, w.pop, w.dom, w.target, w.loss)
        res.append(srv.wait(t).copy())
        srv.close()
    return res


def test_alone_and_in_the_mix_are_identical(env):
    """Each result is bitwise the same served alone and served together with
    the others (several slabs per request, requests joining mid-flight)."""
    tgp, ctx, torch = env
    works = mixed_work(env, 1)
    slab = float(1 << 21)  # small slabs: the larger requests take several steps
    say("alone")
    alone = serve_alone(env, works, slab)
    say("mix")
    srv = tgp.Server(ctx, 1 << 30, 8)
    srv.set_slab_work(slab)
    tickets = [srv.submit(i, w.pop, w.dom, w.target, w.loss) for i, w in enumerate(works)]
    mix = [srv.wait(t).copy() for t in tickets]
    infos = [srv.ticket_info(t) for t in tickets]
    st = srv.stats()
    say(st)
    srv.close()
    assert max(i["slabs"] for i in infos) > 1
    assert st["max_active_seen"] > 1 and st["completed"] == len(works)
    for w, a, m, info in zip(works, alone, mix, infos):
        assert np.array_equal(bits(a), bits(m)), (w.shape, info)
    # and the plain launch agrees within the fitness tolerance
    for w, a in zip(works, alone):
        close(a, w.plain(env))


def test_served_against_oracle(env):
    tgp, ctx, torch = env
    srv = tgp.Server(ctx, 1 << 28, 4)
    srv.set_slab_work(float(1 << 16))  # several slabs even on the small grids
    cases = []
    for i, shape in enumerate([(64, 64), (33, 47), (9, 10, 11), (40, 24)]):
        funcs = pg.F18 if i < 3 else pg.F18 + ("warp", "or", "xor", "and")
        pop = pg.ramped_half_and_half(30, 2, 7, 300 + i, funcs, len(shape))
        w = Work(env, pop, shape, pg.TargetSpec(3, 310 + i, pg.F18, len(shape), 1))
        cases.append((w, srv.submit(i, pop, w.dom, w.target, 0)))
    for w, t in cases:
        got = srv.wait(t)
        say(w.shape, srv.ticket_info(t))
        v64, v32, stab, eb = oracle.evaluate(w.pop.tokens, w.pop.offsets, w.shape, bound=True)
        check_fitness(got, w.values(env), v64, stab, eb, w.target_host, w.pop.n_individuals, 1, "rmse",
                      f"served {w.shape}")
    srv.close()


def test_resident_subtrees_are_reused(env):
    """A later generation that shares subtrees reads them from the cache and
    gets the same values as computing them."""
    tgp, ctx, torch = env
    shape = (256, 256)
    pop = pg.ramped_half_and_half(200, 2, 8, 77, pg.F18, 2)
    w = Work(env, pop, shape, pg.TargetSpec(4, 78, pg.F18, 2, 1))
    srv = tgp.Server(ctx, 1 << 30, 4)
    t1 = srv.submit(5, pop, w.dom, w.target, 0)
    f1 = srv.wait(t1).copy()
    t2 = srv.submit(5, pop, w.dom, w.target, 0)
    f2 = srv.wait(t2).copy()
    i1, i2 = srv.ticket_info(t1), srv.ticket_info(t2)
    say(i1, i2, srv.stats())
    assert i1["cache_new"] > 0 and i1["cache_hits"] == 0
    assert i2["cache_hits"] >= i1["cache_new"] and i2["cache_new"] == 0
    assert np.array_equal(bits(f1), bits(f2))
    # a bred next generation also hits part of the cache
    child = pg.breed(pop, pg.Rng(79), pg.F18, 2, max_depth=10, fitness=f1)
    t3 = srv.submit(5, child, w.dom, w.target, 0)
    f3 = srv.wait(t3).copy()
    i3 = srv.ticket_info(t3)
    say(i3)
    close(f3, _plain_of(env, child, w))
    before = srv.stats()["entries"]
    srv.end_run(5)
    after = srv.stats()["entries"]
    assert before > 0 and after == 0
    srv.close()


def _plain_of(env, pop, w):
    tgp, ctx, torch = env
    dag = tgp.build_dag(ctx, pop)
    o = torch.empty(pop.n_individuals, dtype=torch.float64, device="cuda:0")
    tgp.fitness(ctx, dag, w.dom, w.target, w.loss, o)
    torch.cuda.synchronize()
    return o.cpu().numpy()


def test_admission_under_a_small_cache(env):
    """Requests whose cached subtrees do not fit together wait for memory and
    still finish with the right values; one that can never fit fails."""
    tgp, ctx, torch = env
    shape = (256, 256)
    works = []
    for i in range(5):
        pop = pg.ramped_half_and_half(150, 2, 9, 400 + i, pg.F18, 2)
        works.append(Work(env, pop, shape, pg.TargetSpec(4, 420 + i, pg.F18, 2, 1)))
    need = []
    probe = tgp.Server(ctx, 1 << 30, 1)
    for w in works:
        t = probe.submit(0, w.pop, w.dom, w.target, 0)
        probe.wait(t)
        need.append(probe.ticket_info(t)["cache_new"] + probe.ticket_info(t)["cache_hits"])
        probe.end_run(0)
    probe.close()
    row = 256 * 256 * 4
    budget = (max(need) + 2) * row  # room for about one request at a time
    say("slots per request", need, "budget rows", budget // row)
    srv = tgp.Server(ctx, budget, 8)
    results = {}

    def run(i, w):
        t = srv.submit(100 + i, w.pop, w.dom, w.target, 0)
        results[i] = srv.wait(t).copy()

    th = [threading.Thread(target=run, args=(i, w)) for i, w in enumerate(works)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    st = srv.stats()
    say(st)
    assert st["completed"] == len(works) and st["bytes_peak"] <= budget
    for i, w in enumerate(works):
        close(results[i], w.plain(env))
    srv.close()
    # A tree whose register stack must spill more subtrees than the cache
    # holds can never be admitted: each complete binary subtree of depth 10
    # below needs a stack of 11, so each spills one subtree, and the cache
    # holds one row.
    def full(d, v):
        return v if d == 0 else f"add({full(d - 1, v)}, {full(d - 1, v)})"
    deep = pg.parse(f"sub({full(10, 'x')}, {full(10, 'y')})")
    pop = pg.Population(deep, np.array([0, len(deep)], np.int64), 1, 1)
    tiny = tgp.Server(ctx, row, 2)
    t = tiny.submit(0, pop, works[0].dom, works[0].target, 0)
    with pytest.raises(tgp.TgpError) as e:
        tiny.wait(t)
    assert e.value.status == -5
    tiny.close()


def test_request_errors(env):
    tgp, ctx, torch = env
    srv = tgp.Server(ctx, 1 << 26, 2)
    dom2 = tgp.Domain(ctx, (16, 16))
    tgt = torch.zeros(256, dtype=torch.float32, device="cuda:0")
    bad = pg.parse("add(x, z)")
    pop = pg.Population(bad, np.array([0, len(bad)], np.int64), 1, 1)
    t = srv.submit(0, pop, dom2, tgt, 0)
    with pytest.raises(tgp.TgpError) as e:
        srv.wait(t)
    assert e.value.status == -7  # ESHAPE
    toks = pg.parse("add(x, y)")[:2]  # a truncated tree
    pop = pg.Population(toks, np.array([0, len(toks)], np.int64), 1, 1)
    t = srv.submit(0, pop, dom2, tgt, 0)
    with pytest.raises(tgp.TgpError) as e:
        srv.wait(t)
    assert e.value.status == -2  # EPARSE
    # an empty population ends at once
    empty = pg.Population(np.zeros(0, pg.TOKEN_DTYPE), np.zeros(1, np.int64), 0, 1)
    t = srv.submit(0, empty, dom2, tgt, 0)
    assert srv.wait(t, 10_000_000).size == 0
    st = srv.stats()
    assert st["failed"] == 2 and st["completed"] == 1
    srv.close()
