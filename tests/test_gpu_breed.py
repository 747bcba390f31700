"""Genetic operators on the device (tgp_breed through the C ABI) against the
oracle's breeding (oracle/breed.py): bit-exact tokens and offsets for the
same parents, fitness and seed, including the full-size 1000 x 3 population,
chained generations from device-resident parents, and the error paths."""
import numpy as np
import pytest

from oracle import breed as ob
from paper_2103_07512_amd import popgen as pg

pytestmark = pytest.mark.gpu

F18 = [pg.OP_CODE[f] for f in pg.F18]
ALL = sorted(set(pg.OP_CODE[f] for f in pg.OP_CODE if pg.ARITY[pg.OP_CODE[f]] > 0))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_07512_amd import tgp
    assert torch.cuda.is_available()
    return tgp, tgp.Context(0), torch


def _fit_dev(torch, fit):
    return None if fit is None else torch.tensor(np.asarray(fit, np.float64), device="cuda:0")


def _check(env, pop, fit, seed, n_off, **kw):
    tgp, ctx, torch = env
    say("breed", pop.n_individuals, "x", pop.n_channels, "seed", seed, "offspring", n_off, kw)
    off = tgp.Offspring(ctx, pop, _fit_dev(torch, fit), seed=seed, n_offspring=n_off, **kw)
    got_t, got_o = off.to_host()
    kw2 = dict(kw)
    tries = kw2.pop("crossover_tries", 8)
    use_c = kw2.pop("use_constants", True)
    want_t, want_o = ob.breed(pop.tokens, pop.offsets, pop.n_channels, fit, seed, n_off, tries=tries,
                              use_const=use_c, **kw2)
    assert np.array_equal(got_o, want_o)
    assert np.array_equal(got_t.view(np.uint64), np.ascontiguousarray(want_t).view(np.uint64))
    return off, want_t, want_o


def test_breed_default_rates(env):
    pop = pg.ramped_half_and_half(40, 2, 6, 31, pg.F18, 2, 2)
    rng = np.random.default_rng(1)
    fit = rng.random(40)
    fit[[3, 7]] = np.nan
    fit[11] = np.inf
    for seed in (0, 1, 2 ** 63 + 5):
        _check(env, pop, fit, seed, 40, functions=F18, max_depth=8)


def test_breed_crossover_depth_limit(env):
    """Tight depth limit: many crossover draws are rejected, some offspring
    are copies after the last try."""
    pop = pg.ramped_half_and_half(25, 3, 6, 32, pg.F18, 2, 1)
    _check(env, pop, np.arange(25.0), 5, 60, functions=F18, p_crossover=1.0, p_mutation=0.0,
           max_depth=6, crossover_tries=2)


def test_breed_mutation_forms(env):
    pop = pg.ramped_half_and_half(20, 1, 5, 33, pg.F18, 3, 1)
    for mmd, ndim, use_c in ((0, 3, True), (2, 3, False), (4, 1, True), (16, 2, True)):
        _check(env, pop, None, 7 + mmd, 50, functions=ALL, p_crossover=0.0, p_mutation=1.0,
               max_depth=30 if mmd == 16 else 9, max_mutation_depth=mmd, ndim=ndim, use_constants=use_c)


def test_breed_selection_and_sizes(env):
    pop = pg.ramped_half_and_half(15, 0, 4, 34, pg.F18, 2, 2)  # depth 0: single-token trees too
    fit = np.linspace(3.0, 1.0, 15)
    for n_off, t in ((1, 1), (7, 2), (100, 5), (0, 3)):
        _check(env, pop, fit, 11, n_off, functions=F18, tournament=t)


def test_breed_deep_postfix_stacks(env):
    """Parents whose postfix stack is deeper than the shape scan keeps in LDS
    (32 entries) take its global-memory path; offspring still match."""
    def chain(n, op):
        text = "x"
        for i in range(n):
            text = f"{op}({'y' if i % 2 else 'x'}, {text})"
        return text
    texts = [chain(40, "add"), chain(20, "mult"), chain(35, "sub"), "x", chain(33, "max")]
    pop = pg.population_from_texts(texts)
    _check(env, pop, np.array([1.0, 2.0, 0.5, 3.0, 1.5]), 41, 30, functions=F18, max_depth=50)


def test_breed_full_size_population(env):
    """The 1000 x 3 headline population (F18, depths 2-12), one generation."""
    pop = pg.workload_c3()[0]
    rng = np.random.default_rng(3)
    fit = rng.random(pop.n_individuals)
    _check(env, pop, fit, 2024, pop.n_individuals, functions=F18, max_depth=12)


def test_breed_chained_on_device(env):
    """Three generations, each bred from the previous offspring left on the
    device, against the oracle bred from its own previous generation."""
    tgp, ctx, torch = env
    pop = pg.ramped_half_and_half(30, 2, 5, 35, pg.F18, 2, 2)
    parents, host = pop, (pop.tokens, pop.offsets)
    kw = dict(functions=F18, max_depth=7, p_crossover=0.6, p_mutation=0.3)
    keep = []
    for g in range(3):
        fit = np.random.default_rng(g).random(30)
        say("generation", g)
        off = tgp.Offspring(ctx, parents, _fit_dev(torch, fit), seed=100 + g, n_offspring=30, **kw)
        want_t, want_o = ob.breed(host[0], host[1], 2, fit, 100 + g, 30, **kw)
        got_t, got_o = off.to_host()
        assert np.array_equal(got_o, want_o)
        assert np.array_equal(got_t.view(np.uint64), np.ascontiguousarray(want_t).view(np.uint64))
        keep.append(off)
        parents, host = off, (want_t, want_o)


def test_offspring_feeds_the_dag_and_fitness(env):
    """A device-bred population hash-conses and evaluates exactly like the same
    tokens uploaded from the host."""
    tgp, ctx, torch = env
    pop = pg.ramped_half_and_half(50, 2, 6, 36, pg.F18, 2, 1)
    off = tgp.Offspring(ctx, pop, None, seed=9, n_offspring=50, functions=F18, max_depth=8)
    toks, offs = off.to_host()
    d_dev = tgp.Dag(ctx, off)
    d_host = tgp.Dag(ctx, toks, offs, 50, 1)
    assert d_dev.stats() == d_host.stats()
    dom = tgp.Domain(ctx, (64, 48))
    t = torch.zeros(1, dom.cases, dtype=torch.float32, device="cuda:0")
    a = torch.empty(50, dtype=torch.float64, device="cuda:0")
    b = torch.empty(50, dtype=torch.float64, device="cuda:0")
    tgp.fitness(ctx, d_dev, dom, t, tgp.RMSE, a)
    tgp.fitness(ctx, d_host, dom, t, tgp.RMSE, b)
    assert np.array_equal(a.cpu().numpy().view(np.uint64), b.cpu().numpy().view(np.uint64))


def test_breed_errors(env):
    tgp, ctx, torch = env
    pop = pg.ramped_half_and_half(4, 1, 3, 37, pg.F18, 2, 1)
    with pytest.raises(tgp.TgpError) as e:
        tgp.Offspring(ctx, pop, None, seed=1, n_offspring=2, functions=[pg.OP_CODE["add"], 0])
    assert e.value.status == -4  # a terminal is not a function
    with pytest.raises(tgp.TgpError) as e:
        tgp.Offspring(ctx, pop, None, seed=1, n_offspring=2, functions=F18, p_crossover=0.9, p_mutation=0.2)
    assert e.value.status == -1
    with pytest.raises(tgp.TgpError) as e:
        tgp.Offspring(ctx, pop, None, seed=1, n_offspring=2, functions=F18, max_mutation_depth=17)
    assert e.value.status == -1
    bad = pg.Population.from_trees([pg.parse("add(x, y)"), pg.make_tokens([(0, 0, 0.0), (0, 1, 0.0)])], 1)
    say("malformed parent tree")
    with pytest.raises(tgp.TgpError) as e:
        tgp.Offspring(ctx, bad, None, seed=1, n_offspring=3, functions=F18)
    assert e.value.status == -2
    # the context still works afterwards
    _check(env, pop, None, 3, 4, functions=F18)
