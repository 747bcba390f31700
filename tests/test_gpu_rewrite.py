"""Identity rewrites on the GPU (tgp_ctx_set_rewrite): the device DAG equals
oracle.build_dag(rewrite=True) array by array, structurally and with
commutative hashing, and every per-case value and fitness is bitwise the
one the unrewritten DAG gives (NaN positions equal)."""
import numpy as np
import pytest

import oracle
from paper_2103_07512_amd import popgen as pg

import rewrite_cases as rc
from test_gpu_parity import _dag_equal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_07512_amd import tgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return tgp, torch


def _populations():
    yield "patterns F18", pg.population_from_texts(rc.rewrite_texts(11, 400))
    yield "patterns F6 deep", pg.population_from_texts(rc.rewrite_texts(12, 300, depth=8, funcs=pg.F6))
    yield "patterns 3-D", pg.population_from_texts(rc.rewrite_texts(13, 200, nvars=3))
    yield "F18 d2-10", pg.ramped_half_and_half(300, 2, 10, 14, pg.F18, 2)


def _values(tgp, torch, ctx, pop, shape):
    d = tgp.Domain(ctx, shape)
    dag = tgp.build_dag(ctx, pop)
    out = torch.empty(pop.n_roots, d.cases, dtype=torch.float32, device="cuda:0")
    tgp.evaluate(ctx, dag, d, out)
    target = torch.from_numpy(np.cos(np.arange(d.cases, dtype=np.float32))[None, :].copy()).to("cuda:0")
    f = torch.empty(pop.n_individuals, dtype=torch.float64, device="cuda:0")
    tgp.fitness(ctx, dag, d, target, tgp.RMSE, f)
    torch.cuda.synchronize()
    return dag, out.cpu().numpy(), f.cpu().numpy()


@pytest.mark.parametrize("commutative", [False, True])
def test_rewritten_dag_matches_oracle_and_values_unchanged(env, commutative):
    tgp, torch = env
    plain = tgp.Context(0)
    rw = tgp.Context(0)
    rw.set_rewrite(True)
    for c in (plain, rw):
        c.set_hashing(commutative)
    for name, pop in _populations():
        shape = (17, 19, 5) if "3-D" in name else (37, 41)
        dag_p, v_p, f_p = _values(tgp, torch, plain, pop, shape)
        dag_r, v_r, f_r = _values(tgp, torch, rw, pop, shape)
        o = oracle.build_dag(pop.tokens, pop.offsets, commutative=commutative, rewrite=True)
        _dag_equal(dag_r.export(), o, name)
        n_p, n_r = dag_p.stats()["dag_nodes"], dag_r.stats()["dag_nodes"]
        say(name, "commutative" if commutative else "structural", "nodes", n_p, "->", n_r)
        if name.startswith("patterns"):
            assert n_r < n_p
        nan_p = np.isnan(v_p)
        assert np.array_equal(nan_p, np.isnan(v_r)), name
        assert np.array_equal(v_p[~nan_p].view(np.uint32), v_r[~nan_p].view(np.uint32)), name
        assert np.array_equal(np.isnan(f_p), np.isnan(f_r)) and np.array_equal(f_p[~np.isnan(f_p)],
                                                                                f_r[~np.isnan(f_r)]), name
