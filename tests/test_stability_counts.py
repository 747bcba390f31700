"""The oracle's stability counts of every parity workload equal the recorded
ones (tests/golden/stability_counts.txt, written by the oracle alone), and
each workload meets its floor of checked cases and individuals.  A change of
the classifier that silently narrows what the parity tests compare fails
here on the CPU."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import parity_workloads as pw  # noqa: E402

GOLD = pw.golden_counts()


@pytest.mark.parametrize("name", list(pw.WORKLOADS))
def test_counts_equal_recorded(name):
    assert pw.summary(name) == GOLD[name]


@pytest.mark.parametrize("name", list(pw.WORKLOADS))
def test_floors(name):
    cases, ind = pw.checked_shares(GOLD[name])
    fc, fi = pw.FLOORS[name]
    assert cases >= fc and ind >= fi, (name, cases, ind)


@pytest.mark.parametrize("name", list(pw.WORKLOADS))
def test_contract_accepts_fp32_model(name):
    """The parity checks themselves, run on the CPU with the oracle's O32r
    values (every operator correctly rounded to FP32) standing in for the
    device's: an FP32 evaluation of the assumed accuracy passes every case
    and fitness check, and the counts are the recorded ones."""
    import numpy as np

    import _parity
    import oracle
    pop, shape, spec, loss = pw.load(name)
    v64, v32, st, eb = oracle.evaluate(pop.tokens, pop.offsets, shape, bound=True)
    tg = pw.target(spec, shape)
    g = v32.astype(np.float32)
    rc = _parity.check_cases(g, v64, v32, st, eb, name)
    f = oracle.fitness(g.astype(np.float64), tg, pop.n_individuals, pop.n_channels, loss)
    rf = _parity.check_fitness(f, g, v64, st, eb, tg, pop.n_individuals, pop.n_channels, loss, name)
    _parity.reduction_property(f, g, tg, pop.n_individuals, pop.n_channels, loss)
    gold = GOLD[name]
    assert all(rc[k] == gold[k] for k in ("stable", "envelope", "nonfinite", "unchecked"))
    assert all(rf[k] == gold["fit_" + k] for k in ("strict", "envelope", "inf", "partial"))
