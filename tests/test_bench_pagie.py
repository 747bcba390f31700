"""The paper-shaped bench workload renders its target, the Pagie polynomial
(Eq. 1), from an expression that the library evaluates on the device; the
expression must be Eq. 1.  Checked with the oracle against the closed form
1/(1 + x^-4) + 1/(1 + y^-4) on grids of the bench's shape."""
import os
import sys

import numpy as np

import oracle
from paper_2103_07512_amd import popgen as pg

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_pagie_expression_is_eq1():
    pop = pg.population_from_texts([bench.PAGIE])
    for side in (64, 65):
        v = oracle.evaluate(pop.tokens, pop.offsets, (side, side))[0]
        t = np.linspace(-1.0, 1.0, side)
        x, y = np.meshgrid(t, t, indexing="ij")  # axis 0 = x, the last axis fastest
        with np.errstate(divide="ignore"):
            want = 1.0 / (1.0 + x ** -4.0) + 1.0 / (1.0 + y ** -4.0)
        # the grid coordinates are FP32 values of the FP64 grid points
        xf = x.astype(np.float32).astype(np.float64)
        yf = y.astype(np.float32).astype(np.float64)
        with np.errstate(divide="ignore"):
            want32 = 1.0 / (1.0 + xf ** -4.0) + 1.0 / (1.0 + yf ** -4.0)
        assert np.allclose(v, want32.ravel(), rtol=1e-12, atol=1e-15)
        assert np.allclose(v, want.ravel(), rtol=1e-6, atol=1e-7)
