"""The parity contract between the HIP path and the FP64 oracle.

Per case (value v of the GPU; O64, O32r and the running error bound E from
the oracle):
  * on every case the oracle marks STABLE (E <= 5e-6 max(|O64|, 1), clear of
    every discontinuity), |v - O64| / max(|O64|, 1) <= 1e-5;
  * on every case it marks NONFINITE_STABLE, v has the same non-finite class
    (NaN, +inf, -inf) as O32r.
Per individual, with the first-order fitness bound E_F propagated from the
per-case bounds (RMSE: sum |v - t| E / (N F); MSE: 2 sum |v - t| E / N):
  * when all its cases are stable and E_F <= 1e-7 F_O64,
    |F_gpu - F_O64| <= 1e-6 F_O64 (exact 0 when F_O64 = 0);
  * otherwise, when all its cases are stable, |F_gpu - F_O64| <=
    max(1e-6 F_O64, 2 E_F);
  * always, F_gpu equals the FP64 reduction of the GPU's own per-case values
    within 1e-6 relative (a property of the reduction alone).
"""
import numpy as np

import oracle

CASE_TOL = 1e-5
FIT_TOL = 1e-6
FLT_MAX = float(np.finfo(np.float32).max)


def _sum_of_squares(f, n_terms, loss):
    return f * f * n_terms if loss == "rmse" else f * n_terms


def _may_overflow(f, n_terms, loss):
    """True when the FP32 sum of squares of some stripe could reach FLT_MAX."""
    return not _sum_of_squares(f, n_terms, loss) < FLT_MAX * 0.999


def nf_class(a):
    a = np.asarray(a, dtype=np.float64)
    return np.where(np.isnan(a), 1, np.where(np.isposinf(a), 2, np.where(np.isneginf(a), 3, 0)))


def check_cases(gpu, v64, v32r, stab, what=""):
    g = np.asarray(gpu, dtype=np.float64)
    stable = (stab & oracle.STABLE) != 0
    with np.errstate(all="ignore"):
        err = np.abs(g - v64) / np.maximum(np.abs(v64), 1.0)
    bad = stable & ~(err <= CASE_TOL)
    if bad.any():
        r, c = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} stable cases off, first tree {r} case {c}: "
                             f"gpu {g[r, c]!r} oracle {v64[r, c]!r} err {err[r, c]:.3g}")
    nfs = (stab & oracle.NONFINITE_STABLE) != 0
    mism = nfs & (nf_class(g) != nf_class(v32r))
    if mism.any():
        r, c = np.argwhere(mism)[0]
        raise AssertionError(f"{what}: non-finite class differs at tree {r} case {c}: "
                             f"gpu {g[r, c]!r} O32r {v32r[r, c]!r}")
    return dict(cases=int(stable.size), stable=int(stable.sum()), nonfinite_checked=int(nfs.sum()),
                max_err=float(err[stable].max()) if stable.any() else 0.0)


def check_fitness(f_gpu, v64, v32r, stab, ebound, target, n_ind, n_ch, loss, what=""):
    f64 = oracle.fitness(v64, target, n_ind, n_ch, loss)
    stable = ((stab & oracle.STABLE) != 0).reshape(n_ind, -1).all(axis=1)
    n_terms = v64.size // n_ind
    d = np.abs(v64.reshape(n_ind, -1) - np.tile(np.asarray(target, np.float64).reshape(-1), 1)[None, :])
    with np.errstate(all="ignore"):
        s = (d * ebound.reshape(n_ind, -1)).sum(axis=1)
        ef = s / (n_terms * f64) if loss == "rmse" else 2 * s / n_terms
    strict = envelope = 0
    for i in range(n_ind):
        a, g = f64[i], f_gpu[i]
        if not (np.isfinite(a) and stable[i]):
            continue
        if _may_overflow(a, n_terms, loss) and g == np.inf:
            continue
        if a == 0:
            assert g == 0, (what, i, g)
            strict += 1
            continue
        if ef[i] <= 1e-7 * a:
            tol = FIT_TOL * a
            strict += 1
        else:
            tol = max(FIT_TOL * a, 2 * ef[i])
            envelope += 1
        if not abs(g - a) <= tol:
            raise AssertionError(f"{what}: individual {i} fitness gpu {g!r} oracle {a!r} "
                                 f"bound {ef[i]:.3g} tol {tol:.3g}")
    return dict(strict=strict, envelope=envelope)


def reduction_property(f_gpu, gpu_vals, target, n_ind, n_ch, loss):
    """F_gpu against an FP64 numpy reduction of the GPU's own values."""
    g = np.asarray(gpu_vals, dtype=np.float64).reshape(n_ind, n_ch, -1)
    t = np.asarray(target, dtype=np.float64).reshape(1, n_ch, -1)
    with np.errstate(all="ignore"):
        s = ((g - t) ** 2).sum(axis=(1, 2))
        n = g.shape[1] * g.shape[2]
        want = np.sqrt(s / n) if loss == "rmse" else s / n
    want = np.where(np.isfinite(want), want, np.inf)
    for i in range(n_ind):
        if np.isinf(want[i]):
            assert np.isinf(f_gpu[i]) and f_gpu[i] > 0, (i, f_gpu[i])
        elif _may_overflow(want[i], n, loss) and f_gpu[i] == np.inf:
            continue
        else:
            assert abs(f_gpu[i] - want[i]) <= FIT_TOL * want[i], (i, f_gpu[i], want[i])
