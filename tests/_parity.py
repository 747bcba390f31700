"""The parity contract between the HIP path and the FP64 oracle.

Per case (value v of the GPU, O64 / O32r from the oracle):
  * on every case the oracle marks STABLE, |v - O64| / max(|O64|, 1) <= 1e-5;
  * on every case it marks NONFINITE_STABLE, v has the same non-finite class
    (NaN, +inf, -inf) as O32r.
Per individual:
  * when all its cases are stable and the FP32-rounded walk O32r moves its
    fitness by at most 1e-7 relative, |F_gpu - F_O64| <= 1e-6 F_O64 (exact 0
    when F_O64 = 0);
  * otherwise, when F_O64 and F_O32r are both finite, |F_gpu - F_O64| is
    bounded by max(1e-6 F_O64, 4 |F_O32r - F_O64|): the error the paper's
    FP32 tensors would make, with room for one ulp more per operator;
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


def check_fitness(f_gpu, v64, v32r, stab, target, n_ind, n_ch, loss, what=""):
    f64 = oracle.fitness(v64, target, n_ind, n_ch, loss)
    f32 = oracle.fitness(v32r, target, n_ind, n_ch, loss)
    stable = ((stab & oracle.STABLE) != 0).reshape(n_ind, -1).all(axis=1)
    n_terms = v64.size // n_ind
    strict = envelope = 0
    for i in range(n_ind):
        a, b, g = f64[i], f32[i], f_gpu[i]
        if not (np.isfinite(a) and np.isfinite(b)):
            continue
        if _may_overflow(max(a, b), n_terms, loss) and g == np.inf:
            continue
        if stable[i] and abs(b - a) <= 1e-7 * a:
            tol = FIT_TOL * a
            strict += 1
        else:
            tol = max(FIT_TOL * a, 4 * abs(b - a))
            envelope += 1
        if not abs(g - a) <= tol:
            raise AssertionError(f"{what}: individual {i} fitness gpu {g!r} oracle {a!r} "
                                 f"(O32r {b!r}) tol {tol:.3g}")
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
