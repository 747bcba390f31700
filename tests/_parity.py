"""The parity contract between the HIP path and the FP64 oracle.

Per case (value g of the GPU; O64, O32r, the flags and the running error
bound E from the oracle; sc = max(|O64|, 1)):
  * STABLE (E <= 5e-6 sc, clear of every discontinuity): |g - O64| <= 1e-5 sc;
  * ENVELOPE (clear of every discontinuity, 5e-6 sc < E <= sc / 16):
    |g - O64| <= 1e-5 sc + 2 E (first-order analysis, doubled);
  * NONFINITE_STABLE: g has the non-finite class (NaN, +inf, -inf) of O32r;
  * every other case is unchecked per case (its count is reported).
Per individual, with the first-order fitness bound E_F propagated from the
per-case bounds of its checked cases (RMSE: sum |v - t| E / (N F); MSE:
2 sum |v - t| E / N), every individual falls in exactly one class:
  * inf: some case is NONFINITE_STABLE, so the GPU's fitness must be +inf;
  * strict: every case stable and E_F <= 1e-7 F_O64:
    |F_gpu - F_O64| <= 1e-6 F_O64 (exact 0 when F_O64 = 0);
  * envelope: every case stable or envelope:
    |F_gpu - F_O64| <= max(1e-6 F_O64, 2 E_F);
  * partial: some cases unchecked.  The reference is the hybrid fitness H
    of O64 on the checked cases and the GPU's own values on the rest:
    |F_gpu - H| <= max(1e-6 H, 2 E_F), and +inf when H is not finite;
and, for all individuals, F_gpu equals the FP64 reduction of the GPU's own
per-case values within 1e-6 relative (a property of the reduction alone).
An FP32 sum of squares that can reach FLT_MAX may give +inf on the device
where the FP64 sum is finite; such individuals accept +inf.
"""
import numpy as np

import oracle

CASE_TOL = 1e-5
FIT_TOL = 1e-6
FLT_MAX = float(np.finfo(np.float32).max)
CHECKED = oracle.STABLE | oracle.ENVELOPE | oracle.NONFINITE_STABLE


def _sum_of_squares(f, n_terms, loss):
    return f * f * n_terms if loss == "rmse" else f * n_terms


def _may_overflow(f, n_terms, loss):
    """True when the FP32 sum of squares of some stripe could reach FLT_MAX."""
    return not _sum_of_squares(f, n_terms, loss) < FLT_MAX * 0.999


def nf_class(a):
    a = np.asarray(a, dtype=np.float64)
    return np.where(np.isnan(a), 1, np.where(np.isposinf(a), 2, np.where(np.isneginf(a), 3, 0)))


def case_counts(stab):
    """How many cases the per-case contract checks, by kind."""
    s = (stab & oracle.STABLE) != 0
    e = (stab & oracle.ENVELOPE) != 0
    n = (stab & oracle.NONFINITE_STABLE) != 0
    return dict(cases=int(stab.size), stable=int(s.sum()), envelope=int(e.sum()), nonfinite=int(n.sum()),
                unchecked=int((~(s | e | n)).sum()))


def check_cases(gpu, v64, v32r, stab, ebound, what=""):
    g = np.asarray(gpu, dtype=np.float64)
    stable = (stab & oracle.STABLE) != 0
    env = (stab & oracle.ENVELOPE) != 0
    sc = np.maximum(np.abs(v64), 1.0)
    with np.errstate(all="ignore"):
        dev = np.abs(g - v64)
        err = dev / sc
    bad = stable & ~(err <= CASE_TOL)
    if bad.any():
        r, c = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} stable cases off, first tree {r} case {c}: "
                             f"gpu {g[r, c]!r} oracle {v64[r, c]!r} err {err[r, c]:.3g}")
    bad = env & ~(dev <= CASE_TOL * sc + 2.0 * ebound)
    if bad.any():
        r, c = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} envelope cases off, first tree {r} case {c}: "
                             f"gpu {g[r, c]!r} oracle {v64[r, c]!r} bound {ebound[r, c]:.3g}")
    nfs = (stab & oracle.NONFINITE_STABLE) != 0
    mism = nfs & (nf_class(g) != nf_class(v32r))
    if mism.any():
        r, c = np.argwhere(mism)[0]
        raise AssertionError(f"{what}: non-finite class differs at tree {r} case {c}: "
                             f"gpu {g[r, c]!r} O32r {v32r[r, c]!r}")
    out = case_counts(stab)
    out["max_err_stable"] = float(err[stable].max()) if stable.any() else 0.0
    return out


def _fitness_bound(v, eb, target, n_ind, loss, f):
    """First-order bound of each individual's fitness from per-case bounds."""
    d = np.abs(v.reshape(n_ind, -1) - np.asarray(target, np.float64).reshape(1, -1))
    n_terms = d.shape[1]
    with np.errstate(all="ignore"):
        s = (d * eb.reshape(n_ind, -1)).sum(axis=1)
        return s / (n_terms * f) if loss == "rmse" else 2 * s / n_terms


def fitness_classes(v64, stab, ebound, target, n_ind, n_ch, loss):
    """Class of every individual (see the module docstring), from the oracle
    alone: 'inf', 'strict', 'envelope' or 'partial'."""
    st = stab.reshape(n_ind, -1)
    f64 = oracle.fitness(v64, target, n_ind, n_ch, loss)
    ef = _fitness_bound(v64, ebound, target, n_ind, loss, f64)
    nfs = ((st & oracle.NONFINITE_STABLE) != 0).any(axis=1)
    all_stable = ((st & oracle.STABLE) != 0).all(axis=1)
    all_checked = ((st & (oracle.STABLE | oracle.ENVELOPE)) != 0).all(axis=1)
    out = []
    for i in range(n_ind):
        if nfs[i]:
            out.append("inf")
        elif all_stable[i] and np.isfinite(f64[i]) and (f64[i] == 0 or ef[i] <= 1e-7 * f64[i]):
            out.append("strict")
        elif all_checked[i] and np.isfinite(f64[i]):
            out.append("envelope")
        else:
            out.append("partial")
    return out, f64, ef


def fitness_counts(classes):
    return {k: int(sum(1 for c in classes if c == k)) for k in ("strict", "envelope", "inf", "partial")}


def check_fitness(f_gpu, gpu_vals, v64, stab, ebound, target, n_ind, n_ch, loss, what=""):
    classes, f64, ef = fitness_classes(v64, stab, ebound, target, n_ind, n_ch, loss)
    n_terms = v64.size // n_ind
    st = stab.reshape(n_ind, -1)
    checked = (st & (oracle.STABLE | oracle.ENVELOPE)) != 0
    g = np.asarray(gpu_vals, np.float64).reshape(n_ind, -1)
    vv = v64.reshape(n_ind, -1)
    eb = ebound.reshape(n_ind, -1)
    t = np.asarray(target, np.float64).reshape(-1)
    for i, cls in enumerate(classes):
        got = f_gpu[i]
        if cls == "inf":
            assert got == np.inf, f"{what}: individual {i} has a required non-finite case, fitness {got!r}"
            continue
        if cls == "partial":
            hyb = np.where(checked[i], vv[i], g[i])
            ref = oracle.fitness(hyb.reshape(n_ch, -1), target, 1, n_ch, loss)[0]
            e_i = np.where(checked[i], eb[i], 0.0)
            with np.errstate(all="ignore"):
                s = float((np.abs(hyb - t) * e_i).sum())
                e_chk = s / (n_terms * ref) if loss == "rmse" else 2 * s / n_terms
        else:
            ref, e_chk = f64[i], ef[i]
        if not np.isfinite(ref):
            assert got == np.inf, f"{what}: individual {i} reference {ref!r} fitness {got!r}"
            continue
        if _may_overflow(ref, n_terms, loss) and got == np.inf:
            continue
        if ref == 0:
            assert got == 0, f"{what}: individual {i} fitness {got!r}, reference 0"
            continue
        tol = FIT_TOL * ref if cls == "strict" else max(FIT_TOL * ref, 2 * e_chk)
        if not abs(got - ref) <= tol:
            raise AssertionError(f"{what}: individual {i} ({cls}) fitness gpu {got!r} reference {ref!r} "
                                 f"bound {e_chk:.3g} tol {tol:.3g}")
    return fitness_counts(classes)


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
