#!/usr/bin/env python3
"""Benchmark of whole-population GP fitness evaluation on one MI355X.

One step is the whole hot path over one synthetic population whose tokens,
offsets and target are already resident in HBM: hash-consing the population
into its DAG on the GPU, planning the subtree cache and the programs,
filling cached subtrees, the fused interpreter with the error reduction, and
the FP64 finalize.  The headline number is credited node evaluations per
second: distinct DAG nodes x fitness cases / s (each distinct subtree counts
once per case, whether it was computed, cached or shared).

Default workload: 1000 individuals x 3 channel trees, ramped half-and-half
depths 2-12 over the 18-operator set, on a 1024 x 1024 grid in [-1, 1]^2,
MSE against a target image rendered from three seeded depth-8 trees.

Prints one JSON line.  `roofline` is for the dominant kernel (the fused
root-program launch), timed with HIP events on the stream it runs on;
`cpu_baseline` is the FP64 oracle timed on a bounded row sample of the same
workload on the host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("node-evals/s (DAG nodes × fitness cases / s) at 1024² domain; "
          "p50/p99 request latency")
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# 32-bit lane operation per lane per clock (no packed-FP32 issue).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    "c3": "1000 individuals x 3 channel trees, ramped half-and-half depth 2-12, 18 operators, "
          "1024x1024 grid, MSE vs a 3-channel image from seeded depth-8 trees",
    "c2": "500 trees bred by subtree crossover/mutation (depth <= 10, 18 operators), "
          "256x256 grid, RMSE vs a seeded depth-4 tree",
    "c1": "50 ramped half-and-half trees depth 2-6, 6 operators, 64x64 grid, RMSE vs a seeded "
          "depth-4 tree",
    "c4": "64 populations (sizes log-uniform 20-2000, depths 4-14, 18 operators), domains 2-D "
          "32^2-1024^2 or 3-D 64^3, RMSE; one batched persistent step vs 64 plain launches",
}


def load_workload(name):
    from paper_2103_07512_amd import popgen as pg
    if name == "c3":
        pop, dom, spec = pg.workload_c3()
        return pop, dom, spec, 1   # MSE
    if name == "c2":
        pop, dom, spec = pg.workload_c2()
        return pop, dom, spec, 0
    pop, dom, spec = pg.workload_c1()
    return pop, dom, spec, 0


def cpu_baseline(pop, dom, dag_nodes, max_rows=64, budget_s=15.0):
    """Time the FP64 oracle on evenly spaced grid rows (all trees, all channels)."""
    import numpy as np

    import oracle
    rows_total = dom.shape[0]
    row_len = dom.cases // rows_total

    def run(nrows):
        rows = np.unique(np.linspace(0, rows_total - 1, nrows).round().astype(np.int64))
        cases = (rows[:, None] * row_len + np.arange(row_len)[None, :]).ravel()
        t = time.perf_counter()
        oracle.evaluate(pop.tokens, pop.offsets, dom.shape, cases=cases)
        return time.perf_counter() - t, len(cases), len(rows)

    dt, n, nr = run(1)
    if dt < budget_s / 2:
        want = int(min(max_rows, max(1, budget_s / max(dt, 1e-3))))
        if want > 1:
            dt, n, nr = run(want)
    credited = dag_nodes * n / dt
    executed = len(pop.tokens) * n / dt
    return {"value": credited, "unit": "node-evals/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{nr} of {rows_total} grid rows ({n} cases per tree, all {pop.n_roots} trees); "
                      f"FP64 recursive tree walk, no subtree caching; executed tree-node evals/s "
                      f"{executed:.4g}; {dt:.2f} s"}


def bench_c4(args):
    """64 populations: batched (persistent kernels, replayed HIP graph, autotuned
    shape) against one plain tgp_fitness per population, DAG build included."""
    import numpy as np
    import torch

    from paper_2103_07512_amd import popgen as pg
    from paper_2103_07512_amd import tgp

    dev = torch.device("cuda:0")
    work = pg.workload_c4()
    ctx = tgp.Context(0)
    items = []
    for pop, dspec, tspec in work:
        dom = tgp.Domain(ctx, dspec.shape)

        def render(tree, dom=dom):
            d = tgp.Dag(ctx, tree, np.array([0, len(tree)], np.int64), 1)
            v = torch.empty(1, dom.cases, dtype=torch.float32, device=dev)
            tgp.evaluate(ctx, d, dom, v)
            return v[0].cpu().numpy() if bool(torch.isfinite(v).all()) else None

        _, target = pg.pick_target(tspec, render)
        items.append(dict(pop=pop, dom=dom, target=torch.from_numpy(target).to(dev),
                          tok=torch.from_numpy(pop.tokens.view(np.uint8).copy()).to(dev),
                          off=torch.from_numpy(pop.offsets.copy()).to(dev),
                          out=torch.empty(pop.n_individuals, dtype=torch.float64, device=dev)))

    def dags():
        return [tgp.Dag(ctx, it["tok"], it["off"], it["pop"].n_individuals) for it in items]

    def jobs_of(ds):
        return [(d, it["dom"], it["target"], tgp.RMSE, it["out"]) for d, it in zip(ds, items)]

    tune = tgp.autotune(ctx, jobs_of(dags()))
    batch = tgp.Batch(ctx, use_graph=True)

    def step_batched():
        ds = dags()
        batch.run(jobs_of(ds))
        return ds

    def step_plain():
        ds = dags()
        for d, it in zip(ds, items):
            tgp.fitness(ctx, d, it["dom"], it["target"], tgp.RMSE, it["out"])
        return ds

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    t_plain = timed(step_plain)
    plain_fit = [it["out"].cpu().numpy().copy() for it in items]
    t_batch = timed(step_batched)
    batch_fit = [it["out"].cpu().numpy() for it in items]
    ds = dags()
    credited = sum(d.stats()["dag_nodes"] * it["dom"].cases for d, it in zip(ds, items))
    # evaluation only (DAGs built once): the batched step against 64 plain launches
    eval_plain = timed(lambda: [tgp.fitness(ctx, d, it["dom"], it["target"], tgp.RMSE, it["out"])
                                for d, it in zip(ds, items)])
    eval_batch = timed(lambda: batch.run(jobs_of(ds)))
    agree = max(float(np.nanmax(np.abs(a - b) / np.maximum(np.abs(a), 1e-300)))
                if np.isfinite(a).any() else 0.0 for a, b in zip(plain_fit, batch_fit))
    st = batch.stats()
    line = {
        "metric": METRIC, "value": credited / t_batch, "unit": "node-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"], "populations": len(items),
                   "individuals": int(sum(it["pop"].n_individuals for it in items)),
                   "tree_nodes": int(sum(len(it["pop"].tokens) for it in items))},
        "detail": {"plain_value": credited / t_plain, "plain_ms_per_step": t_plain * 1e3,
                   "batched_over_plain": t_plain / t_batch,
                   "eval_only_ms": {"plain": eval_plain * 1e3, "batched": eval_batch * 1e3},
                   "eval_only_batched_over_plain": eval_plain / eval_batch,
                   "autotune": tune, "batch": st, "max_rel_diff_batched_vs_plain": agree},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cases-per-lane", type=int, default=0)
    ap.add_argument("--tiles-per-item", type=int, default=0)
    ap.add_argument("--no-reorder", action="store_true")
    ap.add_argument("--cache-access-cost", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build evaluates a population on a single MI355X "
              f"and has no multi-GPU path (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return bench_c4(args)

    import numpy as np
    import torch

    from paper_2103_07512_amd import popgen as pg
    from paper_2103_07512_amd import tgp

    dev = torch.device("cuda:0")
    pop, dspec, tspec, loss = load_workload(args.workload)
    ctx = tgp.Context(0)
    ctx.set_tuning(args.cases_per_lane, args.tiles_per_item)
    ctx.set_plan(not args.no_reorder, args.cache_access_cost)
    dom = tgp.Domain(ctx, dspec.shape)

    def render(tree):
        d = tgp.Dag(ctx, tree, np.array([0, len(tree)], np.int64), 1)
        v = torch.empty(1, dom.cases, dtype=torch.float32, device=dev)
        tgp.evaluate(ctx, d, dom, v)
        ok = bool(torch.isfinite(v).all())
        return v[0].cpu().numpy() if ok else None

    _, target = pg.pick_target(tspec, render)
    target_dev = torch.from_numpy(target).to(dev)
    tok_dev = torch.from_numpy(pop.tokens.view(np.uint8).copy()).to(dev)
    off_dev = torch.from_numpy(pop.offsets.copy()).to(dev)
    out = torch.empty(pop.n_individuals, dtype=torch.float64, device=dev)
    ctx.set_timing(True)

    def step():
        dag = tgp.Dag(ctx, tok_dev, off_dev, pop.n_individuals, pop.n_channels)
        tgp.fitness(ctx, dag, dom, target_dev, loss, out)
        return dag

    for _ in range(args.warmup):
        step().close()
    torch.cuda.synchronize()
    times, stats = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dag = step()
        times.append(ctx.last_timing())
        stats = dag.stats()
        dag.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    work = ctx.last_work()
    fit = out.cpu().numpy()

    ms = wall / args.steps * 1e3
    credited = stats["dag_nodes"] * dom.cases
    value = credited / (ms / 1e3)
    interp_ms = float(np.mean([t["interp_ms"] for t in times]))
    achieved = work["executed_valu_roots"] / (interp_ms / 1e3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "node-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "individuals": pop.n_individuals,
                   "channels": pop.n_channels, "domain": list(dspec.shape),
                   "loss": "mse" if loss else "rmse", "tree_nodes": stats["tree_nodes"],
                   "dag_nodes": stats["dag_nodes"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_interp fitness launch (root programs fused with the reduction)",
                     "kernel_ms": interp_ms},
        "detail": {
            "phases_ms": {k: float(np.mean([t[k] for t in times]))
                          for k in ("build_dag_ms", "plan_ms", "fill_ms", "interp_ms", "finalize_ms")},
            "launch": {k: times[-1][k] for k in ("interp_items", "cases_per_lane", "tiles_per_item")},
            "work": work,
            "executed_node_evals_per_s": work["executed_node_evals"] / (ms / 1e3),
            "finite_fitness": int(np.isfinite(fit).sum()),
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pop, dspec, stats["dag_nodes"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
