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

# Algorithmic cost of one operator application on one fitness case, in VALU
# lane-operations: a fixed table that does not depend on how this library
# compiles the operators (elementary add/sub/mul/min/max 1, abs 1, frac 1,
# clip and if 2, sign 3, protected division 7, sqrt, sin, cos and exp 6, log
# 7, pow 13, mod 12, terminals 0).  The operators outside the 18-operator
# set count the same elementary steps their definitions use: neg 1, mdist
# (add, halve) 2, step 2, tan (sin, cos, division) 19, sstep 4, sstepp 6, len
# (two squares, a sum, sqrt) 9, lerp (difference, frac, product, sum) 4, the
# bitwise operators (two conversions, the operation, one conversion) 4, warp
# (two axis points of 6 and a gather) 14.
ALG_COST = {
    "var": 0, "const": 0, "add": 1, "sub": 1, "mult": 1, "div": 7, "sin": 6, "cos": 6, "tan": 19,
    "exp": 6, "log": 7, "pow": 13, "min": 1, "max": 1, "mdist": 2, "neg": 1, "sqrt": 6, "sign": 3,
    "abs": 1, "clip": 2, "mod": 12, "frac": 1, "if": 2, "step": 2, "sstep": 4, "sstepp": 6, "len": 9,
    "lerp": 4, "or": 4, "xor": 4, "and": 4, "warp": 14,
}


def algorithmic_lane_ops(export):
    """Per-case algorithmic lane-operations of a DAG: every function node
    whose value depends on a variable, each once, at ALG_COST.  Subtrees
    without variables have one value for all cases (the library folds them
    once per call), so they add no per-case work."""
    import numpy as np

    from paper_2103_07512_amd import popgen as pg
    op = export["nodes"]["op"].astype(np.int64)
    kids = export["children"]
    cost = np.array([ALG_COST[pg.OP_NAME[i]] for i in range(len(pg.OP_NAME))], np.float64)
    dep = op == pg.VAR
    # children precede their parents (first-occurrence order)
    for n in np.nonzero(pg.ARITY[op] > 0)[0]:
        k = kids[n]
        dep[n] = dep[k[k >= 0]].any()
    fn = pg.ARITY[op] > 0
    return float(cost[op[fn & dep]].sum()), float(cost[op[fn]].sum())

WORKLOADS = {
    "c3": "1000 individuals x 3 channel trees, ramped half-and-half depth 2-12, 18 operators, "
          "1024x1024 grid, MSE vs a 3-channel image from seeded depth-8 trees",
    "c2": "500 trees bred by subtree crossover/mutation (depth <= 10, 18 operators), "
          "256x256 grid, RMSE vs a seeded depth-4 tree",
    "c1": "50 ramped half-and-half trees depth 2-6, 6 operators, 64x64 grid, RMSE vs a seeded "
          "depth-4 tree",
    "c4": "64 populations (sizes log-uniform 20-2000, depths 4-14, 18 operators), domains 2-D "
          "32^2-1024^2 or 3-D 64^3, RMSE; one batched step (stack form, cases per lane and launch "
          "form autotuned) vs 64 plain launches",
    "evolve": "a GP run on the headline workload kept on the GPU: each generation hash-conses and "
              "evaluates the population (1000 x 3 trees, 1024x1024, MSE) and breeds the next one "
              "on the device (tournament 3, crossover 0.8, mutation 0.1, depth <= 12, 18 operators)",
    "p": "the paper's tree-evaluation experiment shape: 5 populations of 50 individuals, ramped "
         "half-and-half depths 2-12, 18 operators, RMSE against the Pagie polynomial on 2-D grids "
         "of 64^2 to 2048^2 cases in [-1, 1]^2",
    "c5": "16 concurrent GP runs (grids 512^2-4096^2, populations log-uniform 200-2000, bred "
          "closed-loop from returned fitness, depth <= 12, 18 operators), RMSE; served with "
          "continuous batching and a resident subtree cache",
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
    print(json.dumps(run_c4(args)), flush=True)


def run_c4(args):
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
    return line


# Pagie polynomial (Eq. 1), 1/(1 + x^-4) + 1/(1 + y^-4) = x^4/(1 + x^4) + y^4/(1 + y^4),
# as an expression the library itself renders on the device
PAGIE = ("add(div(mult(mult(x, x), mult(x, x)), add(1.0, mult(mult(x, x), mult(x, x)))), "
         "div(mult(mult(y, y), mult(y, y)), add(1.0, mult(mult(y, y), mult(y, y)))))")


def bench_p(args):
    """The paper's tree-evaluation experiment shape (Table 2): the same 5
    populations of 50 individuals on each grid from 64^2 to 2048^2, RMSE
    against the Pagie polynomial.  A step evaluates the 5 populations on one
    grid (DAG build from device-resident tokens, plan, fill, fused fitness);
    per grid it reports the mean and spread of one population's evaluation
    and the credited node-evals/s.  The paper's seconds (other hardware,
    other systems) are context only."""
    import numpy as np
    import torch

    from paper_2103_07512_amd import popgen as pg
    from paper_2103_07512_amd import tgp

    dev = torch.device("cuda:0")
    ctx = tgp.Context(0)
    pops = [pg.ramped_half_and_half(50, 2, 12, 20 + r, pg.F18, 2) for r in range(5)]
    dev_tok = [(torch.from_numpy(p.tokens.view(np.uint8).copy()).to(dev), torch.from_numpy(p.offsets.copy()).to(dev))
               for p in pops]
    target_pop = pg.population_from_texts([PAGIE])
    out = torch.empty(50, dtype=torch.float64, device=dev)
    rows, tot_credited, tot_s = [], 0, 0.0
    for side in (64, 128, 256, 512, 1024, 2048):
        dom = tgp.Domain(ctx, (side, side))
        tdag = tgp.build_dag(ctx, target_pop)
        target = torch.empty(1, dom.cases, dtype=torch.float32, device=dev)
        tgp.evaluate(ctx, tdag, dom, target)
        tdag.close()

        def one(r):
            dag = tgp.Dag(ctx, dev_tok[r][0], dev_tok[r][1], 50, 1)
            tgp.fitness(ctx, dag, dom, target, tgp.RMSE, out)
            return dag

        for _ in range(args.warmup):
            for r in range(5):
                one(r).close()
        torch.cuda.synchronize()
        times, credited = [], 0
        for _ in range(args.steps):
            for r in range(5):
                t0 = time.perf_counter()
                dag = one(r)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                credited += dag.stats()["dag_nodes"] * dom.cases
                dag.close()
        s_sum = float(np.sum(times))
        rows.append({"side": side, "cases": dom.cases, "ms_per_population_mean": 1e3 * float(np.mean(times)),
                     "ms_per_population_std": 1e3 * float(np.std(times)),
                     "ms_per_5_populations": 5e3 * float(np.mean(times)),
                     "node_evals_per_s": credited / s_sum})
        tot_credited += credited
        tot_s += s_sum
        print(f"[p] {side}^2: {rows[-1]['ms_per_population_mean']:.3f} ms per population", file=sys.stderr,
              flush=True)
    line = {
        "metric": "node-evals/s (DAG nodes x fitness cases / s) over the six grids",
        "value": tot_credited / tot_s,
        "unit": "node-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * tot_s / (args.steps * 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["p"], "populations": 5, "individuals": 50,
                   "tree_nodes": [int(len(p.tokens)) for p in pops]},
        "roofline": None,
        "cpu_baseline": None,
        "detail": {"by_grid": rows},
    }
    print(json.dumps(line), flush=True)


def bench_evolve(args):
    """Generations of a GP run that never leave the GPU: DAG build from the
    device-resident population, plan, fitness, then tgp_breed on the device
    from that fitness.  Reports node-evals/s over whole generations and the
    breeding kernels' times; the oracle's breeding (host) is timed beside it."""
    import numpy as np
    import torch

    from oracle import breed as oracle_breed
    from paper_2103_07512_amd import popgen as pg
    from paper_2103_07512_amd import tgp

    dev = torch.device("cuda:0")
    pop, dspec, tspec, loss = load_workload("c3")
    F = [pg.OP_CODE[f] for f in pg.F18]
    params = dict(functions=F, tournament=3, p_crossover=0.8, p_mutation=0.1, max_depth=12,
                  max_mutation_depth=4, ndim=2)
    ctx = tgp.Context(0)
    dom = tgp.Domain(ctx, dspec.shape)

    def render(tree):
        d = tgp.Dag(ctx, tree, np.array([0, len(tree)], np.int64), 1)
        v = torch.empty(1, dom.cases, dtype=torch.float32, device=dev)
        tgp.evaluate(ctx, d, dom, v)
        return v[0].cpu().numpy() if bool(torch.isfinite(v).all()) else None

    _, target = pg.pick_target(tspec, render)
    target_dev = torch.from_numpy(target).to(dev)
    out = torch.empty(pop.n_individuals, dtype=torch.float64, device=dev)
    ctx.set_timing(True)
    parents = pop
    rows = []
    keep = None
    n_gen = args.warmup + args.steps
    torch.cuda.synchronize()
    for g in range(n_gen):
        if g == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        tg = time.perf_counter()
        dag = tgp.Dag(ctx, parents) if isinstance(parents, tgp.Offspring) else tgp.Dag.from_population(ctx, parents)
        tgp.fitness(ctx, dag, dom, target_dev, loss, out)
        tm_eval = ctx.last_timing()
        st = dag.stats()
        dag.close()
        tb = time.perf_counter()
        child = tgp.Offspring(ctx, parents, out, seed=1000 + g, n_offspring=pop.n_individuals, **params)
        tm = ctx.last_timing()
        torch.cuda.synchronize()
        rows.append(dict(dag_nodes=st["dag_nodes"], tree_nodes=st["tree_nodes"],
                         breed_host_ms=(time.perf_counter() - tb) * 1e3,
                         generation_ms=(time.perf_counter() - tg) * 1e3,
                         interp_ms=tm_eval["interp_ms"], plan_ms=tm_eval["plan_ms"],
                         build_dag_ms=tm_eval["build_dag_ms"],
                         breed_shape_ms=tm["breed_shape_ms"], breed_plan_ms=tm["breed_plan_ms"],
                         breed_write_ms=tm["breed_write_ms"], offspring_tokens=child.n_tokens,
                         best=float(np.nanmin(out.cpu().numpy()))))
        keep = parents
        parents = child
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = rows[args.warmup:]
    credited = sum(r["dag_nodes"] for r in timed) * dom.cases
    ms = wall / args.steps * 1e3
    # the breeding kernels: parent tokens read and the shapes written (shape),
    # the child trees read from the parents and written (copy), per launch
    last = timed[-1]
    par_tokens = sum(r["tree_nodes"] for r in timed) / len(timed)
    kid_tokens = float(np.mean([r["offspring_tokens"] for r in timed]))
    shape_ms = float(np.mean([r["breed_shape_ms"] for r in timed]))
    write_ms = float(np.mean([r["breed_write_ms"] for r in timed]))
    shape_bytes = par_tokens * (8 + 12)
    write_bytes = kid_tokens * 16
    # oracle breeding of one generation on the host, from the last parents
    cpu = None
    if not args.no_cpu_baseline and isinstance(keep, tgp.Offspring):
        toks, offs = keep.to_host()
        fit = out.cpu().numpy()
        c0 = time.perf_counter()
        oracle_breed.breed(toks, offs, pop.n_channels, fit, 1, pop.n_individuals,
                           tries=8, use_const=True, **{k: v for k, v in params.items()})
        cpu_s = time.perf_counter() - c0
        cpu = {"value": pop.n_individuals / cpu_s, "unit": "offspring/s", "cores": 1, "kind": "oracle",
               "sample": f"one generation of {pop.n_individuals} offspring (x{pop.n_channels} trees) bred "
                         f"by the oracle from the device-bred parents"}
    breed_ms = float(np.mean([r["breed_shape_ms"] + r["breed_plan_ms"] + r["breed_write_ms"] for r in timed]))
    line = {
        "metric": METRIC, "value": credited / (ms / 1e3), "unit": "node-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["evolve"], "individuals": pop.n_individuals,
                   "channels": pop.n_channels, "domain": list(dspec.shape), "generations": args.steps},
        "roofline": {"bound": "hbm", "achieved": max(shape_bytes / (shape_ms / 1e3), write_bytes / (write_ms / 1e3)) / 1e9
                     if shape_ms > 0 and write_ms > 0 else None,
                     "peak": 8000.0, "unit": "GB/s", "frac": None, "traffic": None,
                     "kernel": "breeding: k_shape (20 B per parent token) and k_breed_write (16 B per "
                               "offspring token); the larger of the two rates",
                     "kernel_ms": {"shape": shape_ms, "write": write_ms}},
        "cpu_baseline": cpu,
        "detail": {"generations": rows, "breed_device_ms": breed_ms,
                   "breed_offspring_per_s": pop.n_individuals / (breed_ms / 1e3) if breed_ms > 0 else None,
                   "breed_host_ms": float(np.mean([r["breed_host_ms"] for r in timed]))},
    }
    if line["roofline"]["achieved"] is not None:
        line["roofline"]["frac"] = line["roofline"]["achieved"] / 8000.0
    print(json.dumps(line), flush=True)


def kernel_source_hash():
    """Hash of the sources that make up the fused interpreter kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_interp.hip", "interp_gen.inc", "ops_device.h", "tgp_internal.h", "fp32_math.h",
              "div_magic.h"):
        with open(os.path.join(ROOT, "paper_2103_07512_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded(profile, tag):
    """A record line ('TAG {json}') of a committed counter summary, when the
    counters were taken on the kernel as it is now (else None)."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for ln in fh:
            if ln.startswith(tag + " "):
                rec = json.loads(ln[len(tag) + 1:])
    if not rec or rec.get("kernel_source") != kernel_source_hash():
        return None
    rec["source"] = "profiles/" + profile
    return rec


def serve_c5(generations, loads, with_plain, warm_generations=2, log=None, configure=None):
    """The serving workload: 16 GP runs, one request per generation each.

    Pass 1 runs the closed loop (submit, wait, breed the next generation from
    the returned fitness) and records every population.  Breeding is
    deterministic given the fitness, so later passes replay the recorded
    populations with the same per-run order:
      * capacity: every run resubmits as soon as its previous request ends;
      * loaded: exponential think times between a result and the next
        request, with the mean set so that the offered work is `load` times
        the measured capacity; latency percentiles (submit to fitness on the
        host) over the requests after the warm-up generations;
      * plain: one tgp_fitness per request, one after the other.
    Each pass starts from an empty server.  Returns a dict.
    """
    import threading

    import numpy as np
    import torch

    from paper_2103_07512_amd import popgen as pg
    from paper_2103_07512_amd import tgp

    def say(*a):
        if log:
            print(*a, file=log, flush=True)

    dev = torch.device("cuda:0")
    runs = pg.workload_c5()
    ctx = tgp.Context(0)
    doms, targets = {}, {}
    for spec in runs:
        dom = tgp.Domain(ctx, spec.shape)

        def render(tree, dom=dom):
            d = tgp.Dag(ctx, tree, np.array([0, len(tree)], np.int64), 1)
            v = torch.empty(1, dom.cases, dtype=torch.float32, device=dev)
            tgp.evaluate(ctx, d, dom, v)
            return v[0].cpu().numpy() if bool(torch.isfinite(v).all()) else None

        _, tgt = pg.pick_target(spec.target, render)
        doms[spec.run] = dom
        targets[spec.run] = torch.from_numpy(tgt).to(dev)
    torch.cuda.synchronize()

    pops = {spec.run: [] for spec in runs}
    fits = {spec.run: [] for spec in runs}

    def closed_loop(srv, spec):
        pop = spec.first_population()
        rng = pg.Rng(spec.breed_seed)
        for g in range(generations):
            pops[spec.run].append(pop)
            t = srv.submit(spec.run, pop, doms[spec.run], targets[spec.run], tgp.RMSE)
            f = srv.wait(t).copy()
            fits[spec.run].append(f)
            if g + 1 < generations:
                pop = pg.breed(pop, rng, pg.F18, 2, max_depth=spec.max_depth, fitness=f)

    def run_threads(target_fn):
        # a request that fails ends its run's thread: report it instead of
        # timing the runs that are left
        errors = []

        def guarded(spec):
            try:
                target_fn(spec)
            except Exception as e:  # noqa: BLE001
                errors.append(f"run {spec.run}: {e}")

        th = [threading.Thread(target=guarded, args=(spec,)) for spec in runs]
        t0 = time.perf_counter()
        for x in th:
            x.start()
        for x in th:
            x.join()
        if errors:
            raise RuntimeError(f"{len(errors)} serving run(s) failed; first: {errors[0]}")
        return time.perf_counter() - t0

    say("c5: closed loop with breeding")
    srv = tgp.Server(ctx, 0, 16)
    wall_gen = run_threads(lambda spec: closed_loop(srv, spec))
    srv.close()

    def replay(think_mean_s):
        srv = tgp.Server(ctx, 0, 16)
        if configure:
            configure(srv)
        infos, same = [], [True]
        lock = threading.Lock()

        def one(spec):
            rng = np.random.default_rng(spec.think_seed)
            for g, pop in enumerate(pops[spec.run]):
                t = srv.submit(spec.run, pop, doms[spec.run], targets[spec.run], tgp.RMSE)
                f = srv.wait(t)
                info = srv.ticket_info(t)
                ok = np.array_equal(np.asarray(f).view(np.uint64), fits[spec.run][g].view(np.uint64))
                with lock:
                    infos.append((g, info))
                    same[0] &= bool(ok)
                if think_mean_s > 0:
                    time.sleep(float(rng.exponential(think_mean_s)))

        wall = run_threads(one)
        st = srv.stats()
        srv.close()
        credited = sum(i["credited_node_evals"] for _, i in infos)
        lat = np.array([i["latency_ms"] for g, i in infos if g >= warm_generations])
        counted = int(lat.size)
        ph = {"to_admission": [i["admit_ms"] - i["submit_ms"] for _, i in infos],
              "prep": [i["prep_ms"] for _, i in infos],
              "admitted_to_first_step": [i["start_ms"] - i["admit_ms"] for _, i in infos],
              "running": [i["done_ms"] - i["start_ms"] for _, i in infos]}
        phases = {k: {"mean_ms": float(np.mean(v)), "p50_ms": float(np.median(v))} for k, v in ph.items()}
        return dict(wall_s=wall, node_evals_per_s=credited / wall, requests=len(infos),
                    requests_counted=counted, phases=phases,
                    p50_ms=float(np.percentile(lat, 50)) if lat.size else None,
                    p99_ms=float(np.percentile(lat, 99)) if lat.size else None,
                    same_as_closed_loop=same[0], server=st, credited=credited)

    say("c5: capacity")
    cap = replay(0.0)
    capacity = cap["node_evals_per_s"]
    n_req = cap["requests"]
    mean_work = cap["credited"] / n_req
    out = {"generations": generations, "runs": len(runs), "requests": n_req,
           "closed_loop_wall_s": wall_gen, "capacity": cap, "loaded": []}
    for rho in loads:
        think = len(runs) * mean_work / (rho * capacity)
        say(f"c5: offered load {rho} (mean think {think * 1e3:.1f} ms)")
        r = replay(think)
        r.update(offered_load=rho, mean_think_ms=think * 1e3)
        out["loaded"].append(r)
    if with_plain:
        say("c5: plain")
        total, t0 = 0, time.perf_counter()
        o = torch.empty(2048, dtype=torch.float64, device=dev)
        agree = True
        ctx.set_timing(True)
        host_ms = gpu_ms = 0.0
        for spec in runs:
            for g, pop in enumerate(pops[spec.run]):
                dag = tgp.build_dag(ctx, pop)
                tgp.fitness(ctx, dag, doms[spec.run], targets[spec.run], tgp.RMSE, o)
                f = o[:pop.n_individuals].cpu().numpy()
                tm = ctx.last_timing()
                host_ms += tm["build_dag_ms"] + tm["plan_ms"]
                gpu_ms += tm["fill_ms"] + tm["interp_ms"] + tm["finalize_ms"]
                total += dag.stats()["dag_nodes"] * doms[spec.run].cases
                a, b = f, fits[spec.run][g]
                fin = np.isfinite(b)
                agree &= bool(np.array_equal(np.isfinite(a), fin) and
                              np.all(np.abs(a[fin] - b[fin]) <= 1e-6 * np.abs(b[fin])))
                dag.close()
        wall = time.perf_counter() - t0
        ctx.set_timing(False)
        out["plain"] = dict(wall_s=wall, node_evals_per_s=total / wall, agree_within_1e6=agree,
                            build_and_plan_ms=host_ms, kernels_ms=gpu_ms)
        out["served_over_plain"] = capacity / (total / wall)
    return out


def bench_c5(args):
    loads = [float(x) for x in args.loads.split(",") if x.strip()]
    res = serve_c5(args.generations, loads, not args.no_plain, log=sys.stderr)
    cap = res["capacity"]
    line = {
        "metric": METRIC, "value": cap["node_evals_per_s"], "unit": "node-evals/s", "n_gpus": 1,
        "steps": res["requests"], "warmup": 0, "ms_per_step": cap["wall_s"] * 1e3 / res["requests"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"], "runs": res["runs"], "generations": res["generations"]},
        "latency": [{"offered_load": r["offered_load"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                     "node_evals_per_s": r["node_evals_per_s"]} for r in res["loaded"]],
        "detail": res,
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
    ap.add_argument("--lds-stack", action="store_true", help="operand stack in LDS instead of registers")
    ap.add_argument("--generations", type=int, default=20, help="serving workload: generations per run")
    ap.add_argument("--loads", default="0.5,0.7,0.9", help="serving workload: offered loads")
    ap.add_argument("--no-plain", action="store_true", help="serving workload: skip the plain pass")
    ap.add_argument("--no-latency", action="store_true",
                    help="default workload: skip the short serving run that gives p50/p99 latency")
    ap.add_argument("--latency-generations", type=int, default=22,
                    help="default workload: generations per run of the serving leg (16 runs, the "
                         "first 2 generations not counted: 320 requests counted per offered load)")
    ap.add_argument("--no-batched", action="store_true",
                    help="default workload: skip the batched-vs-plain leg (64 populations)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build evaluates a population on a single MI355X "
              f"and has no multi-GPU path (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "evolve":
        return bench_evolve(args)
    if args.workload == "p":
        return bench_p(args)

    import numpy as np
    import torch

    from paper_2103_07512_amd import popgen as pg
    from paper_2103_07512_amd import tgp

    dev = torch.device("cuda:0")
    pop, dspec, tspec, loss = load_workload(args.workload)
    ctx = tgp.Context(0)
    ctx.set_tuning(args.cases_per_lane, args.tiles_per_item)
    ctx.set_plan(not args.no_reorder, args.cache_access_cost)
    ctx.set_stack(args.lds_stack)
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

    # Evaluation only (DAG and plan kept from the last step) and end to end
    # (host tokens in, host fitness out, PCIe copies included).
    dag = tgp.Dag(ctx, tok_dev, off_dev, pop.n_individuals, pop.n_channels)
    tgp.fitness(ctx, dag, dom, target_dev, loss, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        tgp.fitness(ctx, dag, dom, target_dev, loss, out)
    torch.cuda.synchronize()
    eval_only_ms = (time.perf_counter() - t1) / args.steps * 1e3
    dag.close()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        d2 = tgp.Dag(ctx, pop.tokens, pop.offsets, pop.n_individuals, pop.n_channels)
        tgp.fitness(ctx, d2, dom, target_dev, loss, out)
        host_fit = out.cpu().numpy()
        d2.close()
    end_to_end_ms = (time.perf_counter() - t1) / args.steps * 1e3

    ms = wall / args.steps * 1e3
    credited = stats["dag_nodes"] * dom.cases
    value = credited / (ms / 1e3)
    interp_ms = float(np.mean([t["interp_ms"] for t in times]))
    fill_ms = float(np.mean([t["fill_ms"] for t in times]))
    d_last = tgp.Dag(ctx, tok_dev, off_dev, pop.n_individuals, pop.n_channels)
    per_case, per_case_all = algorithmic_lane_ops(d_last.export())
    d_last.close()
    alg = per_case * dom.cases  # every DAG node is evaluated over every case of the grid
    achieved = alg / ((fill_ms + interp_ms) / 1e3) / 1e12
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
                     "unit": "T lane-op/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_interp evaluation launches of a step: the cache-fill launches and "
                               "the fused fitness launch (root programs with the error reduction)",
                     "kernel_ms": fill_ms + interp_ms, "kernel_ms_fitness_launch": interp_ms,
                     "kernel_ms_fill": fill_ms,
                     "work": "algorithmic lane-ops = cases x sum over variable-dependent DAG function "
                             "nodes of a fixed per-operator cost (bench.py ALG_COST); folded "
                             "variable-free subtrees count 0",
                     "algorithmic_lane_ops": alg,
                     "frac_counting_folded_nodes": per_case_all * dom.cases / ((fill_ms + interp_ms) / 1e3)
                     / 1e12 / VALU_PEAK_TOPS},
        "detail": {
            "phases_ms": {k: float(np.mean([t[k] for t in times]))
                          for k in ("build_dag_ms", "plan_ms", "plan_fold_ms", "plan_decide_ms", "plan_emit_ms", "fill_ms", "interp_ms", "finalize_ms")},
            "launch": {k: times[-1][k] for k in ("interp_items", "cases_per_lane", "tiles_per_item")},
            "work": work,
            "executed_node_evals_per_s": work["executed_node_evals"] / (ms / 1e3),
            "eval_only_ms": eval_only_ms,
            "end_to_end_host_ms": end_to_end_ms,
            "end_to_end_host_node_evals_per_s": stats["dag_nodes"] * dom.cases / (end_to_end_ms / 1e3),
            "finite_fitness": int(np.isfinite(fit).sum()),
        },
    }
    if args.calibrate_copy:
        # A copy of known size for scaling the FETCH_SIZE / WRITE_SIZE counters.
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    traffic = recorded("k_interp_c3_hbm_traffic.md", "TRAFFIC")
    if traffic is not None:
        line["roofline"]["traffic"] = traffic["bytes_per_launch"]
        line["roofline"]["traffic_source"] = traffic["source"]
    # the cache path: the fill launches' algorithmic bytes (the rows they
    # write) over their HIP-event time, against the 8 TB/s HBM peak; the
    # counters' byte count (reads of lower rows included) beside it
    cp = {"kernel": "k_interp cache-fill launches of a step (one per cache level)",
          "algorithmic_write_bytes": work["cache_bytes_written"], "ms": fill_ms,
          "achieved_GB_per_s": work["cache_bytes_written"] / (fill_ms / 1e3) / 1e9 if fill_ms > 0 else None,
          "peak_GB_per_s": 8000.0}
    cp["frac"] = cp["achieved_GB_per_s"] / cp["peak_GB_per_s"] if cp["achieved_GB_per_s"] else None
    if traffic is not None and fill_ms > 0:
        cp["measured_bytes"] = traffic["fill_fetch_bytes"] + traffic["fill_write_bytes"]
        cp["measured_GB_per_s"] = cp["measured_bytes"] / (fill_ms / 1e3) / 1e9
        cp["source"] = traffic["source"]
    line["cache_path"] = cp
    issue = recorded("k_interp_c3_valu.md", "VALU")
    if issue is not None:
        # the fitness launch's issue counters, beside the algorithmic fraction
        line["roofline"]["counters_fitness_launch"] = {
            k: issue[k] for k in ("valu_insts", "salu_insts", "branch_insts", "launch_ms", "valubusy_pct", "source")}
    if not args.no_latency:
        loads = [float(x) for x in args.loads.split(",") if x.strip()]
        res = serve_c5(args.latency_generations, loads, False)
        line["latency"] = {
            "workload": WORKLOADS["c5"] + f"; {args.latency_generations} generations per run, "
                        f"the first 2 not counted",
            "by_offered_load": [{"offered_load": r["offered_load"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                                 "requests_counted": r["requests_counted"],
                                 "node_evals_per_s": r["node_evals_per_s"],
                                 "same_as_closed_loop": r["same_as_closed_loop"]} for r in res["loaded"]],
            "served_node_evals_per_s_at_capacity": res["capacity"]["node_evals_per_s"]}
        for r in res["loaded"]:
            if abs(r["offered_load"] - 0.7) < 1e-9:
                line["latency"].update(offered_load=0.7, p50_ms=r["p50_ms"], p99_ms=r["p99_ms"])
    if not args.no_batched:
        c4 = run_c4(argparse.Namespace(steps=max(3, args.steps // 2), warmup=1))
        dt = c4["detail"]
        line["batched"] = {
            "workload": WORKLOADS["c4"], "batched_node_evals_per_s": c4["value"],
            "plain_node_evals_per_s": dt["plain_value"],
            "end_to_end_batched_over_plain": dt["batched_over_plain"],
            "eval_only_ms": dt["eval_only_ms"],
            "eval_only_batched_over_plain": dt["eval_only_batched_over_plain"],
            "autotuned": dt["autotune"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pop, dspec, stats["dag_nodes"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
