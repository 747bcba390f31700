"""FP64 CPU oracle for whole-population GP fitness evaluation.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this package; the product path never does.  It
shares no code with the HIP library and imports nothing from it.

    evaluate(...)   per-case values of every tree (oracle.c, plain FP64 walk,
                    optionally with the FP32-shaped variants and stability flags)
    fitness(...)    RMSE / MSE per individual in FP64 (oracle.c)
    build_dag(...)  Handley's population DAG by hash-consing (dag.py)
    breed.breed(...) one generation of tournament selection, subtree crossover,
                    subtree mutation and reproduction on counter-based draws
                    (breed.py)
"""
from .core import (build, coords, evaluate, fitness, library_path, max_threads,
                   render_target, target_renderer, STABLE, NONFINITE_STABLE, ENVELOPE)
from .dag import build_dag, tree_stack_depth

__all__ = ["build", "coords", "evaluate", "fitness", "library_path", "max_threads",
           "render_target", "target_renderer", "build_dag", "tree_stack_depth", "STABLE", "NONFINITE_STABLE",
           "ENVELOPE"]
