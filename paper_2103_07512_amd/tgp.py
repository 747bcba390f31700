"""Python binding of libtgp (ctypes): argument marshalling only.

Every step of the evaluation runs in the HIP library; this module converts
numpy / torch arguments to the pointers and sizes of the C ABI in
include/tgp.h and turns non-zero status codes into exceptions.  Device
buffers are torch tensors on the context's GPU; the context orders its work
on the current torch stream of that device unless told otherwise.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_HERE, "libtgp.so")

TOKEN_DTYPE = np.dtype([("op", "u1"), ("var", "u1"), ("pad", "<u2"), ("value", "<f4")])
RMSE, MSE = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
STATUS = {0: "TGP_OK", -1: "TGP_EINVAL", -2: "TGP_EPARSE", -3: "TGP_EDEPTH", -4: "TGP_EOP",
          -5: "TGP_ENOMEM", -6: "TGP_EHIP", -7: "TGP_ESHAPE", -8: "TGP_EBUSY"}


# Set when the interpreter starts to exit: handles that are still open are
# then left to the process exit (destroying them would call into a HIP
# runtime that torch may already have torn down).
_exiting = False


def _mark_exiting():
    global _exiting
    _exiting = True


atexit.register(_mark_exiting)


class TgpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Population(ctypes.Structure):
    _fields_ = [("n_individuals", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("tokens", ctypes.c_void_p),
                ("memory", ctypes.c_int32)]


class DagStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "tree_nodes", "tree_internal", "dag_nodes", "dag_internal", "shared_internal",
        "max_stack", "max_height", "n_roots", "max_var")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class WorkStats(ctypes.Structure):
    _fields_ = [("credited_node_evals", ctypes.c_int64), ("executed_node_evals", ctypes.c_int64),
                ("cached_nodes", ctypes.c_int64), ("stack_spills", ctypes.c_int64),
                ("cache_levels", ctypes.c_int64),
                ("programs", ctypes.c_int64), ("instructions", ctypes.c_int64),
                ("algorithmic_valu", ctypes.c_double), ("executed_valu_fill", ctypes.c_double),
                ("executed_valu_roots", ctypes.c_double), ("cache_bytes_read", ctypes.c_int64),
                ("cache_bytes_written", ctypes.c_int64), ("folded_nodes", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("build_dag_ms", ctypes.c_double), ("plan_ms", ctypes.c_double),
                ("fill_ms", ctypes.c_double), ("interp_ms", ctypes.c_double),
                ("finalize_ms", ctypes.c_double), ("interp_items", ctypes.c_int64),
                ("cases_per_lane", ctypes.c_int32), ("tiles_per_item", ctypes.c_int32),
                ("plan_fold_ms", ctypes.c_double), ("plan_decide_ms", ctypes.c_double),
                ("plan_emit_ms", ctypes.c_double), ("breed_shape_ms", ctypes.c_double),
                ("breed_plan_ms", ctypes.c_double), ("breed_write_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class BreedParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_offspring", ctypes.c_int32), ("tournament", ctypes.c_int32),
                ("p_crossover", ctypes.c_double), ("p_mutation", ctypes.c_double),
                ("max_depth", ctypes.c_int32), ("max_mutation_depth", ctypes.c_int32),
                ("crossover_tries", ctypes.c_int32), ("ndim", ctypes.c_int32),
                ("use_constants", ctypes.c_int32), ("n_functions", ctypes.c_int32),
                ("functions", ctypes.c_void_p)]


class Job(ctypes.Structure):
    _fields_ = [("dag", ctypes.c_void_p), ("domain", ctypes.c_void_p), ("target_dev", ctypes.c_void_p),
                ("loss", ctypes.c_int32), ("out_dev", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("jobs", ctypes.c_int64), ("pairs", ctypes.c_int64), ("items", ctypes.c_int64),
                ("levels", ctypes.c_int64), ("captures", ctypes.c_int64), ("replays", ctypes.c_int64),
                ("credited_node_evals", ctypes.c_int64), ("pack_ms", ctypes.c_double),
                ("tiles_per_item", ctypes.c_int32), ("cases_per_lane", ctypes.c_int32),
                ("persistent", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("cases_per_lane", ctypes.c_int32), ("tiles_cap", ctypes.c_int32),
                ("persistent", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("stack_lds", ctypes.c_int32), ("best_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
I32, I64 = ctypes.c_int32, ctypes.c_int64

# (name, restype, argtypes) of every exported function of include/tgp.h
class TicketInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slabs", ctypes.c_int32),
                ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("prep_ms", ctypes.c_double),
                ("dag_nodes", ctypes.c_int64),
                ("credited_node_evals", ctypes.c_int64), ("cache_hits", ctypes.c_int32),
                ("cache_new", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "completed", "failed", "steps", "slabs", "cache_hits", "cache_new",
        "evictions", "entries", "bytes_in_use", "bytes_peak", "bytes_capacity",
        "credited_node_evals")] + [("max_active_seen", ctypes.c_int32), ("pad", ctypes.c_int32),
                                   ("step_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_ if n != "pad"}


SIGNATURES = [
    ("tgp_ctx_create", I32, [ctypes.c_int, P, PP]),
    ("tgp_ctx_destroy", None, [P]),
    ("tgp_ctx_set_stream", I32, [P, P]),
    ("tgp_last_error", ctypes.c_char_p, [P]),
    ("tgp_ctx_set_cache_budget", I32, [P, ctypes.c_size_t]),
    ("tgp_ctx_set_tuning", I32, [P, I32, I32]),
    ("tgp_ctx_set_plan", I32, [P, I32, ctypes.c_double]),
    ("tgp_ctx_set_stack", I32, [P, I32]),
    ("tgp_ctx_set_folding", I32, [P, I32]),
    ("tgp_ctx_set_hashing", I32, [P, I32]),
    ("tgp_ctx_set_rewrite", I32, [P, I32]),
    ("tgp_debug_set_hash_bits", I32, [I32]),
    ("tgp_domain_create", I32, [P, I32, P, P, P, PP]),
    ("tgp_domain_destroy", None, [P]),
    ("tgp_domain_cases", I64, [P]),
    ("tgp_build_dag", I32, [P, ctypes.POINTER(_Population), PP]),
    ("tgp_breed", I32, [P, ctypes.POINTER(_Population), P, ctypes.POINTER(BreedParams), PP]),
    ("tgp_offspring_population", I32, [P, ctypes.POINTER(_Population)]),
    ("tgp_offspring_export", I32, [P, ctypes.POINTER(ctypes.c_int64), P, P]),
    ("tgp_offspring_destroy", None, [P]),
    ("tgp_dag_stats_get", I32, [P, ctypes.POINTER(DagStats)]),
    ("tgp_dag_export", I32, [P, P, P, P, P, P]),
    ("tgp_dag_destroy", None, [P]),
    ("tgp_evaluate", I32, [P, P, P, P]),
    ("tgp_fitness", I32, [P, P, P, P, I32, P]),
    ("tgp_fitness_noalloc", I32, [P, P, P, P, I32, P]),
    ("tgp_last_work", I32, [P, ctypes.POINTER(WorkStats)]),
    ("tgp_ctx_set_timing", I32, [P, I32]),
    ("tgp_last_timing", I32, [P, ctypes.POINTER(Timing)]),
    ("tgp_batch_create", I32, [P, I32, PP]),
    ("tgp_batch_run", I32, [P, I32, ctypes.POINTER(Job)]),
    ("tgp_batch_destroy", None, [P]),
    ("tgp_fitness_batch", I32, [P, I32, ctypes.POINTER(Job)]),
    ("tgp_ctx_set_batch_form", I32, [P, I32]),
    ("tgp_batch_stats_get", I32, [P, ctypes.POINTER(BatchStats)]),
    ("tgp_autotune", I32, [P, I32, ctypes.POINTER(Job), ctypes.c_char_p, ctypes.POINTER(TuneResult)]),
    ("tgp_server_create", I32, [P, ctypes.c_size_t, I32, PP]),
    ("tgp_server_destroy", None, [P]),
    ("tgp_server_set_slab_work", I32, [P, ctypes.c_double]),
    ("tgp_server_set_launch", I32, [P, I32, I32]),
    ("tgp_server_submit", I32, [P, I64, ctypes.POINTER(_Population), P, P, I32, P,
                                ctypes.POINTER(I64)]),
    ("tgp_server_wait", I32, [P, I64, I64]),
    ("tgp_server_end_run", I32, [P, I64]),
    ("tgp_server_last_error", ctypes.c_char_p, [P]),
    ("tgp_server_ticket_info", I32, [P, I64, ctypes.POINTER(TicketInfo)]),
    ("tgp_server_stats_get", I32, [P, ctypes.POINTER(ServerStats)]),
]


def lib():
    """Load libtgp.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(f"{LIBRARY} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIBRARY)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != 0:
        msg = lib().tgp_last_error(ctx)
        raise TgpError(status, msg.decode() if msg else "")


def _stream_of(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """tgp_ctx: a device, a HIP stream and the library's scratch memory."""

    def __init__(self, device: int = 0, stream=None):
        self.device = device
        h = ctypes.c_void_p()
        s = _stream_of(device) if stream is None else ctypes.c_void_p(stream)
        _check(lib().tgp_ctx_create(device, s, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().tgp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(lib().tgp_ctx_set_stream(self.h, ctypes.c_void_p(stream)), self.h)

    def set_cache_budget(self, nbytes: int):
        _check(lib().tgp_ctx_set_cache_budget(self.h, nbytes), self.h)

    def set_tuning(self, cases_per_lane: int = 0, tiles_per_item: int = 0):
        _check(lib().tgp_ctx_set_tuning(self.h, cases_per_lane, tiles_per_item), self.h)

    def set_plan(self, reorder_children: bool = True, cache_access_cost: float = 20.0):
        _check(lib().tgp_ctx_set_plan(self.h, 1 if reorder_children else 0, cache_access_cost), self.h)

    def set_hashing(self, commutative: bool = False):
        """Hash-cons up to the operand order of commuting operators."""
        _check(lib().tgp_ctx_set_hashing(self.h, 1 if commutative else 0), self.h)

    def set_rewrite(self, on: bool = True):
        """Apply the identity rewrites while hash-consing (tgp_ctx_set_rewrite)."""
        _check(lib().tgp_ctx_set_rewrite(self.h, 1 if on else 0), self.h)

    def set_folding(self, on: bool = True):
        """Evaluate constant subtrees once and use their values as constants."""
        _check(lib().tgp_ctx_set_folding(self.h, 1 if on else 0), self.h)

    def set_stack(self, lds: bool = False):
        """Operand stack in LDS (True) or in registers (False, the default)."""
        _check(lib().tgp_ctx_set_stack(self.h, 1 if lds else 0), self.h)

    def set_batch_form(self, persistent: bool = True):
        _check(lib().tgp_ctx_set_batch_form(self.h, 1 if persistent else 0), self.h)

    def set_timing(self, enable: bool = True):
        _check(lib().tgp_ctx_set_timing(self.h, 1 if enable else 0), self.h)

    def last_timing(self) -> dict:
        t = Timing()
        _check(lib().tgp_last_timing(self.h, ctypes.byref(t)), self.h)
        return t.as_dict()

    def last_work(self) -> dict:
        w = WorkStats()
        _check(lib().tgp_last_work(self.h, ctypes.byref(w)), self.h)
        return w.as_dict()


def debug_set_hash_bits(bits: int):
    _check(lib().tgp_debug_set_hash_bits(bits))


class Domain:
    """tgp_domain: an N-D grid of fitness cases (coordinates on the device)."""

    def __init__(self, ctx: Context, shape, lo=None, hi=None):
        self.ctx = ctx
        shape = np.ascontiguousarray(shape, dtype=np.int64)
        self.shape = tuple(int(v) for v in shape)
        lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
        hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().tgp_domain_create(ctx.h, len(shape), shape.ctypes.data,
                                       None if lo_a is None else lo_a.ctypes.data,
                                       None if hi_a is None else hi_a.ctypes.data,
                                       ctypes.byref(h)), ctx.h)
        self.h = h
        self.cases = int(lib().tgp_domain_cases(h))

    def close(self):
        # a handle outlived by its context: the context's destruction has
        # already released its device memory (the library must not see it)
        if self.h and not self.ctx.h:
            self.h = None
        if self.h:
            lib().tgp_domain_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def _population_struct(tokens, offsets, n_individuals: int, n_channels: int):
    """(struct, arrays to keep alive) for host numpy arrays or device tensors."""
    pop = _Population()
    pop.n_individuals = n_individuals
    pop.n_channels = n_channels
    keep = []
    if hasattr(tokens, "data_ptr"):          # torch tensors on the device
        pop.memory = MEM_DEVICE
        pop.offsets = offsets.data_ptr()
        pop.tokens = tokens.data_ptr()
    else:
        t = np.ascontiguousarray(tokens, dtype=TOKEN_DTYPE)
        o = np.ascontiguousarray(offsets, dtype=np.int64)
        keep += [t, o]
        pop.memory = MEM_HOST
        pop.offsets = o.ctypes.data
        pop.tokens = t.ctypes.data
    return pop, keep


class Dag:
    """tgp_dag: a population hash-consed on the GPU.  tokens/offsets are host
    arrays, device tensors, or tokens is an Offspring (offsets unused)."""

    def __init__(self, ctx: Context, tokens, offsets=None, n_individuals: int = 0, n_channels: int = 1):
        self.ctx = ctx
        if isinstance(tokens, Offspring):
            pop, keep = tokens.population_struct(), [tokens]
            n_individuals, n_channels = tokens.n_individuals, tokens.n_channels
        else:
            pop, keep = _population_struct(tokens, offsets, n_individuals, n_channels)
        h = ctypes.c_void_p()
        _check(lib().tgp_build_dag(ctx.h, ctypes.byref(pop), ctypes.byref(h)), ctx.h)
        self.h = h
        self.n_individuals = n_individuals
        self.n_channels = n_channels

    @staticmethod
    def from_population(ctx: Context, pop) -> "Dag":
        return Dag(ctx, pop.tokens, pop.offsets, pop.n_individuals, pop.n_channels)

    def stats(self) -> dict:
        s = DagStats()
        _check(lib().tgp_dag_stats_get(self.h, ctypes.byref(s)))
        return s.as_dict()

    def export(self) -> dict:
        st = self.stats()
        U, R = st["dag_nodes"], st["n_roots"]
        nodes = np.zeros(U, TOKEN_DTYPE)
        children = np.zeros((U, 3), np.int32)
        roots = np.zeros(R, np.int32)
        mult = np.zeros(U, np.int32)
        indeg = np.zeros(U, np.int32)
        _check(lib().tgp_dag_export(self.h, nodes.ctypes.data, children.ctypes.data,
                                    roots.ctypes.data, mult.ctypes.data, indeg.ctypes.data))
        return dict(nodes=nodes, children=children, roots=roots, multiplicity=mult,
                    indegree=indeg, **st)

    def close(self):
        # a handle outlived by its context: the context's destruction has
        # already released its device memory (the library must not see it)
        if self.h and not self.ctx.h:
            self.h = None
        if self.h:
            lib().tgp_dag_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def build_dag(ctx: Context, pop) -> Dag:
    return Dag.from_population(ctx, pop)


def evaluate(ctx: Context, dag: Dag, dom: Domain, out):
    """Per-case values of every tree into out (torch float32, [n_roots, cases])."""
    _check(lib().tgp_evaluate(ctx.h, dag.h, dom.h, ctypes.c_void_p(out.data_ptr())), ctx.h)
    return out


def fitness(ctx: Context, dag: Dag, dom: Domain, target, loss: int, out):
    """RMSE/MSE per individual into out ([n_individuals] float64): a device
    torch tensor (queued, returns at once) or a host array, numpy or CPU
    torch (the call blocks until the values are there)."""
    if isinstance(out, np.ndarray):
        if out.dtype != np.float64 or not out.flags.c_contiguous or not out.flags.writeable:
            raise ValueError("out must be a writeable C-contiguous float64 array")
        if out.size < dag.n_individuals:
            raise ValueError("out is smaller than the number of individuals")
        ptr = out.ctypes.data
    else:
        ptr = out.data_ptr()
    _check(lib().tgp_fitness(ctx.h, dag.h, dom.h, ctypes.c_void_p(target.data_ptr()), loss,
                             ctypes.c_void_p(ptr)), ctx.h)
    return out


def fitness_noalloc(ctx: Context, dag: Dag, dom: Domain, target, loss: int, out):
    """tgp_fitness_noalloc: the same fitness into a device tensor out, with
    no device allocation (the DAG must already be planned for this domain
    size, e.g. by one fitness() call; scratch is a fixed per-GPU array)."""
    _check(lib().tgp_fitness_noalloc(ctx.h, dag.h, dom.h, ctypes.c_void_p(target.data_ptr()), loss,
                                     ctypes.c_void_p(out.data_ptr())), ctx.h)
    return out


def _jobs(jobs):
    """jobs: iterable of (dag, domain, target tensor, loss, out tensor)."""
    jobs = list(jobs)
    arr = (Job * max(1, len(jobs)))()
    for i, (dag, dom, target, loss, out) in enumerate(jobs):
        arr[i].dag = dag.h
        arr[i].domain = dom.h
        arr[i].target_dev = target.data_ptr()
        arr[i].loss = loss
        arr[i].out_dev = out.data_ptr()
    return arr, len(jobs)


class Batch:
    """tgp_batch: persistent, graph-replayed fitness of many populations."""

    def __init__(self, ctx: Context, use_graph: bool = True):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().tgp_batch_create(ctx.h, 1 if use_graph else 0, ctypes.byref(h)), ctx.h)
        self.h = h

    def run(self, jobs):
        arr, n = _jobs(jobs)
        _check(lib().tgp_batch_run(self.h, n, arr), self.ctx.h)

    def stats(self) -> dict:
        st = BatchStats()
        _check(lib().tgp_batch_stats_get(self.h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        # a handle outlived by its context: the context's destruction has
        # already released its device memory (the library must not see it)
        if self.h and not self.ctx.h:
            self.h = None
        if self.h:
            lib().tgp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def fitness_batch(ctx: Context, jobs):
    arr, n = _jobs(jobs)
    _check(lib().tgp_fitness_batch(ctx.h, n, arr), ctx.h)


def autotune(ctx: Context, jobs, cache_path=None) -> dict:
    arr, n = _jobs(jobs)
    r = TuneResult()
    _check(lib().tgp_autotune(ctx.h, n, arr, cache_path.encode() if cache_path else None,
                              ctypes.byref(r)), ctx.h)
    return r.as_dict()


class Server:
    """tgp_server: continuous-batching fitness service for many concurrent GP runs.

    submit() copies a host population and returns a ticket at once; wait()
    blocks (with the GIL released) until that request's fitness values are in
    its output array.  Safe to call from several Python threads.
    """

    def __init__(self, ctx: Context, cache_budget_bytes: int = 0, max_active: int = 0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().tgp_server_create(ctx.h, cache_budget_bytes, max_active, ctypes.byref(h)), ctx.h)
        self.h = h
        self._keep = {}

    def _check(self, status):
        if status != 0:
            msg = lib().tgp_server_last_error(self.h)
            raise TgpError(status, msg.decode() if msg else "")

    def set_slab_work(self, node_evals: float):
        self._check(lib().tgp_server_set_slab_work(self.h, float(node_evals)))

    def set_launch(self, persistent: int = -1, tiles_per_item: int = 0):
        self._check(lib().tgp_server_set_launch(self.h, persistent, tiles_per_item))

    def submit(self, run_id: int, pop, domain: Domain, target, loss: int = RMSE, out=None):
        """Queue pop (popgen.Population or (tokens, offsets, n_ind, n_ch)); returns the ticket.

        out: float64 numpy array of n_individuals (allocated when None),
        written when the request ends; keep it until wait() returns."""
        if isinstance(pop, tuple):
            tokens, offsets, n_ind, n_ch = pop
        else:
            tokens, offsets, n_ind, n_ch = pop.tokens, pop.offsets, pop.n_individuals, pop.n_channels
        t = np.ascontiguousarray(tokens, dtype=TOKEN_DTYPE)
        o = np.ascontiguousarray(offsets, dtype=np.int64)
        if out is None:
            out = np.empty(n_ind, np.float64)
        assert out.dtype == np.float64 and out.flags.c_contiguous and out.size >= n_ind
        p = _Population()
        p.n_individuals = n_ind
        p.n_channels = n_ch
        p.offsets = o.ctypes.data
        p.tokens = t.ctypes.data
        p.memory = MEM_HOST
        ticket = I64()
        self._check(lib().tgp_server_submit(self.h, run_id, ctypes.byref(p), domain.h,
                                            ctypes.c_void_p(target.data_ptr()), loss,
                                            out.ctypes.data, ctypes.byref(ticket)))
        self._keep[ticket.value] = (out, target, domain)
        return ticket.value

    def wait(self, ticket: int, timeout_us: int = -1):
        """The request's fitness array; TgpError (status TGP_EBUSY) on time-out."""
        self._check(lib().tgp_server_wait(self.h, ticket, timeout_us))
        return self._keep.pop(ticket)[0]

    def end_run(self, run_id: int):
        self._check(lib().tgp_server_end_run(self.h, run_id))

    def ticket_info(self, ticket: int) -> dict:
        t = TicketInfo()
        self._check(lib().tgp_server_ticket_info(self.h, ticket, ctypes.byref(t)))
        return t.as_dict()

    def stats(self) -> dict:
        st = ServerStats()
        self._check(lib().tgp_server_stats_get(self.h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        # (a server keeps contexts of its own, so it is destroyed even when
        # the context it was made from is gone)
        if self.h:
            lib().tgp_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class Offspring:
    """tgp_offspring: one generation bred on the device (tgp_breed) from
    parents (a host Population, an Offspring, or (tokens, offsets,
    n_individuals, n_channels) device tensors) and their fitness (a device
    float64 tensor, or None)."""

    def __init__(self, ctx: Context, parents, fitness=None, *, seed: int, n_offspring: int, functions,
                 tournament: int = 3, p_crossover: float = 0.8, p_mutation: float = 0.1,
                 max_depth: int = 10, max_mutation_depth: int = 4, crossover_tries: int = 8,
                 ndim: int = 2, use_constants: bool = True):
        self.ctx = ctx
        self.h = None
        if isinstance(parents, Offspring):
            pop, keep = parents.population_struct(), [parents]
        elif isinstance(parents, tuple):
            pop, keep = _population_struct(*parents)
        else:
            pop, keep = _population_struct(parents.tokens, parents.offsets, parents.n_individuals,
                                           parents.n_channels)
        codes = np.array([int(f) for f in functions], np.uint8)  # operator codes
        p = BreedParams()
        p.seed = seed & ((1 << 64) - 1)
        p.n_offspring = n_offspring
        p.tournament = tournament
        p.p_crossover = p_crossover
        p.p_mutation = p_mutation
        p.max_depth = max_depth
        p.max_mutation_depth = max_mutation_depth
        p.crossover_tries = crossover_tries
        p.ndim = ndim
        p.use_constants = 1 if use_constants else 0
        p.n_functions = len(codes)
        p.functions = codes.ctypes.data
        fit = fitness.data_ptr() if fitness is not None else None
        h = ctypes.c_void_p()
        _check(lib().tgp_breed(ctx.h, ctypes.byref(pop), fit, ctypes.byref(p), ctypes.byref(h)), ctx.h)
        self.h = h
        self.n_individuals = n_offspring
        self.n_channels = pop.n_channels
        del keep

    def population_struct(self) -> "_Population":
        pop = _Population()
        _check(lib().tgp_offspring_population(self.h, ctypes.byref(pop)))
        return pop

    @property
    def n_tokens(self) -> int:
        n = ctypes.c_int64()
        _check(lib().tgp_offspring_export(self.h, ctypes.byref(n), None, None))
        return n.value

    def to_host(self):
        """(tokens, offsets) as numpy arrays."""
        n = self.n_tokens
        offs = np.zeros(self.n_individuals * self.n_channels + 1, np.int64)
        toks = np.zeros(n, TOKEN_DTYPE)
        m = ctypes.c_int64()
        _check(lib().tgp_offspring_export(self.h, ctypes.byref(m), offs.ctypes.data, toks.ctypes.data),
               self.ctx.h)
        return toks, offs

    def close(self):
        # a handle outlived by its context: the context's destruction has
        # already released its device memory (the library must not see it)
        if self.h and not self.ctx.h:
            self.h = None
        if self.h:
            lib().tgp_offspring_destroy(self.h)
            self.h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def breed(ctx: Context, parents, fitness=None, **params) -> Offspring:
    return Offspring(ctx, parents, fitness, **params)
