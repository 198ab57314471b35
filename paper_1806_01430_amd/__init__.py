"""Python binding of libofl (GA-driven GPU offload of loop nests, MI355X).

Argument marshalling only: every step of the offload path (verdicts, plans,
kernels, host nests, timing, the GA) runs inside the C-ABI library declared in
``include/ofl.h``.  PyTorch supplies device memory and the stream.  Loading
fails loudly when ``libofl.so`` has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libofl.so")
APPS_DIR = os.path.join(HERE, "apps")

OK = 0
E = {-1: "E_ARG", -2: "E_IO", -3: "E_PARSE", -4: "E_IR", -5: "E_GENE_LEN", -6: "E_GENE_BIT",
     -7: "E_NOT_PARALLEL", -8: "E_BUF", -9: "E_HIP", -10: "E_TIMEOUT", -11: "E_MISMATCH",
     -12: "E_STATE", -13: "E_NOMEM", -14: "E_RANGE", -15: "E_UNSUPPORTED"}
PARALLEL, PARALLEL_REDUCTION, REJECT = 0, 1, 2
R_NONE, R_DATA_DEP, R_EXTERNAL_CALL, R_BREAK = 0, 1, 2, 3
RESIDENT, PER_REGION, SECTIONS = 0, 1, 2
PRESTAGED, KEEP_OUTPUTS, GRAPH, BATCHED, PROGRESS, CONCURRENT = 1, 2, 4, 8, 16, 32
ST_OK, ST_TIMEOUT, ST_FAILED, ST_MISMATCH = 0, 1, 2, 3
BATCH_LOOP, BATCH_GROUPED, BATCH_GROUPED_GRAPH = 0, 1, 2
_NP_DTYPE = {0: np.float32, 1: np.float64, 2: np.uint16}

# names declared in include/ofl.h (checked by the ABI test)
EXPORTS = ["ofl_app_load", "ofl_app_load_json", "ofl_app_free", "ofl_app_info", "ofl_nest_info",
           "ofl_nest_name", "ofl_buf_info", "ofl_buf_name", "ofl_buf_dims", "ofl_set_input", "ofl_mask_to_gene",
           "ofl_plan_transfers", "ofl_run_pattern", "ofl_eval_population", "ofl_ga_run",
           "ofl_ga_run_table", "ofl_read_buffer", "ofl_set_kernel_timing", "ofl_set_kernel_timing_op",
           "ofl_set_kernel_timing_sample", "ofl_kernel_stats",
           "ofl_batch_create", "ofl_batch_free", "ofl_batch_info", "ofl_batch_buf_info", "ofl_batch_buf_dims",
           "ofl_batch_buf_name", "ofl_batch_setup", "ofl_batch_run", "ofl_batch_get_config",
           "ofl_batch_set_config", "ofl_batch_tune", "ofl_sweep19", "ofl_sweep19_noalloc", "ofl_status_str",
           "ofl_last_error"]


class OflError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s (%s): %s" % (what, E.get(code, code), last_error()))


class RunOpts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("flags", ctypes.c_int32), ("deadline_s", ctypes.c_double),
                ("verify_rtol", ctypes.c_double)]


class RunStats(ctypes.Structure):
    _fields_ = [("t_total_s", ctypes.c_double), ("bytes_h2d", ctypes.c_uint64), ("bytes_d2h", ctypes.c_uint64),
                ("n_copies", ctypes.c_int32), ("n_launches", ctypes.c_int32), ("n_host_nests", ctypes.c_int32),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class EvalOpts(ctypes.Structure):
    _fields_ = [("reps", ctypes.c_int32), ("warmup", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("deadline_s", ctypes.c_double), ("verify_rtol", ctypes.c_double)]


class GaParams(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("T", ctypes.c_int32), ("Pc", ctypes.c_double), ("Pm", ctypes.c_double),
                ("p", ctypes.c_double), ("seed", ctypes.c_uint64), ("reps", ctypes.c_int32),
                ("warmup", ctypes.c_int32), ("policy", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("deadline_factor", ctypes.c_double), ("timeout_s", ctypes.c_double),
                ("verify_rtol", ctypes.c_double), ("cache_path", ctypes.c_char_p)]


class GaResult(ctypes.Structure):
    _fields_ = [("best_gene", ctypes.POINTER(ctypes.c_uint8)), ("pop_trace", ctypes.POINTER(ctypes.c_uint8)),
                ("time_trace", ctypes.POINTER(ctypes.c_double)), ("status_trace", ctypes.POINTER(ctypes.c_int32)),
                ("best_time", ctypes.c_double), ("best_fitness", ctypes.c_double), ("t_all0", ctypes.c_double),
                ("n_measured", ctypes.c_int32), ("n_generations", ctypes.c_int32),
                ("search_wall_s", ctypes.c_double), ("time_to_best_s", ctypes.c_double)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("gemm_cfg", ctypes.c_int32), ("gemm_blocks_per_cu", ctypes.c_int32),
                ("stencil_rows", ctypes.c_int32), ("stencil_planes", ctypes.c_int32),
                ("stencil_blocks_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("t_total_s", ctypes.c_double), ("n_launches", ctypes.c_int32), ("n_submissions", ctypes.c_int32),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_int32), ("cfg", BatchConfig), ("ms", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_U8P = ctypes.POINTER(ctypes.c_uint8)


def lib():
    """The loaded libofl.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libofl.so is not built: run `python -m paper_1806_01430_amd.build`")
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes libofl bind to that one, so the process holds a single
        # runtime whichever module the caller imported first
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "ofl_app_load": (_I, [ctypes.c_char_p, ctypes.c_uint64, ctypes.POINTER(_P)]),
            "ofl_app_load_json": (_I, [ctypes.c_char_p, ctypes.c_uint64, ctypes.POINTER(_P)]),
            "ofl_app_free": (None, [_P]),
            "ofl_app_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
            "ofl_nest_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
            "ofl_nest_name": (_I, [_P, _I, ctypes.c_char_p, _I]),
            "ofl_buf_info": (_I, [_P, _I, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
            "ofl_buf_name": (_I, [_P, _I, ctypes.c_char_p, _I]),
            "ofl_buf_dims": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int64), _I, ctypes.POINTER(_I)]),
            "ofl_set_input": (_I, [_P, _I, _P, ctypes.c_uint64]),
            "ofl_mask_to_gene": (_I, [_P, _U8P, _I, _U8P]),
            "ofl_plan_transfers": (_I, [_P, _U8P, _I, _I, _I, ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I)]),
            "ofl_run_pattern": (_I, [_P, _U8P, _I, ctypes.POINTER(_P), _I, _P, ctypes.POINTER(RunOpts),
                                     ctypes.POINTER(RunStats)]),
            "ofl_eval_population": (_I, [_P, _U8P, _I, _I, ctypes.POINTER(_P), _I, _P, ctypes.POINTER(EvalOpts),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)]),
            "ofl_ga_run": (_I, [_P, ctypes.POINTER(GaParams), ctypes.POINTER(_P), _I, _P,
                                ctypes.POINTER(GaResult)]),
            "ofl_ga_run_table": (_I, [_I, ctypes.POINTER(GaParams), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(_I), ctypes.POINTER(GaResult)]),
            "ofl_read_buffer": (_I, [_P, _I, _P, ctypes.c_uint64]),
            "ofl_set_kernel_timing": (_I, [_P, _I]),
            "ofl_set_kernel_timing_op": (_I, [_P, ctypes.c_char_p]),
            "ofl_set_kernel_timing_sample": (_I, [_P, ctypes.c_int32, ctypes.c_int32]),
            "ofl_kernel_stats": (_I, [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_double)]),
            "ofl_batch_create": (_I, [ctypes.c_char_p, _I, ctypes.POINTER(ctypes.c_char_p), _I,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(_P)]),
            "ofl_batch_free": (None, [_P]),
            "ofl_batch_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
            "ofl_batch_buf_info": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I),
                                        ctypes.POINTER(_I)]),
            "ofl_batch_buf_dims": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_int64), _I]),
            "ofl_batch_buf_name": (_I, [_P, _I, ctypes.c_char_p, _I]),
            "ofl_batch_setup": (_I, [_P, ctypes.POINTER(_P), _I, _P]),
            "ofl_batch_run": (_I, [_P, ctypes.POINTER(_P), _I, _P, _I, ctypes.POINTER(BatchStats)]),
            "ofl_batch_get_config": (_I, [_P, ctypes.POINTER(BatchConfig)]),
            "ofl_batch_set_config": (_I, [_P, ctypes.POINTER(BatchConfig)]),
            "ofl_batch_tune": (_I, [_P, ctypes.POINTER(_P), _I, _P, _I, ctypes.POINTER(TuneEntry), _I,
                                    ctypes.POINTER(_I)]),
            "ofl_sweep19": (_I, [_P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _P, _P]),
            "ofl_sweep19_noalloc": (_I, [_P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _P, _P]),
            "ofl_status_str": (ctypes.c_char_p, [_I]),
            "ofl_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().ofl_last_error().decode(errors="replace")


def _check(rc, what):
    if rc != OK:
        raise OflError(rc, what)


def _u8(arr):
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    return a, a.ctypes.data_as(_U8P)


def app_path(name):
    return os.path.join(APPS_DIR, name + ".json")


def app_doc(app, sets=()):
    """Application description (a dict) from a name under apps/, a JSON file
    or a C source (parsed by cfront), with NAME=VALUE parameter overrides."""
    import json
    if app.endswith(".c"):
        from .cfront import load
        doc = load(app)
    else:
        with open(app if app.endswith(".json") else app_path(app)) as f:
            doc = json.load(f)
    for kv in sets:
        k, v = kv.split("=", 1)
        doc["params"][k] = int(v)
    return doc


def ga_params(M=12, T=12, Pc=0.9, Pm=0.05, p=0.5, seed=1, reps=3, warmup=1, policy=RESIDENT, flags=0,
              deadline_factor=0.0, timeout_s=0.0, cache_path=None, verify_rtol=0.0):
    return GaParams(M, T, Pc, Pm, p, seed, reps, warmup, policy, flags, deadline_factor, timeout_s, verify_rtol,
                    cache_path.encode() if cache_path else None)


def _ga_result_arrays(a, M, T):
    best = np.zeros(a, np.uint8)
    pops = np.zeros(T * M * a, np.uint8)
    times = np.zeros(T * M, np.float64)
    stats = np.zeros(T * M, np.int32)
    res = GaResult(best.ctypes.data_as(_U8P), pops.ctypes.data_as(_U8P),
                   times.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   stats.ctypes.data_as(ctypes.POINTER(_I)), 0, 0, 0, 0, 0, 0, 0)
    return res, best, pops, times, stats


def _ga_result_dict(res, best, pops, times, stats, a, M):
    G = res.n_generations
    return {"best_gene": tuple(int(x) for x in best), "best_time": res.best_time,
            "best_fitness": res.best_fitness, "t_all0": res.t_all0, "n_measured": res.n_measured,
            "n_generations": G, "search_wall_s": res.search_wall_s, "time_to_best_s": res.time_to_best_s,
            "pops": pops[:G * M * a].reshape(G, M, a).copy(), "times": times[:G * M].reshape(G, M).copy(),
            "status": stats[:G * M].reshape(G, M).copy()}


def ga_run_table(gene_len, params, t_table, status_table=None):
    """The library's GA over an injected time table (host only)."""
    t = np.ascontiguousarray(t_table, np.float64)
    if t.size != (1 << gene_len):
        raise ValueError("table must hold 2^gene_len times")
    st_ptr = None
    if status_table is not None:
        st = np.ascontiguousarray(status_table, np.int32)
        st_ptr = st.ctypes.data_as(ctypes.POINTER(_I))
    res, best, pops, times, stats = _ga_result_arrays(gene_len, params.M, params.T)
    _check(lib().ofl_ga_run_table(gene_len, ctypes.byref(params), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  st_ptr, ctypes.byref(res)), "ofl_ga_run_table")
    return _ga_result_dict(res, best, pops, times, stats, gene_len, params.M)


class App:
    """One loaded application (owns an ofl_app handle)."""

    def __init__(self, src, seed=1):
        L = lib()
        h = _P()
        if isinstance(src, str) and src.endswith(".c"):
            src = app_doc(src)
        if isinstance(src, dict):
            import json
            src = json.dumps(src)
        if src.lstrip().startswith("{"):
            rc = L.ofl_app_load_json(src.encode(), seed, ctypes.byref(h))
        else:
            rc = L.ofl_app_load(src.encode(), seed, ctypes.byref(h))
        _check(rc, "ofl_app_load")
        self._h = h
        n, a, b = _I(), _I(), _I()
        _check(L.ofl_app_info(h, ctypes.byref(n), ctypes.byref(a), ctypes.byref(b)), "ofl_app_info")
        self.n_nests, self.gene_len, self.n_bufs = n.value, a.value, b.value
        self.seed = seed

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ofl_app_free(h)
            self._h = None

    # ---------------------------------------------------------- introspection
    def nest_info(self, i):
        v, r, g = _I(), _I(), _I()
        _check(lib().ofl_nest_info(self._h, i, ctypes.byref(v), ctypes.byref(r), ctypes.byref(g)), "ofl_nest_info")
        return v.value, r.value, g.value

    def nest_name(self, i):
        buf = ctypes.create_string_buffer(256)
        _check(lib().ofl_nest_name(self._h, i, buf, 256), "ofl_nest_name")
        return buf.value.decode()

    def verdicts(self):
        return [self.nest_info(i) for i in range(self.n_nests)]

    def buf_info(self, b):
        nb, dt, out = ctypes.c_uint64(), _I(), _I()
        _check(lib().ofl_buf_info(self._h, b, ctypes.byref(nb), ctypes.byref(dt), ctypes.byref(out)), "ofl_buf_info")
        return nb.value, dt.value, bool(out.value)

    def buf_name(self, b):
        buf = ctypes.create_string_buffer(256)
        _check(lib().ofl_buf_name(self._h, b, buf, 256), "ofl_buf_name")
        return buf.value.decode()

    def buf_dims(self, b):
        dims = (ctypes.c_int64 * 8)()
        nd = _I()
        _check(lib().ofl_buf_dims(self._h, b, dims, 8, ctypes.byref(nd)), "ofl_buf_dims")
        return tuple(dims[i] for i in range(nd.value))

    def buf_index(self, name):
        for b in range(self.n_bufs):
            if self.buf_name(b) == name:
                return b
        raise KeyError(name)

    def set_input(self, b, array):
        """Set-up content of buffer b (dtype and size must match the buffer)."""
        if isinstance(b, str):
            b = self.buf_index(b)
        nbytes, dt, _ = self.buf_info(b)
        a = np.ascontiguousarray(array, dtype=_NP_DTYPE[dt])
        if a.nbytes != nbytes:
            raise ValueError("input has %d bytes, buffer %d" % (a.nbytes, nbytes))
        _check(lib().ofl_set_input(self._h, b, a.ctypes.data_as(_P), a.nbytes), "ofl_set_input")

    def mask_to_gene(self, mask):
        m, mp = _u8(mask)
        g = np.zeros(self.gene_len, np.uint8)
        _check(lib().ofl_mask_to_gene(self._h, mp, len(m), g.ctypes.data_as(_U8P)), "ofl_mask_to_gene")
        return tuple(int(x) for x in g)

    def plan_transfers(self, gene, policy=RESIDENT, flags=0):
        g, gp = _u8(gene)
        h2d, d2h, nc = ctypes.c_uint64(), ctypes.c_uint64(), _I()
        _check(lib().ofl_plan_transfers(self._h, gp, len(g), policy, flags, ctypes.byref(h2d), ctypes.byref(d2h),
                                        ctypes.byref(nc)), "ofl_plan_transfers")
        return h2d.value, d2h.value, nc.value

    # ---------------------------------------------------------- device side
    def alloc_device_buffers(self, device="cuda"):
        """One torch uint8 tensor per application buffer (caller-owned memory)."""
        import torch
        return [torch.empty(max(self.buf_info(b)[0], 16), dtype=torch.uint8, device=device)
                for b in range(self.n_bufs)]

    @staticmethod
    def _ptrs(bufs):
        arr = (_P * len(bufs))(*[ctypes.c_void_p(t.data_ptr()) for t in bufs])
        return arr

    @staticmethod
    def _stream(stream):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        return ctypes.c_void_p(stream.cuda_stream)

    def run_pattern(self, gene, bufs, stream=None, policy=RESIDENT, flags=0, deadline_s=0.0, check=True,
                    verify_rtol=0.0):
        g, gp = _u8(gene)
        st = RunStats()
        opts = RunOpts(policy, flags, deadline_s, verify_rtol)
        rc = lib().ofl_run_pattern(self._h, gp, len(g), self._ptrs(bufs), len(bufs), self._stream(stream),
                                   ctypes.byref(opts), ctypes.byref(st))
        if check:
            _check(rc, "ofl_run_pattern")
        d = st.as_dict()
        d["rc"] = rc
        return d

    def eval_population(self, genes, bufs, stream=None, reps=3, warmup=1, policy=RESIDENT, flags=0,
                        deadline_s=0.0, verify_rtol=0.0):
        G = np.ascontiguousarray(np.asarray(genes, np.uint8).reshape(-1, self.gene_len))
        t = np.zeros(G.shape[0], np.float64)
        s = np.zeros(G.shape[0], np.int32)
        opts = EvalOpts(reps, warmup, policy, flags, deadline_s, verify_rtol)
        _check(lib().ofl_eval_population(self._h, G.ctypes.data_as(_U8P), G.shape[0], self.gene_len,
                                         self._ptrs(bufs), len(bufs), self._stream(stream), ctypes.byref(opts),
                                         t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         s.ctypes.data_as(ctypes.POINTER(_I))), "ofl_eval_population")
        return t, s

    def ga_run(self, params, bufs, stream=None):
        a = self.gene_len
        res, best, pops, times, stats = _ga_result_arrays(a, params.M, params.T)
        _check(lib().ofl_ga_run(self._h, ctypes.byref(params), self._ptrs(bufs), len(bufs), self._stream(stream),
                                ctypes.byref(res)), "ofl_ga_run")
        return _ga_result_dict(res, best, pops, times, stats, a, params.M)

    def read_buffer(self, b):
        if isinstance(b, str):
            b = self.buf_index(b)
        nbytes, dt, _ = self.buf_info(b)
        out = np.empty(self.buf_dims(b), _NP_DTYPE[dt])
        _check(lib().ofl_read_buffer(self._h, b, out.ctypes.data_as(_P), out.nbytes), "ofl_read_buffer")
        return out

    def read_all(self):
        return {self.buf_name(b): self.read_buffer(b) for b in range(self.n_bufs)}

    def set_kernel_timing(self, enable=True):
        _check(lib().ofl_set_kernel_timing(self._h, 1 if enable else 0), "ofl_set_kernel_timing")

    def set_kernel_timing_op(self, op=None):
        """Time only nests of the kinds in `op` (comma-separated; None: every kind)."""
        _check(lib().ofl_set_kernel_timing_op(self._h, op.encode() if op else None), "ofl_set_kernel_timing_op")

    def set_kernel_timing_sample(self, stride=1, phase=0):
        """Time only executions phase, phase + stride, ... of each timed kind in a run."""
        _check(lib().ofl_set_kernel_timing_sample(self._h, stride, phase), "ofl_set_kernel_timing_sample")

    def kernel_stats(self, op):
        """(timed executions of nests of kind `op`, their total kernel ms)."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(lib().ofl_kernel_stats(self._h, op.encode(), ctypes.byref(n), ctypes.byref(ms)), "ofl_kernel_stats")
        return n.value, ms.value


def sweep19(p, q, res, slot=0, stream=None, noalloc=False):
    """One sweep of the 19-point nest on torch tensors p, q (float32, I x J x
    K, on the GPU) adding its FP64 residual into res[slot] (float64 tensor on
    the GPU); launches on the stream, returns without synchronising.
    noalloc=True calls ofl_sweep19_noalloc (the library's fixed scratch)."""
    import torch
    I, J, K = p.shape
    if tuple(q.shape) != (I, J, K):
        raise ValueError("p and q differ in shape")
    if p.dtype != torch.float32 or q.dtype != torch.float32 or res.dtype != torch.float64:
        raise ValueError("p, q must be float32 and res float64")
    if not (p.is_contiguous() and q.is_contiguous()) or not 0 <= slot < res.numel():
        raise ValueError("p, q must be contiguous and slot inside res")
    name = "ofl_sweep19_noalloc" if noalloc else "ofl_sweep19"
    _check(getattr(lib(), name)(_P(p.data_ptr()), _P(q.data_ptr()), I, J, K, _P(res.data_ptr() + 8 * slot),
                                App._stream(stream)), name)


class Batch:
    """Instances of one application description with per-instance parameter
    values and seeds, every nest on the GPU (owns an ofl_batch handle)."""

    def __init__(self, src, params, seeds):
        """src: description (dict or JSON text); params: list of dicts (one per
        instance, same keys); seeds: one integer per instance."""
        import json
        if isinstance(src, dict):
            src = json.dumps(src)
        n = len(params)
        names = sorted(params[0]) if n else []
        for p in params:
            if sorted(p) != names:
                raise ValueError("every instance must set the same parameters")
        cn = (ctypes.c_char_p * max(1, len(names)))(*[x.encode() for x in names])
        vals = np.ascontiguousarray([[int(p[k]) for k in names] for p in params], np.int64).reshape(-1)
        sd = np.ascontiguousarray(seeds, np.uint64)
        if sd.size != n:
            raise ValueError("one seed per instance")
        h = _P()
        _check(lib().ofl_batch_create(src.encode(), n, cn, len(names), vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      sd.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ctypes.byref(h)),
               "ofl_batch_create")
        self._h = h
        ni, nb, nn = _I(), _I(), _I()
        _check(lib().ofl_batch_info(h, ctypes.byref(ni), ctypes.byref(nb), ctypes.byref(nn)), "ofl_batch_info")
        self.n_inst, self.n_bufs, self.n_nests = ni.value, nb.value, nn.value
        buf = ctypes.create_string_buffer(256)
        self.buf_names = []
        for b in range(self.n_bufs):
            _check(lib().ofl_batch_buf_name(h, b, buf, 256), "ofl_batch_buf_name")
            self.buf_names.append(buf.value.decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ofl_batch_free(h)
            self._h = None

    def buf_info(self, inst, b):
        nbytes, dt, rank = ctypes.c_uint64(), _I(), _I()
        _check(lib().ofl_batch_buf_info(self._h, inst, b, ctypes.byref(nbytes), ctypes.byref(dt), ctypes.byref(rank)),
               "ofl_batch_buf_info")
        dims = (ctypes.c_int64 * max(1, rank.value))()
        _check(lib().ofl_batch_buf_dims(self._h, inst, b, dims, rank.value), "ofl_batch_buf_dims")
        return nbytes.value, _NP_DTYPE[dt.value], tuple(dims[i] for i in range(rank.value))

    def alloc_device_buffers(self, device="cuda"):
        """Per instance, one torch uint8 tensor per buffer (caller-owned)."""
        import torch
        return [[torch.empty(max(self.buf_info(i, b)[0], 16), dtype=torch.uint8, device=device)
                 for b in range(self.n_bufs)] for i in range(self.n_inst)]

    @staticmethod
    def _ptrs(bufs):
        flat = [t for row in bufs for t in row]
        return (_P * len(flat))(*[ctypes.c_void_p(t.data_ptr()) for t in flat]), len(flat)

    def setup(self, bufs, stream=None):
        p, n = self._ptrs(bufs)
        _check(lib().ofl_batch_setup(self._h, p, n, App._stream(stream)), "ofl_batch_setup")

    def run(self, bufs, mode=BATCH_GROUPED_GRAPH, stream=None):
        p, n = self._ptrs(bufs)
        st = BatchStats()
        _check(lib().ofl_batch_run(self._h, p, n, App._stream(stream), mode, ctypes.byref(st)), "ofl_batch_run")
        return st.as_dict()

    @property
    def config(self):
        c = BatchConfig()
        _check(lib().ofl_batch_get_config(self._h, ctypes.byref(c)), "ofl_batch_get_config")
        return c.as_dict()

    def set_config(self, **kw):
        c = BatchConfig(**{**self.config, **kw})
        _check(lib().ofl_batch_set_config(self._h, ctypes.byref(c)), "ofl_batch_set_config")

    def tune(self, bufs, reps=3, stream=None):
        p, n = self._ptrs(bufs)
        cap = 512
        ents = (TuneEntry * cap)()
        cnt = _I()
        _check(lib().ofl_batch_tune(self._h, p, n, App._stream(stream), reps, ents, cap, ctypes.byref(cnt)),
               "ofl_batch_tune")
        return [{"phase": ("gemm", "stencil")[e.phase], **e.cfg.as_dict(), "ms": e.ms}
                for e in ents[:min(cap, cnt.value)]]

    def read(self, bufs, inst, name):
        """Host copy of buffer `name` of instance `inst` (synchronises)."""
        import torch
        b = self.buf_names.index(name) if isinstance(name, str) else name
        nbytes, dt, dims = self.buf_info(inst, b)
        torch.cuda.synchronize()
        raw = bufs[inst][b][:nbytes].cpu().numpy()
        return raw.view(dt).reshape(dims).copy()
