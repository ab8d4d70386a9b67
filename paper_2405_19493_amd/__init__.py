"""Python binding of libzg (the MI355X ziggurat Gaussian generator).

Argument marshalling only: every step of generation runs in the HIP kernels
of libzg.so.  torch provides device memory and streams.  The functions keep
the C-ABI names (zg_fill, zg_fill_streams, ...); tensors are passed for
device buffers and the current torch stream is used unless one is given.

The library must be built (python -m paper_2405_19493_amd.build); importing
fails loudly when it is missing.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime libzg shares with torch)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "zg.h")

ZG_OK = 0
ZG_EINVAL = -1
ZG_ERANGE = -2
ZG_ENOMEM = -3
ZG_EHIP = -4
ZG_EBUSY = -5
ZG_ENOENT = -6
ZG_ESTATE = -7

ZG_SPLITMIX64 = 1
ZG_JAVA_LCG48 = 2
ZG_ZIGGURAT = 0
ZG_POLAR = 1
ZG_MCFARLAND = 2
ZG_MZ_BUCKETS = 256
ZG_MZ_LAYERS = 253
ZG_F64 = 0
ZG_F32 = 1
ZG_FLAG_BUDGET = 1
ZG_FLAG_RANGE = 2
ZG_KNOB_DMAX = 1
ZG_KNOB_SEQ_SPANS = 2
ZG_SEQ_MAX_N = 1000000
ZG_SEQ_NOALLOC_MAX_N = 268435456
ZG_OP_FILL = 0
ZG_OP_MUTATE = 1
ZG_NO_HANDLE = -1
ZG_MAX_BATCH = 32768
ZG_TUNE_FILL_F64, ZG_TUNE_FILL_F32, ZG_TUNE_POLAR, ZG_TUNE_MUTATE, ZG_TUNE_BATCH, ZG_TUNE_FILL_MZ = range(6)
ZG_TUNE_CLASSES = 6
ZG_SERVE_BATCHED = 0
ZG_SERVE_PER_REQUEST = 1
ZG_SM64_WINDOW = 1 << 40
ZG_LCG_WINDOW = 2147483547


class ZgError(RuntimeError):
    def __init__(self, status, what, detail=""):
        self.status = status
        msg = f"{what}: {_strerror(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class TableView(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_double),
        ("v", ctypes.c_double),
        ("W", ctypes.c_double * 128),
        ("y", ctypes.c_double * 128),
        ("dy", ctypes.c_double * 128),
        ("w53", ctypes.c_double * 128),
        ("w24d", ctypes.c_double * 128),
        ("w24", ctypes.c_float * 128),
        ("k53", ctypes.c_uint64 * 128),
        ("k24", ctypes.c_uint32 * 128),
    ]


class MzTableView(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double),
        ("xs", ctypes.c_double * 256),
        ("ox", ctypes.c_double * 254),
        ("odx", ctypes.c_double * 254),
        ("oy", ctypes.c_double * 254),
        ("ody", ctypes.c_double * 254),
        ("thr", ctypes.c_uint64 * 256),
        ("kind", ctypes.c_uint8 * 254),
        ("alias", ctypes.c_uint8 * 256),
    ]


class EaParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("generation", ctypes.c_uint64),
                ("stream", ctypes.c_uint32), ("tournament", ctypes.c_uint32),
                ("rate", ctypes.c_double), ("sigma", ctypes.c_double),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [
        ("out", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("first_index", ctypes.c_uint64),
        ("sigma", ctypes.c_double),
        ("stream", ctypes.c_uint32),
        ("handle", ctypes.c_int32),
        ("dtype", ctypes.c_uint8),
        ("method", ctypes.c_uint8),
        ("kind", ctypes.c_uint8),
        ("op", ctypes.c_uint8),
        ("reserved", ctypes.c_uint32),
    ]


class Tune(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("batch_blocks_per_cu", ctypes.c_uint32), ("queue_cap", ctypes.c_uint32),
                ("drain_waves", ctypes.c_uint32), ("group_steps", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_cap_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("batch_window_us", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ServerRequest(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("handle", ctypes.c_uint32), ("dtype", ctypes.c_uint8),
                ("method", ctypes.c_uint8), ("reserved", ctypes.c_uint16),
                ("arrival_s", ctypes.c_double)]


class Completion(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("done", ctypes.c_int32), ("d_out", ctypes.c_void_p),
                ("first_index", ctypes.c_uint64), ("arrival_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("complete_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("variates", ctypes.c_uint64), ("inflight_bytes", ctypes.c_uint64),
                ("peak_inflight_bytes", ctypes.c_uint64), ("p50_latency_s", ctypes.c_double),
                ("p99_latency_s", ctypes.c_double), ("max_latency_s", ctypes.c_double),
                ("first_arrival_s", ctypes.c_double), ("last_complete_s", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libzg.so is not built at {LIB_PATH}; run `python -m paper_2405_19493_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, U64, U32, I32, D = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double
    sigs = {
        "zg_build_table": [P],
        "zg_build_mz_table": [P],
        "zg_create": [ctypes.c_int, P],
        "zg_destroy": [P],
        "zg_table": [P, P],
        "zg_fill": [P, P, U64, ctypes.c_int, ctypes.c_int, ctypes.c_int, U64, U32, U64, P],
        "zg_fill_streams": [P, P, U64, U32, ctypes.c_int, ctypes.c_int, ctypes.c_int, U64, U32, U64, P],
        "zg_uniform_words": [P, P, U64, ctypes.c_int, U64, U32, U32, U64, P],
        "zg_fill_sequential": [P, P, U64, ctypes.c_int, U64, U32, U64, P, P, U64, P],
        "zg_fill_sequential_noalloc": [P, P, U64, ctypes.c_int, U64, U32, U64, P, P],
        "zg_sequential_workspace": [U64, P],
        "zg_mutate": [P, P, U64, D, ctypes.c_int, U64, U32, U64, P],
        "zg_ea_step": [P, P, P, P, P, U32, U32, P, P],
        "zg_decide_words": [P, P, U64, P, P, P],
        "zg_error_flags": [P, P, ctypes.c_int],
        "zg_set_test_knob": [P, ctypes.c_int, ctypes.c_int64],
        "zg_stream_open": [P, U64, U32, ctypes.c_int, ctypes.c_int, ctypes.c_int, P],
        "zg_stream_close": [P, U32],
        "zg_stream_fill": [P, U32, P, U64, ctypes.c_int, ctypes.c_int, P],
        "zg_stream_get_counter": [P, U32, P],
        "zg_stream_set_counter": [P, U32, U64],
        "zg_batch": [P, P, U32, P, P],
        "zg_fill_each": [P, P, U32, P],
        "zg_get_tune": [P, ctypes.c_int, P],
        "zg_set_tune": [P, ctypes.c_int, P],
        "zg_autotune": [P, ctypes.c_char_p, U64, ctypes.c_int],
        "zg_server_create": [P, P, P],
        "zg_server_submit": [P, P, P],
        "zg_server_poll": [P, U64, P],
        "zg_server_wait": [P, U64, D, P],
        "zg_server_release": [P, U64],
        "zg_server_drain": [P],
        "zg_server_stats_get": [P, P],
        "zg_server_destroy": [P],
        "zg_server_replay": [P, P, U32, P, D],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = I32
    lib.zg_strerror.argtypes = [I32]
    lib.zg_strerror.restype = ctypes.c_char_p
    lib.zg_last_error.argtypes = [P]
    lib.zg_last_error.restype = ctypes.c_char_p
    if hasattr(lib, "zg_server_now"):
        lib.zg_server_now.argtypes = [P]
        lib.zg_server_now.restype = D
    return lib


lib = _load()


def _strerror(status):
    return lib.zg_strerror(status).decode()


def _check(status, what, ctx=None):
    if status != ZG_OK:
        detail = lib.zg_last_error(ctx).decode() if (ctx and status == ZG_EHIP) else ""
        raise ZgError(status, what, detail)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    if t.dtype == torch.float64:
        return ZG_F64
    if t.dtype == torch.float32:
        return ZG_F32
    raise ValueError("output tensor must be float64 or float32")


def zg_build_table():
    """Host-only table build (no device needed)."""
    t = TableView()
    _check(lib.zg_build_table(ctypes.byref(t)), "zg_build_table")
    return t


def zg_build_mz_table():
    """Host-only build of the modified ziggurat's table (no device needed)."""
    t = MzTableView()
    _check(lib.zg_build_mz_table(ctypes.byref(t)), "zg_build_mz_table")
    return t


class Context:
    """A libzg context on one HIP device (zg_create / zg_destroy)."""

    def __init__(self, device=0):
        if not torch.cuda.is_available():
            raise RuntimeError("libzg needs a HIP device; none is visible")
        self.device = device
        h = ctypes.c_void_p()
        _check(lib.zg_create(device, ctypes.byref(h)), "zg_create")
        self.h = h

    def close(self):
        if self.h:
            lib.zg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _c(self, st, what):
        _check(st, what, self.h)

    # -------------------------------------------------------------- table
    def zg_table(self):
        t = TableView()
        self._c(lib.zg_table(self.h, ctypes.byref(t)), "zg_table")
        return t

    # --------------------------------------------------------- generation
    def zg_fill(self, out, method=ZG_ZIGGURAT, kind=ZG_SPLITMIX64, seed=0, stream=0,
                first_index=0, hip_stream=None):
        self._c(lib.zg_fill(self.h, _ptr(out), out.numel(), _dtype_code(out), method, kind,
                            seed & (2**64 - 1), stream, first_index, _stream(hip_stream)),
                "zg_fill")
        return out

    def zg_fill_streams(self, out, n_per_stream, n_streams, method=ZG_ZIGGURAT,
                        kind=ZG_SPLITMIX64, seed=0, stream0=0, first_index=0, hip_stream=None):
        if out.numel() < n_per_stream * n_streams:
            raise ValueError("output tensor too small")
        self._c(lib.zg_fill_streams(self.h, _ptr(out), n_per_stream, n_streams, _dtype_code(out),
                                    method, kind, seed & (2**64 - 1), stream0, first_index,
                                    _stream(hip_stream)), "zg_fill_streams")
        return out

    def zg_uniform_words(self, out, kind=ZG_SPLITMIX64, seed=0, stream=0, draw=0, first_index=0,
                         hip_stream=None):
        if out.dtype not in (torch.int64, torch.uint64):
            raise ValueError("words need an int64/uint64 tensor")
        self._c(lib.zg_uniform_words(self.h, _ptr(out), out.numel(), kind, seed & (2**64 - 1),
                                     stream, draw, first_index, _stream(hip_stream)),
                "zg_uniform_words")
        return out

    def zg_fill_sequential(self, out, kind=ZG_SPLITMIX64, seed=0, stream=0, first_word=0,
                           next_word=None, work=None, hip_stream=None):
        """out (float64) <- successive variates reading one generator in order
        from word position first_word; next_word: optional 1-element int64
        device tensor receiving the position after the last word read; work:
        optional uint8 device tensor of zg_sequential_workspace(n) bytes
        (else one is allocated here, on the output's device)."""
        if out.dtype != torch.float64:
            raise ValueError("sequential fills are float64")
        if work is None and out.numel() > 0:
            work = torch.empty(max(zg_sequential_workspace(out.numel()), 1), dtype=torch.uint8,
                               device=out.device)
        wp, wb = (None, 0) if work is None else (_ptr(work), work.numel() * work.element_size())
        self._c(lib.zg_fill_sequential(self.h, _ptr(out), out.numel(), kind, seed & (2**64 - 1),
                                       stream, first_word,
                                       _ptr(next_word) if next_word is not None else None, wp,
                                       wb, _stream(hip_stream)), "zg_fill_sequential")
        return out

    def zg_fill_sequential_noalloc(self, out, kind=ZG_SPLITMIX64, seed=0, stream=0,
                                   first_word=0, next_word=None, hip_stream=None):
        """zg_fill_sequential with the library's device-resident workspace
        (nothing is allocated)."""
        if out.dtype != torch.float64:
            raise ValueError("sequential fills are float64")
        self._c(lib.zg_fill_sequential_noalloc(
            self.h, _ptr(out), out.numel(), kind, seed & (2**64 - 1), stream, first_word,
            _ptr(next_word) if next_word is not None else None, _stream(hip_stream)),
            "zg_fill_sequential_noalloc")
        return out

    def zg_mutate(self, x, sigma, kind=ZG_SPLITMIX64, seed=0, stream=0, first_index=0,
                  hip_stream=None):
        if x.dtype != torch.float64:
            raise ValueError("mutation works on float64")
        self._c(lib.zg_mutate(self.h, _ptr(x), x.numel(), float(sigma), kind, seed & (2**64 - 1),
                              stream, first_index, _stream(hip_stream)), "zg_mutate")
        return x

    def zg_ea_step(self, parents, fitness, children, winners=None, tournament=2, rate=0.05,
                   sigma=0.1, lo=-5.0, hi=5.0, seed=0, stream=0, generation=0,
                   hip_stream=None):
        """One EA generation (zg_ea_step): parents (pop x genes float64, C
        order), fitness (pop float64) -> children (pop x genes), winners
        (pop int32, optional)."""
        if parents.dtype != torch.float64 or children.dtype != torch.float64 or \
                fitness.dtype != torch.float64:
            raise ValueError("the EA step works on float64")
        if parents.dim() != 2 or parents.shape != children.shape or \
                fitness.numel() != parents.shape[0]:
            raise ValueError("parents and children: pop x genes; fitness: pop")
        if not (parents.is_contiguous() and children.is_contiguous() and fitness.is_contiguous()):
            raise ValueError("contiguous tensors only")
        if winners is not None and (winners.dtype != torch.int32 or
                                    winners.numel() != parents.shape[0]):
            raise ValueError("winners: pop int32")
        p = EaParams(seed & (2**64 - 1), generation, stream, tournament, float(rate),
                     float(sigma), float(lo), float(hi))
        pop, genes = parents.shape
        self._c(lib.zg_ea_step(self.h, _ptr(parents), _ptr(fitness), _ptr(children),
                               _ptr(winners) if winners is not None else None, pop, genes,
                               ctypes.byref(p), _stream(hip_stream)), "zg_ea_step")
        return children

    def zg_decide_words(self, words, cls, x, hip_stream=None):
        self._c(lib.zg_decide_words(self.h, _ptr(words), words.numel(), _ptr(cls), _ptr(x),
                                    _stream(hip_stream)), "zg_decide_words")

    def zg_error_flags(self, clear=True):
        f = ctypes.c_uint32()
        self._c(lib.zg_error_flags(self.h, ctypes.byref(f), 1 if clear else 0), "zg_error_flags")
        return f.value

    def zg_set_test_knob(self, knob, value):
        self._c(lib.zg_set_test_knob(self.h, knob, value), "zg_set_test_knob")

    # ----------------------------------------------------------- counters
    def zg_stream_open(self, seed, stream, kind=ZG_SPLITMIX64, dtype=ZG_F64, method=ZG_ZIGGURAT):
        """A counter handle bound to (seed, stream, kind) and one output mode
        (dtype, method); requests in another mode are refused."""
        h = ctypes.c_uint32()
        self._c(lib.zg_stream_open(self.h, seed & (2**64 - 1), stream, kind, dtype, method,
                                   ctypes.byref(h)), "zg_stream_open")
        return h.value

    def zg_stream_close(self, handle):
        self._c(lib.zg_stream_close(self.h, handle), "zg_stream_close")

    def zg_stream_fill(self, handle, out, method=ZG_ZIGGURAT, hip_stream=None):
        self._c(lib.zg_stream_fill(self.h, handle, _ptr(out), out.numel(), _dtype_code(out),
                                   method, _stream(hip_stream)), "zg_stream_fill")
        return out

    def zg_stream_get_counter(self, handle):
        c = ctypes.c_uint64()
        self._c(lib.zg_stream_get_counter(self.h, handle, ctypes.byref(c)),
                "zg_stream_get_counter")
        return c.value

    def zg_stream_set_counter(self, handle, counter):
        self._c(lib.zg_stream_set_counter(self.h, handle, counter), "zg_stream_set_counter")

    # -------------------------------------------------------------- batch
    @staticmethod
    def zg_batch_prepare(requests):
        """The C request array of a list of request dicts (reusable across
        zg_batch calls)."""
        arr = (Request * len(requests))()
        for i, r in enumerate(requests):
            out = r["out"]
            arr[i].out = out.data_ptr() if out is not None else None
            arr[i].n = r.get("n", out.numel() if out is not None else 0)
            arr[i].seed = r.get("seed", 0) & (2**64 - 1)
            arr[i].first_index = r.get("first_index", 0)
            arr[i].sigma = r.get("sigma", 0.0)
            arr[i].stream = r.get("stream", 0)
            arr[i].handle = r.get("handle", ZG_NO_HANDLE)
            arr[i].dtype = r.get("dtype", _dtype_code(out) if out is not None else ZG_F64)
            arr[i].method = r.get("method", ZG_ZIGGURAT)
            arr[i].kind = r.get("kind", ZG_SPLITMIX64)
            arr[i].op = r.get("op", ZG_OP_FILL)
        return arr

    def zg_batch(self, requests, want_first=False, hip_stream=None):
        """requests: list of dicts with keys out (tensor), n, seed, stream,
        first_index, sigma, handle, dtype, method, kind, op; or an array from
        zg_batch_prepare."""
        arr = requests if isinstance(requests, ctypes.Array) else self.zg_batch_prepare(requests)
        first = (ctypes.c_uint64 * len(requests))() if want_first else None
        self._c(lib.zg_batch(self.h, arr, len(requests), first, _stream(hip_stream)), "zg_batch")
        return list(first) if want_first else None

    def zg_fill_each(self, requests, hip_stream=None):
        """Each request of a list (or an array from zg_batch_prepare) as its
        own plain launch, in order, from one C loop."""
        arr = requests if isinstance(requests, ctypes.Array) else self.zg_batch_prepare(requests)
        self._c(lib.zg_fill_each(self.h, arr, len(requests), _stream(hip_stream)), "zg_fill_each")

    # ------------------------------------------------------------- tuning
    def zg_get_tune(self, cls):
        """(tile, waves_per_block, batch_blocks_per_cu, queue_cap, drain_waves,
        group_steps) of a tuning class."""
        t = Tune()
        self._c(lib.zg_get_tune(self.h, cls, ctypes.byref(t)), "zg_get_tune")
        return (t.tile, t.waves_per_block, t.batch_blocks_per_cu, t.queue_cap, t.drain_waves,
                t.group_steps)

    def zg_set_tune(self, cls, tile, waves_per_block, batch_blocks_per_cu=2, queue_cap=0,
                    drain_waves=0, group_steps=4):
        t = Tune(tile, waves_per_block, batch_blocks_per_cu, queue_cap, drain_waves, group_steps)
        self._c(lib.zg_set_tune(self.h, cls, ctypes.byref(t)), "zg_set_tune")

    def zg_autotune(self, cache_path=None, nbytes=0, use_cache=True):
        p = cache_path.encode() if cache_path else None
        self._c(lib.zg_autotune(self.h, p, nbytes, 1 if use_cache else 0), "zg_autotune")


def _completion(c):
    return {"status": c.status, "done": bool(c.done), "d_out": c.d_out or 0,
            "first_index": c.first_index, "arrival_s": c.arrival_s, "admit_s": c.admit_s,
            "complete_s": c.complete_s}


class Server:
    """The serving loop of a context (zg_server_*): counter-keyed requests in,
    outputs in a device arena, completions polled from the device."""

    def __init__(self, ctx, mem_cap_bytes=1 << 30, max_inflight=4096, max_batch=1024,
                 batch_window_us=200, n_streams=2, mode=ZG_SERVE_BATCHED):
        self.ctx = ctx
        cfg = ServerConfig(mem_cap_bytes, max_inflight, max_batch, batch_window_us, n_streams,
                           mode, 0)
        h = ctypes.c_void_p()
        ctx._c(lib.zg_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)), "zg_server_create")
        self.h = h

    def submit(self, handle, n, dtype=ZG_F64, method=ZG_ZIGGURAT, arrival_s=0.0):
        r = ServerRequest(n, handle, dtype, method, 0, float(arrival_s))
        t = ctypes.c_uint64()
        self.ctx._c(lib.zg_server_submit(self.h, ctypes.byref(r), ctypes.byref(t)),
                    "zg_server_submit")
        return t.value

    def poll(self, ticket):
        c = Completion()
        self.ctx._c(lib.zg_server_poll(self.h, ticket, ctypes.byref(c)), "zg_server_poll")
        return _completion(c)

    def wait(self, ticket, timeout_s=30.0):
        c = Completion()
        self.ctx._c(lib.zg_server_wait(self.h, ticket, float(timeout_s), ctypes.byref(c)),
                    "zg_server_wait")
        return _completion(c)

    def release(self, ticket):
        self.ctx._c(lib.zg_server_release(self.h, ticket), "zg_server_release")

    def drain(self):
        self.ctx._c(lib.zg_server_drain(self.h), "zg_server_drain")

    def now(self):
        return lib.zg_server_now(self.h)

    def replay(self, handles, sizes, dtypes, arrivals, timeout_s=600.0, want_first=False):
        """Open-loop replay of a trace (numpy arrays of equal length; arrival
        times in seconds from the call)."""
        n = len(sizes)
        arr = (ServerRequest * n)()
        for k in range(n):
            arr[k].n = int(sizes[k])
            arr[k].handle = int(handles[k])
            arr[k].dtype = int(dtypes[k])
            arr[k].method = ZG_ZIGGURAT
            arr[k].arrival_s = float(arrivals[k])
        first = (ctypes.c_uint64 * n)() if want_first else None
        self.ctx._c(lib.zg_server_replay(self.h, arr, n, first, float(timeout_s)),
                    "zg_server_replay")
        return list(first) if want_first else None

    def stats(self):
        st = ServerStats()
        self.ctx._c(lib.zg_server_stats_get(self.h, ctypes.byref(st)), "zg_server_stats_get")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def output(self, completion, n, dtype=ZG_F64):
        """A zero-copy torch view of a completed request's arena memory; it is
        valid until the ticket is released."""

        class _View:
            pass

        v = _View()
        v.__cuda_array_interface__ = {
            "shape": (n,), "typestr": "<f8" if dtype == ZG_F64 else "<f4",
            "data": (completion["d_out"], False), "version": 2, "strides": None}
        return torch.as_tensor(v, device="cuda")

    def close(self):
        if self.h:
            lib.zg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = [n for n in dir() if n.startswith(("zg_", "ZG_"))] + ["Context", "Server", "ZgError",
                                                                 "lib"]


def zg_sequential_workspace(n):
    """Workspace bytes of a sequential fill of n variates."""
    b = ctypes.c_uint64()
    st = lib.zg_sequential_workspace(n, ctypes.byref(b))
    if st != ZG_OK:
        raise ZgError(st, "zg_sequential_workspace")
    return int(b.value)
