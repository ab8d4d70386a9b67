"""ctypes front end of the C oracle (oracle/zg_oracle.c).

TEST INFRASTRUCTURE ONLY.  Builds the oracle with gcc (-O2 -ffp-contract=off)
into oracle/libzg_oracle.so and exposes numpy-returning wrappers.  The table it
uses is the stored 60-digit oracle table (oracle/table_b128.json), never the
product library's.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import table_mp, table_mz

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "zg_oracle.c")
LIB = os.path.join(HERE, "libzg_oracle.so")

SM64 = 1
LCG48 = 2
DMAX = 256


def build(force=True):
    """Compile the oracle shared library (always recompiles when force)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-pthread", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class OrcTable(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_double),
        ("W", ctypes.c_double * 128),
        ("y", ctypes.c_double * 128),
        ("dy", ctypes.c_double * 128),
        ("w53", ctypes.c_double * 128),
        ("w24d", ctypes.c_double * 128),
        ("w24", ctypes.c_float * 128),
        ("k53", ctypes.c_uint64 * 128),
        ("k24", ctypes.c_uint32 * 128),
    ]


_lib = None
_table = None
_table_dict = None

u64 = ctypes.c_uint64
u32 = ctypes.c_uint32
i32 = ctypes.c_int
vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        L.orc_sm64_word.argtypes = [u64, u32, u64, u32]
        L.orc_sm64_word.restype = u64
        L.orc_lcg_word.argtypes = [u64, u32, u64, u32]
        L.orc_lcg_word.restype = u64
        L.orc_lcg_state.argtypes = [u64, u64]
        L.orc_lcg_state.restype = u64
        L.orc_lcg_state0.argtypes = [u64]
        L.orc_lcg_state0.restype = u64
        L.orc_lcg_step.argtypes = [u64]
        L.orc_lcg_step.restype = u64
        L.orc_lcg_affine.argtypes = [u64, vp, vp]
        L.orc_lcg_affine.restype = None
        L.orc_lcg_seq_doubles.argtypes = [u64, u64, vp]
        L.orc_lcg_seq_doubles.restype = None
        L.orc_lcg_seq_ints.argtypes = [u64, u64, vp]
        L.orc_lcg_seq_ints.restype = None
        L.orc_zig_f64.argtypes = [vp, i32, u64, u32, u64, u32, vp]
        L.orc_zig_f64.restype = ctypes.c_double
        L.orc_decide_word.argtypes = [vp, u64, vp]
        L.orc_decide_word.restype = i32
        L.orc_zig_f64_tape.argtypes = [vp, vp, u32, u32, vp, vp, u32, vp]
        L.orc_zig_f64_tape.restype = ctypes.c_double
        L.orc_attempt.argtypes = [vp, i32, u64, u64, u64, vp]
        L.orc_attempt.restype = i32
        L.orc_enum_attempt.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp]
        L.orc_enum_attempt.restype = i32
        L.orc_polar_core.argtypes = [ctypes.c_double, ctypes.c_double, vp, vp]
        L.orc_polar_core.restype = i32
        L.orc_fill_f64.argtypes = [vp, i32, u64, u32, u64, u64, u32, vp, vp, i32]
        L.orc_fill_f64.restype = u64
        L.orc_fill_f32.argtypes = [vp, i32, u64, u32, u64, u64, u32, vp, vp, vp, i32]
        L.orc_fill_f32.restype = u64
        L.orc_fill_polar.argtypes = [i32, u64, u32, u64, u64, u32, vp, vp, i32]
        L.orc_fill_polar.restype = u64
        L.orc_mutate.argtypes = [vp, i32, u64, u32, u64, u64, u32, ctypes.c_double, vp, vp, i32]
        L.orc_mutate.restype = u64
        L.orc_words.argtypes = [i32, u64, u32, u32, u64, u64, vp]
        L.orc_words.restype = None
        L.orc_fill_streams_f64.argtypes = [vp, i32, u64, u32, u32, u64, u64, u32, vp, vp, i32]
        L.orc_fill_streams_f64.restype = u64
        L.orc_fill_streams_f32.argtypes = [vp, i32, u64, u32, u32, u64, u64, u32, vp, vp, vp, i32]
        L.orc_fill_streams_f32.restype = u64
        L.orc_fill_streams_polar.argtypes = [i32, u64, u32, u32, u64, u64, u32, vp, vp, i32]
        L.orc_fill_streams_polar.restype = u64
        L.orc_seq_f64.argtypes = [vp, i32, u64, u32, u64, u64, vp, u64, vp, vp, vp, vp]
        L.orc_seq_f64.restype = u64
        L.orc_lcg_long.argtypes = [u64, u32, u64, u32]
        L.orc_lcg_long.restype = u64
        L.orc_long_word.argtypes = [i32, u64, u32, u64, u32]
        L.orc_long_word.restype = u64
        L.orc_mz_f64.argtypes = [vp, i32, u64, u32, u64, u32, vp]
        L.orc_mz_f64.restype = ctypes.c_double
        L.orc_mz_f64_tape.argtypes = [vp, vp, u32, u32, vp, vp, u32, vp]
        L.orc_mz_f64_tape.restype = ctypes.c_double
        L.orc_mz_first.argtypes = [vp, u64, vp, vp]
        L.orc_mz_first.restype = i32
        L.orc_mz_region.argtypes = [vp, u64, u64]
        L.orc_mz_region.restype = i32
        L.orc_mz_attempt.argtypes = [vp, i32, u64, u64, vp]
        L.orc_mz_attempt.restype = i32
        L.orc_mz_enum.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.orc_mz_enum.restype = i32
        L.orc_ea_step.argtypes = [vp, vp, vp, vp, vp, vp, u32, u32, u32, u64, u32, u64, u64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, u32, i32]
        L.orc_ea_step.restype = u64
        L.orc_fill_streams_mz.argtypes = [vp, i32, u64, u32, u32, u64, u64, u32, vp, vp, i32]
        L.orc_fill_streams_mz.restype = u64
        _lib = L
    return _lib


class OrcMzTable(ctypes.Structure):
    """The C struct of McFarland's modified ziggurat table (orc_mz_table)."""
    _fields_ = [
        ("n_buckets", ctypes.c_int), ("n_layers", ctypes.c_int), ("bits", ctypes.c_int),
        ("ubits", ctypes.c_int),
        ("xs", ctypes.c_double * 256), ("x0", ctypes.c_double),
        ("ox", ctypes.c_double * 257), ("odx", ctypes.c_double * 257),
        ("oy", ctypes.c_double * 257), ("ody", ctypes.c_double * 257),
        ("kind", ctypes.c_int * 257), ("thr", ctypes.c_uint64 * 256),
        ("alias", ctypes.c_int * 256),
    ]


_mz_table = None


def mz_struct(t):
    """The C struct of a modified-ziggurat table dict (oracle/table_mz.py)."""
    T = OrcMzTable()
    T.n_buckets, T.n_layers, T.bits, T.ubits = t["n_buckets"], t["n_layers"], t["bits"], t["ubits"]
    for i, v in enumerate(t["xs"]):
        T.xs[i] = v
    T.x0 = t["x0"]
    for k in range(t["n_layers"] + 1):
        T.ox[k], T.odx[k], T.oy[k], T.ody[k] = t["ox"][k], t["odx"][k], t["oy"][k], t["ody"][k]
        T.kind[k] = t["kind"][k]
    for j in range(t["n_buckets"]):
        T.thr[j] = int(t["thr"][j])
        T.alias[j] = t["alias"][j]
    return T


def mz_table():
    """The stored 256-bucket modified-ziggurat table as the C struct."""
    global _mz_table
    if _mz_table is None:
        _mz_table = mz_struct(table_mz.load())
    return _mz_table


def long_word(kind, seed, s, v, d):
    """nextLong word of draw d (the modified ziggurat's words)."""
    return int(lib().orc_long_word(kind, seed & (2**64 - 1), s, v, d))


def fill_mz(kind, seed, s, first, n, dmax=DMAX, nthreads=0, T=None):
    """Modified-ziggurat variates first..first+n-1 of one stream; returns
    (values, outcome codes, errors)."""
    return fill_streams_mz(kind, seed, s, 1, first, n, dmax, nthreads, T)


def fill_streams_mz(kind, seed, s0, n_streams, first, n_per, dmax=DMAX, nthreads=0, T=None):
    n = n_streams * n_per
    out = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_streams_mz(ctypes.byref(T or mz_table()), kind, seed & (2**64 - 1),
                                     s0, n_streams, first, n_per, dmax, _p(out), _p(cls),
                                     _threads(nthreads))
    return out, cls, int(errs)


def mz_tape(tape, dmax=DMAX, T=None, L=None):
    """One modified-ziggurat variate from crafted words; (value, outcome code,
    draw indices read)."""
    L = L or lib()
    arr = np.ascontiguousarray(tape, dtype=np.uint64)
    reads = np.zeros(4 * dmax + 8, dtype=np.uint32)
    nreads = ctypes.c_uint32()
    cls = ctypes.c_uint8()
    x = L.orc_mz_f64_tape(ctypes.byref(T or mz_table()), _p(arr), arr.size, dmax,
                          ctypes.byref(cls), _p(reads), reads.size, ctypes.byref(nreads))
    return x, cls.value, reads[:min(nreads.value, reads.size)].tolist()


def mz_enum(T, edges, L=None):
    """Exhaustive enumeration of a tiny modified-ziggurat format through the
    oracle's own steps (orc_mz_enum): (layer weights per signed bin, region
    counts per sign [r][neg], accepted weights per region and bin of the
    magnitude, accepted totals per region)."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    nb = e.size - 1
    nl = T.n_layers
    lb = np.zeros(nb, dtype=np.uint64)
    cnt = np.zeros(2 * (nl + 1), dtype=np.uint64)
    acc = np.zeros((nl + 1) * nb, dtype=np.uint64)
    tot = np.zeros(nl + 1, dtype=np.uint64)
    rc = (L or lib()).orc_mz_enum(ctypes.byref(T), _p(e), nb, _p(lb), _p(cnt), _p(acc), _p(tot))
    if rc == -1:
        raise ValueError("format too large to enumerate")
    if rc != 0:
        raise ValueError("a region index outside the table")
    return lb, cnt.reshape(nl + 1, 2), acc.reshape(nl + 1, nb), tot


def table_dict():
    """The stored oracle table (correctly rounded entries) as a dict."""
    global _table_dict
    if _table_dict is None:
        _table_dict = table_mp.load_table()
    return _table_dict


def table():
    """The stored oracle table as the C struct."""
    global _table
    if _table is None:
        t = table_dict()
        T = OrcTable()
        T.r = t["r"]
        for i in range(128):
            T.W[i] = t["W"][i]
            T.y[i] = t["y"][i]
            T.dy[i] = t["dy"][i]
            T.w53[i] = t["w53"][i]
            T.w24d[i] = t["w24d"][i]
            T.w24[i] = t["w24f"][i] * 2.0 ** -24
            T.k53[i] = t["k53"][i]
            T.k24[i] = t["k24"][i]
        _table = T
    return _table


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _threads(nthreads):
    return nthreads if nthreads else min(os.cpu_count() or 1, 64)


def word(kind, seed, s, v, d):
    L = lib()
    f = L.orc_lcg_word if kind == LCG48 else L.orc_sm64_word
    return int(f(seed & (2**64 - 1), s, v, d))


def words(kind, seed, s, d, first, n):
    out = np.empty(n, dtype=np.uint64)
    lib().orc_words(kind, seed & (2**64 - 1), s, d, first, n, _p(out))
    return out


def lcg_seq_doubles(seed, n):
    out = np.empty(n, dtype=np.uint64)
    lib().orc_lcg_seq_doubles(seed & (2**64 - 1), n, _p(out))
    return out


def lcg_seq_ints(seed, n):
    out = np.empty(n, dtype=np.int32)
    lib().orc_lcg_seq_ints(seed & (2**64 - 1), n, _p(out))
    return out


def lcg_affine(k):
    A = ctypes.c_uint64()
    C = ctypes.c_uint64()
    lib().orc_lcg_affine(k, ctypes.byref(A), ctypes.byref(C))
    return A.value, C.value


def fill_f64(kind, seed, s, first, n, dmax=DMAX, nthreads=0):
    """FP64 ziggurat variates first..first+n-1; returns (values, outcome codes, errors)."""
    out = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_f64(ctypes.byref(table()), kind, seed & (2**64 - 1), s, first, n,
                              dmax, _p(out), _p(cls), _threads(nthreads))
    return out, cls, int(errs)


def fill_streams_f64(kind, seed, s0, n_streams, first, n_per, dmax=DMAX, nthreads=0):
    """FP64 ziggurat variates first..first+n_per-1 of streams s0..s0+n_streams-1,
    stream-major; returns (values, outcome codes, errors)."""
    n = n_streams * n_per
    out = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_streams_f64(ctypes.byref(table()), kind, seed & (2**64 - 1), s0,
                                      n_streams, first, n_per, dmax, _p(out), _p(cls),
                                      _threads(nthreads))
    return out, cls, int(errs)


def fill_streams_f32(kind, seed, s0, n_streams, first, n_per, dmax=DMAX, nthreads=0):
    """FP32 mode over streams s0..s0+n_streams-1, stream-major; returns (values f32,
    FP64 value of the same decision, outcome codes, errors)."""
    n = n_streams * n_per
    out = np.empty(n, dtype=np.float32)
    out64 = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_streams_f32(ctypes.byref(table()), kind, seed & (2**64 - 1), s0,
                                      n_streams, first, n_per, dmax, _p(out), _p(out64), _p(cls),
                                      _threads(nthreads))
    return out, out64, cls, int(errs)


def fill_streams_polar(kind, seed, s0, n_streams, first, n_per, dmax=DMAX, nthreads=0):
    """Polar method over streams s0..s0+n_streams-1, stream-major; returns
    (values, outcome codes, errors)."""
    n = n_streams * n_per
    out = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_streams_polar(kind, seed & (2**64 - 1), s0, n_streams, first, n_per,
                                        dmax, _p(out), _p(cls), _threads(nthreads))
    return out, cls, int(errs)


def fill_f32(kind, seed, s, first, n, dmax=DMAX, nthreads=0):
    """FP32 ziggurat variates; returns (values f32, FP64 value of the same
    decision, outcome codes, errors)."""
    out = np.empty(n, dtype=np.float32)
    out64 = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_f32(ctypes.byref(table()), kind, seed & (2**64 - 1), s, first, n,
                              dmax, _p(out), _p(out64), _p(cls), _threads(nthreads))
    return out, out64, cls, int(errs)


def fill_polar(kind, seed, s, first, n, dmax=DMAX, nthreads=0):
    out = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    errs = lib().orc_fill_polar(kind, seed & (2**64 - 1), s, first, n, dmax, _p(out),
                                _p(cls), _threads(nthreads))
    return out, cls, int(errs)


def ea_rate53(rate):
    """The 53-bit mutation threshold of a per-gene rate: floor(rate 2^53),
    clamped to [0, 2^53]."""
    return max(0, min(1 << 53, int(float(rate) * 2.0 ** 53)))


def ea_step(parents, fitness, k, seed, stream, gen, rate, sigma, lo, hi, dmax=DMAX,
            nthreads=0, L=None):
    """One EA generation (orc_ea_step): parents (pop x genes float64) and
    fitness (pop) -> (children, winners, per-gene outcome codes, errors)."""
    P = np.ascontiguousarray(parents, dtype=np.float64)
    F = np.ascontiguousarray(fitness, dtype=np.float64)
    pop, genes = P.shape
    C = np.empty_like(P)
    W = np.empty(pop, dtype=np.uint32)
    cls = np.empty(P.shape, dtype=np.uint8)
    errs = (L or lib()).orc_ea_step(ctypes.byref(table()), _p(P), _p(F), _p(C), _p(W), _p(cls),
                                    pop, genes, k, seed & (2**64 - 1), stream, gen,
                                    ea_rate53(rate), sigma, lo, hi, dmax, _threads(nthreads))
    return C, W, cls, int(errs)


def mutate(x, kind, seed, s, first, sigma, dmax=DMAX, nthreads=0):
    """Returns a mutated copy of x (float64 array) and the outcome codes."""
    y = np.array(x, dtype=np.float64, copy=True)
    cls = np.empty(y.size, dtype=np.uint8)
    errs = lib().orc_mutate(ctypes.byref(table()), kind, seed & (2**64 - 1), s, first, y.size,
                            dmax, sigma, _p(y), _p(cls), _threads(nthreads))
    return y, cls, int(errs)


def decide_word(W, L=None):
    x = ctypes.c_double()
    c = (L or lib()).orc_decide_word(ctypes.byref(table()), W, ctypes.byref(x))
    return int(c), x.value


def zig_f64_tape(tape, dmax=DMAX, table_=None, L=None):
    """One FP64 variate from crafted words (word d = tape[d], 0 past the end).
    Returns (value, outcome code, list of the draw indices read in order)."""
    L = L or lib()
    arr = np.ascontiguousarray(tape, dtype=np.uint64)
    reads = np.zeros(4 * dmax + 8, dtype=np.uint32)
    nreads = ctypes.c_uint32()
    cls = ctypes.c_uint8()
    x = L.orc_zig_f64_tape(ctypes.byref(table_ or table()), _p(arr), arr.size, dmax,
                           ctypes.byref(cls), _p(reads), reads.size, ctypes.byref(nreads))
    return x, cls.value, reads[:min(nreads.value, reads.size)].tolist()


def small_table(twin_table):
    """The C table struct for a small twin table (n layers, thresholds and
    widths at its j width); layers past n stay zero."""
    T = OrcTable()
    T.r = twin_table.r
    for i in range(twin_table.n):
        T.W[i] = twin_table.W[i]
        T.y[i] = twin_table.y[i]
        T.dy[i] = twin_table.dy[i]
        T.w53[i] = twin_table.w[i]
        T.k53[i] = twin_table.k[i]
    return T


def attempt(T, i, j, W1, W2, L=None):
    """One attempt of the C oracle (orc_attempt): (code, x) with code 0 fast,
    1 wedge accept, 2 tail accept, 5 wedge reject, 6 tail reject."""
    x = ctypes.c_double()
    c = (L or lib()).orc_attempt(ctypes.byref(T), i, j, W1, W2, ctypes.byref(x))
    return int(c), x.value


def enum_attempt(T, n, jbits, ubits, edges, L=None):
    """Exhaustive enumeration of one attempt of the C oracle on a small table
    (orc_enum_attempt).  Returns (accepted weight, accepted weight per bin of
    |x|, accepted base-strip weight, total weight)."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    acc_bin = np.zeros(max(e.size - 1, 1), dtype=np.uint64)
    out = np.zeros(3, dtype=np.uint64)
    rc = (L or lib()).orc_enum_attempt(ctypes.byref(T), n, jbits, ubits, _p(e), e.size,
                                       _p(acc_bin), _p(out))
    if rc != 0:
        raise AssertionError("base-strip decisions depend on j")
    return int(out[0]), [int(c) for c in acc_bin], int(out[1]), int(out[2])


def load_variant(path):
    """Loads another build of the oracle source (a planted mistake in a copy,
    for the mutant tests) with the same signatures."""
    global _lib
    saved = _lib
    try:
        _lib = None
        src_lib = LIB
        globals()["LIB"] = path
        return lib()
    finally:
        globals()["LIB"] = src_lib
        _lib = saved


def polar_core(u1, u2):
    o1 = ctypes.c_double()
    o2 = ctypes.c_double()
    ok = lib().orc_polar_core(u1, u2, ctypes.byref(o1), ctypes.byref(o2))
    return bool(ok), o1.value, o2.value


def seq_f64(kind, seed, s, first, n, words=None, limit=None):
    """Sequential consumption: n variates taken from one generator in order
    (stream s of (seed, kind) from word position `first`, or, with kind 0,
    the crafted uint64 array `words`).  Returns (values, outcome codes, each
    variate's first position, the position after the last word read, the
    number of variates the generator could not complete)."""
    out = np.empty(n, dtype=np.float64)
    cls = np.empty(n, dtype=np.uint8)
    starts = np.empty(n, dtype=np.uint64)
    nxt = ctypes.c_uint64()
    arr = None
    if kind == 0:
        arr = np.ascontiguousarray(words, dtype=np.uint64)
        lim = arr.size if limit is None else limit
    else:
        lim = (2**64 - 1) if limit is None else limit
    fails = lib().orc_seq_f64(ctypes.byref(table()), kind, seed & (2**64 - 1), s, first, n,
                              _p(arr), lim, _p(out), _p(cls), _p(starts), ctypes.byref(nxt))
    return out, cls, starts, int(nxt.value), int(fails)
