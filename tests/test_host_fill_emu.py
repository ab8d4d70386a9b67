"""The plain fill kernels' device source, built for the CPU with a HIP
stand-in (tests/host/shim) and AddressSanitizer, run through launch_fill:
the wave-specialised kernel (streaming waves publishing slow elements in an
LDS ring, drain waves resolving them) and the block-pooled kernel give every
element bit for bit as the oracle does, for FP64, FP32, mutation and the
modified ziggurat, both
uniform kinds, unaligned heads, multi-stream jobs with ragged streams, tiny
jobs and a job whose slow elements wrap the ring several times; no access
leaves its buffer and every wave leaves its loops.  The workgroups of a grid
run one after the other here, with their waves as concurrent threads, so the
ring protocol runs under real concurrency (not the GPU's scheduling)."""
import os

import numpy as np
import pytest

import kernel_emu


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("fill_emu"))
    try:
        exe = kernel_emu.build(d)
    except RuntimeError as e:
        pytest.fail(str(e))
    return d, exe


# op (0 FP64, 1 FP32, 3 mutation, 4 modified ziggurat), kind, seed, s0, n_streams, n_per, first, head,
# drain waves (0 = pooled kernel), steps per group, compute units (persistent
# workgroups)
CASES = [
    (0, 1, 7, 0, 1, 262144 + 37, 0, 1, 4, 4, 4),
    (0, 1, 99, 17, 701, 333, 5, 0, 2, 8, 3),
    (0, 2, 123456789, 3, 1, 100003, 1000, 1, 1, 2, 2),
    (1, 1, 8, 0, 4001, 37, 0, 3, 4, 1, 4),
    (1, 2, 11, 9, 1, 70001, 3, 2, 3, 4, 2),
    (3, 1, 1000, 3, 1, 131072 + 5, 0, 1, 4, 2, 4),
    (0, 1, 5, 2, 1, 5, 77, 1, 4, 4, 4),
    (0, 1, 5, 2, 1, 1, 0, 1, 4, 4, 4),
    (1, 1, 5, 2, 1, 3, 0, 2, 8, 4, 4),
    (0, 1, 42, 0, 1, 1_000_000, 0, 0, 4, 4, 2),
    (0, 1, 99, 17, 701, 333, 5, 1, 0, 2, 3),
    (1, 1, 8, 0, 4001, 37, 0, 1, 0, 8, 4),
    (0, 2, 77, 1, 3, 50001, 9, 1, 0, 1, 2),
    (4, 1, 7, 0, 1, 262144 + 37, 0, 1, 4, 4, 4),
    (4, 1, 99, 17, 701, 333, 5, 0, 2, 8, 3),
    (4, 2, 123456789, 3, 1, 100003, 1000, 1, 1, 2, 2),
    (4, 1, 5, 2, 1, 1, 0, 1, 4, 4, 4),
    (4, 1, 99, 17, 701, 333, 5, 1, 0, 2, 3),
    (4, 2, 77, 1, 3, 50001, 9, 1, 0, 1, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[
    "f64-sm64-ragged", "f64-multistream", "f64-lcg", "f32-multistream", "f32-lcg", "mutate",
    "f64-tiny", "f64-one", "f32-three", "f64-ring-wraps", "pooled-f64", "pooled-f32",
    "pooled-lcg-one-step", "mz-sm64", "mz-multistream", "mz-lcg", "mz-one", "mz-pooled",
    "mz-pooled-lcg"])
def test_fill_kernels_equal_oracle(emu, orc, case):
    op, kind, seed, s0, ns, n_per, first, head, drain, gsteps, cus = case
    d, exe = emu
    n = ns * n_per
    tag = "_".join(str(c) for c in case)
    out = os.path.join(d, f"out_{tag}.bin")
    args = ["fill", op, kind, seed, s0, ns, n_per, first, head, drain, gsteps, out]
    x0 = None
    if op == 3:
        rng = np.random.Generator(np.random.PCG64(5))
        x0 = rng.uniform(-5, 5, n)
        inp = os.path.join(d, f"in_{tag}.bin")
        x0.tofile(inp)
        args.append(inp)
    else:
        args.append("-")
    r = kernel_emu.run(exe, args, cus=cus)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "flags=0" in r.stderr, r.stderr
    if op == 1:
        got = np.fromfile(out, dtype=np.float32)
        want, _, _cls, errs = orc.fill_streams_f32(kind, seed, s0, ns, first, n_per)
    elif op == 3:
        got = np.fromfile(out, dtype=np.float64)
        want, _cls, errs = orc.mutate(x0, kind, seed, s0, first, 0.1)
    elif op == 4:
        got = np.fromfile(out, dtype=np.float64)
        want, _cls, errs = orc.fill_streams_mz(kind, seed, s0, ns, first, n_per)
    else:
        got = np.fromfile(out, dtype=np.float64)
        want, _cls, errs = orc.fill_streams_f64(kind, seed, s0, ns, first, n_per)
    assert errs == 0
    assert got.size == n
    bits = np.uint32 if op == 1 else np.uint64
    same = got.view(bits) == want.view(bits)
    assert same.all(), (int((~same).sum()), np.flatnonzero(~same)[:10])


@pytest.mark.parametrize("waves,drain,res", [(2, 4, 1), (6, 3, 3), (4, 1, 8)],
                         ids=["two-waves-drain-clamped", "six-waves", "four-waves-eight-per-cu"])
def test_ws_fill_small_workgroups_equal_oracle(emu, orc, waves, drain, res):
    """The wave-specialised fill in workgroups of 2 to 6 waves (drain waves
    clamped to leave one streaming wave), 1, 3 or 8 per compute unit (the
    stand-in reports room for 8): the same bits as the oracle."""
    d, exe = emu
    n_per, ns = 333, 301
    out = os.path.join(d, f"out_ws_{waves}_{drain}_{res}.bin")
    env = dict(EMU_WAVES=str(waves), EMU_RES=str(res), EMU_OCC="8")
    r = kernel_emu.run(exe, ["fill", 0, 1, 99, 17, ns, n_per, 5, 1, drain, 2, out, "-"], cus=3,
                       env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "flags=0" in r.stderr, r.stderr
    got = np.fromfile(out, dtype=np.float64)
    want, _cls, errs = orc.fill_streams_f64(1, 99, 17, ns, 5, n_per)
    assert errs == 0
    assert got.view(np.uint64).tolist() == want.view(np.uint64).tolist()
