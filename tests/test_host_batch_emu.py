"""The batch class kernels' device source, built for the CPU with the HIP
stand-in and AddressSanitizer (tests/host/kernel_emu.cpp, mode batch), run
through launch_batch_class over requests laid out as zg_batch lays them out.
The wave-specialised class kernel (streaming waves taking (item, group)
units, ring and retry entries that name their request, drain waves reading
each entry's job from its request) and the block-pooled one give every
element of every request bit for bit as the oracle does: FP64, FP32 and
mutation, both uniform kinds, requests of 1 element to several tiles,
unaligned heads, grids smaller than the item count, and a ring that wraps;
no access leaves its buffer and every wave leaves its loops."""
import os

import numpy as np
import pytest

import kernel_emu


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("batch_emu"))
    try:
        exe = kernel_emu.build(d)
    except RuntimeError as e:
        pytest.fail(str(e))
    return d, exe


SIZES = [1, 2, 37, 255, 256, 257, 4095, 20000, 70001, 262147]
SMALL = [1, 3, 5, 64, 100, 129, 300, 511, 700, 1000] * 4

# op (0 FP64, 1 FP32, 3 mutation), kind, sizes, ws, waves, drain waves,
# steps per group, tile (elements per wave), grid (workgroups)
CASES = [
    (0, 1, SIZES, 1, 8, 2, 2, 256, 3),
    (0, 1, SIZES, 1, 16, 4, 4, 1024, 2),
    (0, 1, SIZES, 0, 8, 0, 4, 256, 3),
    (1, 1, SIZES, 1, 8, 3, 1, 256, 4),
    (3, 1, SIZES, 1, 8, 2, 2, 512, 3),
    (0, 2, SIZES[:9], 1, 8, 2, 2, 256, 3),
    (1, 2, SIZES[:9], 1, 4, 1, 8, 256, 2),
    (0, 1, SMALL, 1, 8, 1, 2, 256, 5),
    (1, 1, SMALL, 1, 16, 8, 8, 2048, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[
    "f64-ws", "f64-ws-default-shape", "f64-pooled", "f32-ws", "mutate-ws", "f64-lcg-ws",
    "f32-lcg-ws", "f64-many-small", "f32-many-small-one-workgroup"])
def test_batch_class_kernels_equal_oracle(emu, orc, case):
    op, kind, sizes, ws, waves, drain, gsteps, tile, grid = case
    d, exe = emu
    per16 = 4 if op == 1 else 2
    spec = [(op, kind, n, 1000 + k, k, k % per16) for k, n in enumerate(sizes)]
    tag = "_".join(str(c) for c in (op, kind, len(sizes), ws, waves, drain, gsteps, tile, grid))
    sp = os.path.join(d, f"spec_{tag}.txt")
    with open(sp, "w") as f:
        for row in spec:
            f.write(" ".join(str(v) for v in row) + "\n")
    out = os.path.join(d, f"out_{tag}.bin")
    inp = os.path.join(d, f"in_{tag}.bin")
    x0 = None
    if op == 3:
        x0 = np.random.Generator(np.random.PCG64(6)).uniform(-5, 5, sum(sizes))
        x0.tofile(inp)
    r = kernel_emu.run(exe, ["batch", ws, waves, drain, gsteps, tile, grid, sp, out,
                             inp if op == 3 else "-"])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "flags=0" in r.stderr, r.stderr
    got = np.fromfile(out, dtype=np.float32 if op == 1 else np.float64)
    assert got.size == sum(sizes)
    at = 0
    for k, (op_, kind_, n, seed, stream, head) in enumerate(spec):
        if op == 1:
            want, _, _, errs = orc.fill_f32(kind, seed, stream, 0, n)
        elif op == 3:
            want, _, errs = orc.mutate(x0[at:at + n], kind, seed, stream, 0, 0.1)
        else:
            want, _, errs = orc.fill_f64(kind, seed, stream, 0, n)
        assert errs == 0
        bits = np.uint32 if op == 1 else np.uint64
        g = got[at:at + n]
        same = g.view(bits) == want.view(bits)
        assert same.all(), (k, n, head, int((~same).sum()), np.flatnonzero(~same)[:8])
        at += n
