"""The EA generation kernel's device source, built for the CPU with the HIP
stand-in and AddressSanitizer (tests/host/kernel_emu.cpp, mode ea), run
through launch_ea: winners and children equal the oracle's bit for bit, with
tournaments of 1 to 70 draws (more draws than lanes), NaN and tied fitness,
one-gene genomes and ragged gene counts, and rates up to 1 (several rounds of
64 mutating genes per chunk group, and leftovers carried between groups);
no access leaves its buffer."""
import os

import numpy as np
import pytest

import kernel_emu


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("ea_emu"))
    try:
        exe = kernel_emu.build(d)
    except RuntimeError as e:
        pytest.fail(str(e))
    return d, exe


CASES = [(37, 70, 2, 3, 0.1, 0.5, -2.0, 2.0, False), (5, 1, 1, 0, 1.0, 3.0, -1.0, 1.0, False),
         (300, 129, 4, 7, 0.05, 0.1, -5.0, 5.0, True), (64, 64, 70, 1, 0.5, 1.0, -1.5, 1.5, True),
         (20, 700, 3, 2, 0.9, 0.2, -3.0, 3.0, False), (9, 769, 2, 5, 1.0, 0.5, -4.0, 4.0, False)]


@pytest.mark.parametrize("case", CASES, ids=["ragged", "one-gene", "nan", "wide-tournament",
                                              "most-mutate", "all-mutate"])
def test_ea_kernel_equals_oracle(emu, orc, case):
    pop, genes, k, gen, rate, sigma, lo, hi, nanfit = case
    d, exe = emu
    rng = np.random.Generator(np.random.PCG64(pop))
    P = rng.uniform(-2, 2, (pop, genes))
    F = np.floor(rng.uniform(0, 10, pop))   # ties
    if nanfit:
        F[::3] = np.nan
    files = [os.path.join(d, f"{n}_{pop}.bin") for n in ("p", "f", "c", "w")]
    P.tofile(files[0])
    F.tofile(files[1])
    r = kernel_emu.run(exe, ["ea", pop, genes, k, 123, 10, gen, rate, sigma, lo, hi, *files])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "flags=0" in r.stderr
    C = np.fromfile(files[2], dtype=np.float64).reshape(pop, genes)
    W = np.fromfile(files[3], dtype=np.uint32)
    Co, Wo, _cls, errs = orc.ea_step(P, F, k, 123, 10, gen, rate, sigma, lo, hi)
    assert errs == 0
    assert np.array_equal(W, Wo)
    assert C.tobytes() == Co.tobytes()
