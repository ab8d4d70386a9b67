"""The sequential passes' device source, built for the CPU with a HIP
stand-in (tests/host/shim) and AddressSanitizer, at more than 1024
workgroups (so the scan pass composes several workgroup maps per thread):
every access stays in its buffer, and every value and the position after the
last word read equal the oracle's sequential routine.  To reach that many
workgroups at a size the CPU runs in seconds, the test build uses one window
of 64 positions per chunk (the source with that one constant changed)."""
import os
import subprocess

import numpy as np
import pytest

import kernel_emu


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("seq_emu"))
    try:
        exe = kernel_emu.build(d, seq_windows=1)
    except RuntimeError as e:
        pytest.fail(str(e))
    return d, exe


@pytest.mark.parametrize("kind,seed,s,first,n", [(1, 7, 0, 0, 1_000_000)])
def test_sequential_source_beyond_1024_workgroups(emu, orc, kind, seed, s, first, n):
    d, exe = emu
    out = os.path.join(d, f"out_{kind}.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe, str(n), str(kind), str(seed), str(s), str(first), out],
                       capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    wg = int(r.stderr.split("workgroups=")[1].split()[0])
    assert wg > 1024, r.stderr
    raw = np.fromfile(out, dtype=np.uint64)
    nxt, g = int(raw[0]), raw[1:]
    o, cls, starts, o_next, fails = orc.seq_f64(kind, seed, s, first, n)
    assert fails == 0
    assert np.array_equal(g, o.view(np.uint64))
    assert nxt == o_next


@pytest.mark.parametrize("n_wg", [1, 1024, 1025, 4096, 17220, 65536])
def test_scan_pass_composes_many_maps_per_thread(emu, n_wg):
    """The scan pass alone over synthetic workgroup maps (random counts and
    exits), from one workgroup up to 64 maps per thread (17220 is the plan of
    2^28 variates): each workgroup's entry and the scan total equal the maps
    composed one at a time, and no access leaves its buffer."""
    d, exe = emu
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe, "scan", str(n_wg), str(n_wg + 7)], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith(f"scan ok n_wg={n_wg}"), r.stdout
