"""The serving loop's host code (context, batch planner, staging slots and
their graphs, zg_server_*) built for the CPU against the runtime stand-in in
tests/host/rt_shim, under ThreadSanitizer and under AddressSanitizer with
UndefinedBehaviorSanitizer: several client threads submit, wait and release
while the batcher and completion threads run; then the C-driven replay, and
a replay whose deadline passes so that the server releases late requests.
Every range follows its handle's submission order, every output element is
the one its range gives, nothing stays in flight, and the sanitizers report
nothing.  Run with up to 4 HIP streams per server (the stand-in build raises
the stream cap that the GPU build keeps at 2)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2405_19493_amd", "csrc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SOURCES = [os.path.join(CSRC, f) for f in ("zg_api.cpp", "zg_batch.cpp", "zg_server.cpp",
                                           "zg_table.cpp")]


def _build(dst, sanitize):
    exe = os.path.join(dst, "server_rt_" + sanitize.replace(",", "_"))
    r = subprocess.run([CLANG, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}",
                        "-fno-omit-frame-pointer", "-DZG_SERVER_MAX_STREAMS=4",
                        "-I", os.path.join(HERE, "host", "rt_shim"), *SOURCES,
                        os.path.join(HERE, "host", "server_rt.cpp"), "-o", exe, "-lpthread"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stdout[-3000:] + r.stderr[-3000:])
    return exe


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    if not shutil.which(CLANG) and not os.path.exists(CLANG):
        pytest.skip("clang++ with the sanitizer runtimes is not installed")
    d = str(tmp_path_factory.mktemp("server_rt"))
    return {"thread": _build(d, "thread"), "address": _build(d, "address,undefined")}


# streams, client threads, requests per client, handles, mode (0 batched, 1 per request)
CASES = [(4, 8, 300, 32, 0), (4, 4, 200, 16, 1), (2, 8, 300, 32, 0), (1, 4, 150, 8, 0)]


@pytest.mark.parametrize("san", ["thread", "address"])
@pytest.mark.parametrize("case", CASES, ids=["4streams", "4streams-per-request", "2streams",
                                             "1stream"])
def test_server_host_code_under_sanitizers(builds, san, case):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([builds[san], *map(str, case)], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "server ok" in r.stdout, r.stdout + r.stderr[-3000:]
    for bad in ("WARNING: ThreadSanitizer", "ERROR: AddressSanitizer", "runtime error:",
                "ERROR: LeakSanitizer"):
        assert bad not in r.stderr, r.stderr[-6000:]
