"""Builds the device source of libzg for the CPU (tests/host/kernel_emu.cpp
with the HIP stand-in in tests/host/shim) under AddressSanitizer.  Used by
the CPU tests of the kernels' index arithmetic and work-queue protocols."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2405_19493_amd", "csrc")
INCLUDE = os.path.join(HERE, "..", "include")


def build(dst, seq_windows=None):
    """Writes the host build of the kernel source into dst and compiles the
    emulator; seq_windows replaces the windows per sequential chunk (so that a
    small job plans many workgroups).  Returns the executable's path, or
    raises with the compiler's output."""
    k = open(os.path.join(CSRC, "zg_kernels.hip")).read()
    k = k.replace("extern __shared__", "extern").replace("__shared__", "static")
    k = k.replace("#include <hip/hip_runtime.h>", '#include "hip/hip_runtime.h"')
    open(os.path.join(dst, "zg_kernels_emu.cpp"), "w").write(k)
    h = open(os.path.join(CSRC, "zg_internal.h")).read()
    h = h.replace('"../../include/zg.h"', '"zg.h"')
    if seq_windows is not None:
        assert "constexpr uint32_t SEQ_WINDOWS = 16;" in h
        h = h.replace("constexpr uint32_t SEQ_WINDOWS = 16;",
                      f"constexpr uint32_t SEQ_WINDOWS = {int(seq_windows)};")
    open(os.path.join(dst, "zg_internal.h"), "w").write(h)
    for name, src in (("zg_table.cpp", CSRC), ("zg.h", INCLUDE)):
        open(os.path.join(dst, name), "w").write(open(os.path.join(src, name)).read())
    exe = os.path.join(dst, "kernel_emu")
    r = subprocess.run(["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address",
                        "-fno-omit-frame-pointer", "-I", os.path.join(HERE, "host", "shim"),
                        "-I", dst, os.path.join(HERE, "host", "kernel_emu.cpp"), "-o", exe,
                        "-lpthread"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stdout[-3000:] + r.stderr[-3000:])
    return exe


def run(exe, args, cus=None, timeout=600, env=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", **(env or {}))
    if cus is not None:
        env["EMU_CUS"] = str(cus)
    return subprocess.run([exe, *[str(a) for a in args]], capture_output=True, text=True,
                          timeout=timeout, env=env)
