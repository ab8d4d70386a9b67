"""The built library exports every function include/zg.h declares (no GPU
needed: the symbols are read from the shared object's dynamic table)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zg.h")
LIB = os.path.join(ROOT, "paper_2405_19493_amd", "libzg.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"^\s*(?:zg_status|const char\s*\*|double)\s*(zg_\w+)\s*\(", text, flags=re.M))
    return names


def test_header_declares_the_boundary():
    names = declared()
    for need in ("zg_create", "zg_destroy", "zg_table", "zg_fill", "zg_fill_streams",
                 "zg_uniform_words", "zg_mutate", "zg_batch", "zg_stream_open", "zg_stream_fill",
                 "zg_server_create", "zg_server_submit", "zg_server_poll", "zg_server_destroy",
                 "zg_error_flags", "zg_decide_words", "zg_strerror", "zg_fill_sequential",
                 "zg_sequential_workspace"):
        assert need in names, need


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libzg.so is not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = sorted(declared() - exported)
    assert not missing, missing
