"""The library used from plain C (tests/c_abi/cuckoo_then_iceberg.c): it
compiles with the host C compiler against include/cpht.h alone, and on a GPU
the program's answers are all as expected."""
from __future__ import annotations

import os
import subprocess

import pytest

from tests.c_abi import build as cbuild


def test_c_example_compiles_against_the_header(tmp_path):
    out = cbuild.build(str(tmp_path / "example"))
    assert os.path.exists(out)


@pytest.mark.gpu
def test_c_example_runs(gpu):
    exe = cbuild.BIN
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(cbuild.SRC):
        exe = cbuild.build()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("c-abi ok")
