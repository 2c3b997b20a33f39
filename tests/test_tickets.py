"""The serving loop's ticket table on the host: built with g++ from its header
alone (no device code) and run; more requests are submitted than the table
keeps, and memory must stay bounded."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ticket_table_bounded(tmp_path):
    exe = tmp_path / "ticket_table_test"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-Wextra", "-Werror",
                           "-I", os.path.join(ROOT, "paper_2406_09255_amd", "csrc"),
                           os.path.join(ROOT, "tests", "tickets", "ticket_table_test.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "ticket table ok" in r.stdout
