"""Host-only unit tests of C++ pieces of the library that need no GPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_01117_amd", "csrc")


def test_arena_bookkeeping(tmp_path):
    """The server's first-fit arena: no overlap, refusal only when nothing
    fits, exact used/peak accounting, full coalescing after release; built
    with the address and undefined-behaviour sanitizers."""
    exe = tmp_path / "test_arena"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-I", CSRC,
                           os.path.join(ROOT, "tests", "cpp", "test_arena.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "arena ok" in out.stdout
