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


# ------------------------------------------------------------ bench.py host legs

def test_bench_refuses_more_than_one_gpu():
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stdout


def test_bench_thread_axis_is_bitwise_stable():
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_2307_01117_amd import inputs
    u0 = inputs.make_initial("uniform", 50_001, 1)
    rep = bench.cpu_threads(u0, 0.5, 3, "ring_50001", max_threads=2)
    assert rep["kind"] == "oracle_threads" and rep["threads"][0] == 1
    for name, s in rep["samples"].items():
        assert s["bitwise_equal_across_threads"], name
        assert len(s["value"]) == len(rep["threads"]) and min(s["value"]) > 0
        assert len(s["value_simd"]) == len(rep["threads"]) and min(s["value_simd"]) > 0


def test_inplace_solve_rejects_arrays_it_cannot_write():
    """The binding's in-place plain form refuses, before any library call,
    arrays whose memory the library could not advance in place."""
    import numpy as np
    import pytest
    from paper_2307_01117_amd import heat
    ro = np.zeros(8)
    ro.flags.writeable = False
    for bad in (np.zeros(8, np.float32), np.zeros((4, 4))[:, 0], ro, [0.0] * 8):
        with pytest.raises(ValueError):
            heat.solve(bad, 1, 0.5, 1, inplace=True)
