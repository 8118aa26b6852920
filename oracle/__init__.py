"""CPU oracle for the periodic 1D heat stencil -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline legs of
``bench.py`` (``cpu_baseline``, ``cpu_threads``) may import this package.  The GPU library never imports, links or
calls it and shares no code with it.

Two independent implementations of the same definition live here:

* ``heat_oracle.c`` (plain C, built with ``-O2 -ffp-contract=off``), loaded
  through ctypes: ``solve``, ``solve_parts``, ``solve_threads`` (one POSIX
  thread per segment, ghost cells through queues; with ``simd=True`` its
  segment sweep is the vectorised one of ``heat_cpu_simd.c``, built with
  ``-O3``, bit-identical), ``cone``, ``solve_f32``,
  ``cone_f32``, ``solve_f32c``, ``cone_f32c`` (and, composed around the
  binary32 ones in NumPy, the mean-shifted storage ``solve_f32_shifted``,
  ``solve_f32c_shifted``);
* NumPy ring shifts (``np_solve``, ``np_solve_f32``, ``np_solve_f32c``), one
  ufunc per arithmetic operation, so every operation is rounded on its own
  exactly as in the C code.

Both follow the paper's Section 2 ("Model problem"): Eq. (heat:discrete) with
r = alpha*dt/h^2, the periodic boundary u(t, x) = u(t, L + x), and the
segment-plus-ghost-zone parallel algorithm of that section's last paragraph.
The FP32 and compensated-FP32 forms are the library's reduced-precision forms
of the same update; their definition is in ``heat_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heat_oracle.c")
_SRC_SIMD = os.path.join(_HERE, "heat_cpu_simd.c")
_LIB = os.path.join(_HERE, "libheat_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile heat_oracle.c (-O2, scalar) and heat_cpu_simd.c (-O3, the
    vectorised segment sweep) with gcc, both with no FMA contraction and no
    fast-math, and link them into one library."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        fp = ["-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
              "-fPIC"]
        with tempfile.TemporaryDirectory() as d:
            o1, o2 = os.path.join(d, "oracle.o"), os.path.join(d, "simd.o")
            subprocess.check_call(["gcc", "-O2", *fp, "-pthread", "-c", "-o", o1, _SRC])
            subprocess.check_call(["gcc", "-O3", *fp, "-c", "-o", o2, _SRC_SIMD])
            subprocess.check_call(["gcc", "-shared", "-pthread", "-o", tmp, o1, o2, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    d, f, i64 = ctypes.c_double, ctypes.c_float, ctypes.c_int64
    p = ctypes.c_void_p
    lib.heat_oracle_solve.argtypes = [p, p, i64, d, i64]
    lib.heat_oracle_solve.restype = None
    lib.heat_oracle_solve_parts.argtypes = [p, p, i64, i64, d, i64]
    lib.heat_oracle_solve_parts.restype = None
    lib.heat_oracle_solve_threads.argtypes = [p, p, i64, i64, d, i64]
    lib.heat_oracle_solve_threads.restype = ctypes.c_int
    lib.heat_oracle_solve_threads_simd.argtypes = [p, p, i64, i64, d, i64]
    lib.heat_oracle_solve_threads_simd.restype = ctypes.c_int
    lib.heat_oracle_cone.argtypes = [p, i64, d]
    lib.heat_oracle_cone.restype = d
    lib.heat_oracle_solve_f32.argtypes = [p, p, i64, f, i64]
    lib.heat_oracle_solve_f32.restype = None
    lib.heat_oracle_cone_f32.argtypes = [p, i64, f]
    lib.heat_oracle_cone_f32.restype = f
    lib.heat_oracle_solve_f32c.argtypes = [p, p, p, i64, d, i64, i64]
    lib.heat_oracle_solve_f32c.restype = None
    lib.heat_oracle_cone_f32c.argtypes = [p, i64, d, i64]
    lib.heat_oracle_cone_f32c.restype = f
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(u) -> np.ndarray:
    return np.ascontiguousarray(u, dtype=np.float64)


def _f32(u) -> np.ndarray:
    return np.ascontiguousarray(u, dtype=np.float32)


# ---------------------------------------------------------------- C oracle

def solve(u0, r: float, nt: int) -> np.ndarray:
    """nt steps of Eq. (heat:discrete) on the periodic ring, binary64."""
    a = _f64(u0)
    out = np.empty_like(a)
    if a.size:
        _load().heat_oracle_solve(_ptr(a), _ptr(out), a.size, float(r), int(nt))
    return out


def solve_parts(u0, nparts: int, r: float, nt: int) -> np.ndarray:
    """Segmented solver with a ghost-zone exchange every step (Section 2)."""
    a = _f64(u0)
    if not 1 <= nparts <= a.size:
        raise ValueError("need 1 <= nparts <= N")
    out = np.empty_like(a)
    _load().heat_oracle_solve_parts(_ptr(a), _ptr(out), a.size, int(nparts), float(r), int(nt))
    return out


def solve_threads(u0, nparts: int, r: float, nt: int, simd: bool = False) -> np.ndarray:
    """The same segmented solver with one thread per segment and the ghost
    cells passed through single-producer single-consumer queues, as the
    paper's CPU codes run it (Section 2, last paragraph).  ``simd``: the
    segment sweep vectorised, as the paper's SIMD build of its Rust code
    (Section 3); bit-identical."""
    a = _f64(u0)
    if not 1 <= nparts <= min(a.size, 4096) or nt < 0:
        raise ValueError("need 1 <= nparts <= min(N, 4096) and nt >= 0")
    out = np.empty_like(a)
    lib = _load()
    fn = lib.heat_oracle_solve_threads_simd if simd else lib.heat_oracle_solve_threads
    rc = fn(_ptr(a), _ptr(out), a.size, int(nparts), float(r), int(nt))
    if rc != 0:
        raise MemoryError(f"threaded oracle failed ({rc}): no memory or threads")
    return out


def cone_window(u0: np.ndarray, i: int, nt: int) -> np.ndarray:
    """The 2*nt+1 initial values around cell i, taken around the ring."""
    n = u0.size
    idx = (np.arange(i - nt, i + nt + 1, dtype=np.int64)) % n
    return u0[idx]


def cone(u0, i: int, r: float, nt: int) -> float:
    """Value of cell i after nt steps, from its light cone only (binary64)."""
    w = _f64(cone_window(np.asarray(u0), int(i), int(nt)))
    return float(_load().heat_oracle_cone(_ptr(w), int(nt), float(r)))


def solve_f32(u0, r: float, nt: int) -> np.ndarray:
    """Plain binary32 form: c + r*((q - c) - (c - l))."""
    a = _f32(u0)
    out = np.empty_like(a)
    if a.size:
        _load().heat_oracle_solve_f32(_ptr(a), _ptr(out), a.size, np.float32(r), int(nt))
    return out


def cone_f32(u0, i: int, r: float, nt: int) -> np.float32:
    w = _f32(cone_window(np.asarray(u0), int(i), int(nt)))
    return np.float32(_load().heat_oracle_cone_f32(_ptr(w), int(nt), np.float32(r)))


def solve_f32c(u0, r: float, nt: int, T: int, return_pair: bool = False):
    """Compensated binary32 form in rounds of T steps.

    With ``return_pair`` the last fold is skipped and (u, e) is returned, whose
    unevaluated sum carries the compensated state.
    """
    a = _f32(u0)
    out = np.empty_like(a)
    e = np.empty_like(a) if return_pair else None
    if a.size:
        _load().heat_oracle_solve_f32c(_ptr(a), _ptr(out), _ptr(e) if e is not None else None,
                                       a.size, float(r), int(nt), int(T))
    return (out, e) if return_pair else out


def cone_f32c(u0, i: int, r: float, nt: int, T: int) -> np.float32:
    w = _f32(cone_window(np.asarray(u0), int(i), int(nt)))
    return np.float32(_load().heat_oracle_cone_f32c(_ptr(w), int(nt), float(r), int(T)))


# -------------------------------------------------------- mean-shifted storage
# The binary32 forms applied to offsets from a constant s: v0 = fl32(u0 - s)
# (difference in binary64, then rounded to nearest even), the binary32 form
# on v, and u = s + v in binary64.  A constant is a fixed point of the update
# (its second difference is zero), so in exact arithmetic s + v evolves
# exactly as u does; s = 0 is the plain rounding and widening.

def to_offsets(u0, shift: float) -> np.ndarray:
    a = _f64(u0)
    if shift == 0:
        return a.astype(np.float32)
    return (a - np.float64(shift)).astype(np.float32)


def from_offsets(v, shift: float) -> np.ndarray:
    w = np.asarray(v, dtype=np.float32).astype(np.float64)
    if shift == 0:
        return w
    return np.float64(shift) + w


def solve_f32_shifted(u0, r: float, nt: int, shift: float) -> np.ndarray:
    """Plain binary32 form on offsets from ``shift``; binary64 result."""
    return from_offsets(solve_f32(to_offsets(u0, shift), r, nt), shift)


def solve_f32c_shifted(u0, r: float, nt: int, T: int, shift: float) -> np.ndarray:
    """Compensated binary32 form on offsets from ``shift``; binary64 result."""
    return from_offsets(solve_f32c(to_offsets(u0, shift), r, nt, T), shift)


# -------------------------------------------------------- NumPy second oracle

def np_solve(u0, r: float, nt: int) -> np.ndarray:
    """Same definition with NumPy ring shifts; one rounding per ufunc."""
    a = _f64(u0).copy()
    r = np.float64(r)
    for _ in range(int(nt)):
        left = np.roll(a, 1)     # left[i]  = a[i-1 mod N]
        right = np.roll(a, -1)   # right[i] = a[i+1 mod N]
        a = a + r * ((left - 2.0 * a) + right)
    return a


def np_solve_f32(u0, r: float, nt: int) -> np.ndarray:
    a = _f32(u0).copy()
    r = np.float32(r)
    for _ in range(int(nt)):
        left = np.roll(a, 1)
        right = np.roll(a, -1)
        a = a + r * ((right - a) - (a - left))
    return a


def fma32(a, b, c) -> np.ndarray:
    """fl32(a*b + c) with one rounding (binary32 fused multiply-add), for
    binary32 arrays: a*b is exact in binary64 (two 24-bit significands); the
    binary64 sum s and its exact error err (TwoSum) give a*b + c = s + err
    exactly, and rounding s to binary32 rounds the exact sum the same way
    unless s lies exactly halfway between two binary32 neighbours and err is
    not zero -- then the exact sum lies on err's side of that midpoint."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    c = np.asarray(c, dtype=np.float32)
    p = a.astype(np.float64) * b.astype(np.float64)
    c64 = c.astype(np.float64)
    s = p + c64
    bp = s - p
    err = (p - (s - bp)) + (c64 - bp)
    r = s.astype(np.float32)
    r64 = r.astype(np.float64)
    lo = np.nextafter(r, np.float32(-np.inf))
    hi = np.nextafter(r, np.float32(np.inf))
    tie_lo = (s == (r64 + lo.astype(np.float64)) * 0.5) & (err < 0)
    tie_hi = (s == (r64 + hi.astype(np.float64)) * 0.5) & (err > 0)
    return np.where(tie_lo, lo, np.where(tie_hi, hi, r))


def np_solve_f32c(u0, r: float, nt: int, T: int) -> np.ndarray:
    u = _f32(u0).copy()
    rh = np.float32(r)
    rl = np.float32(float(r) - float(rh))
    done = 0
    while done < nt:
        s = min(T, nt - done)
        e = np.zeros_like(u)
        for _ in range(s):
            l, q = np.roll(u, 1), np.roll(u, -1)
            el, eq = np.roll(e, 1), np.roll(e, -1)
            L = ((q - u) + (eq - e)) - ((u - l) + (e - el))
            t = fma32(rh, L, u)
            res = fma32(rh, L, u - t)
            e = fma32(rl, L, res) + e
            u = t
        u = u + e
        done += s
    return u
