"""ctypes binding of libheat.so (the HIP library built from csrc/).

Argument marshalling only: every step of the computation runs in the
library's kernels.  The names follow include/heat.h.  If the library is not
built, every call raises -- there is no CPU fallback.

Device arrays are torch tensors on the current HIP device (torch supplies
memory and streams only); the stream defaults to torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheat.so")

HEAT_OK, HEAT_PENDING = 0, 1
HEAT_EINVAL, HEAT_ENOMEM, HEAT_EBUSY, HEAT_ENOENT, HEAT_EDEVICE, HEAT_ECANCELED = -1, -2, -3, -4, -5, -6
FP64, FP32, FP32C = 0, 1, 2
KERNEL_AUTO, KERNEL_STEP, KERNEL_TB, KERNEL_RESIDENT = 0, 1, 2, 3
EXCHANGE_AUTO, EXCHANGE_NONE, EXCHANGE_LDS, EXCHANGE_LDS_DEEP = 0, 1, 2, 3
BATCH_WAIT, BATCH_PERSISTENT, BATCH_GRAPH = 1, 2, 4

PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp32c": FP32C}

# every symbol declared in include/heat.h
EXPORTS = [
    "heat_solve", "heat_solve_dev", "heat_solve_dev_cfg", "heat_plan", "heat_checksum_dev",
    "heat_solve_batch", "heat_solve_batch_dev", "heat_server_create", "heat_submit",
    "heat_poll", "heat_wait", "heat_cancel", "heat_server_get_stats", "heat_server_destroy",
    "heat_last_error", "heat_version", "heat_device_info", "heat_copy_dev",
    "heat_autotune", "heat_tune_save", "heat_tune_load", "heat_solve_dev_noalloc",
    "heat_autotune_batch", "heat_autotune_resident",
]

NOALLOC_SCRATCH_BYTES = 64 << 20   # HEAT_NOALLOC_SCRATCH_BYTES


class HeatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"heat error {code}: {msg}")
        self.code = code


class heat_config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("cells_per_lane", ctypes.c_int32),
                ("steps_per_round", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("register_form", ctypes.c_int32), ("exchange", ctypes.c_int32)]


class heat_plan_info(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("cells_per_lane", ctypes.c_int32),
                ("steps_per_round", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("register_form", ctypes.c_int32), ("exchange_steps", ctypes.c_int32),
                ("tile_cells", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("rounds", ctypes.c_int64)]


class heat_problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("nparts", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("r", ctypes.c_double), ("nt", ctypes.c_int64), ("u0", ctypes.c_void_p),
                ("u_out", ctypes.c_void_p), ("sum0", ctypes.c_double), ("sum_nt", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("latency_s", ctypes.c_double), ("shift", ctypes.c_double)]


class heat_ring(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("nt", ctypes.c_int64), ("r", ctypes.c_double),
                ("precision", ctypes.c_int32), ("nparts", ctypes.c_int32),
                ("d_u", ctypes.c_void_p), ("d_work", ctypes.c_void_p)]


class heat_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("cancelled", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("cell_updates", ctypes.c_uint64), ("hbm_budget", ctypes.c_size_t),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("active", ctypes.c_int32), ("queued", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libheat.so and declare the signatures of include/heat.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2307_01117_amd.build`")
    # torch (which supplies device memory and streams) ships its own HIP and
    # ROCr runtimes under the same sonames as the ones the library links:
    # loading torch first makes the library bind to those, so the process
    # holds one runtime (loaded the other way round, torch's runtime finds
    # no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    lib.heat_version.restype = ctypes.c_char_p
    built = lib.heat_version().decode().rsplit(" ", 1)[-1]
    from paper_2307_01117_amd.build import source_digest
    if built != source_digest():
        raise RuntimeError(f"{path} was built from other sources (src {built[:16]}, tree "
                           f"{source_digest()[:16]}): rebuild with "
                           "`python -m paper_2307_01117_amd.build`")
    i32, i64, d, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    pd = ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "heat_solve": ([vp, i64, i32, d, i64], i32),
        "heat_solve_dev": ([vp, i64, i32, d, i64, i32, vp, pd, pd], i32),
        "heat_solve_dev_noalloc": ([vp, i64, i32, d, i64, i32, vp, vp], i32),
        "heat_solve_dev_cfg": ([vp, vp, i64, i32, d, i64, i32, P(heat_config), vp, pd, pd], i32),
        "heat_plan": ([i64, i64, i32, P(heat_config), P(heat_plan_info)], i32),
        "heat_checksum_dev": ([vp, i64, i32, vp, pd], i32),
        "heat_solve_batch": ([P(heat_problem), i32], i32),
        "heat_solve_batch_dev": ([P(heat_ring), i32, vp, i32], i32),
        "heat_server_create": ([ctypes.c_size_t, i32, i32, P(vp)], i32),
        "heat_submit": ([vp, P(heat_problem), P(ctypes.c_uint64)], i32),
        "heat_poll": ([vp, ctypes.c_uint64], i32),
        "heat_wait": ([vp, ctypes.c_uint64], i32),
        "heat_cancel": ([vp, ctypes.c_uint64], i32),
        "heat_server_get_stats": ([vp, P(heat_server_stats)], i32),
        "heat_server_destroy": ([vp], i32),
        "heat_last_error": ([], ctypes.c_char_p),
        "heat_version": ([], ctypes.c_char_p),
        "heat_device_info": ([P(i32), P(i32), P(i32), P(i32), P(ctypes.c_size_t),
                              P(ctypes.c_size_t)], i32),
        "heat_copy_dev": ([vp, vp, ctypes.c_size_t, vp], i32),
        "heat_autotune": ([i32, i64, i32, P(heat_config), pd], i32),
        "heat_autotune_batch": ([i32, i64, i32, P(i32), P(i32), P(i32), pd], i32),
        "heat_autotune_resident": ([i32, i64, i32, P(heat_config), P(i64), pd], i32),
        "heat_tune_save": ([ctypes.c_char_p], i32),
        "heat_tune_load": ([ctypes.c_char_p], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    # launch shapes measured on MI355X by `python -m paper_2307_01117_amd.autotune`
    table = os.path.join(_HERE, "tune_mi355x.txt")
    if not os.environ.get("HEAT_TUNE_TABLE") and os.path.exists(table):
        _check(lib.heat_tune_load(os.fsencode(table)))
    return lib


def last_error() -> str:
    return load().heat_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise HeatError(rc, last_error())
    return rc


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _cfg(kernel=0, cells_per_lane=0, steps_per_round=0, waves_per_group=0, register_form=0,
         exchange=0):
    if not (kernel or cells_per_lane or steps_per_round or waves_per_group or register_form
            or exchange):
        return None
    return ctypes.byref(heat_config(kernel, cells_per_lane, steps_per_round, waves_per_group,
                                    register_form, exchange))


def autotune_resident(precision: int, N: int, install: bool = True):
    """Time the resident kernel's shapes at N cells against the round kernel
    the planner runs; returns (best resident config dict, minimum run length
    recorded (0: none), round-kernel time / resident time over 1,024 steps)."""
    cfg = heat_config()
    mn = ctypes.c_int64()
    g = ctypes.c_double()
    _check(load().heat_autotune_resident(int(precision), int(N), int(bool(install)),
                                         ctypes.byref(cfg), ctypes.byref(mn), ctypes.byref(g)))
    return {f: getattr(cfg, f) for f, _ in heat_config._fields_}, mn.value, g.value


def autotune(precision: int, N: int, install: bool = True):
    """Time every launch shape on an N-cell ring; returns (config dict, GCUP/s)."""
    cfg = heat_config()
    g = ctypes.c_double()
    _check(load().heat_autotune(int(precision), int(N), int(bool(install)), ctypes.byref(cfg),
                                ctypes.byref(g)))
    return {f: getattr(cfg, f) for f, _ in heat_config._fields_}, g.value


def autotune_batch(precision: int, N: int, install: bool = True):
    """Time every batch kernel class on a batch of N-cell rings; returns
    ({"cells_per_lane", "waves_per_tile", "steps_per_round"}, GCUP/s)."""
    K, G, T = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    g = ctypes.c_double()
    _check(load().heat_autotune_batch(int(precision), int(N), int(bool(install)),
                                      ctypes.byref(K), ctypes.byref(G), ctypes.byref(T),
                                      ctypes.byref(g)))
    return {"cells_per_lane": K.value, "waves_per_tile": G.value,
            "steps_per_round": T.value}, g.value


def tune_save(path: str) -> None:
    _check(load().heat_tune_save(os.fsencode(path)))


def tune_load(path: str) -> None:
    _check(load().heat_tune_load(os.fsencode(path)))


def version() -> str:
    return load().heat_version().decode()


def device_info() -> dict:
    vals = [ctypes.c_int32() for _ in range(4)] + [ctypes.c_size_t() for _ in range(2)]
    _check(load().heat_device_info(*[ctypes.byref(v) for v in vals]))
    keys = ["cus", "lds_bytes", "wave_size", "clock_khz", "mem_total", "mem_free"]
    return {k: v.value for k, v in zip(keys, vals)}


def plan(N: int, nt: int, precision: int = FP64, **cfg) -> dict:
    out = heat_plan_info()
    _check(load().heat_plan(int(N), int(nt), int(precision), _cfg(**cfg), ctypes.byref(out)))
    return {f: getattr(out, f) for f, _ in heat_plan_info._fields_}


def solve(u: np.ndarray, nparts: int, r: float, nt: int, inplace: bool = False) -> np.ndarray:
    """Plain form on a host binary64 array.  By default the input is copied
    and the result returned; with ``inplace`` a writeable C-contiguous
    float64 array is advanced in place (no host copy) and returned."""
    if inplace:
        if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.flags.c_contiguous
                and u.flags.writeable):
            raise ValueError("inplace needs a writeable C-contiguous float64 numpy array")
        a = u
    else:
        a = np.ascontiguousarray(u, dtype=np.float64).copy()
    _check(load().heat_solve(a.ctypes.data, a.size, int(nparts), float(r), int(nt)))
    return a


def solve_dev(d_u, nparts: int, r: float, nt: int, precision: int | None = None, stream=None,
              sums: bool = False, work=None, **cfg):
    """Device form on a torch tensor (float64 for FP64, float32 for FP32 forms),
    advanced in place.  With ``sums`` returns (sum0, sum_nt) and waits."""
    import torch
    if precision is None:
        precision = FP64 if d_u.dtype == torch.float64 else FP32
    want = torch.float64 if precision == FP64 else torch.float32
    if d_u.dtype != want or not d_u.is_contiguous() or not d_u.is_cuda:
        raise ValueError("d_u must be a contiguous device tensor of the precision's dtype")
    if work is not None and (work.dtype != want or work.numel() < d_u.numel()):
        raise ValueError("work must be a device tensor of the same dtype and size")
    s0, s1 = ctypes.c_double(), ctypes.c_double()
    ps0 = ctypes.byref(s0) if sums else None
    ps1 = ctypes.byref(s1) if sums else None
    _check(load().heat_solve_dev_cfg(d_u.data_ptr(), work.data_ptr() if work is not None else None,
                                     d_u.numel(), int(nparts), float(r), int(nt), int(precision),
                                     _cfg(**cfg), _stream_handle(stream), ps0, ps1))
    return (s0.value, s1.value) if sums else None


def solve_dev_noalloc(d_u, nparts: int, r: float, nt: int, precision: int | None = None,
                      stream=None, sums_out=None) -> None:
    """Device form that allocates nothing (static library scratch): d_u as in
    solve_dev; ``sums_out`` None or a float64 device tensor of at least 2
    elements that receives (sum0, sum_nt) on the stream.  Never waits."""
    import torch
    if precision is None:
        precision = FP64 if d_u.dtype == torch.float64 else FP32
    want = torch.float64 if precision == FP64 else torch.float32
    if d_u.dtype != want or not d_u.is_contiguous() or not d_u.is_cuda:
        raise ValueError("d_u must be a contiguous device tensor of the precision's dtype")
    if sums_out is not None and (sums_out.dtype != torch.float64 or not sums_out.is_cuda
                                 or not sums_out.is_contiguous() or sums_out.numel() < 2):
        raise ValueError("sums_out must be a contiguous float64 device tensor of 2 elements")
    _check(load().heat_solve_dev_noalloc(d_u.data_ptr(), d_u.numel(), int(nparts), float(r),
                                         int(nt), int(precision), _stream_handle(stream),
                                         sums_out.data_ptr() if sums_out is not None else None))


def copy_dev(src, dst, stream=None) -> None:
    """Streaming device-to-device copy (bandwidth probe)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    _check(load().heat_copy_dev(src.data_ptr(), dst.data_ptr(), nbytes, _stream_handle(stream)))


def checksum_dev(d_u, precision: int | None = None, stream=None) -> float:
    import torch
    if precision is None:
        precision = FP64 if d_u.dtype == torch.float64 else FP32
    out = ctypes.c_double()
    _check(load().heat_checksum_dev(d_u.data_ptr(), d_u.numel(), int(precision),
                                    _stream_handle(stream), ctypes.byref(out)))
    return out.value


@dataclass
class BatchResult:
    u: np.ndarray
    sum0: float
    sum_nt: float
    status: int
    latency_s: float = 0.0


def solve_batch(problems) -> list:
    """Batching form on host arrays.  ``problems``: iterable of dicts with
    u0, nparts, r, nt and optional precision and shift (binary32 forms: the
    state is stored as offsets from it).  Returns BatchResult list."""
    probs = list(problems)
    arr = (heat_problem * len(probs))()
    keep = []
    for i, p in enumerate(probs):
        u0 = np.ascontiguousarray(p["u0"], dtype=np.float64)
        out = np.empty_like(u0)
        keep.append((u0, out))
        arr[i] = heat_problem(u0.size, int(p.get("nparts", 1)), int(p.get("precision", FP64)),
                              float(p["r"]), int(p["nt"]), u0.ctypes.data, out.ctypes.data,
                              0.0, 0.0, 0, 0, 0.0, float(p.get("shift", 0.0)))
    rc = load().heat_solve_batch(arr, len(probs))
    res = [BatchResult(keep[i][1], arr[i].sum0, arr[i].sum_nt, arr[i].status)
           for i in range(len(probs))]
    _check(rc)
    return res


def solve_batch_dev(rings, stream=None, wait: bool = True, persistent: bool = False,
                    graph: bool = False):
    """Device batching form.  ``rings``: iterable of (d_u, d_work, nt, r, precision)
    with torch tensors; all rings advance together, one launch per round
    (or one persistent launch with ``persistent``)."""
    rings = list(rings)
    arr = (heat_ring * len(rings))()
    for i, (d_u, d_work, nt, r, prec) in enumerate(rings):
        arr[i] = heat_ring(d_u.numel(), int(nt), float(r), int(prec), 1, d_u.data_ptr(),
                           d_work.data_ptr() if d_work is not None else None)
    flags = (BATCH_WAIT if wait else 0) | (BATCH_PERSISTENT if persistent else 0) | \
        (BATCH_GRAPH if graph else 0)
    _check(load().heat_solve_batch_dev(arr, len(rings), _stream_handle(stream), flags))


class Server:
    """Continuous-batching server (heat_server_*)."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 0, max_queue: int = 0):
        self._h = ctypes.c_void_p()
        _check(load().heat_server_create(int(hbm_budget), int(max_slots), int(max_queue),
                                         ctypes.byref(self._h)))
        self._live = {}

    def submit(self, u0: np.ndarray, nt: int, r: float, precision: int = FP64, nparts: int = 1,
               out: np.ndarray | None = None, shift: float = 0.0) -> int:
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        if out is None:
            out = np.empty_like(u0)
        p = heat_problem(u0.size, int(nparts), int(precision), float(r), int(nt), u0.ctypes.data,
                         out.ctypes.data, 0.0, 0.0, 0, 0, 0.0, float(shift))
        t = ctypes.c_uint64()
        _check(load().heat_submit(self._h, ctypes.byref(p), ctypes.byref(t)))
        self._live[t.value] = (p, u0, out)
        return t.value

    def _result(self, t):
        p, _, out = self._live.pop(t)
        return BatchResult(out, p.sum0, p.sum_nt, p.status, p.latency_s)

    def _settle(self, ticket: int, rc: int):
        # HEAT_ENOENT: unknown, or consumed by a call on another thread, which
        # owns the buffers' entry; any other code means this call consumed it
        if rc != HEAT_ENOENT:
            self._live.pop(ticket, None)
        raise HeatError(rc, last_error())

    def poll(self, ticket: int):
        rc = load().heat_poll(self._h, ctypes.c_uint64(ticket))
        if rc == HEAT_PENDING:
            return None
        if rc < 0:
            self._settle(ticket, rc)
        return self._result(ticket)

    def wait(self, ticket: int):
        rc = load().heat_wait(self._h, ctypes.c_uint64(ticket))
        if rc < 0:
            self._settle(ticket, rc)
        return self._result(ticket)

    def cancel(self, ticket: int) -> None:
        rc = load().heat_cancel(self._h, ctypes.c_uint64(ticket))
        if rc < 0:
            self._settle(ticket, rc)
        self._live.pop(ticket, None)

    def stats(self) -> dict:
        s = heat_server_stats()
        _check(load().heat_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in heat_server_stats._fields_}

    def close(self) -> None:
        if self._h:
            _check(load().heat_server_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
