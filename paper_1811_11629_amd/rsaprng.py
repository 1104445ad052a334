"""ctypes binding of librsaprng.so (argument marshalling only).

Every function named ``rsaprng_*`` here calls the C function of the same name
declared in include/rsaprng.h.  Device buffers are torch tensors on a ROCm
device (their data_ptr() is passed through); streams are torch.cuda.Stream
objects or raw hipStream_t integers.  Nothing is computed in Python: if the
shared library is missing the import of a function raises, there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Iterable, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RSAPRNG_LIB") or os.path.join(HERE, "librsaprng.so")

BLOCK_LOG2 = 20
Q = 9223372036854775783
A = 2307085864
VECTOR_MAX_MV = 1 << 24          # limits of rsaprng_generate_vector
VECTOR_MAX_COUNT = 1 << 56
VECTOR_MAX_END = 1 << 62

OK = 0
STATUS = {
    0: "RSAPRNG_OK", -1: "RSAPRNG_E_NOT_PRIME", -2: "RSAPRNG_E_EQUAL_PRIMES",
    -3: "RSAPRNG_E_PRIME_RANGE", -4: "RSAPRNG_E_BAD_EXPONENT", -5: "RSAPRNG_E_BAD_SEED",
    -6: "RSAPRNG_E_RANGE", -7: "RSAPRNG_E_NULL", -8: "RSAPRNG_E_ALIGN", -9: "RSAPRNG_E_OOM",
    -10: "RSAPRNG_E_HIP", -11: "RSAPRNG_E_BUSY", -12: "RSAPRNG_E_ARG", -13: "RSAPRNG_E_DEVICE",
    -14: "RSAPRNG_E_NO_DEVICE",
    -15: "RSAPRNG_E_TOO_LARGE",
}
globals().update({name[len("RSAPRNG_"):]: code for code, name in STATUS.items() if code})
VARIANT_AUTO, VARIANT_MONT, VARIANT_CRT = 0, 1, 2
MODE_GENERATE, MODE_CONSUME = 0, 1


class RsaprngError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, STATUS.get(code, "?"), code))


class rsaprng_params(C.Structure):
    _fields_ = [("n", C.c_uint64), ("m0", C.c_uint64), ("s0", C.c_uint64), ("ce", C.c_uint64),
                ("ninv", C.c_uint32), ("e", C.c_uint32), ("p", C.c_uint32), ("q", C.c_uint32),
                ("nd", C.c_double), ("pd", C.c_double), ("qd", C.c_double),
                ("pinv", C.c_double), ("qinv", C.c_double), ("qinvp", C.c_double),
                ("kp", C.c_double), ("kq", C.c_double), ("nrcp", C.c_double),
                ("ep", C.c_uint32), ("eq", C.c_uint32),
                ("kp_lo", C.c_double), ("kp_hi", C.c_double), ("kp_quo", C.c_double),
                ("kq_lo", C.c_double), ("kq_hi", C.c_double), ("kq_quo", C.c_double),
                ("gp_lo", C.c_double), ("gp_hi", C.c_double), ("gp_quo", C.c_double),
                ("nrcp_lo", C.c_double)]


class rsaprng_req(C.Structure):
    _fields_ = [("h", C.c_void_p), ("k0", C.c_uint64), ("count", C.c_uint64),
                ("out_off", C.c_uint64)]


class rsaprng_pool_req(C.Structure):
    _fields_ = [("inst", C.c_uint32), ("reserved", C.c_uint32), ("k0", C.c_uint64),
                ("count", C.c_uint64), ("out_off", C.c_uint64)]


class rsaprng_config(C.Structure):
    _fields_ = [("variant", C.c_int), ("lanes_per_tile", C.c_int), ("per_lane", C.c_int),
                ("persistent", C.c_int), ("wg_per_cu", C.c_int), ("order", C.c_int),
                ("prefix", C.c_int), ("chunks_per_wave", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class rsaprng_server_opts(C.Structure):
    _fields_ = [("arena_bytes", C.c_size_t), ("iter_outputs", C.c_uint64),
                ("chunk_outputs", C.c_uint64), ("max_queue", C.c_size_t),
                ("cfg", rsaprng_config), ("policy", C.c_int)]


SRV_ROUND_ROBIN, SRV_SHORTEST_FIRST = 0, 1


class rsaprng_completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("c", C.c_void_p), ("r", C.c_void_p), ("count", C.c_uint64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


STATS_WORDS = 3 + 1 + 1 + 1 + 6 + 1024   # uint64 words of rsaprng_stats
STATS_BYTES = STATS_WORDS * 8

_lock = threading.Lock()
_lib = None

_u64, _u32, _i32, _dbl, _sz, _vp = C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_size_t, C.c_void_p
BAT_TESTS = ("frequency", "serial2", "serial3", "serial4", "serial5", "serial6", "poker",
             "max_of_32", "collisions", "gaps", "collisions_msb")
BATTERY_BYTES = 16 + 4 * (4 * (1 << 20) + 2 * 1000000 + 8 + 1024 + 256 + 128 + 256)


class rsaprng_battery_result(C.Structure):
    _fields_ = [("chi2", _dbl * len(BAT_TESTS)), ("dof", _dbl * len(BAT_TESTS)),
                ("p", _dbl * len(BAT_TESTS)), ("samples", _u64 * len(BAT_TESTS))]


_SIGS = {
    "rsaprng_params_init": (_i32, [_u64, _u64, _u64, _u64, _u64, C.POINTER(rsaprng_params)]),
    "rsaprng_is_prime": (_i32, [_u64]),
    "rsaprng_skip_at": (_u64, [_u64, _u64]),
    "rsaprng_block_seed": (_u64, [_u64, _u64]),
    "rsaprng_create": (_vp, [_u64, _u64, _u64, _u64]),
    "rsaprng_create_ex": (_vp, [_u64, _u64, _u64, _u64, _u64]),
    "rsaprng_last_error": (_i32, []),
    "rsaprng_strerror": (C.c_char_p, [_i32]),
    "rsaprng_destroy": (None, [_vp]),
    "rsaprng_get_params": (_i32, [_vp, C.POINTER(rsaprng_params)]),
    "rsaprng_generate": (_i32, [_vp, _u64, _u64, _vp, _vp, _vp]),
    "rsaprng_generate_vector": (_i32, [_vp, _u64, _u64, _u64, _vp, _vp, _i32, _vp]),
    "rsaprng_generate_batch": (_i32, [C.POINTER(rsaprng_req), _sz, _vp, _vp, _vp]),
    "rsaprng_consume": (_i32, [_vp, _u64, _u64, _vp, _vp]),
    "rsaprng_pool_create": (_vp, [_sz, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64),
                                  C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_sz)]),
    "rsaprng_pool_create_dual": (_vp, [_sz] + [_vp] * 6 + [C.POINTER(_sz)]),
    "rsaprng_dual_exponent": (_i32, [_u64, _u64, _u64, _u64, C.POINTER(_u64)]),
    "rsaprng_params_init_dual": (_i32, [_u64] * 6 + [C.POINTER(rsaprng_params)]),
    "rsaprng_pool_destroy": (None, [_vp]),
    "rsaprng_pool_size": (_sz, [_vp]),
    "rsaprng_pool_generate": (_i32, [_vp, C.POINTER(rsaprng_pool_req), _sz, _vp, _vp,
                                     C.POINTER(rsaprng_config), _vp]),
    "rsaprng_pool_generate_noalloc": (_i32, [_vp, C.POINTER(rsaprng_pool_req), _sz, _vp, _vp,
                                             C.POINTER(rsaprng_config), _vp]),
    "rsaprng_pool_consume": (_i32, [_vp, C.POINTER(rsaprng_pool_req), _sz, _vp,
                                    C.POINTER(rsaprng_config), _vp]),
    "rsaprng_batch_create": (_i32, [_vp, C.POINTER(rsaprng_pool_req), _sz, _i32, _vp, _vp, _vp,
                                    C.POINTER(rsaprng_config), _vp, C.POINTER(_vp)]),
    "rsaprng_batch_run": (_i32, [_vp, _vp]),
    "rsaprng_batch_check": (_i32, [_vp]),
    "rsaprng_batch_run_timed": (_i32, [_vp, _vp]),
    "rsaprng_batch_kernel_ms": (_i32, [_vp, C.POINTER(_dbl), C.POINTER(_i32)]),
    "rsaprng_batch_destroy": (None, [_vp]),
    "rsaprng_autotune": (_i32, [_vp, C.POINTER(rsaprng_pool_req), _sz, _i32, _vp, _vp, _vp,
                                C.c_char_p, _vp, C.POINTER(rsaprng_config), C.POINTER(_dbl)]),
    "rsaprng_server_create": (_i32, [_vp, C.POINTER(rsaprng_server_opts), C.POINTER(_vp)]),
    "rsaprng_server_submit": (_i32, [_vp, _u32, _u64, _u64, _u64]),
    "rsaprng_server_poll": (_i32, [_vp, C.POINTER(rsaprng_completion), _sz]),
    "rsaprng_pool_battery": (_i32, [_vp, C.POINTER(rsaprng_pool_req), _sz, _vp,
                                     C.POINTER(rsaprng_config), _vp]),
    "rsaprng_battery_report": (_i32, [_vp, C.POINTER(rsaprng_battery_result)]),
    "rsaprng_battery_values": (_i32, [_vp, _u64, _vp, _vp]),
    "rsaprng_chi2_sf": (_dbl, [_dbl, _dbl]),
    "rsaprng_prime_count": (_i32, [_u64, _u64, _i32, C.POINTER(_u64), _vp]),
    "rsaprng_next_primes": (_i32, [_vp, _u64, _i32, _vp, _i32, _vp, _vp]),
    "rsaprng_server_read": (_i32, [_vp, _u64, _u64, _u64, _vp, _vp, _vp]),
    "rsaprng_server_release": (_i32, [_vp, _u64]),
    "rsaprng_server_replay": (_i32, [_vp, _sz, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rsaprng_server_simulate": (C.c_int64, [C.POINTER(rsaprng_config), _u64, _u64, _u64, _i32,
                                            _sz, _vp, _vp, _vp, _u64, _vp, _sz]),
    "rsaprng_server_now": (_dbl, [_vp]),
    "rsaprng_server_stats": (_i32, [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64),
                                    C.POINTER(_u64)]),
    "rsaprng_server_destroy": (None, [_vp]),
    "rsaprng_check_device_error": (_i32, [_vp]),
    "rsaprng_debug_encrypt": (_i32, [_u64, _u64, _u64, _i32, _vp, _vp, _vp, _u64, _vp]),
    "rsaprng_version": (C.c_char_p, []),
    "rsaprng_probe": (_i32, [_i32, _u64, _vp, _vp, C.POINTER(_dbl), _vp]),
}


def lib():
    """Load librsaprng.so; raises if it has not been built (no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("librsaprng.so not built: run __graft_entry__.build() "
                                  "or python paper_1811_11629_amd/build.py")
            # torch ships its own HIP runtime; load it first so that the library
            # binds to the same one (the process can then use both)
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise RsaprngError(rc, what)


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None / an int passed through)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s) -> Optional[int]:
    if s is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:
            return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _u64arr(vals: Sequence[int]):
    arr = (C.c_uint64 * len(vals))(*[int(v) for v in vals])
    return arr


def config(variant=0, lanes_per_tile=0, per_lane=0, persistent=0, wg_per_cu=0, order=0, prefix=0,
           chunks_per_wave=0):
    return rsaprng_config(variant, lanes_per_tile, per_lane, persistent, wg_per_cu, order, prefix,
                          chunks_per_wave)


# --------------------------------------------------------------------------
# functions with the C names
# --------------------------------------------------------------------------

def rsaprng_params_init(p, q, e, m0, s0=1) -> rsaprng_params:
    out = rsaprng_params()
    _check(lib().rsaprng_params_init(p, q, e, m0, s0, C.byref(out)), "rsaprng_params_init")
    return out


def rsaprng_is_prime(n: int) -> bool:
    return bool(lib().rsaprng_is_prime(n))


def rsaprng_skip_at(s0: int, k: int) -> int:
    return lib().rsaprng_skip_at(s0, k)


def rsaprng_block_seed(s0: int, b: int) -> int:
    return lib().rsaprng_block_seed(s0, b)


def rsaprng_strerror(code: int) -> str:
    return lib().rsaprng_strerror(code).decode()


def rsaprng_version() -> str:
    return lib().rsaprng_version().decode()


class Generator:
    """An rsaprng_t handle (one instance)."""

    def __init__(self, handle: int):
        self.h = handle

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rsaprng_destroy(self.h)
            self.h = None

    @property
    def params(self) -> rsaprng_params:
        out = rsaprng_params()
        _check(lib().rsaprng_get_params(self.h, C.byref(out)), "rsaprng_get_params")
        return out


def rsaprng_create(p, q, e, seed) -> Generator:
    h = lib().rsaprng_create(p, q, e, seed)
    if not h:
        raise RsaprngError(lib().rsaprng_last_error(), "rsaprng_create")
    return Generator(h)


def rsaprng_create_ex(p, q, e, m0, s0=1) -> Generator:
    h = lib().rsaprng_create_ex(p, q, e, m0, s0)
    if not h:
        raise RsaprngError(lib().rsaprng_last_error(), "rsaprng_create_ex")
    return Generator(h)


def rsaprng_generate(gen: Generator, k0: int, count: int, out_u64=None, out_f64=None,
                     stream=None) -> None:
    _check(lib().rsaprng_generate(gen.h, k0, count, _ptr(out_u64), _ptr(out_f64), _stream(stream)),
           "rsaprng_generate")


def rsaprng_generate_vector(gen: Generator, mv: int, f0: int, count: int, out_u64=None,
                            out_f64=None, variant: int = 0, stream=None) -> None:
    """Vector mode: outputs f0 .. f0 + count - 1 of mv substreams, f = (t - 1) mv + g."""
    _check(lib().rsaprng_generate_vector(gen.h, mv, f0, count, _ptr(out_u64), _ptr(out_f64),
                                         variant, _stream(stream)), "rsaprng_generate_vector")


def rsaprng_generate_batch(reqs: Sequence, out_u64=None, out_f64=None, stream=None) -> None:
    """reqs: sequence of (Generator, k0, count, out_off)."""
    arr = (rsaprng_req * len(reqs))(*[rsaprng_req(g.h, k0, cnt, off) for g, k0, cnt, off in reqs])
    _check(lib().rsaprng_generate_batch(arr, len(reqs), _ptr(out_u64), _ptr(out_f64),
                                        _stream(stream)), "rsaprng_generate_batch")


def rsaprng_consume(gen: Generator, k0: int, count: int, stats, stream=None) -> None:
    _check(lib().rsaprng_consume(gen.h, k0, count, _ptr(stats), _stream(stream)), "rsaprng_consume")


def rsaprng_check_device_error(stream=None) -> None:
    _check(lib().rsaprng_check_device_error(_stream(stream)), "rsaprng_check_device_error")


def rsaprng_debug_encrypt(p, q, e, variant, m, c=None, r=None, stream=None) -> None:
    _check(lib().rsaprng_debug_encrypt(p, q, e, variant, _ptr(m), _ptr(c), _ptr(r), m.numel(),
                                       _stream(stream)), "rsaprng_debug_encrypt")


class Pool:
    """An rsaprng_pool_t: a device-resident table of instances."""

    def __init__(self, p: Sequence[int], q: Sequence[int], e: Sequence[int], seed: Sequence[int],
                 s0: Optional[Sequence[int]] = None):
        n = len(p)
        err = C.c_size_t(0)
        h = lib().rsaprng_pool_create(n, _u64arr(p), _u64arr(q), _u64arr(e), _u64arr(seed),
                                      _u64arr(s0) if s0 is not None else None, C.byref(err))
        if not h:
            raise RsaprngError(lib().rsaprng_last_error(), "rsaprng_pool_create[%d]" % err.value)
        self.h = h
        self.size = n

    @classmethod
    def dual(cls, p, q, ep, eq, seed, s0=None) -> "Pool":
        """A pool of instances with exponents ep mod p and eq mod q."""
        self = cls.__new__(cls)
        n = len(p)
        err = C.c_size_t(0)
        h = lib().rsaprng_pool_create_dual(n, _u64arr(p), _u64arr(q), _u64arr(ep), _u64arr(eq),
                                           _u64arr(seed), _u64arr(s0) if s0 is not None else None,
                                           C.byref(err))
        if not h:
            raise RsaprngError(lib().rsaprng_last_error(),
                               "rsaprng_pool_create_dual[%d]" % err.value)
        self.h = h
        self.size = n
        return self

    @classmethod
    def from_instances(cls, insts) -> "Pool":
        return cls([i.p for i in insts], [i.q for i in insts], [i.e for i in insts],
                   [i.m0 for i in insts], [i.s0 for i in insts])

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rsaprng_pool_destroy(self.h)
            self.h = None


def pool_reqs(reqs: Iterable) -> "C.Array":
    """(inst, k0, count, out_off) tuples -> rsaprng_pool_req array."""
    reqs = list(reqs)
    return (rsaprng_pool_req * len(reqs))(*[rsaprng_pool_req(i, 0, k0, c, o) for i, k0, c, o in reqs])


def rsaprng_pool_generate(pool: Pool, reqs, out_u64=None, out_f64=None, cfg=None, stream=None):
    arr = reqs if isinstance(reqs, C.Array) else pool_reqs(reqs)
    _check(lib().rsaprng_pool_generate(pool.h, arr, len(arr), _ptr(out_u64), _ptr(out_f64),
                                       C.byref(cfg) if cfg is not None else None, _stream(stream)),
           "rsaprng_pool_generate")


def rsaprng_pool_generate_noalloc(pool: Pool, reqs, out_u64=None, out_f64=None, cfg=None,
                                  stream=None):
    arr = reqs if isinstance(reqs, C.Array) else pool_reqs(reqs)
    _check(lib().rsaprng_pool_generate_noalloc(pool.h, arr, len(arr), _ptr(out_u64),
                                               _ptr(out_f64),
                                               C.byref(cfg) if cfg is not None else None,
                                               _stream(stream)),
           "rsaprng_pool_generate_noalloc")


def rsaprng_pool_consume(pool: Pool, reqs, stats, cfg=None, stream=None):
    arr = reqs if isinstance(reqs, C.Array) else pool_reqs(reqs)
    _check(lib().rsaprng_pool_consume(pool.h, arr, len(arr), _ptr(stats),
                                      C.byref(cfg) if cfg is not None else None, _stream(stream)),
           "rsaprng_pool_consume")


class Batch:
    """An rsaprng_batch_t: a prepared, graph-captured launch."""

    def __init__(self, pool: Pool, reqs, mode=MODE_GENERATE, out_u64=None, out_f64=None,
                 stats=None, cfg=None, stream=None):
        arr = reqs if isinstance(reqs, C.Array) else pool_reqs(reqs)
        h = C.c_void_p()
        _check(lib().rsaprng_batch_create(pool.h, arr, len(arr), mode, _ptr(out_u64), _ptr(out_f64),
                                          _ptr(stats), C.byref(cfg) if cfg is not None else None,
                                          _stream(stream), C.byref(h)), "rsaprng_batch_create")
        self.h = h.value
        self.pool = pool          # keep the pool alive
        self._keep = (out_u64, out_f64, stats)

    def run(self, stream=None):
        _check(lib().rsaprng_batch_run(self.h, _stream(stream)), "rsaprng_batch_run")

    def check(self):
        _check(lib().rsaprng_batch_check(self.h), "rsaprng_batch_check")

    def run_timed(self, stream=None):
        """Enqueue the launch without the graph, with events between its kernels."""
        _check(lib().rsaprng_batch_run_timed(self.h, _stream(stream)), "rsaprng_batch_run_timed")

    def kernel_ms(self):
        """Average per-kernel ms of the timed runs since the last call:
        {setup, prefix, tiles, finalize, runs}."""
        ms = (_dbl * 4)()
        runs = _i32(0)
        _check(lib().rsaprng_batch_kernel_ms(self.h, ms, C.byref(runs)), "rsaprng_batch_kernel_ms")
        return {"setup": ms[0], "prefix": ms[1], "tiles": ms[2], "finalize": ms[3],
                "runs": runs.value}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rsaprng_batch_destroy(self.h)
            self.h = None


def rsaprng_autotune(pool: Pool, reqs, mode=MODE_GENERATE, out_u64=None, out_f64=None, stats=None,
                     cache_path: Optional[str] = None, stream=None):
    arr = reqs if isinstance(reqs, C.Array) else pool_reqs(reqs)
    best = rsaprng_config()
    ms = C.c_double(0)
    _check(lib().rsaprng_autotune(pool.h, arr, len(arr), mode, _ptr(out_u64), _ptr(out_f64),
                                  _ptr(stats), cache_path.encode() if cache_path else None,
                                  _stream(stream), C.byref(best), C.byref(ms)), "rsaprng_autotune")
    return best, ms.value


def stats_tensor(n: int, device="cuda"):
    import torch
    return torch.zeros((n, STATS_WORDS), dtype=torch.int64, device=device)


def stats_decode(t) -> List[dict]:
    """Host copy of rsaprng_stats records -> dicts (sum_fx as a Python int)."""
    import numpy as np
    a = t.detach().cpu().numpy().view(np.uint64).reshape(-1, STATS_WORDS)
    out = []
    for row in a:
        fx = int(row[0]) | (int(row[1]) << 64) | (int(row[2]) << 128)
        out.append({"sum_fx": fx, "lt_half": int(row[3]), "count": int(row[4]),
                    "sum": float(row[5:6].view(np.float64)[0]),
                    "hist": row[12:12 + 1024].copy()})
    return out


def server_simulate(k0, count, arrive_iter, arena_elems, iter_outputs=0, chunk_outputs=0,
                    hold_iters=0, cfg=None, policy=SRV_ROUND_ROBIN):
    """Host-only dry run of the server's scheduler; returns an (nchunks, 7) uint64
    array: request, iteration, first index, count, arena offset, flags, slot."""
    import numpy as np
    k0 = np.ascontiguousarray(k0, dtype=np.uint64)
    count = np.ascontiguousarray(count, dtype=np.uint64)
    arrive_iter = np.ascontiguousarray(arrive_iter, dtype=np.uint64)
    c = cfg if cfg is not None else rsaprng_config()
    n = len(k0)
    nch = lib().rsaprng_server_simulate(C.byref(c), arena_elems, iter_outputs, chunk_outputs,
                                        policy, n, k0.ctypes.data, count.ctypes.data,
                                        arrive_iter.ctypes.data, hold_iters, None, 0)
    if nch < 0:
        raise RsaprngError(int(nch), "rsaprng_server_simulate")
    log = np.zeros((max(nch, 1), 7), dtype=np.uint64)
    nch2 = lib().rsaprng_server_simulate(C.byref(c), arena_elems, iter_outputs, chunk_outputs,
                                         policy, n, k0.ctypes.data, count.ctypes.data,
                                         arrive_iter.ctypes.data, hold_iters, log.ctypes.data,
                                         nch)
    assert nch2 == nch
    return log[:nch]


def battery_tensor(device="cuda"):
    """A device buffer holding one rsaprng_battery record."""
    import torch
    return torch.empty(BATTERY_BYTES, dtype=torch.uint8, device=device)


def rsaprng_pool_battery(pool: "Pool", reqs, rec, cfg=None, stream=None) -> None:
    arr = reqs if isinstance(reqs, C.Array) else pool_reqs(reqs)
    _check(lib().rsaprng_pool_battery(pool.h, arr, len(arr), _ptr(rec),
                                      C.byref(cfg) if cfg is not None else None, _stream(stream)),
           "rsaprng_pool_battery")


def rsaprng_battery_values(r, rec, count=None, stream=None) -> None:
    """The battery over a device array of values (r[j] at index j)."""
    n = r.numel() if count is None else count
    _check(lib().rsaprng_battery_values(_ptr(r), n, _ptr(rec), _stream(stream)),
           "rsaprng_battery_values")


def battery_report(rec) -> dict:
    """Chi-squared, dof, p-value and sample count per test from a battery record
    (device tensor or host bytes)."""
    import numpy as np
    if hasattr(rec, "cpu"):
        import torch
        torch.cuda.synchronize()
        host = rec.cpu().numpy().tobytes()
    else:
        host = bytes(rec)
    buf = np.frombuffer(host, dtype=np.uint8).copy()
    out = rsaprng_battery_result()
    _check(lib().rsaprng_battery_report(buf.ctypes.data, C.byref(out)), "rsaprng_battery_report")
    return {name: {"chi2": out.chi2[i], "dof": out.dof[i], "p": out.p[i],
                   "samples": out.samples[i]} for i, name in enumerate(BAT_TESTS)}


def rsaprng_chi2_sf(chi2: float, dof: float) -> float:
    return lib().rsaprng_chi2_sf(chi2, dof)


def rsaprng_params_init_dual(p, q, ep, eq, m0, s0=1) -> rsaprng_params:
    out = rsaprng_params()
    _check(lib().rsaprng_params_init_dual(p, q, ep, eq, m0, s0, C.byref(out)),
           "rsaprng_params_init_dual")
    return out


def rsaprng_dual_exponent(p: int, q: int, ep: int, eq: int) -> int:
    out = C.c_uint64(0)
    _check(lib().rsaprng_dual_exponent(p, q, ep, eq, C.byref(out)), "rsaprng_dual_exponent")
    return out.value


def rsaprng_prime_count(lo: int, hi: int, safe: bool = False, stream=None) -> int:
    """Number of primes (safe primes) in [lo, hi), hi <= 2^32, counted on the device."""
    out = C.c_uint64(0)
    _check(lib().rsaprng_prime_count(lo, hi, 1 if safe else 0, C.byref(out), _stream(stream)),
           "rsaprng_prime_count")
    return out.value


def rsaprng_next_primes(x, out, safe: bool = False, exps=(), stream=None) -> None:
    """out[i] = smallest qualifying prime >= x[i] (device tensors of int64), or 0."""
    n = len(x)
    arr = (C.c_uint32 * max(1, len(exps)))(*exps)
    _check(lib().rsaprng_next_primes(_ptr(x), n, 1 if safe else 0, arr, len(exps), _ptr(out),
                                     _stream(stream)), "rsaprng_next_primes")


# Limits of rsaprng_pool_generate_noalloc (its fixed scratch).
NOALLOC_SCRATCH_BYTES = 32 << 20
NOALLOC_MAX_CHAINS = 16384

PROBES = {"v_fma_f64": 0, "v_mul_f64": 1, "v_add_f64": 2, "v_rndne_f64": 3,
          "v_mad_u64_u32": 4, "v_mul_lo_u32": 5, "v_mul_hi_u32": 6, "v_add_u32": 7,
          "v_cvt_f64_u32": 8, "v_lshl_add_u64": 9, "v_mul_u32_u24": 10}
PROBE_STORE_TILE, PROBE_STORE_LINEAR = 16, 17
PROBE_STORE_TILE_PLAIN, PROBE_STORE_BLOCK16, PROBE_STORE_BLOCK16_PLAIN = 18, 19, 20


def rsaprng_probe(kind: int, n: int, out_u64=None, out_f64=None, stream=None) -> float:
    """Enqueue one throughput probe; returns the work it does (lane-instructions
    of the probed class, or bytes written)."""
    work = C.c_double(0)
    _check(lib().rsaprng_probe(kind, n, _ptr(out_u64), _ptr(out_f64), C.byref(work),
                               _stream(stream)), "rsaprng_probe")
    return work.value


class Server:
    """An rsaprng_server_t (continuous batching over a pool)."""

    def __init__(self, pool: Pool, arena_bytes: int, iter_outputs=0, chunk_outputs=0, max_queue=0,
                 cfg=None, policy=SRV_ROUND_ROBIN):
        opts = rsaprng_server_opts(arena_bytes, iter_outputs, chunk_outputs, max_queue,
                                   cfg if cfg is not None else rsaprng_config(), policy)
        h = C.c_void_p()
        _check(lib().rsaprng_server_create(pool.h, C.byref(opts), C.byref(h)),
               "rsaprng_server_create")
        self.h = h.value
        self.pool = pool

    def submit(self, inst: int, k0: int, count: int, tag: int) -> int:
        return lib().rsaprng_server_submit(self.h, inst, k0, count, tag)

    def poll(self, max_n: int = 1024) -> List[rsaprng_completion]:
        buf = (rsaprng_completion * max_n)()
        n = lib().rsaprng_server_poll(self.h, buf, max_n)
        if n < 0:
            raise RsaprngError(n, "rsaprng_server_poll")
        return [buf[i] for i in range(n)]

    def read(self, tag: int, out_u64=None, out_f64=None, offset: int = 0, count=None,
             stream=None) -> None:
        """Copy a completed request's outputs into out_u64 / out_f64 (torch tensors
        or numpy arrays, host or device)."""
        def addr(x):
            if x is None:
                return None
            if hasattr(x, "data_ptr"):
                return x.data_ptr()
            return x.ctypes.data
        if count is None:
            count = len(out_u64 if out_u64 is not None else out_f64)
        _check(lib().rsaprng_server_read(self.h, tag, offset, count, addr(out_u64),
                                         addr(out_f64), _stream(stream)),
               "rsaprng_server_read")

    def release(self, tag: int) -> None:
        _check(lib().rsaprng_server_release(self.h, tag), "rsaprng_server_release")

    def replay(self, inst, k0, count, t_arrival):
        """Open-loop replay of a request trace (numpy arrays); returns (t_admit, t_done)
        in seconds from the start of the replay."""
        import numpy as np
        inst = np.ascontiguousarray(inst, dtype=np.uint32)
        k0 = np.ascontiguousarray(k0, dtype=np.uint64)
        count = np.ascontiguousarray(count, dtype=np.uint64)
        t_arrival = np.ascontiguousarray(t_arrival, dtype=np.float64)
        n = len(inst)
        t_admit = np.zeros(n)
        t_done = np.zeros(n)
        _check(lib().rsaprng_server_replay(self.h, n, inst.ctypes.data, k0.ctypes.data,
                                           count.ctypes.data, t_arrival.ctypes.data,
                                           t_admit.ctypes.data, t_done.ctypes.data),
               "rsaprng_server_replay")
        return t_admit, t_done

    def now(self) -> float:
        return lib().rsaprng_server_now(self.h)

    def stats(self):
        it, outs, w, a = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().rsaprng_server_stats(self.h, C.byref(it), C.byref(outs), C.byref(w),
                                          C.byref(a)), "rsaprng_server_stats")
        return {"iterations": it.value, "outputs": outs.value, "waiting": w.value,
                "active": a.value}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rsaprng_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
