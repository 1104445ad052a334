"""ctypes wrapper of the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  The shared library
is compiled with gcc on first use (or by the repository's build step).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

Q = 9223372036854775783
A = 2307085864
BLOCK_LOG2 = 20
BLOCK = 1 << BLOCK_LOG2

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (always when force, else only if stale)."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Stats(C.Structure):
    _fields_ = [("sum_fx", C.c_uint64 * 3), ("lt_half", C.c_uint64), ("hist", C.c_uint64 * 1024)]

    def as_dict(self):
        fx = self.sum_fx[0] | (self.sum_fx[1] << 64) | (self.sum_fx[2] << 128)
        return {"sum_fx": fx, "lt_half": int(self.lt_half),
                "hist": np.ctypeslib.as_array(self.hist).astype(np.uint64).copy()}


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            u64, i32, dbl = C.c_uint64, C.c_int, C.c_double
            P64 = C.POINTER(C.c_uint64)
            PD = C.POINTER(C.c_double)
            sig = {
                "oracle_mulmod": (u64, [u64, u64, u64]),
                "oracle_powmod": (u64, [u64, u64, u64]),
                "oracle_gcd": (u64, [u64, u64]),
                "oracle_inverse": (u64, [u64, u64]),
                "oracle_is_prime": (i32, [u64]),
                "oracle_check_params": (i32, [u64, u64, u64]),
                "oracle_decryption_exponent": (u64, [u64, u64, u64, i32]),
                "oracle_lcg_next": (u64, [u64]),
                "oracle_lcg_next_schrage": (u64, [u64]),
                "oracle_skip": (u64, [u64, u64]),
                "oracle_block_seed": (u64, [u64, u64]),
                "oracle_block_seed_walk": (u64, [u64, u64]),
                "oracle_ratio": (dbl, [u64, u64]),
                "oracle_generate": (i32, [u64] * 7 + [P64, PD]),
                "oracle_messages": (i32, [u64] * 6 + [P64]),
                "oracle_paper_algorithm1": (i32, [u64] * 6 + [P64, PD]),
                "oracle_encrypt_array": (None, [u64, u64, P64, P64, u64]),
                "oracle_consume": (i32, [u64] * 7 + [C.POINTER(Stats)]),
                "oracle_stats_of": (None, [PD, u64, C.POINTER(Stats)]),
                "oracle_count_primes": (u64, [u64, u64, i32]),
                "oracle_battery_add": (i32, [u64] * 7 + [C.c_void_p]),
                "oracle_battery_values": (i32, [PD, u64, u64, C.c_void_p]),
                "oracle_next_prime": (u64, [u64, i32, C.c_void_p, i32]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _p64(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64)) if a is not None else None


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class OracleError(RuntimeError):
    pass


def mulmod(x, y, m): return lib().oracle_mulmod(x, y, m)
def powmod(x, e, m): return lib().oracle_powmod(x, e, m)
def gcd(x, y): return lib().oracle_gcd(x, y)
def inverse(x, m): return lib().oracle_inverse(x, m)
def is_prime(n): return bool(lib().oracle_is_prime(n))
def check_params(p, q, e): return lib().oracle_check_params(p, q, e)
def decryption_exponent(p, q, e, use_lambda=True): return lib().oracle_decryption_exponent(p, q, e, int(use_lambda))
def lcg_next(s): return lib().oracle_lcg_next(s)
def lcg_next_schrage(s): return lib().oracle_lcg_next_schrage(s)
def skip(s0, k): return lib().oracle_skip(s0, k)
def block_seed(s0, b): return lib().oracle_block_seed(s0, b)
def block_seed_walk(s0, b): return lib().oracle_block_seed_walk(s0, b)
def ratio(c, n): return lib().oracle_ratio(c, n)


def generate(p, q, e, m0, s0, k0, count, want_c=True, want_r=True):
    c = np.empty(count, dtype=np.uint64) if want_c else None
    r = np.empty(count, dtype=np.float64) if want_r else None
    rc = lib().oracle_generate(p, q, e, m0, s0, k0, count, _p64(c), _pd(r))
    if rc:
        raise OracleError("oracle_generate rc=%d" % rc)
    return c, r


def substream_seed(s0, mv, g):
    """Skip seed of substream g of mv (Parallelization section, stream splitting):
    s0 a^(g floor((Q-1)/mv)) mod Q."""
    return mulmod(s0, powmod(A, g * ((Q - 1) // mv), Q), Q)


def generate_vector(p, q, e, m0, s0, mv, f0, count, want_c=True, want_r=True):
    """Vector mode (Parallelization section, eq. vectorize): mv substreams advanced
    together, substream g being the sequence with skip seed substream_seed(s0, mv, g)
    and message seed m0.  The t-th vector call (t >= 1) returns substream g's output
    after t updates, i.e. its index t; flattened, f = (t - 1) mv + g.  Returns
    outputs f0 .. f0 + count - 1."""
    c = np.empty(count, dtype=np.uint64) if want_c else None
    r = np.empty(count, dtype=np.float64) if want_r else None
    if count == 0:
        return c, r
    t_lo, g_lo = f0 // mv + 1, f0 % mv
    t_hi, g_hi = (f0 + count - 1) // mv + 1, (f0 + count - 1) % mv
    for j in range(min(count, mv)):
        g = (g_lo + j) % mv
        first = t_lo if g >= g_lo else t_lo + 1
        last = t_hi if g <= g_hi else t_hi - 1
        if first > last:
            continue
        n = last - first + 1
        cg, rg = generate(p, q, e, m0, substream_seed(s0, mv, g), first, n, want_c, want_r)
        start = (first - 1) * mv + g - f0
        if want_c:
            c[start:start + (n - 1) * mv + 1:mv] = cg
        if want_r:
            r[start:start + (n - 1) * mv + 1:mv] = rg
    return c, r


def messages(p, q, m0, s0, k0, count):
    m = np.empty(count, dtype=np.uint64)
    rc = lib().oracle_messages(p, q, m0, s0, k0, count, _p64(m))
    if rc:
        raise OracleError("oracle_messages rc=%d" % rc)
    return m


def paper_algorithm1(p, q, e, m0, s0, count):
    c = np.empty(count, dtype=np.uint64)
    r = np.empty(count, dtype=np.float64)
    rc = lib().oracle_paper_algorithm1(p, q, e, m0, s0, count, _p64(c), _pd(r))
    if rc:
        raise OracleError("oracle_paper_algorithm1 rc=%d" % rc)
    return c, r


def encrypt_array(n, e, m):
    m = np.ascontiguousarray(m, dtype=np.uint64)
    c = np.empty_like(m)
    lib().oracle_encrypt_array(n, e, _p64(m), _p64(c), m.size)
    return c


def consume(p, q, e, m0, s0, k0, count):
    st = Stats()
    rc = lib().oracle_consume(p, q, e, m0, s0, k0, count, C.byref(st))
    if rc:
        raise OracleError("oracle_consume rc=%d" % rc)
    return st.as_dict()


def stats_of(r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    st = Stats()
    lib().oracle_stats_of(_pd(r), r.size, C.byref(st))
    return st.as_dict()


def generate_instance(inst, k0, count, want_c=True, want_r=True):
    """Convenience: an object with p, q, e, m0, s0 attributes."""
    return generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count, want_c, want_r)


def count_primes(lo, hi, safe=False):
    """Primes (or safe primes) in [lo, hi), hi <= 2^32, by a segmented sieve."""
    return lib().oracle_count_primes(lo, hi, 1 if safe else 0)


def next_prime(x, safe=False, exps=()):
    """Smallest p >= x below 2^32, prime (safe if asked), p mod f != 1 for f in exps; 0 if none."""
    arr = (C.c_uint32 * max(1, len(exps)))(*exps)
    return lib().oracle_next_prime(x, 1 if safe else 0, arr, len(exps))


BATTERY_FIELDS = [("outputs", 1, np.uint64), ("reserved", 1, np.uint64),
                  ("freq", 1 << 20, np.uint32), ("serial2", 1 << 20, np.uint32),
                  ("serial3", 1000000, np.uint32), ("serial4", 1 << 20, np.uint32),
                  ("serial5", 1 << 20, np.uint32), ("serial6", 1000000, np.uint32),
                  ("poker", 8, np.uint32), ("maxt", 1024, np.uint32),
                  ("coll", 256, np.uint32), ("runs", 128, np.uint32),
                  ("coll_msb", 256, np.uint32)]
BATTERY_BYTES = sum(n * np.dtype(t).itemsize for _, n, t in BATTERY_FIELDS)


def battery_decode(buf):
    """bytes of a battery record -> dict of numpy arrays (shared layout with C)."""
    out, off = {}, 0
    raw = np.frombuffer(buf, dtype=np.uint8)
    for name, n, t in BATTERY_FIELDS:
        size = n * np.dtype(t).itemsize
        out[name] = raw[off:off + size].view(t).copy()
        off += size
    return out


def battery_values(r, k0=0):
    """Battery counts of the given values, standing at indices k0 .. k0 + len(r) - 1."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    buf = np.zeros(BATTERY_BYTES, dtype=np.uint8)
    rc = lib().oracle_battery_values(_pd(r), k0, r.size, buf.ctypes.data)
    if rc:
        raise ValueError("oracle_battery_values: %d" % rc)
    return battery_decode(buf.tobytes())


def battery(ranges):
    """Battery counts over [(instance, k0, count), ...], accumulated into one record."""
    buf = np.zeros(BATTERY_BYTES, dtype=np.uint8)
    for inst, k0, count in ranges:
        rc = lib().oracle_battery_add(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count,
                                      buf.ctypes.data)
        if rc:
            raise ValueError("oracle_battery_add: %d" % rc)
    return battery_decode(buf.tobytes())
