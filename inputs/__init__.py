"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the generator itself (no skip recurrence, no
modular exponentiation, no floating-point conversion).  It only turns a seed into
workload descriptions: prime pairs, exponents, seeds, start indices and lengths.

Draws come from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), written here from its published definition.
Primality of a 32-bit candidate is decided by trial division with every prime
below 2^16, which is the definition of primality for numbers below 2^32 and
shares nothing with the Miller-Rabin tests used by the oracle and the library.

Recipes (one per workload; the draw order below is part of the definition):

* every workload ``c`` seeds SplitMix64 with ``181111629 + c``;
* a prime draw takes ``u``, forms ``x = 2^31 + (u >> 33)`` and returns the
  smallest prime ``>= x`` that passes the workload's filter; if that prime would
  exceed the largest 32-bit prime 4294967291, a new ``u`` is drawn;
* an instance draws ``p``, then ``q`` (redrawn while ``q == p``), then one more
  ``u`` whose value mod ``n = p*q`` is the message seed ``m_0``; the skip seed is
  ``s_0 = 1``;
* workload-specific draws (exponent, length, start index) follow the instance's
  three draws, in the order documented on each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

MASK64 = (1 << 64) - 1
LARGEST_PRIME_32 = 4294967291
SEED_BASE = 181111629

# Exponent sets of the paper-scale workloads.
SWEEP_EXPONENTS = (3, 5, 17, 257, 65537)
BATCH_EXPONENTS = (3, 5, 7, 17, 257, 65537)


class SplitMix64:
    """SplitMix64: a Weyl sequence with increment 0x9e3779b97f4a7c15 passed through
    a two-multiply finaliser (published constants)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def unit53(self) -> float:
        """A double in [0, 1) from the top 53 bits of one draw."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def _small_primes(limit: int = 1 << 16) -> np.ndarray:
    sieve = np.ones(limit, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    return np.nonzero(sieve)[0].astype(np.float64)


_SMALL = _small_primes()


def is_prime32(x: int) -> bool:
    """Trial division by all primes below 2^16 (exact for 2^16 <= x < 2^32)."""
    if x < 2:
        return False
    if x < (1 << 16):
        return bool(np.any(_SMALL == x))
    xf = float(x)
    # x / p is exact enough that floor() decides divisibility: x < 2^32 and p < 2^16.
    q = np.floor(xf / _SMALL)
    return not bool(np.any(q * _SMALL == xf))


def _is_prime32_many(xs: np.ndarray) -> np.ndarray:
    """Vectorised trial division for an array of candidates in [2^16, 2^32)."""
    xs = xs.astype(np.float64)
    out = np.ones(xs.shape, dtype=bool)
    # cheap pre-filter with the primes below 256, then the full set on survivors
    head = _SMALL[_SMALL < 256]
    q = np.floor(xs[:, None] / head[None, :])
    out &= ~np.any(q * head[None, :] == xs[:, None], axis=1)
    idx = np.nonzero(out)[0]
    tail = _SMALL[_SMALL >= 256]
    for lo in range(0, idx.size, 2048):
        sl = idx[lo:lo + 2048]
        v = xs[sl]
        q = np.floor(v[:, None] / tail[None, :])
        out[sl] &= ~np.any(q * tail[None, :] == v[:, None], axis=1)
    return out


_HERE = os.path.dirname(os.path.abspath(__file__))
_SIEVE_SRC = os.path.join(_HERE, "primes.c")
_SIEVE_LIB = os.path.join(_HERE, "libprimes.so")
_sieve_lock = threading.Lock()
_sieve = None
SIEVE_MIN = 20000   # query counts from which the sieve beats trial division


def build_sieve(force: bool = False) -> str:
    """Compile the segmented-sieve helper (primes.c) with gcc when stale."""
    stale = (not os.path.exists(_SIEVE_LIB) or
             os.path.getmtime(_SIEVE_LIB) < os.path.getmtime(_SIEVE_SRC))
    if force or stale:
        tmp = _SIEVE_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp,
                               _SIEVE_SRC])
        os.replace(tmp, _SIEVE_LIB)
    return _SIEVE_LIB


def _sieve_lib():
    global _sieve
    with _sieve_lock:
        if _sieve is None:
            L = ctypes.CDLL(build_sieve())
            L.next_primes.restype = ctypes.c_int
            L.next_primes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.c_void_p]
            _sieve = L
    return _sieve


def next_primes_sieve(xs, exps: Sequence[int] = ()) -> np.ndarray:
    """Smallest prime >= x with p mod f != 1 for each f in exps, for x in
    [2^31, 2^32), by a segmented sieve (0 where there is none below 2^32)."""
    q = np.ascontiguousarray(xs, dtype=np.uint64)
    if q.size and (int(q.min()) < (1 << 31) or int(q.max()) >= (1 << 32)):
        raise ValueError("sieve queries must lie in [2^31, 2^32)")
    ex = np.ascontiguousarray(list(exps) or [0], dtype=np.uint32)
    out = np.zeros(q.size, dtype=np.uint64)
    rc = _sieve_lib().next_primes(q.ctypes.data, q.size, ex.ctypes.data, len(exps),
                                  out.ctypes.data)
    if rc:
        raise MemoryError("sieve")
    return out.astype(np.int64)


def _next_prime_many(xs: np.ndarray, filt, exps: Optional[Sequence[int]] = None) -> np.ndarray:
    """Smallest prime >= x passing ``filt`` for each x (0 where none <= 4294967291).
    With ``exps`` given (the filter's exponents) and many queries, the segmented
    sieve answers instead of trial division; both give the same exact result."""
    xs = np.asarray(xs, dtype=np.int64)
    if exps is not None and xs.size >= SIEVE_MIN:
        return next_primes_sieve(xs, exps)
    res = np.zeros(xs.shape, dtype=np.int64)
    cand = xs.copy()
    cand[cand % 2 == 0] += 1
    todo = np.arange(xs.size)
    while todo.size:
        c = cand[todo]
        over = c > LARGEST_PRIME_32
        ok = np.zeros(c.shape, dtype=bool)
        live = ~over
        if np.any(live):
            ok[live] = _is_prime32_many(c[live])
            if filt is not None:
                ok[live] &= filt(c[live])
        done = ok | over
        res[todo[ok]] = c[ok]
        cand[todo] += 2
        todo = todo[~done]
    return res


def gcd(a: int, b: int) -> int:
    while b:
        a, b = b, a % b
    return a


@dataclass
class Instance:
    p: int
    q: int
    e: int
    m0: int
    s0: int = 1

    @property
    def n(self) -> int:
        return self.p * self.q


def _filter_mod(exps: Sequence[int]):
    """Filter on p: gcd(f, p-1) == 1 for every listed prime exponent f (p mod f != 1)."""
    def f(c):
        ok = np.ones(c.shape, dtype=bool)
        for ex in exps:
            ok &= (c % ex) != 1
        return ok
    return f


def draw_instances(seed: int, count: int, filt_exps: Sequence[int] = ()) -> List[List[int]]:
    """Draw ``count`` (p, q, m0-draw) triples with SplitMix64(seed).

    Draws are consumed strictly in order: for each instance a p-draw, then
    q-draws, then the m0 draw.  Redraws (p out of range, q == p) consume further
    draws in sequence.  Returns [p, q, u_m0] lists; workloads with more draws per
    instance continue with the same generator via :func:`draw_instances_rng`.
    """
    rng = SplitMix64(seed)
    return draw_instances_rng(rng, count, filt_exps)


def draw_instances_rng(rng: SplitMix64, count: int, filt_exps: Sequence[int] = ()) -> List[list]:
    filt = _filter_mod(filt_exps) if filt_exps else None
    out = []
    # Prime searches are vectorised per instance-batch; the draw sequence is
    # replayed exactly because each instance's draws are consumed in order and
    # the search result only decides whether another draw is needed.
    cache = {}

    def prime_from(u):
        x = (1 << 31) + (u >> 33)
        if x in cache:
            return cache[x]
        r = int(_next_prime_many(np.array([x]), filt)[0])
        cache[x] = r
        return r

    def batch_primes(us):
        xs = np.array([(1 << 31) + (u >> 33) for u in us], dtype=np.int64)
        need = [i for i, x in enumerate(xs) if int(x) not in cache]
        if need:
            ps = _next_prime_many(xs[need], filt, tuple(filt_exps))
            for i, pv in zip(need, ps):
                cache[int(xs[i])] = int(pv)

    # Look-ahead: pre-compute prime searches for a window of future draws so the
    # sequential loop below hits the cache almost always.
    look = SplitMix64(0)
    look.state = rng.state
    batch_primes([look.next() for _ in range(min(4 * count + 64, 1 << 20))])

    for _ in range(count):
        while True:
            p = prime_from(rng.next())
            if p:
                break
        while True:
            q = prime_from(rng.next())
            if q and q != p:
                break
        um = rng.next()
        out.append([p, q, um])
    return out


def smallest_valid_e(p: int, q: int) -> int:
    e = 3
    phi = (p - 1) * (q - 1)
    while gcd(e, phi) != 1:
        e += 2
    return e


def lam(p: int, q: int) -> int:
    return (p - 1) * (q - 1) // gcd(p - 1, q - 1)


# --------------------------------------------------------------------------
# Paper-scale workloads
# --------------------------------------------------------------------------

def config1() -> Instance:
    """Plain single instance: e = smallest odd >= 3 coprime to (p-1)(q-1); 2^20 outputs."""
    (p, q, um), = draw_instances(SEED_BASE + 1, 1)
    return Instance(p, q, smallest_valid_e(p, q), um % (p * q))


def config2(count: int = 1024) -> List[Instance]:
    """Plain multi-instance: e = 3 for every instance (p, q = 2 mod 3)."""
    recs = draw_instances(SEED_BASE + 2, count, (3,))
    return [Instance(p, q, 3, um % (p * q)) for p, q, um in recs]


CONFIG2_SUBSTREAMS = 256
CONFIG2_SUBSTREAM_LEN = 1 << 12


def config3(count: int = 4096) -> List[Instance]:
    """Exponent sweep: primes valid for every e in {3, 5, 17, 257, 65537}; e is set per run."""
    recs = draw_instances(SEED_BASE + 3, count, SWEEP_EXPONENTS)
    return [Instance(p, q, 3, um % (p * q)) for p, q, um in recs]


@dataclass
class BatchRequest:
    inst: int
    k0: int
    count: int


def _draw_batch_e(rng: SplitMix64, p: int, q: int) -> int:
    lm = lam(p, q)
    while True:
        e = BATCH_EXPONENTS[rng.next() % len(BATCH_EXPONENTS)]
        if gcd(e, lm) == 1:
            return e


def config4(count: int = 10000):
    """Batched uneven.  First every instance's (p, q, m0) draws; then, instance by
    instance: e drawn uniformly from the six exponents (redrawn until
    gcd(e, lambda) = 1), the length draw len = floor(2^(8 + 14 u)) with u from the
    top 53 bits, and the start draw k0 = u64 >> 24 in [0, 2^40)."""
    rng = SplitMix64(SEED_BASE + 4)
    recs = draw_instances_rng(rng, count, ())
    insts, reqs = [], []
    for i, (p, q, um) in enumerate(recs):
        e = _draw_batch_e(rng, p, q)
        length = int(2.0 ** (8 + 14 * rng.unit53()))
        k0 = rng.next() >> 24
        insts.append(Instance(p, q, e, um % (p * q)))
        reqs.append(BatchRequest(i, k0, length))
    return insts, reqs


def config5_instances(count: int = 100000):
    """Served pool: every instance's (p, q, m0) draws, then each instance's e draw
    as in the batched workload."""
    rng = SplitMix64(SEED_BASE + 5)
    recs = draw_instances_rng(rng, count, ())
    insts = []
    for p, q, um in recs:
        insts.append(Instance(p, q, _draw_batch_e(rng, p, q), um % (p * q)))
    return insts, rng


def config5_requests(rng: SplitMix64, n_inst: int, n_req: int) -> List[BatchRequest]:
    """Served requests: instance uniform, k0 = u >> 24, count = floor(2^(10 + 14 u))."""
    out = []
    for _ in range(n_req):
        inst = rng.next() % n_inst
        k0 = rng.next() >> 24
        cnt = int(2.0 ** (10 + 14 * rng.unit53()))
        out.append(BatchRequest(inst, k0, cnt))
    return out


def poisson_arrivals(rng: SplitMix64, rate: float, n: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: exponential gaps -ln(1-u)/rate."""
    t = 0.0
    out = np.empty(n)
    for i in range(n):
        t += -np.log1p(-rng.unit53()) / rate
        out[i] = t
    return out


def small_instances(seed: int, count: int, bits: int = 14, e: Optional[int] = None):
    """Tiny-prime instances (primes in [2^(bits-1), 2^bits)) for brute-force checks.

    The prime search uses the same trial division; e is the smallest valid odd
    exponent unless given.
    """
    rng = SplitMix64(seed)
    out = []
    while len(out) < count:
        lo = 1 << (bits - 1)
        p = lo + (rng.next() >> (64 - (bits - 1)))
        while not is_prime32(p):
            p += 1
        q = lo + (rng.next() >> (64 - (bits - 1)))
        while not is_prime32(q):
            q += 1
        if p == q or p >= (1 << bits) or q >= (1 << bits):
            continue
        ee = e if e is not None else smallest_valid_e(p, q)
        if gcd(ee, (p - 1) * (q - 1)) != 1:
            continue
        out.append(Instance(p, q, ee, rng.next() % (p * q)))
    return out


def edge_instances() -> List[Instance]:
    """Moduli at the ends of the range: n just below 2^64 and n just above 2^62."""
    big = [4294967291, 4294967279]          # the two largest 32-bit primes
    small = [2147483659, 2147483693]        # the two smallest primes above 2^31
    out = []
    for p, q in (big, small, (big[0], small[0])):
        n = p * q
        out.append(Instance(p, q, smallest_valid_e(p, q), (n - 12345) % n))
    return out
