"""Parameter generation on the host side: the oracle's prime counts equal the
counts the paper prints, the library's 32-bit primality code (compiled for the
host from the same header the kernels use) equals the oracle, and the oracle's
next-prime search equals the workload generator's independent trial division."""
import ctypes as C
import json
import os
import random
import subprocess

import numpy as np
import pytest

import inputs
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_prime_counts.json")))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("ph") / "libprimes_harness.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                           "-I" + os.path.join(ROOT, "paper_1811_11629_amd", "csrc"), "-o", out,
                           os.path.join(ROOT, "tests", "native", "primes_harness.cpp")])
    L = C.CDLL(out)
    L.harness_count.restype = C.c_uint64
    L.harness_count.argtypes = [C.c_uint64, C.c_uint64, C.c_int]
    L.harness_is_prime.restype = C.c_int
    L.harness_is_prime.argtypes = [C.c_uint32]
    return L


def test_oracle_counts_equal_the_papers():
    lo, hi = GOLDEN["lo"], GOLDEN["hi"]
    assert oracle.count_primes(lo, hi) == GOLDEN["primes"]
    assert oracle.count_primes(lo, hi, safe=True) == GOLDEN["safe_primes"]


def test_oracle_count_small_cases():
    # pi(x) at textbook points and the safe primes below 1000 by definition
    assert [oracle.count_primes(0, x) for x in (10, 100, 1000, 10 ** 6)] == [4, 25, 168, 78498]
    brute = [p for p in range(2, 1000) if oracle.is_prime(p) and oracle.is_prime((p - 1) // 2)]
    assert oracle.count_primes(0, 1000, safe=True) == len(brute) == 25
    assert oracle.count_primes(5, 6, safe=True) == 1 and oracle.count_primes(0, 5, safe=True) == 0


def test_library_primality_code_on_host(harness):
    for n in list(range(0, 100000)) + [2 ** 32 - 5, 4294967291, 4294967279, 2 ** 31 + 11,
                                      3215031751, 2 ** 31 - 1, 2 ** 32 - 1]:
        assert harness.harness_is_prime(n) == oracle.is_prime(n), n
    rng = random.Random(11)
    windows = [(0, 1 << 18), (2 ** 31, 2 ** 31 + (1 << 18)), (2 ** 32 - (1 << 18), 2 ** 32)]
    windows += [(x, x + 200003) for x in (rng.randrange(2 ** 31, 2 ** 32 - 300000) for _ in range(3))]
    for lo, hi in windows:
        for safe in (0, 1):
            assert harness.harness_count(lo, hi, safe) == oracle.count_primes(lo, hi, safe), (lo, safe)


def test_oracle_next_prime_equals_trial_division():
    rng = inputs.SplitMix64(77)
    xs = np.array([(1 << 31) + (rng.next() >> 33) for _ in range(300)], dtype=np.int64)
    for exps in ((), (3,), inputs.SWEEP_EXPONENTS):
        filt = inputs._filter_mod(exps) if exps else None
        ref = inputs._next_prime_many(xs, filt)
        got = [oracle.next_prime(int(x), exps=exps) for x in xs]
        assert list(ref) == got, exps
    assert oracle.next_prime(4294967292) == 0 and oracle.next_prime(4294967291) == 4294967291
    assert oracle.next_prime(0, safe=True) == 5 and oracle.next_prime(8, safe=True) == 11
