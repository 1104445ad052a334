"""GPU parameter generation against the paper's counts and the oracle."""
import json
import os

import numpy as np
import pytest

import inputs
import oracle
from gpu_helpers import log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_prime_counts.json")))


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def test_full_range_counts_equal_the_papers(R):
    log("prime_count [2^31, 2^32)")
    assert R.rsaprng_prime_count(GOLDEN["lo"], GOLDEN["hi"]) == GOLDEN["primes"]
    log("safe prime_count [2^31, 2^32)")
    assert R.rsaprng_prime_count(GOLDEN["lo"], GOLDEN["hi"], safe=True) == GOLDEN["safe_primes"]


def test_window_counts_match_oracle(R):
    rng = inputs.SplitMix64(3)
    windows = [(0, 1), (0, 2), (0, 30), (0, 1 << 20), (5, 6), (7, 8), (2 ** 32 - 12345, 2 ** 32),
               (2 ** 31 - 77, 2 ** 31 + 77)]
    windows += [(x, x + 1000003) for x in ((1 << 31) + (rng.next() >> 33) for _ in range(4))]
    for lo, hi in windows:
        for safe in (False, True):
            log("prime_count window", lo, hi, safe)
            assert R.rsaprng_prime_count(lo, min(hi, 1 << 32), safe) == \
                oracle.count_primes(lo, min(hi, 1 << 32), safe), (lo, hi, safe)


def test_next_primes_match_oracle(R):
    import torch
    rng = inputs.SplitMix64(19)
    xs = [(1 << 31) + (rng.next() >> 33) for _ in range(1500)]
    xs += [0, 1, 2, 3, 4, 2 ** 32 - 5, 2 ** 32 - 4, 4294967291, 4294967279, 2 ** 32 - 1]
    x = torch.tensor(xs, dtype=torch.int64, device="cuda")
    out = torch.empty_like(x)
    for safe in (False, True):
        for exps in ((), (3,), inputs.SWEEP_EXPONENTS):
            log("next_primes", safe, exps)
            R.rsaprng_next_primes(x, out, safe=safe, exps=exps)
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint64)
            for i, xi in enumerate(xs):
                assert int(got[i]) == oracle.next_prime(xi, safe, exps), (xi, safe, exps)


def test_errors(R):
    import torch
    x = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(R.RsaprngError):
        R.rsaprng_next_primes(x, x, exps=(3, 1))           # f < 2
    with pytest.raises(R.RsaprngError):
        R.rsaprng_next_primes(x, x, exps=tuple(range(3, 21, 2)))  # more than 8
    with pytest.raises(R.RsaprngError):
        R.rsaprng_prime_count(10, 2 ** 32 + 1)
