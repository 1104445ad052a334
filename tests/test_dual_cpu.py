"""Dual-exponent instances (the footnote on CRT exponents): the combined
exponent, the footnote's identity m^e = Garner(m^ep mod p, m^eq mod q) on the
oracle, and the validation rule."""
import math
import random

import pytest

import oracle
from crt_helpers import combined_exponent as _combined


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def _safe_primes(count, seed):
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        p = oracle.next_prime(rng.randrange(2 ** 31, 2 ** 32 - 10 ** 7), safe=True)
        if p and p not in out:
            out.append(p)
    return out


def test_combined_exponent(R):
    ps = _safe_primes(6, 1)
    for i in range(0, 6, 2):
        p, q = ps[i], ps[i + 1]
        for ep, eq in ((3, 5), (5, 3), (17, 65537), (7, 7), (257, 3)):
            e = R.rsaprng_dual_exponent(p, q, ep, eq)
            assert e == _combined(p, q, ep, eq)
            assert e % (p - 1) == ep % (p - 1) and e % (q - 1) == eq % (q - 1)
            assert math.gcd(e, (p - 1) * (q - 1) // math.gcd(p - 1, q - 1)) == 1


def test_footnote_identity_on_oracle():
    # c = m^e mod n for the combined e equals Garner's recombination of
    # m^ep mod p and m^eq mod q (Python integers, independent of the oracle)
    ps = _safe_primes(4, 2)
    p, q = ps[0], ps[1]
    n = p * q
    for ep, eq in ((3, 5), (17, 3)):
        e = _combined(p, q, ep, eq)
        rng = random.Random(ep * 1000 + eq)
        ms = [rng.randrange(n) for _ in range(200)]
        cs = oracle.encrypt_array(n, e, ms)
        for m, c in zip(ms, cs):
            cp, cq = pow(m % p, ep, p), pow(m % q, eq, q)
            t = (cp - cq) * pow(q, -1, p) % p
            assert int(c) == t * q + cq


def test_validation(R):
    p, q = _safe_primes(2, 3)
    P = R.rsaprng_params_init_dual(p, q, 3, 5, 12345)
    assert (P.ep, P.eq, P.e, P.n) == (3, 5, 0, p * q)
    for ep, eq in ((2, 3), (3, (q - 1) // 2), (0, 3), (3, 2 ** 32 + 1)):
        with pytest.raises(R.RsaprngError) as ei:
            R.rsaprng_params_init_dual(p, q, ep, eq, 1)
        assert ei.value.code == -4, (ep, eq)
    # primes whose p - 1 and q - 1 share the factor 3: ep = eq mod 6 is needed
    p2 = oracle.next_prime(2 ** 31 + 1000, exps=(5, 7))
    while (p2 - 1) % 3:
        p2 = oracle.next_prime(p2 + 1, exps=(5, 7))
    q2 = oracle.next_prime(p2 + 1, exps=(5, 7))
    while (q2 - 1) % 3:
        q2 = oracle.next_prime(q2 + 1, exps=(5, 7))
    assert math.gcd(p2 - 1, q2 - 1) % 6 == 0
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_dual_exponent(p2, q2, 5, 7)          # 5 != 7 mod 6
    assert ei.value.code == -4
    assert R.rsaprng_dual_exponent(p2, q2, 5, 11) == _combined(p2, q2, 5, 11)
