"""The seeded workload generators: the segmented sieve used for large draws
gives exactly what trial division gives, and the draws are deterministic."""
import numpy as np

import inputs


def test_sieve_equals_trial_division():
    rng = inputs.SplitMix64(31337)
    xs = [(1 << 31) + (rng.next() >> 33) for _ in range(1500)]
    # the ends of the range: the first candidates, the last prime and beyond it
    xs += [1 << 31, (1 << 31) + 1, inputs.LARGEST_PRIME_32 - 20, inputs.LARGEST_PRIME_32,
           inputs.LARGEST_PRIME_32 + 1, (1 << 32) - 1]
    xs = np.array(xs, dtype=np.int64)
    for exps in [(), (3,), inputs.SWEEP_EXPONENTS]:
        filt = inputs._filter_mod(exps) if exps else None
        a = inputs.next_primes_sieve(xs, exps)
        b = inputs._next_prime_many(xs, filt)
        assert np.array_equal(a, b), exps
        for x, pv in zip(xs[:50], a[:50]):
            assert inputs.is_prime32(int(pv)) and pv >= x
    assert inputs.next_primes_sieve([inputs.LARGEST_PRIME_32 + 1])[0] == 0


def test_large_draws_use_the_same_primes():
    # a draw large enough to take the sieve path equals the trial-division draw
    rng_a = inputs.SplitMix64(7)
    rng_b = inputs.SplitMix64(7)
    a = inputs.draw_instances_rng(rng_a, 6000, (3,))
    saved = inputs.SIEVE_MIN
    try:
        inputs.SIEVE_MIN = 1 << 62
        b = inputs.draw_instances_rng(rng_b, 6000, (3,))
    finally:
        inputs.SIEVE_MIN = saved
    assert a == b and rng_a.state == rng_b.state


def test_served_workload_shapes():
    insts, rng = inputs.config5_instances(200)
    reqs = inputs.config5_requests(rng, len(insts), 2000)
    cnt = np.array([r.count for r in reqs])
    assert cnt.min() >= 1 << 10 and cnt.max() < 1 << 24
    assert all(0 <= r.k0 < 1 << 40 and 0 <= r.inst < 200 for r in reqs)
    for i in insts:
        assert i.e in inputs.BATCH_EXPONENTS and inputs.gcd(i.e, inputs.lam(i.p, i.q)) == 1
    t = inputs.poisson_arrivals(rng, 100.0, 5000)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0) and abs(gaps.mean() * 100.0 - 1.0) < 0.05
