"""Host checks of the lazy skip step the tile kernels use, and of the cases
that exercise its exact redo on the GPU (tests/lazy_skip_cases.py).

The kernels step the skips as r = 25 H + L with a s = H 2^63 + L, which is
congruent to a s mod Q = 2^63 - 25 (Implementation section) and below
2^63 + 2^37, and accept a run of such steps only when every value's upper
32 bits stay below those of Q.  The step is modelled here from that definition
and compared with the oracle's reduced step."""
import random

import oracle
from tests import lazy_skip_cases as L

Q, A = oracle.Q, oracle.A
HI_Q = Q >> 32
M64 = (1 << 64) - 1


def lazy_step(s):
    """The kernels' step without the final reduction, limb by limb."""
    t0 = A * (s & 0xffffffff)
    t1 = A * (s >> 32) + (t0 >> 32)
    assert t1 < 1 << 63
    H = t1 >> 31
    low = ((t1 & 0x7fffffff) << 32) | (t0 & 0xffffffff)
    return 25 * H + low


def test_lazy_step_congruent_and_bounded():
    rng = random.Random(1811)
    samples = [rng.randrange(Q) for _ in range(20000)]
    samples += [0, 1, Q - 1, Q - 2, (1 << 63) - (1 << 32), 1 << 62]
    for s in samples:
        r = lazy_step(s)
        assert r % Q == oracle.lcg_next(s)
        assert r < (1 << 63) + (1 << 37)
        if (r >> 32) < HI_Q:
            assert r < Q and r == oracle.lcg_next(s)
    # a lazy value is a valid input again: chains of lazy steps stay congruent
    s = rng.randrange(Q)
    r = s
    for _ in range(1000):
        r = lazy_step(r)
        s = oracle.lcg_next(s)
        assert r % Q == s and r < (1 << 63) + (1 << 37)
    # the largest inputs of the bound
    for r in ((1 << 63) + (1 << 37) - 1, Q, Q + 12345):
        assert lazy_step(r) % Q == oracle.lcg_next(r % Q)


def test_cases_put_their_values_where_stated():
    for k, v in L.UNREDUCED + L.HIGH_REDUCED:
        s0 = L.seed_for(k, v)
        assert oracle.skip(s0, k) == v


def test_unreduced_cases_are_unreduced():
    # the lazy step into each case's index gives v + Q, so the kernels must redo
    for k, v in L.UNREDUCED:
        s0 = L.seed_for(k, v)
        prev = oracle.skip(s0, k - 1)
        r = lazy_step(prev)
        assert r == v + Q, (k, v)
        assert (r >> 32) >= HI_Q
    for k, v in L.HIGH_REDUCED:
        s0 = L.seed_for(k, v)
        r = lazy_step(oracle.skip(s0, k - 1))
        assert r == v and (r >> 32) == HI_Q


def test_ranges_cover_the_cases():
    insts, cases = L.instances()
    for j, (k, _) in enumerate(cases):
        rs = [(k0, c) for i, k0, c in L.ranges_for(cases) if i == j]
        assert any(k0 <= k < k0 + c for k0, c in rs), k
        if (k + 20000) >> 20 == k >> 20:
            assert any(k0 > k and (k0 >> 20) == (k >> 20) for k0, _ in rs)
