"""Instances whose skip sequence takes chosen values at chosen indices.

The skips are s_k = s0 a^k mod Q (Implementation section), so the seed
s0 = v a^-k mod Q puts the value v at index k.  The tile kernels step the skips
without the final reduction mod Q and redo a lane's walk with reduced steps
when one of its values may be >= Q (a value whose upper 32 bits reach those of
Q).  These cases put such values inside and before requested ranges, at several
positions of a lane's run of skips, so that the redo is what produces the
outputs there:

- a small v: the unreduced step gives v + Q (checked on the host by
  tests/test_lazy_skip_cpu.py);
- v = Q - 1 - j: a reduced value with the upper word of Q, which the test
  cannot tell from an unreduced one.
"""
import inputs
import oracle

Q = oracle.Q
A = oracle.A
B = 1 << 20

# (index, value): positions 1, 2, 7 of a run of 8 skips, the middle and last
# of a run of 128 (the prefix pass of the 8192-index tiles), the last index of
# a 2^20 block, and an index far into the sequence
UNREDUCED = ((9, 1000), (8 * 37 + 2, 2001), (8 * 100 + 7, 77), (128 * 5 + 64, 123456),
             (128 * 9 + 127, 5), (B - 1, 999), (3 * B + 8 * 1000 + 5, 31337),
             ((1 << 40) + 8 * 5 + 3, 4242))
HIGH_REDUCED = ((8 * 11 + 3, Q - 1), (128 * 3 + 1, Q - 2))


def seed_for(k: int, v: int) -> int:
    """s0 with s0 a^k = v (mod Q)."""
    s0 = v * pow(A, -k, Q) % Q
    assert 1 <= s0 < Q
    return s0


def instances(exps=(3,)):
    """One instance per case, on the prime pairs of the exponent sweep (valid for
    3, 5, 17, 257 and 65537), the exponents taken from exps in turn; returns
    (instances, the case of each)."""
    cases = UNREDUCED + HIGH_REDUCED
    base = inputs.config3(len(cases))
    out = []
    for j, (b, (k, v)) in enumerate(zip(base, cases)):
        out.append(inputs.Instance(b.p, b.q, exps[j % len(exps)], b.m0, seed_for(k, v)))
    return out, cases


def ranges_for(cases):
    """Requested ranges per case: one around the index, one starting after it in
    the same block (its lead-in walks over the index), one from the block start."""
    out = []
    for j, (k, _) in enumerate(cases):
        blk = k & ~(B - 1)
        out.append((j, max(k - 300, 0), 1000))
        after = k + 20000 if (k + 20000) >> 20 == k >> 20 else k + 1
        out.append((j, after, 3000))
        out.append((j, blk, min(k - blk + 700, 40000) if k - blk < 39000 else 4096))
    return out
