"""Pins of the CPU oracle against facts the paper and elementary number theory fix.

None of these re-type the oracle's own formula: each compares it with a
different computation that must agree (the paper's CRT algorithm, decryption,
a brute-force permutation check, exact rational arithmetic, number facts the
paper states) so that a dropped term, wrong sign, wrong index or swapped
operand in the oracle fails at least one of them.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import inputs
import oracle

Q = oracle.Q
A = oracle.A
B = oracle.BLOCK


# ---------------------------------------------------------------------------
# Number facts of the Implementation section
# ---------------------------------------------------------------------------

def _mr_py(n, bases=(2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)):
    """Deterministic Miller-Rabin for n < 3.3e24 (independent of the oracle's C code)."""
    if n < 2:
        return False
    for b in bases:
        if n % b == 0:
            return n == b
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for b in bases:
        x = pow(b, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


Q_MINUS_1_FACTORS = {2: 1, 3: 4, 17: 1, 23: 1, 319279: 1, 456065899: 1}


def test_skip_modulus_is_largest_prime_below_2_63():
    # Q = 2^63 - 25 is prime and the largest prime below 2^63 (Implementation section).
    assert Q == 2 ** 63 - 25
    assert _mr_py(Q)
    for x in range(Q + 1, 2 ** 63):
        assert not _mr_py(x)


def test_q_minus_1_has_no_factor_in_32_bit_prime_range():
    # The full period (Q-1)n needs Q-1 coprime to every prime in [2^31, 2^32].
    prod = 1
    for f, k in Q_MINUS_1_FACTORS.items():
        assert inputs.is_prime32(f)
        prod *= f ** k
    assert prod == Q - 1
    assert all(not (2 ** 31 <= f <= 2 ** 32) for f in Q_MINUS_1_FACTORS)


def _is_primitive_root(g):
    return all(pow(g, (Q - 1) // f, Q) != 1 for f in Q_MINUS_1_FACTORS)


def test_recommended_multiplier_is_restricted_primitive_root():
    # a = 2307085864 (L'Ecuyer, Blouin, Couture) is a primitive root mod Q, lies in
    # [2^31, 2^32] and gives q2 < q1, the restriction that keeps Schrage's form in 64 bits.
    assert A == 2307085864
    assert _is_primitive_root(A)
    q1, q2 = Q // A, Q % A
    assert 2 ** 31 <= A <= 2 ** 32 and q2 < q1


def test_footnote_multipliers():
    # Footnote on Sezgin & Sezgin's table: eight of the nine listed multipliers are
    # primitive roots mod Q; 3163786287 is not (its (Q-1)/2 power is 1).  Recorded as a
    # reading of a misprint in the paper.
    listed = [3157107955, 3163786287, 3200261722, 3211103532, 3338736601,
              3423977237, 3465965455, 3474009732, 3512424704]
    prim = {g: _is_primitive_root(g) for g in listed}
    assert [g for g, ok in prim.items() if not ok] == [3163786287]
    assert pow(3163786287, (Q - 1) // 2, Q) == 1
    # the five "intentionally bad" roots of the Tests section are primitive too
    assert all(_is_primitive_root(g) for g in (3, 6, 7, 10, 11))
    assert not _is_primitive_root(2) and not _is_primitive_root(4)


# ---------------------------------------------------------------------------
# Skip generator
# ---------------------------------------------------------------------------

EDGE_S = [1, 2, Q - 1, Q - 2, Q // A - 1, Q // A, Q // A + 1, 2 ** 62, 2 ** 32 - 1, 2 ** 32, 12345]


def test_lcg_three_ways():
    # 128-bit product, the paper's Schrage decomposition, and Python integers agree.
    rng = random.Random(1)
    for s in EDGE_S + [rng.randrange(1, Q) for _ in range(20000)]:
        want = A * s % Q
        assert oracle.lcg_next(s) == want
        assert oracle.lcg_next_schrage(s) == want


def test_skip_jump_equals_walk():
    # s_k = s0 a^k mod Q: the jump equals k single steps (eq. congruentialgenerator1).
    for s0 in (1, 987654321, Q - 1):
        s = s0
        for k in range(1, 3000):
            s = oracle.lcg_next(s)
            if k % 97 == 0 or k < 5:
                assert oracle.skip(s0, k) == s


def test_skip_period():
    # a primitive: s_{k + Q - 1} = s_k, and a^((Q-1)/2) = -1.
    assert oracle.skip(1, Q - 1) == 1
    assert oracle.skip(5, Q - 1 + 17) == oracle.skip(5, 17)
    assert oracle.skip(1, (Q - 1) // 2) == Q - 1


def test_block_seed_closed_form_equals_walk():
    # G_b by the geometric-series closed form equals the exact integer sum of the
    # walked skips, reduced mod Q (eq. pseudoskip).
    for s0 in (1, 31337):
        for b in (1, 2):
            assert oracle.block_seed(s0, b) == oracle.block_seed_walk(s0, b)
    assert oracle.block_seed(1, 0) == 0


def test_block_seed_chains_across_blocks():
    # G_{b+1} = G_b + (sum of the skips of block b+1) mod Q, for blocks far from 0,
    # where the skips of the block are produced by the jump and walked.
    s0 = 7
    for b in (5, 123456, 2 ** 20 + 3):
        k = b * B
        s = oracle.skip(s0, k)
        total = 0
        for _ in range(B):
            s = oracle.lcg_next(s)
            total += s
        assert (oracle.block_seed(s0, b) + total) % Q == oracle.block_seed(s0, b + 1)


# ---------------------------------------------------------------------------
# Messages and ciphertexts
# ---------------------------------------------------------------------------

def _c1():
    return inputs.config1()


def test_paper_algorithm1_equals_definition_block0():
    # The paper's algorithm (1) (Schrage step, CRT residues, two 32-bit
    # exponentiations, Garner, divide) returns c_1, c_2, ...; the oracle's direct
    # evaluation mod n must match it bit for bit over block 0.
    cases = [_c1()] + inputs.config2(4) + inputs.edge_instances()
    sweep = inputs.config3(2)
    for e in inputs.SWEEP_EXPONENTS:
        for i in sweep:
            cases.append(inputs.Instance(i.p, i.q, e, i.m0))
    for j, inst in enumerate(cases):
        count = B - 1 if j == 0 else 1 << 14
        c_ref, r_ref = oracle.paper_algorithm1(inst.p, inst.q, inst.e, inst.m0, inst.s0, count)
        c, r = oracle.generate_instance(inst, 1, count)
        assert np.array_equal(c, c_ref), inst
        assert np.array_equal(r.view(np.uint64), r_ref.view(np.uint64)), inst


def test_message_steps_are_skips():
    # Inside a block m_k - m_{k-1} = s_k (mod n); at a block start the message is
    # m0 + G_b with G_b from the walk (P1), and after it the steps resume.
    inst = _c1()
    n = inst.n
    for k0 in (1, 5000, B - 3, 3 * B - 2, 77 * B + 11):
        m = oracle.messages(inst.p, inst.q, inst.m0, inst.s0, k0 - 1, 6)
        for i in range(1, 6):
            k = k0 - 1 + i
            if k % B == 0:
                g = oracle.block_seed_walk(inst.s0, k // B) if k // B <= 3 else oracle.block_seed(inst.s0, k // B)
                assert int(m[i]) == (inst.m0 + g) % n
            else:
                assert (int(m[i]) - int(m[i - 1])) % n == oracle.skip(inst.s0, k) % n


def test_decryption_recovers_messages():
    # c^d mod n = m with d = e^-1 mod lambda(n) and mod phi(n) (eqs. decrypt, decryptproof).
    insts = [_c1()] + inputs.config2(3) + inputs.edge_instances()
    insts += [inputs.Instance(i.p, i.q, e, i.m0) for i in inputs.config3(1) for e in inputs.SWEEP_EXPONENTS]
    for inst in insts:
        n = inst.n
        phi = (inst.p - 1) * (inst.q - 1)
        lam = phi // math.gcd(inst.p - 1, inst.q - 1)
        for k0 in (0, B - 50, 9 * B + 5, (1 << 40) + 3):
            m = oracle.messages(inst.p, inst.q, inst.m0, inst.s0, k0, 100)
            c, _ = oracle.generate_instance(inst, k0, 100, want_r=False)
            for mod in (lam, phi):
                d = pow(inst.e, -1, mod)
                assert [pow(int(x), d, n) for x in c] == [int(x) for x in m]
        assert oracle.decryption_exponent(inst.p, inst.q, inst.e, True) == pow(inst.e, -1, lam)
        assert oracle.decryption_exponent(inst.p, inst.q, inst.e, False) == pow(inst.e, -1, phi)


def test_encryption_is_bijection_small_primes():
    # Encryption permutes Z_n when gcd(e, phi) = 1 (bijection statement); brute force
    # with 10-12 bit primes (every one of the up to 2^24 messages).
    for bits in (10, 11, 12):
        for inst in inputs.small_instances(100 + bits, 2, bits=bits):
            for e in (inst.e, 65537):
                if math.gcd(e, (inst.p - 1) * (inst.q - 1)) != 1:
                    continue
                m = np.arange(inst.n, dtype=np.uint64)
                c = oracle.encrypt_array(inst.n, e, m)
                assert np.array_equal(np.sort(c), m)


def test_encryption_not_bijection_when_rule_fails():
    # Negative control: e = 3 with p = 1 (mod 3) collapses three messages onto one.
    p = next(x for x in range(4099, 8000) if inputs.is_prime32(x) and x % 3 == 1)
    q = next(x for x in range(5003, 8000) if inputs.is_prime32(x) and x % 3 == 2)
    n = p * q
    c = oracle.encrypt_array(n, 3, np.arange(n, dtype=np.uint64))
    assert np.unique(c).size < n


def test_parameter_rule():
    c1 = _c1()
    assert oracle.check_params(c1.p, c1.q, c1.e) == 0
    assert oracle.check_params(c1.p, c1.q, 1) == 0          # weakened e = 1 is allowed
    assert oracle.check_params(c1.p, c1.p, 3) == -2
    assert oracle.check_params(c1.p, c1.q + 1, 3) in (-1, -3)
    assert oracle.check_params(c1.p, 2 ** 31 - 1, 3) == -3
    assert oracle.check_params(c1.p, c1.q, 2) == -4
    assert oracle.check_params(c1.p, c1.q, 0) == -4
    # gcd(e, lambda) = 1 <=> gcd(e, phi) = 1 on random draws, and the oracle agrees
    rng = random.Random(5)
    ps = [i.p for i in inputs.config3(64)] + [i.p for i in inputs.config2(64)]
    for _ in range(300):
        p, q = rng.choice(ps), rng.choice(ps)
        if p == q:
            continue
        e = rng.randrange(1, 200) | 1
        phi = (p - 1) * (q - 1)
        lam = phi // math.gcd(p - 1, q - 1)
        assert (math.gcd(e, phi) == 1) == (math.gcd(e, lam) == 1)
        assert (oracle.check_params(p, q, e) == 0) == (math.gcd(e, lam) == 1)


def _sieve(lo, hi):
    """Primality flags for [lo, hi) by a segmented sieve of Eratosthenes."""
    flags = np.ones(hi - lo, dtype=bool)
    lim = int(math.isqrt(hi)) + 1
    base = np.ones(lim + 1, dtype=bool)
    base[:2] = False
    for i in range(2, int(lim ** 0.5) + 1):
        if base[i]:
            base[i * i::i] = False
    for pr in np.nonzero(base)[0]:
        pr = int(pr)
        start = max(pr * pr, (lo + pr - 1) // pr * pr)
        flags[start - lo::pr] = False
    return flags


def test_miller_rabin_matches_sieve():
    # Miller-Rabin with the five smallest bases is exact below 2^32 (Implementation
    # section): compare with a sieve at both ends of the 32-bit prime range.
    for lo in (2 ** 31, 2 ** 32 - 2 ** 18):
        hi = lo + 2 ** 18
        flags = _sieve(lo, hi)
        got = np.array([oracle.is_prime(x) for x in range(lo, hi)])
        assert np.array_equal(got, flags)
    # strong pseudoprime to bases 2, 3, 5, 7: needs base 11
    assert not oracle.is_prime(3215031751)
    # 64-bit branch (twelve bases)
    assert oracle.is_prime(Q) and oracle.is_prime(2 ** 61 - 1)
    assert not oracle.is_prime(4294967291 * 4294967279)
    rng = random.Random(3)
    for _ in range(2000):
        x = rng.randrange(2 ** 32, 2 ** 64) | 1
        assert oracle.is_prime(x) == _mr_py(x)


def test_cribs():
    # m = 0, 1, n-1 encrypt to themselves for every allowed e (Pseudorandom skips).
    inst = _c1()
    n = inst.n
    for m0, want in ((0, 0), (1, 1), (n - 1, n - 1)):
        c, r = oracle.generate(inst.p, inst.q, inst.e, m0, 1, 0, 1)
        assert int(c[0]) == want
    # r_0 for the three cribs: 0, RN(1)/RN(n), and the guard value (RN(n-1) = RN(n)).
    assert oracle.ratio(0, n) == 0.0
    assert oracle.ratio(1, n) == 1.0 / float(n)
    assert float(n - 1) == float(n)
    assert oracle.ratio(n - 1, n) == float.fromhex("0x1.fffffffffffffp-1")


def test_exponent_one_returns_messages():
    # e = 1 is the paper's weakened generator: c_k = m_k.
    inst = _c1()
    for k0 in (0, B - 7, 4 * B + 100):
        m = oracle.messages(inst.p, inst.q, inst.m0, inst.s0, k0, 2000)
        c, _ = oracle.generate(inst.p, inst.q, 1, inst.m0, inst.s0, k0, 2000, want_r=False)
        assert np.array_equal(c, m)


def test_period_precondition():
    # gcd(Q(Q-1)/2, n) = 1 for every drawn modulus, so the period is (Q-1)n.
    b = Q * (Q - 1) // 2
    for inst in [_c1()] + inputs.config2(64) + inputs.config3(64):
        assert math.gcd(b, inst.n) == 1


# ---------------------------------------------------------------------------
# Floating point
# ---------------------------------------------------------------------------

def _rn_int(x):
    """Round a non-negative integer to 53 significant bits, ties to even (integer only)."""
    if x < (1 << 53):
        return x
    sh = x.bit_length() - 53
    q, rem = x >> sh, x & ((1 << sh) - 1)
    half = 1 << (sh - 1)
    if rem > half or (rem == half and q & 1):
        q += 1
    return q << sh


def _is_correctly_rounded_quotient(r, a, b):
    """r == RN(a/b) for doubles a, b (exact rational check with ties to even)."""
    exact = Fraction(a) / Fraction(b)
    fr = Fraction(r)
    lo = Fraction(np.nextafter(r, -np.inf)) if r > 0 else None
    hi = Fraction(np.nextafter(r, np.inf))
    dist = abs(fr - exact)
    if lo is not None and abs(lo - exact) < dist:
        return False
    if abs(hi - exact) < dist:
        return False
    if (lo is not None and abs(lo - exact) == dist) or abs(hi - exact) == dist:
        return (int(np.float64(r).view(np.uint64)) & 1) == 0
    return True


def test_ratio_is_rn_of_rn_quotient():
    insts = [_c1()] + inputs.edge_instances() + inputs.config2(4)
    for inst in insts:
        n = inst.n
        c, r = oracle.generate_instance(inst, 3 * B - 40, 2000)
        assert float(n) == _rn_int(n)
        for ci, ri in zip(c[:400], r[:400]):
            ci = int(ci)
            cd = float(ci)
            assert cd == _rn_int(ci)
            if cd == float(n):
                assert ri == float.fromhex("0x1.fffffffffffffp-1")
            else:
                assert ri < 1.0
                assert _is_correctly_rounded_quotient(float(ri), cd, float(n))


def test_ratio_guard_only_when_rn_equal():
    inst = inputs.edge_instances()[0]        # n close to 2^64: ulp(n) = 2048
    n = inst.n
    for c in list(range(n - 3000, n)) + [n // 2, 1, 0]:
        r = oracle.ratio(c, n)
        assert 0.0 <= r < 1.0
        assert (r == float.fromhex("0x1.fffffffffffffp-1") and float(c) == float(n)) or float(c) != float(n)


# ---------------------------------------------------------------------------
# Statistics of the fused-consume mode
# ---------------------------------------------------------------------------

def test_stats_exact_sum_histogram():
    inst = inputs.config2(1)[0]
    count = 50000
    _, r = oracle.generate_instance(inst, 12345, count, want_c=False)
    st = oracle.consume(inst.p, inst.q, inst.e, inst.m0, inst.s0, 12345, count)
    exact = sum(Fraction(float(x)) for x in r)
    assert Fraction(st["sum_fx"], 1 << 128) == exact
    hist = np.bincount(np.floor(r * 1024).astype(np.int64), minlength=1024)
    assert np.array_equal(st["hist"], hist.astype(np.uint64))
    assert st["lt_half"] == int(np.sum(r < 0.5))
    # stats_of on an explicit array agrees
    st2 = oracle.stats_of(r)
    assert st2["sum_fx"] == st["sum_fx"] and np.array_equal(st2["hist"], st["hist"])


def test_uniformity_chi_square():
    # chi^2 of r_k in 1024 bins; p-value inside the paper's [1e-6, 1 - 1e-6] band.
    from scipy.stats import chi2
    insts = inputs.config2(4)
    for inst in insts:
        st = oracle.consume(inst.p, inst.q, inst.e, inst.m0, inst.s0, 0, 1 << 20)
        h = st["hist"].astype(np.float64)
        exp = h.sum() / 1024
        x2 = float(((h - exp) ** 2 / exp).sum())
        pv = chi2.sf(x2, 1023)
        assert 1e-6 < pv < 1 - 1e-6, (inst, x2, pv)
        frac = st["lt_half"] / (1 << 20)
        assert abs(frac - 0.5) < 5 * 0.5 / 1024
