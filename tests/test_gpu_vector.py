"""Vector mode on the GPU (rsaprng_generate_vector) against the oracle, bit for
bit: one to 2^24 substreams, windows that start and end inside a vector call,
vector calls that cross a block re-seeding, starts deep inside a block, every
exponent class, both exponentiation variants; large launches on sampled
outputs."""
import math

import numpy as np
import pytest

import inputs
import oracle
from gpu_helpers import assert_same, dev_f64, dev_u64, host_f64, host_u64, log

pytestmark = pytest.mark.gpu

B = 1 << 20


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def _gen(R, inst, s0=1):
    return R.rsaprng_create_ex(inst.p, inst.q, inst.e, inst.m0, s0)


def _run(R, g, mv, f0, count, variant):
    c, r = dev_u64(count), dev_f64(count)
    R.rsaprng_generate_vector(g, mv, f0, count, c, r, variant=variant)
    R.rsaprng_check_device_error()
    return host_u64(c, count), host_f64(r, count)


CASES = [
    (1, 0, 5000),
    (3, 0, 3 * 3000 + 2),
    (64, 7, 64 * 2000 + 5),
    (100, 100 * (B - 300) + 37, 100 * 600),       # calls cross the re-seeding at t = 2^20
    (1000, 5, 999),                                 # one partial call
    (1000, 1000 * 5 + 990, 20),                     # two partial calls, wraps at g = mv
    (4096, 0, 4096 * 300),
    (1 << 24, (1 << 24) * 3 - 500, 1000),           # the largest M_v
    (8, 8 * (3 * B + 500000), 8 * 100000),          # deep inside a block
    (7, 7 * (B - 1) - 3, 7 * (B + 10)),             # a whole block of calls
    (512, 512 * (B - 1000), 512 * 3000),            # wider segments (lead-in of a block)
]


@pytest.mark.parametrize("mv,f0,count", CASES)
def test_vector_matches_oracle(R, mv, f0, count):
    inst = inputs.config1()
    g = _gen(R, inst, s0=987654321)
    c_ref, r_ref = oracle.generate_vector(inst.p, inst.q, inst.e, inst.m0, 987654321, mv, f0, count)
    for variant in (1, 2):
        log("vector", mv, f0, count, "variant", variant)
        c, r = _run(R, g, mv, f0, count, variant)
        assert_same(c, r, c_ref, r_ref, "vector mv=%d f0=%d variant %d" % (mv, f0, variant))


def test_vector_every_exponent(R):
    base = inputs.config3(1)[0]
    lam = (base.p - 1) * (base.q - 1) // math.gcd(base.p - 1, base.q - 1)
    for e in (1, 3, 5, 7, 17, 257, 65537, 11, 101):
        if math.gcd(e, lam) != 1:
            continue
        inst = inputs.Instance(base.p, base.q, e, base.m0)
        g = _gen(R, inst)
        mv, f0, count = 96, 96 * (B - 20) + 50, 96 * 45
        c_ref, r_ref = oracle.generate_vector(inst.p, inst.q, e, inst.m0, 1, mv, f0, count)
        for variant in (1, 2):
            log("vector exponent", e, "variant", variant)
            c, r = _run(R, g, mv, f0, count, variant)
            assert_same(c, r, c_ref, r_ref, "vector e=%d variant %d" % (e, variant))


@pytest.mark.parametrize("mv,f0,count", [
    (4096, 4096 * (B - 100), 4096 * 300),           # 2^11-index segments
    (1 << 21, (1 << 21) * (B - 4), (1 << 21) * 8),  # 2^19-index segments (the widest)
])
def test_vector_large_sampled(R, mv, f0, count):
    inst = inputs.config1()
    g = _gen(R, inst)
    log("vector large", mv, f0, count)
    c, r = _run(R, g, mv, f0, count, 0)
    rng = np.random.default_rng(mv)
    idx = np.concatenate([[0, count - 1], rng.integers(0, count, 120)])
    for j in idx:
        cj, rj = oracle.generate_vector(inst.p, inst.q, inst.e, inst.m0, 1, mv, f0 + int(j), 1)
        assert int(c[j]) == int(cj[0]) and r[j] == rj[0], (mv, f0, int(j))


def test_vector_null_outputs_and_errors(R):
    import torch
    inst = inputs.config1()
    g = _gen(R, inst)
    mv, f0, count = 33, 1000, 5000
    c_ref, r_ref = oracle.generate_vector(inst.p, inst.q, inst.e, inst.m0, 1, mv, f0, count)
    c = dev_u64(count)
    R.rsaprng_generate_vector(g, mv, f0, count, c, None)
    r = dev_f64(count)
    R.rsaprng_generate_vector(g, mv, f0, count, None, r)
    assert_same(host_u64(c, count), host_f64(r, count), c_ref, r_ref, "null outputs")
    R.rsaprng_generate_vector(g, mv, f0, 0, c, r)          # empty: no-op
    x = torch.zeros(4, dtype=torch.int64, device="cuda")
    for bad_mv in (0, R.VECTOR_MAX_MV + 1):
        with pytest.raises(R.RsaprngError):
            R.rsaprng_generate_vector(g, bad_mv, 0, 4, x, None)
    with pytest.raises(R.RsaprngError):
        R.rsaprng_generate_vector(g, 4, R.VECTOR_MAX_END - 3, 4, x, None)
    with pytest.raises(R.RsaprngError):
        R.rsaprng_generate_vector(g, 4, 0, 4, x, None, variant=3)
