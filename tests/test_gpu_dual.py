"""Dual-exponent instances on the GPU against the oracle run with the combined
exponent e (e = ep mod (p-1), e = eq mod (q-1)), found by the Chinese remainder
theorem in plain Python: the footnote's construction must give exactly m^e mod n."""
import random

import numpy as np
import pytest

import oracle
from crt_helpers import combined_exponent
from gpu_helpers import assert_same, dev_f64, dev_u64, host_f64, host_u64, log

pytestmark = pytest.mark.gpu

B = 1 << 20
PAIRS = ((3, 5), (5, 3), (17, 3), (3, 65537), (257, 17), (7, 7))


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def _instances():
    rng = random.Random(2024)
    ps = []
    while len(ps) < 2 * len(PAIRS):
        p = oracle.next_prime(rng.randrange(2 ** 31, 2 ** 32 - 10 ** 7), safe=True)
        if p and p not in ps:
            ps.append(p)
    out = []
    for j, (ep, eq) in enumerate(PAIRS):
        p, q = ps[2 * j], ps[2 * j + 1]
        out.append((p, q, ep, eq, rng.randrange(p * q)))
    return out


@pytest.mark.parametrize("cfg_kw", [dict(variant=2), dict(variant=2, prefix=2),
                                    dict(variant=1, prefix=1)])
def test_dual_pool_generate_and_consume(R, cfg_kw):
    insts = _instances()
    pool = R.Pool.dual([i[0] for i in insts], [i[1] for i in insts], [i[2] for i in insts],
                       [i[3] for i in insts], [i[4] for i in insts])
    ranges = [(j, k0, cnt) for j in range(len(insts))
              for k0, cnt in ((0, 5000), (B - 777, 3000), ((1 << 41) + 5, 4099))]
    total = sum(c for _, _, c in ranges)
    oc, orr = dev_u64(total), dev_f64(total)
    reqs, off = [], 0
    for j, k0, cnt in ranges:
        reqs.append((j, k0, cnt, off))
        off += cnt
    cfg = R.config(**cfg_kw)
    log("dual generate", cfg_kw)
    R.rsaprng_pool_generate(pool, reqs, oc, orr, cfg=cfg)
    R.rsaprng_check_device_error()
    c, r = host_u64(oc, total), host_f64(orr, total)
    off = 0
    for j, k0, cnt in ranges:
        p, q, ep, eq, m0 = insts[j]
        e = combined_exponent(p, q, ep, eq)
        cref, rref = oracle.generate(p, q, e, m0, 1, k0, cnt)
        assert_same(c[off:off + cnt], r[off:off + cnt], cref, rref, "dual %s inst %d" % (cfg_kw, j))
        off += cnt
    # consume over the same ranges, one record per range
    st = R.stats_tensor(len(ranges))
    log("dual consume", cfg_kw)
    R.rsaprng_pool_consume(pool, [(j, k0, cnt, idx) for idx, (j, k0, cnt) in enumerate(ranges)],
                           st, cfg=cfg)
    R.rsaprng_check_device_error()
    got = R.stats_decode(st)
    for idx, (j, k0, cnt) in enumerate(ranges):
        p, q, ep, eq, m0 = insts[j]
        ref = oracle.consume(p, q, combined_exponent(p, q, ep, eq), m0, 1, k0, cnt)
        assert got[idx]["sum_fx"] == ref["sum_fx"] and np.array_equal(got[idx]["hist"], ref["hist"])
