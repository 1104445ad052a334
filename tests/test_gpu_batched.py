"""The batched uneven workload's shape on the GPU: the first 500 requests of the
10,000-instance batched workload (their drawn exponent mix, lengths
log-uniform in [2^8, 2^22] and starts below 2^40; about 2.4e8 outputs) through
the autotuner and then a graph-captured batch with its chosen configuration.
Every output the autotuner leaves and every output of two graph replays (with
eager work between them) is compared bit for bit with the oracle; and the
autotuner in consume mode over mixed exponents, record by record."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import inputs
from tests.gpu_helpers import assert_same, dev_f64, dev_u64, host_f64, host_u64, log, oracle_gen

pytestmark = pytest.mark.gpu

N_REQ = 500


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1811_11629_amd import rsaprng
    assert torch.cuda.is_available()
    rsaprng.lib()
    return rsaprng


@pytest.fixture(scope="module")
def workload():
    insts, reqs4 = inputs.config4()
    reqs, off = [], 0
    for r in reqs4[:N_REQ]:
        reqs.append((r.inst, r.k0, r.count, off))
        off += r.count
    # the oracle's outputs, on the host's threads
    threads = min(16, os.cpu_count() or 1)

    def one(q):
        i, k0, cnt, _ = q
        return oracle_gen(insts[i], k0, cnt)

    with cf.ThreadPoolExecutor(threads) as ex:
        ref = list(ex.map(one, reqs))
    return insts, reqs, off, ref


def _compare(reqs, ref, oc, orr, total, what):
    c, r = host_u64(oc, total), host_f64(orr, total)
    for (i, k0, cnt, o), (cref, rref) in zip(reqs, ref):
        assert_same(c[o:o + cnt], r[o:o + cnt], cref, rref, "%s inst %d k0 %d" % (what, i, k0))


def test_batched_uneven_autotune_and_graph(R, workload):
    import torch
    insts, reqs, total, ref = workload
    es = sorted({insts[i].e for i, _, _, _ in reqs})
    log("batched uneven subset: %d requests, %d outputs, e in %s" % (len(reqs), total, es))
    pool = R.Pool.from_instances(insts)
    stream = torch.cuda.Stream()
    oc, orr = dev_u64(total), dev_f64(total)
    log("autotune over the subset")
    best, ms = R.rsaprng_autotune(pool, reqs, R.MODE_GENERATE, oc, orr, stream=stream)
    stream.synchronize()
    log("autotuner chose %s (%.3f ms); comparing its output" % (best.as_dict(), ms))
    _compare(reqs, ref, oc, orr, total, "autotuner output")
    b = R.Batch(pool, reqs, R.MODE_GENERATE, oc, orr, cfg=best, stream=stream)
    for rep in range(2):
        oc.fill_(-1)
        orr.fill_(float("nan"))
        scratch = torch.randn(1 << 20, device="cuda")        # eager work between replays
        (scratch * 2).sum().item()
        log("graph replay %d" % rep)
        b.run(stream)
        stream.synchronize()
        b.check()
        _compare(reqs, ref, oc, orr, total, "graph replay %d" % rep)
    R.rsaprng_check_device_error(stream)


def test_consume_autotune_matches_oracle(R):
    """The autotuner in consume mode over mixed exponents and ragged ranges: the
    records it leaves, and those of a graph-captured batch with its choice, equal
    the oracle's statistics record by record."""
    import torch
    from fractions import Fraction

    from tests.gpu_helpers import oracle_stats
    base = inputs.config3(8)
    es = (3, 5, 17, 257, 65537, 7)
    insts = [inputs.Instance(b.p, b.q, es[i % len(es)], b.m0) for i, b in enumerate(base)]
    B = 1 << 20
    ranges = [(i, k0, cnt) for i in range(len(insts))
              for k0, cnt in ((0, 1 << 16), (B - 2500, 7000), ((1 << 40) + 3 * i, 5000 + i))]
    reqs = [(j, k0, cnt, idx) for idx, (j, k0, cnt) in enumerate(ranges)]
    refs = [oracle_stats(insts[j], k0, cnt) for j, k0, cnt in ranges]
    pool = R.Pool.from_instances(insts)
    stream = torch.cuda.Stream()
    st = R.stats_tensor(len(ranges))

    def check(what):
        got = R.stats_decode(st)
        for idx, ref in enumerate(refs):
            g = got[idx]
            assert g["count"] == ranges[idx][2], (what, idx)
            assert g["sum_fx"] == ref["sum_fx"], (what, idx)
            assert g["lt_half"] == ref["lt_half"], (what, idx)
            assert np.array_equal(g["hist"], ref["hist"]), (what, idx)
            assert g["sum"] == float(Fraction(ref["sum_fx"], 1 << 128)), (what, idx)

    log("consume autotune: %d records" % len(ranges))
    best, ms = R.rsaprng_autotune(pool, reqs, R.MODE_CONSUME, stats=st, stream=stream)
    stream.synchronize()
    check("autotuner")
    b = R.Batch(pool, reqs, R.MODE_CONSUME, stats=st, cfg=best, stream=stream)
    st.fill_(-1)                      # the launch clears its records itself
    torch.cuda.synchronize()
    log("consume batch with %s" % best.as_dict())
    b.run(stream)
    stream.synchronize()
    b.check()
    check("batch")
    R.rsaprng_check_device_error(stream)
