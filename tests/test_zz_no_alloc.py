"""The no-allocation entry point (rsaprng_pool_generate_noalloc) against
rsaprng_pool_generate, bit for bit, on two calls in a row (the second smaller),
through the C ABI; its size limit and error codes."""
import numpy as np
import pytest

import inputs
from tests.gpu_helpers import assert_same, dev_f64, dev_u64, host_f64, host_u64, log, oracle_gen

pytestmark = pytest.mark.gpu

B = 1 << 20
SENTINEL = 0x5A5A5A5A5A5A5A5A


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1811_11629_amd import rsaprng
    assert torch.cuda.is_available()
    rsaprng.lib()
    return rsaprng


def _instances():
    base = inputs.config3()[:24]
    es = (3, 5, 17, 65537, 3, 257)
    return [inputs.Instance(b.p, b.q, es[i % len(es)], b.m0) for i, b in enumerate(base)]


def _requests(rng, n_inst, n_req, max_count):
    """Ragged requests packed back to back, every other one at an odd element:
    block crossings, starts deep in a block, k near 2^63 and near 2^64, runs of
    requests that continue each other (merged into one range)."""
    reqs, off = [], 1
    for j in range(n_req):
        i = int(rng.integers(n_inst))
        cnt = int(rng.integers(1, max_count))
        kind = j % 5
        if kind == 0:
            k0 = int(rng.integers(1 << 24))
        elif kind == 1:
            k0 = int(rng.integers(1, 8)) * B - cnt // 2          # crosses a block start
        elif kind == 2:
            k0 = (1 << 63) + int(rng.integers(1 << 30))
        elif kind == 3:
            k0 = (1 << 64) - cnt                                  # ends at the last index
        else:
            k0 = int(rng.integers(1 << 40))
        reqs.append((i, k0, cnt, off))
        off += cnt
        if kind == 4:                                             # a continuation
            c2 = int(rng.integers(1, max_count))
            reqs.append((i, k0 + cnt, c2, off))
            off += c2
        off += j & 1                                              # odd / even starts
    return reqs, off


def _run(R, fn, pool, reqs, total, cfg, stream):
    import torch
    oc, orr = dev_u64(total), dev_f64(total)
    oc.fill_(SENTINEL)
    orr.view(torch.int64).fill_(SENTINEL)
    torch.cuda.synchronize()
    fn(pool, reqs, oc, orr, cfg=cfg, stream=stream)
    return oc, orr


def test_noalloc_matches_pool_generate(R, monkeypatch):
    import torch
    insts = _instances()
    pool = R.Pool.from_instances(insts)
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(20260)
    cfgs = [None,
            R.config(variant=2, prefix=0, lanes_per_tile=256, chunks_per_wave=1),
            R.config(variant=2, prefix=0, lanes_per_tile=512, chunks_per_wave=2, persistent=1),
            R.config(variant=2, prefix=2, lanes_per_tile=512, chunks_per_wave=2),
            R.config(variant=1, prefix=2, lanes_per_tile=256, chunks_per_wave=4, persistent=1),
            R.config(variant=2, prefix=1, lanes_per_tile=256),           # one pass -> two passes
            # 16 indices per lane: two passes, where the reference gives every
            # exponent class a launch of its own and the no-allocation call
            # (which plans no classes) takes the per-tile dispatch kernel; and
            # chain-serial, run as two chunks of 8 for mixed exponents
            R.config(variant=2, prefix=0, lanes_per_tile=256, per_lane=16, chunks_per_wave=2),
            R.config(variant=2, prefix=2, lanes_per_tile=256, per_lane=16, chunks_per_wave=1)]
    monkeypatch.setenv("RSAPRNG_CLASS_MIN_TILES", "0")
    for ci, cfg in enumerate(cfgs):
        # two calls in a row on one stream, the second smaller, both left in flight
        # before either is read back
        calls = [_requests(rng, len(insts), 40, 300000), _requests(rng, len(insts), 7, 5000)]
        got = []
        for n, (reqs, total) in enumerate(calls):
            log("noalloc cfg %d call %d: %d requests, %d outputs" % (ci, n, len(reqs), total))
            got.append(_run(R, R.rsaprng_pool_generate_noalloc, pool, reqs, total, cfg, stream))
        for n, (reqs, total) in enumerate(calls):
            log("pool_generate cfg %d call %d" % (ci, n))
            ref = _run(R, R.rsaprng_pool_generate, pool, reqs, total, cfg, stream)
            stream.synchronize()
            R.rsaprng_check_device_error(stream)
            c, r = host_u64(got[n][0]), host_f64(got[n][1])
            cref, rref = host_u64(ref[0]), host_f64(ref[1])
            assert_same(c, r, cref, rref, "noalloc vs pool_generate cfg %d call %d" % (ci, n))
            # the ranges hold outputs (not the sentinel), and the gaps kept it
            written = np.zeros(total, dtype=bool)
            for i, k0, cnt, o in reqs:
                written[o:o + cnt] = True
            assert (c[~written] == SENTINEL).all()
            # and a few outputs against the oracle
            for i, k0, cnt, o in reqs[:3]:
                cr, rr = oracle_gen(insts[i], k0, min(cnt, 64))
                assert_same(c[o:o + len(cr)], r[o:o + len(cr)], cr, rr, "oracle cfg %d" % ci)


def test_noalloc_limits(R):
    import torch
    insts = _instances()
    pool = R.Pool.from_instances(insts)
    oc, orr = dev_u64(4), dev_f64(4)
    log("noalloc: too many chains")
    reqs = [(j % len(insts), j * B, 1, 0) for j in range(R.NOALLOC_MAX_CHAINS + 1)]
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_pool_generate_noalloc(pool, reqs, oc, orr)
    assert ei.value.code == R.E_TOO_LARGE
    log("noalloc: tile arrays beyond the scratch")
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_pool_generate_noalloc(pool, [(0, 0, 1 << 31, 0)], oc, orr)
    assert ei.value.code == R.E_TOO_LARGE
    log("noalloc: bad arguments")
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_pool_generate_noalloc(pool, [(len(insts), 0, 10, 0)], oc, orr)
    assert ei.value.code == R.E_ARG
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_pool_generate_noalloc(pool, [(0, 2, (1 << 64) - 1, 0)], oc, orr)
    assert ei.value.code == R.E_RANGE
    # nothing was enqueued by the failed calls, and a good call still works
    log("noalloc: a call after the errors")
    R.rsaprng_pool_generate_noalloc(pool, [(1, 5, 4, 0)], oc, orr)
    torch.cuda.synchronize()
    cr, rr = oracle_gen(insts[1], 5, 4)
    assert_same(host_u64(oc, 4), host_f64(orr, 4), cr, rr, "after errors")
