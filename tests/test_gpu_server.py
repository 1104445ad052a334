"""GPU tests of the served form: every request served in a mix equals the
oracle bit for bit and equals the same request served alone; continuation
across iterations (saved chain state) is exercised by small chunks, and
admission by a small arena."""
import time

import numpy as np
import pytest

import inputs
from gpu_helpers import assert_same, log, oracle_gen

pytestmark = pytest.mark.gpu

T = 4096
BLOCK = 1 << 20


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


@pytest.fixture(scope="module")
def pool_insts():
    insts, _ = inputs.config5_instances(48)
    return insts


def make_requests(n, seed, n_inst, max_log2=17):
    rng = inputs.SplitMix64(seed)
    reqs = []
    for i in range(n):
        inst = rng.next() % n_inst
        k0 = rng.next() >> 24
        cnt = 1 + int(2.0 ** (max_log2 * rng.unit53()))
        if i % 9 == 0:
            k0 = (k0 | (BLOCK - 1)) - (rng.next() % 3000)     # crosses a block end
        if i % 13 == 0:
            k0 &= ~(BLOCK - 1)                                 # starts at a block start
        if i % 17 == 0:
            cnt = BLOCK - (k0 % BLOCK)                         # ends at a block end
        reqs.append((inst, k0, cnt))
    return reqs


def serve(R, server, reqs, tag0=0, deadline_s=90.0):
    """Submit all requests, wait for all completions; returns {index: (c, r)}."""
    for i, (inst, k0, cnt) in enumerate(reqs):
        rc = server.submit(inst, k0, cnt, tag0 + i)
        assert rc == 0, (i, rc)
    out = {}
    t_end = time.time() + deadline_s
    while len(out) < len(reqs):
        assert time.time() < t_end, "server did not finish: %d of %d" % (len(out), len(reqs))
        got = server.poll(256)
        if not got:
            time.sleep(0.001)
        for comp in got:
            i = comp.tag - tag0
            cnt = reqs[i][2]
            assert comp.count == cnt
            assert comp.t_submit <= comp.t_admit <= comp.t_done
            c = np.zeros(cnt, dtype=np.uint64)
            r = np.zeros(cnt, dtype=np.float64)
            server.read(comp.tag, c, r)
            server.release(comp.tag)
            out[i] = (c, r)
    return out


CFGS = {
    "crt-twopass": dict(variant=2),
    "mont-lookback-16": dict(variant=1, lanes_per_tile=256, per_lane=16, prefix=1),
    "crt-512": dict(variant=2, lanes_per_tile=512),
    "crt-serial": dict(variant=2, prefix=2),
    "mont-serial-512": dict(variant=1, lanes_per_tile=512, prefix=2),
    "crt-twopass-shortest-first": dict(variant=2),
    "crt-twopass-16": dict(variant=2, lanes_per_tile=256, per_lane=16, chunks_per_wave=2,
                           prefix=0),
    "crt-twopass-16-exponent-classes": dict(variant=2, lanes_per_tile=256, per_lane=16,
                                            chunks_per_wave=2, prefix=0),
}


@pytest.mark.parametrize("name", list(CFGS))
def test_mix_matches_oracle_and_alone(R, pool_insts, name, monkeypatch):
    # "exponent-classes": every iteration's exponent classes take launches of
    # their own (the default keeps small classes in one per-tile launch)
    monkeypatch.setenv("RSAPRNG_CLASS_MIN_TILES", "0" if "exponent-classes" in name else "16384")
    cfg = R.config(**CFGS[name])
    reqs = make_requests(90, 777 + len(name), len(pool_insts))
    log("server mix", name, "requests", len(reqs), "outputs", sum(r[2] for r in reqs))
    pool = R.Pool.from_instances(pool_insts)
    policy = R.SRV_SHORTEST_FIRST if "shortest-first" in name else R.SRV_ROUND_ROBIN
    srv = R.Server(pool, arena_bytes=16 * (1 << 21), iter_outputs=24 * T,
                   chunk_outputs=3 * T + 123, cfg=cfg, policy=policy)
    try:
        mix = serve(R, srv, reqs)
        st = srv.stats()
        assert st["iterations"] > 20 and st["outputs"] == sum(r[2] for r in reqs)
        for i, (inst, k0, cnt) in enumerate(reqs):
            c_ref, r_ref = oracle_gen(pool_insts[inst], k0, cnt)
            assert_same(mix[i][0], mix[i][1], c_ref, r_ref, "%s mix req %d" % (name, i))
        # the same requests one at a time
        for i in range(0, len(reqs), 6):
            alone = serve(R, srv, [reqs[i]], tag0=10000 + i)
            assert_same(alone[0][0], alone[0][1], mix[i][0], mix[i][1], "alone %d" % i)
    finally:
        srv.close()


def test_late_arrivals_and_replay(R, pool_insts):
    pool = R.Pool.from_instances(pool_insts)
    srv = R.Server(pool, arena_bytes=16 * (1 << 21), iter_outputs=1 << 18, chunk_outputs=1 << 16)
    try:
        reqs = make_requests(40, 4242, len(pool_insts), max_log2=18)
        log("server replay", len(reqs))
        rng = inputs.SplitMix64(99)
        t_arr = inputs.poisson_arrivals(rng, 2000.0, len(reqs))
        inst = np.array([r[0] for r in reqs])
        k0 = np.array([r[1] for r in reqs], dtype=np.uint64)
        cnt = np.array([r[2] for r in reqs], dtype=np.uint64)
        t_admit, t_done = srv.replay(inst, k0, cnt, t_arr)
        assert np.all(t_admit >= t_arr - 1e-6) and np.all(t_done >= t_admit)
        st = srv.stats()
        assert st["waiting"] == 0 and st["active"] == 0
        # the server is still usable and still exact afterwards
        out = serve(R, srv, reqs[:5])
        for i in range(5):
            c_ref, r_ref = oracle_gen(pool_insts[reqs[i][0]], reqs[i][1], reqs[i][2])
            assert_same(out[i][0], out[i][1], c_ref, r_ref, "after replay %d" % i)
    finally:
        srv.close()


def test_server_errors(R, pool_insts):
    pool = R.Pool.from_instances(pool_insts[:4])
    srv = R.Server(pool, arena_bytes=16 * 10000)
    try:
        assert srv.submit(4, 0, 10, 1) == R.E_ARG            # no such instance
        assert srv.submit(0, 0, 0, 1) == R.E_ARG             # empty
        assert srv.submit(0, 0, 10001, 1) == R.E_RANGE       # larger than the arena
        assert srv.submit(0, (1 << 64) - 1, 2, 1) == R.E_RANGE
        with pytest.raises(R.RsaprngError):
            srv.release(12345)
        with pytest.raises(R.RsaprngError):
            srv.read(12345, np.zeros(1, dtype=np.uint64))
        out = serve(R, srv, [(1, (1 << 64) - 700, 700)])
        c_ref, r_ref = oracle_gen(pool_insts[1], (1 << 64) - 700, 700)
        assert_same(out[0][0], out[0][1], c_ref, r_ref, "top of range")
    finally:
        srv.close()

