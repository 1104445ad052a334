"""GPU statistical battery (fused consumer) against the oracle, bit for bit
(frequency, serial, poker, max-of-32, collisions, gaps), and the p-values of a
larger run inside the paper's pass band."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_helpers import log

pytestmark = pytest.mark.gpu

B = 1 << 20


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def _decode(rec):
    import torch
    torch.cuda.synchronize()
    return oracle.battery_decode(rec.cpu().numpy().tobytes())


# the battery always runs the chain-serial kernel; a two-pass request maps onto it
SHAPES = ((256, 8, 2, 2), (256, 8, 4, 2), (512, 8, 2, 2), (256, 8, 4, 0))


def test_battery_matches_oracle(R):
    insts = inputs.config3(3)
    cases = [inputs.Instance(i.p, i.q, e, i.m0) for i in insts for e in (3, 17)]
    T2 = 20 << 14   # a leading-bit collision trial
    ranges = [(0, 5, 70000), (1, B - 4000 + 3, 9000), (2, (1 << 40) + 11, 33333), (3, 0, 4096),
              (4, 7, 1), (5, (1 << 63) + 1, 50000), (0, 3 * B, 5000),
              (4, 2 * B - 3 * (1 << 14) - 5, 6 * (1 << 14) + 10),  # trials on both sides of a re-seeding
              # leading-bit trials: 1 and 2 of a block (0 cut), exactly trial 0, a block's
              # tail into the next block's trial 0
              (1, 5 * B + T2 - 3, 2 * T2 + 10), (2, 7 * B, T2), (3, 9 * B + 3 * T2 - 5, B - 3 * T2 + T2 + 9),
              # adjacent requests are counted one by one: groups across their boundary are not
              (5, 11 * B + 100, 500), (5, 11 * B + 600, 700), (5, 11 * B + 1300, 64 * 3 + 7)]
    ref = oracle.battery([(cases[j], k0, cnt) for j, k0, cnt in ranges])
    pool = R.Pool.from_instances(cases)
    rec = R.battery_tensor()
    for shape in SHAPES:
        log("battery", shape)
        cfg = R.config(variant=2, lanes_per_tile=shape[0], per_lane=shape[1],
                       chunks_per_wave=shape[2], prefix=shape[3])
        R.rsaprng_pool_battery(pool, [(j, k0, cnt, 0) for j, k0, cnt in ranges], rec, cfg=cfg)
        R.rsaprng_check_device_error()
        got = _decode(rec)
        # the output count is the requests' total; the frequency bins prove each was counted
        assert int(got["freq"].sum(dtype=np.uint64)) == int(got["outputs"][0])
        assert int(got["coll_msb"].sum()) == 4
        for name in ref:
            if name == "reserved":
                continue
            assert np.array_equal(got[name], ref[name]), (shape, name)


def test_battery_pvalues_in_band(R):
    insts = inputs.config3(8)
    pool = R.Pool.from_instances(insts)
    rec = R.battery_tensor()
    reqs = [(j, 0, 1 << 24, 0) for j in range(len(insts))]   # 2^27 outputs
    log("battery p-values", len(reqs))
    R.rsaprng_pool_battery(pool, reqs, rec)
    R.rsaprng_check_device_error()
    rep = R.battery_report(rec)
    for name, v in rep.items():
        assert v["samples"] > 0, name
        # the paper's criterion: no p-value below 1e-6 or above 1 - 1e-6
        assert 1e-6 < v["p"] < 1 - 1e-6, (name, v)


def test_battery_persistent_many_chains(R):
    # more chains than resident work-groups (one per CU with the urn bitmap), so
    # work-groups walk several chains and must leave LDS clean between them
    insts = inputs.config3(6)
    ranges = [(j % 6, (j * 37 % 64) * (1 << 15) + (j % 3) * 5, (1 << 15) + 77 * (j % 4))
              for j in range(320)]
    ref = oracle.battery([(insts[j], k0, cnt) for j, k0, cnt in ranges])
    pool = R.Pool.from_instances(insts)
    rec = R.battery_tensor()
    for persistent in (1, 0):
        log("battery persistent", persistent, len(ranges))
        cfg = R.config(variant=2, prefix=2, lanes_per_tile=256, chunks_per_wave=2,
                       persistent=persistent)
        R.rsaprng_pool_battery(pool, [(j, k0, cnt, 0) for j, k0, cnt in ranges], rec, cfg=cfg)
        R.rsaprng_check_device_error()
        got = _decode(rec)
        assert int(got["coll"].sum()) > 0 and int(got["runs"].sum()) > 0
        for name in ref:
            if name == "reserved":
                continue
            assert np.array_equal(got[name], ref[name]), (persistent, name)


def test_battery_of_stored_values(R):
    import torch
    inst = inputs.config3(1)[0]
    # a generated range from index 0: the stored values' battery equals the fused one
    n = B + (20 << 14) + 77    # four leading-bit trials, the last block ragged
    pool = R.Pool.from_instances([inst])
    c = torch.empty(n, dtype=torch.int64, device="cuda")
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    R.rsaprng_pool_generate(pool, [(0, 0, n, 0)], c, r)
    rec_v, rec_f = R.battery_tensor(), R.battery_tensor()
    log("battery of stored values", n)
    R.rsaprng_battery_values(r, rec_v)
    R.rsaprng_pool_battery(pool, [(0, 0, n, 0)], rec_f)
    R.rsaprng_check_device_error()
    got_v, got_f = _decode(rec_v), _decode(rec_f)
    ref = oracle.battery_values(r.cpu().numpy())
    assert int(ref["coll_msb"].sum()) == 4
    for name in ref:
        if name == "reserved":
            continue
        assert np.array_equal(got_v[name], ref[name]), name
        assert np.array_equal(got_f[name], ref[name]), name
    # the flattened vector-mode output: substreams seen interleaved
    g = R.rsaprng_create_ex(inst.p, inst.q, inst.e, inst.m0, 1)
    m = (20 << 14) + 999
    rv = torch.empty(m, dtype=torch.float64, device="cuda")
    R.rsaprng_generate_vector(g, 64, 12345, m, None, rv)
    log("battery of vector-mode values", m)
    R.rsaprng_battery_values(rv, rec_v)
    R.rsaprng_check_device_error()
    got = _decode(rec_v)
    ref = oracle.battery_values(rv.cpu().numpy())
    for name in ref:
        if name == "reserved":
            continue
        assert np.array_equal(got[name], ref[name]), name
    assert int(got["coll"].sum()) == 20 and int(got["coll_msb"].sum()) == 1
    assert int(got["outputs"][0]) == m
