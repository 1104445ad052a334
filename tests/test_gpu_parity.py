"""GPU parity: the HIP path (called through the C ABI) against the CPU oracle.

Every comparison is bit-exact: c_k as integers and r_k as IEEE bit patterns.
Each case logs its name before touching the GPU.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_helpers import (assert_same, dev_f64, dev_u64, host_f64, host_u64, log, oracle_gen,
                               oracle_stats)

pytestmark = pytest.mark.gpu

B = 1 << 20


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1811_11629_amd import rsaprng
    assert torch.cuda.is_available()
    rsaprng.lib()
    return rsaprng


# Every kernel shape the library builds: (lanes, per_lane, chunks_per_wave, prefix),
# prefix 0 two passes, 1 one pass with look-back, 2 chain-serial.
SHAPES = ((256, 8, 1, 0), (256, 8, 2, 0), (256, 8, 4, 0), (512, 8, 2, 0), (256, 16, 2, 0),
          (256, 8, 1, 1), (512, 8, 1, 1), (256, 16, 1, 1), (256, 8, 2, 2), (256, 8, 4, 2),
          (512, 8, 2, 2), (256, 16, 1, 2), (512, 16, 1, 2))


def _variants(R):
    return [(R.VARIANT_MONT, "mont64"), (R.VARIANT_CRT, "crt-fp64")]


def _gen_pool(R, insts, ranges, cfg):
    """Generate through a pool: ranges = [(inst_index, k0, count)] packed back to back."""
    total = sum(c for _, _, c in ranges)
    oc, orr = dev_u64(total), dev_f64(total)
    reqs, off = [], 0
    for i, k0, c in ranges:
        reqs.append((i, k0, c, off))
        off += c
    pool = R.Pool.from_instances(insts)
    R.rsaprng_pool_generate(pool, reqs, oc, orr, cfg=cfg)
    R.rsaprng_check_device_error()
    return host_u64(oc, total), host_f64(orr, total), reqs


def _check_ranges(insts, ranges, c, r, what):
    off = 0
    for i, k0, cnt in ranges:
        cref, rref = oracle_gen(insts[i], k0, cnt)
        assert_same(c[off:off + cnt], r[off:off + cnt], cref, rref, "%s inst %d k0 %d" % (what, i, k0))
        off += cnt


def test_config1_full_block(R):
    inst = inputs.config1()
    log("config1 full block 2^20 via rsaprng_generate", inst)
    g = R.rsaprng_create(inst.p, inst.q, inst.e, inst.m0)
    oc, orr = dev_u64(B), dev_f64(B)
    R.rsaprng_generate(g, 0, B, oc, orr)
    R.rsaprng_check_device_error()
    cref, rref = oracle_gen(inst, 0, B)
    assert_same(host_u64(oc), host_f64(orr), cref, rref, "config1")


@pytest.mark.parametrize("k0,count", [
    (0, 1), (1, 1), (4095, 2), (4096, 4096), (B - 5, 10), (3 * B + 7, 3 * 4096 + 5),
    (B - 4096 * 3 - 1, 4096 * 6 + 3), ((1 << 40) + 123, 10000), ((1 << 40) - 1, 70000),
    ((1 << 64) - 3000, 3000), ((1 << 63) + 12345, 5000),
])
def test_ragged_ranges_both_variants(R, k0, count):
    inst = inputs.config1()
    cref, rref = oracle_gen(inst, k0, count)
    for var, name in _variants(R):
        for shape in SHAPES:
            for prefix in (shape[3],):
                log("ragged", name, shape, "prefix", prefix, k0, count)
                cfg = R.config(variant=var, lanes_per_tile=shape[0], per_lane=shape[1],
                               chunks_per_wave=shape[2], prefix=prefix)
                c, r, _ = _gen_pool(R, [inst], [(0, k0, count)], cfg)
                assert_same(c, r, cref, rref, "%s %s %d k0=%d" % (name, shape, prefix, k0))


def test_edge_moduli_and_cribs(R):
    insts = inputs.edge_instances()
    extra = []
    for i in insts:
        n = i.n
        for m0 in (0, 1, n - 1, n - 2):
            extra.append(inputs.Instance(i.p, i.q, i.e, m0))
    allv = insts + extra
    ranges = [(j, k0, 5000) for j in range(len(allv)) for k0 in (0, 7 * B - 100)]
    for var, name in _variants(R):
        log("edge moduli / cribs", name)
        c, r, _ = _gen_pool(R, allv, ranges, R.config(variant=var))
        _check_ranges(allv, ranges, c, r, "edge " + name)
        # the cribs m0 = 0, 1, n - 1 encrypt to themselves at k = 0 (Pseudorandom skips)
        for j, i in enumerate(allv):
            if i.m0 in (0, 1, i.n - 1):
                assert int(c[2 * j * 5000]) == i.m0


def test_every_exponent(R, monkeypatch):
    base = inputs.config3(2)
    es = [1, 3, 5, 7, 17, 257, 65537, 9, 11, 13, 101, 2 ** 31 + 11]
    insts = []
    for b in base:
        for e in es:
            lam = (b.p - 1) * (b.q - 1) // math.gcd(b.p - 1, b.q - 1)
            if math.gcd(e, lam) == 1:
                insts.append(inputs.Instance(b.p, b.q, e, b.m0))
    ranges = [(j, k0, 3000) for j in range(len(insts)) for k0 in (0, 5 * B + 17)]
    for var, name in _variants(R):
        log("every exponent", name, len(insts))
        c, r, _ = _gen_pool(R, insts, ranges, R.config(variant=var))
        _check_ranges(insts, ranges, c, r, "exponents " + name)
    # two passes with 16 indices per lane: one launch per exponent class (the
    # unrolled ladders, then every other exponent in one class; the library
    # gives small classes no launch of their own unless told to), or all in
    # the per-tile dispatch kernel; ranges packed so that about half start at
    # odd output elements
    odd = [(j, k0, 3001 + 2 * j) for j in range(len(insts)) for k0 in (7, 2 * B - 4000)]
    cfg16 = R.config(variant=R.VARIANT_CRT, lanes_per_tile=256, per_lane=16, chunks_per_wave=2,
                     prefix=0)
    for min_tiles in ("0", "16384"):
        monkeypatch.setenv("RSAPRNG_CLASS_MIN_TILES", min_tiles)
        log("every exponent, exponent classes of at least", min_tiles, "tiles", len(insts))
        c, r, _ = _gen_pool(R, insts, odd, cfg16)
        _check_ranges(insts, odd, c, r, "exponent classes, min %s" % min_tiles)


def test_exponent_one_is_message(R):
    inst = inputs.config1()
    i1 = inputs.Instance(inst.p, inst.q, 1, inst.m0)
    log("e = 1")
    c, r, _ = _gen_pool(R, [i1], [(0, 0, 20000), (0, 3 * B - 5000, 10000)], R.config())
    m = np.concatenate([oracle.messages(i1.p, i1.q, i1.m0, 1, 0, 20000),
                        oracle.messages(i1.p, i1.q, i1.m0, 1, 3 * B - 5000, 10000)])
    assert np.array_equal(c, m)


def test_generate_batch_handles(R):
    insts = inputs.config2(6) + inputs.edge_instances()
    gens = [R.rsaprng_create_ex(i.p, i.q, i.e, i.m0, 1) for i in insts]
    ranges = [(j, (j * 7919 * 4096 + j * 13) % (1 << 36), 4096 * (j % 3) + 777 * j + 1)
              for j in range(len(insts))]
    total = sum(c for _, _, c in ranges)
    oc, orr = dev_u64(total), dev_f64(total)
    reqs, off = [], 0
    for j, k0, cnt in ranges:
        reqs.append((gens[j], k0, cnt, off))
        off += cnt
    log("rsaprng_generate_batch", len(reqs))
    R.rsaprng_generate_batch(reqs, oc, orr)
    R.rsaprng_check_device_error()
    _check_ranges(insts, ranges, host_u64(oc, total), host_f64(orr, total), "generate_batch")


def test_substreams_config2_subset_all_shapes(R):
    # 8 instances of the multi-instance workload, each split into 256 substreams of
    # 4096 starting at k0 = j 2^12; every kernel configuration must give the oracle's bytes.
    insts = inputs.config2(8)
    ranges = [(i, j * 4096, 4096) for i in range(len(insts)) for j in range(256)]
    refs = [oracle_gen(i, 0, B) for i in insts]
    cref = np.concatenate([x[0] for x in refs])
    rref = np.concatenate([x[1] for x in refs])
    from paper_1811_11629_amd import rsaprng
    for var in (R.VARIANT_MONT, R.VARIANT_CRT):
        for shape in SHAPES:
            for pers in (0, 1):
                for prefix in (shape[3],):
                    log("config2 subset", var, shape, pers, prefix)
                    cfg = R.config(variant=var, lanes_per_tile=shape[0], per_lane=shape[1],
                                   chunks_per_wave=shape[2], persistent=pers, order=pers,
                                   prefix=prefix)
                    c, r, _ = _gen_pool(R, insts, ranges, cfg)
                    assert_same(c, r, cref, rref, "config2 %s %s %s %s" % (var, shape, pers, prefix))


def test_odd_output_offsets_every_shape(R):
    # Ranges packed back to back after ranges of odd length start at odd
    # elements of the output arrays: full chunks there take the fast path's
    # 8-byte stores (store_chunk), on every shape of both variants.
    insts = inputs.config2(4)
    ranges = [(0, 0, 1), (1, 4096, 3 * 8192 + 1), (2, B - 8192 * 2, 8192 * 5), (3, 77, 40001),
              (0, 5 * B + 3, 2 * 8192 + 511)]
    offs, o = [], 0
    for _, _, cnt in ranges:
        offs.append(o)
        o += cnt
    assert any(x % 2 for x in offs)
    for var, name in _variants(R):
        for shape in SHAPES:
            log("odd offsets", name, shape)
            cfg = R.config(variant=var, lanes_per_tile=shape[0], per_lane=shape[1],
                           chunks_per_wave=shape[2], prefix=shape[3])
            c, r, _ = _gen_pool(R, insts, ranges, cfg)
            _check_ranges(insts, ranges, c, r, "odd offsets %s %s" % (name, shape))


def test_exponent_specialised_chain_serial(R):
    # Launches whose instances all have e = 3 take the chain-serial kernels
    # specialised to that exponent (skips kept for the output pass); ragged
    # ranges put partial chunks and partial steps at both ends of each chain.
    # A pool that mixes e = 3 and e = 5 takes the per-chain exponent paths (16
    # indices per lane: two chunks of 8, the same tile).
    insts3 = inputs.config2(6)
    ranges = [(0, 0, B), (1, 17, 5000), (2, B - 777, 4096 + 1000), (3, 3 * B + 8191, 8193),
              (4, 12345, 2 * 8192 + 64 * 8 + 3), (5, (1 << 40) + 5, 70001)]
    # the exponent-sweep instances are valid for e = 5
    mixed = insts3[:3] + [inputs.Instance(i.p, i.q, 5, i.m0) for i in inputs.config3(3)]
    for shape in ((256, 8, 2), (512, 8, 2), (256, 16, 1), (512, 16, 1)):
        for pers in (0, 1):
            cfg = R.config(variant=R.VARIANT_CRT, lanes_per_tile=shape[0], per_lane=shape[1],
                           chunks_per_wave=shape[2], persistent=pers, order=pers, prefix=2)
            log("e=3 specialised", shape, pers)
            c, r, _ = _gen_pool(R, insts3, ranges, cfg)
            _check_ranges(insts3, ranges, c, r, "e=3 specialised %s %d" % (shape, pers))
            log("mixed exponents", shape, pers)
            c, r, _ = _gen_pool(R, mixed, ranges, cfg)
            _check_ranges(mixed, ranges, c, r, "mixed %s %d" % (shape, pers))


def test_unreduced_lazy_skips_every_shape(R):
    # Skip values the kernels' lazy steps leave unreduced (v + Q for a small v),
    # or reduced with the upper word of Q, inside requested ranges and inside
    # the lead-in before them, at several positions of a lane's run: the exact
    # redo of those walks must give the oracle's bytes, in every shape of both
    # variants, on a pool of e = 3 (the specialised chain-serial kernels) and on
    # one of mixed exponents (the per-chain paths and the general kernels).
    from tests import lazy_skip_cases as LC
    pools = [("e=3", LC.instances((3,))), ("mixed", LC.instances((3, 5, 17, 257, 65537)))]
    for what, (insts, cases) in pools:
        ranges = LC.ranges_for(cases)
        refs = [oracle_gen(insts[i], k0, cnt) for i, k0, cnt in ranges]
        cref = np.concatenate([x[0] for x in refs])
        rref = np.concatenate([x[1] for x in refs])
        for var, name in _variants(R):
            for shape in SHAPES:
                for pers in (0, 1):
                    log("unreduced skips", what, name, shape, pers)
                    cfg = R.config(variant=var, lanes_per_tile=shape[0], per_lane=shape[1],
                                   chunks_per_wave=shape[2], prefix=shape[3], persistent=pers,
                                   order=pers)
                    c, r, _ = _gen_pool(R, insts, ranges, cfg)
                    assert_same(c, r, cref, rref,
                                "unreduced skips %s %s %s %d" % (what, name, shape, pers))
        st_refs = [oracle_stats(insts[i], k0, cnt) for i, k0, cnt in ranges]
        pool = R.Pool.from_instances(insts)
        for var, name in _variants(R):
            for shape in SHAPES:
                log("unreduced skips consume", what, name, shape)
                st = R.stats_tensor(len(ranges))
                cfg = R.config(variant=var, lanes_per_tile=shape[0], per_lane=shape[1],
                               chunks_per_wave=shape[2], prefix=shape[3])
                R.rsaprng_pool_consume(pool, [(i, k0, cnt, idx)
                                              for idx, (i, k0, cnt) in enumerate(ranges)],
                                       st, cfg=cfg)
                R.rsaprng_check_device_error()
                got = R.stats_decode(st)
                for idx, ref in enumerate(st_refs):
                    g = got[idx]
                    assert g["sum_fx"] == ref["sum_fx"], (what, name, shape, idx)
                    assert g["lt_half"] == ref["lt_half"], (what, name, shape, idx)
                    assert np.array_equal(g["hist"], ref["hist"]), (what, name, shape, idx)


def test_consume_matches_oracle(R):
    import torch
    insts = inputs.config3(3)
    cases = []
    for i in insts:
        for e in (3, 17, 65537):
            cases.append(inputs.Instance(i.p, i.q, e, i.m0))
    ranges = [(j, k0, cnt) for j in range(len(cases))
              for k0, cnt in ((0, 1 << 18), (B - 3000, 9000), ((1 << 40) + 5, 4097))]
    pool = R.Pool.from_instances(cases)
    for (var, name), (shape, prefix) in [(v, sp) for v in _variants(R)
                                         for sp in (((256, 8, 4), 0), ((256, 8, 1), 1),
                                                    ((512, 8, 2), 0), ((256, 16, 1), 1),
                                                    ((256, 8, 4), 2), ((512, 8, 2), 2),
                                                    ((256, 8, 2), 2))]:
        log("consume", name, shape, prefix)
        st = R.stats_tensor(len(ranges))
        R.rsaprng_pool_consume(pool, [(j, k0, cnt, idx) for idx, (j, k0, cnt) in enumerate(ranges)],
                               st, cfg=R.config(variant=var, lanes_per_tile=shape[0],
                                                per_lane=shape[1], chunks_per_wave=shape[2],
                                                prefix=prefix))
        R.rsaprng_check_device_error()
        got = R.stats_decode(st)
        for idx, (j, k0, cnt) in enumerate(ranges):
            ref = oracle_stats(cases[j], k0, cnt)
            g = got[idx]
            assert g["count"] == cnt
            assert g["sum_fx"] == ref["sum_fx"], (name, idx)
            assert g["lt_half"] == ref["lt_half"]
            assert np.array_equal(g["hist"], ref["hist"])
            # the double is the exact sum rounded once (Fraction -> float rounds correctly)
            assert g["sum"] == float(Fraction(ref["sum_fx"], 1 << 128))


def test_consume_one_exponent_sixteen_per_lane(R):
    # Consume launches whose instances share one exponent take chain-serial
    # kernels specialised to it with 16 indices per lane: each unrolled
    # exponent, ragged ranges (lead-in, block crossing, partial chunks at both
    # ends), persistent and not, record by record against the oracle.
    base = inputs.config3(4)
    sevens = [i for i in inputs.config4(200)[0] if i.e == 7][:4]
    pools = [(e, [inputs.Instance(b.p, b.q, e, b.m0) for b in base])
             for e in (3, 5, 17, 257, 65537)] + [(7, sevens)]
    for e, insts in pools:
        ranges = [(j, k0, cnt) for j in range(len(insts))
                  for k0, cnt in ((0, 1 << 16), (B - 2500, 7000), ((1 << 40) + 3 * j + 1, 5000 + 17 * j))]
        refs = [oracle_stats(insts[j], k0, cnt) for j, k0, cnt in ranges]
        pool = R.Pool.from_instances(insts)
        for pers in (0, 1):
            log("consume one exponent, 16 per lane", e, pers)
            st = R.stats_tensor(len(ranges))
            cfg = R.config(variant=R.VARIANT_CRT, lanes_per_tile=256, per_lane=16, chunks_per_wave=1,
                           prefix=2, persistent=pers, order=pers)
            R.rsaprng_pool_consume(pool, [(j, k0, cnt, idx) for idx, (j, k0, cnt) in enumerate(ranges)],
                                   st, cfg=cfg)
            R.rsaprng_check_device_error()
            got = R.stats_decode(st)
            for idx, ref in enumerate(refs):
                g = got[idx]
                assert g["count"] == ranges[idx][2], (e, pers, idx)
                assert g["sum_fx"] == ref["sum_fx"], (e, pers, idx)
                assert g["lt_half"] == ref["lt_half"], (e, pers, idx)
                assert np.array_equal(g["hist"], ref["hist"]), (e, pers, idx)


def test_consume_persistent_many_chains(R):
    # one work-group per compute unit walks tiles of many chains in turn: each
    # tile's statistics must land in its own record, in every shape and variant
    insts = inputs.config3(24)
    ranges = []
    for j in range(len(insts)):
        ranges.append((j, (j * 7919) % B, 3 * 4096 + 17 * j))
        ranges.append((j, (1 << 33) + j * 12345, 2 * B // 3))
    refs = [oracle_stats(insts[j], k0, cnt) for j, k0, cnt in ranges]
    pool = R.Pool.from_instances(insts)
    for var, name in _variants(R):
        for shape, prefix in [((sh[0], sh[1], sh[2]), sh[3]) for sh in SHAPES]:
            log("consume persistent", name, shape, prefix)
            st = R.stats_tensor(len(ranges))
            cfg = R.config(variant=var, lanes_per_tile=shape[0], per_lane=shape[1],
                           chunks_per_wave=shape[2], prefix=prefix, persistent=1, wg_per_cu=1,
                           order=1)
            R.rsaprng_pool_consume(pool, [(j, k0, cnt, idx)
                                          for idx, (j, k0, cnt) in enumerate(ranges)], st, cfg=cfg)
            R.rsaprng_check_device_error()
            got = R.stats_decode(st)
            for idx, ref in enumerate(refs):
                g = got[idx]
                assert g["count"] == ranges[idx][2], (name, shape, idx)
                assert g["sum_fx"] == ref["sum_fx"], (name, shape, idx)
                assert g["lt_half"] == ref["lt_half"], (name, shape, idx)
                assert np.array_equal(g["hist"], ref["hist"]), (name, shape, idx)


def test_consume_single_handle(R):
    inst = inputs.config1()
    g = R.rsaprng_create(inst.p, inst.q, inst.e, inst.m0)
    st = R.stats_tensor(1)
    log("rsaprng_consume single")
    R.rsaprng_consume(g, 12345, 300000, st)
    R.rsaprng_check_device_error()
    got = R.stats_decode(st)[0]
    ref = oracle_stats(inst, 12345, 300000)
    assert got["sum_fx"] == ref["sum_fx"] and np.array_equal(got["hist"], ref["hist"])
    assert got["lt_half"] == ref["lt_half"] and got["count"] == 300000


def test_graph_batch_replays(R):
    import torch
    insts = inputs.config2(4)
    ranges = [(i, k0, 50000) for i in range(4) for k0 in (0, 2 * B + 33)]
    total = sum(c for _, _, c in ranges)
    pool = R.Pool.from_instances(insts)
    reqs, off = [], 0
    for i, k0, c in ranges:
        reqs.append((i, k0, c, off))
        off += c
    oc, orr = dev_u64(total), dev_f64(total)
    for var, prefix in ((R.VARIANT_MONT, 0), (R.VARIANT_CRT, 1), (R.VARIANT_CRT, 0),
                        (R.VARIANT_CRT, 2), (R.VARIANT_MONT, 2)):
        log("graph batch", var, prefix)
        b = R.Batch(pool, reqs, R.MODE_GENERATE, oc, orr,
                    cfg=R.config(variant=var, persistent=1, prefix=prefix))
        for rep in range(3):
            oc.fill_(-1)
            orr.fill_(-1.0)
            torch.cuda.synchronize()
            b.run()
            torch.cuda.synchronize()
            b.check()
            _check_ranges(insts, ranges, host_u64(oc, total), host_f64(orr, total),
                          "graph replay %d" % rep)
            x = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
            assert math.isfinite(x)
        # the timed (eager) form of the same launch writes the same outputs
        oc.fill_(-1)
        orr.fill_(-1.0)
        torch.cuda.synchronize()
        b.run_timed()
        b.run_timed()
        kt = b.kernel_ms()
        b.check()
        assert kt["runs"] == 2 and kt["tiles"] > 0 and kt["setup"] > 0 and kt["finalize"] >= 0
        _check_ranges(insts, ranges, host_u64(oc, total), host_f64(orr, total), "timed run")
        assert b.kernel_ms()["runs"] == 0


def test_debug_encrypt_bijection(R):
    import torch
    for bits in (12, 13):
        for inst in inputs.small_instances(500 + bits, 2, bits=bits):
            n = inst.n
            m = torch.arange(n, dtype=torch.int64, device="cuda")
            for var, name in _variants(R):
                log("bijection", bits, name, n)
                c = torch.empty_like(m)
                R.rsaprng_debug_encrypt(inst.p, inst.q, inst.e, var, m, c)
                torch.cuda.synchronize()
                srt, _ = torch.sort(c)
                assert torch.equal(srt, m)
                sample = np.arange(0, n, max(1, n // 5000), dtype=np.uint64)
                ref = oracle.encrypt_array(n, inst.e, sample)
                got = c.cpu().numpy().view(np.uint64)[sample.astype(np.int64)]
                assert np.array_equal(got, ref)


def test_errors(R):
    import torch
    inst = inputs.config1()
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_create(inst.p, inst.p, 3, 1)
    assert ei.value.code == -2
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_create(inst.p, inst.q, 2, 1)
    assert ei.value.code == -4
    g = R.rsaprng_create(inst.p, inst.q, inst.e, 5)
    buf = torch.empty(1000, dtype=torch.int64, device="cuda")
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_generate(g, 0, 10, buf.data_ptr() + 4, None)
    assert ei.value.code == -8
    with pytest.raises(R.RsaprngError) as ei:
        R.rsaprng_generate(g, (1 << 64) - 5, 10, buf, None)
    assert ei.value.code == -6
    R.rsaprng_generate(g, 0, 0, buf, None)   # no-op
    torch.cuda.synchronize()
