"""The statistical battery on the host: the chi-squared tail against scipy,
the report on constructed records, and the oracle's counts against a direct
restatement of the grouping rules on a short ragged range."""
import numpy as np
import pytest
import scipy.stats as st

import inputs
import oracle


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def test_chi2_tail_matches_scipy(R):
    for x, k in [(3.0, 3), (10.0, 3), (0.5, 1), (1000.0, 1023), (1100.0, 1023),
                 (1048575.0, 1048575), (1050000.0, 1048575), (999000.0, 999999), (200.0, 50)]:
        assert abs(R.rsaprng_chi2_sf(x, k) - st.chi2.sf(x, k)) < 1e-9 * max(1.0, st.chi2.sf(x, k))


def test_report_on_constructed_records(R):
    rec = np.zeros(R.BATTERY_BYTES, dtype=np.uint8)
    fields = oracle.BATTERY_FIELDS
    offs, off = {}, 0
    for name, n, t in fields:
        offs[name] = (off, n, t)
        off += n * np.dtype(t).itemsize
    view = {name: rec[o:o + n * np.dtype(t).itemsize].view(t) for name, (o, n, t) in offs.items()}
    view["freq"][:] = 7                      # perfectly uniform: chi2 = 0, p = 1
    view["maxt"][:512] = 3                   # half the bins empty
    view["maxt"][512:] = 1
    view["poker"][2:6] = [40, 1000, 5000, 6000]
    out = R.battery_report(rec.tobytes())
    assert out["frequency"]["chi2"] == 0.0 and out["frequency"]["p"] == 1.0
    m = view["maxt"].astype(float)
    e = m.mean()
    assert abs(out["max_of_32"]["chi2"] - ((m - e) ** 2 / e).sum()) < 1e-9
    pr = np.array([16 + 3600, 84000, 436800, 524160]) / 16.0 ** 5
    o = np.array([40, 1000, 5000, 6000], dtype=float)
    x = ((o - o.sum() * pr) ** 2 / (o.sum() * pr)).sum()
    assert abs(out["poker"]["chi2"] - x) < 1e-9 and out["poker"]["dof"] == 3
    assert abs(out["poker"]["p"] - st.chi2.sf(x, 3)) < 1e-12


def _bin(r, b):
    return min(int(r * b), b - 1)


def test_oracle_battery_matches_definition():
    inst = inputs.config1()
    k0, count = (1 << 20) - 1000 + 3, 3000      # unaligned, crosses a block re-seeding
    _, r = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count)
    got = oracle.battery([(inst, k0, count)])
    freq = np.zeros(1 << 20, dtype=np.uint64)
    for v in r:
        freq[_bin(v, 1 << 20)] += 1
    assert np.array_equal(got["freq"], freq) and int(got["outputs"][0]) == count
    last = k0 + count - 1
    s2, poker, maxt = {}, np.zeros(8, dtype=int), {}
    for k8 in range((k0 + 7) // 8 * 8, last - 6, 8):
        x = r[k8 - k0:k8 - k0 + 8]
        for t in range(4):
            c = _bin(x[2 * t], 1024) * 1024 + _bin(x[2 * t + 1], 1024)
            s2[c] = s2.get(c, 0) + 1
        poker[len({_bin(v, 16) for v in x[:5]})] += 1
    for k32 in range((k0 + 31) // 32 * 32, last - 30, 32):
        t = float(max(r[k32 - k0:k32 - k0 + 32]))
        for _ in range(5):
            t = t * t                           # M^32 by five squarings, as defined
        c = _bin(t, 1024)
        maxt[c] = maxt.get(c, 0) + 1
    assert {int(i): int(v) for i, v in enumerate(got["serial2"]) if v} == s2
    assert np.array_equal(got["poker"], poker)
    assert {int(i): int(v) for i, v in enumerate(got["maxt"]) if v} == maxt


# The serial test in D dimensions (Tests section, D = 2 .. 6): tuples of D
# consecutive outputs inside each aligned block of 8 indices, at offsets
# 0, D, 2D, ... while the tuple fits in the block, with b bins per coordinate;
# a cell is the tuple's mixed-radix number, first index most significant.
SERIAL = {2: 1024, 3: 100, 4: 32, 5: 16, 6: 10}


def _serial_cells(x, d, b):
    cells = []
    for off in range(0, 8 - d + 1, d):
        cell = 0
        for v in x[off:off + d]:
            cell = cell * b + _bin(v, b)
        cells.append(cell)
    return cells


def test_serial_tables_match_definition():
    inst = inputs.config1()
    # ragged at both ends (not 8-aligned), crossing the re-seeding at 2^20
    k0, count = (1 << 20) - 4093, 8190
    _, r = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count)
    got = oracle.battery([(inst, k0, count)])
    last = k0 + count - 1
    want = {d: {} for d in SERIAL}
    blocks = 0
    for k8 in range(-(-k0 // 8) * 8, last - 6, 8):
        x = [float(v) for v in r[k8 - k0:k8 - k0 + 8]]
        blocks += 1
        for d, b in SERIAL.items():
            for c in _serial_cells(x, d, b):
                want[d][c] = want[d].get(c, 0) + 1
    assert blocks == (last + 1) // 8 - -(-k0 // 8)
    for d, b in SERIAL.items():
        tab = got["serial%d" % d]
        assert tab.size >= b ** d
        have = {int(i): int(v) for i, v in zip(np.nonzero(tab)[0], tab[np.nonzero(tab)[0]])}
        assert have == want[d], "serial D=%d" % d
        assert sum(have.values()) == blocks * (8 // d)


def test_serial_cell_order_detects_transposition():
    # the restatement must tell a first-index-most-significant cell from its
    # reverse and from a wrong radix, so a consistent misreading of either
    # in the oracle fails the test above
    x = [0.015, 0.34, 0.72, 0.5, 0.99, 0.001, 0.25, 0.6]
    assert _serial_cells(x, 3, 100) == [1 * 10000 + 34 * 100 + 72, 50 * 10000 + 99 * 100 + 0]
    assert _serial_cells(x, 6, 10) == [((((0 * 10 + 3) * 10 + 7) * 10 + 5) * 10 + 9) * 10 + 0]
    assert _serial_cells(x, 5, 16) == [((((0 * 16 + 5) * 16 + 11) * 16 + 8) * 16 + 15)]
    assert _serial_cells(x, 4, 32) == [(((0 * 32 + 10) * 32 + 23) * 32 + 16),
                                       (((31 * 32 + 0) * 32 + 8) * 32 + 19)]


def test_oracle_collisions_and_gaps_match_definition():
    inst = inputs.config1()
    k0, count = (1 << 14) * 3 - 777, (1 << 14) * 3 + 1000   # three whole trials, ragged ends
    _, r = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count)
    got = oracle.battery([(inst, k0, count)])
    last = k0 + count - 1
    coll = np.zeros(256, dtype=int)
    for kt in range((k0 + (1 << 14) - 1) >> 14 << 14, last - (1 << 14) + 2, 1 << 14):
        urns = {_bin(v, 1 << 20) for v in r[kt - k0:kt - k0 + (1 << 14)]}
        coll[min((1 << 14) - len(urns), 255)] += 1
    assert coll.sum() == 3 and np.array_equal(got["coll"], coll)
    runs = np.zeros(128, dtype=int)
    for k64 in range((k0 + 63) // 64 * 64, last - 62, 64):
        bits = [v > 0.5 for v in r[k64 - k0:k64 - k0 + 64]]
        n = 1
        while n < 64 and bits[n] == bits[0]:
            n += 1
        runs[int(bits[0]) * 64 + n - 1] += 1
    assert np.array_equal(got["runs"], runs)


def _collision_distribution(n=1 << 14, m=1 << 20, cmax=600):
    # distribution of the number of collisions, one ball at a time (numpy, float64)
    b = np.zeros(cmax + 2)
    b[0] = 1.0
    for t in range(n):
        c = np.arange(cmax + 1)
        stay = b[:cmax + 1] * (1.0 - np.maximum(t - c, 0) / m)
        move = np.zeros(cmax + 1)
        move[1:] = b[:cmax] * ((t - c[:-1]) / m).clip(min=0)
        b[:cmax + 1] = stay + move
    return b[:cmax + 1]


def test_collision_distribution_and_report(R):
    dist = _collision_distribution()
    n, m = 1 << 14, 1 << 20
    # closed form of the mean: n - m (1 - (1 - 1/m)^n)
    mean_exact = n - m * (1.0 - (1.0 - 1.0 / m) ** n)
    assert abs(dist.sum() - 1.0) < 1e-12
    assert abs((dist * np.arange(dist.size)).sum() - mean_exact) < 1e-6
    # a record whose collision counts follow the distribution closely: p far from 0
    rec = np.zeros(R.BATTERY_BYTES, dtype=np.uint8)
    offs, off = {}, 0
    for name, k, t in oracle.BATTERY_FIELDS:
        offs[name] = (off, k, t)
        off += k * np.dtype(t).itemsize
    view = {name: rec[o:o + k * np.dtype(t).itemsize].view(t) for name, (o, k, t) in offs.items()}
    trials = 1 << 20
    expect = np.concatenate([dist[:255], [dist[255:].sum()]]) * trials
    view["coll"][:] = np.rint(expect).astype(np.uint32)
    out = R.battery_report(rec.tobytes())
    assert out["collisions"]["samples"] == int(view["coll"].sum())
    assert out["collisions"]["p"] > 0.99 and out["collisions"]["dof"] > 20
    # shifting every count by one class is detected
    view["coll"][:] = np.rint(np.concatenate([[0], expect[:-1]])).astype(np.uint32)
    assert R.battery_report(rec.tobytes())["collisions"]["p"] < 1e-6
    # the leading-bit collision test takes the same distribution
    view["coll_msb"][:] = np.rint(expect).astype(np.uint32)
    out = R.battery_report(rec.tobytes())
    assert out["collisions_msb"]["samples"] == int(view["coll_msb"].sum())
    assert out["collisions_msb"]["p"] > 0.99 and out["collisions_msb"]["dof"] > 20
    view["coll_msb"][:] = 0
    # gaps: counts at their expectations give p near 1; too many short runs do not
    view["coll"][:] = 0
    g = np.array([2.0 ** -(L + 1) if L < 64 else 2.0 ** -64 for L in range(1, 65)]) * (1 << 24)
    view["runs"][:64] = np.rint(g).astype(np.uint32)
    view["runs"][64:] = np.rint(g).astype(np.uint32)
    assert R.battery_report(rec.tobytes())["gaps"]["p"] > 0.99
    view["runs"][0] += 100000
    assert R.battery_report(rec.tobytes())["gaps"]["p"] < 1e-6


MSB_BALL, MSB_TRIAL, BLOCK = 20, 20 << 14, 1 << 20


def _msb_trial_c(vals):
    """C for one trial of the leading-bit collision test: 2^14 balls of 20
    values, the urn the 20 leading bits (value j of the ball -> bit j)."""
    bits = (np.asarray(vals) >= 0.5).astype(np.int64).reshape(1 << 14, MSB_BALL)
    urns = bits @ (1 << np.arange(MSB_BALL, dtype=np.int64))
    return (1 << 14) - np.unique(urns).size


def test_oracle_collisions_msb_match_definition():
    # trials 1 and 2 of block 3 (trial 0 cut by k0), then past the block's tail
    # into block 4, whose trial 0 is whole
    inst = inputs.config1()
    k0 = 3 * BLOCK + MSB_TRIAL - 5
    count = 4 * BLOCK + MSB_TRIAL + 7 - k0
    _, r = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, count)
    got = oracle.battery([(inst, k0, count)])
    want = np.zeros(256, dtype=int)
    for ts in (3 * BLOCK + MSB_TRIAL, 3 * BLOCK + 2 * MSB_TRIAL, 4 * BLOCK):
        c = _msb_trial_c(r[ts - k0:ts - k0 + MSB_TRIAL])
        want[min(c, 255)] += 1
    assert want.sum() == 3 and np.array_equal(got["coll_msb"], want)


def _balls_to_values(urns):
    # values whose leading bits spell the given urns (0.25 for a 0 bit, 0.75 for a 1)
    u = np.asarray(urns, dtype=np.int64)
    bits = (u[:, None] >> np.arange(MSB_BALL)) & 1
    return np.where(bits.reshape(-1) == 1, 0.75, 0.25)


def test_oracle_collisions_msb_closed_forms():
    g = np.arange(1 << 14)
    # every ball in urn 0: 2^14 - 1 collisions (class 255)
    got = oracle.battery_values(np.full(MSB_TRIAL, 0.25), 0)
    assert got["coll_msb"][255] == 1 and got["coll_msb"].sum() == 1
    # ball g in urn g: no collision
    got = oracle.battery_values(_balls_to_values(g), 0)
    assert got["coll_msb"][0] == 1 and got["coll_msb"].sum() == 1
    # the last 100 balls repeat urn 7: 100 collisions; the same values placed as
    # trial 2 of block 5 count too, as trial 3 (the block's tail) they do not
    urns = np.where(g < (1 << 14) - 100, g, 7)
    vals = _balls_to_values(urns)
    for k0, n in ((0, 1), (5 * BLOCK + 2 * MSB_TRIAL, 1), (3 * MSB_TRIAL, 0), (1, 0)):
        got = oracle.battery_values(vals, k0)
        assert got["coll_msb"][100] == n and got["coll_msb"].sum() == n, k0
    # a value of exactly 1/2 has leading bit 1
    v = _balls_to_values(g)
    v[v == 0.75] = 0.5
    assert oracle.battery_values(v, 0)["coll_msb"][0] == 1
