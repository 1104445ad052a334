"""Host-only tests of the served form's scheduler (the same code the server's
request loop runs), through rsaprng_server_simulate: every request is covered
exactly once by its chunks, chunk boundaries and continuation flags are the
ones the kernels' saved-state protocol needs, admission respects the arena and
requests arriving later join a running batch."""
import numpy as np
import pytest

import inputs

BLOCK = 1 << 20
T = 4096          # tile of the default configuration: 256 lanes x 8 per lane x 2 chunks
CONT, WEND = 1, 2


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def by_request(log, n):
    out = [[] for _ in range(n)]
    for row in log:
        out[int(row[0])].append(tuple(int(x) for x in row))
    return out


def check_schedule(log, k0, count, arrive, arena, iter_outputs, chunk_outputs, hold):
    n = len(k0)
    reqs = by_request(log, n)
    per_iter = {}
    life = []
    for i, ch in enumerate(reqs):
        assert ch, "request %d never scheduled" % i
        its = [c[1] for c in ch]
        assert its == sorted(its) and len(set(its)) == len(its), "one chunk per iteration"
        assert its[0] >= arrive[i]
        off0 = ch[0][4]
        slot = ch[0][6]
        assert off0 + count[i] <= arena
        pos = k0[i]
        end = (k0[i] + count[i])  # may be 2^64
        for j, (_, it, ck0, cn, coff, fl, sl) in enumerate(ch):
            assert ck0 == pos and cn > 0 and cn <= chunk_outputs
            assert coff == off0 + (ck0 - k0[i]) and sl == slot
            last = j == len(ch) - 1
            cend = ck0 + cn
            if not last:
                assert cend % T == 0, "non-final chunk must end on a tile boundary"
            assert bool(fl & CONT) == (ck0 != k0[i] and ck0 % BLOCK != 0)
            assert bool(fl & WEND) == (not last and cend % BLOCK != 0)
            if fl & CONT:
                assert ch[j - 1][5] & WEND and ch[j - 1][1] < it
            per_iter[it] = per_iter.get(it, 0) + cn
            pos = cend
        assert pos == end
        life.append((its[0], its[-1] + 1 + hold, off0, off0 + count[i], slot))
    assert max(per_iter.values()) <= iter_outputs
    # requests alive at the same time hold disjoint arena ranges and slots
    life_sorted = sorted(range(n), key=lambda i: life[i][0])
    for a_i, a in enumerate(life_sorted):
        for b in life_sorted[a_i + 1:]:
            if life[b][0] >= life[a][1]:
                continue
            A, B = life[a], life[b]
            assert A[3] <= B[2] or B[3] <= A[2], (a, b)
            assert A[4] != B[4], (a, b)
    return reqs


def test_random_trace(R):
    rng = inputs.SplitMix64(20240611)
    n = 300
    k0 = [rng.next() >> 24 for _ in range(n)]
    for i in range(0, n, 7):  # some just before a block end
        k0[i] = (k0[i] | (BLOCK - 1)) - (rng.next() % 5000)
    count = [1 + int(2.0 ** (16 * rng.unit53())) for _ in range(n)]
    arrive = np.cumsum([rng.next() % 3 for _ in range(n)]).tolist()
    arena, iter_o, chunk_o, hold = 1 << 19, 10 * T, 3 * T + 123, 2
    log = R.server_simulate(k0, count, arrive, arena, iter_o, chunk_o, hold)
    reqs = check_schedule(log, k0, count, arrive, arena, iter_o, chunk_o, hold)
    assert sum(len(c) for c in reqs) > n + 100  # many requests span several chunks
    assert any(r[5] & CONT for r in log) and any(r[5] & WEND for r in log)


def test_top_of_index_range(R):
    k0 = [(1 << 64) - 5000, (1 << 64) - 1, (1 << 64) - BLOCK - 77]
    count = [5000, 1, BLOCK + 77]
    arrive = [0, 0, 0]
    log = R.server_simulate(k0, count, arrive, 1 << 22, 8 * T, 2 * T)
    check_schedule(log, k0, count, arrive, 1 << 22, 8 * T, 2 * T, 0)


def test_late_arrival_joins_running_batch(R):
    # a long request is running; a short one arriving at iteration 3 runs in the
    # same launches and finishes long before it
    k0 = [12345, 999]
    count = [50 * 4 * T, 2 * T]
    arrive = [0, 3]
    log = R.server_simulate(k0, count, arrive, 1 << 24, 8 * T, 4 * T)
    reqs = by_request(log, 2)
    assert reqs[1][0][1] == 3
    assert reqs[1][-1][1] < reqs[0][-1][1]
    shared = {c[1] for c in reqs[0]} & {c[1] for c in reqs[1]}
    assert 3 in shared


def test_admission_waits_for_arena(R):
    cnt = 10 * T
    k0 = [0, BLOCK, 2 * BLOCK]
    count = [cnt, cnt, cnt]
    arrive = [0, 0, 0]
    hold = 4
    arena = 2 * cnt + T  # room for two
    log = R.server_simulate(k0, count, arrive, arena, 64 * T, 2 * T, hold)
    reqs = check_schedule(log, k0, count, arrive, arena, 64 * T, 2 * T, hold)
    first_done = min(reqs[0][-1][1], reqs[1][-1][1])
    assert reqs[2][0][1] >= first_done + 1 + hold


def test_random_trace_shortest_first(R):
    # the same invariants under the shortest-first policy
    rng = inputs.SplitMix64(20240612)
    n = 300
    k0 = [rng.next() >> 24 for _ in range(n)]
    count = [1 + int(2.0 ** (16 * rng.unit53())) for _ in range(n)]
    arrive = np.cumsum([rng.next() % 3 for _ in range(n)]).tolist()
    arena, iter_o, chunk_o, hold = 1 << 19, 10 * T, 3 * T + 123, 2
    log = R.server_simulate(k0, count, arrive, arena, iter_o, chunk_o, hold,
                            policy=R.SRV_SHORTEST_FIRST)
    check_schedule(log, k0, count, arrive, arena, iter_o, chunk_o, hold)


def test_shortest_first_order(R):
    # five requests arrive together; an iteration holds four tiles: shortest
    # first fills it with the fewest-outputs-left requests, so the short ones
    # finish in the first iterations and the long one last, where round robin
    # gives every request a chunk per iteration
    count = [40 * T, 2 * T, T, 3 * T, T // 2]
    k0 = [i * BLOCK for i in range(5)]
    arrive = [0] * 5
    sf = by_request(R.server_simulate(k0, count, arrive, 1 << 24, 4 * T, 2 * T,
                                      policy=R.SRV_SHORTEST_FIRST), 5)
    done = [ch[-1][1] for ch in sf]
    assert done[4] == 0 and done[2] == 0 and done[1] == 0    # T/2 + T + 2T in iteration 0
    # then 3T takes two iterations of at most one 2T chunk, beside the long one's
    assert done[3] == 2 and done[0] == max(done)
    assert all(ch[0][1] == 0 for ch in sf[1:3])
    assert sf[0][0][1] >= 1                                  # the long one waits
    rr = by_request(R.server_simulate(k0, count, arrive, 1 << 24, 4 * T, 2 * T), 5)
    assert rr[0][0][1] == 0                                  # round robin starts it at once
    with pytest.raises(R.RsaprngError):
        R.server_simulate(k0, count, arrive, 1 << 24, 4 * T, 2 * T, policy=7)


def test_rejects_bad_traces(R):
    with pytest.raises(R.RsaprngError):
        R.server_simulate([0], [10], [0], 5)            # larger than the arena
    with pytest.raises(R.RsaprngError):
        R.server_simulate([0, 0], [1, 1], [3, 1], 100)  # arrivals out of order
    with pytest.raises(R.RsaprngError):
        R.server_simulate([(1 << 64) - 1], [2], [0], 100)  # past 2^64
