#!/usr/bin/env python3
"""Benchmark of the RSA-exponentiation generator on one MI355X.

Headline (one "step"): the multi-instance workload -- 1024 independent seeded
prime pairs, e = 3, each split into 256 substreams of 2^12 starting at
k0 = j 2^12, 2^30 outputs written to HBM as uint64 c_k and binary64 r_k -- run
as one prepared batch with the autotuned kernel configuration, timed as eager
launches with HIP events between its kernels (graph replays of the same batch
are reported beside).  value = outputs per second of the whole step, in
Gnumbers/s.

Also reported (not the headline): the same work as plain per-instance
rsaprng_generate launches round-robin over 4 streams; the exponent sweep in
fused-consume mode (4096 instances x 2^18 outputs per e, no HBM write); the
batched uneven workload (10,000 instances, lengths log-uniform in [2^8, 2^22],
start indices below 2^40) as one graph-captured persistent launch, beside its
plain per-request launches; the served workload (100,000 device-resident
instances, Poisson arrivals, continuous batching: p50/p99 latency and
throughput at a fixed offered load); parameter generation (prime and safe-prime
counts, next-prime queries); the statistical battery as a fused consumer; the
vector mode (M_v substreams of one instance); the roofline of the tile kernel;
and the CPU oracle timed on the host's cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # lane-operations/s: 256 CUs x 64 lanes x 2.4 GHz
B = 1 << 20


def ladder_length(e: int) -> int:
    """L(e): squarings plus multiplies of the binary ladder for e."""
    return e.bit_length() - 1 + bin(e).count("1") - 1


def alg_instr(e: int, consume: bool = False) -> int:
    """Algorithmic VALU lane-instructions per output for exponent e: the cheaper
    of the two forms of the method's arithmetic (64-bit Montgomery products, 18
    per product plus 21 for the skip step, the add mod n, the conversion and the
    quotient; or CRT residues in binary64, 12 per ladder step over both primes
    plus 49 for the skip step, the residue updates, Garner's recombination, the
    conversion and the quotient), plus 12 for the fused statistics in consume
    mode."""
    L = ladder_length(e)
    return min(18 * L + 21, 12 * L + 49) + (12 if consume else 0)


def roofline_of(counts_by_e, seconds, consume, kernel, launch_what):
    """Roofline entry for a launch over outputs of several exponents: the binding
    bound of max(bytes / HBM peak, algorithmic instructions / VALU peak)."""
    n = sum(counts_by_e.values())
    instr = sum(c * alg_instr(e, consume) for e, c in counts_by_e.items())
    nbytes = 0 if consume else 16 * n
    t_alu = instr / (VALU_PEAK_TOPS * 1e12)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    out = {"kernel": kernel, "avg_launch_ms": seconds * 1e3, "launch": launch_what,
           "outputs_per_launch": n, "algorithmic_instr_per_output": instr / n,
           "algorithmic_bytes_per_output": nbytes / n,
           "bound_gnumbers_per_s": n / max(t_alu, t_hbm) / 1e9}
    if t_hbm >= t_alu:
        ach = nbytes / seconds / 1e9
        out.update({"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": ach / HBM_PEAK_GBS, "traffic": None})
    else:
        ach = instr / seconds / 1e12
        out.update({"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                    "unit": "T lane-instr/s", "frac": ach / VALU_PEAK_TOPS, "traffic": None})
    return out


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# The translation units of the generate-mode tile kernels and everything they include.
DEVICE_SOURCES = ("k_crt_gen.hip", "k_mont_gen.hip", "common.h", "devmath.h", "tiles.h",
                  "../../include/rsaprng.h")


def code_only(text: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed to one
    space (string and character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the code (comments and layout aside) of the sources the
    generate-mode tile kernels are compiled from."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1811_11629_amd", "csrc")
    for f in DEVICE_SOURCES:
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(os.path.basename(f).encode() + code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it was
    taken on the current kernel sources and on the same tile kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "tile_kernel_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload)
    if not ent or ent.get("kernel_source_hash") != kernel_source_hash():
        return None
    name = kernel.split(" (")[0]
    # the profiled kernel, or another shape the autotuner may pick, measured by
    # the same two counter passes and calibration on the same sources
    for e in [ent] + list(ent.get("other_kernels", [])):
        if e.get("kernel") == name:
            return e.get("hbm_bytes_per_launch")
    return None


def time_timed(batch, stream, steps, warmup, torch):
    """The timed region of the headline: `steps` launches of the prepared batch,
    each with HIP events between its kernels on `stream`; returns wall seconds
    and the per-kernel averages of those same launches."""
    for _ in range(warmup):
        batch.run_timed(stream)
    batch.kernel_ms()  # discard the warm-up runs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run_timed(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, batch.kernel_ms()


def time_graph(batch, stream, steps, warmup, torch):
    for _ in range(warmup):
        batch.run(stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        batch.run(stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [a.elapsed_time(b) for a, b in evs]
    return wall, kms


def tile_kernel_name(cfg, exponent=0, mode="generate") -> str:
    """The tile kernel of a configuration, as rocprofv3 lists it, following the
    launcher's choice for chain-serial CRT launches: the kernels specialised to
    the launch's one exponent (generate: e = 3 with two chunks of 8 or one of
    16 indices per lane; consume: 256 lanes, one chunk of 16, any unrolled
    exponent), else the per-chain exponent dispatch ((256 or 512, 8, 2) in
    generate mode, (256, 8, 2) in consume mode), with 16 indices per lane
    taken as two chunks of 8 where no kernel of 16 is built.  Two passes with
    16 indices per lane (CRT generate) launch one kernel per exponent class,
    named here with `e` when the launch holds several."""
    form = {0: "k_gen2", 1: "k_gen1", 2: "k_gen3"}[cfg.prefix]
    per, chunks, lanes = cfg.per_lane, cfg.chunks_per_wave, cfg.lanes_per_tile
    ek = ""
    if cfg.prefix == 2 and cfg.variant == 2 and mode in ("generate", "consume"):
        if mode == "generate":
            one = exponent == 3 and (per, chunks) in ((8, 2), (16, 1))
        else:
            one = per == 16 and lanes == 256 and exponent in (3, 5, 7, 17, 257, 65537)
        if one:
            ek = ", %d" % exponent
        else:
            if per == 16:
                per, chunks = 8, 2
            if (per, chunks) == (8, 2) and (mode == "generate" or lanes == 256):
                ek = ", -1"
    elif cfg.prefix == 2 and per == 16:
        per, chunks = 8, 2
    elif cfg.prefix == 0 and per == 16:
        if cfg.variant == 2 and mode == "generate":
            # one launch per exponent class, each specialised to its exponent
            ek = ", %d" % exponent if exponent in (3, 5, 7, 17, 257, 65537) else ", e"
        else:
            per, chunks = 8, 4
    r = "" if cfg.prefix == 1 else ", %d" % chunks
    return "%s<%d, %d%s, %d, %d%s> (%s, %s)" % (
        form, lanes, per, r, cfg.variant, {"generate": 0, "consume": 1}.get(mode, 2),
        ek, "CRT binary64 residues" if cfg.variant == 2 else "Montgomery-64", mode)


def config2_requests():
    import inputs
    reqs = []
    for i in range(1024):
        for j in range(inputs.CONFIG2_SUBSTREAMS):
            k0 = j * inputs.CONFIG2_SUBSTREAM_LEN
            reqs.append((i, k0, inputs.CONFIG2_SUBSTREAM_LEN, i * B + k0))
    return reqs


def verify_config2(insts, oc, orr, n_full=3, n_samples=48):
    """Untimed: whole outputs of a few instances, single samples of others."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(7)
    ok = True
    full = rng.choice(len(insts), n_full, replace=False)
    for i in full:
        inst = insts[int(i)]
        c, r = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, 0, B)
        cg = oc[int(i) * B:(int(i) + 1) * B].cpu().numpy().view(np.uint64)
        rg = orr[int(i) * B:(int(i) + 1) * B].cpu().numpy()
        ok &= bool(np.array_equal(cg, c) and np.array_equal(rg.view(np.uint64), r.view(np.uint64)))
    for _ in range(n_samples):
        i = int(rng.integers(len(insts)))
        k = int(rng.integers(B))
        inst = insts[i]
        c, r = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k, 1)
        cg = int(oc[i * B + k].item()) & ((1 << 64) - 1)
        rg = float(orr[i * B + k].item())
        ok &= (cg == int(c[0]) and rg == float(r[0]))
    return ok


def cpu_baseline(insts, budget_outputs):
    """The oracle, unmodified, over whole instances of the workload on the host's
    cores (and on one core for context)."""
    import concurrent.futures as cf

    import oracle
    threads = min(16, os.cpu_count() or 1)
    n_inst = min(len(insts), max(threads, budget_outputs // B))
    sample = insts[:n_inst]
    oracle.lib()

    def one(inst):
        oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, 0, B)
        return B

    t0 = time.perf_counter()
    c0 = time.process_time()
    with cf.ThreadPoolExecutor(threads) as ex:
        done = sum(ex.map(one, sample))
    dt = time.perf_counter() - t0
    cpu_s = time.process_time() - c0
    t1 = time.perf_counter()
    for inst in sample[:4]:
        one(inst)
    single = 4 * B / (time.perf_counter() - t1) / 1e9
    return {"value": done / dt / 1e9, "unit": "Gnumbers/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the 1024 multi-instance workload's instances, each k in [0, 2^20) "
                      "(c_k and r_k) by the plain C oracle, %d host threads: %.1f s wall, %.1f "
                      "CPU-s" % (len(sample), threads, dt, cpu_s),
            "single_thread_value": single}


def cpu_host_info():
    """The host's processor model, clock and thread count, from lscpu (or
    /proc/cpuinfo)."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k in ("Model name", "CPU max MHz", "CPU MHz", "Socket(s)", "Core(s) per socket",
                     "Thread(s) per core"):
                info[k] = v
    except (OSError, subprocess.SubprocessError):
        pass
    if "Model name" not in info:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        info["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return info


def _oracle_rate(work, threads, fn):
    """Outputs per second (G) of fn over the work items on `threads` host threads."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    if threads == 1:
        n = sum(fn(w) for w in work)
    else:
        with cf.ThreadPoolExecutor(threads) as ex:
            n = sum(ex.map(fn, work))
    dt = time.perf_counter() - t0
    return n / dt / 1e9, n, dt


def cpu_baselines(threads=None):
    """The oracle, unmodified, on bounded samples of the exponent sweep (fused
    statistics), the batched uneven workload and the served request trace, at
    one thread and at the host's thread share."""
    import numpy as np

    import inputs
    import oracle
    threads = threads or min(16, os.cpu_count() or 1)
    oracle.lib()
    out = {"host": cpu_host_info(), "threads": threads}

    def consume(w):
        inst, k0, cnt = w
        oracle.consume(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, cnt)
        return cnt

    def generate(w):
        inst, k0, cnt = w
        oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, cnt)
        return cnt

    base = inputs.config3()
    sweep = {}
    for e in inputs.SWEEP_EXPONENTS:
        insts = [inputs.Instance(b.p, b.q, e, b.m0) for b in base[:64 * threads]]
        work = [(i, 0, 1 << 18) for i in insts]
        v, n, dt = _oracle_rate(work, threads, consume)
        v1, n1, dt1 = _oracle_rate(work[:32], 1, consume)
        sweep["e%d" % e] = {"value": v, "single_thread_value": v1,
                            "sample": "%d instances x 2^18 outputs (fused statistics): %.2f s; "
                                      "one thread: 32 instances, %.2f s" % (len(work), dt, dt1)}
    out["exponent_sweep_consume"] = sweep
    insts4, reqs4 = inputs.config4()
    work = [(insts4[r.inst], r.k0, r.count) for r in reqs4[::10]]
    v, n, dt = _oracle_rate(work, threads, generate)
    v1, n1, dt1 = _oracle_rate(work[::20], 1, generate)
    out["batched_uneven"] = {"value": v, "single_thread_value": v1,
                             "sample": "every 10th request (%d requests, %d outputs, each with its "
                                       "lead-in walk): %.2f s; one thread: every 200th (%d "
                                       "outputs), %.2f s" % (len(work), n, dt, n1, dt1)}
    insts5, rng5 = inputs.config5_instances(100000)
    trace = inputs.config5_requests(rng5, len(insts5), 256)
    work = [(insts5[r.inst], r.k0, r.count) for r in trace]
    v, n, dt = _oracle_rate(work, threads, generate)
    v1, n1, dt1 = _oracle_rate(work[:16], 1, generate)
    out["served"] = {"value": v, "single_thread_value": v1,
                     "sample": "256 served requests back to back (%d outputs): %.2f s; one "
                               "thread: 16 of them (%d outputs), %.2f s" % (n, dt, n1, dt1)}
    out["unit"] = "Gnumbers/s"
    out["kind"] = "oracle"
    return out


def run_plain_config2(R, gens, oc, orr, torch, reps=2):
    streams = [torch.cuda.Stream() for _ in range(4)]
    for g in gens[:8]:
        R.rsaprng_generate(g, 0, B, oc, orr, stream=streams[0])
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        t0 = time.perf_counter()
        for i, g in enumerate(gens):
            R.rsaprng_generate(g, 0, B, oc[i * B:], orr[i * B:], stream=streams[i % 4])
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    for s in streams:
        R.rsaprng_check_device_error(s)
    return best


def verify_consume(R, st, insts, count, threads=None):
    """Untimed: records of the last timed replay against the oracle's statistics
    of the same instances (whole 2^18-index ranges), at the ends of the record
    array and spread through it."""
    import concurrent.futures as cf
    from fractions import Fraction

    import numpy as np

    import oracle
    got = R.stats_decode(st)
    m = len(insts)
    idx = sorted({0, 1, m // 2, m - 1} | {(j * 613) % m for j in range(1, 5)})
    threads = threads or min(16, os.cpu_count() or 1)

    def ref(i):
        it = insts[i]
        return oracle.consume(it.p, it.q, it.e, it.m0, it.s0, 0, count)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        refs = list(ex.map(ref, idx))
    ok = True
    for i, r in zip(idx, refs):
        g = got[i]
        ok = ok and (g["count"] == count and g["sum_fx"] == r["sum_fx"] and
                     g["lt_half"] == r["lt_half"] and np.array_equal(g["hist"], r["hist"]) and
                     g["sum"] == float(Fraction(r["sum_fx"], 1 << 128)))
    return {"records_compared": len(idx), "record_indices": idx, "all_equal": bool(ok),
            "seconds": time.perf_counter() - t0}


def run_consume_sweep(R, torch, stream, steps, exponents=None, cfg=None, verify=True):
    import inputs
    base = inputs.config3()
    out = {}
    st = R.stats_tensor(len(base))
    for e in exponents or inputs.SWEEP_EXPONENTS:
        insts = [inputs.Instance(i.p, i.q, e, i.m0) for i in base]
        pool = R.Pool.from_instances(insts)
        reqs = [(i, 0, 1 << 18, i) for i in range(len(insts))]
        if cfg is None:
            best, _ = R.rsaprng_autotune(pool, reqs, R.MODE_CONSUME, stats=st, stream=stream)
        else:
            best = cfg
        b = R.Batch(pool, reqs, R.MODE_CONSUME, stats=st, cfg=best, stream=stream)
        wall, kms = time_graph(b, stream, max(2, steps // 4), 1, torch)
        b.check()
        n = len(insts) << 18
        ms = sum(kms) / len(kms)
        ver = verify_consume(R, st, insts, 1 << 18) if verify else None
        out["e%d" % e] = {"gnumbers_per_s": n / (ms / 1e3) / 1e9, "ms_per_launch": ms,
                          "verified": ver,
                          "variant": int(best.variant), "config": best.as_dict(),
                          "roofline": roofline_of({e: n}, ms / 1e3, True,
                                                  tile_kernel_name(best, exponent=e, mode="consume"),
                                                  "one graph replay (statistics zeroing, chain "
                                                  "setup, prefix pass, tile kernel, finalisation)")}
        log("consume e=%d: %.1f Gnum/s (%.3f ms)%s" % (
            e, out["e%d" % e]["gnumbers_per_s"], ms,
            "" if ver is None else "; %d records equal the oracle's: %s" % (
                ver["records_compared"], ver["all_equal"])))
        del b, pool
    return out


def verify_requests(insts, reqs, oc, orr, cap_s=120.0, threads=None):
    """Untimed: every output of the given requests, (inst, k0, count, out_off),
    compared bit for bit with the oracle on the host's threads.  Requests are
    taken in the order j = 0, 4, 8, ..., then 1, 5, ..., 2, 6, ..., 3, 7, ...,
    so that if the time cap stops the comparison early, what was compared is
    every 4th request first, a stated deterministic subset."""
    import collections
    import concurrent.futures as cf

    import numpy as np

    import oracle
    threads = threads or min(16, os.cpu_count() or 1)
    order = [j for s in range(4) for j in range(s, len(reqs), 4)]

    def one(j):
        i, k0, cnt, o = reqs[j]
        inst = insts[i]
        cref, rref = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, k0, cnt)
        cg = oc[o:o + cnt].cpu().numpy().view(np.uint64)
        rg = orr[o:o + cnt].cpu().numpy().view(np.uint64)
        return bool(np.array_equal(cg, cref) and np.array_equal(rg, rref.view(np.uint64))), cnt

    t0 = time.perf_counter()
    ok, n_out, n_req = True, 0, 0
    with cf.ThreadPoolExecutor(threads) as ex:
        pend = collections.deque()
        for j in order:
            if time.perf_counter() - t0 > cap_s:
                break
            pend.append(ex.submit(one, j))
            while len(pend) >= 2 * threads:
                eq, cnt = pend.popleft().result()
                ok &= eq
                n_out += cnt
                n_req += 1
        for f in pend:
            eq, cnt = f.result()
            ok &= eq
            n_out += cnt
            n_req += 1
    return {"all_equal": bool(ok), "outputs_compared": n_out, "requests_compared": n_req,
            "requests": len(reqs), "complete": n_req == len(reqs),
            "seconds": time.perf_counter() - t0, "threads": threads,
            "order": "requests j = 0, 4, 8, ... first, then 1 mod 4, 2 mod 4, 3 mod 4; "
                     "time cap %.0f s" % cap_s}


def run_batched_uneven(R, torch, stream, steps, cfg=None, plain=True, verify_cap_s=120.0):
    import inputs
    t0 = time.perf_counter()
    insts, reqs4 = inputs.config4()
    log("batched workload drawn in %.1f s" % (time.perf_counter() - t0))
    total = sum(r.count for r in reqs4)
    reqs, off = [], 0
    for r in reqs4:
        reqs.append((r.inst, r.k0, r.count, off))
        off += r.count
    oc = torch.empty(total, dtype=torch.int64, device="cuda")
    orr = torch.empty(total, dtype=torch.float64, device="cuda")
    pool = R.Pool.from_instances(insts)
    if cfg is None:
        best, _ = R.rsaprng_autotune(pool, reqs, R.MODE_GENERATE, oc, orr, stream=stream)
    else:
        best = cfg
    b = R.Batch(pool, reqs, R.MODE_GENERATE, oc, orr, cfg=best, stream=stream)
    wall, kms = time_graph(b, stream, max(2, steps // 4), 1, torch)
    b.check()
    ms = sum(kms) / len(kms)
    batched = total / (ms / 1e3) / 1e9
    # untimed: the graph's own outputs against the oracle, before anything else
    # writes these buffers
    stream.synchronize()
    ver = verify_requests(insts, reqs, oc, orr, cap_s=verify_cap_s)
    log("batched uneven verified: %d of %d outputs (%d requests) in %.1f s, equal: %s" % (
        ver["outputs_compared"], total, ver["requests_compared"], ver["seconds"], ver["all_equal"]))
    by_e = {}
    for r in reqs4:
        by_e[insts[r.inst].e] = by_e.get(insts[r.inst].e, 0) + r.count
    plain_s = None
    if plain:
        # plain per-request launches, round-robin over 4 streams
        gens = [R.rsaprng_create_ex(i.p, i.q, i.e, i.m0, i.s0) for i in insts]
        streams = [torch.cuda.Stream() for _ in range(4)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for j, (i, k0, cnt, o) in enumerate(reqs):
            R.rsaprng_generate(gens[i], k0, cnt, oc[o:], orr[o:], stream=streams[j % 4])
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t1
        for s in streams:
            R.rsaprng_check_device_error(s)
    res = {"workload": "10000 instances, e from {3,5,7,17,257,65537}, lengths log-uniform in "
                       "[2^8, 2^22], k0 < 2^40, %d outputs u64+f64" % total,
           "batched_gnumbers_per_s": batched, "batched_ms": ms,
           "plain_per_request_gnumbers_per_s": total / plain_s / 1e9 if plain_s else None,
           "batched_vs_plain": (total / (ms / 1e3)) / (total / plain_s) if plain_s else None,
           "config": best.as_dict(), "outputs_by_exponent": {str(k): v for k, v in by_e.items()},
           "verified": ver,
           "roofline": roofline_of(by_e, ms / 1e3, False, tile_kernel_name(best),
                                   "one graph replay (chain setup, prefix pass over the "
                                   "lead-in, tile kernel; with two passes of 16 indices "
                                   "per lane one tile launch per exponent class)")}
    log("batched uneven: %.1f Gnum/s graph" % batched +
        (" vs %.1f plain" % res["plain_per_request_gnumbers_per_s"] if plain_s else ""))
    del b, oc, orr
    torch.cuda.empty_cache()
    return res


def tune_served(R, torch, stream, pool, inst, k0, cnt, chunk):
    """Kernel configuration for the server, tuned on an iteration-like batch: 64
    requests of the trace, each cut to the server's per-iteration chunk."""
    reqs, off = [], 0
    for j in range(64):
        c = int(min(int(cnt[j]), chunk))
        reqs.append((int(inst[j]), int(k0[j]), c, off))
        off += c
    oc = torch.empty(off, dtype=torch.int64, device="cuda")
    orr = torch.empty(off, dtype=torch.float64, device="cuda")
    best, ms = R.rsaprng_autotune(pool, reqs, R.MODE_GENERATE, oc, orr, stream=stream)
    del oc, orr
    torch.cuda.empty_cache()
    return best, ms


def verify_served(srv, insts, inst, k0, cnt, threads=None):
    """Untimed: submit the requests (inst, k0, cnt) together, wait for all of
    them, and compare every output of each (read back from the server's arena)
    bit for bit with the oracle, on the host's threads; then release them."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    threads = threads or min(16, os.cpu_count() or 1)
    base = 1 << 40
    n = len(inst)
    for j in range(n):
        rc = srv.submit(int(inst[j]), int(k0[j]), int(cnt[j]), base + j)
        if rc != 0:
            raise RuntimeError("rsaprng_server_submit returned %d" % rc)
    done = set()
    t0 = time.perf_counter()
    while len(done) < n:
        for c in srv.poll():
            done.add(c.tag - base)
        if time.perf_counter() - t0 > 120:
            raise RuntimeError("served verification: requests did not complete")
        time.sleep(0.0005)

    def one(j):
        c = int(cnt[j])
        cg = np.empty(c, dtype=np.uint64)
        rg = np.empty(c, dtype=np.float64)
        srv.read(base + j, cg, rg)
        inst_ = insts[int(inst[j])]
        cref, rref = oracle.generate(inst_.p, inst_.q, inst_.e, inst_.m0, inst_.s0, int(k0[j]), c)
        return bool(np.array_equal(cg, cref) and
                    np.array_equal(rg.view(np.uint64), rref.view(np.uint64))), c

    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(n)))
    for j in range(n):
        srv.release(base + j)
    return {"all_equal": all(r[0] for r in res), "requests_compared": n,
            "outputs_compared": sum(r[1] for r in res), "seconds": time.perf_counter() - t0,
            "what": "%d requests of a fresh trace submitted together, every output read back "
                    "from the arena" % n}


def run_served(R, torch, stream, rho_main=0.7, sweep=(0.5, 0.9), iter_log2=26, chunk_log2=24,
               verify=True, policy="sf", compare=True, cfg=None):
    """Served workload: 100,000 device-resident instances, requests (instance
    uniform, k0 < 2^40, length log-uniform in [2^10, 2^24)) arriving as a Poisson
    stream; continuous batching with a 64 GiB output arena, iterations of
    2^iter_log2 outputs, at most 2^chunk_log2 per request and iteration, the
    requests with the fewest outputs left first (policy "sf") or round robin
    ("rr").  Offered load is a fraction rho of the server's own saturated
    capacity (every request of a trace submitted at once).  With compare, a
    round-robin server with iterations of 2^27 outputs runs the saturated trace
    and the highest load of the sweep beside it.  cfg: the kernel configuration
    (else the served autotuner's choice)."""
    import numpy as np

    import inputs
    t0 = time.perf_counter()
    insts, rng = inputs.config5_instances(100000)
    log("served pool drawn in %.1f s" % (time.perf_counter() - t0))
    pool = R.Pool.from_instances(insts)
    mean_count = 2.0 ** 10 * (2.0 ** 14 - 1) / (14 * np.log(2.0))   # E[2^(10+14u)], u uniform

    def trace(n):
        reqs = inputs.config5_requests(rng, len(insts), n)
        return (np.array([r.inst for r in reqs], dtype=np.uint32),
                np.array([r.k0 for r in reqs], dtype=np.uint64),
                np.array([r.count for r in reqs], dtype=np.uint64))

    chunk = 1 << chunk_log2
    if cfg is None:
        cfg, tune_ms = tune_served(R, torch, stream, pool, *trace(64), chunk)
    else:
        tune_ms = None
    pol = {"rr": R.SRV_ROUND_ROBIN, "sf": R.SRV_SHORTEST_FIRST}[policy]
    log("served config", cfg.as_dict(), "iteration 2^%d outputs, chunk 2^%d, %s" % (
        iter_log2, chunk_log2, {"rr": "round robin", "sf": "shortest first"}[policy]))
    srv = R.Server(pool, arena_bytes=64 << 30, iter_outputs=1 << iter_log2, chunk_outputs=chunk,
                   cfg=cfg, policy=pol)

    res = {"workload": "100000 instances (e from {3,5,7,17,257,65537}), requests: instance "
                       "uniform, k0 < 2^40, count = floor(2^(10+14u)); Poisson arrivals; "
                       "64 GiB output arena; u64+f64 outputs",
           "config": cfg.as_dict(), "iteration_outputs": 1 << iter_log2,
           "chunk_outputs": chunk,
           "policy": {"rr": "round robin", "sf": "shortest first"}[policy]}
    # saturated capacity: a trace submitted at once
    inst, k0, cnt = trace(40000)
    t_adm, t_done = srv.replay(inst, k0, cnt, np.zeros(len(inst)))
    cap = float(cnt.sum()) / float(t_done.max()) / 1e9
    res["saturated_gnumbers_per_s"] = cap
    by_e = {}
    for i, c in zip(inst, cnt):
        by_e[insts[int(i)].e] = by_e.get(insts[int(i)].e, 0) + int(c)
    res["roofline"] = roofline_of(by_e, float(t_done.max()), False,
                                  tile_kernel_name(cfg) + " per iteration",
                                  "the whole saturated trace (40000 requests submitted at once), "
                                  "wall clock")
    log("served saturated: %.1f Gnum/s over %d requests" % (cap, len(inst)))
    # the same requests as plain per-request launches on one stream
    n_plain = 4000
    oc = torch.empty(int(cnt[:n_plain].max()), dtype=torch.int64, device="cuda")
    orr = torch.empty_like(oc, dtype=torch.float64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j in range(n_plain):
        R.rsaprng_pool_generate(pool, [(int(inst[j]), int(k0[j]), int(cnt[j]), 0)], oc, orr,
                                cfg=cfg, stream=stream)
    torch.cuda.synchronize()
    plain = float(cnt[:n_plain].sum()) / (time.perf_counter() - t1) / 1e9
    R.rsaprng_check_device_error(stream)
    res["plain_per_request_gnumbers_per_s"] = plain
    res["saturated_vs_plain"] = cap / plain
    del oc, orr
    log("plain per-request launches: %.1f Gnum/s" % plain)

    def poisson(rho, warm, steady):
        lam = rho * cap * 1e9 / mean_count
        n = int(lam * (warm + steady))
        inst, k0, cnt = trace(n)
        t_arr = inputs.poisson_arrivals(rng, lam, n)
        t_adm, t_done = srv.replay(inst, k0, cnt, t_arr)
        win = (t_arr >= warm) & (t_arr < warm + steady)
        lat = (t_done - t_arr)[win]
        span = float(t_done.max() - t_arr.min())
        out = {"rho": rho, "arrival_rate_per_s": lam, "requests": n,
               "window_requests": int(win.sum()), "warmup_s": warm, "steady_s": steady,
               "offered_gnumbers_per_s": float(cnt[win].sum()) / steady / 1e9,
               "served_gnumbers_per_s": float(cnt.sum()) / span / 1e9,
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_admit_wait_ms": float((t_adm - t_arr)[win].mean() * 1e3)}
        log("served rho=%.2f: %.1f Gnum/s, p50 %.2f ms, p99 %.2f ms" % (
            rho, out["served_gnumbers_per_s"], out["p50_ms"], out["p99_ms"]))
        return out

    res["headline"] = poisson(rho_main, 2.0, 10.0)
    res["sweep"] = [poisson(r, 1.0, 4.0) for r in sweep]
    if compare:
        main = srv
        srv = R.Server(pool, arena_bytes=64 << 30, iter_outputs=1 << 27, chunk_outputs=chunk,
                       cfg=cfg, policy=R.SRV_ROUND_ROBIN)
        inst, k0, cnt = trace(40000)
        t_adm, t_done = srv.replay(inst, k0, cnt, np.zeros(len(inst)))
        cap_main, cap = cap, float(cnt.sum()) / float(t_done.max()) / 1e9
        log("round robin, iteration 2^27: saturated %.1f Gnum/s" % cap)
        res["round_robin_2p27"] = {"saturated_gnumbers_per_s": cap,
                                   "high_load": poisson(max(sweep), 1.0, 4.0)}
        srv.close()
        srv, cap = main, cap_main
    if verify:
        res["verified"] = verify_served(srv, insts, *trace(256))
        log("served verified: %d requests, %d outputs, equal: %s" % (
            res["verified"]["requests_compared"], res["verified"]["outputs_compared"],
            res["verified"]["all_equal"]))
    st = srv.stats()
    res["iterations"] = st["iterations"]
    srv.close()
    del pool
    return res


def p_in_band(rep):
    """The paper's pass criterion over the tests that counted samples: no
    p-value below 1e-6 or above 1 - 1e-6."""
    return all(1e-6 < v["p"] < 1 - 1e-6 for v in rep.values() if v["samples"] > 0)


def run_battery(R, torch, stream, steps):
    """The statistical battery as a fused consumer over 2^30 outputs (the
    exponent-sweep instances at e = 3, 2^18 indices each) into one record."""
    import inputs
    base = inputs.config3()
    insts = [inputs.Instance(i.p, i.q, 3, i.m0) for i in base]
    pool = R.Pool.from_instances(insts)
    reqs = [(i, 0, 1 << 18, 0) for i in range(len(insts))]
    rec = R.battery_tensor()
    best = None
    t_best = 1e30
    for cfg in (R.config(variant=2, prefix=2, lanes_per_tile=256, chunks_per_wave=4),
                R.config(variant=2, prefix=2, lanes_per_tile=512, chunks_per_wave=2)):
        R.rsaprng_pool_battery(pool, reqs, rec, cfg=cfg, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(2, steps // 4)):
            R.rsaprng_pool_battery(pool, reqs, rec, cfg=cfg, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(2, steps // 4)
        if dt < t_best:
            t_best, best = dt, cfg
    R.rsaprng_check_device_error(stream)
    rep = R.battery_report(rec)
    n = len(insts) << 18
    res = {"workload": "4096 instances, e = 3, k in [0, 2^18): 2^30 outputs into one record",
           "gnumbers_per_s": n / t_best / 1e9, "ms": t_best * 1e3, "config": best.as_dict(),
           "tests": rep, "all_p_in_paper_band": p_in_band(rep),
           # a leading-bit collision trial needs 327680 consecutive indices
           "tests_without_samples": [k for k, v in rep.items() if v["samples"] == 0]}
    log("battery: %.1f Gnum/s (%.2f ms); p-values %s" % (
        res["gnumbers_per_s"], t_best * 1e3, " ".join("%s=%.3f" % (k, v["p"]) for k, v in rep.items())))
    # the same instances over four 2^20 blocks each: 2^34 outputs across three
    # re-seedings per instance, which must leave no trace in any test
    reqs4 = [(i, 0, 1 << 22, 0) for i in range(len(insts))]
    t0 = time.perf_counter()
    R.rsaprng_pool_battery(pool, reqs4, rec, cfg=best, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    R.rsaprng_check_device_error(stream)
    rep4 = R.battery_report(rec)
    res["across_reseeding"] = {
        "workload": "the same 4096 instances, k in [0, 2^22) (four blocks each): 2^34 outputs",
        "seconds": dt, "tests": rep4,
        "all_p_in_paper_band": p_in_band(rep4)}
    log("battery over 2^34 outputs (3 re-seedings per instance, %.2f s): p-values %s" % (
        dt, " ".join("%s=%.3f" % (k, v["p"]) for k, v in rep4.items())))
    del rec, pool
    torch.cuda.empty_cache()
    return res


def run_single(R, torch, stream, steps):
    """The single-instance workload: one rsaprng_generate of k in [0, 2^20) on a
    handle (launch- and latency-bound at this size), timed with events."""
    import numpy as np

    import inputs
    import oracle
    inst = inputs.config1()
    g = R.rsaprng_create_ex(inst.p, inst.q, inst.e, inst.m0, inst.s0)
    c = torch.empty(B, dtype=torch.int64, device="cuda")
    r = torch.empty(B, dtype=torch.float64, device="cuda")
    for _ in range(3):
        R.rsaprng_generate(g, 0, B, c, r, stream=stream)
    reps = max(10, steps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        R.rsaprng_generate(g, 0, B, c, r, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    us = sorted(a.elapsed_time(b) * 1e3 for a, b in evs)[reps // 2]
    cref, rref = oracle.generate(inst.p, inst.q, inst.e, inst.m0, inst.s0, 0, B)
    ok = bool(np.array_equal(c.cpu().numpy().view(np.uint64), cref) and
              np.array_equal(r.cpu().numpy().view(np.uint64), rref.view(np.uint64)))
    R.rsaprng_check_device_error(stream)
    log("single instance: %.1f us per 2^20 outputs (%.1f Gnum/s), verified %s" % (us, B / us / 1e3, ok))
    return {"workload": "one instance (e = %d), k in [0, 2^20), c and r, one rsaprng_generate" % inst.e,
            "us": us, "gnumbers_per_s": B / us / 1e3, "verified": ok}


def run_vector(R, torch, stream, steps):
    """Vector mode: 2^30 outputs of one e = 3 instance split into M_v substreams
    (the paper's vectorised calls), for several M_v; sampled outputs checked."""
    import numpy as np

    import inputs
    import oracle
    inst = inputs.config2(1)[0]
    g = R.rsaprng_create_ex(inst.p, inst.q, inst.e, inst.m0, inst.s0)
    N = 1 << 30
    c = torch.empty(N, dtype=torch.int64, device="cuda")
    r = torch.empty(N, dtype=torch.float64, device="cuda")
    res = {"workload": "one e = 3 instance of the multi-instance workload, 2^30 outputs "
                       "(vector calls 1 .. 2^30 / M_v), uint64 c and binary64 r"}
    rng = np.random.default_rng(11)
    reps = max(2, steps // 4)
    for mv in (8, 64, 4096, 1 << 16):
        R.rsaprng_generate_vector(g, mv, 0, N, c, r, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            R.rsaprng_generate_vector(g, mv, 0, N, c, r, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ok = True
        for f in rng.integers(0, N, 8):
            cj, rj = oracle.generate_vector(inst.p, inst.q, inst.e, inst.m0, inst.s0, mv, int(f), 1)
            ok &= int(c[int(f)].item()) & ((1 << 64) - 1) == int(cj[0]) and \
                float(r[int(f)].item()) == float(rj[0])
        res["mv_%d" % mv] = {"gnumbers_per_s": N / dt / 1e9, "ms": dt * 1e3, "verified_samples": ok}
        log("vector mode M_v=%d: %.1f Gnum/s (%.2f ms), samples %s" % (mv, N / dt / 1e9, dt * 1e3, ok))
        if mv == 64:
            # the battery over the flattened output: 64 substreams seen interleaved
            rec = R.battery_tensor()
            R.rsaprng_battery_values(r, rec, stream=stream)
            rep = R.battery_report(rec)
            res["interstream_battery_mv_64"] = {
                "values": N, "tests": rep,
                "all_p_in_paper_band": p_in_band(rep)}
            log("battery of the M_v=64 interleaved output: p-values %s" % " ".join(
                "%s=%.3f" % (k, v["p"]) for k, v in rep.items()))
            del rec
    R.rsaprng_check_device_error(stream)
    del c, r
    torch.cuda.empty_cache()
    return res


def run_param_gen(R, torch, stream):
    """Parameter generation: primes and safe primes in [2^31, 2^32) counted on the
    device (the paper's counts are the check), and the next prime at or above
    200,000 draws with the e = 3 filter; the oracle's sieve timed on a slice."""
    import numpy as np

    import inputs
    import oracle
    lo, hi = 1 << 31, 1 << 32
    res = {}
    for safe, want in ((False, 98182656), (True, 3060794)):
        R.rsaprng_prime_count(lo, lo + (1 << 24), safe, stream=stream)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = R.rsaprng_prime_count(lo, hi, safe, stream=stream)
        dt = time.perf_counter() - t0
        key = "safe_prime_count" if safe else "prime_count"
        res[key] = {"range": "[2^31, 2^32)", "count": got, "matches_paper": got == want,
                    "ms": dt * 1e3, "gnumbers_tested_per_s": (hi - lo) / dt / 1e9}
        log("%s: %d (%s) in %.1f ms" % (key, got, "= paper" if got == want else "MISMATCH", dt * 1e3))
    rng = inputs.SplitMix64(181111629 + 6)
    x = torch.tensor([(1 << 31) + (rng.next() >> 33) for _ in range(200000)], dtype=torch.int64,
                     device="cuda")
    out = torch.empty_like(x)
    R.rsaprng_next_primes(x, out, exps=(3,), stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R.rsaprng_next_primes(x, out, exps=(3,), stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    got = out.cpu().numpy().view(np.uint64)
    idx = np.random.default_rng(5).choice(len(got), 64, replace=False)
    ok = all(int(got[i]) == oracle.next_prime(int(x[i].item()), False, (3,)) for i in idx)
    res["next_primes"] = {"queries": 200000, "filter": "p mod 3 != 1", "ms": dt * 1e3,
                          "queries_per_s": 200000 / dt, "verified_samples": ok}
    t0 = time.perf_counter()
    oracle.count_primes(lo, lo + (1 << 28))
    dtc = time.perf_counter() - t0
    res["cpu_oracle_sieve"] = {"gnumbers_tested_per_s": (1 << 28) / dtc / 1e9, "cores": 1,
                               "sample": "primes in [2^31, 2^31 + 2^28) by the oracle's sieve"}
    log("next_primes: %.1f ms for 200000 (%s); oracle sieve %.2f Gnum/s" % (
        dt * 1e3, "verified" if ok else "MISMATCH", res["cpu_oracle_sieve"]["gnumbers_tested_per_s"]))
    return res


def run_issue_probe(R, torch, stream, iters=1 << 16, store_elems=1 << 30):
    """The ceilings behind the roofline figures, measured on this device: the
    issue rate of each VALU instruction class the kernels use (lane-instructions
    per second, and the clock it implies if the class issues one lane-operation
    per lane and cycle), and the store bandwidth of the tile kernels' output
    pattern and of a plain linear write."""
    res = {"nominal_lane_instr_per_s": VALU_PEAK_TOPS * 1e12,
           "issue": {}, "store": {}}
    for name, kind in R.PROBES.items():
        R.rsaprng_probe(kind, 64, stream=stream)            # warm-up
        times = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            work = R.rsaprng_probe(kind, iters, stream=stream)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = sorted(times)[1]
        rate = work / (ms / 1e3)
        res["issue"][name] = {"lane_instr_per_s": rate, "ms": ms,
                              "frac_of_nominal": rate / (VALU_PEAK_TOPS * 1e12),
                              "implied_ghz_if_full_rate": rate / (256 * 64) / 1e9}
        log("issue %-16s %.2f T lane-instr/s (%.3f of nominal, %.3f ms)" % (
            name, rate / 1e12, rate / (VALU_PEAK_TOPS * 1e12), ms))
    oc = torch.empty(store_elems, dtype=torch.int64, device="cuda")
    orr = torch.empty(store_elems, dtype=torch.float64, device="cuda")
    for name, kind in (("tile_pattern", R.PROBE_STORE_TILE),
                       ("tile_pattern_regular_stores", R.PROBE_STORE_TILE_PLAIN),
                       ("block16_pattern", R.PROBE_STORE_BLOCK16),
                       ("block16_pattern_regular_stores", R.PROBE_STORE_BLOCK16_PLAIN),
                       ("linear", R.PROBE_STORE_LINEAR)):
        R.rsaprng_probe(kind, store_elems, oc, orr, stream=stream)
        times = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            work = R.rsaprng_probe(kind, store_elems, oc, orr, stream=stream)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = sorted(times)[2]
        res["store"][name] = {"bytes": work, "ms": ms, "gb_per_s": work / (ms / 1e3) / 1e9,
                              "frac_of_hbm_peak": work / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
        log("store %-12s %.0f GB/s (%.3f ms for %.1f GiB)" % (
            name, work / (ms / 1e3) / 1e9, ms, work / 2 ** 30))
    ok = bool((oc[:8].cpu() == torch.arange(8)).all())
    del oc, orr
    torch.cuda.empty_cache()
    res["store_values_checked"] = ok
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device five times (counter calibration)")
    ap.add_argument("--issue-probe", action="store_true",
                    help="only the throughput probes (VALU issue rates, store bandwidth)")
    ap.add_argument("--consume-only", type=int, default=0, metavar="E",
                    help="only the exponent sweep's consume workload at exponent E (with "
                         "--config: that configuration, no autotuning)")
    ap.add_argument("--verify-cap", type=float, default=120.0, metavar="SECONDS",
                    help="time cap of the batched workload's comparison with the oracle")
    ap.add_argument("--served-only", default="", metavar="ITER,CHUNK[,POLICY]",
                    help="only the served workload, with iterations of 2^ITER outputs, "
                         "per-request chunks of 2^CHUNK and POLICY sf (shortest first, the "
                         "default) or rr (round robin) (no comparison with the oracle; with "
                         "--config: that configuration, no autotuning)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched uneven workload, without the plain per-request "
                         "launches (with --config: that configuration, no autotuning)")
    ap.add_argument("--config", default="",
                    help="fixed kernel configuration 'variant,lanes,per_lane,persistent[,prefix[,r]]' "
                         "instead of the autotuner (variant 1 = Montgomery-64, 2 = CRT; prefix 0 "
                         "= two passes, 1 = single pass with look-back, 2 = chain-serial; r = "
                         "chunks per wave)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the generator "
              "shards by instance or index range with no exchange; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    from paper_1811_11629_amd import rsaprng as R

    if args.copy_probe:
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}))
        return

    R.lib()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    fixed = None
    if args.config:
        f = [int(x) for x in args.config.split(",")] + [0, 0]
        v, lanes, per, pers, prefix, r = f[:6]
        fixed = R.config(variant=v, lanes_per_tile=lanes, per_lane=per, persistent=pers,
                         order=pers, prefix=prefix, chunks_per_wave=r)
    if args.issue_probe:
        print(json.dumps(run_issue_probe(R, torch, stream)), flush=True)
        return
    if args.batched_only:
        res = run_batched_uneven(R, torch, stream, args.steps, cfg=fixed, plain=False,
                                 verify_cap_s=args.verify_cap)
        print(json.dumps(res))
        return
    if args.served_only:
        parts = args.served_only.split(",")
        it, ch = int(parts[0]), int(parts[1])
        res = run_served(R, torch, stream, iter_log2=it, chunk_log2=ch, verify=False,
                         policy=parts[2] if len(parts) > 2 else "sf", compare=False, cfg=fixed)
        print(json.dumps(res))
        return
    if args.consume_only:
        res = run_consume_sweep(R, torch, stream, args.steps, exponents=[args.consume_only],
                                cfg=fixed)
        print(json.dumps(res))
        return

    insts = inputs.config2()
    pool = R.Pool.from_instances(insts)
    reqs = R.pool_reqs(config2_requests())
    N = 1024 * B
    oc = torch.empty(N, dtype=torch.int64, device="cuda")
    orr = torch.empty(N, dtype=torch.float64, device="cuda")

    if fixed is not None:
        best = fixed
        log("fixed config", best.as_dict())
    else:
        cache = os.environ.get("RSAPRNG_TUNE_CACHE")
        log("autotuning the multi-instance workload")
        best, best_ms = R.rsaprng_autotune(pool, reqs, R.MODE_GENERATE, oc, orr, cache_path=cache,
                                           stream=stream)
        log("best config", best.as_dict(), "%.3f ms" % best_ms)
    batch = R.Batch(pool, reqs, R.MODE_GENERATE, oc, orr, cfg=best, stream=stream)
    wall, kt = time_timed(batch, stream, args.steps, args.warmup, torch)
    batch.check()
    ms_step = wall / args.steps * 1e3
    value = N / (wall / args.steps) / 1e9
    k_ms = kt["tiles"]
    log("multi-instance: %.3f ms/step, %.1f Gnum/s; kernels (ms): setup %.3f prefix %.3f "
        "tiles %.3f" % (ms_step, value, kt["setup"], kt["prefix"], k_ms))
    gwall, gkms = time_graph(batch, stream, args.steps, 1, torch)
    batch.check()
    log("graph replay: %.3f ms/step" % (gwall / args.steps * 1e3))
    verified = verify_config2(insts, oc, orr)
    log("verified against oracle:", verified)

    alg_bytes = 16 * N                                      # 8 B c_k + 8 B r_k per output
    achieved = alg_bytes / (k_ms / 1e3) / 1e9
    traffic = traffic_from_profiles("multi_instance_e3", tile_kernel_name(best, exponent=3))
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": tile_kernel_name(best, exponent=3),
                "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": k_ms,
                "other_kernels_ms": {"setup": kt["setup"], "prefix": kt["prefix"]},
                "graph_replay_ms_per_step": gwall / args.steps * 1e3}

    extras = {}
    if not args.no_extras:
        gens = [R.rsaprng_create_ex(i.p, i.q, i.e, i.m0, i.s0) for i in insts]
        plain_s = run_plain_config2(R, gens, oc, orr, torch)
        extras["multi_instance_plain_per_instance"] = {
            "gnumbers_per_s": N / plain_s / 1e9, "ms": plain_s * 1e3,
            "launches": 1024, "streams": 4}
        extras["multi_instance_batched_vs_plain"] = (N / (wall / args.steps)) / (N / plain_s)
        del gens
        del batch, oc, orr
        torch.cuda.empty_cache()
        extras["single_instance"] = run_single(R, torch, stream, args.steps)
        extras["exponent_sweep_consume"] = run_consume_sweep(R, torch, stream, args.steps)
        extras["batched_uneven"] = run_batched_uneven(R, torch, stream, args.steps,
                                                      verify_cap_s=args.verify_cap)
        extras["served"] = run_served(R, torch, stream)
        extras["parameter_generation"] = run_param_gen(R, torch, stream)
        extras["battery"] = run_battery(R, torch, stream, args.steps)
        extras["vector_mode"] = run_vector(R, torch, stream, args.steps)

    cpu = None if args.no_cpu else cpu_baseline(insts, 1024 * B)
    if cpu:
        log("cpu oracle: %.3f Gnum/s on %d threads" % (cpu["value"], cpu["cores"]))
        cpu["host"] = cpu_host_info()
        if not args.no_extras:
            extras["cpu_baselines"] = cpu_baselines()
            log("cpu oracle on the other workloads:", json.dumps(
                {k: v["value"] for k, v in extras["cpu_baselines"].items()
                 if isinstance(v, dict) and "value" in v}))

    out = {
        "metric": "Gnumbers/s (u64+FP64) and % of INT-VALU/HBM roofline; batched & served vs plain",
        "value": value, "unit": "Gnumbers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64+f64", "data": "synthetic",
        "config": {"workload": "multi-instance: 1024 seeded prime pairs, e=3, 256 substreams of "
                               "2^12 per instance (k0 = j*2^12), 2^30 outputs as uint64 c_k and "
                               "binary64 r_k; one prepared batch per step, launched eagerly with "
                               "HIP events between its kernels (graph replays of the same batch "
                               "reported beside)",
                   "instances": 1024, "outputs_per_step": N, "exponent": 3,
                   "kernel_config": best.as_dict(), "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "verified": bool(verified),
        "paper_context": "paper: >1e8 numbers/s per 24-core Xeon E5-2680 v3 node (other hardware)",
        "kernel_source_hash": kernel_source_hash(),
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
