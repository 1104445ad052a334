"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++,
host only): the served form's scheduler driven by random request streams with
its invariants checked; the whole host library over a checking stand-in of the
HIP runtime; and the CPU oracle on generation, the battery and prime counts,
its digests equal to the regular build's."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
       "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    return env


def test_scheduler_invariants_under_sanitizers(tmp_path):
    exe = str(tmp_path / "scheduler_harness")
    subprocess.check_call(["g++", "-std=c++17", *SAN,
                           "-I" + os.path.join(ROOT, "paper_1811_11629_amd", "csrc"),
                           "-I" + os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(ROOT, "tests", "native", "scheduler_harness.cpp")])
    for seed in (1, 2, 3):
        r = subprocess.run([exe, str(seed)], capture_output=True, text=True, timeout=300, env=_env())
        assert r.returncode == 0 and r.stdout.startswith("ok"), (seed, r.stdout[-2000:], r.stderr[-4000:])


def test_host_library_under_sanitizers(tmp_path):
    """host.cpp, server.cpp and noalloc.hip built for the host against a checking
    stand-in of the HIP runtime (tests/native/fakehip.cpp): every entry point over
    uneven batched, consume and served request sets, with every simulated output
    checked for its own (instance, index) and no device object left behind."""
    csrc = os.path.join(ROOT, "paper_1811_11629_amd", "csrc")
    native = os.path.join(ROOT, "tests", "native")
    exe = str(tmp_path / "host_harness")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I" + os.path.join(native, "fakehip"),
                           "-I" + csrc, "-I" + os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(native, "host_harness.cpp"),
                           os.path.join(native, "fakehip.cpp"), os.path.join(csrc, "host.cpp"),
                           os.path.join(csrc, "server.cpp"), "-x", "c++",
                           os.path.join(csrc, "noalloc.hip"), "-lpthread"])
    r = subprocess.run([exe, str(tmp_path / "tune.jsonl")], capture_output=True, text=True,
                       timeout=900, env=_env())
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout[-3000:], r.stderr[-6000:])


def _fnv(h, data):
    for b in data:
        h = ((h ^ b) * 1099511628211) & ((1 << 64) - 1)
    return h


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    exe = str(tmp_path / "oracle_harness")
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-ffp-contract=off",
                           "-I" + os.path.join(ROOT, "oracle"), "-o", exe,
                           os.path.join(ROOT, "tests", "native", "oracle_harness.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=_env())
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    got = dict(line.split(" ", 1) for line in r.stdout.strip().splitlines())
    # the same digests from the regular build of the oracle
    p, q, e, m0, cnt = 2147483693, 2147483777, 3, 12345, 40000
    h = 14695981039346656037
    ranges = []
    for k0 in (0, (1 << 20) - 1000, (1 << 63) + 7):
        c, rr = oracle.generate(p, q, e, m0, 1, k0, cnt)
        h = _fnv(h, c.tobytes())
        h = _fnv(h, rr.tobytes())
        ranges.append(k0)
    assert got["generate"] == "%016x" % h
    import inputs
    inst = inputs.Instance(p, q, e, m0)
    rec = oracle.battery([(inst, k0, cnt) for k0 in ranges])
    buf = b"".join(rec[name].tobytes() for name, _, _ in oracle.BATTERY_FIELDS)
    assert len(buf) == oracle.BATTERY_BYTES
    w = np.frombuffer(buf, dtype=np.uint32).astype(np.uint64)
    bs = int((w * np.arange(1, w.size + 1, dtype=np.uint64)).sum(dtype=np.uint64))
    assert got["battery"] == "%016x" % bs
    assert got["primes"] == "%d %d" % (oracle.count_primes(1 << 31, (1 << 31) + 200000),
                                      oracle.count_primes(1 << 31, (1 << 31) + 200000, True))
