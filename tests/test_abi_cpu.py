"""CPU checks of the C-ABI library: it loads, exports every function declared in
include/rsaprng.h, and its host-side logic (validation, per-instance constants,
jumps) agrees with independent computations.  No kernel is launched."""
import ctypes as C
import math
from fractions import Fraction
import os
import re

import pytest

import inputs
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsaprng.h")


@pytest.fixture(scope="module")
def R():
    from paper_1811_11629_amd import rsaprng
    rsaprng.lib()
    return rsaprng


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsaprng_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(R):
    names = declared_functions()
    assert len(names) >= 30
    lib = C.CDLL(R.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows all of them
    assert not [n for n in names if n not in R._SIGS]


def test_version_and_strerror(R):
    assert "gfx950" in R.rsaprng_version()
    for code in range(0, -15, -1):
        assert R.rsaprng_strerror(code) not in ("", "unknown status")


def test_params_constants(R):
    insts = [inputs.config1()] + inputs.config2(8) + inputs.edge_instances()
    for i in insts:
        P = R.rsaprng_params_init(i.p, i.q, i.e, i.m0, 1)
        n = i.n
        assert P.n == n and P.p == i.p and P.q == i.q and P.e == i.e
        assert (P.ninv * n) % (1 << 32) == (1 << 32) - 1            # -n^-1 mod 2^32
        assert P.ce == pow(1 << 64, i.e, n)                         # R^e mod n
        assert P.nd == float(n)                                     # RN(n)
        assert P.pinv == 1.0 / i.p and P.qinv == 1.0 / i.q
        assert int(P.qinvp) == pow(i.q, -1, i.p)
        assert int(P.kp) == (1 << 32) % i.p and int(P.kq) == (1 << 32) % i.q
        assert P.nrcp == 1.0 / float(n)
        # split constants: K = hi + lo, hi a multiple of 2^17, lo < 2^17, quo = RN(K RN(1/P))
        for K, P_, lo, hi, quo in (((1 << 32) % i.p, i.p, P.kp_lo, P.kp_hi, P.kp_quo),
                                   ((1 << 32) % i.q, i.q, P.kq_lo, P.kq_hi, P.kq_quo),
                                   (pow(i.q, -1, i.p), i.p, P.gp_lo, P.gp_hi, P.gp_quo)):
            assert int(lo) + int(hi) == K and int(hi) % (1 << 17) == 0 and 0 <= lo < (1 << 17)
            assert quo == float(K) * (1.0 / P_)
        # nrcp + nrcp_lo approximates 1/nd far beyond double precision
        err = (Fraction(P.nrcp) + Fraction(P.nrcp_lo)) * Fraction(P.nd) - 1
        assert abs(err) < Fraction(1, 1 << 100)


def test_params_validation_codes(R):
    c1 = inputs.config1()
    cases = [
        ((c1.p, c1.p, 3, 1, 1), -2),
        ((c1.p, c1.q, 2, 1, 1), -4),
        ((c1.p, c1.q, 0, 1, 1), -4),
        ((c1.p, (1 << 31) - 1, 3, 1, 1), -3),
        ((c1.p, 1 << 32, 3, 1, 1), -3),
        ((c1.p, c1.q + 2 if not inputs.is_prime32(c1.q + 2) else c1.q + 4, 3, 1, 1), None),
        ((c1.p, c1.q, c1.e, c1.n, 1), -5),
        ((c1.p, c1.q, c1.e, 5, 0), -5),
        ((c1.p, c1.q, c1.e, 5, oracle.Q), -5),
    ]
    for args, code in cases:
        if code is None:
            with pytest.raises(R.RsaprngError) as ei:
                R.rsaprng_params_init(*args)
            assert ei.value.code in (-1, -4)
            continue
        with pytest.raises(R.RsaprngError) as ei:
            R.rsaprng_params_init(*args)
        assert ei.value.code == code, (args, ei.value.code)
    # the library's rule agrees with the oracle's on many (p, q, e)
    ps = [i.p for i in inputs.config3(16)] + [i.q for i in inputs.config2(16)]
    for a_ in ps[:12]:
        for b_ in ps[12:24]:
            for e in (1, 3, 5, 7, 9, 15, 17, 257, 65537):
                lib_ok = True
                try:
                    R.rsaprng_params_init(a_, b_, e, 1, 1)
                except R.RsaprngError:
                    lib_ok = False
                assert lib_ok == (oracle.check_params(a_, b_, e) == 0)


def test_library_miller_rabin(R):
    for x in list(range(2 ** 31, 2 ** 31 + 20000)) + [3215031751, oracle.Q, 2 ** 61 - 1,
                                                      4294967291 * 4294967279]:
        assert R.rsaprng_is_prime(x) == oracle.is_prime(x)


def test_library_jumps_match_oracle(R):
    for s0 in (1, 12345, oracle.Q - 1):
        for k in (0, 1, 2, 1000, 1 << 20, (1 << 40) + 17, (1 << 64) - 1):
            assert R.rsaprng_skip_at(s0, k) == oracle.skip(s0, k)
        for b in (0, 1, 2, 3, 12345, 1 << 40):
            assert R.rsaprng_block_seed(s0, b) == oracle.block_seed(s0, b)


def test_no_fallback_without_library(tmp_path, monkeypatch):
    # the binding raises rather than computing anything when the library is absent
    from paper_1811_11629_amd import rsaprng
    monkeypatch.setattr(rsaprng, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(rsaprng, "_lib", None)
    with pytest.raises(ImportError):
        rsaprng.lib()
