"""The reciprocal-based quotient used by the kernels equals IEEE division.

r = RN(cd / nd) for 0 <= cd <= nd, nd = RN(n) with 2^62 <= n < 2^64, computed as
q0 = RN(cd y + RN(cd yl)), q1 = RN(q0 + (cd - q0 nd) y) with y = RN(1/nd) and
yl = RN(RN(1 - nd y) y) its low part (q0 within one ulp, one Markstein
correction).  Checked on the host CPU (hardware fma) against the IEEE quotient
on random pairs over the whole range of n, on the edges of that range, and on
pairs whose exact quotient lies next to a rounding midpoint.  The same sequence of operations runs on the
GPU; the GPU parity tests compare its r_k bit-exactly with the oracle's IEEE
division.
"""
import os
import subprocess
import tempfile

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include <stdlib.h>
static uint64_t st = 0x243f6a8885a308d3ull;
static uint64_t nxt(void) {  /* SplitMix64 */
  uint64_t z = (st += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double quot(double cd, double nd, double y, double yl) {
  double q0 = fma(cd, y, cd * yl);
  return fma(fma(-q0, nd, cd), y, q0);
}
int main(int argc, char** argv) {
  long N = atol(argv[1]);
  long bad = 0, mid = 0;
  for (long i = 0; i < N; ++i) {
    static const uint64_t edge[] = {(1ull << 62) + 1, (1ull << 63) - 1, (1ull << 63) + 1,
                                    ~0ull, (1ull << 62) + (1ull << 10) + 1, ~0ull - (1ull << 11)};
    uint64_t n = nxt();
    if (n < (1ull << 62)) n |= 1ull << 62;
    if (i % 97 == 0) n = edge[(i / 97) % 6];
    n |= 1;
    double nd = (double)n, y = 1.0 / nd, yl = fma(-y, nd, 1.0) * y;
    uint64_t c;
    switch (i % 4) {
      case 0: c = nxt() % n; break;
      case 1: c = n - 1 - (nxt() % 100000); break;
      case 2: c = nxt() % (1ull << (nxt() % 64 + 1)); break;
      default: c = nxt() % n;
    }
    double cd = (double)c;
    double want = cd / nd, got = quot(cd, nd, y, yl);
    if (memcmp(&want, &got, 8)) { if (bad < 5) printf("bad %llu %llu\n", (unsigned long long)c, (unsigned long long)n); ++bad; }
    /* numerator next to a rounding midpoint of the quotient */
    double q = ldexp((double)(nxt() >> 11), -53 - (int)(nxt() % 20));
    double up = nextafter(q, 2.0);
    double m = q + (up - q) / 2.0;  /* not representable: the rounded midpoint */
    double cm = m * nd;
    for (int d = -2; d <= 2; ++d) {
      double cdm = cm;
      for (int s = 0; s < (d < 0 ? -d : d); ++s) cdm = nextafter(cdm, d < 0 ? 0.0 : 1e300);
      if (cdm > nd || cdm < 0) continue;
      double w2 = cdm / nd, g2 = quot(cdm, nd, y, yl);
      ++mid;
      if (memcmp(&w2, &g2, 8)) { if (bad < 5) printf("bad-mid %a %a\n", cdm, nd); ++bad; }
    }
  }
  printf("checked %ld random, %ld near-midpoint, %ld mismatches\n", N, mid, bad);
  return bad != 0;
}
"""


def test_reciprocal_quotient_equals_ieee_division():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "q.c")
        exe = os.path.join(d, "q")
        with open(src, "w") as f:
            f.write(SRC)
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-mfma",
                               "-o", exe, src, "-lm"])
        r = subprocess.run([exe, "20000000"], capture_output=True, text=True)
        print(r.stdout)
        assert r.returncode == 0, r.stdout
        assert "0 mismatches" in r.stdout
