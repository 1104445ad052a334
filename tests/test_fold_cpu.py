"""The split reduction H K mod P used by the CRT kernels is exact.

For a constant 0 <= K < P < 2^32 split as K = hi + lo (hi a multiple of 2^17,
lo < 2^17) with quo = RN(K RN(1/P)), and an integer |H| < 2^35,

    fold(H) = fma(H, lo, fma(-rint(H quo), P, H hi))

equals H K - qt P for an integer qt and lies in (-P, P).  Checked on the host CPU
(hardware fma, the same sequence of binary64 operations the kernels issue)
against exact integer arithmetic, on random operands and on the extremes of the
stated ranges (H = +-(2^35 - 1), K = P - 1, P near 2^31 and 2^32).
"""
import os
import subprocess
import tempfile

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
static uint64_t st = 0x9e3779b97f4a7c15ull;
static uint64_t nxt(void) {  /* SplitMix64 */
  uint64_t z = (st += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double fold(double H, double P, double lo, double hi, double quo) {
  double qt = rint(H * quo);
  return fma(H, lo, fma(-qt, P, H * hi));
}
int main(int argc, char** argv) {
  long N = atol(argv[1]), bad = 0;
  for (long i = 0; i < N; ++i) {
    uint64_t P = (nxt() >> 32) | (1ull << 31);
    if (i % 5 == 0) P = (i & 1) ? 0xffffffffull : 0x80000001ull;
    uint64_t K = nxt() % P;
    if (i % 7 == 0) K = P - 1;
    int64_t lim = (1ll << 35) - 1;
    int64_t H = (int64_t)(nxt() % (2 * (uint64_t)lim + 1)) - lim;
    if (i % 11 == 0) H = (i & 2) ? lim : -lim;
    double Pd = (double)P, pinv = 1.0 / Pd;
    double lo = (double)(K & ((1ull << 17) - 1)), hi = (double)(K - (K & ((1ull << 17) - 1)));
    double quo = (double)K * pinv;
    double r = fold((double)H, Pd, lo, hi, quo);
    __int128 exact = (__int128)H * (__int128)K;
    __int128 rr = (__int128)r;
    int ok = (double)rr == r && rr > -(__int128)P && rr < (__int128)P &&
             ((exact - rr) % (__int128)P) == 0;
    if (!ok) {
      if (bad < 5) printf("bad H=%lld K=%llu P=%llu r=%.17g\n", (long long)H,
                          (unsigned long long)K, (unsigned long long)P, r);
      ++bad;
    }
  }
  printf("checked %ld, %ld failures\n", N, bad);
  return bad != 0;
}
"""


def test_split_fold_is_exact():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "f.c")
        exe = os.path.join(d, "f")
        with open(src, "w") as f:
            f.write(SRC)
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-mfma",
                               "-o", exe, src, "-lm"])
        r = subprocess.run([exe, "20000000"], capture_output=True, text=True)
        print(r.stdout)
        assert r.returncode == 0, r.stdout
        assert " 0 failures" in r.stdout
