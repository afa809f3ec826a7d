// Host-side check of the library's 64-bit modular arithmetic against 128-bit
// integer division, on random and edge-case operands for primes up to 2^61.
#include <stdio.h>
#include <stdlib.h>
#include <math.h>

#include "../../paper_2605_17222_amd/csrc/modarith.hpp"

typedef unsigned __int128 u128;
using namespace ckks;

static uint64_t s = 0x12345678abcdefull;
static uint64_t rnd() {
  s ^= s << 13; s ^= s >> 7; s ^= s << 17;
  return s;
}

int main() {
  const uint64_t qs[] = {1073692673ull, 1125899906826241ull, 1152921504606584833ull % (1ull << 60) | 1,
                         2305843009213554689ull, 1099511922689ull, 65537ull};
  long fails = 0, checks = 0;
  for (uint64_t q : qs) {
    const u128 r = (~(u128)0) / q;
    uint64_t qinv = q;
    for (int i = 0; i < 6; ++i) qinv *= 2 - q * qinv;
    const uint64_t qn = 0 - qinv;
    for (int it = 0; it < 200000; ++it) {
      uint64_t a = rnd(), b = rnd() % q, w = rnd() % q;
      if (it < 4) { a = it < 2 ? 0 : ~0ull; b = it & 1 ? q - 1 : 0; w = q - 1; }
      // mul_wide
      U128 m = mul_wide(a, b);
      u128 ref = (u128)a * b;
      fails += (m.lo != (uint64_t)ref || m.hi != (uint64_t)(ref >> 64));
      // shoup: any a < 2^64
      uint64_t wp = (uint64_t)(((u128)w << 64) / q);
      uint64_t sl = shoup_lazy(a, w, wp, q);
      fails += !(sl < 2 * q && sl % q == (uint64_t)((u128)a * w % q));
      // barrett128 on any 128-bit value
      U128 x = {rnd(), rnd()};
      if (it % 3 == 0) x.hi %= q;
      u128 xv = ((u128)x.hi << 64) | x.lo;
      fails += barrett128(x, q, (uint64_t)r, (uint64_t)(r >> 64)) != (uint64_t)(xv % q);
      // redc for x < q 2^64
      U128 y = {rnd(), rnd() % q};
      u128 yv = ((u128)y.hi << 64) | y.lo;
      uint64_t rr = redc(y, q, qn);
      // rr * 2^64 == y mod q
      fails += !(rr < q && (uint64_t)((((u128)rr << 64) % q)) == (uint64_t)(yv % q));
      checks += 4;
    }
  }
  // exact FP64 arithmetic for q < 2^46: |x| <= 16 q, w in [0, q)
  const uint64_t fq[] = {1099511922689ull, 1073692673ull, 70368744161281ull, 35184372088321ull};
  for (uint64_t q : fq) {
    const double qd = (double)q, qi = 1.0 / qd;
    for (int it = 0; it < 300000; ++it) {
      const uint64_t w = rnd() % q;
      const double wd = (double)w, wq = wd / qd;
      const int64_t lim = (int64_t)16 * (int64_t)q;
      int64_t x = (int64_t)(rnd() % (2 * (uint64_t)lim)) - lim;
      if (it < 3) x = it == 0 ? lim - 1 : (it == 1 ? -lim + 1 : 0);
      const double r = fp_mulmod((double)x, wd, wq, qd);
      // r must be an exact integer with r = x*w mod q and |r| <= 1.07 q
      const __int128 ref = ((__int128)x * (__int128)w) % (__int128)q;
      const __int128 diff = (__int128)(int64_t)r - ref;
      fails += (r != (double)(int64_t)r) || (diff % (__int128)q != 0) || (fabs(r) > 0.75 * qd);
      const double rr = fp_reduce((double)x, qd, qi);
      fails += (((__int128)(int64_t)rr - x) % (__int128)q != 0) || fabs(rr) > 0.5 * qd + 1;
      const uint64_t c = fp_canon((double)x, qd, qi);
      __int128 xm = x % (__int128)q;
      if (xm < 0) xm += q;
      fails += c != (uint64_t)xm;
      const uint64_t u = rnd() % q;
      fails += u64_to_d(u) != (double)u;
      checks += 4;
    }
  }
  // 30-bit column sums of a basis-conversion inner product: y_j, c_j < 2^60
  for (int it = 0; it < 200000; ++it) {
    uint32_t y0[16], y1[16], c2[16][2];
    uint64_t c[16];
    u128 ref = 0;
    for (int j = 0; j < 16; ++j) {
      uint64_t y = rnd() >> 4, cj = rnd() >> 4;
      if (it < 2) y = cj = (1ull << 60) - 1;  // largest operands
      y0[j] = (uint32_t)(y & ((1ull << 30) - 1));
      y1[j] = (uint32_t)(y >> 30);
      c[j] = cj;
      c2[j][0] = (uint32_t)(cj & ((1ull << 30) - 1));
      c2[j][1] = (uint32_t)(cj >> 30);
      if (j < 9 || it % 2) ref += (u128)y * cj;
    }
    const U128 d = (it % 2) ? dot_split30<16>(y0, y1, c2) : dot_split30<9>(y0, y1, c2);
    fails += d.lo != (uint64_t)ref || d.hi != (uint64_t)(ref >> 64);
    checks += 1;
  }
  printf("%ld checks, %ld failures\n", checks, fails);
  return fails ? 1 : 0;
}
