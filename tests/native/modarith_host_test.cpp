// Host-side check of the library's 64-bit modular arithmetic against 128-bit
// integer division, on random and edge-case operands for primes up to 2^61.
#include <stdio.h>
#include <stdlib.h>

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
  printf("%ld checks, %ld failures\n", checks, fails);
  return fails ? 1 : 0;
}
