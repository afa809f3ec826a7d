// 64-bit modular arithmetic on the gfx950 vector ALU.
//
// Residues are uint64 below primes q < 2^61.  There is no 64x64->128 multiply
// instruction: a full product is four 32x32->64 multiply-adds
// (v_mad_u64_u32).  Three reductions are used, each where it is cheapest:
//  * Shoup multiplication by a constant w with w' = floor(w 2^64 / q) (NTT
//    twiddles, scaling constants): result in [0, 2q).
//  * Montgomery REDC of a 128-bit sum x < q 2^64 (basis conversion, whose
//    constants are stored premultiplied by 2^64): x 2^-64 mod q.
//  * Barrett reduction of any 128-bit value with floor(2^128 / q) (key-switch
//    and plaintext inner products, whose operands are both data).
// Lazy (non-canonical) intermediate ranges are documented at each use.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckks {

struct U128 {
  uint64_t lo, hi;
};

// Full 64x64 -> 128 product from four 32x32 -> 64 multiply-adds.
__host__ __device__ __forceinline__ U128 mul_wide(uint64_t a, uint64_t b) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);          // < 2^64
  const uint64_t u = (uint64_t)a1 * b0 + (uint32_t)t;          // < 2^64
  U128 r;
  r.hi = (uint64_t)a1 * b1 + ((t >> 32) + (u >> 32));
  r.lo = (u << 32) | (uint32_t)p00;
  return r;
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return mul_wide(a, b).hi; }

__host__ __device__ __forceinline__ void add128(U128& acc, U128 v) {
  acc.lo += v.lo;
  acc.hi += v.hi + (acc.lo < v.lo ? 1 : 0);
}

__host__ __device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t q) { return x >= q ? x - q : x; }

__host__ __device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }
__host__ __device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

// a * w mod q in [0, 2q) for any a < 2^64, w < q, wp = floor(w 2^64 / q).
__host__ __device__ __forceinline__ uint64_t shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  return a * w - mulhi64(a, wp) * q;
}
__host__ __device__ __forceinline__ uint64_t shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  return csub(shoup_lazy(a, w, wp, q), q);
}

// x 2^-64 mod q for x < q 2^64, qinv_neg = -q^-1 mod 2^64; result canonical.
__host__ __device__ __forceinline__ uint64_t redc(U128 x, uint64_t q, uint64_t qinv_neg) {
  const uint64_t m = x.lo * qinv_neg;
  const uint64_t t = x.hi + mulhi64(m, q) + (x.lo != 0 ? 1 : 0);
  return csub(t, q);
}

// x mod q for any x < 2^128, with (r_hi, r_lo) = floor(2^128 / q).
// qhat = floor(x r / 2^128) satisfies x/q - 2 < qhat <= x/q, so x - qhat q is
// in [0, 2q) and is computed modulo 2^64.
__host__ __device__ __forceinline__ uint64_t barrett128(U128 x, uint64_t q, uint64_t r_lo, uint64_t r_hi) {
  const uint64_t c0 = mulhi64(x.lo, r_lo);
  const U128 p1 = mul_wide(x.lo, r_hi);
  const U128 p2 = mul_wide(x.hi, r_lo);
  uint64_t s = p1.lo + c0;
  uint64_t carry = s < c0 ? 1 : 0;
  s += p2.lo;
  carry += s < p2.lo ? 1 : 0;
  const uint64_t qhat = x.hi * r_hi + p1.hi + p2.hi + carry;
  return csub(x.lo - qhat * q, q);
}

// ---- exact FP64 arithmetic for primes q < 2^46 ----------------------------
// Residues are doubles holding exact integers.  A product x*w (0 <= w < q) is
// reduced with an FMA two-product, so the remainder is exact:
//   t = rint(x * fl(w/q)),  h + l = t*q exactly,  r = fl(x*w - h) - l.
// |fl(x fl(w/q)) - x w/q| <= |x| 2^-52, so for |x| <= 16 q < 2^50 we get
// |x w/q - t| <= 1/2 + 2^-2 and |r| <= 0.75 q; x*w - h = (x*w - t q) + l with
// |l| <= ulp(h)/2 <= 2^45, so it is an integer below 2^53 and the FMA that
// forms it is exact.

// x < 2^52 as a double: the bits of 2^52 with x as the significand are the
// double 2^52 + x (one OR into the high word), and subtracting 2^52 is exact.
__host__ __device__ __forceinline__ double u64_to_d(uint64_t x) {
  return __builtin_bit_cast(double, x | 0x4330000000000000ull) - 4503599627370496.0;
}

__host__ __device__ __forceinline__ double fp_mulmod(double x, double w, double wq, double q) {
  const double t = rint(x * wq);
  const double h = t * q;
  const double l = fma(t, q, -h);
  return fma(x, w, -h) - l;
}

// x * y mod q for two data operands (no precomputed quotient), q < 2^46,
// |x| <= 4 q, |y| <= q: h = fl(x y) and l = x y - h (exact, |l| <= ulp(h)/2
// <= 2^-53 4 q^2 < 2^-5 q) are the two-product; h/q < 4 q < 2^48, so
// t = rint(h fl(1/q)) is within 1/2 + 2^-4 of h/q and h - t q is an integer
// of magnitude below (1/2 + 2^-4) q: the FMA that forms it is exact; the
// result h - t q + l is congruent to x y and below 0.6 q in magnitude, exact
// as well.
__host__ __device__ __forceinline__ double fp_mulmod_var(double x, double y, double q, double qinv) {
  const double h = x * y;
  const double l = fma(x, y, -h);
  const double t = rint(h * qinv);
  return fma(-t, q, h) + l;
}

// |x| < 2^52 -> x mod q in [-q/2 - 1, q/2 + 1] (an exact FMA: the result is below q).
__host__ __device__ __forceinline__ double fp_reduce(double x, double q, double qinv) {
  return fma(-rint(x * qinv), q, x);
}

// |x| < 2^52 -> canonical residue in [0, q) as uint64 (the residue r is an
// integer below 2^52, so 2^52 + r is exact and its significand is r).
__host__ __device__ __forceinline__ uint64_t fp_canon(double x, double q, double qinv) {
  double r = fp_reduce(x, q, qinv);
  r = r < 0 ? r + q : r;
  r = r >= q ? r - q : r;
  return __builtin_bit_cast(uint64_t, r + 4503599627370496.0) & ((1ull << 52) - 1);
}

// sum_j y_j c_j for NS <= 16 terms with y_j, c_j < 2^60, from 30-bit halves
// (y_j = y1_j 2^30 + y0_j, c_j = c1_j 2^30 + c0_j): every partial product is below
// 2^60, so each of the four column sums stays below 2^64 and a term costs four
// 32x32+64 multiply-adds with no carry handling; the columns are combined
// once: c00 + (c01 + c10) 2^30 + c11 2^60 < 2^125.
// k[j] = {c0, c1}: the constant already split.
template <int NS>
__host__ __device__ __forceinline__ U128 dot_split30(const uint32_t* y0, const uint32_t* y1, const uint32_t (*k)[2]) {
  uint64_t c00 = 0, c01 = 0, c10 = 0, c11 = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const uint32_t k0 = k[j][0], k1 = k[j][1];
    c00 += (uint64_t)y0[j] * k0;
    c01 += (uint64_t)y0[j] * k1;
    c10 += (uint64_t)y1[j] * k0;
    c11 += (uint64_t)y1[j] * k1;
  }
  U128 acc = {c00, 0};
  add128(acc, U128{c01 << 30, c01 >> 34});
  add128(acc, U128{c10 << 30, c10 >> 34});
  add128(acc, U128{c11 << 60, c11 >> 4});
  return acc;
}

// Bit reversal of the low `bits` bits.
__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits) { return __brev(x) >> (32 - bits); }

// NTT-domain automorphism index.  With g the Galois element, position p of
// phi_g(a) holds a at position br((g (2 br(p) + 1) mod 2N - 1) / 2).
__device__ __forceinline__ uint32_t auto_index(uint32_t p, uint32_t g, int log_n) {
  const uint32_t l = bitrev(p, log_n);
  const uint32_t e = (uint32_t)(((uint64_t)g * (2u * l + 1u)) & ((2u << log_n) - 1u));
  return bitrev((e - 1u) >> 1, log_n);
}

// Packed narrow limbs are runs of kPackChunk coefficients: the run's 32-bit
// low words, then its 8-bit high bytes (5 kPackChunk bytes), so one limb is a
// single contiguous stream.
constexpr size_t kPackChunk = 256;

#ifdef __HIPCC__
// Limb l (prime pr) of a polynomial at `poly`, stored packed (the limb starts
// at byte pr.pk_off; a narrow prime's limb is in runs as above) or as
// [limbs][N] 64-bit words.  Both are uniform over a block whose limb index is
// uniform, so a kernel branches once on `narrow` and then issues straight-line
// loads.
struct LimbRef {
  const uint8_t* b;  // first byte of the limb
  bool narrow;       // 32 + 8-bit planes (else N 64-bit words)
};
template <typename PrimeT>  // the library's per-prime table entry (pk_off, narrow)
__device__ __forceinline__ size_t limb_off(int l, size_t n, bool packed, const PrimeT& pr) {
  return packed ? (size_t)pr.pk_off : (size_t)l * n * 8;
}
template <typename PrimeT>
__device__ __forceinline__ LimbRef limb_ref(const void* poly, int l, size_t n, bool packed, const PrimeT& pr) {
  return {reinterpret_cast<const uint8_t*>(poly) + limb_off(l, n, packed, pr), packed && pr.narrow};
}
// Word p of a limb; non-temporal loads, these operands are read once per launch.
template <bool NARROW>
__device__ __forceinline__ uint64_t ld_word(const uint8_t* b, size_t p, size_t n) {
  if constexpr (NARROW) {
    const uint8_t* c = b + (p / kPackChunk) * (5 * kPackChunk);
    const size_t r = p % kPackChunk;
    const uint64_t lo = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(c) + r);
    const uint64_t hi = __builtin_nontemporal_load(c + 4 * kPackChunk + r);
    return lo | (hi << 32);
  } else {
    return __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(b) + p);
  }
}
#endif

}  // namespace ckks
