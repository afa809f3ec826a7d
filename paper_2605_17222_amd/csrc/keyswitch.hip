// HBM-bound element-wise kernels of the LT:
//  * hoisted key-switch inner product (x, y) = sum_b d_b (swk_b0, swk_b1)
//    over the PQ limbs, several keys per digit read, with the add of
//    Algorithm 2 lines 4/9/17 and the automorphism phi_r applied on write;
//  * plaintext multiply-accumulate into several accumulators at once
//    (Algorithm 2 lines 12 and 14);
//  * NTT-domain automorphism as a gather (eq. (7)), with an optional add.
//
// The automorphism is written as a scatter: the value computed at position p
// goes to phi's position of p, pi_{-r}(p).  Eq. (8) shows that an aligned
// block of d_p positions maps onto one aligned block of d_p positions for any
// power of two d_p, so a wavefront of 64 consecutive positions writes one
// aligned 512-byte block: the stores stay coalesced.
//
// Products of two data operands are accumulated as exact 128-bit sums and
// reduced once per output with Barrett's floor(2^128 / q); the number of terms
// t satisfies t q^2 < 2^128 (the host splits larger sums).
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kXcds = 8;  // accelerator complex dies of the device, each with its own L2
static_assert(kKsMacAlign == kThreads * kXcds, "ksmac grid: whole workgroups per XCD");

// Operands read once per launch (keys, digits, plaintexts, products) are
// loaded with the non-temporal hint: they stream through without displacing
// cached data, which lifts the achieved read bandwidth on gfx950.  Outputs
// that the next kernel streams the same way (the rotation products read by
// the multiply-accumulate, the accumulators, the automorphism's result) are
// stored non-temporally too: measured, that speeds up the reader (the MAC
// by about 8%).  The gather's accumulators, which the ModDown that follows
// reads right away, use ordinary stores.
__device__ __forceinline__ uint64_t ld_nt(const uint64_t* p) { return __builtin_nontemporal_load(p); }

// Bytes between the polynomials of a key [beta_max][2] (index 2 b + s):
// packed polynomials of pk_bytes each, or [kmax][N] words each.
__device__ __forceinline__ size_t poly_stride(bool packed, uint64_t pk_bytes, int kmax, size_t n) {
  return packed ? pk_bytes : (size_t)kmax * n * 8;
}

// Key k's limb l of polynomials (2 b, 2 b + 1), b < kbeta <= MB, at position p.
template <bool NARROW, int MB>
__device__ __forceinline__ void ld_key(uint64_t (&k0)[MB], uint64_t (&k1)[MB], const uint8_t* base, size_t stride,
                                       int kbeta, size_t p, size_t n) {
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    if (b < kbeta) {
      k0[b] = ld_word<NARROW>(base + (2 * b) * stride, p, n);
      k1[b] = ld_word<NARROW>(base + (2 * b + 1) * stride, p, n);
    }
  }
}

// The keys of a key-switch launch against the digits d (limb l, position p):
// key k's product with digit set i is written at phi_k's position of p.  MB
// is the launch's largest digit count (kbeta), which sizes the register
// arrays: fewer registers at the common digit counts, higher occupancy.
template <int NDIG, int MB, bool PACKED, bool NARROW>
__device__ __forceinline__ void ks_keys(const KsArgs& a, const PrimeDev& pr, int l, uint32_t p, size_t n, int log_n,
                                        const uint64_t (&d)[NDIG][MB], const uint64_t (&addv)[NDIG]) {
  const uint64_t q = pr.q;
  const size_t lo = limb_off(l, n, PACKED, pr);
  const size_t stride = poly_stride(PACKED, a.pk_poly_bytes, a.kmax, n);
  // key k + 1 is loaded while key k's products are formed (the stores that
  // follow do not delay those loads)
  uint64_t k0[MB] = {}, k1[MB] = {}, n0[MB] = {}, n1[MB] = {};
  ld_key<NARROW, MB>(k0, k1, reinterpret_cast<const uint8_t*>(a.key[0]) + lo, stride, a.kbeta, p, n);
  for (int k = 0; k < a.nkeys; ++k) {
    if (k + 1 < a.nkeys)
      ld_key<NARROW, MB>(n0, n1, reinterpret_cast<const uint8_t*>(a.key[k + 1]) + lo, stride, a.kbeta, p, n);
    const size_t o = (size_t)l * n + auto_index(p, a.gal_inv[k], log_n);
#pragma unroll
    for (int i = 0; i < NDIG; ++i) {
      uint64_t* oa = a.out_a[i][k];
      if (!oa || l >= a.K[i]) continue;
      uint64_t* ob = a.out_b[i][k];
      U128 x = {0, 0}, y = {0, 0};
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        if (b < a.beta[i]) {
          add128(x, mul_wide(d[i][b], k0[b]));
          add128(y, mul_wide(d[i][b], k1[b]));
        }
      }
      __builtin_nontemporal_store(add_mod(barrett128(x, q, pr.r_lo, pr.r_hi), addv[i], q), oa + o);
      __builtin_nontemporal_store(barrett128(y, q, pr.r_lo, pr.r_hi), ob + o);
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      k0[b] = n0[b];
      k1[b] = n1[b];
    }
  }
}

// PACKED: every key of the launch is stored packed.  Limb l is uniform over a
// block, so the narrow/wide choice is made once, outside the key loop.
template <int NDIG, int MB, bool PACKED>
__global__ void __launch_bounds__(kThreads)
    ks_kernel(KsArgs a, const PrimeDev* __restrict__ primes, int log_n, int alpha) {
  const size_t n = (size_t)1 << log_n;
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const PrimeDev& pr = primes[l];
  const uint64_t q = pr.q;

  uint64_t d[NDIG][MB], addv[NDIG];
#pragma unroll
  for (int i = 0; i < NDIG; ++i) {
    addv[i] = 0;
    if (l >= a.K[i]) continue;  // this digit set's level has fewer limbs
#pragma unroll
    for (int b = 0; b < MB; ++b)
      if (b < a.beta[i]) d[i][b] = ld_nt(a.digits[i] + ((size_t)b * a.K[i] + l) * n + p);
    if (a.add[i]) {
      if (a.add_pscaled[i])
        addv[i] = (l < alpha) ? 0 : shoup(ld_nt(a.add[i] + (size_t)(l - alpha) * n + p), pr.pmod, pr.pmod_sh, q);
      else
        addv[i] = ld_nt(a.add[i] + (size_t)l * n + p);
    }
  }
  if constexpr (PACKED) {
    if (pr.narrow)
      ks_keys<NDIG, MB, true, true>(a, pr, l, p, n, log_n, d, addv);
    else
      ks_keys<NDIG, MB, true, false>(a, pr, l, p, n, log_n, d, addv);
  } else {
    ks_keys<NDIG, MB, false, false>(a, pr, l, p, n, log_n, d, addv);
  }
}

template <int NDIG, int MB>
hipError_t launch_ks_mb(const ckks_params* P, const KsArgs& a, hipStream_t s) {
  dim3 grid(P->n / kThreads, a.maxK);
  if (a.key_packed)
    hipLaunchKernelGGL((ks_kernel<NDIG, MB, true>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, P->alpha);
  else
    hipLaunchKernelGGL((ks_kernel<NDIG, MB, false>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, P->alpha);
  return hipGetLastError();
}

template <int NDIG>
hipError_t launch_ks(const ckks_params* P, const KsArgs& a, hipStream_t s) {
  static_assert(kMaxBeta == 4, "one instantiation per digit count");
  switch (a.kbeta) {
    case 1: return launch_ks_mb<NDIG, 1>(P, a, s);
    case 2: return launch_ks_mb<NDIG, 2>(P, a, s);
    case 3: return launch_ks_mb<NDIG, 3>(P, a, s);
    case 4: return launch_ks_mb<NDIG, 4>(P, a, s);
    default: return hipErrorInvalidValue;
  }
}

// One-to-one launches (key k with digit set k only, as in the separate
// giant-step rotations of plain BSGS): each key's digits are loaded inside
// the key loop, so only one digit set is live and occupancy stays high.  The
// operands of key k + 1 are loaded while key k's products are formed.
template <int MB>
struct DiagOps {
  uint64_t k0[MB], k1[MB], d[MB], add;
};

template <bool NARROW, int MB>
__device__ __forceinline__ void diag_load(DiagOps<MB>& o, const KsArgs& a, int k, int l, uint32_t p, size_t n,
                                          size_t lo, size_t stride, int alpha) {
  const int beta = a.beta[k];
  ld_key<NARROW, MB>(o.k0, o.k1, reinterpret_cast<const uint8_t*>(a.key[k]) + lo, stride, beta, p, n);
#pragma unroll
  for (int b = 0; b < MB; ++b)
    if (b < beta) o.d[b] = ld_nt(a.digits[k] + ((size_t)b * a.K[k] + l) * n + p);
  o.add = 0;
  if (a.add[k]) {
    if (a.add_pscaled[k])
      o.add = (l < alpha) ? 0 : ld_nt(a.add[k] + (size_t)(l - alpha) * n + p);
    else
      o.add = ld_nt(a.add[k] + (size_t)l * n + p);
  }
}

template <bool PACKED, bool NARROW, int MB>
__device__ __forceinline__ void diag_keys(const KsArgs& a, const PrimeDev& pr, int l, uint32_t p, size_t n, int log_n,
                                          int alpha) {
  const uint64_t q = pr.q;
  const size_t lo = limb_off(l, n, PACKED, pr);
  const size_t stride = poly_stride(PACKED, a.pk_poly_bytes, a.kmax, n);
  // keys whose digit set has fewer limbs than l are skipped
  int k = 0;
  while (k < a.nkeys && (!a.out_a[k][k] || l >= a.K[k])) ++k;
  if (k == a.nkeys) return;
  DiagOps<MB> cur{}, nxt{};
  diag_load<NARROW, MB>(cur, a, k, l, p, n, lo, stride, alpha);
  while (k < a.nkeys) {
    int k2 = k + 1;
    while (k2 < a.nkeys && (!a.out_a[k2][k2] || l >= a.K[k2])) ++k2;
    if (k2 < a.nkeys) diag_load<NARROW, MB>(nxt, a, k2, l, p, n, lo, stride, alpha);
    const int beta = a.beta[k];
    U128 x = {0, 0}, y = {0, 0};
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b < beta) {
        add128(x, mul_wide(cur.d[b], cur.k0[b]));
        add128(y, mul_wide(cur.d[b], cur.k1[b]));
      }
    }
    uint64_t addv = cur.add;
    if (a.add[k] && a.add_pscaled[k] && l >= alpha) addv = shoup(addv, pr.pmod, pr.pmod_sh, q);
    const size_t o = (size_t)l * n + auto_index(p, a.gal_inv[k], log_n);
    a.out_a[k][k][o] = add_mod(barrett128(x, q, pr.r_lo, pr.r_hi), addv, q);
    a.out_b[k][k][o] = barrett128(y, q, pr.r_lo, pr.r_hi);
    cur = nxt;
    k = k2;
  }
}

template <bool PACKED, int MB>
__global__ void __launch_bounds__(kThreads)
    ks_diag_kernel(KsArgs a, const PrimeDev* __restrict__ primes, int log_n, int alpha) {
  const size_t n = (size_t)1 << log_n;
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const PrimeDev& pr = primes[l];
  if constexpr (PACKED) {
    if (pr.narrow)
      diag_keys<true, true, MB>(a, pr, l, p, n, log_n, alpha);
    else
      diag_keys<true, false, MB>(a, pr, l, p, n, log_n, alpha);
  } else {
    diag_keys<false, false, MB>(a, pr, l, p, n, log_n, alpha);
  }
}

template <int MB>
hipError_t launch_diag_mb(const ckks_params* P, const KsArgs& a, hipStream_t s) {
  dim3 grid(P->n / kThreads, a.maxK);
  if (a.key_packed)
    hipLaunchKernelGGL((ks_diag_kernel<true, MB>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, P->alpha);
  else
    hipLaunchKernelGGL((ks_diag_kernel<false, MB>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, P->alpha);
  return hipGetLastError();
}

// The gather's key loop (limb l, output position p): the operands of key
// k + 1 (its limbs, digits and u0 at its source position) are loaded while
// key k's products are formed.
template <int MB>
struct GatherOps {
  uint64_t k0[MB], k1[MB], d[MB], add;
};

template <bool NARROW, int MB>
__device__ __forceinline__ void gather_load(GatherOps<MB>& o, const KsGatherArgs& a, int k, int l, uint32_t p,
                                            size_t n, int log_n, size_t lo, size_t stride) {
  const uint32_t src = auto_index(p, a.gal[k], log_n);
  const size_t s = (size_t)l * n + src;
  ld_key<NARROW, MB>(o.k0, o.k1, reinterpret_cast<const uint8_t*>(a.key[k]) + lo, stride, a.beta, src, n);
#pragma unroll
  for (int b = 0; b < MB; ++b)
    if (b < a.beta) o.d[b] = ld_nt(a.digits[k] + (size_t)b * a.K * n + s);
  o.add = ld_nt(a.add[k] + s);
}

template <bool PACKED, bool NARROW, int MB>
__device__ __forceinline__ void gather_keys(const KsGatherArgs& a, const PrimeDev& pr, int l, uint32_t p, size_t n,
                                            int log_n, uint64_t& c0, uint64_t& c1) {
  const uint64_t q = pr.q;
  const size_t lo = limb_off(l, n, PACKED, pr);
  const size_t stride = poly_stride(PACKED, a.pk_poly_bytes, a.kmax, n);
  if (a.nk <= 0) return;
  GatherOps<MB> cur{}, nxt{};
  gather_load<NARROW, MB>(cur, a, 0, l, p, n, log_n, lo, stride);
  for (int k = 0; k < a.nk; ++k) {
    if (k + 1 < a.nk) gather_load<NARROW, MB>(nxt, a, k + 1, l, p, n, log_n, lo, stride);
    U128 x = {0, 0}, y = {0, 0};
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b < a.beta) {
        add128(x, mul_wide(cur.d[b], cur.k0[b]));
        add128(y, mul_wide(cur.d[b], cur.k1[b]));
      }
    }
    c0 = add_mod(c0, add_mod(barrett128(x, q, pr.r_lo, pr.r_hi), cur.add, q), q);
    c1 = add_mod(c1, barrett128(y, q, pr.r_lo, pr.r_hi), q);
    cur = nxt;
  }
}

template <bool PACKED, int MB>
__global__ void __launch_bounds__(kThreads)
    ks_gather_kernel(KsGatherArgs a, const PrimeDev* __restrict__ primes, int log_n) {
  const size_t n = (size_t)1 << log_n;
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const PrimeDev& pr = primes[l];
  const size_t o = (size_t)l * n + p;
  uint64_t c0 = a.c0[o], c1 = a.c1[o];
  if constexpr (PACKED) {
    if (pr.narrow)
      gather_keys<true, true, MB>(a, pr, l, p, n, log_n, c0, c1);
    else
      gather_keys<true, false, MB>(a, pr, l, p, n, log_n, c0, c1);
  } else {
    gather_keys<false, false, MB>(a, pr, l, p, n, log_n, c0, c1);
  }
  a.c0[o] = c0;
  a.c1[o] = c1;
}

template <int MB>
hipError_t launch_gather_mb(const ckks_params* P, const KsGatherArgs& a, hipStream_t s) {
  dim3 grid(P->n / kThreads, a.K);
  if (a.key_packed)
    hipLaunchKernelGGL((ks_gather_kernel<true, MB>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n);
  else
    hipLaunchKernelGGL((ks_gather_kernel<false, MB>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n);
  return hipGetLastError();
}

template <int NK>
struct MacOps {
  uint64_t a, b, f[NK];
};

// Index m's operands: (a_m, b_m) (for m = 0 with P c', the raw c' words) and
// the NK plaintext words (0 where a plaintext is absent).
template <int NK, bool PACKED, bool NARROW, typename PrimeT>
__device__ __forceinline__ void mac_load(MacOps<NK>& o, const MacArgs& a, const PrimeT& pr, int m, int l, size_t p,
                                         size_t n, int alpha, size_t fo) {
  const size_t off = (size_t)l * n + p;
  if (m == 0 && a.pscaled0) {
    const int lq = l + a.prime_off - alpha;
    o.a = lq < 0 ? 0 : ld_nt(a.a[0] + (size_t)lq * n + p);
    o.b = lq < 0 ? 0 : ld_nt(a.b[0] + (size_t)lq * n + p);
  } else {
    o.a = ld_nt(a.a[m] + off);
    o.b = ld_nt(a.b[m] + off);
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const uint64_t* __restrict__ fp = a.f[k][m];
    o.f[k] = 0;
    if (fp) {
      if constexpr (PACKED)
        o.f[k] = ld_word<NARROW>(reinterpret_cast<const uint8_t*>(fp) + fo, p, n);
      else
        o.f[k] = ld_nt(fp + off);  // the word offset the (a_m, b_m) loads use
    }
  }
}

// The m-outer loop of the MAC for one limb: (a_m, b_m) and the NK plaintexts
// of index m are folded into NK pairs of 128-bit accumulators while the
// operands of m + 1 are loaded, so few values are live and loads stay in
// flight across iterations.  fo: byte offset of the limb within each
// plaintext.
template <int NK, bool PACKED, bool NARROW, typename PrimeT>
__device__ __forceinline__ void mac_loop(const MacArgs& a, const PrimeT& pr, int l, size_t p, size_t n, int alpha,
                                         size_t fo, U128 (&x)[NK], U128 (&y)[NK]) {
  const uint64_t q = pr.q;
  if (a.nm <= 0) return;
  MacOps<NK> cur{}, nxt{};
  mac_load<NK, PACKED, NARROW>(cur, a, pr, 0, l, p, n, alpha, fo);
  for (int m = 0; m < a.nm; ++m) {
    if (m + 1 < a.nm) mac_load<NK, PACKED, NARROW>(nxt, a, pr, m + 1, l, p, n, alpha, fo);
    uint64_t av = cur.a, bv = cur.b;
    if (m == 0 && a.pscaled0) {
      // (a_0, b_0) = (P c0', P c1'): zero on the special primes.
      av = shoup(av, pr.pmod, pr.pmod_sh, q);
      bv = shoup(bv, pr.pmod, pr.pmod_sh, q);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      if (a.f[k][m]) {
        add128(x[k], mul_wide(av, cur.f[k]));
        add128(y[k], mul_wide(bv, cur.f[k]));
      }
    }
    if (m + 1 < a.nm) cur = nxt;
  }
}

// The MAC loop for packed plaintexts: two iterations unrolled (the packed
// loads take more registers, and a pipelined loop would cost a wave).
template <int NK, bool NARROW, typename PrimeT>
__device__ __forceinline__ void mac_loop_packed(const MacArgs& a, const PrimeT& pr, int l, size_t p, size_t n,
                                                int alpha, size_t fo, U128 (&x)[NK], U128 (&y)[NK]) {
  const uint64_t q = pr.q;
  const size_t off = (size_t)l * n + p;
#pragma unroll 2
  for (int m = 0; m < a.nm; ++m) {
    uint64_t av, bv;
    if (m == 0 && a.pscaled0) {
      // (a_0, b_0) = (P c0', P c1'): zero on the special primes.
      const int lq = l + a.prime_off - alpha;
      av = lq < 0 ? 0 : shoup(ld_nt(a.a[0] + (size_t)lq * n + p), pr.pmod, pr.pmod_sh, q);
      bv = lq < 0 ? 0 : shoup(ld_nt(a.b[0] + (size_t)lq * n + p), pr.pmod, pr.pmod_sh, q);
    } else {
      av = ld_nt(a.a[m] + off);
      bv = ld_nt(a.b[m] + off);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const uint64_t* __restrict__ fp = a.f[k][m];
      if (fp) {
        const uint64_t f = ld_word<NARROW>(reinterpret_cast<const uint8_t*>(fp) + fo, p, n);
        add128(x[k], mul_wide(av, f));
        add128(y[k], mul_wide(bv, f));
      }
    }
  }
}

// F_PACKED: the plaintexts are packed.  The unpacked instantiation holds the
// wide path only (the second path would cost registers and occupancy).
template <int NK, bool F_PACKED>
__global__ void __launch_bounds__(kThreads)
    mac_kernel(MacArgs a, const PrimeDev* __restrict__ primes, int log_n, int alpha) {
  const size_t n = (size_t)1 << log_n;
  const size_t p = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const PrimeDev& pr = primes[l + a.prime_off];
  const uint64_t q = pr.q;
  const size_t off = (size_t)l * n + p;
  const size_t fo = limb_off(l, n, F_PACKED, pr);

  U128 x[NK], y[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) x[k] = y[k] = U128{0, 0};
  if constexpr (F_PACKED) {
    if (pr.narrow)
      mac_loop_packed<NK, true>(a, pr, l, p, n, alpha, fo, x, y);
    else
      mac_loop_packed<NK, false>(a, pr, l, p, n, alpha, fo, x, y);
  } else {
    mac_loop<NK, false, false>(a, pr, l, p, n, alpha, fo, x, y);
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    uint64_t xr = barrett128(x[k], q, pr.r_lo, pr.r_hi);
    uint64_t yr = barrett128(y[k], q, pr.r_lo, pr.r_hi);
    if (a.accumulate) {
      xr = add_mod(xr, a.out0[k][off], q);
      yr = add_mod(yr, a.out1[k][off], q);
    }
    __builtin_nontemporal_store(xr, a.out0[k] + off);
    __builtin_nontemporal_store(yr, a.out1[k] + off);
  }
}

template <int NK>
hipError_t launch_mac(const ckks_params* P, const MacArgs& a, hipStream_t s) {
  dim3 grid(P->n / kThreads, a.K);
  if (a.f_packed)
    hipLaunchKernelGGL((mac_kernel<NK, true>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, P->alpha);
  else
    hipLaunchKernelGGL((mac_kernel<NK, false>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, P->alpha);
  return hipGetLastError();
}

// ---- middle key switch fused with the multiply-accumulate ------------------
// Thread (limb l, output position p) forms every term's (a_m, b_m) at p --
// read for unrotated terms, for rotated ones the key-switch product and add
// at the source position auto_index(p, gal) (a gather: eq. (8) keeps a
// wavefront's 64 positions in one aligned block) -- and folds it into NK
// pairs of 128-bit accumulators right away.  The operands of term m + 1 are
// loaded while term m is folded in; a key shared with the previous term is
// kept in registers instead of loaded again.
template <int NK, int MB>
struct KsMacOps {
  uint64_t k0[MB], k1[MB], d[MB], a, b, f[NK];
};

// Layouts: KN / FN, the keys' / plaintexts' limb l is packed narrow (32-bit
// and 8-bit planes); ko, ks: byte offset of limb l within a key polynomial
// and the bytes between the key's polynomials; fo: byte offset of limb l
// within a plaintext.
template <int NK, int MB, bool KN, bool FN>
__device__ __forceinline__ void ksmac_load(KsMacOps<NK, MB>& o, const KsMacArgs& a, int m, bool load_key, int l,
                                           uint32_t p, size_t n, int log_n, int alpha, size_t ko, size_t ks,
                                           size_t fo) {
  const int kj = a.key_of[m];
  const size_t off = (size_t)l * n + p;
  const int lq = l - alpha;  // Q-basis limb of a pscaled operand (none on the special primes)
  // both words are assigned on every path (values first, one store each), so
  // the operand structs stay in registers
  uint64_t va = 0, vb = 0;
  if (kj < 0) {
    if (a.pscaled[m]) {
      va = lq < 0 ? 0 : ld_nt(a.a[m] + (size_t)lq * n + p);
      vb = lq < 0 ? 0 : ld_nt(a.b[m] + (size_t)lq * n + p);
    } else {
      va = ld_nt(a.a[m] + off);
      vb = ld_nt(a.b[m] + off);
    }
  } else {
    const uint32_t src = auto_index(p, a.gal[kj], log_n);
    if (load_key) ld_key<KN, MB>(o.k0, o.k1, reinterpret_cast<const uint8_t*>(a.key[kj]) + ko, ks, a.beta, src, n);
    // digits and adds are read again by the other rotations of the launch:
    // ordinary loads, kept in L2 (the keys and plaintexts stream through)
#pragma unroll
    for (int b = 0; b < MB; ++b)
      if (b < a.beta) o.d[b] = a.digits[m][((size_t)b * a.K + l) * n + src];
    if (a.pscaled[m])
      va = lq < 0 ? 0 : a.a[m][(size_t)lq * n + src];
    else
      va = a.a[m][(size_t)l * n + src];
  }
  o.a = va;
  o.b = vb;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const uint64_t* __restrict__ fp = a.f[k][m];
    o.f[k] = fp ? ld_word<FN>(reinterpret_cast<const uint8_t*>(fp) + fo, p, n) : 0;
  }
}

// The fold of one limb.  FP (primes below 2^46): operands as exact doubles,
// every product reduced on its own (fp_mulmod_var), sums of at most 16 terms
// of magnitude below q stay exact; about a third of the integer path's
// instructions.  Otherwise 64 x 64 -> 128-bit products summed lazily and
// reduced with Barrett's floor(2^128 / q).
template <int NK, int MB, bool FP, bool PK, bool PF, bool NARROW>
__device__ __forceinline__ void ksmac_body(const KsMacArgs& a, const PrimeDev& pr, int l, uint32_t p, size_t n,
                                           int log_n, int alpha) {
  constexpr bool KN = PK && NARROW, FN = PF && NARROW;
  const size_t ko = limb_off(l, n, PK, pr), ks = poly_stride(PK, a.pk_poly_bytes, a.kmax, n);
  const size_t fo = limb_off(l, n, PF, pr);
  const uint64_t q = pr.q;
  const double qd = pr.qd, qi = pr.qinv_d;
  const double pm = (double)pr.pmod, pmq = pm * qi;  // P mod q (below 2^46 on this path) and P/q
  const size_t off = (size_t)l * n + p;
  U128 x[NK], y[NK];
  double xd[NK], yd[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    x[k] = y[k] = U128{0, 0};
    xd[k] = yd[k] = 0.0;
  }
  double kd0[MB] = {}, kd1[MB] = {};  // FP: the current key as doubles
  KsMacOps<NK, MB> cur{}, nxt{};
  if (a.nm > 0) ksmac_load<NK, MB, KN, FN>(cur, a, 0, true, l, p, n, log_n, alpha, ko, ks, fo);
  for (int m = 0; m < a.nm; ++m) {
    const bool new_key = a.key_of[m] >= 0 && (m == 0 || a.key_of[m - 1] != a.key_of[m]);
    if (m + 1 < a.nm) {
      // a key shared with term m stays in registers
      const bool same = a.key_of[m + 1] >= 0 && a.key_of[m + 1] == a.key_of[m];
      ksmac_load<NK, MB, KN, FN>(nxt, a, m + 1, !same, l, p, n, log_n, alpha, ko, ks, fo);
      if (!FP && same) {  // (the FP path keeps the current key as doubles)
#pragma unroll
        for (int b = 0; b < MB; ++b) {
          nxt.k0[b] = cur.k0[b];
          nxt.k1[b] = cur.k1[b];
        }
      }
    }
    if constexpr (FP) {
      double av, bv;
      if (a.key_of[m] < 0) {
        av = u64_to_d(cur.a);
        bv = u64_to_d(cur.b);
        if (a.pscaled[m]) {  // (P c0', P c1')
          av = fp_mulmod(av, pm, pmq, qd);
          bv = fp_mulmod(bv, pm, pmq, qd);
        }
      } else {
        if (new_key) {
#pragma unroll
          for (int b = 0; b < MB; ++b) {
            kd0[b] = u64_to_d(cur.k0[b]);
            kd1[b] = u64_to_d(cur.k1[b]);
          }
        }
        double u = 0.0, v = 0.0;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
          if (b < a.beta) {
            const double d = u64_to_d(cur.d[b]);
            u += fp_mulmod_var(d, kd0[b], qd, qi);
            v += fp_mulmod_var(d, kd1[b], qd, qi);
          }
        }
        double addv = u64_to_d(cur.a);
        if (a.pscaled[m]) addv = fp_mulmod(addv, pm, pmq, qd);
        // not reduced: |u| < 0.6 beta q <= 2.4 q and |addv| < q, within the
        // 4 q that fp_mulmod_var takes for its first operand
        av = u + addv;
        bv = v;
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        if (a.f[k][m]) {
          const double f = u64_to_d(cur.f[k]);
          xd[k] += fp_mulmod_var(av, f, qd, qi);
          yd[k] += fp_mulmod_var(bv, f, qd, qi);
        }
      }
    } else {
      uint64_t av, bv;
      if (a.key_of[m] < 0) {
        av = cur.a;
        bv = cur.b;
        if (a.pscaled[m]) {  // (P c0', P c1'): zero on the special primes
          av = shoup(av, pr.pmod, pr.pmod_sh, q);
          bv = shoup(bv, pr.pmod, pr.pmod_sh, q);
        }
      } else {
        U128 u = {0, 0}, v = {0, 0};
#pragma unroll
        for (int b = 0; b < MB; ++b) {
          if (b < a.beta) {
            add128(u, mul_wide(cur.d[b], cur.k0[b]));
            add128(v, mul_wide(cur.d[b], cur.k1[b]));
          }
        }
        uint64_t addv = cur.a;
        if (a.pscaled[m]) addv = shoup(addv, pr.pmod, pr.pmod_sh, q);
        av = add_mod(barrett128(u, q, pr.r_lo, pr.r_hi), addv, q);
        bv = barrett128(v, q, pr.r_lo, pr.r_hi);
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        if (a.f[k][m]) {
          add128(x[k], mul_wide(av, cur.f[k]));
          add128(y[k], mul_wide(bv, cur.f[k]));
        }
      }
    }
    if (m + 1 < a.nm) cur = nxt;
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    uint64_t xr, yr;
    if constexpr (FP) {
      xr = fp_canon(xd[k], qd, qi);
      yr = fp_canon(yd[k], qd, qi);
    } else {
      xr = barrett128(x[k], q, pr.r_lo, pr.r_hi);
      yr = barrett128(y[k], q, pr.r_lo, pr.r_hi);
    }
    if (a.accumulate) {
      xr = add_mod(xr, a.out0[k][off], q);
      yr = add_mod(yr, a.out1[k][off], q);
    }
    __builtin_nontemporal_store(xr, a.out0[k] + off);
    __builtin_nontemporal_store(yr, a.out1[k] + off);
  }
}

// Workgroup w of the launch runs on XCD w mod 8 (the dispatcher deals
// workgroups round-robin over the eight XCDs); numbering each XCD's
// workgroups consecutively gives an XCD whole limbs, so the digits and adds
// that a limb's rotations gather again stay in that XCD's L2.  The grid is
// (N / kThreads) x K with N / kThreads a multiple of 8.
// PK / PF: the keys / plaintexts of the launch are packed; a packed narrow
// limb (prime below 2^40, so on the FP64 path) is read from its planes.
template <int NK, int MB, bool PK, bool PF>
__global__ void __launch_bounds__(kThreads)
    ksmac_kernel(KsMacArgs a, const PrimeDev* __restrict__ primes, int log_n, int alpha) {
  const uint32_t w = blockIdx.y * gridDim.x + blockIdx.x;
  const uint32_t per_xcd = gridDim.x * gridDim.y / kXcds;
  const uint32_t v = (w % kXcds) * per_xcd + w / kXcds;
  const uint32_t p = (v % gridDim.x) * kThreads + threadIdx.x;
  const int l = (int)(v / gridDim.x);
  const PrimeDev& pr = primes[l];
  const size_t n = (size_t)1 << log_n;
  if (pr.fp) {
    if constexpr (PK || PF) {
      if (pr.narrow) {
        ksmac_body<NK, MB, true, PK, PF, true>(a, pr, l, p, n, log_n, alpha);
        return;
      }
      // With more than 6 accumulators, three bodies in one kernel make the
      // compiler keep the whole argument block in per-lane scratch; the wide
      // limbs of the FP64 path (primes between 2^40 and 2^46) then take the
      // integer body, which serves any prime.
      if constexpr (NK > 6) {
        ksmac_body<NK, MB, false, PK, PF, false>(a, pr, l, p, n, log_n, alpha);
        return;
      }
    }
    ksmac_body<NK, MB, true, PK, PF, false>(a, pr, l, p, n, log_n, alpha);
  } else {
    ksmac_body<NK, MB, false, PK, PF, false>(a, pr, l, p, n, log_n, alpha);
  }
}

template <int NK, int MB>
void launch_ksmac_mb(const ckks_params* P, const KsMacArgs& a, hipStream_t s) {
  dim3 grid(P->n / kThreads, a.K);
  if (a.key_packed && a.f_packed)
    hipLaunchKernelGGL((ksmac_kernel<NK, MB, true, true>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n,
                       P->alpha);
  else if (a.key_packed)
    hipLaunchKernelGGL((ksmac_kernel<NK, MB, true, false>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n,
                       P->alpha);
  else if (a.f_packed)
    hipLaunchKernelGGL((ksmac_kernel<NK, MB, false, true>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n,
                       P->alpha);
  else
    hipLaunchKernelGGL((ksmac_kernel<NK, MB, false, false>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n,
                       P->alpha);
}

template <int NK>
hipError_t launch_ksmac_nk(const ckks_params* P, const KsMacArgs& a, hipStream_t s) {
  switch (a.beta) {
    case 1: launch_ksmac_mb<NK, 1>(P, a, s); break;
    case 2: launch_ksmac_mb<NK, 2>(P, a, s); break;
    case 3: launch_ksmac_mb<NK, 3>(P, a, s); break;
    case 4: launch_ksmac_mb<NK, 4>(P, a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void __launch_bounds__(kThreads)
    auto_kernel(AutoArgs a, const PrimeDev* __restrict__ primes, int log_n) {
  const size_t n = (size_t)1 << log_n;
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const uint64_t q = primes[l + a.prime_off].q;
  const size_t s = (size_t)l * n + auto_index(p, a.gal, log_n);
  uint64_t v = a.in[s];
  if (a.add) v = add_mod(v, a.add[s], q);
  const size_t o = (size_t)l * n + p;
  if (a.accumulate) v = add_mod(v, a.out[o], q);
  __builtin_nontemporal_store(v, a.out + o);
}

__global__ void __launch_bounds__(kThreads)
    auto_batch_kernel(AutoBatchArgs a, const PrimeDev* __restrict__ primes, int log_n) {
  const size_t n = (size_t)1 << log_n;
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const int e = blockIdx.z;
  const uint64_t q = primes[l + a.prime_off].q;
  const size_t s = (size_t)l * n + auto_index(p, a.gal[e], log_n);
  uint64_t v = ld_nt(a.in[e] + s);
  if (a.add[e]) v = add_mod(v, a.add[e][s], q);
  const size_t o = (size_t)l * n + p;
  if (a.accumulate[e]) v = add_mod(v, a.out[e][o], q);
  __builtin_nontemporal_store(v, a.out[e] + o);
}

}  // namespace

// Bytes of the first `count` limbs of a PQ polynomial, packed or not.
static double limb_bytes(const ckks_params* P, int count, bool packed) {
  double b = 0;
  for (int i = 0; i < count; ++i) b += (packed && P->primes[i] < kNarrowLimit ? 5.0 : 8.0) * P->n;
  return b;
}

hipError_t launch_keyswitch(const ckks_params* P, const KsArgs& a, hipStream_t s) {
  double words = 0;
  for (int i = 0; i < a.ndig; ++i) {
    double per = a.beta[i] + (a.add[i] ? 1 : 0);
    for (int k = 0; k < a.nkeys; ++k) per += a.out_a[i][k] ? 2 : 0;
    words += per * a.K[i];
  }
  double key_bytes = 0;
  for (int k = 0; k < a.nkeys; ++k) key_bytes += 2.0 * a.kbeta * limb_bytes(P, a.maxK, a.key_packed);
  ProfScope prof(CKKS_KERNEL_KEYSWITCH, s, words * P->n * 8 + key_bytes);
  if (a.diag) {
    switch (a.kbeta) {
      case 1: return launch_diag_mb<1>(P, a, s);
      case 2: return launch_diag_mb<2>(P, a, s);
      case 3: return launch_diag_mb<3>(P, a, s);
      case 4: return launch_diag_mb<4>(P, a, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.ndig) {
    case 1: return launch_ks<1>(P, a, s);
    case 2: return launch_ks<2>(P, a, s);
    case 3: return launch_ks<3>(P, a, s);
    case 4: return launch_ks<4>(P, a, s);
    case 5: return launch_ks<5>(P, a, s);
    case 6: return launch_ks<6>(P, a, s);
    case 7: return launch_ks<7>(P, a, s);
    case 8: return launch_ks<8>(P, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_keyswitch_gather(const ckks_params* P, const KsGatherArgs& a, hipStream_t s) {
  double bytes = (double)a.K * P->n * (4.0 + a.nk * (a.beta + 1)) * 8;
  bytes += a.nk * 2.0 * a.beta * limb_bytes(P, a.K, a.key_packed);
  ProfScope prof(CKKS_KERNEL_KEYSWITCH_GATHER, s, bytes);
  switch (a.beta) {
    case 1: return launch_gather_mb<1>(P, a, s);
    case 2: return launch_gather_mb<2>(P, a, s);
    case 3: return launch_gather_mb<3>(P, a, s);
    case 4: return launch_gather_mb<4>(P, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ptmac(const ckks_params* P, const MacArgs& a, hipStream_t s) {
  int nf = 0;
  for (int k = 0; k < a.nk; ++k)
    for (int m = 0; m < a.nm; ++m) nf += a.f[k][m] ? 1 : 0;
  const double words = (double)a.K * P->n * (2.0 * a.nm + 2.0 * a.nk * (a.accumulate ? 2 : 1));
  ProfScope prof(CKKS_KERNEL_PTMAC, s, words * 8 + nf * limb_bytes(P, a.K, a.f_packed && a.prime_off == 0));
  switch (a.nk) {
    case 1: return launch_mac<1>(P, a, s);
    case 2: return launch_mac<2>(P, a, s);
    case 3: return launch_mac<3>(P, a, s);
    case 4: return launch_mac<4>(P, a, s);
    case 5: return launch_mac<5>(P, a, s);
    case 6: return launch_mac<6>(P, a, s);
    case 7: return launch_mac<7>(P, a, s);
    case 8: return launch_mac<8>(P, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ksmac(const ckks_params* P, const KsMacArgs& a, hipStream_t s) {
  // Geometry, checked before anything runs: term and accumulator counts
  // within the tables, every rotated term's key among the launch's keys and
  // consecutive with the other terms of that key, every operand present.
  if (a.nm < 1 || a.nm > kMaxMacM || a.nk < 1 || a.nk > kMaxMacK || a.K < 1 || a.K > a.kmax || a.beta < 1 ||
      a.beta > kMaxBeta || P->n % kKsMacAlign)
    return hipErrorInvalidValue;
  int nkeys = 0, ndig = 0, nadd = 0, nunrot = 0, nf = 0;
  for (int m = 0; m < a.nm; ++m) {
    const int kj = a.key_of[m];
    if (kj >= kMaxMacM || !a.a[m]) return hipErrorInvalidValue;
    if (kj < 0) {
      if (!a.b[m]) return hipErrorInvalidValue;
      ++nunrot;
    } else {
      if (!a.key[kj] || !a.digits[m]) return hipErrorInvalidValue;
      for (int m2 = 0; m2 < m; ++m2)  // a key's terms are consecutive
        if (a.key_of[m2] == kj && a.key_of[m - 1] != kj) return hipErrorInvalidValue;
      bool seen_key = false, seen_dig = false, seen_add = false;
      for (int m2 = 0; m2 < m; ++m2) {
        seen_key = seen_key || a.key_of[m2] == kj;
        seen_dig = seen_dig || (a.key_of[m2] >= 0 && a.digits[m2] == a.digits[m]);
        seen_add = seen_add || (a.key_of[m2] >= 0 && a.a[m2] == a.a[m]);
      }
      nkeys += !seen_key;
      ndig += !seen_dig;
      nadd += !seen_add;
    }
    for (int k = 0; k < a.nk; ++k) nf += a.f[k][m] ? 1 : 0;
  }
  for (int k = 0; k < a.nk; ++k)
    if (!a.out0[k] || !a.out1[k]) return hipErrorInvalidValue;
  // algorithmic bytes: keys, digit sets, adds and unrotated products, the
  // plaintexts, the accumulators, each word once (packed limbs at their size)
  const double words = (double)a.K * ((double)a.beta * ndig + nadd + 2.0 * nunrot + 2.0 * a.nk * (a.accumulate ? 2 : 1));
  const double bytes = words * P->n * 8 + 2.0 * a.beta * nkeys * limb_bytes(P, a.K, a.key_packed) +
                       nf * limb_bytes(P, a.K, a.f_packed);
  ProfScope prof(CKKS_KERNEL_KSMAC, s, bytes);
  switch (a.nk) {
    case 1: return launch_ksmac_nk<1>(P, a, s);
    case 2: return launch_ksmac_nk<2>(P, a, s);
    case 3: return launch_ksmac_nk<3>(P, a, s);
    case 4: return launch_ksmac_nk<4>(P, a, s);
    case 5: return launch_ksmac_nk<5>(P, a, s);
    case 6: return launch_ksmac_nk<6>(P, a, s);
    case 7: return launch_ksmac_nk<7>(P, a, s);
    case 8: return launch_ksmac_nk<8>(P, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_automorph_batch(const ckks_params* P, const AutoBatchArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  if (a.count > kMaxAuto) return hipErrorInvalidValue;
  double words = 0;
  for (int e = 0; e < a.count; ++e) words += 2 + (a.add[e] ? 1 : 0) + (a.accumulate[e] ? 1 : 0);
  ProfScope prof(CKKS_KERNEL_AUTOMORPH, s, words * a.nlimbs * P->n * 8);
  dim3 grid(P->n / kThreads, a.nlimbs, a.count);
  hipLaunchKernelGGL(auto_batch_kernel, grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n);
  return hipGetLastError();
}

hipError_t launch_automorph(const ckks_params* P, const AutoArgs& a, hipStream_t s) {
  dim3 grid(P->n / kThreads, a.nlimbs);
  ProfScope prof(CKKS_KERNEL_AUTOMORPH, s,
                 (double)a.nlimbs * P->n * 8 * (2 + (a.add ? 1 : 0) + (a.accumulate ? 1 : 0)));
  hipLaunchKernelGGL(auto_kernel, grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n);
  return hipGetLastError();
}

}  // namespace ckks
