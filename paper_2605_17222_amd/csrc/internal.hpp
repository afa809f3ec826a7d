// Internal types shared by the host orchestration and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/ckks_lt.h"

namespace ckks {

constexpr int kMaxSrc = 16;    // basis-conversion source limbs
constexpr int kMaxDst = 64;    // basis-conversion destination limbs (alpha + L + 1)
constexpr int kMaxBeta = 4;    // key-switching digits
constexpr int kMaxDig = 8;     // digit sets sharing one key read (hoisting)
constexpr int kMaxKs = 8;      // keys applied to one digit set per launch
constexpr int kMaxMacM = 16;   // plaintext-MAC inputs per launch
constexpr int kMaxMacK = 8;    // plaintext-MAC accumulators per launch

// Per-prime constants, indexed by PQ index (special primes first).
struct PrimeDev {
  uint64_t q;
  uint64_t qinv_neg;       // -q^-1 mod 2^64 (Montgomery REDC)
  uint64_t r_lo, r_hi;     // floor(2^128 / q) (Barrett)
  uint64_t ninv, ninv_sh;  // N^-1 mod q and its Shoup companion
  uint64_t pmod, pmod_sh;  // P mod q (0 on the special primes) and companion
  const uint64_t* tw;      // [4][N]: psi^br(i), Shoup, psi^-br(i), Shoup (integer primes) or
                           // the same powers as doubles and each divided by q (fp primes)
  const double* trow;      // fp primes: row-pass twiddle factors, [2][row_tables_size] (forward,
                           // inverse); see ntt_row_tables_size
  int fp;                  // q < 2^46: NTT butterflies in exact FP64 arithmetic
  int pad;
  double qd, qinv_d;       // q and 1/q as doubles
  double ninv_d, ninv_q;   // N^-1 mod q as a double and divided by q
  uint64_t pk_off;         // byte offset of this limb in a packed PQ polynomial
  int narrow;              // q < 2^40: packed as a 32-bit and an 8-bit plane
  int pk_pad;
};

// Packed storage of resident operands (keys, plaintexts): a limb of a prime
// below 2^40 is N 32-bit low words followed by N 8-bit high bytes (5N
// bytes); other limbs stay N 64-bit words.  A packed PQ polynomial is its
// Kmax limbs back to back (limb i at PrimeDev::pk_off); lower levels read a
// prefix.
constexpr uint64_t kNarrowLimit = 1ull << 40;

constexpr uint64_t kFpPrimeLimit = 1ull << 46;

// The two NTT passes split log2 N = (log2 N - B) + B: the column pass does the
// first log2 N - B stages, the row pass the last B.
__host__ __device__ inline int ntt_row_log(int log_n) { return log_n / 2; }

// Row-pass twiddles factor (fp primes): stage s (0 <= s < B) of row `row` uses
// rho^br(2^(log N - B + s) + row 2^s + y), y < 2^s, with rho = psi or psi^-1
// and br over log2 N bits; it equals G[2^s + y] * R[row][s] mod q with
//   G[2^s + y] = rho^(2^(B-1-s) + br_s(y) 2^(log N - s)),
//   R[row][s]  = rho^(br_(log N - B)(row) 2^(B - s)).
// Per direction: G (2^B doubles), then R as (value, value / q) pairs for each
// (row, s): 2^B + 2 * 2^(log N - B) * B doubles.
__host__ __device__ inline size_t ntt_row_tables_size(int log_n) {
  const int B = ntt_row_log(log_n);
  return ((size_t)1 << B) + 2 * ((size_t)1 << (log_n - B)) * B;
}

// Basis conversion eq. (3) from `ns` source limbs to `nd` destination limbs,
// plus the final factor S^-1 of a division step (eq. (4), eq. (1)).
struct BConvPlan {
  int ns, nd;
  int src[kMaxSrc];                 // PQ indices, in the order of the source limbs
  int dst[kMaxDst];                 // PQ indices
  uint64_t hinv[kMaxSrc];           // (S/s_j)^-1 mod s_j
  uint64_t hinv_sh[kMaxSrc];        // Shoup companion
  uint64_t hmod[kMaxDst][kMaxSrc];  // [S/s_j]_{d_m} * 2^64 mod d_m
  uint64_t sinv[kMaxDst];           // S^-1 mod d_m
  uint64_t sinv_sh[kMaxDst];
  int split30;                      // every source and destination prime < 2^60: the
                                    // inner product may use 30-bit column sums
  uint32_t hk[kMaxDst][kMaxSrc][2];  // hmod split into its 30-bit halves (split30)
};

// A run of `count` limbs stored back to back whose primes are consecutive PQ
// indices starting at prime0.
struct LimbRange {
  const uint64_t* in;
  uint64_t* out;
  const uint64_t* aux;      // division epilogue: the kept limbs, laid out like out
  uint64_t* copy;           // inverse transforms: also store the input limbs here
  const uint64_t* sinv;     // division epilogue: divisor^-1 per limb, and its
  const uint64_t* sinv_sh;  // Shoup companion (device, inside a BConvPlan)
  int prime0;
  int count;
  // Forward transforms: in holds N signed 64-bit coefficients shared by every
  // limb of the range, reduced into each limb's prime as the first pass reads
  // them (|coefficient| < 2^62).
  int signed_in;
  int pad;
};

constexpr int kMaxRanges = 32;
struct NttArgs {
  int nr = 0;
  LimbRange r[kMaxRanges];
};

// Epilogue of the last forward pass: ModDown / rescale division step
// out = (aux - v) * S^-1 mod q.
enum EpiMode { EPI_NONE = 0, EPI_SUBMUL = 1 };

constexpr int kMaxConv = 16;
struct BConvArgs {
  const BConvPlan* plan[kMaxConv];
  const uint64_t* src[kMaxConv];  // source limb j at src + j N
  uint64_t* dst[kMaxConv];        // destination limb m at dst + (plan.dst[m] - dst_shift) N
  // division epilogue (null: none): dst = (aux - conv) * plan.sinv, aux laid
  // out like dst (the kept limbs in the coefficient domain)
  const uint64_t* aux[kMaxConv];
  int dst_shift[kMaxConv];
  int limbs_moved;                // sum over items of ns + nd, + nd with aux (timing only)
  int max_nd;                     // largest nd over the items (sets the grid's destination chunks)
};

// Key-switch inner products of ndig digit sets with nkeys keys: output
// (i, k) is phi_k(add_i + <d_i, key_k>), phi_k(<d_i, key_k>) (null = skipped).
// Digit sets may be at different levels (K_i limbs, beta_i digits): limb l of
// a key is the same prime at every level, so one key read serves them all.
struct KsArgs {
  int ndig, nkeys, kmax, kbeta, maxK;
  int K[kMaxDig], beta[kMaxDig];
  const uint64_t* digits[kMaxDig];  // [beta_i][K_i][N] each
  const uint64_t* add[kMaxDig];     // [K_i][N], or Q-basis [K_i - alpha][N] to be multiplied by P, or null
  int add_pscaled[kMaxDig];
  const uint64_t* key[kMaxKs];      // [beta_max][2][kmax][N], or packed [beta_max][2] polynomials
  int key_packed;                   // every key of the launch is packed (else none is)
  uint64_t pk_poly_bytes;           // bytes of one packed PQ polynomial
  uint32_t gal_inv[kMaxKs];         // Galois element of -r: value at p is stored at auto_index(p, gal_inv)
  int diag;                         // one-to-one: ndig == nkeys and only outputs (k, k) exist
  uint64_t* out_a[kMaxDig][kMaxKs];
  uint64_t* out_b[kMaxDig][kMaxKs];
};

// Outer layer of Algorithm 2 (lines 17-18) for all giant steps at once, as a
// gather: c0[p] += sum_k (u0_k + <d_k, key_k,0>)[src_k(p)],
//         c1[p] += sum_k <d_k, key_k,1>[src_k(p)], src_k = phi index of r_k.
struct KsGatherArgs {
  int nk, beta, K, kmax;
  const uint64_t* digits[kMaxKs];  // [beta][K][N]
  const uint64_t* key[kMaxKs];
  int key_packed;                  // every key of the launch is packed (else none is)
  uint64_t pk_poly_bytes;
  const uint64_t* add[kMaxKs];     // u0_k [K][N]
  uint32_t gal[kMaxKs];            // Galois element of r_k
  uint64_t* c0;
  uint64_t* c1;
};

// Lines 8-14 of Algorithm 2 in one pass (middle key switch fused with the
// plaintext multiply-accumulate).  Term m is either unrotated, (a_m, b_m)
// read at the output position (key_of[m] < 0), or the middle rotation of
// digit set digits[m] by key key_of[m]: at output position p the product
// <d, swk> and the add a[m] are formed at auto_index(p, gal[key]), so the
// rotated (a_m, b_m) exist only in registers.  Terms sharing a key are
// consecutive.
constexpr int kKsMacAlign = 2048;  // N must be a multiple: 256 threads per workgroup x 8 XCDs
struct KsMacArgs {
  int nm, nk, K, beta, kmax;
  int accumulate;                    // add into the outputs
  int key_packed, f_packed;          // every key / every plaintext of the launch is packed (else none is)
  uint64_t pk_poly_bytes;            // bytes of one packed PQ polynomial
  int key_of[kMaxMacM];
  const uint64_t* digits[kMaxMacM];  // rotated terms: [beta][K][N]
  const uint64_t* a[kMaxMacM];       // the add (rotated) or a_m (unrotated); Q-basis c' if pscaled
  const uint64_t* b[kMaxMacM];       // unrotated terms: b_m
  int pscaled[kMaxMacM];             // a (and b) are Q-basis polynomials to be multiplied by P
  const uint64_t* key[kMaxMacM];     // [beta_max][2][kmax][N], or packed [beta_max][2] polynomials
  uint32_t gal[kMaxMacM];            // Galois element of the key's rotation r
  const uint64_t* f[kMaxMacK][kMaxMacM];  // null = absent diagonal
  uint64_t* out0[kMaxMacK];
  uint64_t* out1[kMaxMacK];
};

struct MacArgs {
  int nm, nk, K, prime_off;
  int pscaled0;    // a[0], b[0] are Q-basis polynomials to be multiplied by P
  int accumulate;  // add into the outputs
  int f_packed;    // f are packed PQ polynomials (prime_off = 0)
  const uint64_t* a[kMaxMacM];
  const uint64_t* b[kMaxMacM];
  const uint64_t* f[kMaxMacK][kMaxMacM];  // null = absent diagonal
  uint64_t* out0[kMaxMacK];
  uint64_t* out1[kMaxMacK];
};

struct AutoArgs {
  const uint64_t* in;
  const uint64_t* add;  // may be null
  uint64_t* out;
  int nlimbs, prime_off, accumulate;
  uint32_t gal;         // out[p] = (in + add)[auto_index(p, gal)]
};

// Several automorphisms of nlimbs limbs in one launch (blockIdx.z = entry);
// the entries' outputs must be distinct (they run concurrently).
constexpr int kMaxAuto = 16;
struct AutoBatchArgs {
  int count, nlimbs, prime_off;
  const uint64_t* in[kMaxAuto];
  const uint64_t* add[kMaxAuto];  // may be null
  uint64_t* out[kMaxAuto];
  int accumulate[kMaxAuto];
  uint32_t gal[kMaxAuto];
};

// Brackets one launch with HIP events when its kernel is being timed.
class ProfScope {
 public:
  ProfScope(int id, hipStream_t s, double bytes);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  int id_;
  hipStream_t s_;
  double bytes_;
  void* a_ = nullptr;
  void* b_ = nullptr;
  bool active_ = false;
};

// Plaintext encoding of up to kMaxEnc slot vectors per launch: z[i] holds
// N/2 complex slots (re, im), encoded as rot(z, rot[i]) with scale[i]; y[i]
// is scratch for N/2 complex values; coef[i] receives the N coefficients.
constexpr int kMaxEnc = 32;
struct EncArgs {
  int count;
  const double* z[kMaxEnc];
  int rot[kMaxEnc];
  double scale[kMaxEnc];
  double* y[kMaxEnc];
  int64_t* coef[kMaxEnc];
};

// Device address of the no-allocation entry point's scratch array on
// `device` (which must be current), looked up on first use and kept.
int scratch_address(int device, void** out);

// Kernel launchers.
hipError_t launch_ntt(const struct ::ckks_params* P, bool forward, const NttArgs& a, int total_limbs, int epi,
                      hipStream_t s);
hipError_t launch_bconv(const struct ::ckks_params* P, const BConvArgs& a, int items, int ns, hipStream_t s);
hipError_t launch_keyswitch(const struct ::ckks_params* P, const KsArgs& a, hipStream_t s);
hipError_t launch_keyswitch_gather(const struct ::ckks_params* P, const KsGatherArgs& a, hipStream_t s);
hipError_t launch_ptmac(const struct ::ckks_params* P, const MacArgs& a, hipStream_t s);
hipError_t launch_ksmac(const struct ::ckks_params* P, const KsMacArgs& a, hipStream_t s);
hipError_t launch_automorph(const struct ::ckks_params* P, const AutoArgs& a, hipStream_t s);
hipError_t launch_automorph_batch(const struct ::ckks_params* P, const AutoBatchArgs& a, hipStream_t s);
hipError_t launch_encode_fft(const struct ::ckks_params* P, const EncArgs& a, hipStream_t s);
// count full PQ polynomials [count][Kmax][N] -> packed [count][pk_poly_bytes].
hipError_t launch_pack(const struct ::ckks_params* P, int count, const uint64_t* in, uint8_t* out, hipStream_t s);

}  // namespace ckks

struct ckks_params {
  int device = 0;
  int log_n = 0, n = 0;
  int L = 0, alpha = 0, dnum = 0;
  std::vector<uint64_t> primes;        // PQ order
  ckks::PrimeDev* d_primes = nullptr;  // device [K_max]
  uint64_t* d_tw = nullptr;            // device [K_max][4][N]
  double* d_trow = nullptr;            // device [K_max][2][ntt_row_tables_size]
  ckks::BConvPlan* d_plans = nullptr;  // device plan table
  uint64_t pk_poly_bytes = 0;          // bytes of one packed PQ polynomial (Kmax limbs)
  // Encoding tables (N/2 entries each): perm[j] = t with 5^t = 4 j + 1 mod 2N;
  // enc_tw[e] = e^(-2 pi i e / (N/2)); enc_zinv[k] = zeta^-k / (N/2), as (re, im).
  int* d_enc_perm = nullptr;
  double* d_enc_tw = nullptr;
  double* d_enc_zinv = nullptr;
  std::vector<std::pair<int, int>> plan_shape;  // host copy of each plan's (ns, nd)
  std::vector<uint8_t> plan_split30;            // host copy of each plan's split30
  std::vector<int> plan_decomp;        // level * beta_max + b -> plan index
  std::vector<int> plan_moddown, plan_mdrescale, plan_rescale;  // per level
  int beta_max = 0;
  int K(int level) const { return alpha + level + 1; }
  int beta(int level) const { return (level + alpha) / alpha; }
  int Kmax() const { return alpha + L + 1; }
  const ckks::BConvPlan* plan(int idx) const { return d_plans + idx; }
  // (ns, nd) of a device plan pointer returned by plan(), read on the host
  std::pair<int, int> plan_dims(const ckks::BConvPlan* p) const {
    const ptrdiff_t i = p - d_plans;
    return (i >= 0 && (size_t)i < plan_shape.size()) ? plan_shape[(size_t)i] : std::pair<int, int>(-1, -1);
  }
  bool plan_is_split30(const ckks::BConvPlan* p) const {
    const ptrdiff_t i = p - d_plans;
    return i >= 0 && (size_t)i < plan_split30.size() && plan_split30[(size_t)i];
  }
};
