// CPU oracle for RNS-CKKS homomorphic linear transformations.
//
// TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
// implementation used by the tests, by the smoke check and by the CPU-baseline
// leg of the benchmark to decide what the GPU library must output.  The GPU
// library never links, loads or calls it, and it shares no code with it.
//
// Every modular product is the definition (a*b mod q through 128-bit integer
// division); every transform is the textbook radix-2 negacyclic NTT; every
// basis conversion is eq. (3) written out; ModDown is eq. (4); rescale is
// eq. (1).  The LT algorithms follow the paper's Section II-B (diagonal
// method, BSGS eq. (5)) and Algorithm 2 (triple-hoisted BSGS) step by step.
//
// Conventions the paper leaves open (all chosen once and used everywhere):
//  * residues are canonical in [0, q) (the [.]_q of eq. (3));
//  * psi for (q, N) is g^((q-1)/2N) for the smallest quadratic non-residue
//    g >= 2 of q, a primitive 2N-th root of unity;
//  * NTT layout: position p holds sum_k a_k psi^((2 br(p) + 1) k), br = bit
//    reversal over log2 N bits (the bit-reversed storage of Section V);
//  * automorphism phi_r uses g_r = 5^(r mod N/2) mod 2N (Section II-A); in the
//    NTT domain it is the gather out[p] = in[br((g_r (2 br(p)+1) mod 2N - 1)/2)]
//    (eq. (7) read as out_l = in_l');
//  * PQ limb order is P first: p_0..p_{alpha-1}, q_0..q_l (eq. (4) indexes
//    q_j as limb j + alpha);
//  * switching key for rotation r, digit b: (-a s + e + G_b phi_r(s), a) with
//    G_b = [P]_{q_j} on the q_j of group b and 0 elsewhere; the stored key is
//    the pre-rotated phi_{-r}(swk) of Algorithm 2's input list.
//  * the final line of Algorithm 2 is one ModDown by P*q_l (combined ModDown
//    and rescale).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

typedef unsigned __int128 u128;
typedef std::vector<uint64_t> Vec;

namespace {

// ---------------------------------------------------------------------------
// Integers mod q (q < 2^62).
// ---------------------------------------------------------------------------
inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
inline uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
inline uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
inline uint64_t negmod(uint64_t a, uint64_t q) { return a == 0 ? 0 : q - a; }

uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}
// q prime: Fermat inverse.
uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a % q, q - 2, q); }

// Reduce a signed integer into [0, q).
inline uint64_t from_signed(int64_t v, uint64_t q) {
  int64_t r = v % (int64_t)q;
  return r < 0 ? (uint64_t)(r + (int64_t)q) : (uint64_t)r;
}

bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : bases) if (n % p == 0) return n == p;
  uint64_t d = n - 1; int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; ++i) { x = mulmod(x, x, n); if (x == n - 1) { comp = false; break; } }
    if (comp) return false;
  }
  return true;
}

inline uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, 2014): the oracle's only random source.
// A stream is keyed by (seed, stream id).
// ---------------------------------------------------------------------------
struct Rng {
  uint64_t s;
  Rng(uint64_t seed, uint64_t stream) : s(seed * 0x9E3779B97F4A7C15ull ^ (stream + 0x632BE59BD9B4E019ull) * 0xD1B54A32D192ED03ull) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform01() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }  // in (0,1)
  uint64_t below(uint64_t q) {  // uniform in [0, q) by rejection
    int bits = 64 - __builtin_clzll(q);
    for (;;) { uint64_t x = next() >> (64 - bits); if (x < q) return x; }
  }
  // Rounded Gaussian, rejected beyond 6 sigma (Box-Muller).
  int64_t gauss(double sigma) {
    for (;;) {
      double u1 = uniform01(), u2 = uniform01();
      double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2) * sigma;
      if (std::fabs(z) <= 6.0 * sigma) return (int64_t)std::llround(z);
    }
  }
};

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct PrimeTab {
  uint64_t q, psi, psi_inv, n_inv;
  Vec psi_rev, psi_inv_rev;  // psi^br(i), psi^-br(i) over log2 N bits
};

struct Counters { long decompose = 0, moddown = 0, ks = 0, ntt = 0, intt = 0; std::set<long> keys; };

struct Ctx {
  int logn = 0, n = 0, L = 0, alpha = 0, dnum = 0;
  std::vector<PrimeTab> pq;   // PQ order: p_0..p_{alpha-1}, q_0..q_L
  std::vector<int64_t> s;     // ternary secret, coefficient form
  bool has_secret = false;
  Counters cnt;
  std::string err;
  int K(int level) const { return alpha + level + 1; }
  int beta(int level) const { return (level + 1 + alpha - 1) / alpha; }
  uint64_t q(int pqi) const { return pq[pqi].q; }
};

uint64_t find_psi(uint64_t q, int n) {
  // Smallest quadratic non-residue g >= 2; psi = g^((q-1)/2n) has order 2n.
  for (uint64_t g = 2;; ++g) {
    if (powmod(g, (q - 1) / 2, q) == q - 1) return powmod(g, (q - 1) / (2 * (uint64_t)n), q);
  }
}

// ---------------------------------------------------------------------------
// Negacyclic NTT (in place). Forward: Cooley-Tukey with the table psi^br(i),
// output in the bit-reversed evaluation order stated above.  Inverse:
// Gentleman-Sande with psi^-br(i), then multiplication by N^-1.
// ---------------------------------------------------------------------------
void ntt(const Ctx& c, int pqi, uint64_t* a) {
  const PrimeTab& t = c.pq[pqi];
  const uint64_t q = t.q;
  int len = c.n;
  for (int m = 1; m < c.n; m <<= 1) {
    len >>= 1;
    for (int i = 0; i < m; ++i) {
      uint64_t w = t.psi_rev[m + i];
      uint64_t* x = a + 2 * i * len;
      for (int j = 0; j < len; ++j) {
        uint64_t u = x[j], v = mulmod(x[j + len], w, q);
        x[j] = addmod(u, v, q);
        x[j + len] = submod(u, v, q);
      }
    }
  }
}

void intt(const Ctx& c, int pqi, uint64_t* a) {
  const PrimeTab& t = c.pq[pqi];
  const uint64_t q = t.q;
  int len = 1;
  for (int m = c.n >> 1; m >= 1; m >>= 1) {
    for (int i = 0; i < m; ++i) {
      uint64_t w = t.psi_inv_rev[m + i];
      uint64_t* x = a + 2 * i * len;
      for (int j = 0; j < len; ++j) {
        uint64_t u = x[j], v = x[j + len];
        x[j] = addmod(u, v, q);
        x[j + len] = mulmod(submod(u, v, q), w, q);
      }
    }
    len <<= 1;
  }
  for (int j = 0; j < c.n; ++j) a[j] = mulmod(a[j], t.n_inv, q);
}

// Galois element of rotation r: 5^(r mod N/2) mod 2N.
uint64_t galois(const Ctx& c, long r) {
  long S = c.n / 2;
  long rr = ((r % S) + S) % S;
  return powmod(5, (uint64_t)rr, 2 * (uint64_t)c.n);
}

// NTT-domain automorphism: out[p] = in[br((g (2 br(p) + 1) mod 2N - 1) / 2)].
std::vector<uint32_t> auto_index(const Ctx& c, long r) {
  uint64_t g = galois(c, r);
  uint64_t two_n = 2 * (uint64_t)c.n;
  std::vector<uint32_t> idx(c.n);
  for (int p = 0; p < c.n; ++p) {
    uint64_t l = bitrev(p, c.logn);
    uint64_t e = (g * (2 * l + 1)) % two_n;
    idx[p] = bitrev((uint32_t)((e - 1) / 2), c.logn);
  }
  return idx;
}

void automorph_ntt(const Ctx& c, long r, const uint64_t* in, uint64_t* out, int limbs) {
  std::vector<uint32_t> idx = auto_index(c, r);
  for (int l = 0; l < limbs; ++l)
    for (int p = 0; p < c.n; ++p) out[(size_t)l * c.n + p] = in[(size_t)l * c.n + idx[p]];
}

// Coefficient-domain automorphism a(x) -> a(x^g) mod x^N + 1.
void automorph_coeff(const Ctx& c, int pqi, uint64_t g, const uint64_t* in, uint64_t* out) {
  uint64_t q = c.q(pqi);
  for (uint64_t k = 0; k < (uint64_t)c.n; ++k) {
    uint64_t e = (g * k) % (2 * (uint64_t)c.n);
    if (e < (uint64_t)c.n) out[e] = in[k];
    else out[e - c.n] = negmod(in[k], q);
  }
}

// ---------------------------------------------------------------------------
// Basis conversion, eq. (3): from basis S = {s_j} to basis D = {d_m}.
//   y_j = [ (S/s_j)^-1 x_j ]_{s_j};  out_m = sum_j y_j [S/s_j]_{d_m} mod d_m.
// Inputs are coefficient-domain limbs; `src`/`dst` list PQ indices.
// ---------------------------------------------------------------------------
void bconv(const Ctx& c, const std::vector<int>& src, const uint64_t* x,
           const std::vector<int>& dst, uint64_t* out) {
  const int ns = (int)src.size(), nd = (int)dst.size(), n = c.n;
  // hat_inv[j] = (prod_{i != j} s_i)^-1 mod s_j; hat[m][j] = prod_{i != j} s_i mod d_m
  std::vector<uint64_t> hat_inv(ns);
  for (int j = 0; j < ns; ++j) {
    uint64_t sj = c.q(src[j]), prod = 1;
    for (int i = 0; i < ns; ++i) if (i != j) prod = mulmod(prod, c.q(src[i]) % sj, sj);
    hat_inv[j] = invmod(prod, sj);
  }
  std::vector<uint64_t> hat((size_t)nd * ns);
  for (int m = 0; m < nd; ++m) {
    uint64_t dm = c.q(dst[m]);
    for (int j = 0; j < ns; ++j) {
      uint64_t prod = 1;
      for (int i = 0; i < ns; ++i) if (i != j) prod = mulmod(prod, c.q(src[i]) % dm, dm);
      hat[(size_t)m * ns + j] = prod;
    }
  }
  Vec y((size_t)ns * n);
  for (int j = 0; j < ns; ++j)
    for (int k = 0; k < n; ++k) y[(size_t)j * n + k] = mulmod(x[(size_t)j * n + k], hat_inv[j], c.q(src[j]));
#pragma omp parallel for schedule(static)
  for (int m = 0; m < nd; ++m) {
    uint64_t dm = c.q(dst[m]);
    for (int k = 0; k < n; ++k) {
      uint64_t acc = 0;
      for (int j = 0; j < ns; ++j) acc = addmod(acc, mulmod(y[(size_t)j * n + k] % dm, hat[(size_t)m * ns + j], dm), dm);
      out[(size_t)m * n + k] = acc;
    }
  }
}

std::vector<int> q_basis(const Ctx& c, int level) {
  std::vector<int> b; for (int j = 0; j <= level; ++j) b.push_back(c.alpha + j); return b;
}
std::vector<int> pq_basis(const Ctx& c, int level) {
  std::vector<int> b; for (int i = 0; i < c.alpha + level + 1; ++i) b.push_back(i); return b;
}

void ntt_limbs(Ctx& c, const std::vector<int>& basis, uint64_t* a) {
#pragma omp parallel for schedule(static)
  for (int l = 0; l < (int)basis.size(); ++l) ntt(c, basis[l], a + (size_t)l * c.n);
  c.cnt.ntt += basis.size();
}
void intt_limbs(Ctx& c, const std::vector<int>& basis, uint64_t* a) {
#pragma omp parallel for schedule(static)
  for (int l = 0; l < (int)basis.size(); ++l) intt(c, basis[l], a + (size_t)l * c.n);
  c.cnt.intt += basis.size();
}

// ---------------------------------------------------------------------------
// Decompose (Fig. 1): split the level-l Q-basis polynomial (NTT form) into
// beta digit groups of alpha limbs; ModUp each group to PQ with eq. (3); the
// group's own limbs are taken over unchanged.  Output [beta][K][N], NTT form.
// ---------------------------------------------------------------------------
void decompose(Ctx& c, int level, const uint64_t* x_ntt, uint64_t* digits) {
  const int n = c.n, K = c.K(level), beta = c.beta(level);
  Vec coef(x_ntt, x_ntt + (size_t)(level + 1) * n);
  intt_limbs(c, q_basis(c, level), coef.data());
  for (int b = 0; b < beta; ++b) {
    int lo = b * c.alpha, hi = std::min(lo + c.alpha - 1, level);
    std::vector<int> src, dst;
    for (int j = lo; j <= hi; ++j) src.push_back(c.alpha + j);
    for (int i = 0; i < K; ++i) if (i < c.alpha + lo || i > c.alpha + hi) dst.push_back(i);
    Vec conv((size_t)dst.size() * n);
    bconv(c, src, coef.data() + (size_t)lo * n, dst, conv.data());
    ntt_limbs(c, dst, conv.data());
    uint64_t* d = digits + (size_t)b * K * n;
    for (size_t m = 0; m < dst.size(); ++m) std::memcpy(d + (size_t)dst[m] * n, conv.data() + m * n, n * 8);
    for (int j = lo; j <= hi; ++j) std::memcpy(d + (size_t)(c.alpha + j) * n, x_ntt + (size_t)j * n, n * 8);
  }
  c.cnt.decompose++;
}

// ModDown, eq. (4): PQ (K limbs, NTT) -> Q (level+1 limbs, NTT).
void moddown(Ctx& c, int level, const uint64_t* x, uint64_t* out) {
  const int n = c.n, a = c.alpha;
  std::vector<int> P, Q = q_basis(c, level);
  for (int i = 0; i < a; ++i) P.push_back(i);
  Vec pc(x, x + (size_t)a * n);
  intt_limbs(c, P, pc.data());
  Vec conv((size_t)(level + 1) * n);
  bconv(c, P, pc.data(), Q, conv.data());
  ntt_limbs(c, Q, conv.data());
  for (int j = 0; j <= level; ++j) {
    uint64_t qj = c.q(a + j), pinv = 1;
    for (int i = 0; i < a; ++i) pinv = mulmod(pinv, c.q(i) % qj, qj);
    pinv = invmod(pinv, qj);
    for (int k = 0; k < n; ++k)
      out[(size_t)j * n + k] = mulmod(submod(x[(size_t)(a + j) * n + k], conv[(size_t)j * n + k], qj), pinv, qj);
  }
  c.cnt.moddown++;
}

// Combined ModDown and rescale: eq. (4) with P replaced by P*q_l.
// PQ (K limbs, NTT) -> level-1 (level limbs, NTT).
void moddown_rescale(Ctx& c, int level, const uint64_t* x, uint64_t* out) {
  const int n = c.n, a = c.alpha;
  std::vector<int> src, dst;
  for (int i = 0; i < a; ++i) src.push_back(i);
  src.push_back(a + level);
  for (int j = 0; j < level; ++j) dst.push_back(a + j);
  Vec sc((size_t)(a + 1) * n);
  std::memcpy(sc.data(), x, (size_t)a * n * 8);
  std::memcpy(sc.data() + (size_t)a * n, x + (size_t)(a + level) * n, (size_t)n * 8);
  intt_limbs(c, src, sc.data());
  Vec conv((size_t)level * n);
  bconv(c, src, sc.data(), dst, conv.data());
  ntt_limbs(c, dst, conv.data());
  for (int j = 0; j < level; ++j) {
    uint64_t qj = c.q(a + j), inv = 1;
    for (int s : src) inv = mulmod(inv, c.q(s) % qj, qj);
    inv = invmod(inv, qj);
    for (int k = 0; k < n; ++k)
      out[(size_t)j * n + k] = mulmod(submod(x[(size_t)(a + j) * n + k], conv[(size_t)j * n + k], qj), inv, qj);
  }
  c.cnt.moddown += 1;
}

// Rescale, eq. (1): Q at `level` (NTT) -> level-1.  [q_l^-1 (c_j - c_l)]_{q_j}.
void rescale(Ctx& c, int level, const uint64_t* x, uint64_t* out) {
  const int n = c.n, a = c.alpha;
  Vec last(x + (size_t)level * n, x + (size_t)(level + 1) * n);
  intt(c, a + level, last.data());
  uint64_t ql = c.q(a + level);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < level; ++j) {
    uint64_t qj = c.q(a + j), inv = invmod(ql % qj, qj);
    Vec t(n);
    for (int k = 0; k < n; ++k) t[k] = last[k] % qj;
    ntt(c, a + j, t.data());
    for (int k = 0; k < n; ++k)
      out[(size_t)j * n + k] = mulmod(submod(x[(size_t)j * n + k], t[k], qj), inv, qj);
  }
}

// Key-switch inner product <d, swk> over the K limbs of `level`.
// key layout: [beta_max][2][K_max][N]; digit layout [beta][K][N].
void ks_inner(Ctx& c, int level, const uint64_t* digits, const uint64_t* key, uint64_t* x, uint64_t* y) {
  const int n = c.n, K = c.K(level), beta = c.beta(level), Kmax = c.K(c.L);
#pragma omp parallel for schedule(static)
  for (int l = 0; l < K; ++l) {
    uint64_t q = c.q(l);
    for (int k = 0; k < n; ++k) {
      uint64_t ax = 0, ay = 0;
      for (int b = 0; b < beta; ++b) {
        uint64_t d = digits[((size_t)b * K + l) * n + k];
        ax = addmod(ax, mulmod(d, key[(((size_t)b * 2 + 0) * Kmax + l) * n + k], q), q);
        ay = addmod(ay, mulmod(d, key[(((size_t)b * 2 + 1) * Kmax + l) * n + k], q), q);
      }
      x[(size_t)l * n + k] = ax;
      y[(size_t)l * n + k] = ay;
    }
  }
  c.cnt.ks++;
}

// c += a (limb-wise over a basis given as PQ indices)
void add_inplace(const Ctx& c, const std::vector<int>& basis, uint64_t* acc, const uint64_t* a) {
  for (size_t l = 0; l < basis.size(); ++l) {
    uint64_t q = c.q(basis[l]);
    for (int k = 0; k < c.n; ++k) acc[l * c.n + k] = addmod(acc[l * c.n + k], a[l * c.n + k], q);
  }
}
// acc += a .* f
void mac_inplace(const Ctx& c, const std::vector<int>& basis, uint64_t* acc, const uint64_t* a, const uint64_t* f) {
#pragma omp parallel for schedule(static)
  for (int l = 0; l < (int)basis.size(); ++l) {
    uint64_t q = c.q(basis[l]);
    for (int k = 0; k < c.n; ++k)
      acc[(size_t)l * c.n + k] = addmod(acc[(size_t)l * c.n + k], mulmod(a[(size_t)l * c.n + k], f[(size_t)l * c.n + k], q), q);
  }
}

// ---------------------------------------------------------------------------
// Ciphertext rotation with the pre-rotated key swk~_r = phi_{-r}(swk_r):
//   (x, y) = ModDown(<Decompose(c1), swk~_r>);  Rot = (phi_r(c0 + x), phi_r(y)).
// ---------------------------------------------------------------------------
struct KeyMap { std::map<long, const uint64_t*> m; };

const uint64_t* need_key(Ctx& c, const KeyMap& km, long r) {
  long S = c.n / 2;
  long rr = ((r % S) + S) % S;
  auto it = km.m.find(rr);
  if (it == km.m.end()) throw std::runtime_error("missing rotation key " + std::to_string(rr));
  c.cnt.keys.insert(rr);
  return it->second;
}

void rotate(Ctx& c, int level, const uint64_t* c0, const uint64_t* c1, long r, const KeyMap& km,
            uint64_t* o0, uint64_t* o1) {
  const int n = c.n, K = c.K(level), Lq = level + 1;
  const uint64_t* key = need_key(c, km, r);
  Vec d((size_t)c.beta(level) * K * n), x((size_t)K * n), y((size_t)K * n);
  decompose(c, level, c1, d.data());
  ks_inner(c, level, d.data(), key, x.data(), y.data());
  Vec xd((size_t)Lq * n), yd((size_t)Lq * n);
  moddown(c, level, x.data(), xd.data());
  moddown(c, level, y.data(), yd.data());
  add_inplace(c, q_basis(c, level), xd.data(), c0);
  automorph_ntt(c, r, xd.data(), o0, Lq);
  automorph_ntt(c, r, yd.data(), o1, Lq);
}

// P * x mod PQ for a Q-basis x (level): P-limbs 0, q_j-limbs x_j [P]_{q_j}.
void p_scale(const Ctx& c, int level, const uint64_t* x, uint64_t* out) {
  const int n = c.n, a = c.alpha;
  std::memset(out, 0, (size_t)a * n * 8);
  for (int j = 0; j <= level; ++j) {
    uint64_t qj = c.q(a + j), P = 1;
    for (int i = 0; i < a; ++i) P = mulmod(P, c.q(i) % qj, qj);
    for (int k = 0; k < n; ++k) out[(size_t)(a + j) * n + k] = mulmod(x[(size_t)j * n + k], P, qj);
  }
}

struct Diags {
  int n = 0;                       // number of diagonal slots (n1*n2[*n3])
  std::vector<const uint64_t*> f;  // f[m] = plaintext for index m (NULL = zero diagonal)
};

// Diagonal index t stands for the cyclic offset stride*(t - centre) (mod S).
// Plain Algorithm 2 has stride 1 and centre 0; a strided, centred
// progression serves sparse matrices such as the factors of a DFT.  The
// baby and middle rotations become stride*i and stride*n1*j, and the giant
// rotation of block k becomes G_k = stride*(B k - centre) with B the block
// length (n1 n2 for TH-BSGS, n1 for BSGS); a block whose G_k vanishes mod S
// is added without rotation (the role of the k = 0 block in the plain case).
struct Prog {
  long stride = 1, centre = 0;
};

long mod_slots(const Ctx& c, long r) {
  const long S = c.n / 2;
  return ((r % S) + S) % S;
}

// ---------------------------------------------------------------------------
// Triple-hoisted BSGS (Algorithm 2).  Plaintexts f^_m at PQ (K_max limbs,
// prefix-truncated to the level), m = n1 n2 k + n1 j + i, pre-rotated by
// phi_{-G_k}.
// ---------------------------------------------------------------------------
void lt_th(Ctx& c, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, int n3, Prog pg,
           const Diags& D, const KeyMap& km, uint64_t* o0, uint64_t* o1) {
  const int n = c.n, K = c.K(level), beta = c.beta(level), inner = n1 * n2;
  const size_t PL = (size_t)K * n;
  const std::vector<int> PQ = pq_basis(c, level);
  const long s = pg.stride;
  auto has = [&](int m) { return m < D.n && D.f[m] != nullptr; };
  // Which baby/middle products feed at least one present diagonal.
  std::vector<char> used_m(inner, 0);
  for (int k = 0; k < n3; ++k) for (int m = 0; m < inner; ++m) if (has(k * inner + m)) used_m[m] = 1;
  std::vector<char> used_i(n1, 0), mid_i(n1, 0);  // a_i needed / d_i needed (some j >= 1 uses it)
  for (int m = 0; m < inner; ++m) if (used_m[m]) { used_i[m % n1] = 1; if (m >= n1) mid_i[m % n1] = 1; }
  bool need_d0 = mid_i[0];
  for (int i = 1; i < n1; ++i) need_d0 |= used_i[i];

  std::vector<Vec> A(inner), B(inner);
  // Line 1: d_0 = Decompose(c1').
  Vec d0((size_t)beta * PL);
  if (need_d0) decompose(c, level, c1, d0.data());
  // Line 2: (a_0, b_0) = (P c0', P c1') mod PQ.
  A[0].resize(PL); B[0].resize(PL);
  p_scale(c, level, c0, A[0].data());
  p_scale(c, level, c1, B[0].data());
  std::vector<Vec> Dg(n1);
  // Lines 3-7: inner rotations by s*i share d_0; b_i goes through ModDown then Decompose.
  for (int i = 1; i < n1; ++i) {
    if (!used_i[i]) continue;
    const long r = s * i;
    const uint64_t* key = need_key(c, km, r);
    Vec x(PL), y(PL);
    ks_inner(c, level, d0.data(), key, x.data(), y.data());
    add_inplace(c, PQ, x.data(), A[0].data());
    A[i].resize(PL); B[i].resize(PL);
    automorph_ntt(c, r, x.data(), A[i].data(), K);
    automorph_ntt(c, r, y.data(), B[i].data(), K);
    if (!mid_i[i]) continue;
    Vec bq((size_t)(level + 1) * n);
    moddown(c, level, B[i].data(), bq.data());
    Dg[i].resize((size_t)beta * PL);
    decompose(c, level, bq.data(), Dg[i].data());
  }
  // Lines 8-11: middle rotations by s*n1*j share d_i.
  for (int i = 0; i < n1; ++i) {
    if (!mid_i[i]) continue;
    const uint64_t* di = (i == 0) ? d0.data() : Dg[i].data();
    for (int j = 1; j < n2; ++j) {
      int m = n1 * j + i;
      if (!used_m[m]) continue;
      const long r = s * n1 * j;
      const uint64_t* key = need_key(c, km, r);
      Vec x(PL), y(PL);
      ks_inner(c, level, di, key, x.data(), y.data());
      add_inplace(c, PQ, x.data(), A[i].data());
      A[m].resize(PL); B[m].resize(PL);
      automorph_ntt(c, r, x.data(), A[m].data(), K);
      automorph_ntt(c, r, y.data(), B[m].data(), K);
    }
  }
  // Lines 12-18: (u0_k, u1_k) = sum_{m < n1 n2} (a_m, b_m) f^_{n1 n2 k + m};
  // the block with G_k = 0 is added as is (line 12), every other one after
  // ModDown, Decompose and the hoisted rotation by G_k.
  Vec C0(PL, 0), C1(PL, 0);
  for (int k = 0; k < n3; ++k) {
    bool any = false;
    for (int m = 0; m < inner; ++m) any |= has(k * inner + m);
    if (!any) continue;
    Vec U0(PL, 0), U1(PL, 0);
    for (int m = 0; m < inner; ++m) {
      if (!has(k * inner + m)) continue;
      mac_inplace(c, PQ, U0.data(), A[m].data(), D.f[k * inner + m]);
      mac_inplace(c, PQ, U1.data(), B[m].data(), D.f[k * inner + m]);
    }
    const long G = mod_slots(c, s * ((long)inner * k - pg.centre));
    if (G == 0) {
      add_inplace(c, PQ, C0.data(), U0.data());
      add_inplace(c, PQ, C1.data(), U1.data());
      continue;
    }
    Vec u1q((size_t)(level + 1) * n), d((size_t)beta * PL);
    moddown(c, level, U1.data(), u1q.data());
    decompose(c, level, u1q.data(), d.data());
    const uint64_t* key = need_key(c, km, G);
    Vec x(PL), y(PL), t(PL);
    ks_inner(c, level, d.data(), key, x.data(), y.data());
    add_inplace(c, PQ, x.data(), U0.data());
    automorph_ntt(c, G, x.data(), t.data(), K);
    add_inplace(c, PQ, C0.data(), t.data());
    automorph_ntt(c, G, y.data(), t.data(), K);
    add_inplace(c, PQ, C1.data(), t.data());
  }
  // Line 19: combined ModDown and rescale by P q_l.
  moddown_rescale(c, level, C0.data(), o0);
  moddown_rescale(c, level, C1.data(), o1);
}

// ---------------------------------------------------------------------------
// Double-hoisted BSGS (Algorithm 1) with n1 baby steps and n2 giant steps,
// written from the algorithm itself (not as Algorithm 2 with an empty inner
// layer).  Inputs: keys swk~ for the baby rotations s*i (0 < i < n1) and the
// giant rotations G_j = s*(n1 j - centre); plaintexts f^_{n1 j + i} =
// phi_{-G_j}(f_{n1 j + i}) at PQ (K_max limbs, prefix-truncated).
// Readings: the baby loop starts at i = 1, (a_0, b_0) being P c' itself,
// and the giant block whose rotation vanishes is accumulated without key
// switching (the j = 0 block of the plain algorithm); this gives the
// algorithm's counts, n2 Decompose, n2 + 1 ModDown, n1 + n2 - 2 keys.  The
// last line, ModDown of c0 and c1 followed by the rescale, is one ModDown by
// P q_l when `combined` (the combination the paper applies to Algorithm 2's
// last line), else ModDown and then eq. (1).  Absent diagonals are skipped:
// a block without any contributes zero, a baby step no diagonal uses is
// not computed.
// ---------------------------------------------------------------------------
void lt_dh(Ctx& c, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, Prog pg, const Diags& D,
           const KeyMap& km, bool combined, uint64_t* o0, uint64_t* o1) {
  const int n = c.n, K = c.K(level), beta = c.beta(level);
  const size_t PL = (size_t)K * n;
  const std::vector<int> PQ = pq_basis(c, level);
  auto has = [&](int t) { return t < D.n && D.f[t] != nullptr; };
  std::vector<char> baby(n1, 0);  // a_i, b_i feed some present diagonal
  for (int j = 0; j < n2; ++j)
    for (int i = 0; i < n1; ++i)
      if (has(n1 * j + i)) baby[i] = 1;
  bool any_baby = false;
  for (int i = 1; i < n1; ++i) any_baby |= baby[i] != 0;
  // Line 1: d = Decompose(c1').
  Vec d((size_t)beta * PL);
  if (any_baby) decompose(c, level, c1, d.data());
  // Line 2: (a_0, b_0) = (P c0', P c1') mod PQ.
  std::vector<Vec> A(n1), B(n1);
  A[0].resize(PL);
  B[0].resize(PL);
  p_scale(c, level, c0, A[0].data());
  p_scale(c, level, c1, B[0].data());
  // Lines 3-5: a_i = phi_{s i}(a_0 + <d, swk~_{s i, 0}>), b_i = phi_{s i}(<d, swk~_{s i, 1}>).
  for (int i = 1; i < n1; ++i) {
    if (!baby[i]) continue;
    const long r = pg.stride * i;
    const uint64_t* key = need_key(c, km, r);
    Vec x(PL), y(PL);
    ks_inner(c, level, d.data(), key, x.data(), y.data());
    add_inplace(c, PQ, x.data(), A[0].data());
    A[i].resize(PL);
    B[i].resize(PL);
    automorph_ntt(c, r, x.data(), A[i].data(), K);
    automorph_ntt(c, r, y.data(), B[i].data(), K);
  }
  // Line 6: (c0, c1) = (0, 0).
  Vec C0(PL, 0), C1(PL, 0);
  // Lines 7-12: giant steps.
  for (int j = 0; j < n2; ++j) {
    bool any = false;
    for (int i = 0; i < n1; ++i) any |= has(n1 * j + i);
    if (!any) continue;
    // Line 8: (u0, u1) = sum_i (a_i, b_i) f^_{n1 j + i}.
    Vec U0(PL, 0), U1(PL, 0);
    for (int i = 0; i < n1; ++i) {
      if (!has(n1 * j + i)) continue;
      mac_inplace(c, PQ, U0.data(), A[i].data(), D.f[n1 * j + i]);
      mac_inplace(c, PQ, U1.data(), B[i].data(), D.f[n1 * j + i]);
    }
    const long G = mod_slots(c, pg.stride * ((long)n1 * j - pg.centre));
    if (G == 0) {  // no rotation: accumulated as is
      add_inplace(c, PQ, C0.data(), U0.data());
      add_inplace(c, PQ, C1.data(), U1.data());
      continue;
    }
    // Lines 9-12: u1 = ModDown(u1); d = Decompose(u1);
    // c0 += phi_G(u0 + <d, swk~_{G,0}>); c1 += phi_G(<d, swk~_{G,1}>).
    Vec u1q((size_t)(level + 1) * n), dg((size_t)beta * PL);
    moddown(c, level, U1.data(), u1q.data());
    decompose(c, level, u1q.data(), dg.data());
    const uint64_t* key = need_key(c, km, G);
    Vec x(PL), y(PL), t(PL);
    ks_inner(c, level, dg.data(), key, x.data(), y.data());
    add_inplace(c, PQ, x.data(), U0.data());
    automorph_ntt(c, G, x.data(), t.data(), K);
    add_inplace(c, PQ, C0.data(), t.data());
    automorph_ntt(c, G, y.data(), t.data(), K);
    add_inplace(c, PQ, C1.data(), t.data());
  }
  // Line 13: ct = rescale(ModDown(c0), ModDown(c1)).
  if (combined) {
    moddown_rescale(c, level, C0.data(), o0);
    moddown_rescale(c, level, C1.data(), o1);
  } else {
    Vec m0((size_t)(level + 1) * n), m1((size_t)(level + 1) * n);
    moddown(c, level, C0.data(), m0.data());
    moddown(c, level, C1.data(), m1.data());
    rescale(c, level, m0.data(), o0);
    rescale(c, level, m1.data(), o1);
  }
}

// ---------------------------------------------------------------------------
// Plain BSGS, eq. (5): f^_{n1 j + i} = phi_{-G_j}(f) at Q (L+1 limbs, prefix),
// baby rotations s*i, giant rotations G_j = s*(n1 j - centre).
// ---------------------------------------------------------------------------
void lt_bsgs(Ctx& c, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, Prog pg,
             const Diags& D, const KeyMap& km, uint64_t* o0, uint64_t* o1) {
  const int n = c.n, Lq = level + 1;
  const size_t QL = (size_t)Lq * n;
  const std::vector<int> Q = q_basis(c, level);
  auto has = [&](int m) { return m < D.n && D.f[m] != nullptr; };
  std::vector<char> used_i(n1, 0);
  for (int j = 0; j < n2; ++j) for (int i = 0; i < n1; ++i) if (has(n1 * j + i)) used_i[i] = 1;
  std::vector<Vec> R0(n1), R1(n1);
  R0[0].assign(c0, c0 + QL); R1[0].assign(c1, c1 + QL);
  for (int i = 1; i < n1; ++i) {
    if (!used_i[i]) continue;
    R0[i].resize(QL); R1[i].resize(QL);
    rotate(c, level, c0, c1, pg.stride * i, km, R0[i].data(), R1[i].data());
  }
  Vec A0(QL, 0), A1(QL, 0);
  for (int j = 0; j < n2; ++j) {
    bool any = false;
    for (int i = 0; i < n1; ++i) any |= has(n1 * j + i);
    if (!any) continue;
    Vec S0(QL, 0), S1(QL, 0);
    for (int i = 0; i < n1; ++i) {
      if (!has(n1 * j + i)) continue;
      mac_inplace(c, Q, S0.data(), R0[i].data(), D.f[n1 * j + i]);
      mac_inplace(c, Q, S1.data(), R1[i].data(), D.f[n1 * j + i]);
    }
    const long G = mod_slots(c, pg.stride * ((long)n1 * j - pg.centre));
    if (G == 0) {
      add_inplace(c, Q, A0.data(), S0.data());
      add_inplace(c, Q, A1.data(), S1.data());
    } else {
      Vec T0(QL), T1(QL);
      rotate(c, level, S0.data(), S1.data(), G, km, T0.data(), T1.data());
      add_inplace(c, Q, A0.data(), T0.data());
      add_inplace(c, Q, A1.data(), T1.data());
    }
  }
  rescale(c, level, A0.data(), o0);
  rescale(c, level, A1.data(), o1);
}

// Diagonal method: out = rescale(sum_t Rot(ct, s (t - centre)) f_t), f_t at Q.
void lt_naive(Ctx& c, int level, const uint64_t* c0, const uint64_t* c1, Prog pg, const Diags& D,
              const KeyMap& km, uint64_t* o0, uint64_t* o1) {
  const int n = c.n, Lq = level + 1;
  const size_t QL = (size_t)Lq * n;
  const std::vector<int> Q = q_basis(c, level);
  Vec A0(QL, 0), A1(QL, 0), R0(QL), R1(QL);
  for (int t = 0; t < D.n; ++t) {
    if (!D.f[t]) continue;
    const long d = mod_slots(c, pg.stride * (t - pg.centre));
    if (d == 0) { R0.assign(c0, c0 + QL); R1.assign(c1, c1 + QL); }
    else rotate(c, level, c0, c1, d, km, R0.data(), R1.data());
    mac_inplace(c, Q, A0.data(), R0.data(), D.f[t]);
    mac_inplace(c, Q, A1.data(), R1.data(), D.f[t]);
  }
  rescale(c, level, A0.data(), o0);
  rescale(c, level, A1.data(), o1);
}

// Signed integer coefficients -> NTT-form limbs over a list of PQ indices.
void poly_from_signed(const Ctx& c, const int64_t* coef, int nb, const int* basis, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int l = 0; l < nb; ++l) {
    uint64_t q = c.q(basis[l]);
    for (int k = 0; k < c.n; ++k) out[(size_t)l * c.n + k] = from_signed(coef[k], q);
    ntt(c, basis[l], out + (size_t)l * c.n);
  }
}

Ctx* as_ctx(void* p) { return static_cast<Ctx*>(p); }

KeyMap make_keys(int nkeys, const long* rots, const uint64_t* const* keys) {
  KeyMap km;
  for (int i = 0; i < nkeys; ++i) km.m[rots[i]] = keys[i];
  return km;
}
Diags make_diags(int n, const uint64_t* const* f) {
  Diags D; D.n = n; D.f.assign(f, f + n); return D;
}

}  // namespace

// ===========================================================================
// C interface for the Python test harness.  Every function returns 0 on
// success and a negative value on error (message in orc_last_error).
// ===========================================================================
extern "C" {

static thread_local std::string g_err;
const char* orc_last_error() { return g_err.c_str(); }

#define ORC_TRY(...) try { __VA_ARGS__; return 0; } catch (const std::exception& e) { g_err = e.what(); return -1; }

void* orc_ctx_create(int logn, int nq, const uint64_t* q, int np, const uint64_t* p, int dnum) {
  try {
    if (logn < 2 || logn > 17) throw std::runtime_error("bad log_n");
    Ctx* c = new Ctx;
    c->logn = logn; c->n = 1 << logn; c->L = nq - 1; c->alpha = np; c->dnum = dnum;
    if ((nq + np - 1) / np != dnum) { delete c; throw std::runtime_error("dnum != ceil((L+1)/alpha)"); }
    std::vector<uint64_t> all;
    for (int i = 0; i < np; ++i) all.push_back(p[i]);
    for (int j = 0; j < nq; ++j) all.push_back(q[j]);
    std::set<uint64_t> seen;
    for (uint64_t m : all) {
      if (!is_prime(m) || m % (2 * (uint64_t)c->n) != 1 || m >= (1ull << 61) || !seen.insert(m).second) {
        delete c; throw std::runtime_error("bad prime " + std::to_string(m));
      }
      PrimeTab t;
      t.q = m;
      t.psi = find_psi(m, c->n);
      t.psi_inv = invmod(t.psi, m);
      t.n_inv = invmod((uint64_t)c->n, m);
      t.psi_rev.resize(c->n); t.psi_inv_rev.resize(c->n);
      uint64_t pw = 1, pwi = 1;
      std::vector<uint64_t> pows(c->n), ipows(c->n);
      for (int i = 0; i < c->n; ++i) { pows[i] = pw; ipows[i] = pwi; pw = mulmod(pw, t.psi, m); pwi = mulmod(pwi, t.psi_inv, m); }
      for (int i = 0; i < c->n; ++i) { t.psi_rev[i] = pows[bitrev(i, logn)]; t.psi_inv_rev[i] = ipows[bitrev(i, logn)]; }
      c->pq.push_back(t);
    }
    return c;
  } catch (const std::exception& e) { g_err = e.what(); return nullptr; }
}

void orc_ctx_destroy(void* c) { delete as_ctx(c); }

uint64_t orc_psi(void* c, int pqi) { return as_ctx(c)->pq[pqi].psi; }

int orc_ntt(void* c, int pqi, uint64_t* a) { ORC_TRY(ntt(*as_ctx(c), pqi, a)) }
int orc_intt(void* c, int pqi, uint64_t* a) { ORC_TRY(intt(*as_ctx(c), pqi, a)) }
int orc_automorph_ntt(void* c, long r, const uint64_t* in, uint64_t* out, int limbs) {
  ORC_TRY(automorph_ntt(*as_ctx(c), r, in, out, limbs))
}
int orc_automorph_coeff(void* c, int pqi, uint64_t g, const uint64_t* in, uint64_t* out) {
  ORC_TRY(automorph_coeff(*as_ctx(c), pqi, g, in, out))
}
uint64_t orc_galois(void* c, long r) { return galois(*as_ctx(c), r); }

int orc_bconv(void* c, int ns, const int* src, const uint64_t* x, int nd, const int* dst, uint64_t* out) {
  ORC_TRY(bconv(*as_ctx(c), std::vector<int>(src, src + ns), x, std::vector<int>(dst, dst + nd), out))
}
int orc_decompose(void* c, int level, const uint64_t* x, uint64_t* digits) { ORC_TRY(decompose(*as_ctx(c), level, x, digits)) }
int orc_moddown(void* c, int level, const uint64_t* x, uint64_t* out) { ORC_TRY(moddown(*as_ctx(c), level, x, out)) }
int orc_moddown_rescale(void* c, int level, const uint64_t* x, uint64_t* out) { ORC_TRY(moddown_rescale(*as_ctx(c), level, x, out)) }
int orc_rescale(void* c, int level, const uint64_t* x, uint64_t* out) { ORC_TRY(rescale(*as_ctx(c), level, x, out)) }
int orc_ks_inner(void* c, int level, const uint64_t* digits, const uint64_t* key, uint64_t* x, uint64_t* y) {
  ORC_TRY(ks_inner(*as_ctx(c), level, digits, key, x, y))
}
int orc_p_scale(void* c, int level, const uint64_t* x, uint64_t* out) { ORC_TRY(p_scale(*as_ctx(c), level, x, out)) }

int orc_poly_from_signed(void* cv, const int64_t* coef, int nb, const int* basis, uint64_t* out) {
  ORC_TRY(poly_from_signed(*as_ctx(cv), coef, nb, basis, out))
}

// Ternary secret with Hamming weight h: h distinct positions, uniform signs.
int orc_keygen_secret(void* cv, uint64_t seed, int h) {
  ORC_TRY({
    Ctx& c = *as_ctx(cv);
    if (h < 0 || h > c.n) throw std::runtime_error("bad hamming weight");
    Rng g(seed, 1);
    c.s.assign(c.n, 0);
    int placed = 0;
    while (placed < h) {
      uint64_t pos = g.next() >> (64 - c.logn);
      if (c.s[pos] != 0) continue;
      c.s[pos] = (g.next() >> 63) ? 1 : -1;
      ++placed;
    }
    c.has_secret = true;
  })
}

int orc_get_secret(void* cv, int64_t* out) {
  ORC_TRY({ Ctx& c = *as_ctx(cv); if (!c.has_secret) throw std::runtime_error("no secret"); std::memcpy(out, c.s.data(), c.n * 8); })
}

// Rotation key swk~_r = phi_{-r}(swk_r), layout [beta_max][2][K_max][N] (NTT form).
int orc_gen_rotkey(void* cv, long r, uint64_t seed, double sigma, uint64_t* out) {
  ORC_TRY({
    Ctx& c = *as_ctx(cv);
    if (!c.has_secret) throw std::runtime_error("no secret");
    const int n = c.n, Kmax = c.K(c.L), beta = c.beta(c.L), a = c.alpha;
    const std::vector<int> PQ = pq_basis(c, c.L);
    Vec s_ntt((size_t)Kmax * n);
    for (int l = 0; l < Kmax; ++l) {
      for (int k = 0; k < n; ++k) s_ntt[(size_t)l * n + k] = from_signed(c.s[k], c.q(l));
      ntt(c, l, s_ntt.data() + (size_t)l * n);
    }
    Vec s_rot((size_t)Kmax * n);
    automorph_ntt(c, r, s_ntt.data(), s_rot.data(), Kmax);
    Rng g(seed, 1000 + (uint64_t)((r % (n / 2) + n / 2) % (n / 2)));
    Vec b0((size_t)Kmax * n), b1((size_t)Kmax * n);
    for (int b = 0; b < beta; ++b) {
      for (int l = 0; l < Kmax; ++l)
        for (int k = 0; k < n; ++k) b1[(size_t)l * n + k] = g.below(c.q(l));
      std::vector<int64_t> e(n);
      for (int k = 0; k < n; ++k) e[k] = g.gauss(sigma);
      for (int l = 0; l < Kmax; ++l) {
        uint64_t q = c.q(l);
        uint64_t* row = b0.data() + (size_t)l * n;
        for (int k = 0; k < n; ++k) row[k] = from_signed(e[k], q);
        ntt(c, l, row);
        const uint64_t* sa = b1.data() + (size_t)l * n;
        const uint64_t* ss = s_ntt.data() + (size_t)l * n;
        for (int k = 0; k < n; ++k) row[k] = submod(row[k], mulmod(sa[k], ss[k], q), q);
        int j = l - a;  // q_j index when l >= alpha
        if (j >= 0 && j / a == b) {
          uint64_t P = 1;
          for (int i = 0; i < a; ++i) P = mulmod(P, c.q(i) % q, q);
          const uint64_t* sr = s_rot.data() + (size_t)l * n;
          for (int k = 0; k < n; ++k) row[k] = addmod(row[k], mulmod(P, sr[k], q), q);
        }
      }
      automorph_ntt(c, -r, b0.data(), out + ((size_t)b * 2 + 0) * Kmax * n, Kmax);
      automorph_ntt(c, -r, b1.data(), out + ((size_t)b * 2 + 1) * Kmax * n, Kmax);
    }
  })
}

// Secret-key encryption at `level`: (c0, c1) = (-a s + e + m, a), NTT form.
int orc_encrypt(void* cv, int level, const int64_t* m, uint64_t seed, double sigma, uint64_t* c0, uint64_t* c1) {
  ORC_TRY({
    Ctx& c = *as_ctx(cv);
    if (!c.has_secret) throw std::runtime_error("no secret");
    const int n = c.n, a = c.alpha;
    Rng g(seed, 7);
    std::vector<int64_t> e(n);
    for (int k = 0; k < n; ++k) e[k] = g.gauss(sigma);
    for (int j = 0; j <= level; ++j) {
      uint64_t q = c.q(a + j);
      uint64_t* r1 = c1 + (size_t)j * n;
      uint64_t* r0 = c0 + (size_t)j * n;
      for (int k = 0; k < n; ++k) r1[k] = g.below(q);
      Vec s(n), em(n);
      for (int k = 0; k < n; ++k) { s[k] = from_signed(c.s[k], q); em[k] = addmod(from_signed(e[k], q), from_signed(m[k], q), q); }
      ntt(c, a + j, s.data());
      ntt(c, a + j, em.data());
      for (int k = 0; k < n; ++k) r0[k] = submod(em[k], mulmod(r1[k], s[k], q), q);
    }
  })
}

// Decrypt with limb q_0 only: m = [c0 + c1 s]_{q_0}, centred.
int orc_decrypt(void* cv, const uint64_t* c0, const uint64_t* c1, int64_t* m) {
  ORC_TRY({
    Ctx& c = *as_ctx(cv);
    const int n = c.n, a = c.alpha;
    uint64_t q = c.q(a);
    Vec s(n), t(n);
    for (int k = 0; k < n; ++k) s[k] = from_signed(c.s[k], q);
    ntt(c, a, s.data());
    for (int k = 0; k < n; ++k) t[k] = addmod(c0[k], mulmod(c1[k], s[k], q), q);
    intt(c, a, t.data());
    for (int k = 0; k < n; ++k) m[k] = t[k] > q / 2 ? (int64_t)t[k] - (int64_t)q : (int64_t)t[k];
  })
}

int orc_rotate(void* cv, int level, const uint64_t* c0, const uint64_t* c1, long r, int nkeys, const long* rots,
               const uint64_t* const* keys, uint64_t* o0, uint64_t* o1) {
  ORC_TRY(rotate(*as_ctx(cv), level, c0, c1, r, make_keys(nkeys, rots, keys), o0, o1))
}

int orc_lt_th(void* cv, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, int n3, long stride,
              long centre, int nd, const uint64_t* const* diags, int nkeys, const long* rots,
              const uint64_t* const* keys, uint64_t* o0, uint64_t* o1) {
  ORC_TRY(lt_th(*as_ctx(cv), level, c0, c1, n1, n2, n3, Prog{stride, centre}, make_diags(nd, diags),
                make_keys(nkeys, rots, keys), o0, o1))
}

int orc_lt_dh(void* cv, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, long stride, long centre,
              int combined, int nd, const uint64_t* const* diags, int nkeys, const long* rots,
              const uint64_t* const* keys, uint64_t* o0, uint64_t* o1) {
  ORC_TRY(lt_dh(*as_ctx(cv), level, c0, c1, n1, n2, Prog{stride, centre}, make_diags(nd, diags),
                make_keys(nkeys, rots, keys), combined != 0, o0, o1))
}

int orc_lt_bsgs(void* cv, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, long stride,
                long centre, int nd, const uint64_t* const* diags, int nkeys, const long* rots,
                const uint64_t* const* keys, uint64_t* o0, uint64_t* o1) {
  ORC_TRY(lt_bsgs(*as_ctx(cv), level, c0, c1, n1, n2, Prog{stride, centre}, make_diags(nd, diags),
                  make_keys(nkeys, rots, keys), o0, o1))
}

int orc_lt_naive(void* cv, int level, const uint64_t* c0, const uint64_t* c1, long stride, long centre, int nd,
                 const uint64_t* const* diags, int nkeys, const long* rots, const uint64_t* const* keys,
                 uint64_t* o0, uint64_t* o1) {
  ORC_TRY(lt_naive(*as_ctx(cv), level, c0, c1, Prog{stride, centre}, make_diags(nd, diags),
                   make_keys(nkeys, rots, keys), o0, o1))
}

// Operation counters since the last reset: [decompose, moddown, ks, ntt, intt, distinct keys].
void orc_counters(void* cv, long* out) {
  Ctx& c = *as_ctx(cv);
  out[0] = c.cnt.decompose; out[1] = c.cnt.moddown; out[2] = c.cnt.ks;
  out[3] = c.cnt.ntt; out[4] = c.cnt.intt; out[5] = (long)c.cnt.keys.size();
}
void orc_reset_counters(void* cv) { as_ctx(cv)->cnt = Counters(); }

}  // extern "C"
