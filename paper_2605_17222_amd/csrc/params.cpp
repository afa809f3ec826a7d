// Parameter-set creation: prime validation, psi, twiddle tables and the
// basis-conversion constants of eq. (3) / eq. (4) / eq. (1), uploaded once.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <set>

#include "host_util.hpp"
#include "internal.hpp"

namespace ckks {

namespace {

typedef unsigned __int128 u128;

uint64_t mm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t pw(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = mm(r, b, q);
    b = mm(b, b, q);
  }
  return r;
}

uint64_t inv(uint64_t a, uint64_t q) { return pw(a, q - 2, q); }

// Deterministic Miller-Rabin (exact below 3.3e24 with these witnesses).
bool prime(uint64_t n) {
  static const uint64_t w[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : w)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) d >>= 1, ++s;
  for (uint64_t a : w) {
    uint64_t x = pw(a, d, n);
    if (x == 1 || x == n - 1) continue;
    int i = 1;
    for (; i < s; ++i) {
      x = mm(x, x, n);
      if (x == n - 1) break;
    }
    if (i == s) return false;
  }
  return true;
}

uint64_t shoup_of(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

uint32_t brev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i, x >>= 1) r = (r << 1) | (x & 1);
  return r;
}

// -q^-1 mod 2^64 by Newton iteration (q odd).
uint64_t neg_inv64(uint64_t q) {
  uint64_t x = q;  // correct to 3 bits
  for (int i = 0; i < 6; ++i) x *= 2 - q * x;
  return (uint64_t)0 - x;
}

// Fill a plan for the conversion src -> dst (PQ indices).  sinv: product of
// the source primes inverted modulo each destination prime.
int make_plan(const std::vector<uint64_t>& pr, const std::vector<int>& src, const std::vector<int>& dst,
              BConvPlan* pl) {
  if ((int)src.size() > kMaxSrc || (int)dst.size() > kMaxDst || src.empty()) return CKKS_E_UNSUPPORTED;
  memset(pl, 0, sizeof(*pl));
  pl->ns = (int)src.size();
  pl->nd = (int)dst.size();
  u128 sum = 0;
  for (int j = 0; j < pl->ns; ++j) {
    pl->src[j] = src[j];
    sum += pr[src[j]];
  }
  // REDC of sum_j y_j c_jm needs sum_j s_j <= 2^64.
  if (sum > ((u128)1 << 64)) return CKKS_E_UNSUPPORTED;
  pl->split30 = 1;
  for (int j : src)
    if (pr[j] >= (1ull << 60)) pl->split30 = 0;
  for (int m : dst)
    if (pr[m] >= (1ull << 60)) pl->split30 = 0;
  for (int j = 0; j < pl->ns; ++j) {
    const uint64_t sj = pr[src[j]];
    uint64_t h = 1;
    for (int i = 0; i < pl->ns; ++i)
      if (i != j) h = mm(h, pr[src[i]] % sj, sj);
    pl->hinv[j] = inv(h, sj);
    pl->hinv_sh[j] = shoup_of(pl->hinv[j], sj);
  }
  for (int m = 0; m < pl->nd; ++m) {
    const uint64_t d = pr[dst[m]];
    pl->dst[m] = dst[m];
    const uint64_t r64 = (uint64_t)(((u128)1 << 64) % d);
    uint64_t all = 1;
    for (int j = 0; j < pl->ns; ++j) {
      uint64_t h = 1;
      for (int i = 0; i < pl->ns; ++i)
        if (i != j) h = mm(h, pr[src[i]] % d, d);
      pl->hmod[m][j] = mm(h, r64, d);
      pl->hk[m][j][0] = (uint32_t)(pl->hmod[m][j] & ((1ull << 30) - 1));
      pl->hk[m][j][1] = (uint32_t)(pl->hmod[m][j] >> 30);
      all = mm(all, pr[src[j]] % d, d);
    }
    pl->sinv[m] = inv(all, d);
    pl->sinv_sh[m] = shoup_of(pl->sinv[m], d);
  }
  return CKKS_OK;
}

double as_double(uint64_t x) { return (double)x; }

// Row-pass twiddle factors of one prime and direction (root rho = psi or
// psi^-1); layout as in ntt_row_tables_size.  Returns false if a product
// G * R differs from the full table `full` (rho^br(i) for i < N), which is
// checked for every entry the row pass uses.
bool row_tables(uint64_t q, uint64_t rho, int log_n, const uint64_t* full, double* out) {
  const int B = ntt_row_log(log_n), L1 = log_n - B;
  const uint64_t n = 1ull << log_n, two_n = 2 * n;
  const size_t rows = (size_t)1 << L1;
  std::vector<uint64_t> G((size_t)1 << B, 0), R(rows * B);
  for (int s = 0; s < B; ++s)
    for (uint32_t y = 0; y < (1u << s); ++y) {
      const uint64_t e = ((1ull << (B - 1 - s)) + (uint64_t)brev(y, s) * (n >> s)) % two_n;
      G[(1u << s) + y] = pw(rho, e, q);
    }
  for (size_t row = 0; row < rows; ++row)
    for (int s = 0; s < B; ++s) R[row * B + s] = pw(rho, ((uint64_t)brev((uint32_t)row, L1) << (B - s)) % two_n, q);
  for (size_t row = 0; row < rows; ++row)
    for (int s = 0; s < B; ++s)
      for (uint32_t y = 0; y < (1u << s); ++y) {
        const size_t i = ((size_t)1 << (L1 + s)) + row * ((size_t)1 << s) + y;
        if (mm(G[(1u << s) + y], R[row * B + s], q) != full[i]) return false;
      }
  for (size_t k = 0; k < G.size(); ++k) out[k] = as_double(G[k]);
  double* r = out + G.size();
  for (size_t k = 0; k < R.size(); ++k) {
    r[2 * k] = as_double(R[k]);
    r[2 * k + 1] = as_double(R[k]) / (double)q;
  }
  return true;
}

}  // namespace

int params_create(const ckks_params_desc* d, ckks_params** out) {
  if (!d || !out || !d->q || !d->p) return CKKS_E_INVALID_ARG;
  *out = nullptr;
  if (d->log_n < 12 || d->log_n > 16 || d->n_q < 1 || d->n_p < 1 || d->dnum < 1) return CKKS_E_INVALID_ARG;
  if ((d->n_q + d->n_p - 1) / d->n_p != d->dnum) return CKKS_E_INVALID_ARG;  // digits of alpha primes
  if (d->n_q + d->n_p > kMaxDst) return CKKS_E_UNSUPPORTED;
  ckks_params* P = new ckks_params;
  Cleanup<ckks_params> guard(P);
  P->log_n = d->log_n;
  P->n = 1 << d->log_n;
  P->L = d->n_q - 1;
  P->alpha = d->n_p;
  P->dnum = d->dnum;
  P->beta_max = P->beta(P->L);
  if (P->beta_max > kMaxBeta) return CKKS_E_UNSUPPORTED;
  const uint64_t two_n = 2 * (uint64_t)P->n;
  std::set<uint64_t> seen;
  for (int i = 0; i < d->n_p; ++i) P->primes.push_back(d->p[i]);
  for (int j = 0; j < d->n_q; ++j) P->primes.push_back(d->q[j]);
  for (uint64_t q : P->primes) {
    if (q >= (1ull << 61) || q % two_n != 1 || !prime(q) || !seen.insert(q).second) return CKKS_E_INVALID_ARG;
  }
  const int K = P->Kmax(), n = P->n;
  if (hipGetDevice(&P->device) != hipSuccess) return CKKS_E_DEVICE;

  // psi and twiddle tables.
  std::vector<uint64_t> tw((size_t)K * 4 * n);
  const size_t rts = ntt_row_tables_size(P->log_n);
  std::vector<double> trow((size_t)K * 2 * rts, 0.0);
  std::vector<PrimeDev> pd(K);
  for (int i = 0; i < K; ++i) {
    const uint64_t q = P->primes[i];
    uint64_t psi;
    if (d->psi) {
      psi = d->psi[i] % q;
    } else {
      uint64_t g = 2;
      while (pw(g, (q - 1) / 2, q) != q - 1) ++g;  // smallest quadratic non-residue
      psi = pw(g, (q - 1) / two_n, q);
    }
    if (pw(psi, n, q) != q - 1) return CKKS_E_INVALID_ARG;  // not a primitive 2N-th root
    const uint64_t psi_inv = inv(psi, q);
    uint64_t* t = tw.data() + (size_t)i * 4 * n;
    std::vector<uint64_t> pf(n), pi(n);
    uint64_t a = 1, b = 1;
    for (int k = 0; k < n; ++k) {
      pf[k] = a;
      pi[k] = b;
      a = mm(a, psi, q);
      b = mm(b, psi_inv, q);
    }
    const bool fp = q < kFpPrimeLimit;
    if (fp) {
      std::vector<uint64_t> full_f(n), full_i(n);
      for (int k = 0; k < n; ++k) {
        const uint32_t r = brev(k, P->log_n);
        full_f[k] = pf[r];
        full_i[k] = pi[r];
      }
      double* tr = trow.data() + (size_t)i * 2 * rts;
      if (!row_tables(q, psi, P->log_n, full_f.data(), tr) || !row_tables(q, psi_inv, P->log_n, full_i.data(), tr + rts))
        return CKKS_E_UNSUPPORTED;  // internal consistency check of the factorisation
    }
    auto dbits = [](double x) {
      uint64_t u;
      memcpy(&u, &x, 8);
      return u;
    };
    for (int k = 0; k < n; ++k) {
      const uint32_t r = brev(k, P->log_n);
      if (fp) {
        t[k] = dbits((double)pf[r]);
        t[n + k] = dbits((double)pf[r] / (double)q);
        t[2 * n + k] = dbits((double)pi[r]);
        t[3 * n + k] = dbits((double)pi[r] / (double)q);
      } else {
        t[k] = pf[r];
        t[n + k] = shoup_of(pf[r], q);
        t[2 * n + k] = pi[r];
        t[3 * n + k] = shoup_of(pi[r], q);
      }
    }
    PrimeDev& c = pd[i];
    c.fp = fp ? 1 : 0;
    c.qd = (double)q;
    c.qinv_d = 1.0 / (double)q;
    c.q = q;
    c.qinv_neg = neg_inv64(q);
    const u128 r = (~(u128)0) / q;  // floor(2^128 / q): q odd, does not divide 2^128
    c.r_lo = (uint64_t)r;
    c.r_hi = (uint64_t)(r >> 64);
    c.ninv = inv((uint64_t)n % q, q);
    c.ninv_sh = shoup_of(c.ninv, q);
    c.ninv_d = (double)c.ninv;
    c.ninv_q = (double)c.ninv / (double)q;
    uint64_t Pm = 1;
    for (int k = 0; k < P->alpha; ++k) Pm = mm(Pm, P->primes[k] % q, q);
    c.pmod = i < P->alpha ? 0 : Pm;
    c.pmod_sh = shoup_of(c.pmod, q);
    c.narrow = q < kNarrowLimit ? 1 : 0;
    c.pk_off = P->pk_poly_bytes;
    c.pk_pad = 0;
    P->pk_poly_bytes += (uint64_t)n * (c.narrow ? 5 : 8);
  }

  // Basis-conversion plans.
  std::vector<BConvPlan> plans;
  auto add_plan = [&](const std::vector<int>& src, const std::vector<int>& dst) -> int {
    plans.emplace_back();
    int e = make_plan(P->primes, src, dst, &plans.back());
    if (e != CKKS_OK) return e;
    return (int)plans.size() - 1;
  };
  const int a = P->alpha;
  P->plan_decomp.assign((size_t)(P->L + 1) * P->beta_max, -1);
  P->plan_moddown.assign(P->L + 1, -1);
  P->plan_mdrescale.assign(P->L + 1, -1);
  P->plan_rescale.assign(P->L + 1, -1);
  for (int lv = 0; lv <= P->L; ++lv) {
    const int Kl = P->K(lv);
    for (int b = 0; b < P->beta(lv); ++b) {
      const int lo = b * a, hi = std::min(lo + a - 1, lv);
      std::vector<int> src, dst;
      for (int j = lo; j <= hi; ++j) src.push_back(a + j);
      for (int i = 0; i < Kl; ++i)
        if (i < a + lo || i > a + hi) dst.push_back(i);
      int id = add_plan(src, dst);
      if (id < 0) return id;
      P->plan_decomp[(size_t)lv * P->beta_max + b] = id;
    }
    std::vector<int> ps, qs, qs1;
    for (int i = 0; i < a; ++i) ps.push_back(i);
    for (int j = 0; j <= lv; ++j) qs.push_back(a + j);
    for (int j = 0; j < lv; ++j) qs1.push_back(a + j);
    int id = add_plan(ps, qs);
    if (id < 0) return id;
    P->plan_moddown[lv] = id;
    if (lv >= 1) {
      std::vector<int> pq = ps;
      pq.push_back(a + lv);
      id = add_plan(pq, qs1);
      if (id < 0) return id;
      P->plan_mdrescale[lv] = id;
      id = add_plan(std::vector<int>{a + lv}, qs1);
      if (id < 0) return id;
      P->plan_rescale[lv] = id;
    }
  }

  // Encoding tables.
  const int S = n / 2;
  std::vector<int> perm(S, -1);
  std::vector<double> etw(2 * (size_t)S), ezinv(2 * (size_t)S);
  {
    uint64_t e = 1;
    for (int t = 0; t < S; ++t) {
      perm[(e - 1) / 4] = t;
      e = e * 5 % two_n;
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < S; ++k) {
      const long double a = -2 * pi * (long double)k / (long double)S;
      etw[2 * k] = (double)std::cos(a);
      etw[2 * k + 1] = (double)std::sin(a);
      const long double b = -pi * (long double)k / (long double)n;
      ezinv[2 * k] = (double)(std::cos(b) / S);
      ezinv[2 * k + 1] = (double)(std::sin(b) / S);
    }
  }

  // Upload.
  if (hipMalloc(&P->d_tw, tw.size() * 8) != hipSuccess) return CKKS_E_NOMEM;
  if (hipMalloc(&P->d_trow, trow.size() * 8) != hipSuccess) return CKKS_E_NOMEM;
  if (hipMalloc(&P->d_primes, pd.size() * sizeof(PrimeDev)) != hipSuccess) return CKKS_E_NOMEM;
  for (const BConvPlan& pl : plans) {
    P->plan_shape.push_back({pl.ns, pl.nd});
    P->plan_split30.push_back(pl.split30 ? 1 : 0);
  }
  if (hipMalloc(&P->d_plans, plans.size() * sizeof(BConvPlan)) != hipSuccess) return CKKS_E_NOMEM;
  if (hipMalloc(&P->d_enc_perm, perm.size() * sizeof(int)) != hipSuccess) return CKKS_E_NOMEM;
  if (hipMalloc(&P->d_enc_tw, etw.size() * 8) != hipSuccess) return CKKS_E_NOMEM;
  if (hipMalloc(&P->d_enc_zinv, ezinv.size() * 8) != hipSuccess) return CKKS_E_NOMEM;
  for (int i = 0; i < K; ++i) {
    pd[i].tw = P->d_tw + (size_t)i * 4 * n;
    pd[i].trow = P->d_trow + (size_t)i * 2 * rts;
  }
  if (hipMemcpy(P->d_tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return CKKS_E_DEVICE;
  if (hipMemcpy(P->d_trow, trow.data(), trow.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return CKKS_E_DEVICE;
  if (hipMemcpy(P->d_primes, pd.data(), pd.size() * sizeof(PrimeDev), hipMemcpyHostToDevice) != hipSuccess)
    return CKKS_E_DEVICE;
  if (hipMemcpy(P->d_plans, plans.data(), plans.size() * sizeof(BConvPlan), hipMemcpyHostToDevice) != hipSuccess)
    return CKKS_E_DEVICE;
  if (hipMemcpy(P->d_enc_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_enc_tw, etw.data(), etw.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_enc_zinv, ezinv.data(), ezinv.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return CKKS_E_DEVICE;
  *out = guard.release();
  return CKKS_OK;
}

void params_destroy(ckks_params* P) {
  if (!P) return;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  if (cur != P->device) (void)hipSetDevice(P->device);
  if (P->d_tw) (void)hipFree(P->d_tw);
  if (P->d_trow) (void)hipFree(P->d_trow);
  if (P->d_primes) (void)hipFree(P->d_primes);
  if (P->d_plans) (void)hipFree(P->d_plans);
  if (P->d_enc_perm) (void)hipFree(P->d_enc_perm);
  if (P->d_enc_tw) (void)hipFree(P->d_enc_tw);
  if (P->d_enc_zinv) (void)hipFree(P->d_enc_zinv);
  if (cur >= 0 && cur != P->device) (void)hipSetDevice(cur);
  delete P;
}

uint32_t galois(const ckks_params* P, long r) {
  const long S = P->n / 2;
  const long rr = ((r % S) + S) % S;
  return (uint32_t)pw(5, (uint64_t)rr, 2 * (uint64_t)P->n);
}

}  // namespace ckks
