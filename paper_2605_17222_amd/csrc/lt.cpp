// Host orchestration of the HE-LT on one HIP stream, and the C interface.
//
// Every public call first runs its plan "dry" (no launches) to validate the
// arguments, find the rotation keys it needs and size its workspace, then runs
// it for real; both runs take the same code path, so the sizes always match.
#include <string.h>

#include <map>
#include <vector>

#include "host_util.hpp"
#include "internal.hpp"

namespace ckks {

namespace {

struct Run {
  const ckks_params* P = nullptr;
  hipStream_t s = nullptr;
  Workspace ws;
  bool dry = true;
  int err = CKKS_OK;
  size_t N = 0;

  void fail(int e) {
    if (err == CKKS_OK) err = e;
  }
  void check(hipError_t e) {
    if (e != hipSuccess) fail(CKKS_E_DEVICE);
  }
  uint64_t* limbs(size_t c) { return ws.limbs(c); }
};

// ---- primitive steps ------------------------------------------------------

LimbRange range(const uint64_t* in, uint64_t* out, int prime0, int count, const uint64_t* aux = nullptr,
                uint64_t* copy = nullptr) {
  LimbRange r;
  r.in = in;
  r.out = out;
  r.aux = aux;
  r.prime0 = prime0;
  r.count = count;
  r.copy = copy;
  r.epi0 = 0;
  r.pad = 0;
  return r;
}

void ntt_range(Run& R, bool fwd, int prime0, int count, const uint64_t* in, uint64_t* out) {
  if (R.dry || R.err || count <= 0) return;
  NttArgs a;
  a.nr = 1;
  a.r[0] = range(in, out, prime0, count);
  R.check(launch_ntt(R.P, fwd, a, count, EPI_NONE, nullptr, R.s));
}

// Collects limb ranges into NTT launches (flushing when the table is full).
struct NttBatch {
  Run& R;
  bool fwd;
  int epi;
  const BConvPlan* plan;
  NttArgs a;
  int total = 0;
  NttBatch(Run& r, bool f, int e = EPI_NONE, const BConvPlan* pl = nullptr) : R(r), fwd(f), epi(e), plan(pl) {
    a.nr = 0;
  }
  void add(const LimbRange& r) {
    if (r.count <= 0) return;
    if (a.nr == kMaxRanges) flush();
    a.r[a.nr++] = r;
    total += r.count;
  }
  void flush() {
    if (a.nr && !R.dry && !R.err) R.check(launch_ntt(R.P, fwd, a, total, epi, plan, R.s));
    a.nr = 0;
    total = 0;
  }
  ~NttBatch() { flush(); }
};

// Collects basis conversions with the same number of source limbs.
struct BConvBatch {
  Run& R;
  int ns;
  BConvArgs a;
  int items = 0;
  BConvBatch(Run& r, int n) : R(r), ns(n) { reset(); }
  void reset() {
    memset(&a, 0, sizeof(a));
    items = 0;
  }
  void add(const BConvPlan* plan, int nd, const uint64_t* src, uint64_t* dst, int shift) {
    if (items == kMaxConv) flush();
    a.plan[items] = plan;
    a.src[items] = src;
    a.dst[items] = dst;
    a.dst_shift[items] = shift;
    a.limbs_moved += ns + nd;
    a.max_nd = std::max(a.max_nd, nd);
    ++items;
  }
  void flush() {
    if (items && !R.dry && !R.err) R.check(launch_bconv(R.P, a, items, ns, R.s));
    reset();
  }
  ~BConvBatch() { flush(); }
};

typedef std::vector<std::pair<const uint64_t*, uint64_t*>> IOList;

// Decompose (Fig. 1) of several level-l Q-basis polynomials (NTT form) into
// digits [beta][K][N] each.  The inverse NTT's first pass also stores each
// group's own limbs, unchanged, into its digit (ModUp keeps them, R15).
void decompose(Run& R, int level, const IOList& xs) {
  const ckks_params* P = R.P;
  const int a = P->alpha, K = P->K(level), beta = P->beta(level), Lq = level + 1;
  const size_t N = R.N, mark = R.ws.mark();
  std::vector<uint64_t*> coef(xs.size());
  for (size_t t = 0; t < xs.size(); ++t) coef[t] = R.limbs(Lq);
  if (!R.dry && !R.err) {
    {
      NttBatch inv(R, false);
      for (size_t t = 0; t < xs.size(); ++t)
        for (int b = 0; b < beta; ++b) {
          const int lo = b * a, hi = std::min(lo + a - 1, level);
          inv.add(range(xs[t].first + (size_t)lo * N, coef[t] + (size_t)lo * N, a + lo, hi - lo + 1, nullptr,
                        xs[t].second + ((size_t)b * K + a + lo) * N));
        }
    }
    // Digits with a full group of alpha limbs share launches; a shorter last
    // group has its own.
    const int last = level - (beta - 1) * a + 1;
    {
      BConvBatch full(R, a);
      BConvBatch part(R, last);
      for (size_t t = 0; t < xs.size(); ++t)
        for (int b = 0; b < beta; ++b) {
          const int lo = b * a, hi = std::min(lo + a - 1, level), g = hi - lo + 1;
          const BConvPlan* pl = P->plan(P->plan_decomp[(size_t)level * P->beta_max + b]);
          (g == a ? full : part).add(pl, K - g, coef[t] + (size_t)lo * N, xs[t].second + (size_t)b * K * N, 0);
        }
    }
    NttBatch fwd(R, true);
    for (size_t t = 0; t < xs.size(); ++t)
      for (int b = 0; b < beta; ++b) {
        const int lo = b * a, hi = std::min(lo + a - 1, level);
        uint64_t* d = xs[t].second + (size_t)b * K * N;
        fwd.add(range(d, d, 0, a + lo));
        fwd.add(range(d + (size_t)(a + hi + 1) * N, d + (size_t)(a + hi + 1) * N, a + hi + 1, K - (a + hi + 1)));
      }
  }
  R.ws.reset(mark);
}

void decompose(Run& R, int level, const uint64_t* x, uint64_t* digits) { decompose(R, level, IOList{{x, digits}}); }

enum DivKind { DIV_MODDOWN, DIV_MODDOWN_RESCALE, DIV_RESCALE };

// Division step of eq. (4) / eq. (1), for several inputs of the same kind:
//  DIV_MODDOWN:         x [alpha+l+1] -> out [l+1], divide by P
//  DIV_MODDOWN_RESCALE: x [alpha+l+1] -> out [l],   divide by P q_l
//  DIV_RESCALE:         x [l+1]       -> out [l],   divide by q_l
void divide(Run& R, DivKind kind, int level, const IOList& xs) {
  const ckks_params* P = R.P;
  const int a = P->alpha;
  const size_t N = R.N, mark = R.ws.mark();
  int plan_idx, ns, nout;
  if (kind == DIV_MODDOWN) {
    plan_idx = P->plan_moddown[level];
    ns = a;
    nout = level + 1;
  } else if (kind == DIV_MODDOWN_RESCALE) {
    plan_idx = P->plan_mdrescale[level];
    ns = a + 1;
    nout = level;
  } else {
    plan_idx = P->plan_rescale[level];
    ns = 1;
    nout = level;
  }
  std::vector<uint64_t*> coef(xs.size());
  for (size_t t = 0; t < xs.size(); ++t) coef[t] = R.limbs(ns);
  if (!R.dry && !R.err) {
    const BConvPlan* plan = P->plan(plan_idx);
    {
      NttBatch inv(R, false);
      for (size_t t = 0; t < xs.size(); ++t) {
        const uint64_t* x = xs[t].first;
        if (kind == DIV_RESCALE) {
          inv.add(range(x + (size_t)level * N, coef[t], a + level, 1));
        } else {
          inv.add(range(x, coef[t], 0, a));
          if (kind == DIV_MODDOWN_RESCALE)
            inv.add(range(x + (size_t)(a + level) * N, coef[t] + (size_t)a * N, a + level, 1));
        }
      }
    }
    {
      BConvBatch bc(R, ns);
      for (size_t t = 0; t < xs.size(); ++t) bc.add(plan, nout, coef[t], xs[t].second, a);
    }
    NttBatch fwd(R, true, EPI_SUBMUL, plan);
    for (size_t t = 0; t < xs.size(); ++t) {
      const uint64_t* keep = kind == DIV_RESCALE ? xs[t].first : xs[t].first + (size_t)a * N;
      fwd.add(range(xs[t].second, xs[t].second, a, nout, keep));
    }
  }
  R.ws.reset(mark);
}

void divide(Run& R, DivKind kind, int level, const uint64_t* x, uint64_t* out) {
  divide(R, kind, level, IOList{{x, out}});
}

// Key-switch inner products of several digit sets with several keys, phi on
// write (hoisting: each digit set and each key is read once per launch).
struct KsDigit {
  const uint64_t* digits;
  const uint64_t* add;   // may be null
  bool add_pscaled;
};
struct KsKey {
  const uint64_t* key;
  uint32_t gal_inv;
};
// out[i][k] = {a, b} destination of digit set i with key k (nulls skip).
void keyswitch(Run& R, int level, const std::vector<KsDigit>& dig, const std::vector<KsKey>& keys,
               const std::vector<std::vector<std::pair<uint64_t*, uint64_t*>>>& out, bool accumulate) {
  if (R.dry || R.err || dig.empty() || keys.empty()) return;
  const ckks_params* P = R.P;
  for (size_t i0 = 0; i0 < dig.size(); i0 += kMaxDig) {
    for (size_t k0 = 0; k0 < keys.size(); k0 += kMaxKs) {
      KsArgs ka;
      memset(&ka, 0, sizeof(ka));
      ka.beta = P->beta(level);
      ka.K = P->K(level);
      ka.kmax = P->Kmax();
      ka.accumulate = accumulate ? 1 : 0;
      ka.ndig = (int)std::min(dig.size() - i0, (size_t)kMaxDig);
      ka.nkeys = (int)std::min(keys.size() - k0, (size_t)kMaxKs);
      for (int i = 0; i < ka.ndig; ++i) {
        ka.digits[i] = dig[i0 + i].digits;
        ka.add[i] = dig[i0 + i].add;
        ka.add_pscaled[i] = dig[i0 + i].add_pscaled ? 1 : 0;
        for (int k = 0; k < ka.nkeys; ++k) {
          ka.out_a[i][k] = out[i0 + i][k0 + k].first;
          ka.out_b[i][k] = out[i0 + i][k0 + k].second;
        }
      }
      for (int k = 0; k < ka.nkeys; ++k) {
        ka.key[k] = keys[k0 + k].key;
        ka.gal_inv[k] = keys[k0 + k].gal_inv;
      }
      R.check(launch_keyswitch(P, ka, R.s));
    }
  }
}

struct MacTerm {
  const uint64_t* a;
  const uint64_t* b;
  bool pscaled;
  std::vector<const uint64_t*> f;  // per output k (null = absent)
};

// outs[k] = sum_m terms[m] * f[k], over nlimbs limbs starting at prime_off.
void ptmac(Run& R, int nlimbs, int prime_off, const std::vector<MacTerm>& terms, const std::vector<uint64_t*>& o0,
           const std::vector<uint64_t*>& o1) {
  if (R.dry || R.err) return;
  const int nk_all = (int)o0.size();
  for (int k0 = 0; k0 < nk_all; k0 += kMaxMacK) {
    const int nk = std::min(kMaxMacK, nk_all - k0);
    bool first = true;
    for (size_t m0 = 0; m0 < std::max<size_t>(terms.size(), 1); m0 += kMaxMacM) {
      MacArgs ma;
      memset(&ma, 0, sizeof(ma));
      ma.nk = nk;
      ma.K = nlimbs;
      ma.prime_off = prime_off;
      ma.accumulate = first ? 0 : 1;
      int nm = 0;
      for (size_t m = m0; m < std::min(terms.size(), m0 + kMaxMacM); ++m, ++nm) {
        ma.a[nm] = terms[m].a;
        ma.b[nm] = terms[m].b;
        if (terms[m].pscaled) {
          if (nm != 0) {
            R.fail(CKKS_E_INVALID_ARG);
            return;
          }
          ma.pscaled0 = 1;
        }
        for (int k = 0; k < nk; ++k) ma.f[k][nm] = terms[m].f[k0 + k];
      }
      ma.nm = nm;
      for (int k = 0; k < nk; ++k) {
        ma.out0[k] = o0[k0 + k];
        ma.out1[k] = o1[k0 + k];
      }
      R.check(launch_ptmac(R.P, ma, R.s));
      first = false;
    }
  }
}

void automorph(Run& R, int nlimbs, int prime_off, uint32_t gal, const uint64_t* in, const uint64_t* add,
               uint64_t* out, bool accumulate) {
  if (R.dry || R.err) return;
  AutoArgs aa{in, add, out, nlimbs, prime_off, accumulate ? 1 : 0, gal};
  R.check(launch_automorph(R.P, aa, R.s));
}

// ---- keys -------------------------------------------------------------------

struct KeySet {
  std::map<long, const uint64_t*> m;
  long S = 0;
  const uint64_t* get(Run& R, long r) const {
    const long rr = ((r % S) + S) % S;
    auto it = m.find(rr);
    if (it == m.end() || !it->second) {
      R.fail(CKKS_E_UNSUPPORTED);
      return nullptr;
    }
    return it->second;
  }
};

// Rot(ct, r) = (phi_r(c0 + x), phi_r(y)), (x, y) = ModDown(<Decompose(c1), swk~_r>),
// for several independent rotations at once (each with its own Decompose, as
// plain BSGS and the diagonal method prescribe; only the launches are shared).
struct RotJob {
  const uint64_t* c0;
  const uint64_t* c1;
  long r;
  uint64_t* o0;
  uint64_t* o1;
  bool accumulate;  // o += Rot(ct, r)
};

void rotate(Run& R, int level, const std::vector<RotJob>& jobs, const KeySet& ks) {
  const ckks_params* P = R.P;
  const int K = P->K(level), Lq = level + 1, beta = P->beta(level);
  for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxDig) {
    const size_t nj = std::min(jobs.size() - j0, (size_t)kMaxDig);
    const size_t mark = R.ws.mark();
    std::vector<uint64_t*> D(nj), X(nj), Y(nj), Xq(nj), Yq(nj);
    IOList dc, md;
    std::vector<KsDigit> dig;
    std::vector<KsKey> keys;
    std::vector<std::vector<std::pair<uint64_t*, uint64_t*>>> out(nj);
    for (size_t t = 0; t < nj; ++t) {
      D[t] = R.limbs((size_t)beta * K);
      X[t] = R.limbs(K);
      Y[t] = R.limbs(K);
      Xq[t] = R.limbs(Lq);
      Yq[t] = R.limbs(Lq);
    }
    for (size_t t = 0; t < nj; ++t) {
      const RotJob& J = jobs[j0 + t];
      dc.push_back({J.c1, D[t]});
      md.push_back({X[t], Xq[t]});
      md.push_back({Y[t], Yq[t]});
      dig.push_back(KsDigit{D[t], nullptr, false});
      keys.push_back(KsKey{ks.get(R, J.r), 1u});
      for (size_t u = 0; u < nj; ++u)
        out[t].push_back(u == t ? std::make_pair(X[t], Y[t]) : std::make_pair((uint64_t*)nullptr, (uint64_t*)nullptr));
    }
    decompose(R, level, dc);
    keyswitch(R, level, dig, keys, out, false);
    divide(R, DIV_MODDOWN, level, md);
    for (size_t t = 0; t < nj; ++t) {
      const RotJob& J = jobs[j0 + t];
      const uint32_t g = galois(P, J.r);
      automorph(R, Lq, P->alpha, g, Xq[t], J.c0, J.o0, J.accumulate);
      automorph(R, Lq, P->alpha, g, Yq[t], nullptr, J.o1, J.accumulate);
    }
    R.ws.reset(mark);
  }
}

struct Diag {
  int n = 0;
  const uint64_t* const* pt = nullptr;
  bool has(int m) const { return m >= 0 && m < n && pt[m] != nullptr; }
};

// ---- triple-hoisted BSGS, Algorithm 2 ----------------------------------------
void lt_th(Run& R, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, int n3, const Diag& D,
           const KeySet& ks, uint64_t* o0, uint64_t* o1) {
  const ckks_params* P = R.P;
  const int K = P->K(level), beta = P->beta(level), inner = n1 * n2, Lq = level + 1;
  const size_t N = R.N;
  std::vector<char> used_m(inner, 0), used_i(n1, 0), mid_i(n1, 0), used_k(n3, 0);
  for (int k = 0; k < n3; ++k)
    for (int m = 0; m < inner; ++m)
      if (D.has(k * inner + m)) used_m[m] = 1, used_k[k] = 1;
  for (int m = 0; m < inner; ++m)
    if (used_m[m]) {
      used_i[m % n1] = 1;
      if (m >= n1) mid_i[m % n1] = 1;
    }
  bool need_d0 = mid_i[0];
  for (int i = 1; i < n1; ++i) need_d0 = need_d0 || used_i[i];

  std::vector<uint64_t*> Dg(n1, nullptr), A(inner, nullptr), B(inner, nullptr);
  for (int i = 0; i < n1; ++i)
    if ((i == 0 && need_d0) || (i > 0 && mid_i[i])) Dg[i] = R.limbs((size_t)beta * K);
  for (int m = 1; m < inner; ++m)
    if (used_m[m] || (m < n1 && used_i[m])) {
      A[m] = R.limbs(K);
      B[m] = R.limbs(K);
    }
  std::vector<uint64_t*> U0(n3, nullptr), U1(n3, nullptr);
  for (int k = 0; k < n3; ++k) {
    U0[k] = R.limbs(K);
    U1[k] = R.limbs(K);
  }
  std::vector<uint64_t*> tmpQ(n1, nullptr), tmpK(n3, nullptr), Dk(n3, nullptr);
  for (int i = 1; i < n1; ++i)
    if (mid_i[i]) tmpQ[i] = R.limbs(Lq);
  for (int k = 1; k < n3; ++k)
    if (used_k[k]) {
      tmpK[k] = R.limbs(Lq);
      Dk[k] = R.limbs((size_t)beta * K);
    }

  // Line 1: d_0 = Decompose(c1').
  if (need_d0) decompose(R, level, c1, Dg[0]);
  // Lines 3-5: inner rotations share d_0; a_0 = P c0' is applied inside the kernel.
  {
    std::vector<KsKey> keys;
    std::vector<std::vector<std::pair<uint64_t*, uint64_t*>>> out(1);
    for (int i = 1; i < n1; ++i) {
      if (!used_i[i]) continue;
      keys.push_back(KsKey{ks.get(R, i), galois(P, -i)});
      out[0].push_back({A[i], B[i]});
    }
    keyswitch(R, level, {KsDigit{Dg[0], c0, true}}, keys, out, false);
  }
  // Lines 6-7: d_i = Decompose(ModDown(b_i)), all i at once (independent).
  {
    IOList md, dc;
    for (int i = 1; i < n1; ++i) {
      if (!mid_i[i]) continue;
      md.push_back({B[i], tmpQ[i]});
      dc.push_back({tmpQ[i], Dg[i]});
    }
    if (!md.empty()) {
      divide(R, DIV_MODDOWN, level, md);
      decompose(R, level, dc);
    }
  }
  // Lines 8-11: middle rotations by n1 j share d_i; one launch reads every
  // middle key once for all digit sets d_0 .. d_{n1-1}.
  {
    std::vector<KsDigit> dig;
    std::vector<int> di;
    for (int i = 0; i < n1; ++i)
      if (mid_i[i]) {
        dig.push_back(KsDigit{Dg[i], i == 0 ? c0 : A[i], i == 0});
        di.push_back(i);
      }
    std::vector<KsKey> keys;
    std::vector<int> kj;
    for (int j = 1; j < n2; ++j) {
      bool any = false;
      for (int i : di) any = any || used_m[n1 * j + i];
      if (!any) continue;
      keys.push_back(KsKey{ks.get(R, (long)n1 * j), galois(P, -(long)n1 * j)});
      kj.push_back(j);
    }
    std::vector<std::vector<std::pair<uint64_t*, uint64_t*>>> out(dig.size());
    for (size_t x = 0; x < dig.size(); ++x)
      for (int j : kj) {
        const int m = n1 * j + di[x];
        out[x].push_back(used_m[m] ? std::make_pair(A[m], B[m]) : std::make_pair((uint64_t*)nullptr, (uint64_t*)nullptr));
      }
    keyswitch(R, level, dig, keys, out, false);
  }
  // Lines 12 and 14: all plaintext products at once.
  {
    std::vector<MacTerm> terms;
    std::vector<int> ks_out;
    for (int k = 0; k < n3; ++k)
      if (k == 0 || used_k[k]) ks_out.push_back(k);
    for (int m = 0; m < inner; ++m) {
      if (!used_m[m]) continue;
      MacTerm t;
      t.a = m == 0 ? c0 : A[m];
      t.b = m == 0 ? c1 : B[m];
      t.pscaled = (m == 0);
      for (int k : ks_out) t.f.push_back(D.has(k * inner + m) ? D.pt[k * inner + m] : nullptr);
      terms.push_back(t);
    }
    std::vector<uint64_t*> oo0, oo1;
    for (int k : ks_out) {
      oo0.push_back(U0[k]);
      oo1.push_back(U1[k]);
    }
    if (terms.empty()) {
      // No diagonal at all: the result is the encryption of zero.
      MacTerm t{c0, c1, true, std::vector<const uint64_t*>(ks_out.size(), nullptr)};
      terms.push_back(t);
    }
    ptmac(R, K, 0, terms, oo0, oo1);
  }
  // Lines 13-18: outer rotations by n1 n2 k, all k at once: ModDown and
  // Decompose batched, then one gather kernel adds phi_G(u0 + x), phi_G(y)
  // of every k into (c0, c1).
  {
    IOList md, dc;
    std::vector<int> kk;
    for (int k = 1; k < n3; ++k) {
      if (!used_k[k]) continue;
      md.push_back({U1[k], tmpK[k]});
      dc.push_back({tmpK[k], Dk[k]});
      kk.push_back(k);
    }
    if (!kk.empty()) {
      divide(R, DIV_MODDOWN, level, md);
      decompose(R, level, dc);
      for (size_t k0 = 0; k0 < kk.size(); k0 += kMaxKs) {
        KsGatherArgs ga;
        memset(&ga, 0, sizeof(ga));
        ga.beta = beta;
        ga.K = K;
        ga.kmax = P->Kmax();
        ga.c0 = U0[0];
        ga.c1 = U1[0];
        for (size_t t = k0; t < std::min(kk.size(), k0 + kMaxKs); ++t) {
          const long G = (long)inner * kk[t];
          ga.digits[ga.nk] = Dk[kk[t]];
          ga.key[ga.nk] = ks.get(R, G);
          ga.add[ga.nk] = U0[kk[t]];
          ga.gal[ga.nk] = galois(P, G);
          ++ga.nk;
        }
        if (!R.dry && !R.err) R.check(launch_keyswitch_gather(P, ga, R.s));
      }
    }
  }
  // Line 19: ModDown by P q_l (ModDown and rescale combined).
  divide(R, DIV_MODDOWN_RESCALE, level, IOList{{U0[0], o0}, {U1[0], o1}});
  (void)N;
}

// ---- plain BSGS, eq. (5) -------------------------------------------------------
void lt_bsgs(Run& R, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, const Diag& D,
             const KeySet& ks, uint64_t* o0, uint64_t* o1) {
  const ckks_params* P = R.P;
  const int Lq = level + 1;
  std::vector<char> used_i(n1, 0), used_j(n2, 0);
  for (int j = 0; j < n2; ++j)
    for (int i = 0; i < n1; ++i)
      if (D.has(n1 * j + i)) used_i[i] = 1, used_j[j] = 1;
  std::vector<uint64_t*> R0(n1, nullptr), R1(n1, nullptr), S0(n2, nullptr), S1(n2, nullptr);
  R0[0] = const_cast<uint64_t*>(c0);
  R1[0] = const_cast<uint64_t*>(c1);
  for (int i = 1; i < n1; ++i)
    if (used_i[i]) {
      R0[i] = R.limbs(Lq);
      R1[i] = R.limbs(Lq);
    }
  uint64_t* A0 = R.limbs(Lq);
  uint64_t* A1 = R.limbs(Lq);
  for (int j = 1; j < n2; ++j)
    if (used_j[j]) {
      S0[j] = R.limbs(Lq);
      S1[j] = R.limbs(Lq);
    }
  // Baby steps: ct_i = Rot(ct, i), each with its own Decompose.
  {
    std::vector<RotJob> jobs;
    for (int i = 1; i < n1; ++i)
      if (used_i[i]) jobs.push_back(RotJob{c0, c1, (long)i, R0[i], R1[i], false});
    rotate(R, level, jobs, ks);
  }
  // Inner sums for every giant step at once: A = sum_i ct_i f^_i (j = 0) and
  // S_j = sum_i ct_i f^_{n1 j + i}.
  {
    std::vector<MacTerm> terms;
    std::vector<int> js;
    std::vector<uint64_t*> out0, out1;
    for (int j = 0; j < n2; ++j)
      if (j == 0 || used_j[j]) {
        js.push_back(j);
        out0.push_back(j == 0 ? A0 : S0[j]);
        out1.push_back(j == 0 ? A1 : S1[j]);
      }
    for (int i = 0; i < n1; ++i) {
      if (!used_i[i]) continue;
      MacTerm t{R0[i], R1[i], false, {}};
      for (int j : js) t.f.push_back(D.has(n1 * j + i) ? D.pt[n1 * j + i] : nullptr);
      terms.push_back(t);
    }
    if (terms.empty()) terms.push_back(MacTerm{c0, c1, false, std::vector<const uint64_t*>(js.size(), nullptr)});
    ptmac(R, Lq, P->alpha, terms, out0, out1);
  }
  // Giant steps: A += Rot(S_j, n1 j).
  {
    std::vector<RotJob> jobs;
    for (int j = 1; j < n2; ++j)
      if (used_j[j]) jobs.push_back(RotJob{S0[j], S1[j], (long)n1 * j, A0, A1, true});
    rotate(R, level, jobs, ks);
  }
  divide(R, DIV_RESCALE, level, IOList{{A0, o0}, {A1, o1}});
}

// ---- diagonal method ---------------------------------------------------------
void lt_naive(Run& R, int level, const uint64_t* c0, const uint64_t* c1, const Diag& D, const KeySet& ks,
              uint64_t* o0, uint64_t* o1) {
  const ckks_params* P = R.P;
  const int Lq = level + 1;
  uint64_t* A0 = R.limbs(Lq);
  uint64_t* A1 = R.limbs(Lq);
  std::vector<int> ds;
  for (int d = 1; d < D.n; ++d)
    if (D.has(d)) ds.push_back(d);
  std::vector<uint64_t*> T0(ds.size()), T1(ds.size());
  for (size_t t = 0; t < ds.size(); ++t) {
    T0[t] = R.limbs(Lq);
    T1[t] = R.limbs(Lq);
  }
  std::vector<RotJob> jobs;
  for (size_t t = 0; t < ds.size(); ++t) jobs.push_back(RotJob{c0, c1, (long)ds[t], T0[t], T1[t], false});
  rotate(R, level, jobs, ks);
  std::vector<MacTerm> terms;
  if (D.has(0)) terms.push_back(MacTerm{c0, c1, false, {D.pt[0]}});
  for (size_t t = 0; t < ds.size(); ++t) terms.push_back(MacTerm{T0[t], T1[t], false, {D.pt[ds[t]]}});
  if (terms.empty()) terms.push_back(MacTerm{c0, c1, false, {nullptr}});
  ptmac(R, Lq, P->alpha, terms, {A0}, {A1});
  divide(R, DIV_RESCALE, level, IOList{{A0, o0}, {A1, o1}});
}

// ---- argument checks -----------------------------------------------------------
bool overlap(const void* a, size_t an, const void* b, size_t bn) {
  const uint8_t *x = (const uint8_t*)a, *y = (const uint8_t*)b;
  return x < y + bn && y < x + an;
}

int plan_lt(Run& R, const ckks_ct* in, const ckks_lt_diags* diags, const ckks_rotkeys* keys, int algo,
            ckks_ct* out) {
  const ckks_params* P = R.P;
  if (!in || !diags || !out || !in->c0 || !in->c1 || !out->c0 || !out->c1) return CKKS_E_INVALID_ARG;
  const int level = in->level;
  if (level < 1 || level > P->L) return CKKS_E_INVALID_ARG;
  if (diags->n_diag < 0 || (diags->n_diag > 0 && !diags->pt)) return CKKS_E_INVALID_ARG;
  const size_t in_bytes = (size_t)(level + 1) * R.N * 8, out_bytes = (size_t)level * R.N * 8;
  for (const void* o : {(const void*)out->c0, (const void*)out->c1})
    for (const void* i : {(const void*)in->c0, (const void*)in->c1})
      if (overlap(o, out_bytes, i, in_bytes)) return CKKS_E_INVALID_ARG;
  if (overlap(out->c0, out_bytes, out->c1, out_bytes)) return CKKS_E_INVALID_ARG;
  KeySet ks;
  ks.S = P->n / 2;
  if (keys) {
    if (keys->count < 0 || (keys->count > 0 && (!keys->rot || !keys->key))) return CKKS_E_INVALID_ARG;
    for (int i = 0; i < keys->count; ++i) ks.m[((keys->rot[i] % ks.S) + ks.S) % ks.S] = keys->key[i];
  }
  Diag D;
  D.n = diags->n_diag;
  D.pt = diags->pt;
  R.N = (size_t)P->n;
  R.ws.limb_bytes = R.N * 8;
  if (algo == CKKS_LT_TH_BSGS) {
    const int n1 = diags->n1, n2 = diags->n2, n3 = diags->n3;
    if (n1 < 1 || n2 < 1 || n3 < 1 || (long)n1 * n2 * n3 < diags->n_diag || n1 * n2 > 4096) return CKKS_E_INVALID_ARG;
    // exact 128-bit accumulation over one MAC chunk: kMaxMacM q^2 < 2^128 (q < 2^61)
    lt_th(R, level, in->c0, in->c1, n1, n2, n3, D, ks, out->c0, out->c1);
  } else if (algo == CKKS_LT_BSGS) {
    const int n1 = diags->n1, n2 = diags->n2;
    if (n1 < 1 || n2 < 1 || (long)n1 * n2 < diags->n_diag) return CKKS_E_INVALID_ARG;
    lt_bsgs(R, level, in->c0, in->c1, n1, n2, D, ks, out->c0, out->c1);
  } else if (algo == CKKS_LT_NAIVE) {
    if (diags->n_diag > P->n / 2) return CKKS_E_INVALID_ARG;
    lt_naive(R, level, in->c0, in->c1, D, ks, out->c0, out->c1);
  } else {
    return CKKS_E_INVALID_ARG;
  }
  return R.err;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess || prev == dev || hipSetDevice(dev) != hipSuccess) prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace
}  // namespace ckks

// =============================================================================
// C interface
// =============================================================================
using namespace ckks;

extern "C" {

const char* ckks_strerror(int code) {
  switch (code) {
    case CKKS_OK: return "ok";
    case CKKS_E_INVALID_ARG: return "invalid argument";
    case CKKS_E_UNSUPPORTED: return "unsupported (missing rotation key or shape)";
    case CKKS_E_WORKSPACE: return "workspace too small";
    case CKKS_E_DEVICE: return "HIP runtime error";
    case CKKS_E_NOMEM: return "device allocation failed";
    default: return "unknown error";
  }
}

int ckks_params_create(const ckks_params_desc* desc, ckks_params** out) {
  try {
    return params_create(desc, out);
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

void ckks_params_destroy(ckks_params* params) { params_destroy(params); }

void ckks_params_info(const ckks_params* P, int* log_n, int* n_q, int* n_p) {
  if (!P) return;
  if (log_n) *log_n = P->log_n;
  if (n_q) *n_q = P->L + 1;
  if (n_p) *n_p = P->alpha;
}

int ckks_lt_workspace_size(const ckks_params* P, int level, const ckks_lt_diags* diags, int algo, size_t* bytes) {
  if (!P || !diags || !bytes) return CKKS_E_INVALID_ARG;
  try {
    Run R;
    R.P = P;
    R.dry = true;
    R.N = (size_t)P->n;
    // sizes do not depend on the buffers: plan with placeholder pointers
    static uint64_t dummy[2];
    ckks_ct in{level, 1.0, dummy, dummy + 1}, out{level - 1, 1.0, dummy, dummy + 1};
    // placeholder ciphertexts alias by construction; size the plan directly
    R.ws.limb_bytes = R.N * 8;
    KeySet ks;
    ks.S = P->n / 2;
    Diag D{diags->n_diag, diags->pt};
    if (level < 1 || level > P->L) return CKKS_E_INVALID_ARG;
    R.err = CKKS_OK;
    if (algo == CKKS_LT_TH_BSGS) {
      if (diags->n1 < 1 || diags->n2 < 1 || diags->n3 < 1) return CKKS_E_INVALID_ARG;
      lt_th(R, level, in.c0, in.c1, diags->n1, diags->n2, diags->n3, D, ks, out.c0, out.c1);
    } else if (algo == CKKS_LT_BSGS) {
      if (diags->n1 < 1 || diags->n2 < 1) return CKKS_E_INVALID_ARG;
      lt_bsgs(R, level, in.c0, in.c1, diags->n1, diags->n2, D, ks, out.c0, out.c1);
    } else if (algo == CKKS_LT_NAIVE) {
      lt_naive(R, level, in.c0, in.c1, D, ks, out.c0, out.c1);
    } else {
      return CKKS_E_INVALID_ARG;
    }
    *bytes = R.ws.peak;
    return CKKS_OK;
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_lt_eval(const ckks_params* P, const ckks_ct* in, const ckks_lt_diags* diags, const ckks_rotkeys* keys,
                 int algo, ckks_ct* out, void* ws, size_t ws_bytes, void* stream) {
  if (!P) return CKKS_E_INVALID_ARG;
  try {
    DeviceGuard dg(P->device);
    Run R;
    R.P = P;
    R.s = (hipStream_t)stream;
    R.N = (size_t)P->n;
    R.dry = true;
    int e = plan_lt(R, in, diags, keys, algo, out);
    if (e != CKKS_OK) return e;
    if (R.ws.peak > ws_bytes || (R.ws.peak > 0 && !ws)) return CKKS_E_WORKSPACE;
    Run X;
    X.P = P;
    X.s = R.s;
    X.N = R.N;
    X.dry = false;
    X.ws.base = (uint8_t*)ws;
    e = plan_lt(X, in, diags, keys, algo, out);
    if (e != CKKS_OK) return e;
    out->level = in->level - 1;
    out->scale = in->scale * diags->pt_scale / (double)P->primes[P->alpha + in->level];
    return CKKS_OK;
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_op_workspace_size(const ckks_params* P, int level, size_t* bytes) {
  if (!P || !bytes || level < 0 || level > P->L) return CKKS_E_INVALID_ARG;
  // decompose: Lq limbs; division: alpha + 1 limbs
  const size_t limb = (size_t)P->n * 8;
  *bytes = (size_t)std::max(level + 1, P->alpha + 1) * limb + 256;
  return CKKS_OK;
}

static int op_prologue(const ckks_params* P, int level, void* ws, size_t ws_bytes, Run& R, void* stream) {
  if (!P || level < 0 || level > P->L) return CKKS_E_INVALID_ARG;
  size_t need = 0;
  ckks_op_workspace_size(P, level, &need);
  if (ws_bytes < need || !ws) return CKKS_E_WORKSPACE;
  R.P = P;
  R.s = (hipStream_t)stream;
  R.N = (size_t)P->n;
  R.dry = false;
  R.ws.base = (uint8_t*)ws;
  R.ws.limb_bytes = R.N * 8;
  return CKKS_OK;
}

int ckks_op_ntt(const ckks_params* P, int forward, int first_prime, int n_limbs, const uint64_t* in, uint64_t* out,
                void* stream) {
  if (!P || !in || !out || n_limbs < 0 || first_prime < 0 || first_prime + n_limbs > P->Kmax())
    return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  Run R;
  R.P = P;
  R.s = (hipStream_t)stream;
  R.N = (size_t)P->n;
  R.dry = false;
  ntt_range(R, forward != 0, first_prime, n_limbs, in, out);
  return R.err;
}

int ckks_op_decompose(const ckks_params* P, int level, const uint64_t* x, uint64_t* digits, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!x || !digits) return CKKS_E_INVALID_ARG;
  Run R;
  int e = op_prologue(P, level, ws, ws_bytes, R, stream);
  if (e) return e;
  DeviceGuard dg(P->device);
  decompose(R, level, x, digits);
  return R.err;
}

int ckks_op_moddown(const ckks_params* P, int level, int rescale, const uint64_t* x, uint64_t* out, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!x || !out || (rescale && level < 1)) return CKKS_E_INVALID_ARG;
  Run R;
  int e = op_prologue(P, level, ws, ws_bytes, R, stream);
  if (e) return e;
  DeviceGuard dg(P->device);
  divide(R, rescale ? DIV_MODDOWN_RESCALE : DIV_MODDOWN, level, x, out);
  return R.err;
}

int ckks_op_rescale(const ckks_params* P, int level, const uint64_t* x, uint64_t* out, void* ws, size_t ws_bytes,
                    void* stream) {
  if (!x || !out || level < 1) return CKKS_E_INVALID_ARG;
  Run R;
  int e = op_prologue(P, level, ws, ws_bytes, R, stream);
  if (e) return e;
  DeviceGuard dg(P->device);
  divide(R, DIV_RESCALE, level, x, out);
  return R.err;
}

int ckks_op_keyswitch(const ckks_params* P, int level, const uint64_t* digits, const uint64_t* key, int32_t rot,
                      const uint64_t* add, uint64_t* out_a, uint64_t* out_b, void* stream) {
  if (!P || !digits || !key || !out_a || !out_b || level < 0 || level > P->L) return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  Run R;
  R.P = P;
  R.s = (hipStream_t)stream;
  R.N = (size_t)P->n;
  R.dry = false;
  keyswitch(R, level, {KsDigit{digits, add, false}}, {KsKey{key, galois(P, -(long)rot)}}, {{{out_a, out_b}}},
            false);
  return R.err;
}

int ckks_op_automorph(const ckks_params* P, int32_t rot, int n_limbs, const uint64_t* in, uint64_t* out,
                      void* stream) {
  if (!P || !in || !out || n_limbs < 0 || n_limbs > P->Kmax() || in == out) return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  Run R;
  R.P = P;
  R.s = (hipStream_t)stream;
  R.N = (size_t)P->n;
  R.dry = false;
  automorph(R, n_limbs, 0, galois(P, rot), in, nullptr, out, false);
  return R.err;
}

}  // extern "C"
