// Host orchestration of the HE-LT on one HIP stream, and the C interface.
//
// Every public call first runs its plan "dry" (no launches) to validate the
// arguments, find the rotation keys it needs and size its workspace, then runs
// it for real; both runs take the same code path, so the sizes always match.
//
// All steps take lists of independent jobs (the type-III independence of
// Section IV: rotations with different indices, and different ciphertexts,
// do not depend on each other), possibly at different levels, and pack them
// into as few launches as the kernel argument tables allow.  A single LT and a
// ragged batch of LTs run the same code.
#include <string.h>

#include <algorithm>
#include <cmath>
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
  bool live() const { return !dry && err == CKKS_OK; }
  uint64_t* limbs(size_t c) { return ws.limbs(c); }
};

// ---- launch packing -----------------------------------------------------------

LimbRange range(const uint64_t* in, uint64_t* out, int prime0, int count, const uint64_t* aux = nullptr,
                uint64_t* copy = nullptr, const uint64_t* sinv = nullptr, const uint64_t* sinv_sh = nullptr) {
  LimbRange r;
  r.in = in;
  r.out = out;
  r.aux = aux;
  r.copy = copy;
  r.sinv = sinv;
  r.sinv_sh = sinv_sh;
  r.prime0 = prime0;
  r.count = count;
  r.signed_in = 0;
  r.pad = 0;
  return r;
}

// Collects limb ranges into NTT launches (flushing when the table is full).
struct NttBatch {
  Run& R;
  bool fwd;
  int epi;
  NttArgs a;
  int total = 0;
  NttBatch(Run& r, bool f, int e = EPI_NONE) : R(r), fwd(f), epi(e) { a.nr = 0; }
  void add(const LimbRange& r) {
    if (r.count <= 0) return;
    if (a.nr == kMaxRanges) flush();
    a.r[a.nr++] = r;
    total += r.count;
  }
  void flush() {
    if (a.nr && R.live()) R.check(launch_ntt(R.P, fwd, a, total, epi, R.s));
    a.nr = 0;
    total = 0;
  }
  ~NttBatch() { flush(); }
};

// Collects basis conversions with at most ns source limbs each.
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
  void add(const BConvPlan* plan, int ns_item, int nd, const uint64_t* src, uint64_t* dst, int shift,
           const uint64_t* aux = nullptr) {
    if (items == kMaxConv) flush();
    a.plan[items] = plan;
    a.src[items] = src;
    a.dst[items] = dst;
    a.aux[items] = aux;
    a.dst_shift[items] = shift;
    a.limbs_moved += ns_item + nd + (aux ? nd : 0);
    a.max_nd = std::max(a.max_nd, nd);
    ++items;
  }
  void flush() {
    if (items && R.live()) R.check(launch_bconv(R.P, a, items, ns, R.s));
    reset();
  }
  ~BConvBatch() { flush(); }
};

// An input polynomial at some level and where its result goes.
struct Job {
  int level;
  const uint64_t* in;
  uint64_t* out;
};
typedef std::vector<Job> Jobs;

// ---- Decompose, ModDown, rescale -----------------------------------------------

// Decompose (Fig. 1) of level-l Q-basis polynomials (NTT form) into digits
// [beta_l][alpha+l+1][N].  The inverse NTT's first pass also stores each
// group's own limbs, unchanged, into its digit (ModUp keeps them, R15).
void decompose(Run& R, const Jobs& xs) {
  const ckks_params* P = R.P;
  const int a = P->alpha;
  const size_t N = R.N, mark = R.ws.mark();
  std::vector<uint64_t*> coef(xs.size());
  for (size_t t = 0; t < xs.size(); ++t) coef[t] = R.limbs(xs[t].level + 1);
  if (R.live()) {
    {
      NttBatch inv(R, false);
      for (size_t t = 0; t < xs.size(); ++t) {
        const int level = xs[t].level, K = P->K(level);
        for (int b = 0; b < P->beta(level); ++b) {
          const int lo = b * a, hi = std::min(lo + a - 1, level);
          inv.add(range(xs[t].in + (size_t)lo * N, coef[t] + (size_t)lo * N, a + lo, hi - lo + 1, nullptr,
                        xs[t].out + ((size_t)b * K + a + lo) * N));
        }
      }
    }
    {
      // every digit of every input in one set of launches: a group shorter
      // than alpha (the last one) is padded with zero sources, cheaper than
      // a launch of its own (measured: BConv 0.228 -> 0.210 ms per (4,4,4)
      // LT, where the 7-limb group had a launch of 256 workgroups)
      int gmax = 1;
      for (size_t t = 0; t < xs.size(); ++t) gmax = std::max(gmax, std::min(a, xs[t].level + 1));
      BConvBatch bc(R, gmax);
      for (size_t t = 0; t < xs.size(); ++t) {
        const int level = xs[t].level, K = P->K(level);
        for (int b = 0; b < P->beta(level); ++b) {
          const int lo = b * a, hi = std::min(lo + a - 1, level), g = hi - lo + 1;
          bc.add(P->plan(P->plan_decomp[(size_t)level * P->beta_max + b]), g, K - g, coef[t] + (size_t)lo * N,
                 xs[t].out + (size_t)b * K * N, 0);
        }
      }
    }
    NttBatch fwd(R, true);
    for (size_t t = 0; t < xs.size(); ++t) {
      const int level = xs[t].level, K = P->K(level);
      for (int b = 0; b < P->beta(level); ++b) {
        const int lo = b * a, hi = std::min(lo + a - 1, level);
        uint64_t* d = xs[t].out + (size_t)b * K * N;
        fwd.add(range(d, d, 0, a + lo));
        fwd.add(range(d + (size_t)(a + hi + 1) * N, d + (size_t)(a + hi + 1) * N, a + hi + 1, K - (a + hi + 1)));
      }
    }
  }
  R.ws.reset(mark);
}

enum DivKind { DIV_MODDOWN, DIV_MODDOWN_RESCALE, DIV_RESCALE };

// Division step of eq. (4) / eq. (1):
//  DIV_MODDOWN:         x [alpha+l+1] -> out [l+1], divide by P
//  DIV_MODDOWN_RESCALE: x [alpha+l+1] -> out [l],   divide by P q_l
//  DIV_RESCALE:         x [l+1]       -> out [l],   divide by q_l
// INTT of the dividing limbs -> BConv onto the kept limbs -> NTT whose last
// pass applies out = (kept - conv) * divisor^-1.
void divide(Run& R, DivKind kind, const Jobs& xs) {
  const ckks_params* P = R.P;
  const int a = P->alpha;
  const size_t N = R.N, mark = R.ws.mark();
  const int ns = kind == DIV_MODDOWN ? a : (kind == DIV_MODDOWN_RESCALE ? a + 1 : 1);
  std::vector<uint64_t*> coef(xs.size());
  for (size_t t = 0; t < xs.size(); ++t) coef[t] = R.limbs(ns);
  if (R.live()) {
    auto plan_of = [&](int level) {
      const int idx = kind == DIV_MODDOWN ? P->plan_moddown[level]
                                          : (kind == DIV_MODDOWN_RESCALE ? P->plan_mdrescale[level]
                                                                         : P->plan_rescale[level]);
      return P->plan(idx);
    };
    auto nout_of = [&](int level) { return kind == DIV_MODDOWN ? level + 1 : level; };
    {
      NttBatch inv(R, false);
      for (size_t t = 0; t < xs.size(); ++t) {
        const uint64_t* x = xs[t].in;
        const int level = xs[t].level;
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
      for (size_t t = 0; t < xs.size(); ++t)
        bc.add(plan_of(xs[t].level), ns, nout_of(xs[t].level), coef[t], xs[t].out, a);
    }
    NttBatch fwd(R, true, EPI_SUBMUL);
    for (size_t t = 0; t < xs.size(); ++t) {
      const int level = xs[t].level;
      const BConvPlan* plan = plan_of(level);
      const uint64_t* keep = kind == DIV_RESCALE ? xs[t].in : xs[t].in + (size_t)a * N;
      fwd.add(range(xs[t].out, xs[t].out, a, nout_of(level), keep, nullptr, plan->sinv, plan->sinv_sh));
    }
  }
  R.ws.reset(mark);
}

// ModDown (eq. (4)) and then Decompose (Fig. 1) of level-l PQ polynomials
// (Algorithm 2 lines 6-7 and 15-16) into digits [beta_l][alpha+l+1][N].
// b' = (b_Q - conv(b_P)) P^-1 is the same polynomial whichever domain the
// subtraction runs in (the NTT is linear and bijective), so it runs in the
// coefficient domain: one inverse NTT of all K limbs of b, the conversion
// P -> Q with the subtraction and scaling as its epilogue (b' in coefficient
// form), the digits' conversions from b', and one forward NTT of b' (into
// the digits' own-group limbs) and of the extensions.  The same limb
// transforms as ModDown then Decompose (ModDown's forward NTT of the
// conversion and Decompose's inverse NTT of b' become the inverse NTT of
// b_Q and the forward NTT of b'), in 6 launches instead of 10, each over
// more limbs.
void moddown_decompose(Run& R, const Jobs& xs) {
  const ckks_params* P = R.P;
  const int a = P->alpha;
  const size_t N = R.N, mark = R.ws.mark();
  std::vector<uint64_t*> coef(xs.size()), bq(xs.size());
  for (size_t t = 0; t < xs.size(); ++t) {
    coef[t] = R.limbs(P->K(xs[t].level));
    bq[t] = R.limbs(xs[t].level + 1);
  }
  if (R.live()) {
    {
      NttBatch inv(R, false);
      for (size_t t = 0; t < xs.size(); ++t) inv.add(range(xs[t].in, coef[t], 0, P->K(xs[t].level)));
    }
    {
      BConvBatch bc(R, a);
      for (size_t t = 0; t < xs.size(); ++t)
        bc.add(P->plan(P->plan_moddown[xs[t].level]), a, xs[t].level + 1, coef[t], bq[t], a, coef[t] + (size_t)a * N);
    }
    {
      int gmax = 1;
      for (size_t t = 0; t < xs.size(); ++t) gmax = std::max(gmax, std::min(a, xs[t].level + 1));
      BConvBatch bc(R, gmax);
      for (size_t t = 0; t < xs.size(); ++t) {
        const int level = xs[t].level, K = P->K(level);
        for (int b = 0; b < P->beta(level); ++b) {
          const int lo = b * a, hi = std::min(lo + a - 1, level), g = hi - lo + 1;
          bc.add(P->plan(P->plan_decomp[(size_t)level * P->beta_max + b]), g, K - g, bq[t] + (size_t)lo * N,
                 xs[t].out + (size_t)b * K * N, 0);
        }
      }
    }
    NttBatch fwd(R, true);
    for (size_t t = 0; t < xs.size(); ++t) {
      const int level = xs[t].level, K = P->K(level);
      for (int b = 0; b < P->beta(level); ++b) {
        const int lo = b * a, hi = std::min(lo + a - 1, level);
        uint64_t* d = xs[t].out + (size_t)b * K * N;
        fwd.add(range(bq[t] + (size_t)lo * N, d + (size_t)(a + lo) * N, a + lo, hi - lo + 1));
        fwd.add(range(d, d, 0, a + lo));
        fwd.add(range(d + (size_t)(a + hi + 1) * N, d + (size_t)(a + hi + 1) * N, a + hi + 1, K - (a + hi + 1)));
      }
    }
  }
  R.ws.reset(mark);
}

// ---- key switching --------------------------------------------------------------

// One hoisted key-switch product: out = phi(add + <d, key>), phi(<d, key>),
// with phi given by the Galois element of -r (gal_inv).
struct KsTask {
  const uint64_t* digits;  // [beta_l][K_l][N]
  int level;
  const uint64_t* add;     // null, [K_l][N], or Q-basis [l+1][N] multiplied by P
  bool pscaled;
  const uint64_t* key;
  uint32_t gal_inv;
  uint64_t* oa;
  uint64_t* ob;
  bool key_packed;  // the key is stored packed
};

// Packs tasks into launches of at most kMaxKs distinct keys and kMaxDig
// distinct digit sets, so each key (and each digit set) is read once per
// launch; digit sets of different levels share the key reads (limb l of a
// key is the same prime at every level).
void keyswitch(Run& R, const std::vector<KsTask>& tasks) {
  if (!R.live() || tasks.empty()) return;
  const ckks_params* P = R.P;
  // packed and unpacked keys go to separate launches
  for (int pk = 0; pk < 2; ++pk) {
    std::vector<const uint64_t*> keys;
    for (const KsTask& t : tasks)
      if ((t.key_packed ? 1 : 0) == pk && std::find(keys.begin(), keys.end(), t.key) == keys.end())
        keys.push_back(t.key);
    for (size_t k0 = 0; k0 < keys.size(); k0 += kMaxKs) {
      const size_t k1 = std::min(keys.size(), k0 + kMaxKs);
      std::vector<const uint64_t*> digs;  // digit sets used with this chunk of keys
      for (const KsTask& t : tasks) {
        const size_t ki = std::find(keys.begin(), keys.end(), t.key) - keys.begin();
        if (ki < k0 || ki >= k1) continue;
        if (std::find(digs.begin(), digs.end(), t.digits) == digs.end()) digs.push_back(t.digits);
      }
      for (size_t i0 = 0; i0 < digs.size(); i0 += kMaxDig) {
        const size_t i1 = std::min(digs.size(), i0 + kMaxDig);
        KsArgs ka;
        memset(&ka, 0, sizeof(ka));
        ka.kmax = P->Kmax();
        ka.pk_poly_bytes = P->pk_poly_bytes;
        ka.key_packed = pk;
        ka.nkeys = (int)(k1 - k0);
        ka.ndig = (int)(i1 - i0);
        for (size_t k = k0; k < k1; ++k) ka.key[k - k0] = keys[k];
        int ntask = 0, ndiag = 0;
        for (const KsTask& t : tasks) {
          const size_t ki = std::find(keys.begin(), keys.end(), t.key) - keys.begin();
          const size_t di = std::find(digs.begin(), digs.end(), t.digits) - digs.begin();
          if (ki < k0 || ki >= k1 || di < i0 || di >= i1) continue;
          const int i = (int)(di - i0), k = (int)(ki - k0);
          ka.digits[i] = t.digits;
          ka.K[i] = P->K(t.level);
          ka.beta[i] = P->beta(t.level);
          ka.add[i] = t.add;
          ka.add_pscaled[i] = t.pscaled ? 1 : 0;
          ka.gal_inv[k] = t.gal_inv;
          ka.out_a[i][k] = t.oa;
          ka.out_b[i][k] = t.ob;
          ka.kbeta = std::max(ka.kbeta, ka.beta[i]);
          ka.maxK = std::max(ka.maxK, ka.K[i]);
          ++ntask;
          ndiag += i == k;
        }
        // several keys, each with its own digit set only
        ka.diag = ka.ndig > 1 && ka.ndig == ka.nkeys && ntask == ka.nkeys && ndiag == ntask;
        R.check(launch_keyswitch(P, ka, R.s));
      }
    }
  }
}

// ---- plaintext encoding -------------------------------------------------------

// One plaintext: round(scale sigma^-1(rot(z, rot))) over n_limbs primes from
// first_prime, in NTT form at out; coef (optional) receives the integers.
struct EncItem {
  const double* z;
  long rot;
  double scale;
  int first_prime, n_limbs;
  uint64_t* out;
  int64_t* coef;
};

// FFT passes and forward NTTs (from the signed integers) of up to kMaxEnc
// items per launch.
void encode(Run& R, const std::vector<EncItem>& items) {
  const long S = R.P->n / 2;
  for (size_t i0 = 0; i0 < items.size(); i0 += kMaxEnc) {
    const size_t mark = R.ws.mark();
    const int cnt = (int)std::min<size_t>(kMaxEnc, items.size() - i0);
    EncArgs ea;
    memset(&ea, 0, sizeof(ea));
    ea.count = cnt;
    for (int c = 0; c < cnt; ++c) {
      const EncItem& it = items[i0 + c];
      ea.z[c] = it.z;
      ea.rot[c] = (int)(((it.rot % S) + S) % S);
      ea.scale[c] = it.scale;
      ea.y[c] = reinterpret_cast<double*>(R.limbs(1));  // N/2 complex values
      ea.coef[c] = it.coef ? it.coef : reinterpret_cast<int64_t*>(R.limbs(1));
    }
    if (R.live()) {
      R.check(launch_encode_fft(R.P, ea, R.s));
      // the NTT's first pass reduces the integers into each prime itself
      NttBatch fwd(R, true);
      for (int c = 0; c < cnt; ++c) {
        const EncItem& it = items[i0 + c];
        LimbRange r = range(reinterpret_cast<const uint64_t*>(ea.coef[c]), it.out, it.first_prime, it.n_limbs);
        r.signed_in = 1;
        fwd.add(r);
      }
    }
    R.ws.reset(mark);
  }
}

// ---- plaintext multiply-accumulate --------------------------------------------

struct MacTerm {
  const uint64_t* a;
  const uint64_t* b;
  bool pscaled;
  std::vector<const uint64_t*> f;  // per output k (null = absent)
  std::vector<const double*> z;    // per output k, if encoded on the fly: the slots (null = absent)
};

// How on-the-fly plaintexts are encoded: output k's with rot(z, rot[k]).
struct MacEnc {
  std::vector<long> rot;
  double scale = 0;
};

// outs[k] = sum_m terms[m] * f[k], over nlimbs limbs starting at prime_off.
// Terms with z get their plaintexts encoded right before the launch that
// reads them, into workspace that the next launch reuses.
// f_packed: the resident plaintexts are packed PQ polynomials (prime_off 0).
void ptmac(Run& R, int nlimbs, int prime_off, const std::vector<MacTerm>& terms, const std::vector<uint64_t*>& o0,
           const std::vector<uint64_t*>& o1, const MacEnc* enc = nullptr, bool f_packed = false) {
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
      ma.f_packed = f_packed ? 1 : 0;
      const size_t mark = R.ws.mark();
      std::vector<EncItem> pts;
      int nm = 0;
      for (size_t m = m0; m < std::min(terms.size(), m0 + kMaxMacM); ++m, ++nm) {
        ma.a[nm] = terms[m].a;
        ma.b[nm] = terms[m].b;
        if (terms[m].pscaled) {
          if (nm != 0) {
            R.fail(CKKS_E_INVALID_ARG);
            R.ws.reset(mark);
            return;
          }
          ma.pscaled0 = 1;
        }
        for (int k = 0; k < nk; ++k) {
          ma.f[k][nm] = terms[m].f[k0 + k];
          if (enc && !terms[m].z.empty() && terms[m].z[k0 + k]) {
            uint64_t* buf = R.limbs(nlimbs);
            pts.push_back(EncItem{terms[m].z[k0 + k], enc->rot[k0 + k], enc->scale, prime_off, nlimbs, buf, nullptr});
            ma.f[k][nm] = buf;
          }
        }
      }
      ma.nm = nm;
      for (int k = 0; k < nk; ++k) {
        ma.out0[k] = o0[k0 + k];
        ma.out1[k] = o1[k0 + k];
      }
      encode(R, pts);
      if (R.live()) R.check(launch_ptmac(R.P, ma, R.s));
      R.ws.reset(mark);
      first = false;
    }
  }
}

void automorph(Run& R, int nlimbs, int prime_off, uint32_t gal, const uint64_t* in, const uint64_t* add,
               uint64_t* out, bool accumulate) {
  if (!R.live()) return;
  AutoArgs aa{in, add, out, nlimbs, prime_off, accumulate ? 1 : 0, gal};
  R.check(launch_automorph(R.P, aa, R.s));
}

// ---- keys -----------------------------------------------------------------------

struct KeySet {
  std::map<long, const uint64_t*> m;
  long S = 0;
  bool packed = false;  // every key of the set is stored packed
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
// for several independent rotations at one level (each with its own
// Decompose, as plain BSGS and the diagonal method prescribe; only the
// launches are shared).
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
    Jobs dc, md;
    std::vector<KsTask> tasks;
    for (size_t t = 0; t < nj; ++t) {
      D[t] = R.limbs((size_t)beta * K);
      X[t] = R.limbs(K);
      Y[t] = R.limbs(K);
      Xq[t] = R.limbs(Lq);
      Yq[t] = R.limbs(Lq);
    }
    for (size_t t = 0; t < nj; ++t) {
      const RotJob& J = jobs[j0 + t];
      dc.push_back({level, J.c1, D[t]});
      md.push_back({level, X[t], Xq[t]});
      md.push_back({level, Y[t], Yq[t]});
      tasks.push_back(KsTask{D[t], level, nullptr, false, ks.get(R, J.r), 1u, X[t], Y[t], ks.packed});
    }
    decompose(R, dc);
    keyswitch(R, tasks);
    divide(R, DIV_MODDOWN, md);
    // the phi applications of the chunk, batched into launches whose entries
    // do not overlap: no entry writes what another reads or writes (jobs that
    // accumulate into one output go to consecutive launches, in order)
    AutoBatchArgs ab;
    memset(&ab, 0, sizeof(ab));
    ab.nlimbs = Lq;
    ab.prime_off = P->alpha;
    auto flush = [&]() {
      if (ab.count > 0 && R.live()) R.check(launch_automorph_batch(P, ab, R.s));
      ab.count = 0;
    };
    auto push = [&](const uint64_t* in, const uint64_t* add, uint64_t* out, bool acc, uint32_t g) {
      for (int e = 0; e < ab.count; ++e)
        if (ab.out[e] == out || ab.out[e] == in || (add && ab.out[e] == add) || ab.in[e] == out ||
            ab.add[e] == out) {
          flush();
          break;
        }
      if (ab.count == kMaxAuto) flush();
      ab.in[ab.count] = in;
      ab.add[ab.count] = add;
      ab.out[ab.count] = out;
      ab.accumulate[ab.count] = acc ? 1 : 0;
      ab.gal[ab.count] = g;
      ++ab.count;
    };
    for (size_t t = 0; t < nj; ++t) {
      const RotJob& J = jobs[j0 + t];
      const uint32_t g = galois(P, J.r);
      push(Xq[t], J.c0, J.o0, J.accumulate, g);
      push(Yq[t], nullptr, J.o1, J.accumulate, g);
    }
    flush();
    R.ws.reset(mark);
  }
}

// The diagonals: encoded plaintexts pt, or slot vectors z encoded on the fly
// with scale zscale.
struct Diag {
  int n = 0;
  const uint64_t* const* pt = nullptr;
  const double* const* z = nullptr;
  double zscale = 0;
  bool packed = false;  // pt are packed PQ polynomials
  bool has(int m) const { return m >= 0 && m < n && (z ? z[m] != nullptr : pt[m] != nullptr); }
};

// ---- triple-hoisted BSGS, Algorithm 2, for one or many ciphertexts ----------------

// Index t of the diagonals stands for the cyclic offset stride (t - centre):
// rotations s i (inner), s n1 j (middle) and G_k = s (n1 n2 k - centre)
// (outer); a block whose G_k vanishes mod N/2 is added without rotation.
struct ThItem {
  int level;
  const uint64_t* c0;
  const uint64_t* c1;
  int n1, n2, n3;
  long stride = 1, centre = 0;
  int kdir = -1;  // the block with G_k = 0, or -1
  Diag D;
  const KeySet* ks;
  uint64_t* o0;
  uint64_t* o1;
  // which parts of the algorithm carry a present diagonal
  std::vector<char> used_m, used_i, mid_i, used_k;
  bool need_d0 = false;
  // buffers
  std::vector<uint64_t*> Dg, A, B, U0, U1, Dk;
  bool fused = false;  // lines 8-14 in the fused kernel (fuse_middle)
  uint64_t* acc0 = nullptr;  // (c0, c1) of lines 12-18 at PQ
  uint64_t* acc1 = nullptr;
  long giant(const ckks_params* P, int k) const {
    const long S = P->n / 2;
    return (((stride * ((long)n1 * n2 * k - centre)) % S) + S) % S;
  }
};

// Whether lines 8-14 of an item run fused (ksmac): at most kMaxMacK
// accumulators, so the key-switch products are formed once; resident or
// encoded, plain or packed operands alike.  Also for items of a batch that
// share keys: the unfused key-switch launch reads a shared key once for up
// to kMaxDig digit sets, but the rotation products it stores and the MAC
// reads back cost more (measured: 32 same-shape LTs 738 -> 768 LT/s, the
// 128-item ragged batch 1346 -> 1430 LT/s when fused).  With more than 4
// accumulators the fused kernel runs 2-3 waves per SIMD, and every fused
// launch after the first reads and writes all its accumulators again, so
// such items run fused only when their terms fit one launch (measured at
// level 24: (4,32,8) 9.10 -> 8.20 ms and (1,64,8) 5.33 -> 5.02 ms unfused;
// (1,16,8) 2.05 against 2.08 ms and (1,16,6) 1.53 against 1.66 ms fused).
bool fuse_middle(const ckks_params* P, const ThItem& it) {
  if (P->n % kKsMacAlign) return false;
  int nk = it.kdir < 0 ? 1 : 0, nterms = 0;
  for (int k = 0; k < it.n3; ++k) nk += (k == it.kdir || it.used_k[k]) ? 1 : 0;
  for (int m = 0; m < it.n1 * it.n2; ++m) nterms += it.used_m[m] ? 1 : 0;
  return nk <= kMaxMacK && nterms > 0 && (nk <= 4 || nterms <= kMaxMacM);
}

// Lines 8-14 of one item in one kernel: every used term m = n1 j + i is
// either unrotated (j = 0: (a_i, b_i), or (P c0', P c1') for i = 0) or the
// middle rotation of d_i by s n1 j, formed in registers at each output
// position and multiplied into the outputs kk right away.  Terms go to
// launches of at most kMaxMacM terms (and so keys); the first launch writes
// the outputs, later ones add into them.  Diagonals given as slot vectors
// are encoded right before the launch that reads them (f^ = encode(rot(z,
// -G_k))), into workspace the next launch reuses.
void ksmac(Run& R, ThItem& it, const std::vector<int>& kk) {
  const ckks_params* P = R.P;
  const int inner = it.n1 * it.n2;
  struct Term {
    int m, j, i;
  };
  std::vector<Term> terms;
  for (int j = 0; j < it.n2; ++j)
    for (int i = 0; i < it.n1; ++i)
      if (it.used_m[it.n1 * j + i]) terms.push_back(Term{it.n1 * j + i, j, i});
  bool first = true;
  size_t t0 = 0;
  while (t0 < terms.size()) {
    KsMacArgs a;
    memset(&a, 0, sizeof(a));
    a.nk = (int)kk.size();
    a.K = P->K(it.level);
    a.beta = P->beta(it.level);
    a.kmax = P->Kmax();
    a.accumulate = first ? 0 : 1;
    a.key_packed = it.ks->packed ? 1 : 0;
    a.f_packed = it.D.packed && !it.D.z ? 1 : 0;  // encoded plaintexts are written unpacked
    a.pk_poly_bytes = P->pk_poly_bytes;
    int nkeys = 0, last_j = -1;
    const size_t mark = R.ws.mark();
    std::vector<EncItem> enc;
    size_t t = t0;
    for (; t < terms.size() && a.nm < kMaxMacM; ++t) {
      const Term& tm = terms[t];
      const int m = a.nm;
      if (tm.j == 0) {
        a.key_of[m] = -1;
        a.a[m] = tm.i == 0 ? it.c0 : it.A[tm.i];
        a.b[m] = tm.i == 0 ? it.c1 : it.B[tm.i];
        a.pscaled[m] = tm.i == 0 ? 1 : 0;
      } else {
        if (tm.j != last_j) {
          const long r = it.stride * it.n1 * tm.j;
          a.key[nkeys] = it.ks->get(R, r);
          a.gal[nkeys] = galois(P, r);
          ++nkeys;
          last_j = tm.j;
        }
        a.key_of[m] = nkeys - 1;
        a.digits[m] = it.Dg[tm.i];
        a.a[m] = tm.i == 0 ? it.c0 : it.A[tm.i];
        a.pscaled[m] = tm.i == 0 ? 1 : 0;
      }
      for (size_t k = 0; k < kk.size(); ++k) {
        const int idx = kk[k] * inner + tm.m;
        a.f[k][m] = nullptr;
        if (kk[k] < 0 || !it.D.has(idx)) continue;
        if (it.D.z) {
          uint64_t* buf = R.limbs(a.K);
          enc.push_back(EncItem{it.D.z[idx], -it.giant(P, kk[k]), it.D.zscale, 0, a.K, buf, nullptr});
          a.f[k][m] = buf;
        } else {
          a.f[k][m] = it.D.pt[idx];
        }
      }
      ++a.nm;
    }
    for (size_t k = 0; k < kk.size(); ++k) {
      a.out0[k] = kk[k] >= 0 ? it.U0[kk[k]] : it.acc0;
      a.out1[k] = kk[k] >= 0 ? it.U1[kk[k]] : it.acc1;
    }
    encode(R, enc);
    if (R.live()) R.check(launch_ksmac(P, a, R.s));
    R.ws.reset(mark);
    first = false;
    t0 = t;
  }
}

void lt_th(Run& R, std::vector<ThItem>& items) {
  const ckks_params* P = R.P;
  // Plan every item and take its buffers.
  for (ThItem& it : items) {
    const int K = P->K(it.level), beta = P->beta(it.level), inner = it.n1 * it.n2;
    it.used_m.assign(inner, 0);
    it.used_i.assign(it.n1, 0);
    it.mid_i.assign(it.n1, 0);
    it.used_k.assign(it.n3, 0);
    for (int k = 0; k < it.n3; ++k)
      for (int m = 0; m < inner; ++m)
        if (it.D.has(k * inner + m)) it.used_m[m] = 1, it.used_k[k] = 1;
    for (int m = 0; m < inner; ++m)
      if (it.used_m[m]) {
        it.used_i[m % it.n1] = 1;
        if (m >= it.n1) it.mid_i[m % it.n1] = 1;
      }
    it.need_d0 = it.mid_i[0];
    for (int i = 1; i < it.n1; ++i) it.need_d0 = it.need_d0 || it.used_i[i];
    it.kdir = -1;
    for (int k = 0; k < it.n3 && it.kdir < 0; ++k)
      if (it.giant(P, k) == 0) it.kdir = k;
    it.Dg.assign(it.n1, nullptr);
    it.A.assign(inner, nullptr);
    it.B.assign(inner, nullptr);
    it.fused = fuse_middle(P, it);
    for (int i = 0; i < it.n1; ++i)
      if ((i == 0 && it.need_d0) || (i > 0 && it.mid_i[i])) it.Dg[i] = R.limbs((size_t)beta * K);
    // the inner layer's products (m < n1); the middle layer's only when they
    // are materialised (not fused)
    for (int m = 1; m < inner; ++m)
      if ((m < it.n1 && (it.used_m[m] || it.used_i[m])) || (m >= it.n1 && it.used_m[m] && !it.fused)) {
        it.A[m] = R.limbs(K);
        it.B[m] = R.limbs(K);
      }
    it.U0.assign(it.n3, nullptr);
    it.U1.assign(it.n3, nullptr);
    it.Dk.assign(it.n3, nullptr);
    for (int k = 0; k < it.n3; ++k) {
      if (k != it.kdir && !it.used_k[k]) continue;
      it.U0[k] = R.limbs(K);
      it.U1[k] = R.limbs(K);
      if (k != it.kdir) it.Dk[k] = R.limbs((size_t)beta * K);
    }
    if (it.kdir >= 0) {
      it.acc0 = it.U0[it.kdir];
      it.acc1 = it.U1[it.kdir];
    } else {
      it.acc0 = R.limbs(K);
      it.acc1 = R.limbs(K);
    }
  }
  // Line 1: d_0 = Decompose(c1').
  {
    Jobs dc;
    for (ThItem& it : items)
      if (it.need_d0) dc.push_back({it.level, it.c1, it.Dg[0]});
    decompose(R, dc);
  }
  // Lines 2-5: inner rotations share d_0; a_0 = P c0' is applied inside the kernel.
  {
    std::vector<KsTask> tasks;
    for (ThItem& it : items)
      for (int i = 1; i < it.n1; ++i)
        if (it.used_i[i])
          tasks.push_back(KsTask{it.Dg[0], it.level, it.c0, true, it.ks->get(R, it.stride * i),
                                 galois(P, -it.stride * i), it.A[i], it.B[i], it.ks->packed});
    keyswitch(R, tasks);
  }
  // Lines 6-7: d_i = Decompose(ModDown(b_i)), every i at once.
  {
    Jobs mdc;
    for (ThItem& it : items)
      for (int i = 1; i < it.n1; ++i)
        if (it.mid_i[i]) mdc.push_back({it.level, it.B[i], it.Dg[i]});
    moddown_decompose(R, mdc);
  }
  // Lines 8-14 fused where fuse_middle allows (ksmac above); for the
  // other items the middle key switch runs first.
  // Lines 8-11: middle rotations by s n1 j share d_i; each middle key is read
  // once per launch for all digit sets.
  {
    std::vector<KsTask> tasks;
    for (size_t t = 0; t < items.size(); ++t) {
      ThItem& it = items[t];
      if (it.fused) continue;
      for (int j = 1; j < it.n2; ++j)
        for (int i = 0; i < it.n1; ++i) {
          const int m = it.n1 * j + i;
          if (!it.mid_i[i] || !it.used_m[m]) continue;
          const long r = it.stride * it.n1 * j;
          tasks.push_back(KsTask{it.Dg[i], it.level, i == 0 ? it.c0 : it.A[i], i == 0, it.ks->get(R, r),
                                 galois(P, -r), it.A[m], it.B[m], it.ks->packed});
        }
    }
    keyswitch(R, tasks);
  }
  // Lines 12 and 14: all plaintext products of an item at once (with no
  // unrotated block, the accumulator is one more output with no plaintext,
  // i.e. zero).
  for (size_t t = 0; t < items.size(); ++t) {
    ThItem& it = items[t];
    const int K = P->K(it.level), inner = it.n1 * it.n2;
    std::vector<int> kk;
    for (int k = 0; k < it.n3; ++k)
      if (k == it.kdir || it.used_k[k]) kk.push_back(k);
    if (it.kdir < 0) kk.push_back(-1);
    if (it.fused) {
      ksmac(R, it, kk);
      continue;
    }
    std::vector<MacTerm> terms;
    for (int m = 0; m < inner; ++m) {
      if (!it.used_m[m]) continue;
      MacTerm t{m == 0 ? it.c0 : it.A[m], m == 0 ? it.c1 : it.B[m], m == 0, {}, {}};
      for (int k : kk) {
        const bool h = k >= 0 && it.D.has(k * inner + m);
        if (it.D.z)
          t.z.push_back(h ? it.D.z[k * inner + m] : nullptr);
        t.f.push_back(h && !it.D.z ? it.D.pt[k * inner + m] : nullptr);
      }
      terms.push_back(t);
    }
    // No diagonal at all: the result is an encryption of zero.
    if (terms.empty())
      terms.push_back(MacTerm{it.c0, it.c1, true, std::vector<const uint64_t*>(kk.size(), nullptr), {}});
    std::vector<uint64_t*> o0, o1;
    MacEnc enc;
    enc.scale = it.D.zscale;
    for (int k : kk) {
      o0.push_back(k >= 0 ? it.U0[k] : it.acc0);
      o1.push_back(k >= 0 ? it.U1[k] : it.acc1);
      enc.rot.push_back(k >= 0 ? -it.giant(P, k) : 0);  // f^ = encode(rot(diag, -G_k))
    }
    ptmac(R, K, 0, terms, o0, o1, it.D.z ? &enc : nullptr, it.D.packed);
  }
  // Lines 13-18: outer rotations by G_k: ModDown and Decompose of every
  // (item, k) at once, then per item one gather kernel adds
  // phi_G(u0 + x), phi_G(y) of all its k into (c0, c1).
  {
    Jobs mdc;
    for (ThItem& it : items)
      for (int k = 0; k < it.n3; ++k)
        if (k != it.kdir && it.used_k[k]) mdc.push_back({it.level, it.U1[k], it.Dk[k]});
    moddown_decompose(R, mdc);
    for (ThItem& it : items) {
      std::vector<int> kk;
      for (int k = 0; k < it.n3; ++k)
        if (k != it.kdir && it.used_k[k]) kk.push_back(k);
      for (size_t k0 = 0; k0 < kk.size(); k0 += kMaxKs) {
        KsGatherArgs ga;
        memset(&ga, 0, sizeof(ga));
        ga.beta = P->beta(it.level);
        ga.K = P->K(it.level);
        ga.kmax = P->Kmax();
        ga.pk_poly_bytes = P->pk_poly_bytes;
        ga.key_packed = it.ks->packed ? 1 : 0;
        ga.c0 = it.acc0;
        ga.c1 = it.acc1;
        for (size_t t = k0; t < std::min(kk.size(), k0 + kMaxKs); ++t) {
          const long G = it.giant(P, kk[t]);
          ga.digits[ga.nk] = it.Dk[kk[t]];
          ga.key[ga.nk] = it.ks->get(R, G);
          ga.add[ga.nk] = it.U0[kk[t]];
          ga.gal[ga.nk] = galois(P, G);
          ++ga.nk;
        }
        if (R.live()) R.check(launch_keyswitch_gather(P, ga, R.s));
      }
    }
  }
  // Line 19: ModDown by P q_l (ModDown and rescale combined).
  {
    Jobs md;
    for (ThItem& it : items) {
      md.push_back({it.level, it.acc0, it.o0});
      md.push_back({it.level, it.acc1, it.o1});
    }
    divide(R, DIV_MODDOWN_RESCALE, md);
  }
}

// ---- plain BSGS, eq. (5) -------------------------------------------------------
// Baby rotations s i, giant rotations G_j = s (n1 j - centre); the block whose
// G_j vanishes mod N/2 is added without rotation.
void lt_bsgs(Run& R, int level, const uint64_t* c0, const uint64_t* c1, int n1, int n2, long stride, long centre,
             const Diag& D, const KeySet& ks, uint64_t* o0, uint64_t* o1) {
  const ckks_params* P = R.P;
  const int Lq = level + 1;
  const long S = P->n / 2;
  auto giant = [&](int j) { return (((stride * ((long)n1 * j - centre)) % S) + S) % S; };
  int jdir = -1;
  for (int j = 0; j < n2 && jdir < 0; ++j)
    if (giant(j) == 0) jdir = j;
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
  for (int j = 0; j < n2; ++j)
    if (used_j[j] && j != jdir) {
      S0[j] = R.limbs(Lq);
      S1[j] = R.limbs(Lq);
    }
  // Baby steps: ct_i = Rot(ct, s i), each with its own Decompose.
  {
    std::vector<RotJob> jobs;
    for (int i = 1; i < n1; ++i)
      if (used_i[i]) jobs.push_back(RotJob{c0, c1, stride * i, R0[i], R1[i], false});
    rotate(R, level, jobs, ks);
  }
  // Inner sums for every giant step at once: A = sum_i ct_i f^_{n1 jdir + i}
  // (zero if no block is unrotated) and S_j = sum_i ct_i f^_{n1 j + i}.
  {
    std::vector<MacTerm> terms;
    std::vector<int> js{jdir};
    std::vector<uint64_t*> out0{A0}, out1{A1};
    for (int j = 0; j < n2; ++j)
      if (used_j[j] && j != jdir) {
        js.push_back(j);
        out0.push_back(S0[j]);
        out1.push_back(S1[j]);
      }
    for (int i = 0; i < n1; ++i) {
      if (!used_i[i]) continue;
      MacTerm t{R0[i], R1[i], false, {}, {}};
      for (int j : js) {
        const bool h = j >= 0 && D.has(n1 * j + i);
        if (D.z) t.z.push_back(h ? D.z[n1 * j + i] : nullptr);
        t.f.push_back(h && !D.z ? D.pt[n1 * j + i] : nullptr);
      }
      terms.push_back(t);
    }
    if (terms.empty())
      terms.push_back(MacTerm{c0, c1, false, std::vector<const uint64_t*>(js.size(), nullptr), {}});
    MacEnc enc;  // on-the-fly plaintexts: f^ = encode(rot(diag, -G_j)) at the Q basis
    enc.scale = D.zscale;
    for (int j : js) enc.rot.push_back(j >= 0 ? -giant(j) : 0);
    ptmac(R, Lq, P->alpha, terms, out0, out1, D.z ? &enc : nullptr);
  }
  // Giant steps: A += Rot(S_j, G_j).
  {
    std::vector<RotJob> jobs;
    for (int j = 0; j < n2; ++j)
      if (used_j[j] && j != jdir) jobs.push_back(RotJob{S0[j], S1[j], giant(j), A0, A1, true});
    rotate(R, level, jobs, ks);
  }
  divide(R, DIV_RESCALE, Jobs{{level, A0, o0}, {level, A1, o1}});
}

// ---- diagonal method ---------------------------------------------------------
// out = rescale(sum_t Rot(ct, s (t - centre)) f_t).
void lt_naive(Run& R, int level, const uint64_t* c0, const uint64_t* c1, long stride, long centre, const Diag& D,
              const KeySet& ks, uint64_t* o0, uint64_t* o1) {
  const ckks_params* P = R.P;
  const int Lq = level + 1;
  const long S = P->n / 2;
  uint64_t* A0 = R.limbs(Lq);
  uint64_t* A1 = R.limbs(Lq);
  std::vector<int> ts;
  int tdir = -1;
  for (int t = 0; t < D.n; ++t) {
    if (!D.has(t)) continue;
    if ((((stride * (t - centre)) % S) + S) % S == 0)
      tdir = t;
    else
      ts.push_back(t);
  }
  std::vector<uint64_t*> T0(ts.size()), T1(ts.size());
  for (size_t u = 0; u < ts.size(); ++u) {
    T0[u] = R.limbs(Lq);
    T1[u] = R.limbs(Lq);
  }
  std::vector<RotJob> jobs;
  for (size_t u = 0; u < ts.size(); ++u)
    jobs.push_back(RotJob{c0, c1, stride * (ts[u] - centre), T0[u], T1[u], false});
  rotate(R, level, jobs, ks);
  // on-the-fly plaintexts: f_t = encode(diag_t) at the Q basis (no pre-rotation)
  auto term = [&](const uint64_t* a, const uint64_t* b, int t) {
    return D.z ? MacTerm{a, b, false, {nullptr}, {D.z[t]}} : MacTerm{a, b, false, {D.pt[t]}, {}};
  };
  std::vector<MacTerm> terms;
  if (tdir >= 0) terms.push_back(term(c0, c1, tdir));
  for (size_t u = 0; u < ts.size(); ++u) terms.push_back(term(T0[u], T1[u], ts[u]));
  if (terms.empty()) terms.push_back(MacTerm{c0, c1, false, {nullptr}, {}});
  MacEnc enc;
  enc.scale = D.zscale;
  enc.rot.push_back(0);
  ptmac(R, Lq, P->alpha, terms, {A0}, {A1}, D.z ? &enc : nullptr);
  divide(R, DIV_RESCALE, Jobs{{level, A0, o0}, {level, A1, o1}});
}

// ---- argument checks -------------------------------------------------------------
bool overlap(const void* a, size_t an, const void* b, size_t bn) {
  const uint8_t *x = (const uint8_t*)a, *y = (const uint8_t*)b;
  return x < y + bn && y < x + an;
}

// A zero stride (a zero-initialised struct) reads as 1.
long prog_stride(const ckks_lt_diags* d) { return d->stride == 0 ? 1 : d->stride; }

// Validates one LT's arguments (no device access); fills ks from keys.
int check_item(const ckks_params* P, const ckks_ct* in, const ckks_lt_diags* diags, const ckks_rotkeys* keys,
               int algo, const ckks_ct* out, bool check_buffers, KeySet* ks) {
  if (!in || !diags || !out) return CKKS_E_INVALID_ARG;
  const int level = in->level;
  if (level < 1 || level > P->L) return CKKS_E_INVALID_ARG;
  if (diags->n_diag < 0 || (diags->n_diag > 0 && !diags->pt && !diags->slots) || (diags->pt && diags->slots))
    return CKKS_E_INVALID_ARG;
  if (diags->slots && (!(diags->pt_scale > 0) || !std::isfinite(diags->pt_scale))) return CKKS_E_INVALID_ARG;
  if (diags->pt_packed) {
    if (diags->slots) return CKKS_E_INVALID_ARG;
    if (algo != CKKS_LT_TH_BSGS && algo != CKKS_LT_DH_BSGS) return CKKS_E_UNSUPPORTED;  // PQ-basis plaintexts only
  }
  if (check_buffers) {
    if (!in->c0 || !in->c1 || !out->c0 || !out->c1) return CKKS_E_INVALID_ARG;
    const size_t N = (size_t)P->n;
    const size_t in_bytes = (size_t)(level + 1) * N * 8, out_bytes = (size_t)level * N * 8;
    for (const void* o : {(const void*)out->c0, (const void*)out->c1})
      for (const void* i : {(const void*)in->c0, (const void*)in->c1})
        if (overlap(o, out_bytes, i, in_bytes)) return CKKS_E_INVALID_ARG;
    if (overlap(out->c0, out_bytes, out->c1, out_bytes)) return CKKS_E_INVALID_ARG;
  }
  ks->S = P->n / 2;
  ks->packed = keys && keys->packed;
  if (keys) {
    if (keys->count < 0 || (keys->count > 0 && (!keys->rot || !keys->key))) return CKKS_E_INVALID_ARG;
    for (int i = 0; i < keys->count; ++i) ks->m[((keys->rot[i] % ks->S) + ks->S) % ks->S] = keys->key[i];
  }
  // The progression stride (t - centre) must not repeat an offset mod N/2:
  // at most N/2 / gcd(stride, N/2) indices.
  const long S = P->n / 2;
  const long st = ((prog_stride(diags) % S) + S) % S;
  long g = S, x = st;
  while (x) {
    const long t = g % x;
    g = x;
    x = t;
  }
  const long period = S / g;
  long n_idx = diags->n_diag;
  if (algo == CKKS_LT_TH_BSGS) n_idx = std::max<long>(n_idx, (long)diags->n1 * diags->n2 * diags->n3);
  if (algo == CKKS_LT_BSGS || algo == CKKS_LT_DH_BSGS) n_idx = std::max<long>(n_idx, (long)diags->n1 * diags->n2);
  if (n_idx > period) return CKKS_E_INVALID_ARG;
  if (algo == CKKS_LT_TH_BSGS) {
    const int n1 = diags->n1, n2 = diags->n2, n3 = diags->n3;
    if (n1 < 1 || n2 < 1 || n3 < 1 || (long)n1 * n2 * n3 < diags->n_diag || (long)n1 * n2 * n3 > P->n / 2)
      return CKKS_E_INVALID_ARG;
  } else if (algo == CKKS_LT_BSGS || algo == CKKS_LT_DH_BSGS) {
    const int n1 = diags->n1, n2 = diags->n2;
    if (n1 < 1 || n2 < 1 || (long)n1 * n2 < diags->n_diag || (long)n1 * n2 > P->n / 2) return CKKS_E_INVALID_ARG;
  } else if (algo == CKKS_LT_NAIVE) {
    if (diags->n_diag > P->n / 2) return CKKS_E_INVALID_ARG;
  } else {
    return CKKS_E_INVALID_ARG;
  }
  return CKKS_OK;
}

// DH-BSGS (Algorithm 1) with n1 baby and n2 giant steps is Algorithm 2 with
// an empty inner layer: (n1', n2', n3') = (1, n1, n2).
ThItem th_item(const ckks_ct* in, const ckks_lt_diags* d, const KeySet* ks, ckks_ct* out, bool dh) {
  ThItem it;
  it.level = in->level;
  it.c0 = in->c0;
  it.c1 = in->c1;
  it.n1 = dh ? 1 : d->n1;
  it.n2 = dh ? d->n1 : d->n2;
  it.n3 = dh ? d->n2 : d->n3;
  // With one middle step, (n1, 1, n3) has the terms, rotations and outputs
  // of (1, n1, n3) (index n1 k + i, rotation s i, G_k = s (n1 k - centre),
  // the same products bit for bit); run it that way, so its rotations go
  // through the fused middle layer instead of materialising products.
  if (it.n2 == 1 && it.n1 > 1) {
    it.n2 = it.n1;
    it.n1 = 1;
  }
  it.stride = prog_stride(d);
  it.centre = d->centre;
  it.D.n = d->n_diag;
  it.D.pt = d->pt;
  it.D.z = d->slots;
  it.D.zscale = d->pt_scale;
  it.D.packed = d->pt_packed != 0;
  it.ks = ks;
  it.o0 = out->c0;
  it.o1 = out->c1;
  return it;
}

// Runs (or, dry, plans) LTs of one algorithm.  TH-BSGS items run in lockstep;
// the other algorithms run one item after the other.
void run_items(Run& R, int algo, const std::vector<const ckks_ct*>& in, const std::vector<const ckks_lt_diags*>& dg,
               const std::vector<KeySet>& ks, const std::vector<ckks_ct*>& out) {
  if (algo == CKKS_LT_TH_BSGS || algo == CKKS_LT_DH_BSGS) {
    std::vector<ThItem> items;
    for (size_t t = 0; t < in.size(); ++t)
      items.push_back(th_item(in[t], dg[t], &ks[t], out[t], algo == CKKS_LT_DH_BSGS));
    lt_th(R, items);
    return;
  }
  for (size_t t = 0; t < in.size(); ++t) {
    Diag D;
    D.n = dg[t]->n_diag;
    D.pt = dg[t]->pt;
    D.z = dg[t]->slots;
    D.zscale = dg[t]->pt_scale;
    const long stride = prog_stride(dg[t]), centre = dg[t]->centre;
    if (algo == CKKS_LT_BSGS)
      lt_bsgs(R, in[t]->level, in[t]->c0, in[t]->c1, dg[t]->n1, dg[t]->n2, stride, centre, D, ks[t], out[t]->c0,
              out[t]->c1);
    else
      lt_naive(R, in[t]->level, in[t]->c0, in[t]->c1, stride, centre, D, ks[t], out[t]->c0, out[t]->c1);
  }
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

Run make_run(const ckks_params* P, void* stream, bool dry, void* ws) {
  Run R;
  R.P = P;
  R.s = (hipStream_t)stream;
  R.N = (size_t)P->n;
  R.dry = dry;
  R.ws.base = (uint8_t*)ws;
  R.ws.limb_bytes = R.N * 8;
  return R;
}

// Plans (dry) then runs a list of items; *need receives the workspace bytes.
int eval_items(const ckks_params* P, int algo, const std::vector<const ckks_ct*>& in,
               const std::vector<const ckks_lt_diags*>& dg, const std::vector<KeySet>& ks,
               const std::vector<ckks_ct*>& out, void* ws, size_t ws_bytes, void* stream, bool plan_only,
               size_t* need) {
  Run D = make_run(P, stream, true, nullptr);
  run_items(D, algo, in, dg, ks, out);
  if (need) *need = D.ws.peak;
  if (plan_only) return CKKS_OK;
  if (D.err != CKKS_OK) return D.err;
  if (D.ws.peak > ws_bytes || (D.ws.peak > 0 && !ws)) return CKKS_E_WORKSPACE;
  Run X = make_run(P, stream, false, ws);
  run_items(X, algo, in, dg, ks, out);
  return X.err;
}

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
    case CKKS_E_TIMEOUT: return "request timed out in the queue";
    case CKKS_E_CANCELLED: return "request cancelled";
    case CKKS_PENDING: return "pending";
    case CKKS_RUNNING: return "running";
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
    // Sizes depend only on shapes: plan with placeholder buffers and no keys.
    static uint64_t dummy[4];
    ckks_ct in{level, 1.0, dummy, dummy + 1}, out{level - 1, 1.0, dummy + 2, dummy + 3};
    std::vector<KeySet> ks(1);
    int e = check_item(P, &in, diags, nullptr, algo, &out, false, &ks[0]);
    if (e != CKKS_OK) return e;
    return eval_items(P, algo, {&in}, {diags}, ks, {&out}, nullptr, 0, nullptr, true, bytes);
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_lt_eval(const ckks_params* P, const ckks_ct* in, const ckks_lt_diags* diags, const ckks_rotkeys* keys,
                 int algo, ckks_ct* out, void* ws, size_t ws_bytes, void* stream) {
  if (!P) return CKKS_E_INVALID_ARG;
  try {
    DeviceGuard dg(P->device);
    std::vector<KeySet> ks(1);
    int e = check_item(P, in, diags, keys, algo, out, true, &ks[0]);
    if (e != CKKS_OK) return e;
    e = eval_items(P, algo, {in}, {diags}, ks, {out}, ws, ws_bytes, stream, false, nullptr);
    if (e != CKKS_OK) return e;
    out->level = in->level - 1;
    out->scale = in->scale * diags->pt_scale / (double)P->primes[P->alpha + in->level];
    return CKKS_OK;
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_lt_eval_noalloc(const ckks_params* P, const ckks_ct* in, const ckks_lt_diags* diags,
                         const ckks_rotkeys* keys, int algo, ckks_ct* out, void* stream) {
  if (!P) return CKKS_E_INVALID_ARG;
  void* ws = nullptr;
  {
    DeviceGuard dg(P->device);
    const int e = scratch_address(P->device, &ws);
    if (e != CKKS_OK) return e;
  }
  // ckks_lt_eval plans first and refuses a workspace beyond the scratch
  // before it enqueues anything.
  return ckks_lt_eval(P, in, diags, keys, algo, out, ws, CKKS_LT_NOALLOC_MAX_WS, stream);
}

static int encode_common(const ckks_params* P, int count, const ckks_encode_item* items, double scale,
                         int first_prime, int n_limbs, void* ws, size_t ws_bytes, void* stream, bool plan_only,
                         size_t* need) {
  if (!P || count < 0 || (count > 0 && !items) || !(scale > 0) || !std::isfinite(scale) || first_prime < 0 ||
      n_limbs < 1 || first_prime + n_limbs > P->Kmax())
    return CKKS_E_INVALID_ARG;
  std::vector<EncItem> its;
  for (int i = 0; i < count; ++i) {
    if (!plan_only && (!items[i].slots || !items[i].out)) return CKKS_E_INVALID_ARG;
    its.push_back(EncItem{items[i].slots, (long)items[i].rot, scale, first_prime, n_limbs, items[i].out,
                          plan_only ? nullptr : items[i].coef});
  }
  Run D = make_run(P, stream, true, nullptr);
  encode(D, its);
  if (need) *need = D.ws.peak;
  if (plan_only) return CKKS_OK;
  if (D.ws.peak > ws_bytes || (D.ws.peak > 0 && !ws)) return CKKS_E_WORKSPACE;
  Run X = make_run(P, stream, false, ws);
  encode(X, its);
  return X.err;
}

int ckks_encode_workspace_size(const ckks_params* P, int count, size_t* bytes) {
  if (!bytes) return CKKS_E_INVALID_ARG;
  try {
    std::vector<ckks_encode_item> items((size_t)std::max(count, 0));
    return encode_common(P, count, items.data(), 1.0, 0, 1, nullptr, 0, nullptr, true, bytes);
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_encode(const ckks_params* P, int count, const ckks_encode_item* items, double scale, int first_prime,
                int n_limbs, void* ws, size_t ws_bytes, void* stream) {
  if (!P) return CKKS_E_INVALID_ARG;
  try {
    DeviceGuard dg(P->device);
    return encode_common(P, count, items, scale, first_prime, n_limbs, ws, ws_bytes, stream, false, nullptr);
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_packed_poly_bytes(const ckks_params* P, size_t* bytes) {
  if (!P || !bytes) return CKKS_E_INVALID_ARG;
  *bytes = (size_t)P->pk_poly_bytes;
  return CKKS_OK;
}

int ckks_pack(const ckks_params* P, int count, const uint64_t* in, void* out, void* stream) {
  if (!P || count < 0 || count > 65535 || (count > 0 && (!in || !out))) return CKKS_E_INVALID_ARG;
  if (count == 0) return CKKS_OK;
  const size_t in_bytes = (size_t)count * P->Kmax() * P->n * 8, out_bytes = (size_t)count * P->pk_poly_bytes;
  if (overlap(in, in_bytes, out, out_bytes)) return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  return launch_pack(P, count, in, static_cast<uint8_t*>(out), (hipStream_t)stream) == hipSuccess ? CKKS_OK
                                                                                                   : CKKS_E_DEVICE;
}

static int batch_common(const ckks_params* P, int count, ckks_lt_item* items, int algo, void* ws, size_t ws_bytes,
                        void* stream, bool plan_only, size_t* need) {
  if (!P || count < 0 || (count > 0 && !items)) return CKKS_E_INVALID_ARG;
  std::vector<const ckks_ct*> in;
  std::vector<const ckks_lt_diags*> dg;
  std::vector<ckks_ct*> out;
  std::vector<KeySet> ks;
  std::vector<int> idx;
  ks.reserve(count);
  int first_err = CKKS_OK;
  for (int t = 0; t < count; ++t) {
    KeySet k;
    const int e =
        check_item(P, &items[t].in, &items[t].diags, items[t].keys, algo, &items[t].out, !plan_only, &k);
    items[t].status = e;
    if (e != CKKS_OK) {
      if (first_err == CKKS_OK) first_err = e;
      continue;
    }
    if (!plan_only) {
      // The item planned alone (no launches) finds what only its own keys
      // can tell, e.g. a rotation its split, stride or centre needs and its
      // key set lacks: that item fails, the others still run.
      Run D = make_run(P, stream, true, nullptr);
      run_items(D, algo, {&items[t].in}, {&items[t].diags}, {k}, {&items[t].out});
      if (D.err != CKKS_OK) {
        items[t].status = D.err;
        if (first_err == CKKS_OK) first_err = D.err;
        continue;
      }
    }
    ks.push_back(k);
    in.push_back(&items[t].in);
    dg.push_back(&items[t].diags);
    out.push_back(&items[t].out);
    idx.push_back(t);
  }
  // an output must not overlap any input or another item's output
  if (!plan_only) {
    const size_t N = (size_t)P->n;
    for (size_t a = 0; a < out.size(); ++a) {
      const size_t ob = (size_t)in[a]->level * N * 8;
      for (size_t b = 0; b < in.size(); ++b) {
        const size_t ib = (size_t)(in[b]->level + 1) * N * 8, obb = (size_t)in[b]->level * N * 8;
        for (const void* o : {(const void*)out[a]->c0, (const void*)out[a]->c1}) {
          if (overlap(o, ob, in[b]->c0, ib) || overlap(o, ob, in[b]->c1, ib) ||
              (a != b && (overlap(o, ob, out[b]->c0, obb) || overlap(o, ob, out[b]->c1, obb)))) {
            for (int i : idx) items[i].status = CKKS_E_INVALID_ARG;  // nothing runs
            return CKKS_E_INVALID_ARG;
          }
        }
      }
    }
  }
  if (in.empty()) {
    if (need) *need = 0;
    return first_err;
  }
  const int e = eval_items(P, algo, in, dg, ks, out, ws, ws_bytes, stream, plan_only, need);
  if (plan_only) return e;
  for (size_t t = 0; t < idx.size(); ++t) {
    ckks_lt_item& it = items[idx[t]];
    it.status = e;
    if (e == CKKS_OK) {
      it.out.level = it.in.level - 1;
      it.out.scale = it.in.scale * it.diags.pt_scale / (double)P->primes[P->alpha + it.in.level];
    }
  }
  return e != CKKS_OK ? e : first_err;
}

int ckks_lt_batch_workspace_size(const ckks_params* P, int count, const ckks_lt_item* items, int algo,
                                 size_t* bytes) {
  if (!bytes || count < 0 || (count > 0 && !items)) return CKKS_E_INVALID_ARG;
  try {
    std::vector<ckks_lt_item> copy(items, items + count);
    static uint64_t dummy[4];
    for (auto& it : copy) {
      it.in.c0 = it.in.c1 = dummy;
      it.out.c0 = it.out.c1 = dummy + 2;
      it.keys = nullptr;
    }
    return batch_common(P, count, copy.data(), algo, nullptr, 0, nullptr, true, bytes);
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_lt_eval_batch(const ckks_params* P, int count, ckks_lt_item* items, int algo, void* ws, size_t ws_bytes,
                       void* stream) {
  if (!P) return CKKS_E_INVALID_ARG;
  try {
    DeviceGuard dg(P->device);
    return batch_common(P, count, items, algo, ws, ws_bytes, stream, false, nullptr);
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_op_workspace_size(const ckks_params* P, int level, size_t* bytes) {
  if (!P || !bytes || level < 0 || level > P->L) return CKKS_E_INVALID_ARG;
  // decompose: l+1 limbs; division: alpha + 1 limbs
  const size_t limb = (size_t)P->n * 8;
  *bytes = (size_t)std::max(level + 1, P->alpha + 1) * limb + 256;
  return CKKS_OK;
}

static int op_prologue(const ckks_params* P, int level, void* ws, size_t ws_bytes, Run& R, void* stream) {
  if (!P || level < 0 || level > P->L) return CKKS_E_INVALID_ARG;
  size_t need = 0;
  ckks_op_workspace_size(P, level, &need);
  if (ws_bytes < need || !ws) return CKKS_E_WORKSPACE;
  R = make_run(P, stream, false, ws);
  return CKKS_OK;
}

int ckks_op_ntt(const ckks_params* P, int forward, int first_prime, int n_limbs, const uint64_t* in, uint64_t* out,
                void* stream) {
  if (!P || !in || !out || n_limbs < 0 || first_prime < 0 || first_prime + n_limbs > P->Kmax())
    return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  Run R = make_run(P, stream, false, nullptr);
  {
    NttBatch b(R, forward != 0);
    b.add(range(in, out, first_prime, n_limbs));
  }
  return R.err;
}

int ckks_op_decompose(const ckks_params* P, int level, const uint64_t* x, uint64_t* digits, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!x || !digits) return CKKS_E_INVALID_ARG;
  Run R;
  int e = op_prologue(P, level, ws, ws_bytes, R, stream);
  if (e) return e;
  DeviceGuard dg(P->device);
  decompose(R, Jobs{{level, x, digits}});
  return R.err;
}

int ckks_op_moddown(const ckks_params* P, int level, int rescale, const uint64_t* x, uint64_t* out, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!x || !out || (rescale && level < 1)) return CKKS_E_INVALID_ARG;
  Run R;
  int e = op_prologue(P, level, ws, ws_bytes, R, stream);
  if (e) return e;
  DeviceGuard dg(P->device);
  divide(R, rescale ? DIV_MODDOWN_RESCALE : DIV_MODDOWN, Jobs{{level, x, out}});
  return R.err;
}

int ckks_op_rescale(const ckks_params* P, int level, const uint64_t* x, uint64_t* out, void* ws, size_t ws_bytes,
                    void* stream) {
  if (!x || !out || level < 1) return CKKS_E_INVALID_ARG;
  Run R;
  int e = op_prologue(P, level, ws, ws_bytes, R, stream);
  if (e) return e;
  DeviceGuard dg(P->device);
  divide(R, DIV_RESCALE, Jobs{{level, x, out}});
  return R.err;
}

int ckks_op_keyswitch(const ckks_params* P, int level, const uint64_t* digits, const uint64_t* key, int32_t rot,
                      const uint64_t* add, uint64_t* out_a, uint64_t* out_b, void* stream) {
  if (!P || !digits || !key || !out_a || !out_b || level < 0 || level > P->L) return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  Run R = make_run(P, stream, false, nullptr);
  keyswitch(R, {KsTask{digits, level, add, false, key, galois(P, -(long)rot), out_a, out_b, false}});
  return R.err;
}

int ckks_op_automorph(const ckks_params* P, int32_t rot, int n_limbs, const uint64_t* in, uint64_t* out,
                      void* stream) {
  if (!P || !in || !out || n_limbs < 0 || n_limbs > P->Kmax() || in == out) return CKKS_E_INVALID_ARG;
  DeviceGuard dg(P->device);
  Run R = make_run(P, stream, false, nullptr);
  automorph(R, n_limbs, 0, galois(P, rot), in, nullptr, out, false);
  return R.err;
}

}  // extern "C"
