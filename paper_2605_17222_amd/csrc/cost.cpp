// Operation-count model of the LT algorithms (Table I and the counts of
// Section III) and the split autotuner built on it.
//
// Modular multiplications are counted as in Table II: a limb (I)NTT costs
// (N/2) log2 N, a basis conversion |S| |D| N + |S| N (the products and the
// (S/s_j)^-1 scaling), a key-switch inner product 2 beta K N, the plaintext
// products 2 n K N (PQ basis) or 2 n (l+1) N (Q basis, plain BSGS).
// Decompose = INTT of l+1 limbs, the per-group conversions, NTT of every
// converted limb; ModDown = INTT of alpha limbs, alpha (l+1) N conversion
// products, NTT of l+1 limbs, the final multiplication (l+1) N; the final
// ModDown by P q_l has alpha+1 source and l destination limbs.  With w = 54,
// N = 2^16, L+1 = 32, alpha = 12 this gives Table II's switching-key sizes
// exactly and its DH-BSGS / TH-BSGS multiplication counts within 0.5%.
//
// The predictor estimates a split's time on the device from the same counts:
// limb NTTs x (time per limb NTT) + conversion products x (time per product)
// + the words the key-switch and MAC kernels move (as this library schedules
// them) / (achieved bandwidth) + a latency per active hoisting layer (each
// layer is a chain of dependent launches).  The autotuner picks the split
// with the smallest prediction that needs at most max_keys switching keys.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "../../include/ckks_lt.h"

namespace {

struct Counts {
  double dec, md, mdr, ks, n, keys, mac_limbs;
};

int counts(int algo, int n1, int n2, int n3, int Lq, int K, Counts* c) {
  memset(c, 0, sizeof(*c));
  if (algo == CKKS_LT_TH_BSGS) {
    c->n = (double)n1 * n2 * n3;
    c->dec = n1 + n3 - 1;
    c->md = n1 + n3 - 2;
    c->mdr = 2;
    c->ks = (double)n1 * n2 + n3 - 2;
    c->keys = n1 + n2 + n3 - 3;
    c->mac_limbs = K;
  } else if (algo == CKKS_LT_DH_BSGS) {
    c->n = (double)n1 * n2;
    c->dec = n2;
    c->md = n2 - 1;
    c->mdr = 2;
    c->ks = n1 + n2 - 2;
    c->keys = n1 + n2 - 2;
    c->mac_limbs = K;
  } else if (algo == CKKS_LT_BSGS) {
    c->n = (double)n1 * n2;
    c->dec = n1 + n2 - 2;
    c->md = 2.0 * (n1 + n2 - 2);
    c->mdr = 0;
    c->ks = n1 + n2 - 2;
    c->keys = n1 + n2 - 2;
    c->mac_limbs = Lq;
  } else {
    return CKKS_E_INVALID_ARG;
  }
  return CKKS_OK;
}

}  // namespace

extern "C" {

int ckks_lt_cost_model(int log_n, int level, int alpha, int algo, int n1, int n2, int n3, int word_bits,
                 ckks_lt_cost* out) {
  if (!out || log_n < 1 || log_n > 20 || level < 0 || alpha < 1 || n1 < 1 || n2 < 1 || n3 < 1 || word_bits < 1)
    return CKKS_E_INVALID_ARG;
  if (algo != CKKS_LT_TH_BSGS) n3 = 1;
  const double N = (double)(1 << log_n), ntt = N / 2 * log_n;
  const int Lq = level + 1, K = alpha + Lq, beta = (Lq + alpha - 1) / alpha;
  Counts c;
  const int e = counts(algo, n1, n2, n3, Lq, K, &c);
  if (e != CKKS_OK) return e;
  // Decompose: INTT of Lq limbs; per group g: g (K - g) N products + g N scaling; NTT of K - g limbs.
  double dec = Lq * ntt, dec_ntt = Lq;
  for (int b = 0; b < beta; ++b) {
    const int g = std::min(alpha, Lq - alpha * b);
    dec += (double)g * (K - g) * N + g * N + (K - g) * ntt;
    dec_ntt += K - g;
  }
  const double md = alpha * ntt + (double)alpha * Lq * N + Lq * ntt + Lq * N;
  const double mdr = (alpha + 1) * ntt + (double)(alpha + 1) * (Lq - 1) * N + (Lq - 1) * ntt + (Lq - 1) * N;
  const double ks = 2.0 * beta * K * N;
  memset(out, 0, sizeof(*out));
  out->decompose = c.dec;
  out->moddown = c.md + c.mdr;
  out->keyswitch = c.ks;
  out->keys = (int)c.keys;
  out->modmul = c.dec * dec + c.md * md + c.mdr * mdr + c.ks * ks + 2.0 * c.n * c.mac_limbs * N;
  out->ntt_limbs = c.dec * dec_ntt + c.md * (alpha + Lq) + c.mdr * (alpha + 1 + Lq - 1);
  const double word = word_bits / 8.0;
  out->key_bytes = c.keys * 2.0 * beta * K * N * word;
  out->pt_bytes = c.n * c.mac_limbs * N * word;
  return CKKS_OK;
}

int ckks_lt_predict(int log_n, int level, int alpha, int algo, int n1, int n2, int n3, int n_diag,
                    const ckks_lt_rates* rates, double* seconds) {
  if (!seconds || n_diag < 0 || log_n < 1 || log_n > 20 || level < 0 || alpha < 1 || n1 < 1 || n2 < 1 || n3 < 1)
    return CKKS_E_INVALID_ARG;
  ckks_lt_rates r;
  if (rates) {
    r = *rates;
  } else {
    // Measured on one MI355X (python -m paper_2605_17222_amd.calibrate: 120
    // banded LTs at N = 2^16, levels 8, 16, 24, 16..256 diagonals): the BConv
    // rate from that kernel's own time, the other three fitted to the rest;
    // mean prediction error 6.3% (max 20%), the pick 2.2% slower than the
    // fastest timed split of its group on average (at most 7.4%; identical
    // runs of one split differ by up to 2%).
    r.ntt_limb_s = 1.82e-7;
    r.bconv_product_s = 0.650e-12;
    r.hbm_bytes_per_s = 4.69e12;
    r.layer_s = 97.0e-6;
  }
  if (algo == CKKS_LT_DH_BSGS) {  // Algorithm 2 with an empty inner layer
    n3 = n2;
    n2 = n1;
    n1 = 1;
    algo = CKKS_LT_TH_BSGS;
  }
  if (algo != CKKS_LT_TH_BSGS) n3 = 1;
  // A banded matrix (offsets 0 .. n_diag - 1) leaves the blocks past its
  // last diagonal absent, and the library skips their work (the outer
  // rotations of empty giant-step blocks, the middle rotations and inner
  // products with no diagonal): price the split it really runs.
  if (n_diag > 0) {
    const long inner = (long)n1 * n2;
    if (algo == CKKS_LT_TH_BSGS) n3 = (int)std::min<long>(n3, (n_diag + inner - 1) / inner);
    if (n_diag < inner) {
      n2 = (int)std::min<long>(n2, (n_diag + n1 - 1) / n1);
      n1 = std::min(n1, n_diag);
    }
  }
  // TH-BSGS (n1, 1, n3) runs as (1, n1, n3): the same terms and rotations.
  if (algo == CKKS_LT_TH_BSGS && n2 == 1 && n1 > 1) {
    n2 = n1;
    n1 = 1;
  }
  ckks_lt_cost c;
  const int e = ckks_lt_cost_model(log_n, level, alpha, algo, n1, n2, n3, 64, &c);
  if (e != CKKS_OK) return e;
  const double N = (double)(1 << log_n);
  const double nscale = N * log_n / (65536.0 * 16);
  const int Lq = level + 1, K = alpha + Lq, beta = (Lq + alpha - 1) / alpha;
  double conv = 0;
  for (int g = 0; g < beta; ++g) {
    const int gs = std::min(alpha, Lq - alpha * g);
    conv += (double)gs * (K - gs);
  }
  const double bconv_products = (c.decompose * conv + c.moddown * alpha * Lq) * N;
  // Words moved per coefficient position by the HBM-bound kernels as this
  // library schedules one LT: a key (2 beta K words at this level) is read
  // once per launch for every digit set that uses it (up to 8 digit sets per
  // launch).  With at most 4 accumulators, or at most 8 and terms that fit
  // one launch, the middle key switch runs fused with the multiply-
  // accumulate (lines 8-14 in one kernel per 16 terms): each middle key,
  // digit set and add read once, the rotation products never stored;
  // otherwise every product is written once and read once by the MAC.
  const double keyw = 2.0 * beta * K;
  double words = 0;
  int layers = 0;
  if (algo == CKKS_LT_TH_BSGS) {
    if (n1 > 1) {
      words += beta * K + (n1 - 1) * keyw + (n1 - 1) * 2.0 * K + Lq;
      ++layers;
    }
    if (n2 > 1 && n3 <= 8 && (n3 <= 4 || n1 * n2 <= 16)) {
      // launches of 16 terms, ordered by middle step: each launch reads the
      // digit sets and adds of its terms (up to 16) and each key once, and
      // every launch after the first reads and writes the accumulators
      const int launches = (n1 * n2 + 15) / 16, per = std::min(n1, 16), spans = (n1 + 15) / 16;
      words += (double)spans * (n2 - 1) * keyw + (double)launches * per * (beta + 1.0) * K + 2.0 * n1 * K +
               (double)n_diag * K + 2.0 * n3 * K + (launches - 1) * 4.0 * n3 * K;
      ++layers;
    } else {
      if (n2 > 1) {
        words += ((n1 + 7) / 8) * (n2 - 1) * keyw + n1 * (double)beta * K + n1 * (double)K +
                 (double)n1 * (n2 - 1) * 2.0 * K;
        ++layers;
      }
      words += 2.0 * n1 * n2 * K + (double)n_diag * K + 2.0 * n3 * K;
    }
    if (n3 > 1) {
      words += (n3 - 1) * (beta * (double)K + keyw + K) + 4.0 * K;
      ++layers;
    }
  } else {
    // plain BSGS: every rotation has its own digits, key, (x, y), ModDown
    // and automorphism; the plaintext products are at the Q basis.
    words += (n1 - 1 + n2 - 1) * (beta * (double)K + keyw + 2.0 * K + 5.0 * Lq);
    words += 2.0 * n1 * Lq + (double)n_diag * Lq + 2.0 * n2 * Lq;
    layers = (n1 > 1) + (n2 > 1);
  }
  *seconds = c.ntt_limbs * r.ntt_limb_s * nscale + bconv_products * r.bconv_product_s +
             words * N * 8 / r.hbm_bytes_per_s + layers * r.layer_s;
  return CKKS_OK;
}

int ckks_lt_autotune(int log_n, int level, int alpha, int algo, int n_diag, int max_keys, const ckks_lt_rates* rates,
                     int* n1, int* n2, int* n3, double* predicted_s) {
  if (!n1 || !n2 || !n3 || n_diag < 1 || log_n < 1 || log_n > 20) return CKKS_E_INVALID_ARG;
  double best = -1;
  int b1 = 0, b2 = 0, b3 = 0;
  const int nmax = 2 * n_diag;
  for (int a = 1; a <= n_diag; ++a)
    for (int b = 1; (long)a * b <= nmax; ++b) {
      const int c3max = algo == CKKS_LT_TH_BSGS ? nmax : 1;
      for (int c = 1; c <= c3max && (long)a * b * c <= nmax; ++c) {
        const long tot = (long)a * b * c;
        if (tot < n_diag) continue;
        if (c > 1 && (long)a * b * (c - 1) >= n_diag) break;  // c larger than needed
        ckks_lt_cost cost;
        if (ckks_lt_cost_model(log_n, level, alpha, algo, a, b, c, 64, &cost) != CKKS_OK) continue;
        if (max_keys > 0 && cost.keys > max_keys) continue;
        double t;
        if (ckks_lt_predict(log_n, level, alpha, algo, a, b, c, n_diag, rates, &t) != CKKS_OK) continue;
        if (best < 0 || t < best - 1e-12) {
          best = t;
          b1 = a;
          b2 = b;
          b3 = c;
        }
      }
    }
  if (best < 0) return CKKS_E_UNSUPPORTED;
  *n1 = b1;
  *n2 = b2;
  *n3 = algo == CKKS_LT_TH_BSGS ? b3 : 1;
  if (predicted_s) *predicted_s = best;
  return CKKS_OK;
}

int ckks_th_traffic_model(int log_n, int level, int alpha, int n1, int n2, int n3, int n_diag, int word_bits,
                          const ckks_th_parallelism* par, ckks_th_traffic* out) {
  if (!par || !out || log_n < 1 || log_n > 30 || level < 0 || alpha < 1 || n1 < 1 || n2 < 1 || n3 < 1 ||
      n_diag < 0 || word_bits < 1 || par->m2 < 1 || par->m3 < 1 || par->m5 < 1 || par->m6 < 1)
    return CKKS_E_INVALID_ARG;
  const double Lq = level + 1.0, K = Lq + alpha, beta = ceil(Lq / alpha), n = n_diag;
  auto rounds = [](double a, double b) { return ceil(a / b); };
  const double r2 = rounds(n1 - 1.0, par->m2), r3 = rounds(n2 - 1.0, par->m3);
  const double r5 = rounds((double)n1 * n2, par->m5), r6 = rounds((double)n3, par->m6);
  // Table III, one row per phase: (I)NTT twiddles, LT matrix, switching keys,
  // polynomial reads, polynomial writes
  const double t[6][5] = {
      {3 * Lq + 2 * alpha, 0, 2 * (n1 - 1.0) * beta * K, 2 * Lq, 3 * (n1 - 1.0) * K + 2 * Lq},
      {r2 * K, 0, 0, (n1 - 1.0) * K, (n1 - 1.0) * beta * K},
      {0, 0, 2 * (n2 - 1.0) * beta * K, r3 * n1 * (beta + 1) * K, 2.0 * n1 * n2 * K},
      {K, n * K, 0, 2 * (n1 * (double)n2 + (r5 - 1) * n3) * K, 2 * r5 * n3 * K},
      {r6 * K, 0, 2 * (n3 - 1.0) * beta * K, 2 * (n3 + r6 - 1) * K, 2 * r6 * K},
      {K, 0, 0, 2 * K, 2 * Lq},
  };
  memset(out, 0, sizeof(*out));
  double* col[5] = {&out->twiddle_limbs, &out->matrix_limbs, &out->key_limbs, &out->read_limbs, &out->write_limbs};
  for (int p = 0; p < 6; ++p)
    for (int c = 0; c < 5; ++c) {
      out->phase_limbs[p] += t[p][c];
      *col[c] += t[p][c];
      out->total_limbs += t[p][c];
    }
  out->total_bytes = out->total_limbs * ldexp(1.0, log_n) * word_bits / 8.0;
  return CKKS_OK;
}

}  // extern "C"
