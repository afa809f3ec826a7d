// Negacyclic NTT / inverse NTT over batches of limbs (gfx950).
//
// Layout (bit-reversed storage, Section V): word p of an NTT-form limb holds
// the evaluation at psi^(2 br(p) + 1).  The forward transform is the radix-2
// Cooley-Tukey network with twiddle psi^br(m + i) at stage m (log2 m = s),
// butterfly (x, x + N/2m); the inverse is the Gentleman-Sande network with
// psi^-br(m + i) and a final factor N^-1.  The PE butterflies of Section V
// (a0 +- a1 tf; (a0 + a1), (a0 - a1) tf) are exactly these, with the halving
// collected into N^-1.
//
// A limb of N = N1 N2 words is transformed in two passes of log2 N1 and
// log2 N2 stages (at N = 2^16 a limb is 512 KiB, larger than one workgroup's
// LDS):
//   column pass: the first log2 N1 stages act on the N2 columns (stride N2)
//                independently;
//   row pass:    the last log2 N2 stages act on the N1 rows (contiguous)
//                independently.
// Inside a pass each thread keeps 16 words in registers: 4 stages run in
// registers, the words are exchanged through LDS, and the remaining stages run
// in registers again.
//
// Two arithmetic paths, chosen per limb (uniform over a workgroup):
//  * integer (q >= 2^46): Harvey's lazy butterflies ([0, 4q) forward,
//    [0, 2q) inverse) with Shoup twiddle products;
//  * FP64 (q < 2^46): residues are doubles holding exact integers, the
//    twiddle product is the exact FMA two-product remainder of modarith.hpp,
//    values are re-centred every 4 stages.  Between the two passes such a limb
//    is stored as raw double bits; the final pass writes canonical residues.
//
// Stage s of a sub-transform of P = 2^p points whose global twiddle base is B
// uses twiddle index B 2^s + (x >> (p - s)) for butterfly position x; B = 1
// for the column pass and B = N1 + row for the row pass.  The column pass
// reads its 2^p - 1 twiddles from the full table (shared by all columns, so
// they stay in cache); the row pass of an FP64 limb would read a different
// 2^p - 1 for every row (the whole table, twice the limb's own bytes), so it
// forms them instead as G[s][y] R[row][s] mod q from two small tables (the
// factorisation is described at ntt_row_tables_size).
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

__device__ __forceinline__ double as_d(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ uint64_t as_u(double d) { return (uint64_t)__double_as_longlong(d); }

// SIN (forward column pass only): the input is the range's shared signed
// coefficients (LimbRange::signed_in).
template <int PLOG, int G, bool COL, bool FWD, bool FP, bool SIN>
__device__ __forceinline__ void ntt_body(const LimbRange& R, int limb, const PrimeDev& pr, int log_n, int epi,
                                         uint64_t* lds, double* tws) {
  constexpr int P = 1 << PLOG;
  constexpr int T = P / 16;           // threads per sub-transform
  constexpr int RS = P + P / 16 + 1;  // LDS row stride (padded)
  const uint64_t q = pr.q, q2 = 2 * q;
  const double qd = pr.qd, qi = pr.qinv_d;
  const int n = 1 << log_n;
  const uint64_t* __restrict__ tw = pr.tw + (FWD ? 0 : 2 * (size_t)n);
  const bool first = (COL == FWD);  // first pass of the transform
  const uint64_t* __restrict__ src = (first ? R.in : R.out) + (SIN ? 0 : (size_t)limb * n);
  uint64_t* __restrict__ dst = R.out + (size_t)limb * n;

  const int tid = threadIdx.x;
  int g, j;
  if (COL) {
    g = tid % G;
    j = tid / G;
  } else {
    j = tid % T;
    g = tid / T;
  }
  const int sub = blockIdx.x * G + g;  // column index (column pass) or row index (row pass)
  const int ncols = n >> PLOG;
  const uint32_t base = COL ? 1u : (uint32_t)((n >> PLOG) + sub);
  uint64_t* L = lds + g * RS;

  uint64_t v[16];  // integer residues, or double bits on the FP path
  auto addr = [&](int x) -> size_t { return COL ? (size_t)x * ncols + sub : (size_t)sub * P + x; };

  // FP row pass: the factor tables of this direction, G (P doubles, shared
  // by every row) and the R factors of the workgroup's G rows, staged into
  // LDS once (stage_tw) so that no stage waits on a global load for its
  // twiddles.
  const double* tg = tws;
  const double* tr = tws + P + 2 * g * PLOG;
  auto stage_tw = [&]() {
    if (FP && !COL) {
      const double* __restrict__ gs = pr.trow + (FWD ? 0 : ntt_row_tables_size(log_n));
      const double* __restrict__ rs = gs + P + 2 * (size_t)(blockIdx.x * G) * PLOG;
      for (int e = tid; e < P; e += G * P / 16) tws[e] = gs[e];
      for (int e = tid; e < G * 2 * PLOG; e += G * P / 16) tws[P + e] = rs[e];
      __syncthreads();
    }
  };
  // Twiddle of stage s, group y (index base 2^s + y): the value and its
  // companion (Shoup word, or w/q on the FP path), as raw 64-bit words.
  auto twid = [&](int s, uint32_t y, uint64_t& w, uint64_t& wp) {
    if (FP && !COL) {
      // |w| <= 0.75 q; wq = w/q to within 2 ulp, which keeps the products
      // that use it within the bounds of fp_mulmod.
      const double wv = fp_mulmod(tg[(1u << s) + y], tr[2 * s], tr[2 * s + 1], qd);
      w = as_u(wv);
      wp = as_u(wv * qi);
    } else {
      const uint32_t ti = (base << s) + y;
      w = tw[ti];
      wp = tw[n + ti];
    }
  };

  // One butterfly between registers u and u + d with twiddle (tw_w, tw_p).
  auto bfly = [&](int u, int d, uint64_t tw_w, uint64_t tw_p) {
    if (FP) {
      const double w = as_d(tw_w), wq = as_d(tw_p);
      const double X = as_d(v[u]), Y = as_d(v[u + d]);
      if (FWD) {
        const double r = fp_mulmod(Y, w, wq, qd);
        v[u] = as_u(X + r);
        v[u + d] = as_u(X - r);
      } else {
        v[u] = as_u(X + Y);
        v[u + d] = as_u(fp_mulmod(X - Y, w, wq, qd));
      }
    } else {
      const uint64_t w = tw_w, wp = tw_p;
      if (FWD) {
        uint64_t X = v[u];
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(v[u + d], w, wp, q);
        v[u] = X + t;
        v[u + d] = X - t + q2;
      } else {
        const uint64_t X = v[u], Y = v[u + d];
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        v[u] = sm;
        v[u + d] = shoup_lazy(X - Y + q2, w, wp, q);
      }
    }
  };
  // Stages 0..3 in layout "x = j + T u": group y = u >> (4 - s), 2^s groups.
  auto round1 = [&]() {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = FWD ? k : 3 - k;
      const int d = 8 >> s;
      uint64_t W[8], WP[8];
#pragma unroll
      for (int y = 0; y < (1 << s); ++y) twid(s, (uint32_t)y, W[y], WP[y]);
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (!(u & d)) bfly(u, d, W[u >> (4 - s)], WP[u >> (4 - s)]);
    }
  };
  // Stages 4..PLOG-1 in layout "x = 16 j + u": group (16 j + u) >> sh with
  // sh = PLOG - s <= 4, i.e. (16 j >> sh) + (u >> sh), 16 >> sh groups.
  auto round2 = [&]() {
#pragma unroll
    for (int k = 4; k < PLOG; ++k) {
      const int s = FWD ? k : PLOG - 1 - (k - 4);
      const int d = P >> (s + 1);
      const int sh = PLOG - s;
      const uint32_t y0 = (uint32_t)(16 * j) >> sh;
      uint64_t W[8], WP[8];
#pragma unroll
      for (int c = 0; c < (16 >> sh); ++c) twid(s, y0 + (uint32_t)c, W[c], WP[c]);
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (!(u & d)) bfly(u, d, W[u >> sh], WP[u >> sh]);
    }
  };
  auto recentre = [&]() {
    if (FP) {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = as_u(fp_reduce(as_d(v[u]), qd, qi));
    }
  };
  auto to_lds = [&](bool layout1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) L[lds_pad(layout1 ? (j + T * u) : (16 * j + u))] = v[u];
  };
  auto from_lds = [&](bool layout1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = L[lds_pad(layout1 ? (j + T * u) : (16 * j + u))];
  };
  // Canonical residues arrive as integers; the FP path converts them.
  auto convert_in = [&]() {
    if (FP) {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = as_u(u64_to_d(v[u]));
    }
  };
  // Final values -> canonical residues.
  auto canon = [&](uint64_t x) -> uint64_t {
    if (FP) return fp_canon(as_d(x), qd, qi);
    x = x >= q2 ? x - q2 : x;
    return csub(x, q);
  };

  if (FWD) {
    if constexpr (SIN) {
      // signed coefficients -> residues: |m / q| < 2^33, so the estimated
      // quotient is within one of the floor and r lands in [-q, 2q)
      const int64_t* __restrict__ sc = reinterpret_cast<const int64_t*>(src);
      const int64_t qs = (int64_t)q;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t m = sc[addr(j + T * u)];
        int64_t r = m - (int64_t)floor((double)m * qi) * qs;
        r = r < 0 ? r + qs : r;
        r = r >= qs ? r - qs : r;
        v[u] = (uint64_t)r;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = __builtin_nontemporal_load(src + addr(j + T * u));
    }
    if (!COL) stage_tw();
    if (first) convert_in();
    round1();
    recentre();
    to_lds(true);
    __syncthreads();
    from_lds(false);
    round2();
    if (COL) {
      // intermediate of the transform: lazy integers or double bits
#pragma unroll
      for (int u = 0; u < 16; ++u) dst[addr(16 * j + u)] = v[u];
    } else {
      __syncthreads();
      to_lds(false);
      __syncthreads();
      from_lds(true);
      const uint64_t* aux = (epi == EPI_SUBMUL) ? R.aux + (size_t)limb * n : nullptr;
      uint64_t c = 0, cs = 0;
      if (epi == EPI_SUBMUL) {
        c = R.sinv[limb];
        cs = R.sinv_sh[limb];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int x = j + T * u;
        uint64_t y = canon(v[u]);
        if (epi == EPI_SUBMUL) y = shoup(__builtin_nontemporal_load(aux + addr(x)) - y + q, c, cs, q);
        dst[addr(x)] = y;
      }
    }
  } else {
    if (COL) {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = __builtin_nontemporal_load(src + addr(16 * j + u));
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = __builtin_nontemporal_load(src + addr(j + T * u));
      if (R.copy) {
        uint64_t* __restrict__ cp = R.copy + (size_t)limb * n;
#pragma unroll
        for (int u = 0; u < 16; ++u) cp[addr(j + T * u)] = v[u];
      }
      stage_tw();
      to_lds(true);
      __syncthreads();
      from_lds(false);
      __syncthreads();
    }
    if (first) convert_in();
    round2();
    recentre();
    to_lds(false);
    __syncthreads();
    from_lds(true);
    round1();
    if (!first) {
      // last pass: times N^-1, canonical
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        uint64_t y;
        if (FP)
          y = fp_canon(fp_mulmod(as_d(v[u]), pr.ninv_d, pr.ninv_q, qd), qd, qi);
        else
          y = shoup(v[u], pr.ninv, pr.ninv_sh, q);
        dst[addr(j + T * u)] = y;
      }
    } else {
      recentre();
#pragma unroll
      for (int u = 0; u < 16; ++u) dst[addr(j + T * u)] = v[u];
    }
  }
}

template <int PLOG, int G, bool COL, bool FWD, bool SIN>
__global__ void __launch_bounds__(G*(1 << PLOG) / 16)
    ntt_pass(NttArgs args, const PrimeDev* __restrict__ primes, int log_n, int epi) {
  constexpr int P = 1 << PLOG;
  constexpr int RS = P + P / 16 + 1;
  __shared__ uint64_t lds[G * RS];
  __shared__ double tws[COL ? 1 : P + G * 2 * PLOG];  // FP row pass twiddle factors
  // Which limb (uniform over the workgroup).
  int limb = blockIdx.y;
  int ri = 0;
  while (ri < args.nr - 1 && limb >= args.r[ri].count) {
    limb -= args.r[ri].count;
    ++ri;
  }
  const LimbRange& R = args.r[ri];
  const PrimeDev& pr = primes[R.prime0 + limb];
  if (pr.fp)
    ntt_body<PLOG, G, COL, FWD, true, SIN>(R, limb, pr, log_n, epi, lds, tws);
  else
    ntt_body<PLOG, G, COL, FWD, false, SIN>(R, limb, pr, log_n, epi, lds, tws);
}

// Sub-transforms per workgroup: 4096 / P (16 at N = 2^16: 256 threads,
// 128-byte column segments).  A quarter of that for launches over a few
// limbs (4x the workgroups) was measured slower: the inverse column pass
// over 9-10 limbs 0.106 -> 0.147 ms per (4,4,4) LT, its 32-byte column
// segments costing more than the extra workgroups gain.
template <int PLOG, bool COL, bool FWD>
hipError_t launch_pass(const ckks_params* P, const NttArgs& a, int total, int epi, hipStream_t s) {
  constexpr int Pn = 1 << PLOG;
  constexpr int G = 4096 / Pn;
  const int n = P->n;
  const int subs = n >> PLOG;  // columns (column pass) or rows
  if (subs % G) return hipErrorInvalidValue;
  dim3 grid(subs / G, total);
  const int id = FWD ? (COL ? CKKS_KERNEL_NTT_FWD_COL : CKKS_KERNEL_NTT_FWD_ROW)
                     : (COL ? CKKS_KERNEL_NTT_INV_COL : CKKS_KERNEL_NTT_INV_ROW);
  double words = (double)total * n * (epi == EPI_SUBMUL ? 3 : 2);
  if (!FWD && !COL)
    for (int i = 0; i < a.nr; ++i) words += a.r[i].copy ? (double)a.r[i].count * n : 0;
  // signed input: every range of the launch, forward transforms only
  const bool sin = a.r[0].signed_in != 0;
  for (int i = 1; i < a.nr; ++i)
    if ((a.r[i].signed_in != 0) != sin) return hipErrorInvalidValue;
  if (sin && !FWD) return hipErrorInvalidValue;
  ProfScope prof(id, s, words * 8);
  if constexpr (COL && FWD) {
    if (sin) {
      hipLaunchKernelGGL((ntt_pass<PLOG, G, COL, FWD, true>), grid, dim3(G * Pn / 16), 0, s, a, P->d_primes,
                         P->log_n, epi);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((ntt_pass<PLOG, G, COL, FWD, false>), grid, dim3(G * Pn / 16), 0, s, a, P->d_primes,
                     P->log_n, epi);
  return hipGetLastError();
}

template <int PA, int PB>
hipError_t launch_both(const ckks_params* P, bool forward, const NttArgs& a, int total, int epi, hipStream_t s) {
  hipError_t e;
  if (forward) {
    e = launch_pass<PA, true, true>(P, a, total, EPI_NONE, s);
    if (e != hipSuccess) return e;
    return launch_pass<PB, false, true>(P, a, total, epi, s);
  }
  e = launch_pass<PB, false, false>(P, a, total, EPI_NONE, s);
  if (e != hipSuccess) return e;
  return launch_pass<PA, true, false>(P, a, total, EPI_NONE, s);
}

}  // namespace

hipError_t launch_ntt(const ckks_params* P, bool forward, const NttArgs& a, int total_limbs, int epi,
                      hipStream_t s) {
  if (total_limbs <= 0) return hipSuccess;
  switch (P->log_n) {
    case 12: return launch_both<6, 6>(P, forward, a, total_limbs, epi, s);
    case 13: return launch_both<7, 6>(P, forward, a, total_limbs, epi, s);
    case 14: return launch_both<7, 7>(P, forward, a, total_limbs, epi, s);
    case 15: return launch_both<8, 7>(P, forward, a, total_limbs, epi, s);
    case 16: return launch_both<8, 8>(P, forward, a, total_limbs, epi, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ckks
