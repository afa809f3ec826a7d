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
// A limb of N words is viewed as 16 rows of N/16 contiguous words (at
// N = 2^16 a limb is 512 KiB, larger than one workgroup's LDS), and each
// transform is two passes:
//   column pass: the first 4 stages act on the N/16 columns of 16 words
//                (stride N/16) independently: one thread holds a whole
//                column in registers, no exchange;
//   row pass:    the last log2 N - 4 stages act on the 16 rows of P = N/16
//                words independently: a workgroup holds G = 4096/P rows in
//                LDS, each thread 16 words in registers; up to three rounds
//                of at most 4 stages run in registers, separated by LDS
//                exchanges.
// The split puts 4 of the 16 stages of a transform in the column pass so
// that the basis conversions of Decompose and ModDown (bconv.hip) can finish
// an inverse transform and start a forward one on a tile of coefficient
// positions that stays in registers (the column stages of 16 rows), leaving
// only the row passes as separate launches.
//
// Arithmetic:
//  * column stages: integer Harvey lazy butterflies with Shoup twiddles
//    (PrimeDev::ctw) for every prime ([0, 4q) forward, [0, 2q) inverse);
//  * row stages, q >= 2^46: the same integer butterflies, twiddles from the
//    full table (value and Shoup word);
//  * row stages, q < 2^46: exact FP64 modular products (modarith.hpp), values
//    re-centred after every round, twiddles formed as G[s][y] R[row][s] mod q
//    from two small tables (ntt_row_tables_size) rather than read from the
//    full table.
// Between the passes a limb of an FP64 prime is stored as raw double bits
// (forward: canonical residues as doubles; inverse: re-centred values), an
// integer prime's limb as lazy residues.  The last pass writes canonical
// residues.
//
// Row-pass indexing: a row of P = 2^PLOG points, T = P/16 threads, Tb = T/16.
// Stage s of the row pass (global stage 4 + s) pairs x and x + P/2^(s+1) and
// uses twiddle index (base << s) + (x >> (PLOG - s)), base = 16 + row.  The
// three register layouts of a thread j (u = 0 .. 15):
//   A: x = j + T u                          stages 0 .. 3   (u distance 8 >> s)
//   B: x = (j / Tb) T + u Tb + (j % Tb)     stages 4 .. 7   (u distance 8 >> (s - 4))
//   C: x = 16 j + u                         stages 8 .. PLOG-1
// (at PLOG = 8, Tb = 1 and B is C).  Loads and stores use layout A, which is
// coalesced (consecutive threads, consecutive words).
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

__device__ __forceinline__ double as_d(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ uint64_t as_u(double d) { return (uint64_t)__double_as_longlong(d); }

constexpr int kColThreads = 128;  // threads (columns) per column-pass workgroup

// ---- column pass ------------------------------------------------------------
// One thread per column: 16 words at x = c + (N/16) r, r = 0 .. 15, all four
// stages in registers.  Forward stage s pairs rows r and r + (8 >> s) with
// twiddle index 2^s + (r >> (4 - s)); the inverse runs the stages backwards.
// SIN (forward only): the input is N signed 64-bit coefficients shared by
// every limb of the range, reduced into the limb's prime here.
template <bool FWD, bool SIN>
__global__ void __launch_bounds__(kColThreads)
    ntt_col(NttArgs args, const PrimeDev* __restrict__ primes, int log_n) {
  int limb = blockIdx.y;
  int ri = 0;
  while (ri < args.nr - 1 && limb >= args.r[ri].count) {
    limb -= args.r[ri].count;
    ++ri;
  }
  const LimbRange& R = args.r[ri];
  const PrimeDev& pr = primes[R.prime0 + limb];
  const int n = 1 << log_n;
  const size_t n2 = (size_t)n >> kColLog;
  const size_t c = (size_t)blockIdx.x * kColThreads + threadIdx.x;
  const uint64_t q = pr.q, q2 = 2 * q;
  const uint64_t* __restrict__ tw = pr.ctw[FWD ? 0 : 1][0];
  const uint64_t* __restrict__ tp = pr.ctw[FWD ? 0 : 1][1];
  uint64_t v[16];
  if (FWD) {
    if constexpr (SIN) {
      // |m / q| < 2^33: the estimated quotient is within one of the floor
      const int64_t* __restrict__ sc = reinterpret_cast<const int64_t*>(R.in);
      const int64_t qs = (int64_t)q;
      const double qi = pr.qinv_d;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = sc[c + n2 * r];
        int64_t x = m - (int64_t)floor((double)m * qi) * qs;
        x = x < 0 ? x + qs : x;
        x = x >= qs ? x - qs : x;
        v[r] = (uint64_t)x;
      }
    } else {
      const uint64_t* __restrict__ src = R.in + (size_t)limb * n;
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = __builtin_nontemporal_load(src + c + n2 * r);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int d = 8 >> s;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r & d) continue;
        const int ti = (1 << s) + (r >> (4 - s));
        uint64_t X = v[r];
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(v[r + d], tw[ti], tp[ti], q);
        v[r] = X + t;
        v[r + d] = X - t + q2;
      }
    }
    uint64_t* __restrict__ dst = R.out + (size_t)limb * n;
    if (pr.fp) {
      // the FP64 row pass takes canonical residues as doubles
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        uint64_t x = v[r] >= q2 ? v[r] - q2 : v[r];
        x = csub(x, q);
        dst[c + n2 * r] = as_u(u64_to_d(x));
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) dst[c + n2 * r] = v[r];
    }
  } else {
    const uint64_t* __restrict__ src = R.in + (size_t)limb * n;
    if (pr.fp) {
      const double qd = pr.qd, qi = pr.qinv_d;
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = fp_canon(as_d(__builtin_nontemporal_load(src + c + n2 * r)), qd, qi);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = __builtin_nontemporal_load(src + c + n2 * r);
    }
#pragma unroll
    for (int s = 3; s >= 0; --s) {
      const int d = 8 >> s;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r & d) continue;
        const int ti = (1 << s) + (r >> (4 - s));
        const uint64_t X = v[r], Y = v[r + d];
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        v[r] = sm;
        v[r + d] = shoup_lazy(X - Y + q2, tw[ti], tp[ti], q);
      }
    }
    uint64_t* __restrict__ dst = R.out + (size_t)limb * n;
#pragma unroll
    for (int r = 0; r < 16; ++r) dst[c + n2 * r] = shoup(v[r], pr.ninv, pr.ninv_sh, q);
  }
}

// ---- row pass ---------------------------------------------------------------
template <int PLOG, bool FWD, bool FP>
__device__ __forceinline__ void row_body(const LimbRange& R, int limb, const PrimeDev& pr, int log_n, int epi,
                                         uint64_t* lds) {
  constexpr int P = 1 << PLOG;
  constexpr int T = P / 16;            // threads per row
  constexpr int G = 256 / T;           // rows per workgroup
  constexpr int TB = T / 16;           // layout B's inner count
  constexpr int RS = P + P / 16 + 1;   // LDS row stride (padded)
  constexpr bool HAS_C = PLOG > 8;     // a third round (else B is C)
  const uint64_t q = pr.q, q2 = 2 * q;
  const double qd = pr.qd, qi = pr.qinv_d;
  const int n = 1 << log_n;
  const int tid = threadIdx.x;
  const int g = tid / T, j = tid % T;
  const int row = blockIdx.x * G + g;
  const uint32_t base = 16u + (uint32_t)row;
  const int ja = j / TB, jb = j % TB;  // layout B coordinates
  uint64_t* L = lds + g * RS;
  const uint64_t* __restrict__ tw = pr.tw + (FWD ? 0 : 2 * (size_t)n);
  const double* __restrict__ tg = nullptr;
  const double* __restrict__ tr = nullptr;
  if (FP) {
    tg = pr.trow + (FWD ? 0 : ntt_row_tables_size(log_n));
    tr = tg + P + 2 * (size_t)row * PLOG;
  }
  uint64_t v[16];  // integer residues, or double bits on the FP path

  auto xA = [&](int u) { return j + T * u; };

  // Twiddle of row stage s, group y: value and companion (Shoup word, or
  // w/q on the FP path) as raw words.
  auto twid = [&](int s, uint32_t y, uint64_t& w, uint64_t& wp) {
    if (FP) {
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
      if (FWD) {
        uint64_t X = v[u];
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(v[u + d], tw_w, tw_p, q);
        v[u] = X + t;
        v[u + d] = X - t + q2;
      } else {
        const uint64_t X = v[u], Y = v[u + d];
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        v[u] = sm;
        v[u + d] = shoup_lazy(X - Y + q2, tw_w, tw_p, q);
      }
    }
  };
  // One stage s of the row pass in a layout where element u's butterfly
  // partner is u + 2^(sh-1) and its group is g0 + (u >> sh): 16 >> sh groups
  // (at most 8) per thread and stage.
  auto stage = [&](int s, int sh, uint32_t g0) {
    // the stage's twiddles are loaded here, not hoisted above earlier stages
    // (which would hold several stages' twiddles in registers at once)
    asm volatile("" ::: "memory");
    uint64_t W[8], WP[8];
#pragma unroll
    for (int k = 0; k < (16 >> sh); ++k) twid(s, g0 + (uint32_t)k, W[k], WP[k]);
    const int d = 1 << (sh - 1);
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (!(u & d)) bfly(u, d, W[u >> sh], WP[u >> sh]);
  };
  auto roundA = [&](int k) {  // k-th stage of round A in execution order
    const int s = FWD ? k : 3 - k;
    stage(s, 4 - s, 0u);
  };
  auto roundB = [&](int k) {
    const int s = FWD ? 4 + k : 7 - k;
    stage(s, 8 - s, (uint32_t)ja << (s - 4));
  };
  auto roundC = [&](int k) {
    const int s = FWD ? 8 + k : PLOG - 1 - k;
    stage(s, PLOG - s, (uint32_t)(16 * j) >> (PLOG - s));
  };
  auto recentre = [&]() {
    if (FP) {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = as_u(fp_reduce(as_d(v[u]), qd, qi));
    }
  };
  // LDS word of element u in each layout, lds_pad(x(u)) written as a
  // per-thread base plus a compile-time offset (T, Tb powers of two, T >= 16,
  // Tb dividing 16 or a multiple of it), so the accesses use immediate
  // offsets rather than one address register per word.
  const int lbA = j + (j >> 4);
  const int lbB = ja * (T + T / 16) + jb + (TB >= 16 ? (jb >> 4) : 0);
  const int lbC = 17 * j;
  auto offA = [&](int u) { return u * (T + T / 16); };
  auto offB = [&](int u) { return u * TB + ((u * TB) >> 4); };
  auto offC = [&](int u) { return u; };
  auto to_lds = [&](int b, auto off) {
#pragma unroll
    for (int u = 0; u < 16; ++u) L[b + off(u)] = v[u];
  };
  auto from_lds = [&](int b, auto off) {
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = L[b + off(u)];
  };
  auto exchange = [&](int bf, auto of, int bt, auto ot) {
    to_lds(bf, of);
    __syncthreads();
    from_lds(bt, ot);
    __syncthreads();
  };

  const uint64_t* __restrict__ src = R.in + (size_t)limb * n + (size_t)row * P;
  uint64_t* __restrict__ dst = R.out + (size_t)limb * n + (size_t)row * P;
  // word u of layout A in a row buffer: a uniform base plus a 32-bit byte
  // offset (no 64-bit address registers per word)
  auto wA = [&](const uint64_t* b, int u) -> uint64_t* {
    return reinterpret_cast<uint64_t*>(const_cast<char*>(reinterpret_cast<const char*>(b)) +
                                       (uint32_t)(8 * xA(u)));
  };
  if (FWD) {
    // input: the column pass's output (lazy residues, or doubles on the FP path)
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = __builtin_nontemporal_load(wA(src, u));
#pragma unroll
    for (int k = 0; k < 4; ++k) roundA(k);
    recentre();
    exchange(lbA, offA, lbB, offB);
#pragma unroll
    for (int k = 0; k < 4; ++k) roundB(k);
    if (HAS_C) {
      recentre();
      exchange(lbB, offB, lbC, offC);
#pragma unroll
      for (int k = 0; k < PLOG - 8; ++k) roundC(k);
      exchange(lbC, offC, lbA, offA);
    } else {
      exchange(lbB, offB, lbA, offA);
    }
    const uint64_t* aux = (epi == EPI_SUBMUL) ? R.aux + (size_t)limb * n + (size_t)row * P : nullptr;
    uint64_t c = 0, cs = 0;
    if (epi == EPI_SUBMUL) {
      c = R.sinv[limb];
      cs = R.sinv_sh[limb];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      uint64_t y;
      if (FP) {
        y = fp_canon(as_d(v[u]), qd, qi);
      } else {
        y = v[u] >= q2 ? v[u] - q2 : v[u];
        y = csub(y, q);
      }
      if (epi == EPI_SUBMUL) y = shoup(__builtin_nontemporal_load(wA(aux, u)) - y + q, c, cs, q);
      *wA(dst, u) = y;
    }
  } else {
    // input: canonical NTT-form residues
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = __builtin_nontemporal_load(wA(src, u));
    if (R.copy) {
      uint64_t* __restrict__ cp = R.copy + (size_t)limb * n + (size_t)row * P;
#pragma unroll
      for (int u = 0; u < 16; ++u) *wA(cp, u) = v[u];
    }
    if (FP) {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = as_u(u64_to_d(v[u]));
    }
    if (HAS_C) {
      exchange(lbA, offA, lbC, offC);
#pragma unroll
      for (int k = 0; k < PLOG - 8; ++k) roundC(k);
      recentre();
      exchange(lbC, offC, lbB, offB);
    } else {
      exchange(lbA, offA, lbB, offB);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) roundB(k);
    recentre();
    exchange(lbB, offB, lbA, offA);
#pragma unroll
    for (int k = 0; k < 4; ++k) roundA(k);
    recentre();
    // output: lazy residues, or re-centred doubles, for the column pass
#pragma unroll
    for (int u = 0; u < 16; ++u) *wA(dst, u) = v[u];
  }
}

template <int PLOG, bool FWD>
__global__ void __launch_bounds__(256) ntt_row(NttArgs args, const PrimeDev* __restrict__ primes, int log_n, int epi) {
  constexpr int P = 1 << PLOG;
  constexpr int G = 4096 / P;
  constexpr int RS = P + P / 16 + 1;
  __shared__ uint64_t lds[G * RS];
  int limb = blockIdx.y;
  int ri = 0;
  while (ri < args.nr - 1 && limb >= args.r[ri].count) {
    limb -= args.r[ri].count;
    ++ri;
  }
  const LimbRange& R = args.r[ri];
  const PrimeDev& pr = primes[R.prime0 + limb];
  if (pr.fp)
    row_body<PLOG, FWD, true>(R, limb, pr, log_n, epi, lds);
  else
    row_body<PLOG, FWD, false>(R, limb, pr, log_n, epi, lds);
}

bool ranges_ok(const NttArgs& a, int total) {
  if (a.nr < 1 || a.nr > kMaxRanges) return false;
  int sum = 0;
  for (int i = 0; i < a.nr; ++i) {
    if (a.r[i].count < 0 || !a.r[i].in || !a.r[i].out) return false;
    sum += a.r[i].count;
  }
  return sum == total;
}

hipError_t launch_col(const ckks_params* P, bool fwd, const NttArgs& a, int total, hipStream_t s) {
  const int n2 = P->n >> kColLog;
  if (n2 % kColThreads || !ranges_ok(a, total)) return hipErrorInvalidValue;
  const bool sin = a.r[0].signed_in != 0;
  for (int i = 1; i < a.nr; ++i)
    if ((a.r[i].signed_in != 0) != sin) return hipErrorInvalidValue;
  if (sin && !fwd) return hipErrorInvalidValue;
  dim3 grid(n2 / kColThreads, total);
  ProfScope prof(fwd ? CKKS_KERNEL_NTT_FWD_COL : CKKS_KERNEL_NTT_INV_COL, s, (double)total * P->n * 2 * 8);
  if (fwd && sin)
    hipLaunchKernelGGL((ntt_col<true, true>), grid, dim3(kColThreads), 0, s, a, P->d_primes, P->log_n);
  else if (fwd)
    hipLaunchKernelGGL((ntt_col<true, false>), grid, dim3(kColThreads), 0, s, a, P->d_primes, P->log_n);
  else
    hipLaunchKernelGGL((ntt_col<false, false>), grid, dim3(kColThreads), 0, s, a, P->d_primes, P->log_n);
  return hipGetLastError();
}

template <int PLOG>
hipError_t launch_row_t(const ckks_params* P, bool fwd, const NttArgs& a, int total, int epi, hipStream_t s) {
  constexpr int G = 4096 / (1 << PLOG);
  static_assert(16 % G == 0, "rows per workgroup");
  dim3 grid(16 / G, total);
  double words = (double)total * P->n * (epi == EPI_SUBMUL ? 3 : 2);
  if (!fwd)
    for (int i = 0; i < a.nr; ++i) words += a.r[i].copy ? (double)a.r[i].count * P->n : 0;
  ProfScope prof(fwd ? CKKS_KERNEL_NTT_FWD_ROW : CKKS_KERNEL_NTT_INV_ROW, s, words * 8);
  if (fwd)
    hipLaunchKernelGGL((ntt_row<PLOG, true>), grid, dim3(256), 0, s, a, P->d_primes, P->log_n, epi);
  else
    hipLaunchKernelGGL((ntt_row<PLOG, false>), grid, dim3(256), 0, s, a, P->d_primes, P->log_n, epi);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ntt_row(const ckks_params* P, bool forward, const NttArgs& a, int total_limbs, int epi,
                          hipStream_t s) {
  if (total_limbs <= 0) return hipSuccess;
  if (!ranges_ok(a, total_limbs) || (epi == EPI_SUBMUL && !forward)) return hipErrorInvalidValue;
  for (int i = 0; i < a.nr; ++i)
    if (a.r[i].signed_in || (epi == EPI_SUBMUL && (!a.r[i].aux || !a.r[i].sinv || !a.r[i].sinv_sh)) ||
        (a.r[i].copy && forward))
      return hipErrorInvalidValue;
  switch (P->log_n) {
    case 12: return launch_row_t<8>(P, forward, a, total_limbs, epi, s);
    case 13: return launch_row_t<9>(P, forward, a, total_limbs, epi, s);
    case 14: return launch_row_t<10>(P, forward, a, total_limbs, epi, s);
    case 15: return launch_row_t<11>(P, forward, a, total_limbs, epi, s);
    case 16: return launch_row_t<12>(P, forward, a, total_limbs, epi, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ntt(const ckks_params* P, bool forward, const NttArgs& a, int total_limbs, int epi,
                      hipStream_t s) {
  if (total_limbs <= 0) return hipSuccess;
  hipError_t e;
  if (forward) {
    // the column pass transforms in place into out; the row pass then reads out
    e = launch_col(P, true, a, total_limbs, s);
    if (e != hipSuccess) return e;
    NttArgs b = a;
    for (int i = 0; i < b.nr; ++i) {
      b.r[i].in = b.r[i].out;
      b.r[i].signed_in = 0;
    }
    return launch_ntt_row(P, true, b, total_limbs, epi, s);
  }
  if (epi != EPI_NONE) return hipErrorInvalidValue;
  e = launch_ntt_row(P, false, a, total_limbs, EPI_NONE, s);
  if (e != hipSuccess) return e;
  NttArgs b = a;
  for (int i = 0; i < b.nr; ++i) {
    b.r[i].in = b.r[i].out;
    b.r[i].copy = nullptr;
  }
  return launch_col(P, false, b, total_limbs, s);
}

}  // namespace ckks
