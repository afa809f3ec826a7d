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
// in registers again.  Butterflies use Harvey's lazy ranges ([0, 4q) forward,
// [0, 2q) inverse) and Shoup twiddle products; values are made canonical only
// on the final pass.
//
// Stage s of a sub-transform of P = 2^p points whose global twiddle base is B
// uses twiddle index B 2^s + (x >> (p - s)) for butterfly position x; B = 1
// for the column pass and B = N1 + row for the row pass.
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

template <int P>
__device__ __forceinline__ int lds_pad(int i) {
  return i + (i >> 4);
}

template <int PLOG, int G, bool COL, bool FWD>
__global__ void __launch_bounds__(G*(1 << PLOG) / 16)
    ntt_pass(NttArgs args, const PrimeDev* __restrict__ primes, int log_n, int epi,
             const BConvPlan* __restrict__ plan) {
  constexpr int P = 1 << PLOG;
  constexpr int T = P / 16;           // threads per sub-transform
  constexpr int RS = P + P / 16 + 1;  // LDS row stride (padded)
  __shared__ uint64_t lds[G * RS];

  // Which limb (uniform over the workgroup).
  int limb = blockIdx.y;
  int ri = 0;
  while (ri < args.nr - 1 && limb >= args.r[ri].count) {
    limb -= args.r[ri].count;
    ++ri;
  }
  const LimbRange& R = args.r[ri];
  const PrimeDev& pr = primes[R.prime0 + limb];
  const uint64_t q = pr.q, q2 = 2 * q;
  const int n = 1 << log_n;
  const uint64_t* __restrict__ tw = pr.tw + (FWD ? 0 : 2 * (size_t)n);
  const uint64_t* __restrict__ src = ((COL == FWD) ? R.in : R.out) + (size_t)limb * n;
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
  const int sub = blockIdx.x * G + g;       // column index (COL) or row index (row pass)
  const int ncols = n >> PLOG;              // N2 when COL
  // Global twiddle base of this sub-transform.
  const uint32_t base = COL ? 1u : (uint32_t)((n >> PLOG) + sub);
  uint64_t* L = lds + g * RS;

  uint64_t v[16];

  auto addr = [&](int x) -> size_t { return COL ? (size_t)x * ncols + sub : (size_t)sub * P + x; };

  // Round over local stages [s_lo, s_hi) (forward) in layout "x = j + T u".
  auto fwd_round1 = [&]() {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int d = 8 >> s;  // u-distance
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (u & d) continue;
        const uint32_t ti = (base << s) + (uint32_t)(u >> (4 - s));
        const uint64_t w = tw[ti], wp = tw[n + ti];
        uint64_t X = v[u], Y = v[u + d];
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(Y, w, wp, q);
        v[u] = X + t;
        v[u + d] = X - t + q2;
      }
    }
  };
  // Local stages 4 .. PLOG-1 in layout "x = 16 j + u".
  auto fwd_round2 = [&]() {
#pragma unroll
    for (int s = 4; s < PLOG; ++s) {
      const int d = P >> (s + 1);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (u & d) continue;
        const uint32_t ti = (base << s) + (uint32_t)((16 * j + u) >> (PLOG - s));
        const uint64_t w = tw[ti], wp = tw[n + ti];
        uint64_t X = v[u], Y = v[u + d];
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(Y, w, wp, q);
        v[u] = X + t;
        v[u + d] = X - t + q2;
      }
    }
  };
  auto inv_round2 = [&]() {
#pragma unroll
    for (int s = PLOG - 1; s >= 4; --s) {
      const int d = P >> (s + 1);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (u & d) continue;
        const uint32_t ti = (base << s) + (uint32_t)((16 * j + u) >> (PLOG - s));
        const uint64_t w = tw[ti], wp = tw[n + ti];
        const uint64_t X = v[u], Y = v[u + d];
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        v[u] = sm;
        v[u + d] = shoup_lazy(X - Y + q2, w, wp, q);
      }
    }
  };
  auto inv_round1 = [&]() {
#pragma unroll
    for (int s = 3; s >= 0; --s) {
      const int d = 8 >> s;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (u & d) continue;
        const uint32_t ti = (base << s) + (uint32_t)(u >> (4 - s));
        const uint64_t w = tw[ti], wp = tw[n + ti];
        const uint64_t X = v[u], Y = v[u + d];
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        v[u] = sm;
        v[u + d] = shoup_lazy(X - Y + q2, w, wp, q);
      }
    }
  };
  // Exchange layouts through LDS.
  auto to_lds = [&](bool from_round1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = from_round1 ? (j + T * u) : (16 * j + u);
      L[lds_pad<P>(x)] = v[u];
    }
  };
  auto from_lds = [&](bool to_round1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = to_round1 ? (j + T * u) : (16 * j + u);
      v[u] = L[lds_pad<P>(x)];
    }
  };
  const bool last = (COL != FWD);  // second pass of the transform

  if (FWD) {
    // load in layout j + T u (coalesced for both passes)
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = src[addr(j + T * u)];
    fwd_round1();
    to_lds(true);
    __syncthreads();
    from_lds(false);
    fwd_round2();
    if (COL) {
      // layout 16 j + u is coalesced across g for the column pass
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
        c = plan->sinv[R.epi0 + limb];
        cs = plan->sinv_sh[R.epi0 + limb];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int x = j + T * u;
        uint64_t y = v[u];
        y = y >= q2 ? y - q2 : y;
        y = csub(y, q);
        if (epi == EPI_SUBMUL) y = shoup(aux[addr(x)] - y + q, c, cs, q);
        dst[addr(x)] = y;
      }
    }
  } else {
    if (COL) {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = src[addr(16 * j + u)];
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = src[addr(j + T * u)];
      to_lds(true);
      __syncthreads();
      from_lds(false);
      __syncthreads();
    }
    inv_round2();
    to_lds(false);
    __syncthreads();
    from_lds(true);
    inv_round1();
    if (last) {
#pragma unroll
      for (int u = 0; u < 16; ++u) dst[addr(j + T * u)] = shoup(v[u], pr.ninv, pr.ninv_sh, q);
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) dst[addr(j + T * u)] = v[u];
    }
  }
}

template <int PLOG, bool COL, bool FWD>
hipError_t launch_pass(const ckks_params* P, const NttArgs& a, int total, int epi, const BConvPlan* plan,
                       hipStream_t s) {
  constexpr int Pn = 1 << PLOG;
  constexpr int G = 4096 / Pn;
  const int n = P->n;
  const int subs = n >> PLOG;  // columns (COL) or rows
  if (subs % G) return hipErrorInvalidValue;
  dim3 grid(subs / G, total);
  const int id = FWD ? (COL ? CKKS_KERNEL_NTT_FWD_COL : CKKS_KERNEL_NTT_FWD_ROW)
                     : (COL ? CKKS_KERNEL_NTT_INV_COL : CKKS_KERNEL_NTT_INV_ROW);
  ProfScope prof(id, s, (double)total * n * 8 * (epi == EPI_SUBMUL ? 3 : 2));
  hipLaunchKernelGGL((ntt_pass<PLOG, G, COL, FWD>), grid, dim3(G * Pn / 16), 0, s, a, P->d_primes, P->log_n,
                     epi, plan);
  return hipGetLastError();
}

template <int PA, int PB>
hipError_t launch_both(const ckks_params* P, bool forward, const NttArgs& a, int total, int epi,
                       const BConvPlan* plan, hipStream_t s) {
  hipError_t e;
  if (forward) {
    e = launch_pass<PA, true, true>(P, a, total, EPI_NONE, nullptr, s);
    if (e != hipSuccess) return e;
    return launch_pass<PB, false, true>(P, a, total, epi, plan, s);
  }
  e = launch_pass<PB, false, false>(P, a, total, EPI_NONE, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_pass<PA, true, false>(P, a, total, EPI_NONE, nullptr, s);
}

}  // namespace

hipError_t launch_ntt(const ckks_params* P, bool forward, const NttArgs& a, int total_limbs, int epi,
                      const BConvPlan* epi_plan, hipStream_t s) {
  if (total_limbs <= 0) return hipSuccess;
  switch (P->log_n) {
    case 12: return launch_both<6, 6>(P, forward, a, total_limbs, epi, epi_plan, s);
    case 13: return launch_both<7, 6>(P, forward, a, total_limbs, epi, epi_plan, s);
    case 14: return launch_both<7, 7>(P, forward, a, total_limbs, epi, epi_plan, s);
    case 15: return launch_both<8, 7>(P, forward, a, total_limbs, epi, epi_plan, s);
    case 16: return launch_both<8, 8>(P, forward, a, total_limbs, epi, epi_plan, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ckks
