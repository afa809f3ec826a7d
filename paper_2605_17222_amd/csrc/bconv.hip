// Basis conversion, eq. (3):  y_j = [(S/s_j)^-1 x_j]_{s_j},
//                             out_m = sum_j y_j [S/s_j]_{d_m} mod d_m.
// Coefficient-domain limbs; each thread owns one coefficient position with
// all source limbs of that position in registers (the type-II dependency of
// Section IV: every limb of a coefficient is needed).  The constants
// [S/s_j]_{d_m} are stored times 2^64 mod d_m, so one Montgomery REDC of the
// exact 128-bit sum gives the canonical result; this needs sum_j s_j <= 2^64,
// which parameter creation checks.  The number of source limbs is a template
// parameter so the inner product is fully unrolled and its constants come in
// with wide scalar loads.  Several conversions (the digits of Decompose) run
// in one launch, one per blockIdx.y; blockIdx.z splits the destination limbs
// into chunks so that a launch has enough workgroups to fill 256 CUs.
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 27;     // most destination limbs per workgroup (grid.z splits the rest)
constexpr int kMinWgs = 2048;  // workgroups a launch is split to reach (8 per CU)
constexpr int kMinChunk = 6;   // fewest destination limbs per workgroup when splitting for that

// S30: every plan of the launch is split30 (all its primes below 2^60), so
// only the 30-bit halves of the y_j are kept (half the registers of the
// general kernel, which holds the full words for the 128-bit products).
template <int NS, bool S30>
__global__ void __launch_bounds__(kThreads)
    bconv_kernel(BConvArgs a, const PrimeDev* __restrict__ primes, int log_n, int chunk) {
  const int item = blockIdx.y;
  const BConvPlan* __restrict__ plan = a.plan[item];
  const uint64_t* __restrict__ src = a.src[item];
  uint64_t* __restrict__ dst = a.dst[item];
  const uint64_t* __restrict__ aux = a.aux[item];
  const int shift = a.dst_shift[item];
  const size_t n = (size_t)1 << log_n;
  const size_t p = (size_t)blockIdx.x * kThreads + threadIdx.x;
  // m1 <= m0 when this item has fewer destination limbs than the launch's
  // widest item: then the chunk is empty (cnt = 0) and only the shared
  // staging below runs (with nothing to stage).
  const int m0 = blockIdx.z * chunk;
  const int m1 = max(m0, min(plan->nd, m0 + chunk));
  const int cnt = m1 - m0;  // 0 .. chunk <= kChunk

  // The chunk's constants and primes, staged once per workgroup: read from
  // global memory inside the destination loop they would make every
  // iteration wait for a load.
  __shared__ uint64_t cst[kChunk][NS];
  __shared__ uint32_t cst2[kChunk][NS][2];
  __shared__ uint64_t qd[kChunk][2];
  const int tid = (int)threadIdx.x;
  for (int e = tid; e < cnt * NS; e += kThreads) {
    const int mm = e / NS, j = e % NS;
    cst[mm][j] = plan->hmod[m0 + mm][j];
    cst2[mm][j][0] = plan->hk[m0 + mm][j][0];
    cst2[mm][j][1] = plan->hk[m0 + mm][j][1];
  }
  for (int e = tid; e < cnt; e += kThreads) {
    const PrimeDev& pd = primes[plan->dst[m0 + e]];
    qd[e][0] = pd.q;
    qd[e][1] = pd.qinv_neg;
  }
  __syncthreads();

  // An item with fewer source limbs than the launch's NS (a digit group
  // shorter than alpha) has zeros in the remaining places: every product
  // with them vanishes.
  const int nsi = plan->ns;
  auto yj = [&](int j) -> uint64_t {
    return j < nsi ? shoup(src[(size_t)j * n + p], plan->hinv[j], plan->hinv_sh[j], primes[plan->src[j]].q) : 0;
  };
  if constexpr (S30) {
    // all primes below 2^60: the inner product from 30-bit column sums
    uint32_t y0[NS], y1[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const uint64_t v = yj(j);
      y0[j] = (uint32_t)(v & ((1ull << 30) - 1));
      y1[j] = (uint32_t)(v >> 30);
    }
    for (int m = m0; m < m1; ++m) {
      const int di = plan->dst[m];
      const size_t o = (size_t)(di - shift) * n + p;
      const uint64_t q = qd[m - m0][0];
      uint64_t v = redc(dot_split30<NS>(y0, y1, cst2[m - m0]), q, qd[m - m0][1]);
      if (aux) v = shoup(aux[o] - v + q, plan->sinv[m], plan->sinv_sh[m], q);
      dst[o] = v;
    }
    return;
  }
  uint64_t y[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) y[j] = yj(j);
  for (int m = m0; m < m1; ++m) {
    const int di = plan->dst[m];
    const size_t o = (size_t)(di - shift) * n + p;
    const uint64_t q = qd[m - m0][0], qn = qd[m - m0][1];
    const uint64_t* c = cst[m - m0];
    U128 acc = mul_wide(y[0], c[0]);
#pragma unroll
    for (int j = 1; j < NS; ++j) add128(acc, mul_wide(y[j], c[j]));
    uint64_t v = redc(acc, q, qn);
    if (aux) v = shoup(aux[o] - v + q, plan->sinv[m], plan->sinv_sh[m], q);
    dst[o] = v;
  }
}

template <int NS>
hipError_t launch_ns(const ckks_params* P, const BConvArgs& a, int items, hipStream_t s) {
  // Destination chunks: at most kChunk limbs each; a launch with few
  // workgroups (few conversions) is split further, down to kMinChunk limbs
  // per chunk, until it has about kMinWgs (each chunk converts its sources
  // again, a small cost against the destinations' inner products).
  const int wgs = P->n / kThreads * items;
  int nch = (a.max_nd + kChunk - 1) / kChunk;
  nch = std::max(nch, std::min((kMinWgs + wgs - 1) / wgs, (a.max_nd + kMinChunk - 1) / kMinChunk));
  const int chunk = (a.max_nd + nch - 1) / nch;
  nch = (a.max_nd + chunk - 1) / chunk;
  dim3 grid(P->n / kThreads, items, nch);
  bool s30 = true;
  for (int i = 0; i < items; ++i) s30 = s30 && P->plan_is_split30(a.plan[i]);
  if (s30)
    hipLaunchKernelGGL((bconv_kernel<NS, true>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, chunk);
  else
    hipLaunchKernelGGL((bconv_kernel<NS, false>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n, chunk);
  return hipGetLastError();
}

}  // namespace

// Every item of one launch has at most `ns` source limbs (the kernel's
// unrolled count; shorter items are padded with zeros).
hipError_t launch_bconv(const ckks_params* P, const BConvArgs& a, int items, int ns, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  // Launch geometry, checked on the host before anything runs: every item's
  // plan converts from 1 .. ns limbs into at most max_nd <= kMaxDst limbs
  // (so each workgroup's chunk [m0, m1) lies inside the plan and the grid
  // covers every destination), its buffers are set and the position grid
  // covers N exactly.
  if (items > kMaxConv || a.max_nd < 1 || a.max_nd > kMaxDst || P->n % kThreads) return hipErrorInvalidValue;
  for (int i = 0; i < items; ++i) {
    const std::pair<int, int> d = P->plan_dims(a.plan[i]);
    if (d.first < 1 || d.first > ns || d.second < 1 || d.second > a.max_nd || !a.src[i] || !a.dst[i])
      return hipErrorInvalidValue;
  }
  ProfScope prof(CKKS_KERNEL_BCONV, s, (double)a.limbs_moved * P->n * 8);
  switch (ns) {
    case 1: return launch_ns<1>(P, a, items, s);
    case 2: return launch_ns<2>(P, a, items, s);
    case 3: return launch_ns<3>(P, a, items, s);
    case 4: return launch_ns<4>(P, a, items, s);
    case 5: return launch_ns<5>(P, a, items, s);
    case 6: return launch_ns<6>(P, a, items, s);
    case 7: return launch_ns<7>(P, a, items, s);
    case 8: return launch_ns<8>(P, a, items, s);
    case 9: return launch_ns<9>(P, a, items, s);
    case 10: return launch_ns<10>(P, a, items, s);
    case 11: return launch_ns<11>(P, a, items, s);
    case 12: return launch_ns<12>(P, a, items, s);
    case 13: return launch_ns<13>(P, a, items, s);
    case 14: return launch_ns<14>(P, a, items, s);
    case 15: return launch_ns<15>(P, a, items, s);
    case 16: return launch_ns<16>(P, a, items, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ckks
