// Basis conversion, eq. (3):  y_j = [(S/s_j)^-1 x_j]_{s_j},
//                             out_m = sum_j y_j [S/s_j]_{d_m} mod d_m.
// Coefficient-domain limbs; one thread per coefficient position, all source
// limbs of that position in registers (the type-II dependency of Section IV:
// every limb of a coefficient is needed).  The constants [S/s_j]_{d_m} are
// stored times 2^64 mod d_m, so one Montgomery REDC of the 128-bit sum gives
// the canonical result; this needs sum_j s_j <= 2^64, which parameter
// creation checks.  Several conversions (the digits of Decompose) run in one
// launch, one per blockIdx.y.
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads)
    bconv_kernel(BConvArgs a, const PrimeDev* __restrict__ primes, int log_n) {
  const int item = blockIdx.y;
  const BConvPlan* __restrict__ plan = a.plan[item];
  const uint64_t* __restrict__ src = a.src[item];
  uint64_t* __restrict__ dst = a.dst[item];
  const int shift = a.dst_shift[item];
  const size_t n = (size_t)1 << log_n;
  const size_t p = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int ns = plan->ns, nd = plan->nd;

  uint64_t y[kMaxSrc];
#pragma unroll
  for (int j = 0; j < kMaxSrc; ++j) {
    if (j < ns) {
      const PrimeDev& ps = primes[plan->src[j]];
      y[j] = shoup(src[(size_t)j * n + p], plan->hinv[j], plan->hinv_sh[j], ps.q);
    }
  }
  for (int m = 0; m < nd; ++m) {
    const int di = plan->dst[m];
    const uint64_t q = primes[di].q, qn = primes[di].qinv_neg;
    U128 acc = {0, 0};
#pragma unroll
    for (int j = 0; j < kMaxSrc; ++j)
      if (j < ns) add128(acc, mul_wide(y[j], plan->hmod[m][j]));
    dst[(size_t)(di - shift) * n + p] = redc(acc, q, qn);
  }
}

}  // namespace

hipError_t launch_bconv(const ckks_params* P, const BConvArgs& a, int items, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  dim3 grid(P->n / kThreads, items);
  ProfScope prof(CKKS_KERNEL_BCONV, s, (double)a.limbs_moved * P->n * 8);
  hipLaunchKernelGGL(bconv_kernel, grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n);
  return hipGetLastError();
}

}  // namespace ckks
