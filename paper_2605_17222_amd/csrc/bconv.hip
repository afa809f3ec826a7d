// Basis conversion, eq. (3), fused with the column stages of the transforms
// around it.
//
//   y_j   = [(S/s_j)^-1 x_j]_{s_j}               (x_j: coefficients of source limb j)
//   out_m = sum_j y_j [S/s_j]_{d_m}  mod d_m      (each destination limb m)
//
// The conversion needs every source limb of a coefficient (the type-II
// dependency of Section IV), the NTT needs a whole limb (type I).  With the
// transforms split as 16 columns-stages x row stages (ntt.hip), a workgroup
// owns a tile of 64 columns x 16 rows = 1024 coefficient positions, which is
// closed under both the column stages and the conversion:
//   1. for each source limb: load the tile of its inverse row-pass output,
//      run the inverse transform's 4 column stages, and fold N^-1 into the
//      factor (S/s_j)^-1 (one Shoup product): y_j, kept in registers;
//   2. for each destination limb of the workgroup's chunk: the inner product
//      of eq. (3), the forward transform's 4 column stages, store (its row
//      pass follows as a separate launch).
// So a Decompose or ModDown reads the source limbs once and writes each
// destination limb once between its two row passes, instead of three HBM
// round trips (inverse column pass, conversion, forward column pass).
//
// Thread t of the workgroup holds column 64 blockIdx.x + t/4, rows
// 4 (t % 4) + u, u = 0..3: the four threads of a column are one quad of lanes,
// so the two column stages that cross threads exchange operands with DPP quad
// permutations (lane xor 1, lane xor 2); the other two stay in registers.
//
// The inner product: constants [S/s_j]_{d_m} are stored times 2^64 mod d_m, so
// one Montgomery REDC of the exact 128-bit sum gives the canonical result
// (sum_j s_j <= 2^64, checked at parameter creation).  When every prime is
// below 2^60 the sum is formed from four 30-bit column sums without carries
// (dot_split30).  The number of source limbs is a template parameter, so the
// source registers are indexed statically.  Several conversions (the digits
// of Decompose, many ciphertexts) run in one launch, one per blockIdx.y;
// blockIdx.z splits the destination limbs into chunks (each chunk redoes
// step 1) so that small launches still fill the device.
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

constexpr int kThreads = 256;
constexpr int kTileCols = kThreads / 4;  // columns per workgroup
constexpr int kChunkMax = 32;            // destination limbs per workgroup at most

__device__ __forceinline__ double as_d(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ uint64_t as_u(double d) { return (uint64_t)__double_as_longlong(d); }

// The value of the lane whose quad index is this lane's xor M (M = 1 or 2).
template <int M>
__device__ __forceinline__ uint64_t quad_xor(uint64_t x) {
  constexpr int ctrl = M == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)x, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), ctrl, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int NS>
__global__ void __launch_bounds__(kThreads)
    bconv_kernel(BConvArgs a, const PrimeDev* __restrict__ primes, int log_n) {
  const int item = blockIdx.y;
  const BConvPlan* __restrict__ plan = a.plan[item];
  const int nd = plan->nd;
  const int m0 = blockIdx.z * a.chunk;
  const int cnt = min(nd, m0 + a.chunk) - m0;  // uniform over the workgroup
  if (cnt <= 0) return;                        // this item has fewer destination limbs
  const uint64_t* __restrict__ src = a.src[item];
  uint64_t* __restrict__ dst = a.dst[item];
  const int shift = a.dst_shift[item];
  const size_t n = (size_t)1 << log_n, n2 = n >> kColLog;
  const int tid = (int)threadIdx.x;
  const int qi4 = tid & 3;  // quad index: rows 4 qi4 .. 4 qi4 + 3
  const size_t col = (size_t)blockIdx.x * kTileCols + (tid >> 2);
  // Byte offsets of the thread's four positions within a limb (below 2^32):
  // a uniform limb base plus a 32-bit offset, so no 64-bit address registers.
  uint32_t bo[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) bo[u] = (uint32_t)((col + n2 * (size_t)(4 * qi4 + u)) * 8);
  auto at = [&](const uint64_t* base, int u) {
    return reinterpret_cast<uint64_t*>(const_cast<char*>(reinterpret_cast<const char*>(base)) + bo[u]);
  };

  // Constants staged once per workgroup (read from global memory where they
  // are used, the loads would be hoisted and held in registers): for each
  // source its prime, N^-1 (S/s_j)^-1 and the inverse column twiddles; for
  // each destination of the chunk the inner-product constants, its prime and
  // Montgomery word, and the forward column twiddles (value, Shoup word).
  __shared__ uint64_t stw[NS][2][16];
  __shared__ uint64_t sc[NS][4];  // q, hinvn, hinvn_sh, fp
  __shared__ double sd[NS][2];    // q, 1/q as doubles
  __shared__ uint32_t hk[kChunkMax][NS][2];
  __shared__ uint64_t dq[kChunkMax][2];
  __shared__ uint64_t dtw[kChunkMax][2][16];
  __shared__ int dfp[kChunkMax];
  for (int e = tid; e < NS * 32; e += kThreads) {
    const int j = e / 32, k = e % 32;
    stw[j][k / 16][k % 16] = primes[plan->src[j]].ctw[1][k / 16][k % 16];
  }
  for (int j = tid; j < NS; j += kThreads) {
    const PrimeDev& ps = primes[plan->src[j]];
    sc[j][0] = ps.q;
    sc[j][1] = plan->hinvn[j];
    sc[j][2] = plan->hinvn_sh[j];
    sc[j][3] = (uint64_t)ps.fp;
    sd[j][0] = ps.qd;
    sd[j][1] = ps.qinv_d;
  }
  for (int e = tid; e < cnt * NS; e += kThreads) {
    const int mm = e / NS, j = e % NS;
    hk[mm][j][0] = plan->hk[m0 + mm][j][0];
    hk[mm][j][1] = plan->hk[m0 + mm][j][1];
  }
  for (int e = tid; e < cnt * 32; e += kThreads) {
    const int mm = e / 32, k = e % 32;
    dtw[mm][k / 16][k % 16] = primes[plan->dst[m0 + mm]].ctw[0][k / 16][k % 16];
  }
  for (int e = tid; e < cnt; e += kThreads) {
    const PrimeDev& pd = primes[plan->dst[m0 + e]];
    dq[e][0] = pd.q;
    dq[e][1] = pd.qinv_neg;
    dfp[e] = pd.fp;
  }
  __syncthreads();

  // Step 1: the sources' inverse column stages and y_j = (S/s_j)^-1 N^-1 x_j.
  const bool lo1 = !(qi4 & 1), lo2 = !(qi4 & 2);  // lower row of the cross-thread pairs
  uint32_t y0[NS][4], y1[NS][4];
#pragma clang loop unroll(full)
  for (int j = 0; j < NS; ++j) {
    const uint64_t q = sc[j][0], q2 = 2 * q;
    const uint64_t* __restrict__ sj = src + (size_t)j * n;
    uint64_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(at(sj, u));
    if (sc[j][3]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = fp_canon(as_d(v[u]), sd[j][0], sd[j][1]);
    }
    const uint64_t* tw = stw[j][0];
    const uint64_t* tp = stw[j][1];
    // Gentleman-Sande stages 3, 2 (rows r, r + 1 and r, r + 2: in registers)
#pragma unroll
    for (int u = 0; u < 4; u += 2) {
      const int ti = 8 + 2 * qi4 + (u >> 1);
      const uint64_t X = v[u], Y = v[u + 1];
      uint64_t sm = X + Y;
      sm = sm >= q2 ? sm - q2 : sm;
      v[u] = sm;
      v[u + 1] = shoup_lazy(X - Y + q2, tw[ti], tp[ti], q);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int ti = 4 + qi4;
      const uint64_t X = v[u], Y = v[u + 2];
      uint64_t sm = X + Y;
      sm = sm >= q2 ? sm - q2 : sm;
      v[u] = sm;
      v[u + 2] = shoup_lazy(X - Y + q2, tw[ti], tp[ti], q);
    }
    // stages 1 and 0 (rows r, r + 4: quad xor 1; r, r + 8: quad xor 2): each
    // lane forms its own output of the butterfly from both operands
    {
      const int ti = 2 + (qi4 >> 1);
      const uint64_t w = tw[ti], wp = tp[ti];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t o = v[u], p = quad_xor<1>(o);
        const uint64_t X = lo1 ? o : p, Y = lo1 ? p : o;
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        const uint64_t df = shoup_lazy(X - Y + q2, w, wp, q);
        v[u] = lo1 ? sm : df;
      }
    }
    {
      const uint64_t w = tw[1], wp = tp[1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t o = v[u], p = quad_xor<2>(o);
        const uint64_t X = lo2 ? o : p, Y = lo2 ? p : o;
        uint64_t sm = X + Y;
        sm = sm >= q2 ? sm - q2 : sm;
        const uint64_t df = shoup_lazy(X - Y + q2, w, wp, q);
        v[u] = lo2 ? sm : df;
      }
    }
    const uint64_t h = sc[j][1], hs = sc[j][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t y = shoup(v[u], h, hs, q);
      y0[j][u] = (uint32_t)(y & ((1ull << 30) - 1));
      y1[j][u] = (uint32_t)(y >> 30);
      // materialise y here: otherwise its computation sinks to the uses and
      // every source's operands and constants stay live until then
      asm volatile("" : "+v"(y0[j][u]), "+v"(y1[j][u]));
    }
  }

  // Step 2: every destination of the chunk.
  const bool split30 = plan->split30 != 0;
#pragma unroll 1
  for (int mm = 0; mm < cnt; ++mm) {
    // y is re-read here each iteration as far as the compiler knows, so
    // nothing derived from it (widened copies) is hoisted out of the loop
    // and held in extra registers
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int u = 0; u < 4; ++u) asm volatile("" : "+v"(y0[j][u]), "+v"(y1[j][u]));
    const uint64_t q = dq[mm][0], qn = dq[mm][1], q2 = 2 * q;
    uint64_t v[4];
    if (split30) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        uint32_t a0[NS], a1[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          a0[j] = y0[j][u];
          a1[j] = y1[j][u];
        }
        v[u] = redc(dot_split30<NS>(a0, a1, hk[mm]), q, qn);
      }
    } else {
      const uint64_t* hm = plan->hmod[m0 + mm];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        U128 acc = {0, 0};
#pragma unroll
        for (int j = 0; j < NS; ++j) add128(acc, mul_wide(((uint64_t)y1[j][u] << 30) | y0[j][u], hm[j]));
        v[u] = redc(acc, q, qn);
      }
    }
    const uint64_t* tw = dtw[mm][0];
    const uint64_t* tp = dtw[mm][1];
    // Cooley-Tukey stages 0 and 1 (cross-thread), then 2 and 3 (in registers)
    {
      const uint64_t w = tw[1], wp = tp[1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t o = v[u], p = quad_xor<2>(o);
        uint64_t X = lo2 ? o : p;
        const uint64_t Y = lo2 ? p : o;
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(Y, w, wp, q);
        v[u] = lo2 ? X + t : X - t + q2;
      }
    }
    {
      const int ti = 2 + (qi4 >> 1);
      const uint64_t w = tw[ti], wp = tp[ti];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t o = v[u], p = quad_xor<1>(o);
        uint64_t X = lo1 ? o : p;
        const uint64_t Y = lo1 ? p : o;
        X = X >= q2 ? X - q2 : X;
        const uint64_t t = shoup_lazy(Y, w, wp, q);
        v[u] = lo1 ? X + t : X - t + q2;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int ti = 4 + qi4;
      uint64_t X = v[u];
      X = X >= q2 ? X - q2 : X;
      const uint64_t t = shoup_lazy(v[u + 2], tw[ti], tp[ti], q);
      v[u] = X + t;
      v[u + 2] = X - t + q2;
    }
#pragma unroll
    for (int u = 0; u < 4; u += 2) {
      const int ti = 8 + 2 * qi4 + (u >> 1);
      uint64_t X = v[u];
      X = X >= q2 ? X - q2 : X;
      const uint64_t t = shoup_lazy(v[u + 1], tw[ti], tp[ti], q);
      v[u] = X + t;
      v[u + 1] = X - t + q2;
    }
    uint64_t* __restrict__ dm = dst + (size_t)(plan->dst[m0 + mm] - shift) * n;
    if (dfp[mm]) {
      // the FP64 row pass takes canonical residues as doubles
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        uint64_t x = v[u] >= q2 ? v[u] - q2 : v[u];
        *at(dm, u) = as_u(u64_to_d(csub(x, q)));
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) *at(dm, u) = v[u];
    }
  }
}

template <int NS>
hipError_t launch_ns(const ckks_params* P, const BConvArgs& a, int items, hipStream_t s) {
  dim3 grid((P->n >> kColLog) / kTileCols, items, (a.max_nd + a.chunk - 1) / a.chunk);
  hipLaunchKernelGGL((bconv_kernel<NS>), grid, dim3(kThreads), 0, s, a, P->d_primes, P->log_n);
  return hipGetLastError();
}

}  // namespace

int bconv_chunk_max() { return kChunkMax; }

// All items of one launch have the same number of source limbs `ns`.
hipError_t launch_bconv(const ckks_params* P, const BConvArgs& a, int items, int ns, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  // Launch geometry, checked on the host before anything runs: every item's
  // plan converts from exactly ns limbs into at most max_nd <= kMaxDst limbs,
  // the chunk fits the staged constants, its buffers are set, and the
  // position tiles cover the N/16 columns exactly.
  if (items > kMaxConv || a.max_nd < 1 || a.max_nd > kMaxDst || a.chunk < 1 || a.chunk > kChunkMax ||
      (P->n >> kColLog) % kTileCols)
    return hipErrorInvalidValue;
  for (int i = 0; i < items; ++i) {
    const std::pair<int, int> d = P->plan_dims(a.plan[i]);
    if (d.first != ns || d.second < 1 || d.second > a.max_nd || !a.src[i] || !a.dst[i]) return hipErrorInvalidValue;
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
