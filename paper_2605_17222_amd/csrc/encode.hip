// Plaintext encoding on the device (Section II-A): the integer polynomial
// m = round(scale * sigma^-1(z)) of a vector z of N/2 complex slots (the
// forward NTT then reduces m into each prime as its first pass reads it).
//
// Slot t is m(zeta^(5^t)), zeta = e^(i pi / N).  With e_t = 5^t mod 2N = 4 j_t + 1
// (5^t is 1 mod 4, and t -> j_t permutes [0, N/2)) and u_k = m_k + i m_(k+N/2),
//   z_t = sum_(k < N/2) u_k zeta^k e^(2 pi i j_t k / (N/2)),
// so with z'_(j_t) = z_t the inverse is one length-S = N/2 DFT:
//   u_k = zeta^-k / S * sum_j z'_j e^(-2 pi i j k / S).
// The DFT runs as two passes over S = A B (four-step FFT): j = B j1 + j2,
// k = k1 + A k2; pass 1 transforms each column j2 over j1 (length A) and
// multiplies by w^(j2 k1) (w = e^(-2 pi i / S)); pass 2 transforms each row k1
// over j2 (length B).  Each sub-transform is an in-place radix-2 FFT in LDS.
// Rounding is half away from zero.
#include "internal.hpp"
#include "modarith.hpp"

namespace ckks {

namespace {

struct Cx {
  double re, im;
};

__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx ld(const double* p) { return {p[0], p[1]}; }

__device__ __forceinline__ uint32_t brev_bits(uint32_t x, int bits) { return __brev(x) >> (32 - bits); }

// Radix-2 decimation-in-time FFT of P points held in LDS in bit-reversed
// order; on return L holds the DFT in natural order.  Each of the P/2 lanes of
// a sub-transform does one butterfly per stage.
template <int LOGP>
__device__ __forceinline__ void lds_fft(Cx* L, int lane, const double* __restrict__ tw, int log_s) {
  constexpr int P = 1 << LOGP;
  // A lane reads and writes only its own pair within a stage.
#pragma unroll
  for (int s = 1; s <= LOGP; ++s) {
    const int half = 1 << (s - 1);
    const int pos = lane & (half - 1);
    const int i0 = ((lane >> (s - 1)) << s) + pos, i1 = i0 + half;
    // e^(-2 pi i pos / 2^s) = w^(pos S / 2^s)
    const Cx w = ld(tw + 2 * ((size_t)pos << (log_s - s)));
    const Cx x0 = L[i0], x1 = cmul(L[i1], w);
    L[i0] = {x0.re + x1.re, x0.im + x1.im};
    L[i1] = {x0.re - x1.re, x0.im - x1.im};
    __syncthreads();
  }
  (void)P;
}

// Pass 1: block (x, y) transforms columns j2 = x G + g of item y.
template <int LOGA, int LOGB>
__global__ void __launch_bounds__(256) enc_pass1(EncArgs a, const int* __restrict__ perm,
                                                 const double* __restrict__ tw, int log_s) {
  constexpr int A = 1 << LOGA, B = 1 << LOGB;
  constexpr int G = 512 / A;  // columns per workgroup
  __shared__ Cx lds[G][A];
  const int it = blockIdx.y;
  const int S = 1 << log_s;
  const int lane = threadIdx.x % (A / 2), g = threadIdx.x / (A / 2);
  const int j2 = blockIdx.x * G + g;
  const double* __restrict__ z = a.z[it];
  const int rot = a.rot[it];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j1 = lane + h * (A / 2);
    const int t = perm[B * j1 + j2];
    lds[g][brev_bits((uint32_t)j1, LOGA)] = ld(z + 2 * (size_t)((t + rot) & (S - 1)));
  }
  __syncthreads();
  lds_fft<LOGA>(lds[g], lane, tw, log_s);
  double* __restrict__ y = a.y[it];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k1 = lane + h * (A / 2);
    const Cx v = cmul(lds[g][k1], ld(tw + 2 * (size_t)((j2 * k1) & (S - 1))));
    y[2 * ((size_t)k1 * B + j2)] = v.re;
    y[2 * ((size_t)k1 * B + j2) + 1] = v.im;
  }
}

// Pass 2: block (x, y) transforms rows k1 = x G + g of item y, then forms
// u_k = zeta^-k / S * U_k and the rounded coefficients m_k, m_(k+S).
template <int LOGA, int LOGB>
__global__ void __launch_bounds__(256) enc_pass2(EncArgs a, const double* __restrict__ tw,
                                                 const double* __restrict__ zinv, int log_s) {
  constexpr int A = 1 << LOGA, B = 1 << LOGB;
  constexpr int G = 512 / B;  // rows per workgroup
  __shared__ Cx lds[G][B];
  const int it = blockIdx.y;
  const int S = 1 << log_s;
  const int lane = threadIdx.x % (B / 2), g = threadIdx.x / (B / 2);
  const int k1 = blockIdx.x * G + g;
  const double* __restrict__ y = a.y[it];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j2 = lane + h * (B / 2);
    lds[g][brev_bits((uint32_t)j2, LOGB)] = ld(y + 2 * ((size_t)k1 * B + j2));
  }
  __syncthreads();
  lds_fft<LOGB>(lds[g], lane, tw, log_s);
  const double scale = a.scale[it];
  int64_t* __restrict__ coef = a.coef[it];
  // |scale u| beyond 2^62 is outside the documented range; clamp so the
  // conversion stays defined.
  constexpr double kLim = 4611686018427387904.0;  // 2^62
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k2 = lane + h * (B / 2);
    const int k = k1 + A * k2;
    const Cx u = cmul(lds[g][k2], ld(zinv + 2 * (size_t)k));
    const double mr = fmin(fmax(round(scale * u.re), -kLim), kLim);
    const double mi = fmin(fmax(round(scale * u.im), -kLim), kLim);
    coef[k] = (int64_t)mr;
    coef[k + S] = (int64_t)mi;
  }
}

template <int LOGA, int LOGB>
hipError_t launch_enc(const ckks_params* P, const EncArgs& a, hipStream_t s) {
  constexpr int A = 1 << LOGA, B = 1 << LOGB;
  const int log_s = P->log_n - 1;
  if (LOGA + LOGB != log_s) return hipErrorInvalidValue;
  {
    ProfScope prof(CKKS_KERNEL_ENCODE_FFT, s, (double)a.count * (P->n * 8.0) * 2);
    hipLaunchKernelGGL((enc_pass1<LOGA, LOGB>), dim3(B / (512 / A), a.count), dim3(256), 0, s, a, P->d_enc_perm,
                       P->d_enc_tw, log_s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  ProfScope prof(CKKS_KERNEL_ENCODE_FFT, s, (double)a.count * (P->n * 8.0) * 2);
  hipLaunchKernelGGL((enc_pass2<LOGA, LOGB>), dim3(A / (512 / B), a.count), dim3(256), 0, s, a, P->d_enc_tw,
                     P->d_enc_zinv, log_s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_encode_fft(const ckks_params* P, const EncArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  switch (P->log_n) {
    case 12: return launch_enc<6, 5>(P, a, s);
    case 13: return launch_enc<6, 6>(P, a, s);
    case 14: return launch_enc<7, 6>(P, a, s);
    case 15: return launch_enc<7, 7>(P, a, s);
    case 16: return launch_enc<8, 7>(P, a, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {

// Block (x, l, c): positions x*256.. of limb l of polynomial c.
__global__ void __launch_bounds__(256)
    pack_kernel(const uint64_t* __restrict__ in, uint8_t* __restrict__ out, const PrimeDev* __restrict__ primes,
                int kmax, int log_n, uint64_t poly_bytes) {
  const size_t n = (size_t)1 << log_n;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int l = blockIdx.y;
  const size_t c = blockIdx.z;
  const PrimeDev& pr = primes[l];
  const uint64_t v = in[(c * kmax + l) * n + p];
  uint8_t* b = out + c * poly_bytes + pr.pk_off;
  if (pr.narrow) {
    uint8_t* c = b + (p / kPackChunk) * (5 * kPackChunk);
    reinterpret_cast<uint32_t*>(c)[p % kPackChunk] = (uint32_t)v;
    c[4 * kPackChunk + p % kPackChunk] = (uint8_t)(v >> 32);
  } else {
    reinterpret_cast<uint64_t*>(b)[p] = v;
  }
}

}  // namespace

hipError_t launch_pack(const ckks_params* P, int count, const uint64_t* in, uint8_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3(P->n / 256, P->Kmax(), count), dim3(256), 0, s, in, out, P->d_primes,
                     P->Kmax(), P->log_n, P->pk_poly_bytes);
  return hipGetLastError();
}

}  // namespace ckks
