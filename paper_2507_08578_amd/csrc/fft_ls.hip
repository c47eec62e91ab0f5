// FP32 plane kernel for square boxes N1 = N2 = P^2 whose 1D transforms trade
// data through LDS instead of cross-lane shuffles ("four-step" split
// N = P x P).  One transform is held by P lanes of a wavefront:
//   step 1: lane b holds x[P a + b] (a < P), a P-point DFT in registers over
//           a, the twiddle w_N^(b k1), and a write back transposed,
//   step 2: lane k1 reads the P values of row k1, a second P-point DFT,
//           outputs X[k1 + P k2] in natural order.
// Step 1 of a forward transform takes exactly the layout step 2 of a
// backward one leaves, so a row goes backward, x V/N_box, forward without
// leaving the registers except for the two exchanges.  The N2 transforms of
// the extent columns run in place in the plane's extent array E (the
// positions a lane writes in step 1 are the ones it read); the N1 rows use
// a per-group exchange buffer.  Lanes of one group always sit in one
// wavefront, whose LDS operations execute in order, so the exchanges need
// only a compiler-level wavefront fence.
#include "fft_common.h"

using namespace pwfft;

namespace {

constexpr int kLsWaves = 10;
constexpr int kLsThreads = kLsWaves * 64;

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v[k] *= w_N^(S b k), k = 1..P-1, with w[k-1] = exp(-2 pi i b k / N)
template <int P, int S>
__device__ __forceinline__ void ls_twiddle(float2 (&v)[P], const float2 (&w)[P - 1]) {
#pragma unroll
  for (int k = 1; k < P; ++k) v[k] = S > 0 ? conj_mul(v[k], w[k - 1]) : cmul(v[k], w[k - 1]);
}

// In-place transform (sign S) of the length-P^2 sequence seq[0 .. P^2) in LDS
// by the P lanes of a group (lane lb): natural order in, natural order out.
template <int P, int S>
__device__ __forceinline__ void ls_fft_inplace(float2* seq, int lb, const float2 (&w)[P - 1]) {
  float2 v[P];
#pragma unroll
  for (int a = 0; a < P; ++a) v[a] = seq[P * a + lb];
  dft_reg<P, S>(v);
  ls_twiddle<P, S>(v, w);
#pragma unroll
  for (int k = 0; k < P; ++k) seq[P * k + lb] = v[k];
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < P; ++b) v[b] = seq[P * lb + b];
  dft_reg<P, S>(v);
  wave_lds_fence();
#pragma unroll
  for (int k = 0; k < P; ++k) seq[lb + P * k] = v[k];
  wave_lds_fence();
}

// Transform (sign S) of the sequence whose element P a + lb sits in v[a] of
// lane lb; the exchange goes through buf (P^2 entries).  Result: v[k] holds
// element lb + P k.
template <int P, int S>
__device__ __forceinline__ void ls_fft_regs(float2 (&v)[P], float2* buf, int lb,
                                            const float2 (&w)[P - 1]) {
  dft_reg<P, S>(v);
  ls_twiddle<P, S>(v, w);
#pragma unroll
  for (int k = 0; k < P; ++k) buf[P * k + lb] = v[k];
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < P; ++b) v[b] = buf[P * lb + b];
  dft_reg<P, S>(v);
  wave_lds_fence();
}

template <int P>
__device__ __forceinline__ void plane_ls_body(const BoxPlan& Pl, const float2* __restrict__ tw,
                                              const float* __restrict__ vs, float2* __restrict__ T,
                                              int j3, int b) {
  constexpr int N = P * P, TRS = N + 1, GPW = 64 / P;
  extern __shared__ __align__(16) char lds_raw[];
  float2* E = reinterpret_cast<float2*>(lds_raw);                      // xr x TRS
  float2* X = E + (size_t)Pl.xr * TRS;                                 // groups x N
  int* slot = reinterpret_cast<int*>(X + (size_t)kLsWaves * GPW * N);  // N
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, lw = tid & 63;
  const int gw = lw / P, lb = lw - gw * P;
  const bool act = gw < GPW;
  const int grp = wave * GPW + gw, ngr = (nt >> 6) * GPW;
  float2* tp = T + (size_t)b * Pl.n3 * Pl.ncols + (size_t)j3 * Pl.ncols;
  for (int i = tid; i < Pl.xr * TRS; i += nt) E[i] = czero<float2>();
  for (int i = tid; i < N; i += nt) slot[i] = -1;
  __syncthreads();
  for (int e = tid; e < Pl.xr; e += nt) slot[Pl.ext_m1[e]] = e;
  for (int c = tid; c < Pl.ncols; c += nt) E[Pl.col_e[c] * TRS + Pl.col_m2[c]] = tp[c];
  __syncthreads();
  float2 w[P - 1];
#pragma unroll
  for (int k = 1; k < P; ++k) w[k - 1] = tw[(lb * k) % N];
  // backward along N2 on every extent column
  if (act)
    for (int e = grp; e < Pl.xr; e += ngr) ls_fft_inplace<P, +1>(E + e * TRS, lb, w);
  __syncthreads();
  // rows: backward along N1, x V/N_box, forward along N1
  if (act) {
    int sl[P];   // extent slot of positions P a + lb (the same set on output: lb + P k)
#pragma unroll
    for (int a = 0; a < P; ++a) sl[a] = slot[P * a + lb];
    float2* buf = X + (size_t)grp * N;
    const float* vp = vs + (size_t)j3 * N * N;
    for (int row = grp; row < N; row += ngr) {
      float2 v[P];
#pragma unroll
      for (int a = 0; a < P; ++a) v[a] = sl[a] >= 0 ? E[sl[a] * TRS + row] : czero<float2>();
      ls_fft_regs<P, +1>(v, buf, lb, w);
      const float* vr = vp + (size_t)row * N + lb;
#pragma unroll
      for (int k = 0; k < P; ++k) v[k] = cscale(v[k], vr[P * k]);
      ls_fft_regs<P, -1>(v, buf, lb, w);
      // v[k] holds position lb + P k: slot sl[k]
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (sl[k] >= 0) E[sl[k] * TRS + row] = v[k];
    }
  }
  __syncthreads();
  // forward along N2
  if (act)
    for (int e = grp; e < Pl.xr; e += ngr) ls_fft_inplace<P, -1>(E + e * TRS, lb, w);
  __syncthreads();
  for (int c = tid; c < Pl.ncols; c += nt) tp[c] = E[Pl.col_e[c] * TRS + Pl.col_m2[c]];
}

template <int P>
__global__ void __launch_bounds__(kLsThreads)
k_plane_ls(BoxPlan Pl, const float2* __restrict__ tw, const float* __restrict__ vs,
           float2* __restrict__ T) {
  plane_ls_body<P>(Pl, tw, vs, T, blockIdx.x, blockIdx.y);
}

constexpr int kLsP = 12;   // N1 = N2 = 144

}  // namespace

size_t fft_plane_ls_lds(const BoxPlan& p) {
  constexpr int N = kLsP * kLsP, GPW = 64 / kLsP;
  return (size_t)p.xr * (N + 1) * sizeof(float2) + (size_t)kLsWaves * GPW * N * sizeof(float2) +
         (size_t)N * sizeof(int);
}

bool fft_plane_ls_supported(const BoxPlan& p, size_t lds_limit) {
  return p.n1 == kLsP * kLsP && p.n2 == kLsP * kLsP && fft_plane_ls_lds(p) <= lds_limit;
}

hipError_t launch_fft_plane_ls32(const BoxPlan& p, int nb, const float* vscaled, float2* T,
                                 hipStream_t s) {
  if (p.n1 != kLsP * kLsP || p.n2 != p.n1 || p.ax1.tw32 == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plane_ls<kLsP>, dim3(p.n3, nb), dim3(kLsThreads), fft_plane_ls_lds(p), s, p,
                     p.ax1.tw32, vscaled, T);
  return hipGetLastError();
}

hipError_t fft_ls_set_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_plane_ls<kLsP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
