// FP32 plane kernel for square boxes N1 = N2 = P^2 whose 1D transforms trade
// data through LDS instead of cross-lane shuffles ("four-step" split
// N = P x P).  One transform is held by P lanes of a wavefront:
//   step 1: lane b holds x[P a + b] (a < P), a P-point DFT in registers over
//           a, the twiddle w_N^(b k1), and a write back transposed,
//   step 2: lane k1 reads the P values of row k1, a second P-point DFT,
//           outputs X[k1 + P k2] in natural order.
// Step 1 of a forward transform takes exactly the layout step 2 of a
// backward one leaves, so a row goes backward, x V/N_box, forward without
// leaving the registers except for the two exchanges.  Every exchange goes
// through a per-group buffer whose rows are padded so that the step-2 reads
// fall in distinct banks; the N2 transforms of the extent columns read and
// write the plane's extent array E in natural order.  Lanes of one group always sit in one
// wavefront, whose LDS operations execute in order, so the exchanges need
// only a compiler-level wavefront fence.
#include "fft_common.h"

#include <algorithm>

using namespace pwfft;

namespace {

// Up to 16 wavefronts per workgroup; the launch takes as many as the LDS
// budget leaves room for after the extent array (each wavefront adds the
// exchange buffers of its 64 / P groups).
constexpr int kLsMaxWaves = 16;
constexpr int kLsMinWaves = 4;

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

// Exchange buffer of one group: the P x P intermediate, row k at offset
// P k + k / 4.  The extra entry every fourth row spreads the rows a group
// reads column-wise in step 2 (lane r reads row r) over distinct LDS banks.
template <int P>
__host__ __device__ constexpr int ls_row_off(int k) { return P * k + k / 4; }
template <int P>
__host__ __device__ constexpr int ls_buf_len() { return ls_row_off<P>(P - 1) + P; }
// Distance between the buffers of neighbouring groups: one entry more than a
// buffer, so the five groups of a wavefront start on staggered banks.
template <int P>
__host__ __device__ constexpr int ls_buf_stride() { return ls_buf_len<P>() + 1; }

// Index a of the P values a lane holds lies in the outer quarters of the
// sequence: P a + lb in [0, N/4) or [3N/4, N), i.e. centred index in [-N/4, N/4).
template <int P>
__host__ __device__ constexpr bool ls_quarter(int a) { return a < P / 4 || a >= P - P / 4; }

// Step 1 on v (the P values x[P a + lb] of lane lb): P-point DFT, twiddle,
// store row-wise into buf; step 2: lane lb reads intermediate row lb and
// transforms it.  Result: v[k] holds element lb + P k.  ZIN: the input is
// zero outside the outer quarters (those v[a] are not read; the DFT folds the
// zeros away).  Callers that use only the outer-quarter outputs leave the
// rest unused and the compiler drops their arithmetic.
template <int P, int S, bool ZIN = false>
__device__ __forceinline__ void ls_fft_regs(float2 (&v)[P], float2* buf, int lb,
                                            const float2 (&w)[P - 1]) {
  if constexpr (ZIN) {
#pragma unroll
    for (int a = 0; a < P; ++a)
      if (!ls_quarter<P>(a)) v[a] = czero<float2>();
  }
  dft_reg<P, S>(v);
  ls_twiddle<P, S>(v, w);
#pragma unroll
  for (int k = 0; k < P; ++k) buf[ls_row_off<P>(k) + lb] = v[k];
  wave_lds_fence();
  const float2* row = buf + ls_row_off<P>(lb);
#pragma unroll
  for (int b = 0; b < P; ++b) v[b] = row[b];
  dft_reg<P, S>(v);
  wave_lds_fence();
}

// Transform (sign S) of the length-P^2 sequence seq[0 .. P^2) in LDS by the P
// lanes of a group, through the group's exchange buffer: natural order in,
// natural order out.  ZIN: input zero outside the outer quarters; QOUT: only
// the outer-quarter outputs are written.
template <int P, int S, bool ZIN, bool QOUT>
__device__ __forceinline__ void ls_fft_seq(float2* seq, float2* buf, int lb,
                                           const float2 (&w)[P - 1]) {
  float2 v[P];
#pragma unroll
  for (int a = 0; a < P; ++a)
    if (!ZIN || ls_quarter<P>(a)) v[a] = seq[P * a + lb];
  ls_fft_regs<P, S, ZIN>(v, buf, lb, w);
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (!QOUT || ls_quarter<P>(k)) seq[lb + P * k] = v[k];
}

// Columns handled together by the groups of one wavefront are kColSpacing
// apart in E: 12 x (P^2 + 1) complex entries is 24 dwords past a multiple of
// 64 banks, so the groups' contiguous 24-dword slices tile the banks.
constexpr int kColSpacing = 12;

// Columns of the sphere per thread kept in registers from one plane to the
// next (the next plane's are loaded while the current one is transformed);
// plans with more columns load the rest directly.
constexpr int kLsPre = 4;

// Q: every sphere point's centred m1 and m2 lie in [-N/4, N/4) (always so
// when the box holds the density's sphere), which prunes the transforms:
// the backward N2 and N1 passes start from data zero outside the outer
// quarters, the forward ones are needed only there.
//
// Persistent: workgroup g takes planes L = g, g + G, ... of the n3 x nb
// (z-plane, band) planes, L = b n3 + j3.
template <int P, bool Q>
__global__ void __launch_bounds__(kLsMaxWaves * 64)
k_plane_ls(BoxPlan Pl, const float2* __restrict__ tw, const float* __restrict__ vs,
           float2* __restrict__ T, int nplanes) {
  constexpr int N = P * P, TRS = N + 1, GPW = 64 / P, XS = ls_buf_stride<P>();
  // the unpruned transforms need the registers: no prefetch there
  constexpr int KP = Q ? kLsPre : 0;
  constexpr int KPA = KP > 0 ? KP : 1;
  extern __shared__ __align__(16) char lds_raw[];
  float2* E = reinterpret_cast<float2*>(lds_raw);                      // xr x TRS
  const int tid = threadIdx.x, nt = blockDim.x;
  float2* X = E + (size_t)Pl.xr * TRS;                                 // groups x N
  int* slot = reinterpret_cast<int*>(X + (size_t)(nt >> 6) * GPW * XS);  // N
  const int wave = tid >> 6, lw = tid & 63;
  const int gw = lw / P, lb = lw - gw * P;
  const bool act = gw < GPW;
  const int nw = nt >> 6;
  const int grp = wave * GPW + gw;
  float2* buf = X + (size_t)grp * XS;
  // Work items are dealt in tasks of GPW items, one per group of the
  // wavefront that takes the task, spaced so that the groups' LDS accesses
  // fall on different banks.  Rows: task t holds rows t + rstride gw.
  // Extent columns: tasks come in rounds of kColSpacing, task t of round r
  // holds columns r kColSpacing GPW + t + kColSpacing gw.
  const int rstride = (N + GPW - 1) / GPW;
  const int ctasks = kColSpacing * ((Pl.xr + kColSpacing * GPW - 1) / (kColSpacing * GPW));
  const int64_t plane_elems = Pl.ldt;
  // per plane invariants: extent slots, twiddles, this thread's column positions in E
  for (int i = tid; i < N; i += nt) slot[i] = -1;
  __syncthreads();
  for (int e = tid; e < Pl.xr; e += nt) slot[Pl.ext_m1[e]] = e;
  int cpos[KPA];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int c = tid + k * nt;
    cpos[k] = c < Pl.ncols ? Pl.col_e[c] * TRS + Pl.col_m2[c] : 0;
  }
  float2 w[P - 1];
#pragma unroll
  for (int k = 1; k < P; ++k) w[k - 1] = tw[(lb * k) % N];
  // plane L's row of T: band b = L / n3, z-plane j3 = L % n3, i.e. offset L ldt
  float2 pre[KPA];
  auto fetch = [&](int L) {
    if (L < nplanes) {
      const float2* tq = T + (size_t)L * plane_elems;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int c = tid + k * nt;
        if (c < Pl.ncols) pre[k] = tq[c];
      }
    }
  };
  fetch(blockIdx.x);
  for (int L = blockIdx.x; L < nplanes; L += gridDim.x) {
    const int j3 = L % Pl.n3;
    float2* tp = T + (size_t)L * plane_elems;
    __syncthreads();   // the previous plane's gather is done with E
    if constexpr (Q) {
      // the backward N2 pass reads only the outer quarters of each column
      constexpr int H = N / 4;
      for (int i = tid; i < Pl.xr * 2 * H; i += nt) {
        const int e = i / (2 * H), j = i - e * (2 * H);
        E[e * TRS + (j < H ? j : j + N - 2 * H)] = czero<float2>();
      }
    } else {
      for (int i = tid; i < Pl.xr * TRS; i += nt) E[i] = czero<float2>();
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (tid + k * nt < Pl.ncols) E[cpos[k]] = pre[k];
    for (int c = tid + KP * nt; c < Pl.ncols; c += nt)
      E[Pl.col_e[c] * TRS + Pl.col_m2[c]] = tp[c];
    __syncthreads();
    fetch(L + gridDim.x);   // next plane's columns, in flight during the transforms
    // backward along N2 on every extent column
    if (act)
      for (int t = wave; t < ctasks; t += nw) {
        const int e = (t / kColSpacing) * (kColSpacing * GPW) + t % kColSpacing + kColSpacing * gw;
        if (e < Pl.xr) ls_fft_seq<P, +1, Q, false>(E + e * TRS, buf, lb, w);
      }
    __syncthreads();
    // rows: backward along N1, x V/N_box, forward along N1
    if (act) {
      int sl[P];   // extent slot of positions P a + lb (the same set on output: lb + P k)
#pragma unroll
      for (int a = 0; a < P; ++a) sl[a] = slot[P * a + lb];
      const float* vp = vs + (size_t)j3 * N * N;
      for (int t = wave; t < rstride; t += nw) {
        const int row = t + rstride * gw;
        if (row >= N) continue;
        float2 v[P];
#pragma unroll
        for (int a = 0; a < P; ++a)
          if (!Q || ls_quarter<P>(a)) v[a] = sl[a] >= 0 ? E[sl[a] * TRS + row] : czero<float2>();
        ls_fft_regs<P, +1, Q>(v, buf, lb, w);
        const float* vr = vp + (size_t)row * N + lb;
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = cscale(v[k], vr[P * k]);
        ls_fft_regs<P, -1>(v, buf, lb, w);
        // v[k] holds position lb + P k: slot sl[k]
#pragma unroll
        for (int k = 0; k < P; ++k)
          if ((!Q || ls_quarter<P>(k)) && sl[k] >= 0) E[sl[k] * TRS + row] = v[k];
      }
    }
    __syncthreads();
    // forward along N2
    if (act)
      for (int t = wave; t < ctasks; t += nw) {
        const int e = (t / kColSpacing) * (kColSpacing * GPW) + t % kColSpacing + kColSpacing * gw;
        if (e < Pl.xr) ls_fft_seq<P, -1, false, Q>(E + e * TRS, buf, lb, w);
      }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (tid + k * nt < Pl.ncols) tp[tid + k * nt] = E[cpos[k]];
    for (int c = tid + KP * nt; c < Pl.ncols; c += nt)
      tp[c] = E[Pl.col_e[c] * TRS + Pl.col_m2[c]];
  }
}

constexpr int kLsP = 12;   // N1 = N2 = 144

size_t g_ls_lds_limit = 64 * 1024;
int g_ls_cus = 256;   // compute units of the device (set with the LDS limit)

size_t ls_lds_bytes(const BoxPlan& p, int waves) {
  constexpr int N = kLsP * kLsP, GPW = 64 / kLsP;
  return (size_t)p.xr * (N + 1) * sizeof(float2) +
         (size_t)waves * GPW * ls_buf_stride<kLsP>() * sizeof(float2) + (size_t)N * sizeof(int);
}

// the most wavefronts whose buffers fit next to this plan's extent array
int ls_waves(const BoxPlan& p, size_t lds_limit) {
  int w = kLsMaxWaves;
  while (w >= kLsMinWaves && ls_lds_bytes(p, w) > lds_limit) --w;
  return w;
}

}  // namespace

size_t fft_plane_ls_lds(const BoxPlan& p) { return ls_lds_bytes(p, ls_waves(p, g_ls_lds_limit)); }

bool fft_plane_ls_supported(const BoxPlan& p, size_t lds_limit) {
  return p.n1 == kLsP * kLsP && p.n2 == kLsP * kLsP && ls_waves(p, lds_limit) >= kLsMinWaves;
}

hipError_t launch_fft_plane_ls32(const BoxPlan& p, int nb, const float* vscaled, float2* T,
                                 hipStream_t s) {
  const int waves = ls_waves(p, g_ls_lds_limit);
  if (p.n1 != kLsP * kLsP || p.n2 != p.n1 || p.ax1.tw32 == nullptr || waves < kLsMinWaves)
    return hipErrorInvalidValue;
  if (nb <= 0) return hipSuccess;
  // persistent grid: as many workgroups as are resident at once (LDS: one
  // per CU at C5 sizes; VGPRs: at most 16 wavefronts per CU)
  const size_t lds = ls_lds_bytes(p, waves);
  const int per_cu = std::max(1, std::min((int)(g_ls_lds_limit / lds), 16 / waves));
  const int64_t nplanes = (int64_t)p.n3 * nb;
  const int grid = (int)std::min<int64_t>(nplanes, (int64_t)g_ls_cus * per_cu);
  if (p.quarter12)
    hipLaunchKernelGGL((k_plane_ls<kLsP, true>), dim3(grid), dim3(waves * 64), lds, s, p,
                       p.ax1.tw32, vscaled, T, (int)nplanes);
  else
    hipLaunchKernelGGL((k_plane_ls<kLsP, false>), dim3(grid), dim3(waves * 64), lds, s, p,
                       p.ax1.tw32, vscaled, T, (int)nplanes);
  return hipGetLastError();
}

hipError_t fft_ls_set_lds_limit(size_t bytes) {
  g_ls_lds_limit = bytes;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    g_ls_cus = cus;
  hipError_t e = hipFuncSetAttribute((const void*)k_plane_ls<kLsP, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_plane_ls<kLsP, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
