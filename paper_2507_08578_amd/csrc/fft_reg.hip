// Register-resident variants of the three FFT-route kernels for the box
// lengths listed in kFastSizes.  Each 1D transform of length N = G R lives
// in the registers of G lanes of one wavefront (R values per lane): an
// R-point DFT in registers, then log2(G) radix-2 stages across lanes with
// wavefront shuffles (pwfft::lane_fft_bwd / lane_fft_fwd).  LDS holds only
// the data that must change hands between axes:
//   col kernels : a tile of columns (one column per lane group),
//   plane kernel: the extent array E[e][m2] of one z-plane; every N2
//                 transform and every N1 row (backward, x V/N_box, forward)
//                 reads its input from E and writes its output back in place.
#include "fft_common.h"

#include <algorithm>

using namespace pwfft;

namespace {

constexpr int kColThreads = 256;
constexpr int kPlaneMaxThreads = 512;

// S: storage type of the block psi (C, or bf16 pairs widened on load).
template <int N3, class C, class S = C>
__device__ __forceinline__ void col_inv_reg_body(const BoxPlan& P, const C* __restrict__ tw3,
                                                 const S* __restrict__ psi, int64_t ldpsi,
                                                 C* __restrict__ T, int cb, int b) {
  constexpr int G = lane_group(N3), R = N3 / G, CT = kColThreads / G, TRS = N3 + 1;
  __shared__ C tile[CT * TRS];
  const int c0 = cb * CT;
  const int ncl = min(CT, P.ncols - c0);
  const S* src = psi + (size_t)b * ldpsi;
  const int grp = threadIdx.x / G, lb = threadIdx.x % G;
  if (!P.runs) {
    for (int i = threadIdx.x; i < CT * TRS; i += blockDim.x) tile[i] = czero<C>();
    __syncthreads();
    const int k0 = P.col_start[c0], k1 = P.col_start[c0 + ncl];
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x)
      tile[(P.pt_col[k] - c0) * TRS + P.pt_m3[k]] = ld_c(src[P.pt_perm[k]]);
    __syncthreads();
  }
  if (grp < ncl) {
    C v[R];
    C* col = tile + grp * TRS;
    LaneTw<R, G, C> tw;
    tw.load(lb, tw3);
    if (P.runs) {
      // one lane group per column, its points consecutive in psi and in
      // centred m3 from lo: lane lb loads box positions G a + lb straight
      // into registers (zero outside the run)
      const int c = c0 + grp, ks = P.col_start[c], len = P.col_start[c + 1] - ks;
      const int lo = P.col_m3lo[c];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const int m = G * a + lb;
        const int j = (m <= N3 / 2 ? m : m - N3) - lo;
        v[a] = (unsigned)j < (unsigned)len ? ld_c(src[ks + j]) : czero<C>();
      }
    } else {
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = col[G * a + lb];
    }
    lane_fft_bwd<R, G>(v, lb, tw);
    const int base = R * brev<G>(lb);
#pragma unroll
    for (int q = 0; q < R; ++q) col[q + base] = v[q];
  }
  __syncthreads();
  // rows of CT columns (no division by the tile's column count): lane lc
  // of every CT-lane slice writes column lc of row j3
  C* dst = T + (size_t)b * N3 * P.ldt + c0;
  {
    const int lc = threadIdx.x % CT;
    if (lc < ncl)
      for (int j3 = threadIdx.x / CT; j3 < N3; j3 += kColThreads / CT)
        dst[(size_t)j3 * P.ldt + lc] = tile[lc * TRS + j3];
  }
}

template <int N3, class C, class S = C>
__global__ void __launch_bounds__(kColThreads)
k_col_inv_reg(BoxPlan P, const C* __restrict__ tw3, const S* __restrict__ psi, int64_t ldpsi,
              C* __restrict__ T) {
  col_inv_reg_body<N3, C, S>(P, tw3, psi, ldpsi, T, blockIdx.x, blockIdx.y);
}

// S: storage type of the blocks in, prev and out.
template <int N3, class C, class S = C>
__device__ __forceinline__ void col_fwd_reg_body(const BoxPlan& P, const C* __restrict__ tw3,
                                                 const C* __restrict__ T,
                                                 const real_t<C>* __restrict__ kin, const S* in,
                                                 int64_t ldin, const S* prev, int64_t ldprev,
                                                 S* out, int64_t ldout, double alpha_d,
                                                 double beta_d, double gamma_d,
                                                 const double* __restrict__ coef, int cb, int b) {
  using Rl = real_t<C>;
  constexpr int G = lane_group(N3), R = N3 / G, CT = kColThreads / G, TRS = N3 + 1;
  __shared__ C tile[CT * TRS];
  if (coef) {
    alpha_d = coef[0];
    beta_d = coef[1];
    gamma_d = coef[2];
  }
  const Rl alpha = (Rl)alpha_d, beta = (Rl)beta_d, gamma = (Rl)gamma_d;
  const int c0 = cb * CT;
  const int ncl = min(CT, P.ncols - c0);
  const C* srcT = T + (size_t)b * N3 * P.ldt + c0;
  {
    const int lc = threadIdx.x % CT;
    if (lc < ncl)
      for (int j3 = threadIdx.x / CT; j3 < N3; j3 += kColThreads / CT)
        tile[lc * TRS + j3] = srcT[(size_t)j3 * P.ldt + lc];
  }
  __syncthreads();
  const int grp = threadIdx.x / G, lb = threadIdx.x % G;
  if (grp < ncl) {
    C v[R];
    C* col = tile + grp * TRS;
    const int base = R * brev<G>(lb);
    LaneTw<R, G, C> tw;
    tw.load(lb, tw3);
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = col[q + base];
    lane_fft_fwd<R, G>(v, lb, tw);
#pragma unroll
    for (int a = 0; a < R; ++a) col[G * a + lb] = v[a];
  }
  __syncthreads();
  const S* inb = in + (size_t)b * ldin;
  S* outb = out + (size_t)b * ldout;
  const S* prevb = prev ? prev + (size_t)b * ldprev : nullptr;
  auto emit = [&](int g, const C& loc) {
    const C x = ld_c(inb[g]);
    const Rl t = kin[g];
    C val;
    val.x = alpha * (loc.x + t * x.x) + beta * x.x;
    val.y = alpha * (loc.y + t * x.y) + beta * x.y;
    if (prevb) {
      const C p = ld_c(prevb[g]);
      val.x += gamma * p.x;
      val.y += gamma * p.y;
    }
    outb[g] = st_c<S>(val);
  };
  if (P.runs) {
    // one lane group per column: its points are consecutive in psi and in m3
    if (grp < ncl) {
      const int c = c0 + grp, ks = P.col_start[c], len = P.col_start[c + 1] - ks;
      const int lo = P.col_m3lo[c];
      for (int j = lb; j < len; j += G) {
        const int m = lo + j;
        emit(ks + j, tile[grp * TRS + (m < 0 ? m + N3 : m)]);
      }
    }
  } else {
    const int k0 = P.col_start[c0], k1 = P.col_start[c0 + ncl];
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x)
      emit(P.pt_perm[k], tile[(P.pt_col[k] - c0) * TRS + P.pt_m3[k]]);
  }
}

template <int N3, class C, class S = C>
__global__ void __launch_bounds__(kColThreads)
k_col_fwd_reg(BoxPlan P, const C* __restrict__ tw3, const C* __restrict__ T,
              const real_t<C>* __restrict__ kin, const S* in, int64_t ldin, const S* prev,
              int64_t ldprev, S* out, int64_t ldout, double alpha_d, double beta_d,
              double gamma_d, const double* __restrict__ coef) {
  col_fwd_reg_body<N3, C, S>(P, tw3, T, kin, in, ldin, prev, ldprev, out, ldout, alpha_d, beta_d,
                             gamma_d, coef, blockIdx.x, blockIdx.y);
}

template <int N1, int N2, int GMAX, class C>
__device__ __forceinline__ void plane_reg_body(const BoxPlan& P, const C* __restrict__ tw1,
                                               const C* __restrict__ tw2,
                                               const real_t<C>* __restrict__ vs,
                                               C* __restrict__ T, int j3, int b) {
  constexpr int G1 = lane_group(N1, GMAX), R1 = N1 / G1;
  constexpr int G2 = lane_group(N2, GMAX), R2 = N2 / G2;
  constexpr int TRS = N2 + 1;
  extern __shared__ __align__(16) char lds_raw[];
  C* E = reinterpret_cast<C*>(lds_raw);                            // xr x TRS
  int* slot = reinterpret_cast<int*>(E + (size_t)P.xr * TRS);      // N1 entries
  const int tid = threadIdx.x, nt = blockDim.x;
  C* tp = T + (size_t)b * P.n3 * P.ldt + (size_t)j3 * P.ldt;
  for (int i = tid; i < P.xr * TRS; i += nt) E[i] = czero<C>();
  for (int i = tid; i < N1; i += nt) slot[i] = -1;
  __syncthreads();
  for (int e = tid; e < P.xr; e += nt) slot[P.ext_m1[e]] = e;
  for (int c = tid; c < P.ncols; c += nt) E[P.col_e[c] * TRS + P.col_m2[c]] = tp[c];
  __syncthreads();
  // backward along N2 for every extent column (in place, one column per lane group)
  {
    const int grp = tid / G2, lb = tid % G2, ngr = nt / G2;
    const int base = R2 * brev<G2>(lb);
    LaneTw<R2, G2, C> tw;
    tw.load(lb, tw2);
    for (int e = grp; e < P.xr; e += ngr) {
      C v[R2];
      C* col = E + e * TRS;
#pragma unroll
      for (int a = 0; a < R2; ++a) v[a] = col[G2 * a + lb];
      lane_fft_bwd<R2, G2>(v, lb, tw);
#pragma unroll
      for (int q = 0; q < R2; ++q) col[q + base] = v[q];
    }
  }
  __syncthreads();
  // rows: backward along N1, x V/N_box, forward along N1; only extent entries live in E
  {
    const int grp = tid / G1, lb = tid % G1, ngr = nt / G1;
    const int base = R1 * brev<G1>(lb);
    LaneTw<R1, G1, C> tw;
    tw.load(lb, tw1);
    const real_t<C>* vp = vs + (size_t)j3 * N2 * N1;
    for (int row = grp; row < N2; row += ngr) {
      C v[R1];
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        const int s = slot[G1 * a + lb];
        v[a] = s >= 0 ? E[s * TRS + row] : czero<C>();
      }
      lane_fft_bwd<R1, G1>(v, lb, tw);
      const real_t<C>* vr = vp + (size_t)row * N1 + base;
#pragma unroll
      for (int q = 0; q < R1; ++q) v[q] = cscale(v[q], vr[q]);
      lane_fft_fwd<R1, G1>(v, lb, tw);
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        const int s = slot[G1 * a + lb];
        if (s >= 0) E[s * TRS + row] = v[a];
      }
    }
  }
  __syncthreads();
  // forward along N2
  {
    const int grp = tid / G2, lb = tid % G2, ngr = nt / G2;
    const int base = R2 * brev<G2>(lb);
    LaneTw<R2, G2, C> tw;
    tw.load(lb, tw2);
    for (int e = grp; e < P.xr; e += ngr) {
      C v[R2];
      C* col = E + e * TRS;
#pragma unroll
      for (int q = 0; q < R2; ++q) v[q] = col[q + base];
      lane_fft_fwd<R2, G2>(v, lb, tw);
#pragma unroll
      for (int a = 0; a < R2; ++a) col[G2 * a + lb] = v[a];
    }
  }
  __syncthreads();
  for (int c = tid; c < P.ncols; c += nt) tp[c] = E[P.col_e[c] * TRS + P.col_m2[c]];
}

template <int N1, int N2, int GMAX, class C>
__global__ void __launch_bounds__(kPlaneMaxThreads)
k_plane_reg(BoxPlan P, const C* __restrict__ tw1, const C* __restrict__ tw2,
            const real_t<C>* __restrict__ vs, C* __restrict__ T) {
  plane_reg_body<N1, N2, GMAX, C>(P, tw1, tw2, vs, T, blockIdx.x, blockIdx.y);
}

// ---- fused-batch variants: item = blockIdx.z, all items share the box lengths
template <class C>
__device__ __forceinline__ const C* tw_of(const FftAxis& ax);
template <>
__device__ __forceinline__ const double2* tw_of<double2>(const FftAxis& ax) { return ax.tw; }
template <>
__device__ __forceinline__ const float2* tw_of<float2>(const FftAxis& ax) { return ax.tw32; }

template <class C>
__device__ __forceinline__ C* item_block(const ItemDev& d, int sel);
template <>
__device__ __forceinline__ double2* item_block<double2>(const ItemDev& d, int sel) {
  return item_blk64(d, sel);
}
template <>
__device__ __forceinline__ float2* item_block<float2>(const ItemDev& d, int sel) {
  return item_blk32(d, sel);
}
template <class C>
__device__ __forceinline__ C* item_T(const ItemDev& d);
template <>
__device__ __forceinline__ double2* item_T<double2>(const ItemDev& d) { return d.T; }
template <>
__device__ __forceinline__ float2* item_T<float2>(const ItemDev& d) { return d.T32; }
template <class C>
__device__ __forceinline__ const real_t<C>* item_kin(const ItemDev& d);
template <>
__device__ __forceinline__ const double* item_kin<double2>(const ItemDev& d) { return d.kin; }
template <>
__device__ __forceinline__ const float* item_kin<float2>(const ItemDev& d) { return d.kin32; }
template <class C>
__device__ __forceinline__ const real_t<C>* item_vs(const ItemDev& d);
template <>
__device__ __forceinline__ const double* item_vs<double2>(const ItemDev& d) { return d.vs; }
template <>
__device__ __forceinline__ const float* item_vs<float2>(const ItemDev& d) { return d.vs32; }

template <int N3, class C>
__global__ void __launch_bounds__(kColThreads)
kb_col_inv_reg(const ItemDev* __restrict__ D, int sel_in) {
  constexpr int CT = kColThreads / lane_group(N3);
  const ItemDev& d = D[blockIdx.z];
  if ((int)blockIdx.y >= d.nb || (int)blockIdx.x * CT >= d.plan.ncols) return;
  col_inv_reg_body<N3, C>(d.plan, tw_of<C>(d.plan.ax3), item_block<C>(d, sel_in), d.npw,
                          item_T<C>(d), blockIdx.x, blockIdx.y);
}

template <int N3, class C>
__global__ void __launch_bounds__(kColThreads)
kb_col_fwd_reg(const ItemDev* __restrict__ D, int sel_in, int sel_out, int sel_prev, double alpha,
               double beta, double gamma, int coef_step) {
  constexpr int CT = kColThreads / lane_group(N3);
  const ItemDev& d = D[blockIdx.z];
  if ((int)blockIdx.y >= d.nb || (int)blockIdx.x * CT >= d.plan.ncols) return;
  col_fwd_reg_body<N3, C>(d.plan, tw_of<C>(d.plan.ax3), item_T<C>(d), item_kin<C>(d),
                          item_block<C>(d, sel_in), d.npw, item_block<C>(d, sel_prev), d.npw,
                          item_block<C>(d, sel_out), d.npw, alpha, beta, gamma,
                          coef_step >= 0 ? d.coef + 3 * coef_step : nullptr, blockIdx.x,
                          blockIdx.y);
}

template <int N1, int N2, int GMAX, class C>
__global__ void __launch_bounds__(kPlaneMaxThreads)
kb_plane_reg(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.z];
  if ((int)blockIdx.y >= d.nb || (int)blockIdx.x >= d.plan.n3) return;
  plane_reg_body<N1, N2, GMAX, C>(d.plan, tw_of<C>(d.plan.ax1), tw_of<C>(d.plan.ax2),
                                  item_vs<C>(d), item_T<C>(d), blockIdx.x, blockIdx.y);
}

size_t plane_reg_lds(const BoxPlan& p, size_t elem) {
  return (size_t)p.xr * (p.n2 + 1) * elem + (size_t)p.n1 * sizeof(int);
}

int plane_reg_threads(const BoxPlan& p, int gmax) {
  const int g1 = lane_group(p.n1, gmax), g2 = lane_group(p.n2, gmax);
  int t = std::max(p.xr * g2, p.n2 * g1);
  t = ((t + 63) / 64) * 64;
  return std::min(t, kPlaneMaxThreads);
}

#define PW_FAST_SIZES(X) X(24) X(30) X(32) X(36) X(48) X(64) X(72) X(96) X(120) X(128) X(144) X(160)
// sizes whose 8-lane variant differs from the 16-lane one and fits the
// registers: FP64, and FP32 (half the registers per value)
#define PW_NARROW_SIZES64(X) X(48) X(64) X(96)
#define PW_NARROW_SIZES32(X) X(48) X(64) X(96) X(120) X(128) X(144) X(160)

}  // namespace

bool fft_reg_col_supported(int n3) {
#define CASE(N) if (n3 == N) return true;
  PW_FAST_SIZES(CASE)
#undef CASE
  return false;
}

bool fft_reg_plane_narrow(const BoxPlan& p, bool fp32) {
#define CASE(N) if (p.n1 == N && p.n2 == N) return true;
  if (fp32) {
    PW_NARROW_SIZES32(CASE)
  } else {
    PW_NARROW_SIZES64(CASE)
  }
#undef CASE
  return false;
}

bool fft_reg_plane_supported(const BoxPlan& p, size_t lds_limit) {
  if (p.n1 != p.n2) return false;
  bool ok = false;
#define CASE(N) if (p.n1 == N) ok = true;
  PW_FAST_SIZES(CASE)
#undef CASE
  return ok && plane_reg_lds(p, sizeof(cplx)) <= lds_limit;
}

namespace {

template <class C>
const C* axis_tw(const FftAxis& ax);
template <>
const double2* axis_tw<double2>(const FftAxis& ax) { return ax.tw; }
template <>
const float2* axis_tw<float2>(const FftAxis& ax) { return ax.tw32; }

template <class C, class S = C>
hipError_t col_inv_reg(const BoxPlan& p, int nb, const S* psi, int64_t ldpsi, C* T, hipStream_t s) {
#define CASE(N)                                                                              \
  if (p.n3 == N) {                                                                           \
    constexpr int CT = kColThreads / lane_group(N);                                          \
    dim3 grid((p.ncols + CT - 1) / CT, nb);                                                  \
    hipLaunchKernelGGL((k_col_inv_reg<N, C, S>), grid, dim3(kColThreads), 0, s, p,           \
                       axis_tw<C>(p.ax3), psi, ldpsi, T);                                    \
    return hipGetLastError();                                                                \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <class C, class S = C>
hipError_t col_fwd_reg(const BoxPlan& p, int nb, const C* T, const real_t<C>* kin, const S* in,
                       int64_t ldin, const S* prev, int64_t ldprev, S* out, int64_t ldout,
                       const Epilogue& ep, hipStream_t s) {
#define CASE(N)                                                                               \
  if (p.n3 == N) {                                                                            \
    constexpr int CT = kColThreads / lane_group(N);                                           \
    dim3 grid((p.ncols + CT - 1) / CT, nb);                                                   \
    hipLaunchKernelGGL((k_col_fwd_reg<N, C, S>), grid, dim3(kColThreads), 0, s, p,            \
                       axis_tw<C>(p.ax3), T, kin, in, ldin, prev, ldprev, out, ldout, ep.alpha,  \
                       ep.beta, ep.gamma, ep.coef);                                           \
    return hipGetLastError();                                                                 \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

// variant 0: lane groups of up to 16 lanes; variant 1: up to 8 lanes (more
// values per lane, fewer cross-lane stages).
template <class C>
hipError_t plane_reg(const BoxPlan& p, int variant, int nb, const real_t<C>* vscaled, C* T,
                     hipStream_t s) {
  const size_t lds = plane_reg_lds(p, sizeof(C));
  const int gmax = variant == 1 ? 8 : 16;
  const int threads = plane_reg_threads(p, gmax);
  const C* tw1 = axis_tw<C>(p.ax1);
  const C* tw2 = axis_tw<C>(p.ax2);
  if (variant == 1) {
#define CASE(N)                                                                                \
    if (p.n1 == N && p.n2 == N) {                                                              \
      hipLaunchKernelGGL((k_plane_reg<N, N, 8, C>), dim3(p.n3, nb), dim3(threads), lds, s, p,  \
                         tw1, tw2, vscaled, T);                                                \
      return hipGetLastError();                                                                \
    }
    if constexpr (sizeof(C) == sizeof(double2)) {
      PW_NARROW_SIZES64(CASE)
    } else {
      PW_NARROW_SIZES32(CASE)
    }
#undef CASE
    return hipErrorInvalidValue;
  }
#define CASE(N)                                                                                \
  if (p.n1 == N && p.n2 == N) {                                                                \
    hipLaunchKernelGGL((k_plane_reg<N, N, 16, C>), dim3(p.n3, nb), dim3(threads), lds, s, p,   \
                       tw1, tw2, vscaled, T);                                                  \
    return hipGetLastError();                                                                  \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <class C>
hipError_t set_plane_lds(size_t bytes) {
#define CASE(N)                                                                              \
  {                                                                                          \
    hipError_t e = hipFuncSetAttribute((const void*)k_plane_reg<N, N, 16, C>,                \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); \
    if (e != hipSuccess) return e;                                                           \
    e = hipFuncSetAttribute((const void*)kb_plane_reg<N, N, 16, C>,                          \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);         \
    if (e != hipSuccess) return e;                                                           \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
#define CASE(N)                                                                              \
  {                                                                                          \
    hipError_t e = hipFuncSetAttribute((const void*)k_plane_reg<N, N, 8, C>,                 \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); \
    if (e != hipSuccess) return e;                                                           \
    e = hipFuncSetAttribute((const void*)kb_plane_reg<N, N, 8, C>,                           \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);         \
    if (e != hipSuccess) return e;                                                           \
  }
  if constexpr (sizeof(C) == sizeof(double2)) {
    PW_NARROW_SIZES64(CASE)
  } else {
    PW_NARROW_SIZES32(CASE)
  }
#undef CASE
  return hipSuccess;
}

}  // namespace

namespace {
template <class C>
hipError_t fused_col_inv_reg(const FusedFft& f, const ItemDev* D, int sel_in, hipStream_t s) {
#define CASE(N)                                                                             \
  if (f.n3 == N) {                                                                          \
    constexpr int CT = kColThreads / lane_group(N);                                         \
    dim3 grid((f.ncols_max + CT - 1) / CT, f.nb_max, f.nitems);                             \
    hipLaunchKernelGGL((kb_col_inv_reg<N, C>), grid, dim3(kColThreads), 0, s, D, sel_in);   \
    return hipGetLastError();                                                               \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <class C>
hipError_t fused_col_fwd_reg(const FusedFft& f, const ItemDev* D, int sel_in, int sel_out,
                             int sel_prev, double alpha, double beta, double gamma, int coef_step,
                             hipStream_t s) {
#define CASE(N)                                                                              \
  if (f.n3 == N) {                                                                           \
    constexpr int CT = kColThreads / lane_group(N);                                          \
    dim3 grid((f.ncols_max + CT - 1) / CT, f.nb_max, f.nitems);                              \
    hipLaunchKernelGGL((kb_col_fwd_reg<N, C>), grid, dim3(kColThreads), 0, s, D, sel_in,      \
                       sel_out, sel_prev, alpha, beta, gamma, coef_step);                     \
    return hipGetLastError();                                                                \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <class C>
hipError_t fused_plane_reg(const FusedFft& f, int variant, const ItemDev* D, hipStream_t s) {
  BoxPlan shape{};
  shape.n1 = f.n1;
  shape.n2 = f.n2;
  shape.n3 = f.n3;
  shape.xr = f.xr_max;
  const size_t lds = plane_reg_lds(shape, sizeof(C));
  const int threads = plane_reg_threads(shape, variant == 1 ? 8 : 16);
  dim3 grid(f.n3_max, f.nb_max, f.nitems);
  if (variant == 1) {
#define CASE(N)                                                                               \
    if (f.n1 == N && f.n2 == N) {                                                             \
      hipLaunchKernelGGL((kb_plane_reg<N, N, 8, C>), grid, dim3(threads), lds, s, D);         \
      return hipGetLastError();                                                               \
    }
    if constexpr (sizeof(C) == sizeof(double2)) {
      PW_NARROW_SIZES64(CASE)
    } else {
      PW_NARROW_SIZES32(CASE)
    }
#undef CASE
    return hipErrorInvalidValue;
  }
#define CASE(N)                                                                               \
  if (f.n1 == N && f.n2 == N) {                                                               \
    hipLaunchKernelGGL((kb_plane_reg<N, N, 16, C>), grid, dim3(threads), lds, s, D);          \
    return hipGetLastError();                                                                 \
  }
  PW_FAST_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_fused_col_inv_reg(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                    hipStream_t s) {
  return fp32 ? fused_col_inv_reg<float2>(f, D, sel_in, s) : fused_col_inv_reg<double2>(f, D, sel_in, s);
}
hipError_t launch_fused_col_fwd_reg(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                    int sel_out, int sel_prev, double alpha, double beta,
                                    double gamma, int coef_step, hipStream_t s) {
  return fp32 ? fused_col_fwd_reg<float2>(f, D, sel_in, sel_out, sel_prev, alpha, beta, gamma,
                                          coef_step, s)
              : fused_col_fwd_reg<double2>(f, D, sel_in, sel_out, sel_prev, alpha, beta, gamma,
                                           coef_step, s);
}
hipError_t launch_fused_plane_reg(const FusedFft& f, bool fp32, const ItemDev* D, hipStream_t s) {
  return fp32 ? fused_plane_reg<float2>(f, f.plane_variant32, D, s)
              : fused_plane_reg<double2>(f, f.plane_variant, D, s);
}

hipError_t launch_fft_col_inv_reg(const BoxPlan& p, int nb, const cplx* psi, int64_t ldpsi, cplx* T,
                                  hipStream_t s) {
  return col_inv_reg<double2>(p, nb, psi, ldpsi, T, s);
}
hipError_t launch_fft_col_inv_reg32(const BoxPlan& p, int nb, const float2* psi, int64_t ldpsi,
                                    float2* T, hipStream_t s) {
  return col_inv_reg<float2>(p, nb, psi, ldpsi, T, s);
}

hipError_t launch_fft_col_fwd_reg(const BoxPlan& p, int nb, const cplx* T, const double* kin,
                                  const cplx* in, int64_t ldin, const cplx* prev, int64_t ldprev,
                                  cplx* out, int64_t ldout, const Epilogue& ep, hipStream_t s) {
  return col_fwd_reg<double2>(p, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
}
hipError_t launch_fft_col_fwd_reg32(const BoxPlan& p, int nb, const float2* T, const float* kin,
                                    const float2* in, int64_t ldin, const float2* prev,
                                    int64_t ldprev, float2* out, int64_t ldout, const Epilogue& ep,
                                    hipStream_t s) {
  return col_fwd_reg<float2>(p, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
}

hipError_t launch_fft_col_inv_reg16(const BoxPlan& p, int nb, const bf16c* psi, int64_t ldpsi,
                                    float2* T, hipStream_t s) {
  return col_inv_reg<float2, bf16c>(p, nb, psi, ldpsi, T, s);
}
hipError_t launch_fft_col_fwd_reg16(const BoxPlan& p, int nb, const float2* T, const float* kin,
                                    const bf16c* in, int64_t ldin, const bf16c* prev,
                                    int64_t ldprev, bf16c* out, int64_t ldout, const Epilogue& ep,
                                    hipStream_t s) {
  return col_fwd_reg<float2, bf16c>(p, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
}

hipError_t launch_fft_plane_reg(const BoxPlan& p, int variant, int nb, const double* vscaled,
                                cplx* T, hipStream_t s) {
  return plane_reg<double2>(p, variant, nb, vscaled, T, s);
}
hipError_t launch_fft_plane_reg32(const BoxPlan& p, int variant, int nb, const float* vscaled,
                                  float2* T, hipStream_t s) {
  return plane_reg<float2>(p, variant, nb, vscaled, T, s);
}

hipError_t fft_reg_set_lds_limits(size_t bytes) {
  hipError_t e = set_plane_lds<double2>(bytes);
  if (e != hipSuccess) return e;
  return set_plane_lds<float2>(bytes);
}
