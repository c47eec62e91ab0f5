// Electron density of a block of bands (section 2.4, Eq. nandtau; the band
// sum of Eq. extfpmd_density in section 2.3 without its free-electron term):
//   n(r_j) = (1/Omega) sum_b w_b |psi_b(r_j)|^2,
// psi_b(r_j) the unnormalised backward transform (e^{+2 pi i m.j/N}) of the
// band's sphere coefficients, w_b its occupation times k-point weight.
//
// Route per chunk of bands (the column stage is the FFT route's own):
//   col_inv       : sphere -> T[b][j3][c], backward along N3;
//   density plane : one workgroup per (z-plane j3, band group g, part of the
//                   plane's rows) takes the chunk's bands b = g, g + ngroup,
//                   ...: backward along N2 on the plane's extent columns and
//                   along N1 on each of its rows,
//                   w_b |.|^2 summed in registers over those bands, then
//                   added once to the group's own partial array
//                   part[g][j3][j2][j1] (no atomics: each element has one
//                   writer);
//   reduce        : n = (1/Omega) sum_g part[g] in group order (+ n when
//                   accumulating over k-points).
// Every sum runs in a fixed order, so the result does not depend on timing.
#include "fft_common.h"

#include <algorithm>

using namespace pwfft;

namespace {

constexpr int kDensThreads = 512;

// Row parts per plane: a thread's sums (rows x R values) and one transform's
// registers must fit 256 VGPRs; from N = 128 on, the rows of a plane are
// split between two (N = 160: three) workgroups, each repeating the plane's
// N2 transforms.
constexpr int dens_parts(int n) { return n >= 160 ? 3 : n >= 128 ? 2 : 1; }
// Rows of every part but the last (which takes the rest): whole rounds of the
// 32 lane groups where that helps (N = 144: 64 + 80 rows, five rounds where
// 72 + 72 took six).
constexpr int dens_split(int n) { return n == 144 ? 64 : (n + dens_parts(n) - 1) / dens_parts(n); }

// Register plane kernel for N1 = N2 = N: each length-N transform in the
// registers of one lane group (pwfft::lane_fft_bwd); E[e][m2] in LDS holds
// the plane's extent columns between the two axes.  Workgroup (j3, g NH + h)
// takes row part h (rows h S .. h S + S - 1, the last part up to N - 1) of
// the bands of group g.  A thread owns rows h S + grp + k NGR (k < RPT) of its
// part and N1 outputs base .. base + R - 1 of each: the same elements for
// every band, so its sums stay in registers.
template <int N, int GMAX>
__global__ void __launch_bounds__(kDensThreads)
k_density_reg(BoxPlan P, const double2* __restrict__ tw, const double2* __restrict__ T, int nbc,
              const double* __restrict__ w, int ngroup, double* __restrict__ part, int add) {
  constexpr int G = lane_group(N, GMAX), R = N / G, TRS = N + 1;
  constexpr int NH = dens_parts(N), S = dens_split(N), NL = N - (NH - 1) * S;   // last part: NL rows
  constexpr int NR = S > NL ? S : NL;                                            // largest part
  constexpr int NGR = kDensThreads / G, RPT = (NR + NGR - 1) / NGR;
  extern __shared__ __align__(16) char lds_raw[];
  double2* E = reinterpret_cast<double2*>(lds_raw);                   // xr x TRS
  int* slot = reinterpret_cast<int*>(E + (size_t)P.xr * TRS);         // N entries
  const int tid = threadIdx.x, j3 = blockIdx.x, g = blockIdx.y / NH, h = blockIdx.y % NH;
  const int grp = tid / G, lb = tid % G, base = R * brev<G>(lb);
  const int row0 = h * S, row1 = h == NH - 1 ? N : row0 + S;
  for (int i = tid; i < N; i += kDensThreads) slot[i] = -1;
  __syncthreads();
  for (int e = tid; e < P.xr; e += kDensThreads) slot[P.ext_m1[e]] = e;
  LaneTw<R, G, double2> t;   // N1 = N2: one table serves both axes
  t.load(lb, tw);
  double acc[RPT][R];
#pragma unroll
  for (int k = 0; k < RPT; ++k)
#pragma unroll
    for (int q = 0; q < R; ++q) acc[k][q] = 0.0;
  for (int b = g; b < nbc; b += ngroup) {
    const double2* tp = T + ((size_t)b * P.n3 + j3) * P.ldt;
    __syncthreads();   // the previous band's rows are done with E; slot is complete
    for (int i = tid; i < P.xr * TRS; i += kDensThreads) E[i] = czero<double2>();
    __syncthreads();
    for (int c = tid; c < P.ncols; c += kDensThreads) E[P.col_e[c] * TRS + P.col_m2[c]] = tp[c];
    __syncthreads();
    for (int e = grp; e < P.xr; e += NGR) {   // backward along N2, in place
      double2 v[R];
      double2* col = E + e * TRS;
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = col[G * a + lb];
      lane_fft_bwd<R, G>(v, lb, t);
#pragma unroll
      for (int q = 0; q < R; ++q) col[q + base] = v[q];
    }
    __syncthreads();
    const double wb = w[b];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {           // backward along N1, |.|^2
      const int row = row0 + grp + k * NGR;
      if (row < row1) {                        // uniform over the lane group
        double2 v[R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
          const int s = slot[G * a + lb];
          v[a] = s >= 0 ? E[s * TRS + row] : czero<double2>();
        }
        lane_fft_bwd<R, G>(v, lb, t);
#pragma unroll
        for (int q = 0; q < R; ++q) acc[k][q] += wb * (v[q].x * v[q].x + v[q].y * v[q].y);
      }
    }
  }
  double* pp = part + ((size_t)g * P.n3 + j3) * N * N;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int row = row0 + grp + k * NGR;
    if (row < row1) {
      double* dst = pp + (size_t)row * N + base;
#pragma unroll
      for (int q = 0; q < R; ++q) dst[q] = (add ? dst[q] : 0.0) + acc[k][q];
    }
  }
}

// rho[i] = scale sum_{g < ngroup} part[g][i]  (+ rho[i] when accumulating);
// ngroup = 0 writes scale * 0.
__global__ void __launch_bounds__(256)
k_density_reduce(int64_t nbox, int ngroup, const double* __restrict__ part, double scale,
                 double* __restrict__ rho, int accumulate) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nbox;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < ngroup; ++g) s += part[(size_t)g * nbox + i];
    rho[i] = accumulate ? rho[i] + scale * s : scale * s;
  }
}

size_t density_reg_lds(const BoxPlan& p) {
  return (size_t)p.xr * (p.n2 + 1) * sizeof(double2) + (size_t)p.n1 * sizeof(int);
}

// the box lengths with register-resident transforms (the FFT route's list)
#define PW_DENSITY_SIZES(X) X(24) X(30) X(32) X(36) X(48) X(64) X(72) X(96) X(120) X(128) X(144) X(160)

}  // namespace

hipError_t launch_density_planes_reg(const BoxPlan& p, int nbc, const cplx* T, const double* w,
                                     int ngroup, double* part, int add, hipStream_t s) {
  if (p.n1 != p.n2) return hipErrorInvalidValue;
  const size_t lds = density_reg_lds(p);
#define CASE(N)                                                                                 \
  if (p.n1 == N) {                                                                              \
    hipLaunchKernelGGL((k_density_reg<N, 16>), dim3(p.n3, ngroup * dens_parts(N)),              \
                       dim3(kDensThreads), lds, s, p, p.ax1.tw, T, nbc, w, ngroup, part, add);  \
    return hipGetLastError();                                                                   \
  }
  PW_DENSITY_SIZES(CASE)
#undef CASE
  return hipErrorInvalidValue;
}

int density_row_parts(const BoxPlan& p) { return dens_parts(p.n1); }

bool density_reg_supported(const BoxPlan& p, size_t lds_limit) {
  if (p.n1 != p.n2) return false;
  bool ok = false;
#define CASE(N) if (p.n1 == N) ok = true;
  PW_DENSITY_SIZES(CASE)
#undef CASE
  return ok && density_reg_lds(p) <= lds_limit;
}

hipError_t density_set_lds_limit(size_t bytes) {
#define CASE(N)                                                                              \
  {                                                                                          \
    hipError_t e = hipFuncSetAttribute((const void*)k_density_reg<N, 16>,                   \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); \
    if (e != hipSuccess) return e;                                                           \
  }
  PW_DENSITY_SIZES(CASE)
#undef CASE
  return hipSuccess;
}

hipError_t launch_density_reduce(int64_t nbox, int ngroup, const double* part, double scale,
                                 double* rho, int accumulate, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((nbox + 255) / 256, 8192);
  hipLaunchKernelGGL(k_density_reduce, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                     nbox, ngroup, part, scale, rho, accumulate);
  return hipGetLastError();
}
