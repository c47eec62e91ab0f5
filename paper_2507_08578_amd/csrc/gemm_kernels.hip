// Complex FP64 matrix products on the gfx950 matrix cores (MFMA), used for
// the dense contractions of the path: the projections c = P^H psi ("cprj",
// section 5.2, Eq. ham-nl), the non-local expansion H psi += P (E c), the
// Gram matrices Y^H Y and Y^H (H Y), and the subspace rotations Y Q, Y U^{-1}.
//
// v_mfma_f64_16x16x4f64 operand layout on gfx950 (checked on the device):
//   A operand : lane l holds A[i = l % 16][k = l / 16]
//   B operand : lane l holds B[k = l / 16][j = l % 16]
//   result    : lane l, element r holds D[i = l / 16 + 4 r][j = l % 16]
// A complex product is four real MFMAs into two accumulators:
//   re += ar br - ai bi,  im += ar bi + ai br.
#include "pw_internal.h"

#include <algorithm>

typedef double d4 __attribute__((ext_vector_type(4)));
// complex value in registers and LDS as a native 2-vector: loads, stores and
// selects stay in registers (struct copies through cplx can leave the staging
// arrays in scratch memory)
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d2 ld2(const cplx* p) { return *reinterpret_cast<const d2*>(p); }

namespace {

constexpr int kBM = 64;       // workgroup tile rows
constexpr int kBN = 64;       // workgroup tile columns
constexpr int kThreads = 256; // 4 waves, 2 x 2, each a 32 x 32 sub-tile
constexpr int kKcNN = 8;      // complex K per LDS stage (A B)
constexpr int kKcCN = 16;     // complex K per LDS stage (A^H B)
constexpr int kTargetBlocks = 2048;

__device__ __forceinline__ void cmfma(d4& re, d4& im, double ar, double ai, double br, double bi) {
  re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, re, 0, 0, 0);
  re = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, re, 0, 0, 0);
  im = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, im, 0, 0, 0);
  im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, im, 0, 0, 0);
}

// C = alpha A B + beta C; A m x k (lda), B k x n (ldb), column-major.
// Workgroup tile (32 TM) x (32 TN): 4 waves in 2 x 2, each (16 TM) x (16 TN)
// built from TM x TN MFMA tiles; K staged KC complex at a time.
template <int TM, int TN, int KC>
__device__ __forceinline__ void gemm_nn_tile(int64_t M, int64_t N, int64_t K, double alpha,
                                             const cplx* __restrict__ A, int64_t lda,
                                             const cplx* __restrict__ B, int64_t ldb, double beta,
                                             cplx* __restrict__ C, int64_t ldc, int bx, int by) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  __shared__ d2 As[KC][BM];
  __shared__ d2 Bs[KC][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t i0 = (int64_t)by * BM, j0 = (int64_t)bx * BN;
  d4 accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      accr[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      acci[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const int lr = lane & 15, lk = lane >> 4;
  // global -> register prefetch of the next K stage overlaps this stage's MFMAs
  constexpr int QA = BM * KC / kThreads, QB = BN * KC / kThreads;
  static_assert(QA * kThreads == BM * KC && QB * kThreads == BN * KC, "tile split");
  d2 ra[QA], rb[QB];
  // Every lane loads from a clamped in-bounds address, so the K loop has no
  // branches (branches around the loads make the compiler copy the
  // accumulators out of and back into the matrix-core registers every
  // stage).  Rows of A past M and columns of B past N only feed results that
  // are not stored; B's rows past K are zeroed as the stage goes to LDS.
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int kk = e / BM, ii = e - kk * BM;
      ra[q] = ld2(A + min(i0 + ii, M - 1) + min(k0 + kk, K - 1) * lda);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / KC, kk = e - jj * KC;
      rb[q] = ld2(B + min(k0 + kk, K - 1) + min(j0 + jj, N - 1) * ldb);
    }
  };
  if (K > 0) fetch(0);
  for (int64_t k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int kk = e / BM, ii = e - kk * BM;
      As[kk][ii] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / KC, kk = e - jj * KC;
      Bs[kk][jj] = k0 + kk < K ? rb[q] : d2{0.0, 0.0};
    }
    __syncthreads();
    fetch(k0 + KC);   // after the last stage: clamped loads, never used
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      d2 a[TM], b[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t) a[t] = As[ks + lk][wi * 16 * TM + t * 16 + lr];
#pragma unroll
      for (int t = 0; t < TN; ++t) b[t] = Bs[ks + lk][wj * 16 * TN + t * 16 + lr];
#pragma unroll
      for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
          cmfma(accr[ti][tj], acci[ti][tj], a[ti].x, a[ti].y, b[tj].x, b[tj].y);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < TM; ++ti)
#pragma unroll
    for (int tj = 0; tj < TN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 16 * TM + ti * 16 + lk + 4 * r;
        const int64_t j = j0 + wj * 16 * TN + tj * 16 + lr;
        if (i < M && j < N) {
          cplx v = make_double2(alpha * accr[ti][tj][r], alpha * acci[ti][tj][r]);
          if (beta != 0.0) {
            const cplx c = C[i + j * ldc];
            v.x += beta * c.x;
            v.y += beta * c.y;
          }
          C[i + j * ldc] = v;
        }
      }
}

__device__ __forceinline__ void gemm_nn_body(int64_t M, int64_t N, int64_t K, double alpha,
                                             const cplx* __restrict__ A, int64_t lda,
                                             const cplx* __restrict__ B, int64_t ldb, double beta,
                                             cplx* __restrict__ C, int64_t ldc, int bx, int by) {
  gemm_nn_tile<2, 2, kKcNN>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bx, by);
}

// Workgroups are dealt round-robin over the device's XCDs (each with its own
// L2), block L to XCD L % kXcds.  The launches use 1D grids whose block order
// keeps the blocks that share operand tiles on one XCD and close in time.
constexpr int kXcds = 8;

// the tiles_n column tiles of a row panel on one XCD in a row;
// grid kXcds * tiles_n * ceil(tiles_m / kXcds)
__device__ __forceinline__ bool xcd_panel_tile(int L, int tiles_m, int tiles_n, int* bx, int* by) {
  const int x = L % kXcds, slot = L / kXcds;
  const int panel = x + kXcds * (slot / tiles_n);
  if (panel >= tiles_m) return false;
  *by = panel;
  *bx = slot % tiles_n;
  return true;
}

// all `per` tiles of one K split on one XCD in a row;
// grid kXcds * per * ceil(nsplit / kXcds); returns the tile index within the split
__device__ __forceinline__ bool xcd_split(int L, int per, int nsplit, int* tile, int* z) {
  const int x = L % kXcds, slot = L / kXcds;
  *z = x + kXcds * (slot / per);
  *tile = slot % per;
  return *z < nsplit;
}

__global__ void __launch_bounds__(kThreads)
k_gemm_nn(int64_t M, int64_t N, int64_t K, double alpha, const cplx* __restrict__ A, int64_t lda,
          const cplx* __restrict__ B, int64_t ldb, double beta, cplx* __restrict__ C, int64_t ldc,
          int tiles_m, int tiles_n) {
  int bx, by;
  if (!xcd_panel_tile(blockIdx.x, tiles_m, tiles_n, &bx, &by)) return;
  gemm_nn_body(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bx, by);
}

// 128 x 64 workgroup tiles for tall products (M = plane waves)
__global__ void __launch_bounds__(kThreads)
k_gemm_nn_tall(int64_t M, int64_t N, int64_t K, double alpha, const cplx* __restrict__ A,
               int64_t lda, const cplx* __restrict__ B, int64_t ldb, double beta,
               cplx* __restrict__ C, int64_t ldc, int tiles_m, int tiles_n) {
  int bx, by;
  if (!xcd_panel_tile(blockIdx.x, tiles_m, tiles_n, &bx, &by)) return;
  gemm_nn_tile<4, 2, kKcNN>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bx, by);
}

// Partial or final C = alpha diag(rowscale) A^H B over K range [kb, ke) of split z.
// A k x m (lda), B k x n (ldb).  Element (i, j) goes to out + z*zstride at
// (i - oi0) + (j - oj0) ldo.
__device__ __forceinline__ void gemm_cn_body(int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                             double alpha, const double* __restrict__ alpha_dev,
                                             const double* __restrict__ rowscale,
                                             const cplx* __restrict__ A, int64_t lda,
                                             const cplx* __restrict__ B, int64_t ldb, double beta,
                                             cplx* __restrict__ out, int64_t ldo, int64_t zstride,
                                             int bx, int by, int bz, int64_t oi0 = 0,
                                             int64_t oj0 = 0) {
  if (alpha_dev) alpha = alpha_dev[0];
  __shared__ d2 As[kKcCN][kBM + 1];
  __shared__ d2 Bs[kKcCN][kBN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t i0 = (int64_t)by * kBM, j0 = (int64_t)bx * kBN;
  const int64_t kb = (int64_t)bz * ksplit;
  const int64_t ke = min(K, kb + ksplit);
  d4 accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      acci[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int QA = kBM * kKcCN / kThreads, QB = kBN * kKcCN / kThreads;
  static_assert(QA * kThreads == kBM * kKcCN && QB * kThreads == kBN * kKcCN, "tile split");
  d2 ra[QA], rb[QB];
  // clamped loads, no branches in the K loop; B's rows past the split's
  // end are zeroed as the stage goes to LDS (as in gemm_nn_tile)
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int ii = e / kKcCN, kk = e - ii * kKcCN;
      ra[q] = ld2(A + min(k0 + kk, ke - 1) + min(i0 + ii, M - 1) * lda);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / kKcCN, kk = e - jj * kKcCN;
      rb[q] = ld2(B + min(k0 + kk, ke - 1) + min(j0 + jj, N - 1) * ldb);
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kKcCN) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int ii = e / kKcCN, kk = e - ii * kKcCN;
      As[kk][ii] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / kKcCN, kk = e - jj * kKcCN;
      Bs[kk][jj] = k0 + kk < ke ? rb[q] : d2{0.0, 0.0};
    }
    __syncthreads();
    fetch(k0 + kKcCN);
#pragma unroll
    for (int ks = 0; ks < kKcCN; ks += 4) {
      d2 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[ks + lk][wi * 32 + t * 16 + lr];
        b[t] = Bs[ks + lk][wj * 32 + t * 16 + lr];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)   // conj(A): negate the imaginary part
          cmfma(accr[ti][tj], acci[ti][tj], a[ti].x, -a[ti].y, b[tj].x, b[tj].y);
    }
    __syncthreads();
  }
  cplx* o = out + (int64_t)bz * zstride;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + ti * 16 + lk + 4 * r;
        const int64_t j = j0 + wj * 32 + tj * 16 + lr;
        if (i < M && j < N) {
          const double s = alpha * (rowscale ? rowscale[i] : 1.0);
          cplx v = make_double2(s * accr[ti][tj][r], s * acci[ti][tj][r]);
          if (beta != 0.0) {
            const cplx c = o[(i - oi0) + (j - oj0) * ldo];
            v.x += beta * c.x;
            v.y += beta * c.y;
          }
          o[(i - oi0) + (j - oj0) * ldo] = v;
        }
      }
}

__global__ void __launch_bounds__(kThreads)
k_gemm_cn(int64_t M, int64_t N, int64_t K, int64_t ksplit, double alpha,
          const double* __restrict__ alpha_dev, const double* __restrict__ rowscale,
          const cplx* __restrict__ A, int64_t lda, const cplx* __restrict__ B, int64_t ldb,
          double beta, cplx* __restrict__ out, int64_t ldo, int64_t zstride, int upper) {
  if (upper && blockIdx.y > blockIdx.x) return;   // tile strictly below the diagonal
  gemm_cn_body(M, N, K, ksplit, alpha, alpha_dev, rowscale, A, lda, B, ldb, beta, out, ldo, zstride,
               blockIdx.x, blockIdx.y, blockIdx.z);
}

// split partials of A^H B into work (ld M, split stride M N), XCD-grouped 1D grid
__global__ void __launch_bounds__(kThreads)
k_gemm_cn_split(int64_t M, int64_t N, int64_t K, int64_t ksplit, const cplx* __restrict__ A,
                int64_t lda, const cplx* __restrict__ B, int64_t ldb, cplx* __restrict__ work,
                int tiles_m, int tiles_n, int nsplit) {
  int t, z;
  if (!xcd_split(blockIdx.x, tiles_m * tiles_n, nsplit, &t, &z)) return;
  gemm_cn_body(M, N, K, ksplit, 1.0, nullptr, nullptr, A, lda, B, ldb, 0.0, work, M, M * N,
               t % tiles_n, t / tiles_n, z);
}

// C[i + j ldc] = alpha rowscale[i] sum_z work[z][i + j M], z in fixed order;
// Craw (may be null) also receives alpha sum_z work[z][i + j M] (ld ldraw).
__device__ __forceinline__ void splitk_reduce_body(int64_t M, int64_t N, int nsplit,
                                                   const cplx* __restrict__ work, double alpha,
                                                   const double* __restrict__ alpha_dev,
                                                   const double* __restrict__ rowscale,
                                                   double beta, cplx* __restrict__ C, int64_t ldc,
                                                   int bx, cplx* __restrict__ Craw = nullptr,
                                                   int64_t ldraw = 0) {
  if (alpha_dev) alpha = alpha_dev[0];
  const int64_t idx = (int64_t)bx * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t j = idx / M, i = idx - j * M;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < nsplit; ++z) {
    const cplx w = work[(int64_t)z * M * N + idx];
    re += w.x;
    im += w.y;
  }
  if (Craw) Craw[i + j * ldraw] = make_double2(alpha * re, alpha * im);
  const double s = alpha * (rowscale ? rowscale[i] : 1.0);
  cplx v = make_double2(s * re, s * im);
  if (beta != 0.0) {
    const cplx c = C[i + j * ldc];
    v.x += beta * c.x;
    v.y += beta * c.y;
  }
  C[i + j * ldc] = v;
}

__global__ void k_splitk_reduce(int64_t M, int64_t N, int nsplit, const cplx* __restrict__ work,
                                double alpha, const double* __restrict__ alpha_dev,
                                const double* __restrict__ rowscale, double beta,
                                cplx* __restrict__ C, int64_t ldc, cplx* __restrict__ Craw,
                                int64_t ldraw) {
  splitk_reduce_body(M, N, nsplit, work, alpha, alpha_dev, rowscale, beta, C, ldc, blockIdx.x, Craw,
                     ldraw);
}

// C[i + j ldc] = rowscale[i] R[i + j ldr] (the unsplit product's scaled copy)
__global__ void k_rowscale_copy(int64_t M, int64_t N, const cplx* __restrict__ R, int64_t ldr,
                                const double* __restrict__ rowscale, cplx* __restrict__ C,
                                int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t j = idx / M, i = idx - j * M;
  const cplx r = R[i + j * ldr];
  const double sc = rowscale ? rowscale[i] : 1.0;
  C[i + j * ldc] = make_double2(sc * r.x, sc * r.y);
}

// Hermitian products (M = N): only the nact = T (T + 1) / 2 tiles on and
// above the diagonal (T = ceil(M / 64)), enumerated column by column,
// t = bx (bx + 1) / 2 + by for by <= bx.  Split partials are packed per
// active tile: work[(z nact + t) 4096 + ii + 64 jj].
__device__ __forceinline__ void upper_tile(int t, int* by, int* bx) {
  int c = 0;
  while ((c + 1) * (c + 2) / 2 <= t) ++c;
  *bx = c;
  *by = t - c * (c + 1) / 2;
}

__global__ void __launch_bounds__(kThreads)
k_gemm_cn_upper(int64_t M, int64_t K, int64_t ksplit, int nact, int nsplit,
                const cplx* __restrict__ A, int64_t lda, const cplx* __restrict__ B, int64_t ldb,
                cplx* __restrict__ work) {
  int t, z, by, bx;
  if (!xcd_split(blockIdx.x, nact, nsplit, &t, &z)) return;
  upper_tile(t, &by, &bx);
  gemm_cn_body(M, M, K, ksplit, 1.0, nullptr, nullptr, A, lda, B, ldb, 0.0,
               work + (int64_t)t * kBM * kBN, kBM, (int64_t)nact * kBM * kBN, bx, by, z,
               (int64_t)by * kBM, (int64_t)bx * kBN);
}

// C[i + j ldc] = alpha sum_z (packed partials), fixed order, for the
// elements of the active tiles; the rest of C is not written.
__global__ void k_splitk_reduce_upper(int64_t M, int nsplit, int nact, const cplx* __restrict__ work,
                                      double alpha, cplx* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * M) return;
  const int64_t j = idx / M, i = idx - j * M;
  const int by = (int)(i / kBM), bx = (int)(j / kBN);
  if (by > bx) return;
  const int64_t t = (int64_t)bx * (bx + 1) / 2 + by;
  const int64_t loc = (i - (int64_t)by * kBM) + (j - (int64_t)bx * kBN) * kBM;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < nsplit; ++z) {
    const cplx w = work[((int64_t)z * nact + t) * kBM * kBN + loc];
    re += w.x;
    im += w.y;
  }
  C[i + j * ldc] = make_double2(alpha * re, alpha * im);
}

struct SplitPlan {
  int64_t tiles_m, tiles_n, nsplit, ksplit;
};

// The handle's split-K target as the FP64 products use it: values outside
// [1, kTargetBlocks] (the FP32 products accept more) mean kTargetBlocks, as in
// launch_gemm_cn, so fused and per-item launches split alike and stay within
// the workspace sized for kTargetBlocks.
__host__ __device__ inline int fp64_target(int target) {
  return (target < 1 || target > kTargetBlocks) ? kTargetBlocks : target;
}

__host__ __device__ inline SplitPlan split_plan(int64_t m, int64_t n, int64_t k, int target) {
  SplitPlan p;
  p.tiles_m = (m + kBM - 1) / kBM;
  p.tiles_n = (n + kBN - 1) / kBN;
  const int64_t tiles = p.tiles_m * p.tiles_n;
  int64_t want = (target + tiles - 1) / tiles;
  // at least two K stages per split (short splits keep small products latency-light)
  const int64_t maxs = (k + kKcCN * 2 - 1) / (kKcCN * 2) > 1 ? (k + kKcCN * 2 - 1) / (kKcCN * 2) : 1;
  want = want < maxs ? want : maxs;
  if (want >= 2 * kXcds) want -= want % kXcds;   // whole rounds of splits over the XCDs
  if (want < 1) want = 1;
  int64_t ks = (k + want - 1) / want;
  ks = ((ks + kKcCN - 1) / kKcCN) * kKcCN;
  p.ksplit = ks > kKcCN ? ks : kKcCN;
  p.nsplit = (k + p.ksplit - 1) / p.ksplit;
  if (p.nsplit < 1) p.nsplit = 1;
  return p;
}

// ---- fused-batch products (item from the launch's z or y coordinate)
struct CnArgs {
  int64_t M, N, K;
  const cplx* A;
  int64_t lda;
  const cplx* B;
  int64_t ldb;
  cplx* C;
  int64_t ldc;
  const double* rowscale;
  int target;
};

__device__ __forceinline__ CnArgs fused_cn_args(const ItemDev& d, int op, int sel_b) {
  CnArgs a;
  a.B = item_blk64(d, sel_b);
  a.ldb = d.npw;
  a.K = d.npw;
  a.lda = d.npw;
  if (op == GOP_PROJ) {
    a.M = d.nproj;
    a.N = d.nb;
    a.A = d.proj;
    a.C = d.cprj;
    a.ldc = d.nproj;
    a.rowscale = d.ekb;
    a.target = fp64_target(d.gemm_target);
  } else {
    a.M = d.nb;
    a.N = d.nb;
    a.A = d.y;
    a.C = d.sub0;
    a.ldc = d.nb;
    a.rowscale = nullptr;
    a.target = kTargetBlocks;
  }
  return a;
}

__global__ void __launch_bounds__(kThreads)
kb_gemm_cn(const ItemDev* __restrict__ D, int op, int sel_b, double alpha, int coef_step,
           int nsplit_max) {
  const int item = blockIdx.z / nsplit_max, zs = blockIdx.z - item * nsplit_max;
  const ItemDev& d = D[item];
  const CnArgs a = fused_cn_args(d, op, sel_b);
  if (a.M <= 0 || a.N <= 0) return;
  const SplitPlan p = split_plan(a.M, a.N, a.K, a.target);
  if (zs >= p.nsplit || (int64_t)blockIdx.y >= p.tiles_m || (int64_t)blockIdx.x >= p.tiles_n) return;
  const double* alpha_dev = coef_step >= 0 ? d.coef + 3 * coef_step : nullptr;
  if (p.nsplit == 1)
    gemm_cn_body(a.M, a.N, a.K, p.ksplit, alpha, alpha_dev, a.rowscale, a.A, a.lda, a.B, a.ldb, 0.0,
                 a.C, a.ldc, 0, blockIdx.x, blockIdx.y, 0);
  else
    gemm_cn_body(a.M, a.N, a.K, p.ksplit, 1.0, nullptr, nullptr, a.A, a.lda, a.B, a.ldb, 0.0,
                 d.gemm_work, a.M, a.M * a.N, blockIdx.x, blockIdx.y, zs);
}

__global__ void kb_splitk_reduce(const ItemDev* __restrict__ D, int op, int sel_b, double alpha,
                                 int coef_step) {
  const ItemDev& d = D[blockIdx.y];
  const CnArgs a = fused_cn_args(d, op, sel_b);
  if (a.M <= 0 || a.N <= 0) return;
  const SplitPlan p = split_plan(a.M, a.N, a.K, a.target);
  if (p.nsplit == 1) return;
  const double* alpha_dev = coef_step >= 0 ? d.coef + 3 * coef_step : nullptr;
  splitk_reduce_body(a.M, a.N, (int)p.nsplit, d.gemm_work, alpha, alpha_dev, a.rowscale, 0.0, a.C,
                     a.ldc, blockIdx.x);
}

__global__ void __launch_bounds__(kThreads)
kb_gemm_nn(const ItemDev* __restrict__ D, int op, int sel_a, int sel_c) {
  const ItemDev& d = D[blockIdx.z];
  int64_t M = d.npw, N = d.nb, K;
  const cplx* A;
  const cplx* B;
  int64_t ldb;
  cplx* C;
  double beta;
  if (op == GOP_NONLOCAL) {
    K = d.nproj; A = d.proj; B = d.cprj; ldb = d.nproj; C = item_blk64(d, sel_c); beta = 1.0;
  } else if (op == GOP_TRSM) {
    K = d.nb; A = d.y; B = d.dinv; ldb = d.nb; C = d.blk; beta = 0.0;
  } else {
    K = d.nb; A = item_blk64(d, sel_a); B = d.sub1; ldb = d.nb; C = d.blk; beta = 0.0;
  }
  if (K <= 0 || (int64_t)blockIdx.y * kBM >= M || (int64_t)blockIdx.x * kBN >= N) return;
  gemm_nn_body(M, N, K, 1.0, A, d.npw, B, ldb, beta, C, d.npw, blockIdx.x, blockIdx.y);
}

}  // namespace

size_t gemm_cn_work_elems(int64_t m, int64_t n, int64_t k) {
  const SplitPlan p = split_plan(m, n, k, kTargetBlocks);
  return p.nsplit > 1 ? (size_t)(p.nsplit * m * n) : 0;
}

hipError_t launch_gemm_cn(int64_t m, int64_t n, int64_t k, double alpha, const cplx* A, int64_t lda,
                          const cplx* B, int64_t ldb, cplx* C, int64_t ldc, const double* rowscale,
                          cplx* work, hipStream_t s, double beta, const double* alpha_dev,
                          int target, int upper, cplx* craw, int64_t ldraw) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (upper && (m != n || kBM != kBN || rowscale || alpha_dev || beta != 0.0))
    return hipErrorInvalidValue;
  if (craw && (upper || beta != 0.0 || ldraw < m)) return hipErrorInvalidValue;
  if (target < 1 || target > kTargetBlocks) target = kTargetBlocks;
  SplitPlan p = split_plan(m, n, k, target);
  const int64_t T = (m + kBM - 1) / kBM, nact = T * (T + 1) / 2;
  if (T == 1) upper = 0;   // a single tile: nothing to skip
  // packed splits that fit the workspace the full product would use (p.nsplit m n)
  const int64_t cap = p.nsplit * m * n / (nact * kBM * kBN);
  if (upper && work && p.nsplit > 1 && cap >= 1) {
    // as many splits as fill ~target blocks with the active tiles
    const int64_t maxs = (k + kKcCN * 2 - 1) / (kKcCN * 2) > 1 ? (k + kKcCN * 2 - 1) / (kKcCN * 2) : 1;
    int64_t want = (target + nact - 1) / nact;
    want = std::min(want, std::min(maxs, cap));
    if (want >= 2 * kXcds) want -= want % kXcds;
    if (want < 1) want = 1;
    int64_t ks = (k + want - 1) / want;
    ks = ((ks + kKcCN - 1) / kKcCN) * kKcCN;
    ks = std::max<int64_t>(ks, kKcCN);
    const int64_t ns = (k + ks - 1) / ks;
    hipLaunchKernelGGL(k_gemm_cn_upper, dim3((unsigned)(kXcds * nact * ((ns + kXcds - 1) / kXcds))),
                       dim3(kThreads), 0, s, m, k, ks, (int)nact, (int)ns, A, lda, B, ldb, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_splitk_reduce_upper, dim3((unsigned)((m * m + 255) / 256)), dim3(256), 0, s,
                       m, (int)ns, (int)nact, (const cplx*)work, alpha, C, ldc);
    return hipGetLastError();
  }
  if (!work) {   // no workspace: one split over the whole K range
    p.nsplit = 1;
    p.ksplit = k > 0 ? k : 1;
  }
  if (p.nsplit == 1) {
    dim3 grid(p.tiles_n, p.tiles_m, 1);
    if (craw) {   // unscaled product first, then its row-scaled copy
      hipLaunchKernelGGL(k_gemm_cn, grid, dim3(kThreads), 0, s, m, n, k, p.ksplit, alpha, alpha_dev,
                         (const double*)nullptr, A, lda, B, ldb, 0.0, craw, ldraw, (int64_t)0, 0);
      hipLaunchKernelGGL(k_rowscale_copy, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, s, m,
                         n, (const cplx*)craw, ldraw, rowscale, C, ldc);
      return hipGetLastError();
    }
    hipLaunchKernelGGL(k_gemm_cn, grid, dim3(kThreads), 0, s, m, n, k, p.ksplit, alpha, alpha_dev,
                       rowscale, A, lda, B, ldb, beta, C, ldc, (int64_t)0, upper);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)(kXcds * p.tiles_m * p.tiles_n * ((p.nsplit + kXcds - 1) / kXcds)));
  hipLaunchKernelGGL(k_gemm_cn_split, grid, dim3(kThreads), 0, s, m, n, k, p.ksplit, A, lda, B, ldb,
                     work, (int)p.tiles_m, (int)p.tiles_n, (int)p.nsplit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = m * n;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((tot + 255) / 256), dim3(256), 0, s, m, n,
                     (int)p.nsplit, (const cplx*)work, alpha, alpha_dev, rowscale, beta, C, ldc, craw,
                     ldraw);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(int64_t m, int64_t n, int64_t k, double alpha, const cplx* A, int64_t lda,
                          const cplx* B, int64_t ldb, double beta, cplx* C, int64_t ldc,
                          hipStream_t s, int tile) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int tn = (int)((n + kBN - 1) / kBN);
  if (tile == 1) {
    const int tm = (int)((m + 2 * kBM - 1) / (2 * kBM));
    const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
    hipLaunchKernelGGL(k_gemm_nn_tall, grid, dim3(kThreads), 0, s, m, n, k, alpha, A, lda, B, ldb,
                       beta, C, ldc, tm, tn);
    return hipGetLastError();
  }
  const int tm = (int)((m + kBM - 1) / kBM);
  const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
  hipLaunchKernelGGL(k_gemm_nn, grid, dim3(kThreads), 0, s, m, n, k, alpha, A, lda, B, ldb, beta,
                     C, ldc, tm, tn);
  return hipGetLastError();
}

int fused_cn_nsplit(int op, int64_t npw, int64_t nb, int64_t nproj, int target) {
  const SplitPlan p = op == GOP_PROJ ? split_plan(nproj, nb, npw, fp64_target(target))
                                     : split_plan(nb, nb, npw, kTargetBlocks);
  return (int)p.nsplit;
}

hipError_t launch_fused_gemm_cn(int nitems, int64_t m_max, int64_t n_max, int nsplit_max,
                                const ItemDev* D, int op, int sel_b, double alpha, int coef_step,
                                hipStream_t s) {
  if (nitems <= 0 || m_max <= 0 || n_max <= 0) return hipSuccess;
  dim3 grid((n_max + kBN - 1) / kBN, (m_max + kBM - 1) / kBM, nitems * nsplit_max);
  hipLaunchKernelGGL(kb_gemm_cn, grid, dim3(kThreads), 0, s, D, op, sel_b, alpha, coef_step,
                     nsplit_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nsplit_max == 1) return e;
  dim3 rgrid((m_max * n_max + 255) / 256, nitems);
  hipLaunchKernelGGL(kb_splitk_reduce, rgrid, dim3(256), 0, s, D, op, sel_b, alpha, coef_step);
  return hipGetLastError();
}

hipError_t launch_fused_gemm_nn(int nitems, int64_t m_max, int64_t n_max, const ItemDev* D, int op,
                                int sel_a, int sel_c, hipStream_t s) {
  if (nitems <= 0 || m_max <= 0 || n_max <= 0) return hipSuccess;
  dim3 grid((n_max + kBN - 1) / kBN, (m_max + kBM - 1) / kBM, nitems);
  hipLaunchKernelGGL(kb_gemm_nn, grid, dim3(kThreads), 0, s, D, op, sel_a, sel_c);
  return hipGetLastError();
}
