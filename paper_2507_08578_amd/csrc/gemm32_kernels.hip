// Complex matrix products of the low-precision filter path on the gfx950
// matrix cores, FP32 accumulation (the projections c = P^H psi and the
// non-local expansion H psi += P c of section 5.2, Eq. ham-nl, applied to
// complex64 blocks).
//
//   MODE_F32 : FP32 operands, each split exactly into three bfloat16 terms,
//              products on v_mfma_f32_16x16x32_bf16 (six term products per
//              real product, FP32 accumulation: the accuracy of FP32 products
//              at 6/16 of the FP32 MFMA time).  P^H psi (gemm_cn32_s3)
//              and P C (gemm_nn32_s3) read P's terms from copies made once
//              per handle; P^H psi splits psi per stage, and the reduction
//              that forms C stores C's terms.  Gram matrices Y^H Y
//              (gemm_cn32) split both operands per stage.  Without the copies
//              P C runs on v_mfma_f32_16x16x4f32 with FP32 operands.
//   MODE_BF16: v_mfma_f32_16x16x32_bf16, operands rounded to bfloat16
//              (round to nearest even) when the MFMA operands are formed from
//              the FP32 tiles staged in LDS.
// Operand layouts (checked on the device):
//   f32 16x16x4 : A lane l -> A[l%16][l/16], B lane l -> B[l/16][l%16]
//   bf16 16x16x32: A lane l -> A[l%16][8(l/16)+e], B lane l -> B[8(l/16)+e][l%16], e < 8
//   result (both): lane l, element r -> D[4(l/16) + r][l%16]
// A complex product is four real MFMAs into two accumulators:
//   re += ar br - ai bi,  im += ar bi + ai br.
#include "pw_internal.h"

#include <algorithm>

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBM = 64, kBN = 64, kThreads = 256;
constexpr int kTargetBlocks = 4096;
enum { MODE_F32 = 0, MODE_BF16 = 1 };

template <int MODE>
struct KC {
  static constexpr int value = MODE == MODE_F32 ? 16 : 32;   // complex K per LDS stage
};

__device__ __forceinline__ void f4zero(f4& a) { a = f4{0.f, 0.f, 0.f, 0.f}; }

// One complex K-stage of MFMAs for a wave's TM x TN sub-tiles.  As/Bs are LDS
// tiles [k][i] / [k][j] (row pitch pa/pb in float2); conjA negates Im(A).
template <int MODE, bool CONJA, int TM = 2, int TN = 2>
__device__ __forceinline__ void mfma_stage(const float2* As, int pa, const float2* Bs, int pb,
                                           int wi, int wj, int lane, f4 (&ar)[TM][TN],
                                           f4 (&ai)[TM][TN]) {
  const int lr = lane & 15, lk = lane >> 4;
  if constexpr (MODE == MODE_F32) {
#pragma unroll
    for (int ks = 0; ks < KC<MODE>::value; ks += 4) {
      float2 a[TM], b[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        a[t] = As[(ks + lk) * pa + wi * 16 * TM + t * 16 + lr];
        if (CONJA) a[t].y = -a[t].y;
      }
#pragma unroll
      for (int t = 0; t < TN; ++t) b[t] = Bs[(ks + lk) * pb + wj * 16 * TN + t * 16 + lr];
#pragma unroll
      for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
          ar[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti].x, b[tj].x, ar[ti][tj], 0, 0, 0);
          ar[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[ti].y, b[tj].y, ar[ti][tj], 0, 0, 0);
          ai[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti].x, b[tj].y, ai[ti][tj], 0, 0, 0);
          ai[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti].y, b[tj].x, ai[ti][tj], 0, 0, 0);
        }
    }
  } else {
    bf8 are[TM], aim[TM], anim[TM], bre[TN], bim[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float2 a = As[(8 * lk + e) * pa + wi * 16 * TM + t * 16 + lr];
        if (CONJA) a.y = -a.y;
        are[t][e] = (__bf16)a.x;
        aim[t][e] = (__bf16)a.y;
        anim[t][e] = (__bf16)(-a.y);
      }
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 b = Bs[(8 * lk + e) * pb + wj * 16 * TN + t * 16 + lr];
        bre[t][e] = (__bf16)b.x;
        bim[t][e] = (__bf16)b.y;
      }
    }
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < TN; ++tj) {
        ar[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(are[ti], bre[tj], ar[ti][tj], 0, 0, 0);
        ar[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anim[ti], bim[tj], ar[ti][tj], 0, 0, 0);
        ai[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(are[ti], bim[tj], ai[ti][tj], 0, 0, 0);
        ai[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aim[ti], bre[tj], ai[ti][tj], 0, 0, 0);
      }
  }
}

// C = alpha A B + beta C; A m x k (lda), B k x n (ldb), complex64 column-major.
// Workgroup tile (32 TM) x (32 TN), 4 waves in 2 x 2.
template <int MODE, int TM, int TN, class SC = float2>
__device__ __forceinline__ void gemm_nn32_tile(int64_t M, int64_t N, int64_t K, float alpha,
                                               const float2* __restrict__ A, int64_t lda,
                                               const float2* __restrict__ B, int64_t ldb,
                                               float beta, SC* __restrict__ C, int64_t ldc,
                                               int bx, int by) {
  constexpr int Kc = KC<MODE>::value;
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int PA = BM, PB = BN + 1;
  __shared__ float2 As[Kc * PA];
  __shared__ float2 Bs[Kc * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t i0 = (int64_t)by * BM, j0 = (int64_t)bx * BN;
  f4 ar[TM][TN], ai[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      f4zero(ar[a][b]);
      f4zero(ai[a][b]);
    }
  constexpr int QA = BM * Kc / kThreads, QB = BN * Kc / kThreads;
  static_assert(QA * kThreads == BM * Kc && QB * kThreads == BN * Kc, "tile split");
  float2 ra[QA], rb[QB];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int kk = e / BM, ii = e - kk * BM;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      ra[q] = (gi < M && gk < K) ? A[gi + gk * lda] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / Kc, kk = e - jj * Kc;
      const int64_t gk = k0 + kk, gj = j0 + jj;
      rb[q] = (gk < K && gj < N) ? B[gk + gj * ldb] : make_float2(0.f, 0.f);
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < K; k0 += Kc) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int kk = e / BM, ii = e - kk * BM;
      As[kk * PA + ii] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / Kc, kk = e - jj * Kc;
      Bs[kk * PB + jj] = rb[q];
    }
    __syncthreads();
    if (k0 + Kc < K) fetch(k0 + Kc);
    mfma_stage<MODE, false, TM, TN>(As, PA, Bs, PB, wi, wj, lane, ar, ai);
    __syncthreads();
  }
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < TM; ++ti)
#pragma unroll
    for (int tj = 0; tj < TN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 16 * TM + ti * 16 + 4 * lk + r;
        const int64_t j = j0 + wj * 16 * TN + tj * 16 + lr;
        if (i < M && j < N) {
          float2 v = make_float2(alpha * ar[ti][tj][r], alpha * ai[ti][tj][r]);
          if (beta != 0.f) {
            const float2 c = ld_c(C[i + j * ldc]);
            v.x += beta * c.x;
            v.y += beta * c.y;
          }
          C[i + j * ldc] = st_c<SC>(v);
        }
      }
}

template <int MODE>
__device__ __forceinline__ void gemm_nn32_body(int64_t M, int64_t N, int64_t K, float alpha,
                                               const float2* __restrict__ A, int64_t lda,
                                               const float2* __restrict__ B, int64_t ldb,
                                               float beta, float2* __restrict__ C, int64_t ldc,
                                               int bx, int by) {
  gemm_nn32_tile<MODE, 2, 2>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bx, by);
}

// Workgroups are dealt round-robin over the device's XCDs (each with its own
// L2), block L to XCD L % kXcds.  The launches below use 1D grids whose block
// order keeps the blocks that share operand tiles on one XCD and close in
// time, so those tiles come from that XCD's L2 rather than from HBM.
constexpr int kXcds = 8;

// Tall products: the tiles_n column tiles of a row panel on one XCD in a row
// (the panel's rows of A are read once); grid kXcds * tiles_n * ceil(tiles_m / kXcds).
__device__ __forceinline__ bool xcd_panel_tile(int L, int tiles_m, int tiles_n, int* bx, int* by) {
  const int x = L % kXcds, slot = L / kXcds;
  const int panel = x + kXcds * (slot / tiles_n);
  if (panel >= tiles_m) return false;
  *by = panel;
  *bx = slot % tiles_n;
  return true;
}

template <int MODE, class SC = float2>
__global__ void __launch_bounds__(kThreads)
k_gemm_nn32(int64_t M, int64_t N, int64_t K, float alpha, const float2* __restrict__ A,
            int64_t lda, const float2* __restrict__ B, int64_t ldb, float beta,
            SC* __restrict__ C, int64_t ldc, int tiles_m, int tiles_n) {
  int bx, by;
  if (!xcd_panel_tile(blockIdx.x, tiles_m, tiles_n, &bx, &by)) return;
  gemm_nn32_tile<MODE, 2, 2, SC>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bx, by);
}

template <int MODE, class SC = float2>
__global__ void __launch_bounds__(kThreads)
k_gemm_nn32_tall(int64_t M, int64_t N, int64_t K, float alpha, const float2* __restrict__ A,
                 int64_t lda, const float2* __restrict__ B, int64_t ldb, float beta,
                 SC* __restrict__ C, int64_t ldc, int tiles_m, int tiles_n) {
  int bx, by;
  if (!xcd_panel_tile(blockIdx.x, tiles_m, tiles_n, &bx, &by)) return;
  gemm_nn32_tile<MODE, 4, 2, SC>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bx, by);
}

// ---- P^H psi with FP32 operands on the bf16 matrix cores.
// x = h + m + l, h = bf16(x), m = bf16(x - h), l = bf16(x - h - m): both
// differences are exact in FP32, and the three terms hold x's 24 significant
// bits (bf16 has FP32's exponent range).  x y is formed from the six term
// products of weight >= 2^-16 (h h, h m, m h, h l, l h, m m); the dropped
// ones are below 2^-24 |x y|.
constexpr int kB3K = 32;                    // complex K per LDS stage
constexpr int kB3Pitch = kB3K + 8;          // bf16 per LDS row (80 B: rows spread over the banks)
constexpr int kB3Plane = 64 * kB3Pitch;     // one (term, part) plane of a 64-row operand tile

__device__ __forceinline__ f4 mfma6(const bf8 (&x)[3], const bf8 (&y)[3], f4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[2], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[1], acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[0], acc, 0, 0, 0);
}

// x = h + m + l as above (round to nearest even at each step).
__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r = x - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

// Split two consecutive-K complex values of one operand row and store the
// six bf16 pairs (term t, part re/im) at row `row`, K offset kq (even).
__device__ __forceinline__ void b3_store2(__bf16* L, int row, int kq, float4 v) {
  const float x[2][2] = {{v.x, v.z}, {v.y, v.w}};   // [re, im][k, k + 1]
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    bf2 h, m, l;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      __bf16 xh, xm, xl;
      split3(x[c][e], xh, xm, xl);
      h[e] = xh;
      m[e] = xm;
      l[e] = xl;
    }
    *reinterpret_cast<bf2*>(L + (0 * 2 + c) * kB3Plane + row * kB3Pitch + kq) = h;
    *reinterpret_cast<bf2*>(L + (1 * 2 + c) * kB3Plane + row * kB3Pitch + kq) = m;
    *reinterpret_cast<bf2*>(L + (2 * 2 + c) * kB3Plane + row * kB3Pitch + kq) = l;
  }
}

// Fragment of 16 rows (from row r0) for the 16x16x32 bf16 layout: lane
// (lr, lk) takes K values 8 lk .. 8 lk + 7 of row r0 + lr, for each term.
__device__ __forceinline__ void b3_frag(const __bf16* L, int c, int r0, int lr, int lk, bf8 (&f)[3]) {
#pragma unroll
  for (int t = 0; t < 3; ++t)
    f[t] = *reinterpret_cast<const bf8*>(L + (t * 2 + c) * kB3Plane + (r0 + lr) * kB3Pitch + 8 * lk);
}

// ---- Stored three-term operands.  A matrix with R rows and contraction
// length K is kept as chunks of 32 K values: chunk (r, s) holds row r, K
// 32 s .. 32 s + 31, as six planes of 32 bf16 in the order q = 2 t + c (term
// t, part c = re / im), 384 bytes; the chunks of a row follow each other:
//   X3[((r nst + s) 6 + q) 32 + k % 32],  nst = ceil(K / 32).
// Rows are padded to a multiple of 64 and K to 32 nst, with zeros, so the
// 64-row x 32-K tiles of the products are read without bounds checks.
constexpr int kS3Chunk = 6 * 32;   // bf16 per chunk

__host__ __device__ inline int64_t s3_nst(int64_t k) { return (k + 31) / 32; }
__host__ __device__ inline int64_t s3_rows(int64_t r) { return (r + 63) / 64 * 64; }
__device__ __forceinline__ int64_t s3_index(int64_t r, int64_t k, int q, int64_t nst) {
  return ((r * nst + (k >> 5)) * 6 + q) * 32 + (k & 31);
}

// Thread tid's part of a 64-row x 32-K tile: row tid / 4, K 8 (tid % 4) .. + 7
// of the six planes (16-byte pieces of its chunk; `chunk` points at that K
// offset of the row's current chunk).
__device__ __forceinline__ void s3_load(const __bf16* __restrict__ chunk, bf8 (&v)[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) v[q] = *reinterpret_cast<const bf8*>(chunk + q * 32);
}

__device__ __forceinline__ void s3_put(__bf16* L, int row, int k8, const bf8 (&v)[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) *reinterpret_cast<bf8*>(L + q * kB3Plane + row * kB3Pitch + k8) = v[q];
}

// Eight consecutive-K complex values of one row, split into the six planes.
__device__ __forceinline__ void s3_split8(const float2 (&x)[8], bf8 (&v)[6]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    __bf16 h, m, l;
    split3(x[e].x, h, m, l);
    v[0][e] = h;
    v[2][e] = m;
    v[4][e] = l;
    split3(x[e].y, h, m, l);
    v[1][e] = h;
    v[3][e] = m;
    v[5][e] = l;
  }
}

// Partial (split z over K) A^H B as gemm_cn32_body, FP32 operands in three
// bf16 terms.  Each operand tile (64 rows x 32 K) is staged as 1024 pairs of
// consecutive-K values: pair p = tid + 256 q (q < 4) is row p / 16, K 2 (p % 16),
// so the 16-byte loads of a wavefront cover four whole 256-byte row runs.
__device__ __forceinline__ void gemm_cn32_b3_body(int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                                  const float2* __restrict__ A, int64_t lda,
                                                  const float2* __restrict__ B, int64_t ldb,
                                                  float2* __restrict__ out, int bx, int by, int bz) {
  __shared__ __align__(16) __bf16 LA[6 * kB3Plane];
  __shared__ __align__(16) __bf16 LB[6 * kB3Plane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t i0 = (int64_t)by * kBM, j0 = (int64_t)bx * kBN;
  const int64_t kb = (int64_t)bz * ksplit;
  const int64_t ke = min(K, kb + ksplit);
  const int kq = (tid & 15) * 2;
  // acc[0] = Re(conj(a) b) = ar br + ai bi, acc[1] = ar bi, acc[2] = ai br
  f4 acc[3][2][2];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) f4zero(acc[q][a][b]);
  float4 ra[4], rb[4];
  // (k, k + 1) of one row (columns of odd length are only 8-byte aligned)
  auto pair = [&](const float2* __restrict__ X, int64_t ld, int64_t row, int64_t rows,
                  int64_t gk) -> float4 {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    const float2* src = X + gk + row * ld;
    if (row < rows && gk < ke) {
      const float2 a = src[0];
      v.x = a.x;
      v.y = a.y;
    }
    if (row < rows && gk + 1 < ke) {
      const float2 b = src[1];
      v.z = b.x;
      v.w = b.y;
    }
    return v;
  };
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = (tid >> 4) + 16 * q;
      ra[q] = pair(A, lda, i0 + r, M, k0 + kq);
      rb[q] = pair(B, ldb, j0 + r, N, k0 + kq);
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kB3K) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      b3_store2(LA, (tid >> 4) + 16 * q, kq, ra[q]);
      b3_store2(LB, (tid >> 4) + 16 * q, kq, rb[q]);
    }
    __syncthreads();
    if (k0 + kB3K < ke) fetch(k0 + kB3K);
    bf8 a[2][2][3], b[2][2][3];   // [tile][re, im][term]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        b3_frag(LA, c, wi * 32 + t * 16, lr, lk, a[t][c]);
        b3_frag(LB, c, wj * 32 + t * 16, lr, lk, b[t][c]);
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        acc[0][ti][tj] = mfma6(a[ti][0], b[tj][0], acc[0][ti][tj]);
        acc[0][ti][tj] = mfma6(a[ti][1], b[tj][1], acc[0][ti][tj]);
        acc[1][ti][tj] = mfma6(a[ti][0], b[tj][1], acc[1][ti][tj]);
        acc[2][ti][tj] = mfma6(a[ti][1], b[tj][0], acc[2][ti][tj]);
      }
    __syncthreads();
  }
  float2* o = out + (int64_t)bz * M * N;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + ti * 16 + 4 * lk + r;
        const int64_t j = j0 + wj * 32 + tj * 16 + lr;
        if (i < M && j < N)
          o[i + j * M] = make_float2(acc[0][ti][tj][r], acc[1][ti][tj][r] - acc[2][ti][tj][r]);
      }
}

// Partial (split z over K) A^H B with A given as its stored three-term copy
// A3 (rows = the M columns of A, contraction K; the chunk layout above) and B
// (K x N, ldb) complex64, split per stage: thread tid stages chunk row tid / 4
// of A3 and column tid / 4 of B, K 8 (tid % 4) .. + 7 of the stage.  The same
// products as gemm_cn32_b3_body in the same order, so the same result.
// Columns j >= N are read from column N - 1 (they feed only outputs that are
// not stored); K beyond ke reads zero from B.
__device__ __forceinline__ void gemm_cn32_s3_body(int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                                  const __bf16* __restrict__ A3,
                                                  const float2* __restrict__ B, int64_t ldb,
                                                  float2* __restrict__ out, int bx, int by, int bz) {
  __shared__ __align__(16) __bf16 LA[6 * kB3Plane];
  __shared__ __align__(16) __bf16 LB[6 * kB3Plane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int row = tid >> 2, k8 = (tid & 3) * 8;
  const int64_t i0 = (int64_t)by * kBM, j0 = (int64_t)bx * kBN;
  const int64_t kb = (int64_t)bz * ksplit;
  const int64_t ke = min(K, kb + ksplit);
  const int64_t nst = s3_nst(K);
  f4 acc[3][2][2];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) f4zero(acc[q][a][b]);
  const __bf16* pa = A3 + ((i0 + row) * nst + (kb >> 5)) * kS3Chunk + k8;
  const int64_t col = min(j0 + row, N - 1);
  const float2* pb = B + col * ldb + kb + k8;
  bf8 ra[6];
  float2 xb[8];
  auto fetch = [&](int64_t k0) {
    s3_load(pa, ra);
    pa += kS3Chunk;
    if (k0 + kB3K <= ke) {
#pragma unroll
      for (int e = 0; e < 8; ++e) xb[e] = pb[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        xb[e] = k0 + k8 + e < ke ? pb[e] : make_float2(0.f, 0.f);
    }
    pb += kB3K;
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kB3K) {
    s3_put(LA, row, k8, ra);
    {
      bf8 vb[6];
      s3_split8(xb, vb);
      s3_put(LB, row, k8, vb);
    }
    __syncthreads();
    if (k0 + kB3K < ke) fetch(k0 + kB3K);
    bf8 a[2][2][3], b[2][2][3];   // [tile][re, im][term]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        b3_frag(LA, c, wi * 32 + t * 16, lr, lk, a[t][c]);
        b3_frag(LB, c, wj * 32 + t * 16, lr, lk, b[t][c]);
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        acc[0][ti][tj] = mfma6(a[ti][0], b[tj][0], acc[0][ti][tj]);
        acc[0][ti][tj] = mfma6(a[ti][1], b[tj][1], acc[0][ti][tj]);
        acc[1][ti][tj] = mfma6(a[ti][0], b[tj][1], acc[1][ti][tj]);
        acc[2][ti][tj] = mfma6(a[ti][1], b[tj][0], acc[2][ti][tj]);
      }
    __syncthreads();
  }
  float2* o = out + (int64_t)bz * M * N;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + ti * 16 + 4 * lk + r;
        const int64_t j = j0 + wj * 32 + tj * 16 + lr;
        if (i < M && j < N)
          o[i + j * M] = make_float2(acc[0][ti][tj][r], acc[1][ti][tj][r] - acc[2][ti][tj][r]);
      }
}

// Partial (split z over K) A^H B; A k x m (lda), B k x n (ldb); out ld = M.
template <int MODE, class SB = float2>
__device__ __forceinline__ void gemm_cn32_body(int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                               const float2* __restrict__ A, int64_t lda,
                                               const SB* __restrict__ B, int64_t ldb,
                                               float2* __restrict__ out, int bx, int by, int bz) {
  if constexpr (MODE == MODE_F32) {
    static_assert(sizeof(SB) == sizeof(float2), "FP32 operands only");
    gemm_cn32_b3_body(M, N, K, ksplit, A, lda, B, ldb, out, bx, by, bz);
    return;
  }
  constexpr int Kc = KC<MODE>::value;
  constexpr int PA = kBM + 1, PB = kBN + 1;
  __shared__ float2 As[Kc * PA];
  __shared__ float2 Bs[Kc * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t i0 = (int64_t)by * kBM, j0 = (int64_t)bx * kBN;
  const int64_t kb = (int64_t)bz * ksplit;
  const int64_t ke = min(K, kb + ksplit);
  f4 ar[2][2], ai[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      f4zero(ar[a][b]);
      f4zero(ai[a][b]);
    }
  constexpr int QA = kBM * Kc / kThreads, QB = kBN * Kc / kThreads;
  static_assert(QA * kThreads == kBM * Kc && QB * kThreads == kBN * Kc, "tile split");
  float2 ra[QA], rb[QB];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int ii = e / Kc, kk = e - ii * Kc;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      ra[q] = (gi < M && gk < ke) ? A[gk + gi * lda] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / Kc, kk = e - jj * Kc;
      const int64_t gj = j0 + jj, gk = k0 + kk;
      rb[q] = (gj < N && gk < ke) ? ld_c(B[gk + gj * ldb]) : make_float2(0.f, 0.f);
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += Kc) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * kThreads;
      const int ii = e / Kc, kk = e - ii * Kc;
      As[kk * PA + ii] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * kThreads;
      const int jj = e / Kc, kk = e - jj * Kc;
      Bs[kk * PB + jj] = rb[q];
    }
    __syncthreads();
    if (k0 + Kc < ke) fetch(k0 + Kc);
    mfma_stage<MODE, true>(As, PA, Bs, PB, wi, wj, lane, ar, ai);
    __syncthreads();
  }
  float2* o = out + (int64_t)bz * M * N;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + ti * 16 + 4 * lk + r;
        const int64_t j = j0 + wj * 32 + tj * 16 + lr;
        if (i < M && j < N) o[i + j * M] = make_float2(ar[ti][tj][r], ai[ti][tj][r]);
      }
}

// ---- P C with FP32 operands on the bf16 matrix cores, both operands in
// their stored three-term copies: A3 (rows = the M rows of P, contraction K)
// and B3 (rows = the N columns of C, contraction K), formed once per handle
// (P) and by the reduction that produces C.  Nothing is split or bounds-
// checked in the K loop: every stage stages six 16-byte pieces of each.

// out = alpha P C + beta out on a 64 x 64 tile (by: rows of P, bx: columns of C).
__device__ __forceinline__ void gemm_nn32_s3_body(int64_t M, int64_t N, int64_t K, float alpha,
                                                  const __bf16* __restrict__ A3,
                                                  const __bf16* __restrict__ B3, float beta,
                                                  float2* __restrict__ C, int64_t ldc, int bx,
                                                  int by) {
  __shared__ __align__(16) __bf16 LA[6 * kB3Plane];
  __shared__ __align__(16) __bf16 LB[6 * kB3Plane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int row = tid >> 2, k8 = (tid & 3) * 8;
  const int64_t i0 = (int64_t)by * kBM, j0 = (int64_t)bx * kBN;
  const int64_t nst = s3_nst(K);
  // acc[0] = ar br, acc[1] = ai bi, acc[2] = ar bi + ai br
  f4 acc[3][2][2];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) f4zero(acc[q][a][b]);
  const __bf16* pa = A3 + (i0 + row) * nst * kS3Chunk + k8;
  const __bf16* pb = B3 + (j0 + row) * nst * kS3Chunk + k8;
  bf8 ra[6], rb[6];
  s3_load(pa, ra);
  s3_load(pb, rb);
  for (int64_t st = 0; st < nst; ++st) {
    s3_put(LA, row, k8, ra);
    s3_put(LB, row, k8, rb);
    __syncthreads();
    if (st + 1 < nst) {
      pa += kS3Chunk;
      pb += kS3Chunk;
      s3_load(pa, ra);
      s3_load(pb, rb);
    }
    bf8 a[2][2][3], b[2][2][3];   // [tile][re, im][term]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        b3_frag(LA, c, wi * 32 + t * 16, lr, lk, a[t][c]);
        b3_frag(LB, c, wj * 32 + t * 16, lr, lk, b[t][c]);
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        acc[0][ti][tj] = mfma6(a[ti][0], b[tj][0], acc[0][ti][tj]);
        acc[1][ti][tj] = mfma6(a[ti][1], b[tj][1], acc[1][ti][tj]);
        acc[2][ti][tj] = mfma6(a[ti][0], b[tj][1], acc[2][ti][tj]);
        acc[2][ti][tj] = mfma6(a[ti][1], b[tj][0], acc[2][ti][tj]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + ti * 16 + 4 * lk + r;
        const int64_t j = j0 + wj * 32 + tj * 16 + lr;
        if (i < M && j < N) {
          float2 v = make_float2(alpha * (acc[0][ti][tj][r] - acc[1][ti][tj][r]),
                                 alpha * acc[2][ti][tj][r]);
          if (beta != 0.f) {
            const float2 c = C[i + j * ldc];
            v.x += beta * c.x;
            v.y += beta * c.y;
          }
          C[i + j * ldc] = v;
        }
      }
}

__global__ void __launch_bounds__(kThreads)
k_gemm_nn32_s3(int64_t M, int64_t N, int64_t K, float alpha, const __bf16* __restrict__ A3,
               const __bf16* __restrict__ B3, float beta, float2* __restrict__ C, int64_t ldc,
               int tiles_m, int tiles_n) {
  int bx, by;
  if (!xcd_panel_tile(blockIdx.x, tiles_m, tiles_n, &bx, &by)) return;
  gemm_nn32_s3_body(M, N, K, alpha, A3, B3, beta, C, ldc, bx, by);
}

// The stored three-term copy X3 of a complex64 matrix X (R rows, contraction
// K; element (r, k) at X[r sr + k sk]), all s3_rows(R) x 32 nst entries
// written (zero padding included).  A workgroup per 64-row panel and K chunk
// (grid-strided over the chunks), through LDS: reads run along whichever
// index is contiguous in X, writes along K within the chunks.
__global__ void __launch_bounds__(256)
k_split3_s3(int64_t R, int64_t K, const float2* __restrict__ X, int64_t sr, int64_t sk,
            __bf16* __restrict__ X3) {
  __shared__ float2 t[64][33];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int64_t nst = s3_nst(K);
  for (int64_t s = blockIdx.y; s < nst; s += gridDim.y) {
    const int64_t k0 = s * 32;
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int rr = sr == 1 ? (e & 63) : (e >> 5);
      const int kk = sr == 1 ? (e >> 6) : (e & 31);
      const int64_t r = r0 + rr, k = k0 + kk;
      t[rr][kk] = (r < R && k < K) ? X[r * sr + k * sk] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int rr = e >> 5, kk = e & 31;
      const float2 v = t[rr][kk];
      __bf16* o = X3 + ((r0 + rr) * nst + s) * kS3Chunk + kk;
      __bf16 h, m, l;
      split3(v.x, h, m, l);
      o[0 * 32] = h;
      o[2 * 32] = m;
      o[4 * 32] = l;
      split3(v.y, h, m, l);
      o[1 * 32] = h;
      o[3 * 32] = m;
      o[5 * 32] = l;
    }
    __syncthreads();
  }
}

// Split-K products: all tiles of one K split on one XCD in a row; they stream
// the same K range of both operands together, so each K stage is fetched
// once per XCD.  Grid kXcds * tiles_m * tiles_n * ceil(nsplit / kXcds).
__device__ __forceinline__ bool xcd_split_tile(int L, int tiles_m, int tiles_n, int nsplit,
                                               int* bx, int* by, int* bz) {
  const int x = L % kXcds, slot = L / kXcds;
  const int per = tiles_m * tiles_n;
  const int z = x + kXcds * (slot / per);
  if (z >= nsplit) return false;
  const int r = slot % per;
  *by = r / tiles_n;
  *bx = r % tiles_n;
  *bz = z;
  return true;
}

template <int MODE, class SB = float2>
__global__ void __launch_bounds__(kThreads)
k_gemm_cn32(int64_t M, int64_t N, int64_t K, int64_t ksplit, const float2* __restrict__ A,
            int64_t lda, const SB* __restrict__ B, int64_t ldb, float2* __restrict__ out,
            int tiles_m, int tiles_n, int nsplit) {
  int bx, by, bz;
  if (!xcd_split_tile(blockIdx.x, tiles_m, tiles_n, nsplit, &bx, &by, &bz)) return;
  gemm_cn32_body<MODE, SB>(M, N, K, ksplit, A, lda, B, ldb, out, bx, by, bz);
}

__global__ void __launch_bounds__(kThreads)
k_gemm_cn32_s3(int64_t M, int64_t N, int64_t K, int64_t ksplit, const __bf16* __restrict__ A3,
               const float2* __restrict__ B, int64_t ldb, float2* __restrict__ out, int tiles_m,
               int tiles_n, int nsplit) {
  int bx, by, bz;
  if (!xcd_split_tile(blockIdx.x, tiles_m, tiles_n, nsplit, &bx, &by, &bz)) return;
  gemm_cn32_s3_body(M, N, K, ksplit, A3, B, ldb, out, bx, by, bz);
}

// C[i + j ldc] = alpha rowscale[i] sum_z work[z][i + j M] (FP64 sum, fixed order), rounded;
// with c3, also the stored three-term copy of the rounded C^T (rows = the N
// columns of C, contraction M: the B operand of gemm_nn32_s3_body).
__device__ __forceinline__ void splitk_reduce32_body(int64_t M, int64_t N, int nsplit,
                                                     const float2* __restrict__ work, double alpha,
                                                     const double* __restrict__ alpha_dev,
                                                     const double* __restrict__ rowscale,
                                                     float2* __restrict__ C, int64_t ldc,
                                                     __bf16* __restrict__ c3, int bx) {
  if (alpha_dev) alpha = alpha_dev[0];
  const int64_t idx = (int64_t)bx * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t j = idx / M, i = idx - j * M;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < nsplit; ++z) {
    const float2 w = work[(int64_t)z * M * N + idx];
    re += w.x;
    im += w.y;
  }
  const double s = alpha * (rowscale ? rowscale[i] : 1.0);
  const float2 v = make_float2((float)(s * re), (float)(s * im));
  C[i + j * ldc] = v;
  if (c3) {
    __bf16* o = c3 + s3_index(j, i, 0, s3_nst(M));
    __bf16 h, m, l;
    split3(v.x, h, m, l);
    o[0 * 32] = h;
    o[2 * 32] = m;
    o[4 * 32] = l;
    split3(v.y, h, m, l);
    o[1 * 32] = h;
    o[3 * 32] = m;
    o[5 * 32] = l;
  }
}

__global__ void k_splitk_reduce32(int64_t M, int64_t N, int nsplit, const float2* __restrict__ work,
                                  double alpha, const double* __restrict__ alpha_dev,
                                  const double* __restrict__ rowscale, float2* __restrict__ C,
                                  int64_t ldc, __bf16* __restrict__ c3) {
  splitk_reduce32_body(M, N, nsplit, work, alpha, alpha_dev, rowscale, C, ldc, c3, blockIdx.x);
}

struct SplitPlan {
  int64_t tiles_m, tiles_n, nsplit, ksplit;
};

template <int MODE>
__host__ __device__ inline SplitPlan split_plan32(int64_t m, int64_t n, int64_t k, int target) {
  constexpr int Kc = 32;   // complex K per LDS stage of both P^H psi kernels
  SplitPlan p;
  p.tiles_m = (m + kBM - 1) / kBM;
  p.tiles_n = (n + kBN - 1) / kBN;
  const int64_t tiles = p.tiles_m * p.tiles_n;
  int64_t want = (target + tiles - 1) / tiles;
  // at least two K stages per split (short splits keep small products latency-light)
  const int64_t maxs = (k + Kc * 2 - 1) / (Kc * 2) > 1 ? (k + Kc * 2 - 1) / (Kc * 2) : 1;
  want = want < maxs ? want : maxs;
  if (want >= 2 * kXcds) want -= want % kXcds;   // whole rounds of splits over the XCDs
  if (want < 1) want = 1;
  int64_t ks = (k + want - 1) / want;
  ks = ((ks + Kc - 1) / Kc) * Kc;
  p.ksplit = ks > Kc ? ks : Kc;
  p.nsplit = (k + p.ksplit - 1) / p.ksplit;
  if (p.nsplit < 1) p.nsplit = 1;
  return p;
}

// ---- fused-batch products (FP32 / bf16 operands): P^H X into work32, reduced into
// cprj32; X += P cprj32
template <int MODE>
__global__ void __launch_bounds__(kThreads)
kb_gemm_cn32(const ItemDev* __restrict__ D, int sel_b, int nsplit_max) {
  const int item = blockIdx.z / nsplit_max, zs = blockIdx.z - item * nsplit_max;
  const ItemDev& d = D[item];
  if (d.nproj <= 0) return;
  const SplitPlan p = split_plan32<MODE>(d.nproj, d.nb, d.npw, d.gemm_target);
  if (zs >= p.nsplit || (int64_t)blockIdx.y >= p.tiles_m || (int64_t)blockIdx.x >= p.tiles_n) return;
  if constexpr (MODE == MODE_F32)
    gemm_cn32_s3_body(d.nproj, d.nb, d.npw, p.ksplit, reinterpret_cast<const __bf16*>(d.proj3c),
                      item_blk32(d, sel_b), d.npw, d.work32, blockIdx.x, blockIdx.y, zs);
  else
    gemm_cn32_body<MODE>(d.nproj, d.nb, d.npw, p.ksplit, d.proj32, d.npw, item_blk32(d, sel_b),
                         d.npw, d.work32, blockIdx.x, blockIdx.y, zs);
}

template <int MODE>
__global__ void kb_splitk_reduce32(const ItemDev* __restrict__ D, double alpha, int coef_step) {
  const ItemDev& d = D[blockIdx.y];
  if (d.nproj <= 0) return;
  const SplitPlan p = split_plan32<MODE>(d.nproj, d.nb, d.npw, d.gemm_target);
  const double* alpha_dev = coef_step >= 0 ? d.coef + 3 * coef_step : nullptr;
  splitk_reduce32_body(d.nproj, d.nb, (int)p.nsplit, d.work32, alpha, alpha_dev, d.ekb, d.cprj32,
                       d.nproj, MODE == MODE_F32 ? reinterpret_cast<__bf16*>(d.cprj3) : nullptr,
                       blockIdx.x);
}

template <int MODE>
__global__ void __launch_bounds__(kThreads)
kb_gemm_nn32(const ItemDev* __restrict__ D, int sel_c) {
  const ItemDev& d = D[blockIdx.z];
  if (d.nproj <= 0 || (int64_t)blockIdx.y * kBM >= d.npw || (int64_t)blockIdx.x * kBN >= d.nb) return;
  if constexpr (MODE == MODE_F32)
    gemm_nn32_s3_body(d.npw, d.nb, d.nproj, 1.f, reinterpret_cast<const __bf16*>(d.proj3),
                      reinterpret_cast<const __bf16*>(d.cprj3), 1.f, item_blk32(d, sel_c), d.npw,
                      blockIdx.x, blockIdx.y);
  else
    gemm_nn32_body<MODE>(d.npw, d.nb, d.nproj, 1.f, d.proj32, d.npw, d.cprj32, d.nproj, 1.f,
                         item_blk32(d, sel_c), d.npw, blockIdx.x, blockIdx.y);
}

}  // namespace

size_t gemm_cn32_work_elems(int64_t m, int64_t n, int64_t k, int bf16) {
  const SplitPlan p = bf16 ? split_plan32<MODE_BF16>(m, n, k, kTargetBlocks)
                           : split_plan32<MODE_F32>(m, n, k, kTargetBlocks);
  return (size_t)(p.nsplit * m * n);
}

hipError_t launch_gemm_cn32(int bf16, int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                            int64_t lda, const float2* B, int64_t ldb, float2* C, int64_t ldc,
                            const double* rowscale, float2* work, hipStream_t s,
                            const double* alpha_dev, int target) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (target < 1 || target > kTargetBlocks) target = kTargetBlocks;
  const SplitPlan p = bf16 ? split_plan32<MODE_BF16>(m, n, k, target)
                           : split_plan32<MODE_F32>(m, n, k, target);
  const dim3 grid((unsigned)(kXcds * p.tiles_m * p.tiles_n * ((p.nsplit + kXcds - 1) / kXcds)));
  if (bf16)
    hipLaunchKernelGGL(k_gemm_cn32<MODE_BF16>, grid, dim3(kThreads), 0, s, m, n, k, p.ksplit, A, lda,
                       B, ldb, work, (int)p.tiles_m, (int)p.tiles_n, (int)p.nsplit);
  else
    hipLaunchKernelGGL(k_gemm_cn32<MODE_F32>, grid, dim3(kThreads), 0, s, m, n, k, p.ksplit, A, lda,
                       B, ldb, work, (int)p.tiles_m, (int)p.tiles_n, (int)p.nsplit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = m * n;
  hipLaunchKernelGGL(k_splitk_reduce32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, n,
                     (int)p.nsplit, (const float2*)work, alpha, alpha_dev, rowscale, C, ldc,
                     (__bf16*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gemm_cn32_s3(int64_t m, int64_t n, int64_t k, double alpha, const uint16_t* a3,
                               const float2* B, int64_t ldb, float2* C, int64_t ldc,
                               const double* rowscale, float2* work, hipStream_t s,
                               const double* alpha_dev, int target, uint16_t* c3) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (target < 1 || target > kTargetBlocks) target = kTargetBlocks;
  const SplitPlan p = split_plan32<MODE_F32>(m, n, k, target);
  const dim3 grid((unsigned)(kXcds * p.tiles_m * p.tiles_n * ((p.nsplit + kXcds - 1) / kXcds)));
  hipLaunchKernelGGL(k_gemm_cn32_s3, grid, dim3(kThreads), 0, s, m, n, k, p.ksplit,
                     reinterpret_cast<const __bf16*>(a3), B, ldb, work, (int)p.tiles_m,
                     (int)p.tiles_n, (int)p.nsplit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = m * n;
  hipLaunchKernelGGL(k_splitk_reduce32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, n,
                     (int)p.nsplit, (const float2*)work, alpha, alpha_dev, rowscale, C, ldc,
                     reinterpret_cast<__bf16*>(c3));
  return hipGetLastError();
}

hipError_t launch_gemm_cn32_s16(int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                                int64_t lda, const bf16c* B, int64_t ldb, float2* C, int64_t ldc,
                                const double* rowscale, float2* work, hipStream_t s,
                                const double* alpha_dev, int target) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (target < 1 || target > kTargetBlocks) target = kTargetBlocks;
  const SplitPlan p = split_plan32<MODE_BF16>(m, n, k, target);
  const dim3 grid((unsigned)(kXcds * p.tiles_m * p.tiles_n * ((p.nsplit + kXcds - 1) / kXcds)));
  hipLaunchKernelGGL((k_gemm_cn32<MODE_BF16, bf16c>), grid, dim3(kThreads), 0, s, m, n, k,
                     p.ksplit, A, lda, B, ldb, work, (int)p.tiles_m, (int)p.tiles_n,
                     (int)p.nsplit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = m * n;
  hipLaunchKernelGGL(k_splitk_reduce32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, n,
                     (int)p.nsplit, (const float2*)work, alpha, alpha_dev, rowscale, C, ldc,
                     (__bf16*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gemm_nn32_s16(int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                                int64_t lda, const float2* B, int64_t ldb, double beta, bf16c* C,
                                int64_t ldc, hipStream_t s, int tile) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int tn = (int)((n + kBN - 1) / kBN);
  if (tile == 1) {
    const int tm = (int)((m + 2 * kBM - 1) / (2 * kBM));
    const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
    hipLaunchKernelGGL((k_gemm_nn32_tall<MODE_BF16, bf16c>), grid, dim3(kThreads), 0, s, m, n, k,
                       (float)alpha, A, lda, B, ldb, (float)beta, C, ldc, tm, tn);
    return hipGetLastError();
  }
  const int tm = (int)((m + kBM - 1) / kBM);
  const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
  hipLaunchKernelGGL((k_gemm_nn32<MODE_BF16, bf16c>), grid, dim3(kThreads), 0, s, m, n, k,
                     (float)alpha, A, lda, B, ldb, (float)beta, C, ldc, tm, tn);
  return hipGetLastError();
}

hipError_t launch_gemm_nn32(int bf16, int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                            int64_t lda, const float2* B, int64_t ldb, double beta, float2* C,
                            int64_t ldc, hipStream_t s, int tile, const uint16_t* a3,
                            const uint16_t* b3) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int tn = (int)((n + kBN - 1) / kBN);
  if (!bf16 && a3 && b3) {
    const int tm = (int)((m + kBM - 1) / kBM);
    const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
    hipLaunchKernelGGL(k_gemm_nn32_s3, grid, dim3(kThreads), 0, s, m, n, k, (float)alpha,
                       reinterpret_cast<const __bf16*>(a3), reinterpret_cast<const __bf16*>(b3),
                       (float)beta, C, ldc, tm, tn);
    return hipGetLastError();
  }
  if (tile == 1) {
    const int tm = (int)((m + 2 * kBM - 1) / (2 * kBM));
    const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
    if (bf16)
      hipLaunchKernelGGL(k_gemm_nn32_tall<MODE_BF16>, grid, dim3(kThreads), 0, s, m, n, k,
                         (float)alpha, A, lda, B, ldb, (float)beta, C, ldc, tm, tn);
    else
      hipLaunchKernelGGL(k_gemm_nn32_tall<MODE_F32>, grid, dim3(kThreads), 0, s, m, n, k,
                         (float)alpha, A, lda, B, ldb, (float)beta, C, ldc, tm, tn);
    return hipGetLastError();
  }
  const int tm = (int)((m + kBM - 1) / kBM);
  const dim3 grid((unsigned)(kXcds * tn * ((tm + kXcds - 1) / kXcds)));
  if (bf16)
    hipLaunchKernelGGL(k_gemm_nn32<MODE_BF16>, grid, dim3(kThreads), 0, s, m, n, k, (float)alpha, A,
                       lda, B, ldb, (float)beta, C, ldc, tm, tn);
  else
    hipLaunchKernelGGL(k_gemm_nn32<MODE_F32>, grid, dim3(kThreads), 0, s, m, n, k, (float)alpha, A,
                       lda, B, ldb, (float)beta, C, ldc, tm, tn);
  return hipGetLastError();
}

int fused_cn32_nsplit(int bf16, int64_t npw, int64_t nb, int64_t nproj, int target) {
  const SplitPlan p = bf16 ? split_plan32<MODE_BF16>(nproj, nb, npw, target)
                           : split_plan32<MODE_F32>(nproj, nb, npw, target);
  return (int)p.nsplit;
}

hipError_t launch_fused_gemm_cn32(int bf16, int nitems, int64_t m_max, int64_t n_max,
                                  int nsplit_max, const ItemDev* D, int sel_b, double alpha,
                                  int coef_step, hipStream_t s) {
  if (nitems <= 0 || m_max <= 0 || n_max <= 0) return hipSuccess;
  dim3 grid((n_max + kBN - 1) / kBN, (m_max + kBM - 1) / kBM, nitems * nsplit_max);
  if (bf16)
    hipLaunchKernelGGL(kb_gemm_cn32<MODE_BF16>, grid, dim3(kThreads), 0, s, D, sel_b, nsplit_max);
  else
    hipLaunchKernelGGL(kb_gemm_cn32<MODE_F32>, grid, dim3(kThreads), 0, s, D, sel_b, nsplit_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 rgrid((m_max * n_max + 255) / 256, nitems);
  if (bf16)
    hipLaunchKernelGGL(kb_splitk_reduce32<MODE_BF16>, rgrid, dim3(256), 0, s, D, alpha, coef_step);
  else
    hipLaunchKernelGGL(kb_splitk_reduce32<MODE_F32>, rgrid, dim3(256), 0, s, D, alpha, coef_step);
  return hipGetLastError();
}

hipError_t launch_fused_gemm_nn32(int bf16, int nitems, int64_t m_max, int64_t n_max,
                                  const ItemDev* D, int sel_c, hipStream_t s) {
  if (nitems <= 0 || m_max <= 0 || n_max <= 0) return hipSuccess;
  dim3 grid((n_max + kBN - 1) / kBN, (m_max + kBM - 1) / kBM, nitems);
  if (bf16)
    hipLaunchKernelGGL(kb_gemm_nn32<MODE_BF16>, grid, dim3(kThreads), 0, s, D, sel_c);
  else
    hipLaunchKernelGGL(kb_gemm_nn32<MODE_F32>, grid, dim3(kThreads), 0, s, D, sel_c);
  return hipGetLastError();
}

size_t split3_elems(int64_t rows, int64_t k) { return (size_t)(s3_rows(rows) * s3_nst(k) * kS3Chunk); }

hipError_t launch_split3(int64_t rows, int64_t k, const float2* X, int64_t sr, int64_t sk,
                         uint16_t* X3, hipStream_t s) {
  if (rows <= 0 || k <= 0) return hipSuccess;
  const dim3 grid((unsigned)(s3_rows(rows) / 64), (unsigned)std::min<int64_t>(s3_nst(k), 65535));
  hipLaunchKernelGGL(k_split3_s3, grid, dim3(256), 0, s, rows, k, X, sr, sk,
                     reinterpret_cast<__bf16*>(X3));
  return hipGetLastError();
}
