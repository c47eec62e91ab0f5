// Small dense FP64 linear algebra of the subspace steps, plus element-wise
// helpers.  Section 5.1 (Rayleigh-Ritz: a dense Hermitian eigenproblem of
// the block size) and section 5.4 (full-band Cholesky orthogonalisation).
//
//  * chol      : S = U^H U (upper Cholesky), blocked: each 64-wide diagonal
//                block is factored and inverted in LDS by one workgroup; the
//                row panels and trailing updates are MFMA products.
//  * heev      : cyclic two-sided Jacobi with the round-robin (circle)
//                ordering: in each round all n/2 disjoint pairs rotate at
//                once, A <- G^H A G, V <- V G.  For n <= 64 the whole solve
//                runs in one workgroup with A and V in LDS; larger n run a
//                block Jacobi whose block pairs take one such sweep each in
//                LDS, applied to A and V as tiled products.
#include "pw_internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace {

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------------------
// element-wise helpers
// ---------------------------------------------------------------------------
struct KinArgs {
  double b[9];
  double k[3];
};

__global__ void k_kinetic(int64_t npw, const int* __restrict__ miller, KinArgs a,
                          double* __restrict__ kin) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const double u0 = miller[3 * g] + a.k[0], u1 = miller[3 * g + 1] + a.k[1],
               u2 = miller[3 * g + 2] + a.k[2];
  const double qx = u0 * a.b[0] + u1 * a.b[3] + u2 * a.b[6];
  const double qy = u0 * a.b[1] + u1 * a.b[4] + u2 * a.b[7];
  const double qz = u0 * a.b[2] + u1 * a.b[5] + u2 * a.b[8];
  kin[g] = 0.5 * (qx * qx + qy * qy + qz * qz);
}

__global__ void k_scale_copy(int64_t n, const double* __restrict__ src, double scale,
                             double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = scale * src[i];
}

__global__ void __launch_bounds__(1024) k_max_reduce(int64_t n, const double* __restrict__ x,
                                                     double* out) {
  __shared__ double red[1024];
  double m = -DBL_MAX;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, x[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_check_finite(int64_t n, const double* __restrict__ x, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flag, 1);
}

// The Hermitian matrix from its upper triangle: A[j][i] = conj(A[i][j]) for
// i < j, real diagonal (the lower triangle is not read).
__device__ __forceinline__ void hermitize_body(int64_t n, cplx* a, int64_t lda, int bx_) {
  const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  if (i > j) return;
  if (i == j) {
    a[i + j * lda].y = 0.0;
    return;
  }
  a[j + i * lda] = cconj(a[i + j * lda]);
}

__global__ void 
k_hermitize(int64_t n, cplx* a, int64_t lda) {
  hermitize_body(n, a, lda, blockIdx.x);
}

__device__ __forceinline__ void copy_block_body(int64_t rows, int64_t cols, const cplx* __restrict__ src, int64_t lds,
                             cplx* __restrict__ dst, int64_t ldd, int bx_) {
  const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  dst[i + j * ldd] = src[i + j * lds];
}

__global__ void 
k_copy_block(int64_t rows, int64_t cols, const cplx* __restrict__ src, int64_t lds,
                             cplx* __restrict__ dst, int64_t ldd) {
  copy_block_body(rows, cols, src, lds, dst, ldd, blockIdx.x);
}

__global__ void k_scale_rows_cols(int64_t n, const double* __restrict__ d, cplx* a, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  a[i + j * lda] = cscale(a[i + j * lda], d[i] * d[j]);
}

__device__ __forceinline__ void axpby_block_body(int64_t npw, int64_t nb, double a, const cplx* x, int64_t ldx,
                              double b, const cplx* y, int64_t ldy, cplx* out, int64_t ldo,
                              const double* __restrict__ coef, int bx_) {
  const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (idx >= npw * nb) return;
  if (coef) {
    a = coef[0];
    b = coef[1];
  }
  const int64_t j = idx / npw, i = idx - j * npw;
  const cplx u = x[i + j * ldx], v = y[i + j * ldy];
  out[i + j * ldo] = make_double2(a * u.x + b * v.x, a * u.y + b * v.y);
}

__global__ void 
k_axpby_block(int64_t npw, int64_t nb, double a, const cplx* x, int64_t ldx,
                              double b, const cplx* y, int64_t ldy, cplx* out, int64_t ldo,
                              const double* __restrict__ coef) {
  axpby_block_body(npw, nb, a, x, ldx, b, y, ldy, out, ldo, coef, blockIdx.x);
}

__device__ __forceinline__ void residuals_body(int64_t npw, const cplx* __restrict__ W, int64_t ldw, const cplx* __restrict__ Y,
            int64_t ldy, const double* __restrict__ lam, double* __restrict__ resid, int bx_) {
  __shared__ double red[256];
  const int64_t b = bx_;
  const double l = lam[b];
  const cplx* w = W + b * ldw;
  const cplx* y = Y + b * ldy;
  double s = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += blockDim.x) {
    const cplx d = make_double2(w[g].x - l * y[g].x, w[g].y - l * y[g].y);
    s += cabs2(d);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) resid[b] = sqrt(red[0]);
}

__global__ void __launch_bounds__(256) 
k_residuals(int64_t npw, const cplx* __restrict__ W, int64_t ldw, const cplx* __restrict__ Y,
            int64_t ldy, const double* __restrict__ lam, double* __restrict__ resid) {
  residuals_body(npw, W, ldw, Y, ldy, lam, resid, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Blocked Cholesky (S = U^H U) for large n: per diagonal block of kb <= 64
// one workgroup factors it in LDS and inverts the factor; the row panel and
// the trailing update are matrix products (k_gemm_cn) issued by the host.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chol_init_body(int n, const cplx* __restrict__ A, int64_t lda,
                                                    double* tol, int* status) {
  __shared__ double red[1024];
  __shared__ int bad[1024];
  double m = 0.0;
  int b = n;   // first diagonal entry that is NaN or infinite (a non-finite column)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = A[i + (int64_t)i * lda].x;
    m = fmax(m, d);
    if (!isfinite(d)) b = min(b, i);
  }
  red[threadIdx.x] = m;
  bad[threadIdx.x] = b;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      bad[threadIdx.x] = min(bad[threadIdx.x], bad[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tol[0] = (double)n * DBL_EPSILON * red[0];
    status[0] = bad[0] < n ? kCholNonFinite - bad[0] : -1;
  }
}

__global__ void __launch_bounds__(1024) 
k_chol_init(int n, const cplx* __restrict__ A, int64_t lda,
                                                    double* tol, int* status) {
  chol_init_body(n, A, lda, tol, status);
}

// Factor the kb x kb diagonal block at A(k0, k0) (upper triangle read),
// write U back (zeros below its diagonal) and U^{-1} to dinv (ld kb).  A
// pivot at or below tol records k0 + p in status unless an earlier block did.
// 1/sqrt(x) and 1/x for x > 0 (normal): the hardware estimate refined by two
// Newton steps (each doubles the correct bits), much shorter dependency
// chains than the correctly rounded sequences; about 1 ulp.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

// Upper Cholesky of the kb x kb diagonal block at (k0, k0) (kb <= 64; 256
// threads, as both launchers give) and the inverse of its factor into dinv (ld kb).  Right-looking
// with the pivot row left unscaled, a_ij -= conj(a_pi) a_pj / a_pp for
// p < i <= j (thread (ti, tj) of a 16 x 16 grid owns the entries i = ti + 16u,
// j = tj + 16v), one barrier per pivot; the rows are scaled by 1/sqrt(a_pp)
// at the end.  The inverse is formed column by column, each entry's sum
// split over four lanes and joined by shuffles.
__device__ __forceinline__ void chol_diag_body(int kb, int k0, cplx* __restrict__ A, int64_t lda, cplx* __restrict__ dinv,
            const double* __restrict__ tol, int* status) {
  extern __shared__ cplx sm[];
  const int trs = kb + 1;
  cplx* a = sm;
  cplx* x = sm + kb * trs;
  __shared__ double sq[kCholBlock], rs[kCholBlock];   // sqrt(a_pp), 1 / sqrt(a_pp)
  const int tid = threadIdx.x, nt = blockDim.x;
  cplx* Ab = A + k0 + (int64_t)k0 * lda;
  for (int idx = tid; idx < kb * kb; idx += nt) {
    const int j = idx / kb, i = idx - j * kb;
    a[i + j * trs] = (i <= j) ? Ab[i + (int64_t)j * lda] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double t = tol[0];
  const int ti = tid & 15, tj = (tid >> 4) & 15;
  int fail = -1;
  for (int p = 0; p < kb; ++p) {
    const double d = a[p + p * trs].x;   // the same value in every thread
    if (!(d > t)) {
      fail = p;
      break;
    }
    const double rd = rcp_nr(d);
#pragma unroll
    for (int u = 0; u < kCholBlock / 16; ++u) {
      const int i = ti + 16 * u;
      if (i <= p || i >= kb) continue;
      const cplx c = cscale(cconj(a[p + i * trs]), rd);
#pragma unroll
      for (int v = 0; v < kCholBlock / 16; ++v) {
        const int j = tj + 16 * v;
        if (j < i || j >= kb) continue;
        a[i + j * trs] = csub(a[i + j * trs], cmul(c, a[p + j * trs]));
      }
    }
    __syncthreads();
  }
  if (fail >= 0) {
    if (tid == 0 && status[0] == -1) status[0] = k0 + fail;
    return;
  }
  for (int i = tid; i < kb; i += nt) {
    sq[i] = sqrt(a[i + i * trs].x);
    rs[i] = rsqrt_nr(a[i + i * trs].x);
  }
  __syncthreads();
  for (int idx = tid; idx < kb * kb; idx += nt) {
    const int j = idx / kb, i = idx - j * kb;
    cplx u = make_double2(0.0, 0.0);
    if (i == j) u = make_double2(sq[i], 0.0);
    else if (i < j) u = cscale(a[i + j * trs], rs[i]);
    a[i + j * trs] = u;
    Ab[i + (int64_t)j * lda] = u;
  }
  __syncthreads();
  // x = U^{-1}: x_jj = 1/u_jj, x_ij = -(sum_{i <= p < j} x_ip u_pj) / u_jj
  const int i = tid >> 2, q = tid & 3;
  for (int j = 0; j < kb; ++j) {
    double sr = 0.0, si = 0.0;
    if (i < j)
      for (int p = i + q; p < j; p += 4) {
        const cplx xv = x[i + p * trs], uv = a[p + j * trs];
        sr += xv.x * uv.x - xv.y * uv.y;
        si += xv.x * uv.y + xv.y * uv.x;
      }
    sr += __shfl_xor(sr, 1, 64);
    si += __shfl_xor(si, 1, 64);
    sr += __shfl_xor(sr, 2, 64);
    si += __shfl_xor(si, 2, 64);
    if (q == 0 && i < kb) {
      const double rinv = rs[j];
      x[i + j * trs] = i < j ? make_double2(-sr * rinv, -si * rinv)
                             : make_double2(i == j ? rinv : 0.0, 0.0);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kb * kb; idx += nt) {
    const int j = idx / kb, i = idx - j * kb;
    dinv[i + j * kb] = x[i + j * trs];
  }
}

__global__ void __launch_bounds__(256) 
k_chol_diag(int kb, int k0, cplx* __restrict__ A, int64_t lda, cplx* __restrict__ dinv,
            const double* __restrict__ tol, int* status) {
  chol_diag_body(kb, k0, A, lda, dinv, tol, status);
}

__global__ void k_zero_lower(int n, cplx* A, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  if (i > j) A[i + j * lda] = make_double2(0.0, 0.0);
}

__global__ void k_identity_ld(int n, cplx* A, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  A[i + j * lda] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Jacobi
// ---------------------------------------------------------------------------
struct Rot {
  double cs, sn, t;
  cplx ph;     // c / |c|
  bool on;
};

// Round r of the circle method over n2 (even) indices: pair k -> (p < q).
__device__ __forceinline__ void rr_pair(int r, int k, int n2, int* p, int* q) {
  const int m = n2 - 1;
  const int a = k == 0 ? m : (r + k) % m;
  const int b = k == 0 ? r : (r - k + m) % m;
  *p = min(a, b);
  *q = max(a, b);
}

// Rotation J = [[cs, sn ph], [-sn conj(ph), cs]] with J^H [[a, c], [conj c, b]] J diagonal:
// tau = (b - a)/(2|c|), t = sign(tau)/(|tau| + sqrt(1 + tau^2)), cs = 1/sqrt(1+t^2), sn = t cs;
// new diagonal a - t|c|, b + t|c|.  |c| below 1e-150 (|c|^2 near the
// denormal range) counts as zero: no rotation.  (Matrix entries here are
// O(1) Hamiltonian elements.)
__device__ __forceinline__ Rot make_rot(double a, double b, cplx c) {
  // branch-free (callers form several rotations side by side); a zero c
  // selects the identity at the end (the arithmetic before it may be inf/NaN)
  Rot R;
  const double m2 = c.x * c.x + c.y * c.y;
  R.on = m2 > 1e-300;
  const double rmag = rsqrt_nr(m2);
  const double mag = m2 * rmag;
  const double tau = 0.5 * (b - a) * rmag;
  const double at = fabs(tau);
  // for |tau| > 1e100, sqrt(1 + tau^2) = |tau| to working precision
  const double u = 1.0 + tau * tau;
  const double ru = u * rsqrt_nr(u);
  const double root = at > 1e100 ? at : ru;
  const double t = copysign(rcp_nr(at + root), tau);
  const double cs = rsqrt_nr(1.0 + t * t);
  R.cs = R.on ? cs : 1.0;
  R.sn = R.on ? t * cs : 0.0;
  R.t = R.on ? t * mag : 0.0;
  R.ph = R.on ? make_double2(c.x * rmag, c.y * rmag) : make_double2(1.0, 0.0);
  return R;
}

// 2x2 block update X <- Jp^H X Jq, X = [[x11, x12], [x21, x22]]
__device__ __forceinline__ void rot_block(const Rot& P, const Rot& Q, cplx* x11, cplx* x12,
                                          cplx* x21, cplx* x22) {
  // M = X Jq: Jq = [[cs, sn ph], [-sn conj(ph), cs]]
  const cplx q12 = cscale(Q.ph, Q.sn);              // sn ph
  const cplx q21 = cscale(cconj(Q.ph), -Q.sn);      // -sn conj(ph)
  const cplx m11 = cadd(cscale(*x11, Q.cs), cmul(*x12, q21));
  const cplx m12 = cadd(cmul(*x11, q12), cscale(*x12, Q.cs));
  const cplx m21 = cadd(cscale(*x21, Q.cs), cmul(*x22, q21));
  const cplx m22 = cadd(cmul(*x21, q12), cscale(*x22, Q.cs));
  // Jp^H = [[cs, -sn ph], [sn conj(ph), cs]]
  const cplx p12 = cscale(P.ph, -P.sn);
  const cplx p21 = cscale(cconj(P.ph), P.sn);
  *x11 = cadd(cscale(m11, P.cs), cmul(p12, m21));
  *x12 = cadd(cscale(m12, P.cs), cmul(p12, m22));
  *x21 = cadd(cmul(p21, m11), cscale(m21, P.cs));
  *x22 = cadd(cmul(p21, m12), cscale(m22, P.cs));
}

// row update [vp, vq] <- [vp, vq] Jq
__device__ __forceinline__ void rot_row(const Rot& Q, cplx* vp, cplx* vq) {
  const cplx q12 = cscale(Q.ph, Q.sn);
  const cplx q21 = cscale(cconj(Q.ph), -Q.sn);
  const cplx a = *vp, b = *vq;
  *vp = cadd(cscale(a, Q.cs), cmul(b, q21));
  *vq = cadd(cmul(a, q12), cscale(b, Q.cs));
}

constexpr int kJacSmallMax = 64;
constexpr int kJacThreads = 1024;
constexpr int kMaxSweeps = kHeevMaxSweeps;

__device__ __forceinline__ double jac_tol(int n) { return fmax(1e-15, 2.2e-16 * n); }

// Workgroup size of the one-workgroup solve: one thread per 2x2 block of a
// round (h^2, h = ceil(n/2)), a power of two in [64, 1024].
inline int jac_threads(int n) {
  const int h = (n + 1) / 2;
  int t = 64;
  while (t < h * h && t < kJacThreads) t *= 2;
  return t;
}

// Whole Jacobi solve in LDS for n <= 64.
__device__ __forceinline__ void jacobi_small_body(int n, const cplx* __restrict__ Ain, int64_t lda, double* __restrict__ w,
               cplx* __restrict__ Q, int64_t ldq, int* sweeps_out) {
  extern __shared__ cplx sm[];
  const int n2 = n + (n & 1);
  const int h = n2 / 2;
  // A with an odd leading dimension: the 2x2 blocks a round updates sit in
  // columns n + 1 entries apart, which spreads them over the LDS banks
  const int la = n + 1;
  cplx* a = sm;               // n x n, ld la
  cplx* v = sm + n * la;      // n x n, ld n
  __shared__ Rot rots[kJacSmallMax / 2];
  __shared__ int pp[kJacSmallMax / 2], pq[kJacSmallMax / 2];   // this round's pairs
  __shared__ double red[kJacThreads];
  __shared__ double red2[kJacThreads];
  __shared__ int done;
  __shared__ int rank_[kJacSmallMax];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < n * n; idx += nt) {
    const int j = idx / n, i = idx - j * n;
    a[i + j * la] = Ain[i + (int64_t)j * lda];
    v[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) done = 0;
  __syncthreads();
  int sweeps = 0;
  for (; sweeps < kMaxSweeps; ++sweeps) {
    // convergence test before the sweep: 64 fixed partial sums, so the
    // summation order does not depend on the workgroup size
    if (tid < 64) {
      double off = 0.0, tot = 0.0;
      for (int idx = tid; idx < n * n; idx += 64) {
        const int j = idx / n, i = idx - j * n;
        const double m2 = cabs2(a[i + j * la]);
        tot += m2;
        if (i != j) off += m2;
      }
      red[tid] = off;
      red2[tid] = tot;
    }
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
      if (tid < s) {
        red[tid] += red[tid + s];
        red2[tid] += red2[tid + s];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double tl = jac_tol(n);
      done = (red[0] <= tl * tl * red2[0]) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < n2 - 1; ++r) {
      if (tid < h) {
        int p, q;
        rr_pair(r, tid, n2, &p, &q);
        pp[tid] = p;
        pq[tid] = q;
        if (q < n) rots[tid] = make_rot(a[p + p * la].x, a[q + q * la].x, a[p + q * la]);
        else rots[tid] = make_rot(0.0, 0.0, make_double2(0.0, 0.0));
      }
      __syncthreads();
      for (int idx = tid; idx < h * h; idx += nt) {
        const int P = idx / h, Qb = idx - P * h;
        const int p1 = pp[P], q1 = pq[P], p2 = pp[Qb], q2 = pq[Qb];
        const Rot& RP = rots[P];
        const Rot& RQ = rots[Qb];
        if (q1 >= n || q2 >= n) {
          // pairs holding the padding index rotate nothing; update the real rows/cols only
          if (q1 < n && RP.on) {   // Q pair is (p2, pad): column p2 only
            cplx x1 = a[p1 + p2 * la], x2 = a[q1 + p2 * la];
            cplx y1 = x1, y2 = x2;
            // Jp^H [x1; x2]
            const cplx p12 = cscale(RP.ph, -RP.sn), p21 = cscale(cconj(RP.ph), RP.sn);
            y1 = cadd(cscale(x1, RP.cs), cmul(p12, x2));
            y2 = cadd(cmul(p21, x1), cscale(x2, RP.cs));
            a[p1 + p2 * la] = y1;
            a[q1 + p2 * la] = y2;
          } else if (q2 < n && RQ.on) {   // P pair is (p1, pad): row p1 only
            cplx x1 = a[p1 + p2 * la], x2 = a[p1 + q2 * la];
            rot_row(RQ, &x1, &x2);
            a[p1 + p2 * la] = x1;
            a[p1 + q2 * la] = x2;
          }
          continue;
        }
        if (P == Qb) {
          if (RP.on) {
            const double ap = a[p1 + p1 * la].x, aq = a[q1 + q1 * la].x;
            a[p1 + p1 * la] = make_double2(ap - RP.t, 0.0);
            a[q1 + q1 * la] = make_double2(aq + RP.t, 0.0);
            a[p1 + q1 * la] = make_double2(0.0, 0.0);
            a[q1 + p1 * la] = make_double2(0.0, 0.0);
          }
          continue;
        }
        if (!RP.on && !RQ.on) continue;
        cplx x11 = a[p1 + p2 * la], x12 = a[p1 + q2 * la], x21 = a[q1 + p2 * la], x22 = a[q1 + q2 * la];
        rot_block(RP, RQ, &x11, &x12, &x21, &x22);
        a[p1 + p2 * la] = x11;
        a[p1 + q2 * la] = x12;
        a[q1 + p2 * la] = x21;
        a[q1 + q2 * la] = x22;
      }
      for (int idx = tid; idx < n * h; idx += nt) {
        const int Qb = idx / n, i = idx - Qb * n;
        const int p2 = pp[Qb], q2 = pq[Qb];
        if (q2 >= n || !rots[Qb].on) continue;
        cplx x1 = v[i + p2 * n], x2 = v[i + q2 * n];
        rot_row(rots[Qb], &x1, &x2);
        v[i + p2 * n] = x1;
        v[i + q2 * n] = x2;
      }
      __syncthreads();
    }
  }
  // sort ascending (rank by value, ties by index) and write out
  for (int i = tid; i < n; i += nt) {
    const double di = a[i + i * la].x;
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = a[j + j * la].x;
      if (dj < di || (dj == di && j < i)) ++rk;
    }
    rank_[i] = rk;
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) w[rank_[i]] = a[i + i * la].x;
  for (int idx = tid; idx < n * n; idx += nt) {
    const int j = idx / n, i = idx - j * n;
    Q[i + (int64_t)rank_[j] * ldq] = v[i + j * n];
  }
  if (tid == 0) sweeps_out[0] = done ? sweeps : -1;
}

__global__ void 
k_jacobi_small(int n, const cplx* __restrict__ Ain, int64_t lda, double* __restrict__ w,
               cplx* __restrict__ Q, int64_t ldq, int* sweeps_out) {
  jacobi_small_body(n, Ain, lda, w, Q, ldq, sweeps_out);
}

// n > 64: block Jacobi.  The matrix (padded with zero rows and columns to
// n2p, a multiple of 2 kBJ) is cut into blocks of kBJ indices; an outer
// round pairs the blocks by the circle method and, for every pair (I, J) at
// once, runs one cyclic Jacobi sweep on the 2 kBJ x 2 kBJ sub-problem
// A[I u J, I u J] in LDS, accumulating its rotations in a unitary Q_k; then
// A <- G^H A G and V <- V G with G the block-diagonal product of the Q_k, as
// two tiled products.  Every index pair meets in each outer sweep (pairs
// inside a block in every round), so the outer sweeps converge like cyclic
// Jacobi.  Rounds 1 .. nblk - 2 of a sweep each take one launch that also
// applies the previous round's update (k_bj_step); round 0 and the last
// update have launches of their own.  Padding indices have zero rows and
// columns and never rotate.  The
// convergence test runs on the device before every outer sweep; once it
// passes, conv[0] is set and every later launch of the solve returns at
// once, so a fixed number of sweeps can be issued with no host read.
constexpr int kBJ = 16;           // block size
constexpr int kBJS = 2 * kBJ;     // sub-problem size
constexpr int kBJTile = 64;       // row tile of the V update (and the padding of n)

// global index of sub-problem index i of block pair (I, J)
__device__ __forceinline__ int bj_index(int i, int I, int J) {
  return i < kBJ ? I * kBJ + i : J * kBJ + (i - kBJ);
}

// One sweep on each block pair of outer round r (workgroup k: pair k);
// Qout[k] (kBJS x kBJS, column-major) receives the accumulated rotations.
// One thread per 2x2 block of A (kBJ^2 blocks: thread (P, Qb) takes rows
// of pair P and columns of pair Qb of the inner round) and per two (row,
// pair) items of V (rows Qb and Qb + kBJ, pair P).  A is double-buffered:
// each inner round reads one copy and writes the other, so every thread
// forms the two rotations it needs from the entries it reads (the same
// arithmetic on the same values in every thread that forms one) and an
// inner round needs a single barrier.  a0 holds the sub-problem on entry
// (ld kBJS + 1); a1 and v are LDS of the same size.
constexpr int kBJInnerThreads = kBJ * kBJ;
constexpr int kBJLA = kBJS + 1;           // ld of the sub-problem (odd: spreads the LDS banks)
static_assert(2 * kBJInnerThreads == kBJS * kBJ, "V (row, pair) items: two per thread");
static_assert(64 % kBJ == 0, "the lanes P < kBJ of every wavefront hold the pairs' rotations");
__device__ __forceinline__ void bj_inner_sweep(cplx* a0, cplx* a1, cplx* v, cplx* __restrict__ qo) {
  constexpr int LA = kBJLA;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kBJS * kBJS; idx += kBJInnerThreads) {
    const int j = idx / kBJS, i = idx - j * kBJS;
    v[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int P = tid / kBJ, Qb = tid - P * kBJ;
  for (int rr = 0; rr < kBJS - 1; ++rr) {
    const cplx* ac = rr & 1 ? a1 : a0;
    cplx* an = rr & 1 ? a0 : a1;
    int p1, q1, p2, q2;
    rr_pair(rr, P, kBJS, &p1, &q1);
    rr_pair(rr, Qb, kBJS, &p2, &q2);
    // every thread forms the rotation of its pair Qb; RP (pair P) comes from
    // lane P of the same wavefront (its Qb is P)
    const Rot RQ = make_rot(ac[p2 + p2 * LA].x, ac[q2 + q2 * LA].x, ac[p2 + q2 * LA]);
    Rot RP;
    RP.cs = __shfl(RQ.cs, P, 64);
    RP.sn = __shfl(RQ.sn, P, 64);
    RP.t = __shfl(RQ.t, P, 64);
    RP.ph = make_double2(__shfl(RQ.ph.x, P, 64), __shfl(RQ.ph.y, P, 64));
    RP.on = __shfl((int)RQ.on, P, 64) != 0;
    cplx x11 = ac[p1 + p2 * LA], x12 = ac[p1 + q2 * LA];
    cplx x21 = ac[q1 + p2 * LA], x22 = ac[q1 + q2 * LA];
    // an identity rotation (pair off) leaves the values unchanged exactly;
    // the diagonal block reads RQ (= RP there), so both are formed up front
    if (P == Qb) {
      if (RQ.on) {
        x11 = make_double2(x11.x - RQ.t, 0.0);
        x22 = make_double2(x22.x + RQ.t, 0.0);
        x12 = make_double2(0.0, 0.0);
        x21 = make_double2(0.0, 0.0);
      }
    } else {
      rot_block(RP, RQ, &x11, &x12, &x21, &x22);
    }
    an[p1 + p2 * LA] = x11;
    an[p1 + q2 * LA] = x12;
    an[q1 + p2 * LA] = x21;
    an[q1 + q2 * LA] = x22;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int vi = Qb + h * kBJ;
      cplx x1 = v[vi + p1 * kBJS], x2 = v[vi + q1 * kBJS];
      rot_row(RP, &x1, &x2);
      v[vi + p1 * kBJS] = x1;
      v[vi + q1 * kBJS] = x2;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kBJS * kBJS; idx += kBJInnerThreads) qo[idx] = v[idx];
}

// Round 0 of a sweep: the sub-problems read straight from A.
__global__ void __launch_bounds__(kBJInnerThreads)
k_bj_inner(int n2p, int r, const cplx* __restrict__ A, cplx* __restrict__ Qout,
           const int* __restrict__ conv) {
  if (conv[0]) return;
  __shared__ cplx a[2][kBJS * kBJLA];
  __shared__ cplx v[kBJS * kBJS];
  int I, J;
  rr_pair(r, blockIdx.x, n2p / kBJ, &I, &J);
  for (int idx = threadIdx.x; idx < kBJS * kBJS; idx += kBJInnerThreads) {
    const int j = idx / kBJS, i = idx - j * kBJS;
    a[0][i + j * kBJLA] = A[bj_index(i, I, J) + (int64_t)bj_index(j, I, J) * n2p];
  }
  bj_inner_sweep(a[0], a[1], v, Qout + (int64_t)blockIdx.x * kBJS * kBJS);
}

// Two-sided update of outer round r.  Workgroup w < npair^2 takes the
// sub-block of A on block pair p = w / npair (rows) and block pair q =
// w % npair (columns): Aout[idx_p, idx_q] <- Q_p^H Ain[idx_p, idx_q] Q_q,
// both products in LDS.  Workgroup npair^2 + t npair + q takes kBJTile rows
// of V from row t kBJTile: V[rows, idx_q] <- V[rows, idx_q] Q_q.  Each
// workgroup reads and writes only its own elements, so Ain may be Aout.
// sm: LDS of kBJUpdateSm entries.
constexpr int kBJUThreads = 256;
static_assert(kBJUThreads == kBJInnerThreads, "fused step: one workgroup size");
constexpr int kBJUSmA = (kBJS + 1) * kBJS + 2 * kBJS * kBJS, kBJUSmV = kBJTile * kBJS + kBJS * kBJS;
constexpr int kBJUpdateSm = kBJUSmA > kBJUSmV ? kBJUSmA : kBJUSmV;
__device__ __forceinline__ void bj_update_body(int n, int n2p, int r, const cplx* Ain, cplx* Aout,
                                               cplx* __restrict__ V, const cplx* __restrict__ Qk,
                                               int w, cplx* sm) {
  constexpr int LX = kBJS + 1;                         // odd row pitch of the A sub-block
  const int tid = threadIdx.x;
  const int nblk = n2p / kBJ, npair = nblk / 2;
  if (w < npair * npair) {
    const int p = w / npair, q = w - p * npair;
    int Ip, Jp, Iq, Jq;
    rr_pair(r, p, nblk, &Ip, &Jp);
    rr_pair(r, q, nblk, &Iq, &Jq);
    cplx* X = sm;                       // [i + j LX]
    cplx* Qp = sm + LX * kBJS;          // [i + m kBJS] = conj(Q_p(m, i)): the lanes of
    cplx* Qq = Qp + kBJS * kBJS;        //   a wavefront read consecutive i
    const cplx* gp = Qk + (int64_t)p * kBJS * kBJS;
    const cplx* gq = Qk + (int64_t)q * kBJS * kBJS;
    for (int idx = tid; idx < kBJS * kBJS; idx += kBJUThreads) {
      const int j = idx / kBJS, i = idx - j * kBJS;
      X[i + j * LX] = Ain[bj_index(i, Ip, Jp) + (int64_t)bj_index(j, Iq, Jq) * n2p];
      Qp[j + i * kBJS] = cconj(gp[idx]);
      Qq[idx] = gq[idx];
    }
    __syncthreads();
    constexpr int NJ = kBJS * kBJS / kBJUThreads;      // outputs per thread
    constexpr int G = kBJUThreads / kBJS;
    const int i = tid % kBJS, jg = tid / kBJS;
    cplx acc[NJ];
#pragma unroll
    for (int t = 0; t < NJ; ++t) acc[t] = make_double2(0.0, 0.0);
    // T = Q_p^H X
#pragma unroll 8
    for (int m = 0; m < kBJS; ++m) {
      const cplx qh = Qp[i + m * kBJS];
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        const cplx x = X[m + (jg + t * G) * LX];
        acc[t].x += qh.x * x.x - qh.y * x.y;
        acc[t].y += qh.x * x.y + qh.y * x.x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NJ; ++t) X[i + (jg + t * G) * LX] = acc[t];
    __syncthreads();
    // out = T Q_q
#pragma unroll
    for (int t = 0; t < NJ; ++t) acc[t] = make_double2(0.0, 0.0);
#pragma unroll 8
    for (int m = 0; m < kBJS; ++m) {
      const cplx x = X[i + m * LX];
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        const cplx qv = Qq[m + (jg + t * G) * kBJS];
        acc[t].x += x.x * qv.x - x.y * qv.y;
        acc[t].y += x.x * qv.y + x.y * qv.x;
      }
    }
    const int gi = bj_index(i, Ip, Jp);
#pragma unroll
    for (int t = 0; t < NJ; ++t)
      Aout[gi + (int64_t)bj_index(jg + t * G, Iq, Jq) * n2p] = acc[t];
    return;
  }
  const int vw = w - npair * npair;
  const int tile = vw / npair, q = vw - tile * npair;
  int Iq, Jq;
  rr_pair(r, q, nblk, &Iq, &Jq);
  const int r0 = tile * kBJTile;
  cplx* T = sm;                         // [i + m kBJTile]: V[r0 + i, idx_q[m]]
  cplx* Qq = sm + kBJTile * kBJS;       // [m + j kBJS]
  const cplx* gq = Qk + (int64_t)q * kBJS * kBJS;
  for (int idx = tid; idx < kBJTile * kBJS; idx += kBJUThreads) {
    const int m = idx / kBJTile, i = idx - m * kBJTile;
    T[idx] = (r0 + i < n) ? V[(r0 + i) + (int64_t)bj_index(m, Iq, Jq) * n] : make_double2(0.0, 0.0);
  }
  for (int idx = tid; idx < kBJS * kBJS; idx += kBJUThreads) Qq[idx] = gq[idx];
  __syncthreads();
  constexpr int G = kBJUThreads / kBJTile, NJ = kBJS / G;
  const int i = tid % kBJTile, jg = tid / kBJTile;
  cplx acc[NJ];
#pragma unroll
  for (int t = 0; t < NJ; ++t) acc[t] = make_double2(0.0, 0.0);
#pragma unroll 8
  for (int m = 0; m < kBJS; ++m) {
    const cplx x = T[i + m * kBJTile];
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
      const cplx qv = Qq[m + (jg + t * G) * kBJS];
      acc[t].x += x.x * qv.x - x.y * qv.y;
      acc[t].y += x.x * qv.y + x.y * qv.x;
    }
  }
  if (r0 + i < n) {
#pragma unroll
    for (int t = 0; t < NJ; ++t)
      V[(r0 + i) + (int64_t)bj_index(jg + t * G, Iq, Jq) * n] = acc[t];
  }
}

// The update of the last round of a sweep, in place.
__global__ void __launch_bounds__(kBJUThreads)
k_bj_update(int n, int n2p, int r, cplx* __restrict__ A, cplx* __restrict__ V,
            const cplx* __restrict__ Qk, const int* __restrict__ conv) {
  if (conv[0]) return;
  __shared__ cplx sm[kBJUpdateSm];
  bj_update_body(n, n2p, r, A, A, V, Qk, blockIdx.x, sm);
}

// Sub-problem of round r's pair (I, J) of M_r = G^H M G, G the block-
// diagonal unitary of round r - 1 (Qin, its pairs), M = Min, formed by the
// workgroup itself: with block I in round-(r-1) pair p1 (offset o1 = 0 for
// its first block, kBJ for its second) and J in p2, entry (a, b) of the
// (I, I) block is sum conj(Q_p1(m, o1 + a)) M[idx_p1(m), idx_p1(n)]
// Q_p1(n, o1 + b), and so on for (I, J) and (J, J); (J, I) is the conjugate
// transpose of (I, J).  The products run in the order of bj_update_body
// (Q^H M first, then the right factor), the sums over m and n ascending.
// sm: kBJLookSm entries of scratch (disjoint from a0).
constexpr int kBJLookSm = (kBJS + 1) * kBJS + 4 * kBJS * kBJ + kBJ * (kBJS + 1);
__device__ __forceinline__ void bj_lookahead(int n2p, int r, int I, int J, const cplx* __restrict__ Min,
                                             const cplx* __restrict__ Qin, cplx* a0, cplx* sm) {
  constexpr int LX = kBJS + 1, LT = kBJ;
  const int tid = threadIdx.x;
  const int nblk = n2p / kBJ, npair = nblk / 2;
  int p1 = 0, o1 = 0, p2 = 0, o2 = 0;
  for (int k = 0; k < npair; ++k) {
    int Ik, Jk;
    rr_pair(r - 1, k, nblk, &Ik, &Jk);
    if (Ik == I) { p1 = k; o1 = 0; }
    if (Jk == I) { p1 = k; o1 = kBJ; }
    if (Ik == J) { p2 = k; o2 = 0; }
    if (Jk == J) { p2 = k; o2 = kBJ; }
  }
  int I1, J1, I2, J2;
  rr_pair(r - 1, p1, nblk, &I1, &J1);
  rr_pair(r - 1, p2, nblk, &I2, &J2);
  cplx* X = sm;                         // [i + j LX]: a kBJS x kBJS block of Min
  cplx* L1 = X + LX * kBJS;             // [a + m kBJ] = conj(Q_p1(m, o1 + a))
  cplx* L2 = L1 + kBJS * kBJ;           // the same for p2
  cplx* R1 = L2 + kBJS * kBJ;           // [m + b kBJS] = Q_p1(m, o1 + b)
  cplx* R2 = R1 + kBJS * kBJ;
  cplx* T = R2 + kBJS * kBJ;            // [a + j LT]: (Q^H X)(a, j), kBJ x kBJS
  const cplx* q1 = Qin + (int64_t)p1 * kBJS * kBJS;
  const cplx* q2 = Qin + (int64_t)p2 * kBJS * kBJS;
  // three blocks: (I, I) from (p1, p1), (I, J) from (p1, p2), (J, J) from
  // (p2, p2); each block's entries are loaded into registers while the
  // previous block's products run
  constexpr int NX = kBJS * kBJS / kBJInnerThreads;
  typedef double dv2 __attribute__((ext_vector_type(2)));   // native vector: stays in registers
  dv2 xr[NX];
  auto load_x = [&](int blk) {
    const int Ir = blk < 2 ? I1 : I2, Jr = blk < 2 ? J1 : J2;       // row pair of Min
    const int Ic = blk == 0 ? I1 : I2, Jc = blk == 0 ? J1 : J2;     // column pair
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const int idx = tid + t * kBJInnerThreads;
      const int j = idx / kBJS, i = idx - j * kBJS;
      xr[t] = *reinterpret_cast<const dv2*>(Min + bj_index(i, Ir, Jr) + (int64_t)bj_index(j, Ic, Jc) * n2p);
    }
  };
  load_x(0);
  for (int idx = tid; idx < kBJS * kBJ; idx += kBJInnerThreads) {
    const int b = idx / kBJS, m = idx - b * kBJS;
    const cplx v1 = q1[m + (o1 + b) * kBJS], v2 = q2[m + (o2 + b) * kBJS];
    R1[idx] = v1;
    R2[idx] = v2;
    L1[b + m * kBJ] = cconj(v1);
    L2[b + m * kBJ] = cconj(v2);
  }
  for (int blk = 0; blk < 3; ++blk) {
    const cplx* L = blk < 2 ? L1 : L2;
    const cplx* R = blk == 0 ? R1 : R2;
    const int da = blk < 2 ? 0 : kBJ, db = blk == 0 ? 0 : kBJ;      // place in the sub-problem
    __syncthreads();   // X and T free (previous block done; Q copies stored)
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const int idx = tid + t * kBJInnerThreads;
      const int j = idx / kBJS, i = idx - j * kBJS;
      X[i + j * LX] = make_double2(xr[t].x, xr[t].y);
    }
    if (blk < 2) load_x(blk + 1);
    __syncthreads();
    {   // T = L X: kBJ x kBJS, two entries per thread
      const int a = tid % kBJ, j0 = tid / kBJ;
      cplx acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
#pragma unroll 8
      for (int m = 0; m < kBJS; ++m) {
        const cplx qh = L[a + m * kBJ];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const cplx x = X[m + (j0 + t * kBJ) * LX];
          acc[t].x += qh.x * x.x - qh.y * x.y;
          acc[t].y += qh.x * x.y + qh.y * x.x;
        }
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) T[a + (j0 + t * kBJ) * LT] = acc[t];
    }
    __syncthreads();
    {   // S = T R: kBJ x kBJ, one entry per thread
      const int a = tid % kBJ, b = tid / kBJ;
      cplx acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int m = 0; m < kBJS; ++m) {
        const cplx x = T[a + m * LT];
        const cplx qv = R[m + b * kBJS];
        acc.x += x.x * qv.x - x.y * qv.y;
        acc.y += x.x * qv.y + x.y * qv.x;
      }
      a0[(da + a) + (db + b) * kBJLA] = acc;
      if (blk == 1) a0[(db + b) + (da + a) * kBJLA] = cconj(acc);
    }
  }
  __syncthreads();
}

// Outer round r >= 1 of a sweep fused with the update of round r - 1.
// Workgroups [0, npair): the inner sweep of round r, each forming its
// sub-problem of the rotated matrix itself (bj_lookahead from Ain and Qin)
// and writing its rotations to Qout.  Workgroups [npair, npair + ugrid):
// the update of round r - 1 from Ain into Aout (and V) with Qin.  The two
// kinds read the same inputs and write disjoint outputs, so the update of
// one round runs beside the inner sweep of the next.
constexpr int kBJStepSm = kBJUpdateSm > kBJLA * kBJS + kBJLookSm ? kBJUpdateSm : kBJLA * kBJS + kBJLookSm;
static_assert(kBJLookSm >= kBJLA * kBJS + kBJS * kBJS, "the inner sweep's a1 and v fit the scratch");
__global__ void __launch_bounds__(kBJUThreads)
k_bj_step(int n, int n2p, int r, const cplx* __restrict__ Ain, cplx* __restrict__ Aout,
          cplx* __restrict__ V, const cplx* __restrict__ Qin, cplx* __restrict__ Qout,
          const int* __restrict__ conv) {
  if (conv[0]) return;
  __shared__ cplx sm[kBJStepSm];
  const int npair = n2p / kBJ / 2;
  if ((int)blockIdx.x >= npair) {
    bj_update_body(n, n2p, r - 1, Ain, Aout, V, Qin, blockIdx.x - npair, sm);
    return;
  }
  int I, J;
  rr_pair(r, blockIdx.x, n2p / kBJ, &I, &J);
  cplx* a0 = sm;
  cplx* scr = sm + kBJLA * kBJS;
  bj_lookahead(n2p, r, I, J, Ain, Qin, a0, scr);
  bj_inner_sweep(a0, scr, scr + kBJLA * kBJS, Qout + (int64_t)blockIdx.x * kBJS * kBJS);
}

// A0 = [a 0; 0 0] (n2 x n2), V0 = [I 0] (n x n2)
__global__ void k_jacobi_init(int n, int n2, const cplx* __restrict__ a, int64_t lda,
                              cplx* __restrict__ A0, cplx* __restrict__ V0, int* __restrict__ conv) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0) {
    conv[0] = 0;   // converged
    conv[1] = 0;   // sweeps when it converged
  }
  const int64_t na = (int64_t)n2 * n2;
  if (idx < na) {
    const int j = (int)(idx / n2), i = (int)(idx - (int64_t)j * n2);
    A0[idx] = (i < n && j < n) ? a[i + (int64_t)j * lda] : make_double2(0.0, 0.0);
    return;
  }
  const int64_t vi = idx - na;
  if (vi >= (int64_t)n * n2) return;
  const int j = (int)(vi / n), i = (int)(vi - (int64_t)j * n);
  V0[vi] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

// Rank of index p's eigenvalue among 0..n-1 (ties by index).
__global__ void k_jacobi_rank(int n, int ld, const cplx* __restrict__ A, int* __restrict__ rank,
                              const int* __restrict__ conv, int* __restrict__ sweeps_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) sweeps_out[0] = conv[0] ? conv[1] : -1;
  if (p >= n) return;
  const double dp = A[p + (int64_t)p * ld].x;
  int rk = 0;
  for (int q = 0; q < n; ++q) {
    const double dq = A[q + (int64_t)q * ld].x;
    if (dq < dp || (dq == dp && q < p)) ++rk;
  }
  rank[p] = rk;
}

__global__ void k_jacobi_scatter(int n, int ld, const cplx* __restrict__ A,
                                 const cplx* __restrict__ V, const int* __restrict__ rank,
                                 double* __restrict__ w, cplx* __restrict__ Q, int64_t ldq) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int p = (int)(idx / n), i = (int)(idx - (int64_t)p * n);
  const int rp = rank[p];
  Q[i + (int64_t)rp * ldq] = V[i + (int64_t)p * n];
  if (i == 0) w[rp] = A[p + (int64_t)p * ld].x;
}

// Squared off-diagonal and total Frobenius norms of A (n x n), in two fixed-
// order stages: kOffParts workgroups sum interleaved slices into part[2 w],
// part[2 w + 1]; one workgroup adds the parts.
constexpr int kOffParts = 256;
__global__ void __launch_bounds__(256) k_offnorm_part(int n, const cplx* __restrict__ A,
                                                      double* __restrict__ part,
                                                      const int* __restrict__ conv) {
  if (conv[0]) return;
  __shared__ double r1[256], r2[256];
  double off = 0.0, tot = 0.0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < nn;
       idx += (int64_t)kOffParts * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const double m2 = cabs2(A[idx]);
    tot += m2;
    if (i != j) off += m2;
  }
  r1[threadIdx.x] = off;
  r2[threadIdx.x] = tot;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

// ... and sets conv = {1, sweep} when off <= tol2 * total (the test that
// precedes outer sweep `sweep`).
__global__ void __launch_bounds__(kOffParts) k_offnorm_final(const double* __restrict__ part,
                                                            double tol2, int sweep,
                                                            int* __restrict__ conv) {
  if (conv[0]) return;
  __shared__ double r1[kOffParts], r2[kOffParts];
  r1[threadIdx.x] = part[2 * threadIdx.x];
  r2[threadIdx.x] = part[2 * threadIdx.x + 1];
  __syncthreads();
  for (int s = kOffParts / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && r1[0] <= tol2 * r2[0]) {
    conv[1] = sweep;
    conv[0] = 1;
  }
}

// ---------------------------------------------------------------------------
// precision conversions for the low-precision filter path
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_to_f32_body(int64_t rows, int64_t cols, const cplx* __restrict__ x, int64_t ldx,
                               float2* __restrict__ y, int64_t ldy, int bx_) {
  const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  const cplx v = x[i + j * ldx];
  y[i + j * ldy] = make_float2((float)v.x, (float)v.y);
}

__global__ void 
k_block_to_f32(int64_t rows, int64_t cols, const cplx* __restrict__ x, int64_t ldx,
                               float2* __restrict__ y, int64_t ldy) {
  block_to_f32_body(rows, cols, x, ldx, y, ldy, blockIdx.x);
}

__device__ __forceinline__ void block_to_f64_body(int64_t rows, int64_t cols, const float2* __restrict__ x, int64_t ldx,
                               cplx* __restrict__ y, int64_t ldy, int bx_) {
  const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  const float2 v = x[i + j * ldx];
  y[i + j * ldy] = make_double2((double)v.x, (double)v.y);
}

__global__ void 
k_block_to_f64(int64_t rows, int64_t cols, const float2* __restrict__ x, int64_t ldx,
                               cplx* __restrict__ y, int64_t ldy) {
  block_to_f64_body(rows, cols, x, ldx, y, ldy, blockIdx.x);
}

// out = fp32(a x + b y), x and y FP64
__device__ __forceinline__ void axpby_to_f32_body(int64_t rows, int64_t cols, double a, const cplx* __restrict__ x,
                               int64_t ldx, double b, const cplx* __restrict__ y, int64_t ldy,
                               float2* __restrict__ out, int64_t ldo, const double* __restrict__ coef, int bx_) {
  const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  if (coef) {
    a = coef[0];
    b = coef[1];
  }
  const int64_t j = idx / rows, i = idx - j * rows;
  const cplx u = x[i + j * ldx], v = y[i + j * ldy];
  out[i + j * ldo] = make_float2((float)(a * u.x + b * v.x), (float)(a * u.y + b * v.y));
}

__global__ void 
k_axpby_to_f32(int64_t rows, int64_t cols, double a, const cplx* __restrict__ x,
                               int64_t ldx, double b, const cplx* __restrict__ y, int64_t ldy,
                               float2* __restrict__ out, int64_t ldo, const double* __restrict__ coef) {
  axpby_to_f32_body(rows, cols, a, x, ldx, b, y, ldy, out, ldo, coef, blockIdx.x);
}

__global__ void k_real_to_f32(int64_t n, const double* __restrict__ src, double scale,
                              float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)(scale * src[i]);
}

__global__ void k_tw_to_f32(int n, const cplx* __restrict__ src, float2* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

// Chebyshev filter coefficients on the device from the current Ritz values
// (a = largest, a0 = smallest) and the upper bound b: step i (0-based) of the
// scaled recurrence is out = alpha (H in) + beta in + gamma prev with
//   i = 0: alpha = s/e, beta = -s c/e, gamma = 0            (s = e/(a0 - c))
//   i > 0: s' = 1/(2/s_0 - s), alpha = 2 s'/e, beta = -alpha c, gamma = -s s'; s = s'
// If a0 < a < b fails, every step becomes the identity and flag[0] is set.
__device__ __forceinline__ void cheb_coef_body(const double* __restrict__ eig, int nb, const double* __restrict__ upper,
                            int degree, double* __restrict__ coef, int* flag) {
  if (threadIdx.x != 0) return;
  const double a = eig[nb - 1], a0 = eig[0], b = upper[0];
  if (!(a0 < a && a < b)) {
    for (int i = 0; i < degree; ++i) {
      coef[3 * i] = 0.0;
      coef[3 * i + 1] = 1.0;
      coef[3 * i + 2] = 0.0;
    }
    flag[0] = 1;
    return;
  }
  const double e = 0.5 * (b - a), c = 0.5 * (b + a);
  double sigma = e / (a0 - c);
  const double tau = 2.0 / sigma;
  coef[0] = sigma / e;
  coef[1] = -sigma * c / e;
  coef[2] = 0.0;
  for (int i = 1; i < degree; ++i) {
    const double sn = 1.0 / (tau - sigma);
    const double al = 2.0 * sn / e;
    coef[3 * i] = al;
    coef[3 * i + 1] = -al * c;
    coef[3 * i + 2] = -sigma * sn;
    sigma = sn;
  }
}

__global__ void 
k_cheb_coef(const double* __restrict__ eig, int nb, const double* __restrict__ upper,
                            int degree, double* __restrict__ coef, int* flag) {
  cheb_coef_body(eig, nb, upper, degree, coef, flag);
}

// Sticky per-item failure flags of a batched iteration:
// flags[0] = first failing Cholesky pivot + 1 (or -(column + 1) for a Gram
// diagonal entry that is not finite), flags[1] = eigensolver hit the
// sweep limit, flags[2] = bad filter interval (set by k_cheb_coef),
// flags[3] = largest sweep count seen.
__device__ __forceinline__ void batch_flags_body(const int* __restrict__ chol_status, const int* __restrict__ sweeps,
                              int* flags) {
  if (threadIdx.x != 0) return;
  if (chol_status && chol_status[0] != -1 && flags[0] == 0)
    flags[0] = chol_status[0] >= 0 ? chol_status[0] + 1 : chol_status[0] - kCholNonFinite - 1;
  const int sw = sweeps[0];
  if (sw < 0) flags[1] = 1;
  else if (sw > flags[3]) flags[3] = sw;
}

__global__ void 
k_batch_flags(const int* __restrict__ chol_status, const int* __restrict__ sweeps,
                              int* flags) {
  batch_flags_body(chol_status, sweeps, flags);
}

// ---- fused-batch steps: item = blockIdx.y for the element-wise steps (x covers
// the largest item), blockIdx.x for the one-workgroup steps
__global__ void kb_cheb_coef(const ItemDev* __restrict__ D, int degree) {
  const ItemDev& d = D[blockIdx.x];
  cheb_coef_body(d.eig, d.nb, d.upper, degree, d.coef, d.flags + 2);
}

// first filter step from W = H Y: FP64 blk, or FP32 b32[1]
__global__ void kb_filter_first(const ItemDev* __restrict__ D, int fp32) {
  const ItemDev& d = D[blockIdx.y];
  if (fp32)
    axpby_to_f32_body(d.npw, d.nb, 0.0, d.hy, d.npw, 0.0, d.y, d.npw, d.b32[1], d.npw, d.coef,
                      blockIdx.x);
  else
    axpby_block_body(d.npw, d.nb, 0.0, d.hy, d.npw, 0.0, d.y, d.npw, d.blk, d.npw, d.coef,
                     blockIdx.x);
}

__global__ void kb_to_f32(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.y];
  block_to_f32_body(d.npw, d.nb, d.y, d.npw, d.b32[0], d.npw, blockIdx.x);
}

__global__ void kb_to_f64(const ItemDev* __restrict__ D, int sel) {
  const ItemDev& d = D[blockIdx.y];
  block_to_f64_body(d.npw, d.nb, item_blk32(d, sel), d.npw, d.y, d.npw, blockIdx.x);
}

__global__ void kb_copy(const ItemDev* __restrict__ D, int sel_src, int sel_dst) {
  const ItemDev& d = D[blockIdx.y];
  copy_block_body(d.npw, d.nb, item_blk64(d, sel_src), d.npw, item_blk64(d, sel_dst), d.npw,
                  blockIdx.x);
}

__global__ void kb_hermitize(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.y];
  hermitize_body(d.nb, d.sub0, d.nb, blockIdx.x);
}

__global__ void __launch_bounds__(1024) kb_chol_init(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.x];
  chol_init_body(d.nb, d.sub0, d.nb, d.dtol, d.status);
}

__global__ void __launch_bounds__(256) kb_chol_diag(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.x];
  chol_diag_body(d.nb, 0, d.sub0, d.nb, d.dinv, d.dtol, d.status);
}

__global__ void __launch_bounds__(kJacThreads) kb_jacobi(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.x];
  jacobi_small_body(d.nb, d.sub0, d.nb, d.eig, d.sub1, d.nb, d.sweeps);
}

__global__ void __launch_bounds__(256) kb_residuals(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.y];
  if ((int)blockIdx.x >= d.nb) return;
  residuals_body(d.npw, d.hy, d.npw, d.y, d.npw, d.eig, d.resid, blockIdx.x);
}

__global__ void kb_flags(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.x];
  batch_flags_body(d.status, d.sweeps, d.flags);
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_kinetic(int64_t npw, const int* miller, const double* recip9, const double* k3,
                          double* kin, hipStream_t s) {
  KinArgs a;
  for (int i = 0; i < 9; ++i) a.b[i] = recip9[i];
  for (int i = 0; i < 3; ++i) a.k[i] = k3[i];
  hipLaunchKernelGGL(k_kinetic, dim3(nblocks(npw, 256)), dim3(256), 0, s, npw, miller, a, kin);
  return hipGetLastError();
}

hipError_t launch_scale_copy(int64_t n, const double* src, double scale, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(nblocks(n, 256)), dim3(256), 0, s, n, src, scale, dst);
  return hipGetLastError();
}

hipError_t launch_max_reduce(int64_t n, const double* x, double* out1, hipStream_t s) {
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(1024), 0, s, n, x, out1);
  return hipGetLastError();
}

hipError_t launch_check_finite(int64_t n, const double* x, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, dim3(nblocks(n, 256)), dim3(256), 0, s, n, x, flag);
  return hipGetLastError();
}

hipError_t launch_hermitize(int64_t n, cplx* a, int64_t lda, hipStream_t s) {
  hipLaunchKernelGGL(k_hermitize, dim3(nblocks(n * n, 256)), dim3(256), 0, s, n, a, lda);
  return hipGetLastError();
}

hipError_t launch_copy_block(int64_t rows, int64_t cols, const cplx* src, int64_t lds, cplx* dst,
                             int64_t ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_block, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows, cols, src,
                     lds, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_scale_rows_cols(int64_t n, const double* d, cplx* a, int64_t lda, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rows_cols, dim3(nblocks(n * n, 256)), dim3(256), 0, s, n, d, a, lda);
  return hipGetLastError();
}

hipError_t launch_axpby_block(int64_t npw, int64_t nb, double a, const cplx* x, int64_t ldx, double b,
                              const cplx* y, int64_t ldy, cplx* out, int64_t ldo, hipStream_t s,
                              const double* coef) {
  hipLaunchKernelGGL(k_axpby_block, dim3(nblocks(npw * nb, 256)), dim3(256), 0, s, npw, nb, a, x,
                     ldx, b, y, ldy, out, ldo, coef);
  return hipGetLastError();
}

hipError_t launch_batch_flags(const int* chol_status, const int* sweeps, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_flags, dim3(1), dim3(64), 0, s, chol_status, sweeps, flags);
  return hipGetLastError();
}

hipError_t launch_cheb_coef(const double* eig, int nb, const double* upper, int degree, double* coef,
                            int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_cheb_coef, dim3(1), dim3(64), 0, s, eig, nb, upper, degree, coef, flag);
  return hipGetLastError();
}

hipError_t launch_block_to_f32(int64_t rows, int64_t cols, const cplx* x, int64_t ldx, float2* y,
                               int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_to_f32, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows, cols, x,
                     ldx, y, ldy);
  return hipGetLastError();
}

hipError_t launch_block_to_f64(int64_t rows, int64_t cols, const float2* x, int64_t ldx, cplx* y,
                               int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_to_f64, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows, cols, x,
                     ldx, y, ldy);
  return hipGetLastError();
}

hipError_t launch_axpby_to_f32(int64_t rows, int64_t cols, double a, const cplx* x, int64_t ldx,
                               double b, const cplx* y, int64_t ldy, float2* out, int64_t ldo,
                               hipStream_t s, const double* coef) {
  hipLaunchKernelGGL(k_axpby_to_f32, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows, cols, a,
                     x, ldx, b, y, ldy, out, ldo, coef);
  return hipGetLastError();
}

__global__ void k_block_to_b16(int64_t rows, int64_t cols, const cplx* __restrict__ x, int64_t ldx,
                               bf16c* __restrict__ y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  y[i + j * ldy] = st_c<bf16c>(x[i + j * ldx]);
}

__global__ void k_block_b16_to_f64(int64_t rows, int64_t cols, const bf16c* __restrict__ x,
                                   int64_t ldx, cplx* __restrict__ y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  const float2 v = ld_c(x[i + j * ldx]);
  y[i + j * ldy] = make_double2(v.x, v.y);
}

__global__ void k_axpby_to_b16(int64_t rows, int64_t cols, double a, const cplx* __restrict__ x,
                               int64_t ldx, double b, const cplx* __restrict__ y, int64_t ldy,
                               bf16c* __restrict__ out, int64_t ldo, const double* __restrict__ coef) {
  if (coef) {
    a = coef[0];
    b = coef[1];
  }
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  const cplx u = x[i + j * ldx], v = y[i + j * ldy];
  out[i + j * ldo] = st_c<bf16c>(make_double2(a * u.x + b * v.x, a * u.y + b * v.y));
}

hipError_t launch_block_to_b16(int64_t rows, int64_t cols, const cplx* x, int64_t ldx, bf16c* y,
                               int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_to_b16, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows, cols,
                     x, ldx, y, ldy);
  return hipGetLastError();
}

hipError_t launch_block_b16_to_f64(int64_t rows, int64_t cols, const bf16c* x, int64_t ldx, cplx* y,
                                   int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_b16_to_f64, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows,
                     cols, x, ldx, y, ldy);
  return hipGetLastError();
}

hipError_t launch_axpby_to_b16(int64_t rows, int64_t cols, double a, const cplx* x, int64_t ldx,
                               double b, const cplx* y, int64_t ldy, bf16c* out, int64_t ldo,
                               hipStream_t s, const double* coef) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby_to_b16, dim3(nblocks(rows * cols, 256)), dim3(256), 0, s, rows, cols,
                     a, x, ldx, b, y, ldy, out, ldo, coef);
  return hipGetLastError();
}

hipError_t launch_real_to_f32(int64_t n, const double* src, double scale, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_real_to_f32, dim3(nblocks(n, 256)), dim3(256), 0, s, n, src, scale, dst);
  return hipGetLastError();
}

hipError_t launch_tw_to_f32(int n, const cplx* src, float2* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_tw_to_f32, dim3(nblocks(n, 256)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_residuals(int64_t npw, int64_t nb, const cplx* W, int64_t ldw, const cplx* Y,
                            int64_t ldy, const double* lam, double* resid, hipStream_t s) {
  hipLaunchKernelGGL(k_residuals, dim3((unsigned)nb), dim3(256), 0, s, npw, W, ldw, Y, ldy, lam,
                     resid);
  return hipGetLastError();
}

hipError_t launch_chol_init(int64_t n, const cplx* a, int64_t lda, double* tol, int* status,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_chol_init, dim3(1), dim3(1024), 0, s, (int)n, a, lda, tol, status);
  return hipGetLastError();
}

hipError_t launch_chol_diag(int kb, int k0, cplx* a, int64_t lda, cplx* dinv, const double* tol,
                            int* status, hipStream_t s) {
  const size_t lds = (size_t)2 * kb * (kb + 1) * sizeof(cplx);
  hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), lds, s, kb, k0, a, lda, dinv, tol, status);
  return hipGetLastError();
}

hipError_t launch_zero_lower(int64_t n, cplx* a, int64_t lda, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_lower, dim3(nblocks(n * n, 256)), dim3(256), 0, s, (int)n, a, lda);
  return hipGetLastError();
}

hipError_t launch_identity(int64_t n, cplx* a, int64_t lda, hipStream_t s) {
  hipLaunchKernelGGL(k_identity_ld, dim3(nblocks(n * n, 256)), dim3(256), 0, s, (int)n, a, lda);
  return hipGetLastError();
}

// padded size: a multiple of the update tiles (and so of 2 kBJ)
static int64_t bj_padded(int64_t n) { return (n + kBJTile - 1) / kBJTile * kBJTile; }

// Work layout for n > 64: A (n2p x n2p), V (n x n2p), the block pairs'
// unitaries (n2p / kBJS of kBJS x kBJS), n ints of ranks, then two 16-byte
// aligned doubles.
size_t heev_work_bytes(int64_t n) {
  const int64_t n2p = bj_padded(n);
  return (size_t)(2 * n2p * n2p + n * n2p + 2 * n2p * kBJS) * sizeof(cplx) +
         (size_t)(n + 8) * sizeof(int) + 64 + 2 * kOffParts * sizeof(double);
}

hipError_t heev_set_lds_limit(size_t bytes) {
  const void* fns[4] = {(const void*)k_jacobi_small, (const void*)k_chol_diag,
                        (const void*)kb_jacobi, (const void*)kb_chol_diag};
  for (const void* f : fns) {
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, f);
    if (e != hipSuccess) return e;
    const size_t dyn = bytes > at.sharedSizeBytes ? bytes - at.sharedSizeBytes : 0;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_heev_small_async(int64_t n, const cplx* a, int64_t lda, double* w, cplx* q,
                                   int64_t ldq, int* sweeps_dev, hipStream_t s) {
  if (n > kJacSmallMax) return hipErrorInvalidValue;
  const size_t lds = (size_t)(n * (2 * n + 1)) * sizeof(cplx);
  hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(jac_threads((int)n)), lds, s, (int)n, a, lda, w,
                     q, ldq, sweeps_dev);
  return hipGetLastError();
}

hipError_t launch_heev_async(int64_t n, const cplx* a, int64_t lda, double* w, cplx* q,
                             int64_t ldq, void* work, int* sweeps_dev, int max_sweeps,
                             hipStream_t s) {
  if (n <= kJacSmallMax) return launch_heev_small_async(n, a, lda, w, q, ldq, sweeps_dev, s);
  if (max_sweeps < 1 || max_sweeps > kMaxSweeps) return hipErrorInvalidValue;
  const int64_t n2p = bj_padded(n);
  char* base = static_cast<char*>(work);
  const size_t mat_bytes = (size_t)(2 * n2p * n2p + n * n2p + 2 * n2p * kBJS) * sizeof(cplx);
  int* rank = reinterpret_cast<int*>(base + mat_bytes);
  int* conv = rank + n;                  // {converged, sweeps}
  const size_t stat_off = (mat_bytes + (size_t)(n + 8) * sizeof(int) + 15) & ~(size_t)15;
  double* dpart = reinterpret_cast<double*>(base + stat_off) + 2;   // kOffParts pairs
  // A: the matrix at the start of every sweep; A1: the other copy of the
  // fused rounds (each reads one and writes the other, an even number per
  // sweep); Q0 / Q1: the unitaries of consecutive rounds
  cplx* A = reinterpret_cast<cplx*>(base);
  cplx* A1 = A + n2p * n2p;
  cplx* V = A1 + n2p * n2p;
  cplx* Q0 = V + n * n2p;
  cplx* Q1 = Q0 + n2p * kBJS;
  hipLaunchKernelGGL(k_jacobi_init, dim3(nblocks(n2p * n2p + n * n2p, 256)), dim3(256), 0, s,
                     (int)n, (int)n2p, a, lda, A, V, conv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nblk = (int)(n2p / kBJ), npair = nblk / 2;
  const int vtiles = (int)((n + kBJTile - 1) / kBJTile);
  const unsigned ugrid = (unsigned)(npair * npair + vtiles * npair);
  const double tl = std::max(1e-15, 2.2e-16 * (double)n);
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    hipLaunchKernelGGL(k_offnorm_part, dim3(kOffParts), dim3(256), 0, s, (int)n2p, (const cplx*)A,
                       dpart, (const int*)conv);
    hipLaunchKernelGGL(k_offnorm_final, dim3(1), dim3(kOffParts), 0, s, (const double*)dpart,
                       tl * tl, sw, conv);
    if (sw == max_sweeps) break;
    // round 0 from A; rounds 1 .. nblk - 2 each beside the previous round's
    // update (A -> A1 -> A ...: nblk - 2 copies, even); the last update in place
    hipLaunchKernelGGL(k_bj_inner, dim3(npair), dim3(kBJInnerThreads), 0, s, (int)n2p, 0,
                       (const cplx*)A, Q0, (const int*)conv);
    cplx* cur = A;
    cplx* nxt = A1;
    for (int r = 1; r < nblk - 1; ++r) {
      hipLaunchKernelGGL(k_bj_step, dim3((unsigned)npair + ugrid), dim3(kBJUThreads), 0, s, (int)n,
                         (int)n2p, r, (const cplx*)cur, nxt, V, (const cplx*)(r & 1 ? Q0 : Q1),
                         r & 1 ? Q1 : Q0, (const int*)conv);
      std::swap(cur, nxt);
    }
    hipLaunchKernelGGL(k_bj_update, dim3(ugrid), dim3(kBJUThreads), 0, s, (int)n, (int)n2p,
                       nblk - 2, cur, V, (const cplx*)((nblk - 2) & 1 ? Q1 : Q0), (const int*)conv);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_jacobi_rank, dim3(nblocks(n, 256)), dim3(256), 0, s, (int)n, (int)n2p,
                     (const cplx*)A, rank, (const int*)conv, sweeps_dev);
  hipLaunchKernelGGL(k_jacobi_scatter, dim3(nblocks(n * n, 256)), dim3(256), 0, s, (int)n, (int)n2p,
                     (const cplx*)A, (const cplx*)V, (const int*)rank, w, q, ldq);
  return hipGetLastError();
}

hipError_t launch_heev(int64_t n, const cplx* a, int64_t lda, double* w, cplx* q, int64_t ldq,
                       void* work, int* sweeps_dev, int* host_scratch, int* sweeps_done,
                       hipStream_t s) {
  hipError_t e = launch_heev_async(n, a, lda, w, q, ldq, work, sweeps_dev, kMaxSweeps, s);
  if (e == hipSuccess) e = hipMemcpyAsync(host_scratch, sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) *sweeps_done = host_scratch[0];
  return e;
}

// First failure since the last clear wins: rec = {status, op, info}.
__global__ void k_status_record(const int* __restrict__ chol_status, const int* __restrict__ sweeps,
                                int op, int* __restrict__ rec) {
  if (threadIdx.x != 0 || rec[0] != 0) return;
  if (chol_status && chol_status[0] >= 0) {
    rec[0] = 5;   // PW_ERR_NOT_POSDEF
    rec[1] = op;
    rec[2] = chol_status[0];
  } else if (chol_status && chol_status[0] <= kCholNonFinite) {
    rec[0] = 6;   // PW_ERR_NONFINITE
    rec[1] = op;
    rec[2] = kCholNonFinite - chol_status[0];
  } else if (sweeps && sweeps[0] < 0) {
    rec[0] = 7;   // PW_ERR_NO_CONVERGENCE
    rec[1] = op;
    rec[2] = 0;
  }
}

__global__ void k_fill_int(int n, int v, int* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_status_record(const int* chol_status, const int* sweeps, int op, int* rec,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_status_record, dim3(1), dim3(64), 0, s, chol_status, sweeps, op, rec);
  return hipGetLastError();
}

hipError_t launch_fill_int(int n, int v, int* p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, n, v, p);
  return hipGetLastError();
}

// ---- fused-batch step launchers (npw_nb_max = max over items of npw * nb)
hipError_t launch_fused_dense(FusedStep step, int nitems, int64_t npw_nb_max, int nb_max,
                              const ItemDev* D, int arg0, int arg1, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 ew(nblocks(npw_nb_max, 256), nitems);
  switch (step) {
    case FS_CHEB_COEF:
      hipLaunchKernelGGL(kb_cheb_coef, dim3(nitems), dim3(64), 0, s, D, arg0);
      break;
    case FS_FILTER_FIRST:
      hipLaunchKernelGGL(kb_filter_first, ew, dim3(256), 0, s, D, arg0);
      break;
    case FS_TO_F32:
      hipLaunchKernelGGL(kb_to_f32, ew, dim3(256), 0, s, D);
      break;
    case FS_TO_F64:
      hipLaunchKernelGGL(kb_to_f64, ew, dim3(256), 0, s, D, arg0);
      break;
    case FS_COPY:
      hipLaunchKernelGGL(kb_copy, ew, dim3(256), 0, s, D, arg0, arg1);
      break;
    case FS_HERMITIZE:
      hipLaunchKernelGGL(kb_hermitize, dim3(nblocks((int64_t)nb_max * nb_max, 256), nitems),
                         dim3(256), 0, s, D);
      break;
    case FS_CHOL_INIT:
      hipLaunchKernelGGL(kb_chol_init, dim3(nitems), dim3(1024), 0, s, D);
      break;
    case FS_CHOL_DIAG:
      hipLaunchKernelGGL(kb_chol_diag, dim3(nitems), dim3(256),
                         (size_t)2 * nb_max * (nb_max + 1) * sizeof(cplx), s, D);
      break;
    case FS_JACOBI:
      hipLaunchKernelGGL(kb_jacobi, dim3(nitems), dim3(jac_threads(nb_max)),
                         (size_t)(nb_max * (2 * nb_max + 1)) * sizeof(cplx), s, D);
      break;
    case FS_RESIDUALS:
      hipLaunchKernelGGL(kb_residuals, dim3(nb_max, nitems), dim3(256), 0, s, D);
      break;
    case FS_FLAGS:
      hipLaunchKernelGGL(kb_flags, dim3(nitems), dim3(64), 0, s, D);
      break;
  }
  return hipGetLastError();
}
