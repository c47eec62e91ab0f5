// Small dense FP64 linear algebra of the subspace steps, plus element-wise
// helpers.  Section 5.1 (Rayleigh-Ritz: a dense Hermitian eigenproblem of
// the block size) and section 5.4 (full-band Cholesky orthogonalisation).
//
//  * potrf_inv : S = U^H U (upper Cholesky, right-looking) then U^{-1}
//                (column-oriented triangular inverse), one workgroup.
//  * heev      : cyclic two-sided Jacobi with the round-robin (circle)
//                ordering: in each round all n/2 disjoint pairs rotate at
//                once, A <- G^H A G, V <- V G.  For n <= 64 the whole solve
//                runs in one workgroup with A and V in LDS; larger n run one
//                kernel per round over 2x2 blocks of A (ping-pong buffers).
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

// A <- (A + A^H)/2
__global__ void k_hermitize(int64_t n, cplx* a, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  if (i > j) return;
  if (i == j) {
    a[i + j * lda].y = 0.0;
    return;
  }
  const cplx u = a[i + j * lda], l = a[j + i * lda];
  const cplx avg = make_double2(0.5 * (u.x + l.x), 0.5 * (u.y - l.y));
  a[i + j * lda] = avg;
  a[j + i * lda] = cconj(avg);
}

__global__ void k_copy_block(int64_t rows, int64_t cols, const cplx* __restrict__ src, int64_t lds,
                             cplx* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  dst[i + j * ldd] = src[i + j * lds];
}

__global__ void k_scale_rows_cols(int64_t n, const double* __restrict__ d, cplx* a, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  a[i + j * lda] = cscale(a[i + j * lda], d[i] * d[j]);
}

__global__ void k_axpby_block(int64_t npw, int64_t nb, double a, const cplx* x, int64_t ldx,
                              double b, const cplx* y, int64_t ldy, cplx* out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npw * nb) return;
  const int64_t j = idx / npw, i = idx - j * npw;
  const cplx u = x[i + j * ldx], v = y[i + j * ldy];
  out[i + j * ldo] = make_double2(a * u.x + b * v.x, a * u.y + b * v.y);
}

__global__ void __launch_bounds__(256)
k_residuals(int64_t npw, const cplx* __restrict__ W, int64_t ldw, const cplx* __restrict__ Y,
            int64_t ldy, const double* __restrict__ lam, double* __restrict__ resid) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;
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

// ---------------------------------------------------------------------------
// Cholesky (upper, S = U^H U) and triangular inverse, single workgroup.
// A is read from its upper triangle and overwritten by U (strict lower part
// set to zero); X receives U^{-1}.  status[0] = -1 on success, else the index
// of the first pivot whose value is at or below n eps max_i S_ii.
// ---------------------------------------------------------------------------
constexpr int kCholThreads = 1024;

__global__ void __launch_bounds__(kCholThreads)
k_potrf_inv(int n, cplx* A, int64_t lda, cplx* X, int64_t ldx, int* status) {
  extern __shared__ cplx rowk[];   // n entries
  __shared__ double red[kCholThreads];
  __shared__ int fail;
  __shared__ double sh_tol, sh_inv;
  const int tid = threadIdx.x, nt = blockDim.x;
  double m = 0.0;
  for (int i = tid; i < n; i += nt) m = fmax(m, A[i + (int64_t)i * lda].x);
  red[tid] = m;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  if (tid == 0) {
    sh_tol = (double)n * DBL_EPSILON * red[0];
    fail = -1;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = A[k + (int64_t)k * lda].x;
      if (!(d > sh_tol)) {
        fail = k;
      } else {
        const double u = sqrt(d);
        A[k + (int64_t)k * lda] = make_double2(u, 0.0);
        sh_inv = 1.0 / u;
      }
    }
    __syncthreads();
    if (fail >= 0) break;
    const double inv = sh_inv;
    for (int j = k + 1 + tid; j < n; j += nt) {
      const cplx v = cscale(A[k + (int64_t)j * lda], inv);
      A[k + (int64_t)j * lda] = v;
      rowk[j] = v;
    }
    __syncthreads();
    // trailing update of the upper triangle: A[i][j] -= conj(U[k][i]) U[k][j], k < i <= j
    const int mrem = n - k - 1;
    const int64_t tot = (int64_t)mrem * mrem;
    for (int64_t idx = tid; idx < tot; idx += nt) {
      const int jj = (int)(idx / mrem), ii = (int)(idx - (int64_t)jj * mrem);
      if (ii > jj) continue;
      const int i = k + 1 + ii, j = k + 1 + jj;
      const cplx p = cmul(cconj(rowk[i]), rowk[j]);
      cplx a = A[i + (int64_t)j * lda];
      A[i + (int64_t)j * lda] = csub(a, p);
    }
    __syncthreads();
  }
  if (fail >= 0) {
    if (tid == 0) status[0] = fail;
    return;
  }
  // zero the strict lower triangle of U
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += nt) {
    const int j = (int)(idx / n), i = (int)(idx - (int64_t)j * n);
    if (i > j) A[i + (int64_t)j * lda] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  // X = U^{-1}, column by column: X[j][j] = 1/U[j][j];
  // X[i][j] = -(sum_{p=i}^{j-1} X[i][p] U[p][j]) / U[j][j] for i < j.
  for (int j = 0; j < n; ++j) {
    for (int p = tid; p <= j; p += nt) rowk[p] = A[p + (int64_t)j * lda];
    __syncthreads();
    const double ujj = rowk[j].x;
    const double rinv = 1.0 / ujj;
    for (int i = tid; i < n; i += nt) {
      cplx v;
      if (i < j) {
        double sr = 0.0, si = 0.0;
        for (int p = i; p < j; ++p) {
          const cplx x = X[i + (int64_t)p * ldx];
          const cplx u = rowk[p];
          sr += x.x * u.x - x.y * u.y;
          si += x.x * u.y + x.y * u.x;
        }
        v = make_double2(-sr * rinv, -si * rinv);
      } else if (i == j) {
        v = make_double2(rinv, 0.0);
      } else {
        v = make_double2(0.0, 0.0);
      }
      X[i + (int64_t)j * ldx] = v;
    }
    __syncthreads();
  }
  if (tid == 0) status[0] = -1;
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
  int a, b;
  if (k == 0) {
    a = m;
    b = r;
  } else {
    a = (r + k) % m;
    b = (r - k + m) % m;
  }
  *p = min(a, b);
  *q = max(a, b);
}

// Rotation J = [[cs, sn ph], [-sn conj(ph), cs]] with J^H [[a, c], [conj c, b]] J diagonal:
// tau = (b - a)/(2|c|), t = sign(tau)/(|tau| + sqrt(1 + tau^2)), cs = 1/sqrt(1+t^2), sn = t cs;
// new diagonal a - t|c|, b + t|c|.
__device__ __forceinline__ Rot make_rot(double a, double b, cplx c) {
  Rot R;
  const double mag = hypot(c.x, c.y);
  if (!(mag > DBL_MIN)) {
    R.cs = 1.0; R.sn = 0.0; R.t = 0.0; R.ph = make_double2(1.0, 0.0); R.on = false;
    return R;
  }
  const double tau = (b - a) / (2.0 * mag);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  R.cs = 1.0 / sqrt(1.0 + t * t);
  R.sn = t * R.cs;
  R.t = t * mag;
  R.ph = make_double2(c.x / mag, c.y / mag);
  R.on = true;
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
constexpr int kMaxSweeps = 40;

__device__ __forceinline__ double jac_tol(int n) { return fmax(1e-15, 2.2e-16 * n); }

// Whole Jacobi solve in LDS for n <= 64.
__global__ void __launch_bounds__(kJacThreads)
k_jacobi_small(int n, const cplx* __restrict__ Ain, int64_t lda, double* __restrict__ w,
               cplx* __restrict__ Q, int64_t ldq, int* sweeps_out) {
  extern __shared__ cplx sm[];
  const int n2 = n + (n & 1);
  const int h = n2 / 2;
  cplx* a = sm;               // n x n, ld n
  cplx* v = sm + n * n;       // n x n
  __shared__ Rot rots[kJacSmallMax / 2];
  __shared__ double red[kJacThreads];
  __shared__ double red2[kJacThreads];
  __shared__ int done;
  __shared__ int rank_[kJacSmallMax];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < n * n; idx += nt) {
    const int j = idx / n, i = idx - j * n;
    a[idx] = Ain[i + (int64_t)j * lda];
    v[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) done = 0;
  __syncthreads();
  int sweeps = 0;
  for (; sweeps < kMaxSweeps; ++sweeps) {
    // convergence test before the sweep
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < n * n; idx += nt) {
      const int j = idx / n, i = idx - j * n;
      const double m2 = cabs2(a[idx]);
      tot += m2;
      if (i != j) off += m2;
    }
    red[tid] = off;
    red2[tid] = tot;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
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
        if (q < n) rots[tid] = make_rot(a[p + p * n].x, a[q + q * n].x, a[p + q * n]);
        else rots[tid] = make_rot(0.0, 0.0, make_double2(0.0, 0.0));
      }
      __syncthreads();
      for (int idx = tid; idx < h * h; idx += nt) {
        const int P = idx / h, Qb = idx - P * h;
        int p1, q1, p2, q2;
        rr_pair(r, P, n2, &p1, &q1);
        rr_pair(r, Qb, n2, &p2, &q2);
        const Rot& RP = rots[P];
        const Rot& RQ = rots[Qb];
        if (q1 >= n || q2 >= n) {
          // pairs holding the padding index rotate nothing; update the real rows/cols only
          if (q1 < n && RP.on) {   // Q pair is (p2, pad): column p2 only
            cplx x1 = a[p1 + p2 * n], x2 = a[q1 + p2 * n];
            cplx y1 = x1, y2 = x2;
            // Jp^H [x1; x2]
            const cplx p12 = cscale(RP.ph, -RP.sn), p21 = cscale(cconj(RP.ph), RP.sn);
            y1 = cadd(cscale(x1, RP.cs), cmul(p12, x2));
            y2 = cadd(cmul(p21, x1), cscale(x2, RP.cs));
            a[p1 + p2 * n] = y1;
            a[q1 + p2 * n] = y2;
          } else if (q2 < n && RQ.on) {   // P pair is (p1, pad): row p1 only
            cplx x1 = a[p1 + p2 * n], x2 = a[p1 + q2 * n];
            rot_row(RQ, &x1, &x2);
            a[p1 + p2 * n] = x1;
            a[p1 + q2 * n] = x2;
          }
          continue;
        }
        if (P == Qb) {
          if (RP.on) {
            const double ap = a[p1 + p1 * n].x, aq = a[q1 + q1 * n].x;
            a[p1 + p1 * n] = make_double2(ap - RP.t, 0.0);
            a[q1 + q1 * n] = make_double2(aq + RP.t, 0.0);
            a[p1 + q1 * n] = make_double2(0.0, 0.0);
            a[q1 + p1 * n] = make_double2(0.0, 0.0);
          }
          continue;
        }
        if (!RP.on && !RQ.on) continue;
        cplx x11 = a[p1 + p2 * n], x12 = a[p1 + q2 * n], x21 = a[q1 + p2 * n], x22 = a[q1 + q2 * n];
        rot_block(RP, RQ, &x11, &x12, &x21, &x22);
        a[p1 + p2 * n] = x11;
        a[p1 + q2 * n] = x12;
        a[q1 + p2 * n] = x21;
        a[q1 + q2 * n] = x22;
      }
      for (int idx = tid; idx < n * h; idx += nt) {
        const int Qb = idx / n, i = idx - Qb * n;
        int p2, q2;
        rr_pair(r, Qb, n2, &p2, &q2);
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
    const double di = a[i + i * n].x;
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = a[j + j * n].x;
      if (dj < di || (dj == di && j < i)) ++rk;
    }
    rank_[i] = rk;
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) w[rank_[i]] = a[i + i * n].x;
  for (int idx = tid; idx < n * n; idx += nt) {
    const int j = idx / n, i = idx - j * n;
    Q[i + (int64_t)rank_[j] * ldq] = v[i + j * n];
  }
  if (tid == 0) sweeps_out[0] = done ? sweeps : -1;
}

// One round for n > 64: A_out = G^H A_in G over 2x2 blocks; V <- V G in place.
// Threads [0, h*h) own the blocks, [h*h, h*h + n*h) own the V row pairs.
__global__ void k_jacobi_round(int n, int r, const cplx* __restrict__ Ai, cplx* __restrict__ Ao,
                               cplx* __restrict__ V) {
  const int n2 = n + (n & 1);
  const int h = n2 / 2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nblk = (int64_t)h * h;
  auto rot_of = [&](int pair, int* p, int* q) {
    rr_pair(r, pair, n2, p, q);
    if (*q >= n) return make_rot(0.0, 0.0, make_double2(0.0, 0.0));
    return make_rot(Ai[*p + (int64_t)*p * n].x, Ai[*q + (int64_t)*q * n].x, Ai[*p + (int64_t)*q * n]);
  };
  if (idx < nblk) {
    const int P = (int)(idx / h), Qb = (int)(idx - (int64_t)P * h);
    int p1, q1, p2, q2;
    const Rot RP = rot_of(P, &p1, &q1);
    const Rot RQ = rot_of(Qb, &p2, &q2);
    if (q1 >= n && q2 >= n) {
      Ao[p1 + (int64_t)p2 * n] = Ai[p1 + (int64_t)p2 * n];
      return;
    }
    if (q1 >= n) {   // row p1 only, columns (p2, q2)
      cplx x1 = Ai[p1 + (int64_t)p2 * n], x2 = Ai[p1 + (int64_t)q2 * n];
      rot_row(RQ, &x1, &x2);
      Ao[p1 + (int64_t)p2 * n] = x1;
      Ao[p1 + (int64_t)q2 * n] = x2;
      return;
    }
    if (q2 >= n) {   // column p2 only, rows (p1, q1)
      const cplx x1 = Ai[p1 + (int64_t)p2 * n], x2 = Ai[q1 + (int64_t)p2 * n];
      const cplx p12 = cscale(RP.ph, -RP.sn), p21 = cscale(cconj(RP.ph), RP.sn);
      Ao[p1 + (int64_t)p2 * n] = cadd(cscale(x1, RP.cs), cmul(p12, x2));
      Ao[q1 + (int64_t)p2 * n] = cadd(cmul(p21, x1), cscale(x2, RP.cs));
      return;
    }
    cplx x11 = Ai[p1 + (int64_t)p2 * n], x12 = Ai[p1 + (int64_t)q2 * n];
    cplx x21 = Ai[q1 + (int64_t)p2 * n], x22 = Ai[q1 + (int64_t)q2 * n];
    if (P == Qb) {
      if (RP.on) {
        x11 = make_double2(x11.x - RP.t, 0.0);
        x22 = make_double2(x22.x + RP.t, 0.0);
        x12 = make_double2(0.0, 0.0);
        x21 = make_double2(0.0, 0.0);
      }
    } else if (RP.on || RQ.on) {
      rot_block(RP, RQ, &x11, &x12, &x21, &x22);
    }
    Ao[p1 + (int64_t)p2 * n] = x11;
    Ao[p1 + (int64_t)q2 * n] = x12;
    Ao[q1 + (int64_t)p2 * n] = x21;
    Ao[q1 + (int64_t)q2 * n] = x22;
    return;
  }
  const int64_t vi = idx - nblk;
  if (vi >= (int64_t)n * h) return;
  const int Qb = (int)(vi / n), i = (int)(vi - (int64_t)Qb * n);
  int p2, q2;
  const Rot RQ = rot_of(Qb, &p2, &q2);
  if (q2 >= n || !RQ.on) return;
  cplx x1 = V[i + (int64_t)p2 * n], x2 = V[i + (int64_t)q2 * n];
  rot_row(RQ, &x1, &x2);
  V[i + (int64_t)p2 * n] = x1;
  V[i + (int64_t)q2 * n] = x2;
}

__global__ void __launch_bounds__(1024) k_offnorm(int n, const cplx* __restrict__ A, double* out) {
  __shared__ double r1[1024], r2[1024];
  double off = 0.0, tot = 0.0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int64_t j = idx / n, i = idx - j * n;
    const double m2 = cabs2(A[idx]);
    tot += m2;
    if (i != j) off += m2;
  }
  r1[threadIdx.x] = off;
  r2[threadIdx.x] = tot;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r1[0];
    out[1] = r2[0];
  }
}

__global__ void k_identity(int n, cplx* V) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  V[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

__global__ void k_eig_rank(int n, const cplx* __restrict__ A, int* __restrict__ rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = A[i + (int64_t)i * n].x;
  int rk = 0;
  for (int j = 0; j < n; ++j) {
    const double dj = A[j + (int64_t)j * n].x;
    if (dj < di || (dj == di && j < i)) ++rk;
  }
  rank[i] = rk;
}

__global__ void k_eig_scatter(int n, const cplx* __restrict__ A, const cplx* __restrict__ V,
                              const int* __restrict__ rank, double* __restrict__ w,
                              cplx* __restrict__ Q, int64_t ldq) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int j = (int)(idx / n), i = (int)(idx - (int64_t)j * n);
  const int rj = rank[j];
  Q[i + (int64_t)rj * ldq] = V[idx];
  if (i == 0) w[rj] = A[j + (int64_t)j * n].x;
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
                              const cplx* y, int64_t ldy, cplx* out, int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby_block, dim3(nblocks(npw * nb, 256)), dim3(256), 0, s, npw, nb, a, x,
                     ldx, b, y, ldy, out, ldo);
  return hipGetLastError();
}

hipError_t launch_residuals(int64_t npw, int64_t nb, const cplx* W, int64_t ldw, const cplx* Y,
                            int64_t ldy, const double* lam, double* resid, hipStream_t s) {
  hipLaunchKernelGGL(k_residuals, dim3((unsigned)nb), dim3(256), 0, s, npw, W, ldw, Y, ldy, lam,
                     resid);
  return hipGetLastError();
}

hipError_t launch_potrf_inv(int64_t n, cplx* a, int64_t lda, cplx* ainv, int64_t ldi, int* status,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_potrf_inv, dim3(1), dim3(kCholThreads), (size_t)n * sizeof(cplx), s, (int)n,
                     a, lda, ainv, ldi, status);
  return hipGetLastError();
}

size_t heev_work_bytes(int64_t n) {
  return (size_t)(3 * n * n) * sizeof(cplx) + (size_t)(n + 8) * sizeof(int) + 64;
}

// Opt the kernels with large dynamic LDS into `bytes` of LDS per workgroup
// (minus their static shared memory).
hipError_t heev_set_lds_limit(size_t bytes) {
  const void* fns[2] = {(const void*)k_jacobi_small, (const void*)k_potrf_inv};
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

hipError_t launch_heev(int64_t n, cplx* a, int64_t lda, double* w, cplx* q, int64_t ldq, void* work,
                       double* host_scratch, int* sweeps_done, hipStream_t s) {
  // layout: A0, A1, V (n*n cplx each) | n ints (ranks) + flag | 16-byte aligned 2 doubles
  int* dev_int = reinterpret_cast<int*>(static_cast<char*>(work) + (size_t)(3 * n * n) * sizeof(cplx));
  const size_t stat_off = (((size_t)(3 * n * n) * sizeof(cplx) + (size_t)(n + 8) * sizeof(int)) + 15) & ~(size_t)15;
  double* dstat = reinterpret_cast<double*>(static_cast<char*>(work) + stat_off);
  if (n <= kJacSmallMax) {
    const size_t lds = (size_t)(2 * n * n) * sizeof(cplx);
    hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(kJacThreads), lds, s, (int)n, (const cplx*)a,
                       lda, w, q, ldq, dev_int);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int hs = 0;
    e = hipMemcpyAsync(&hs, dev_int, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    *sweeps_done = hs;
    return e;
  }
  cplx* A0 = static_cast<cplx*>(work);
  cplx* A1 = A0 + n * n;
  cplx* V = A1 + n * n;
  hipError_t e = launch_copy_block(n, n, a, lda, A0, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_identity, dim3(nblocks(n * n, 256)), dim3(256), 0, s, (int)n, V);
  const int n2 = (int)(n + (n & 1));
  const int64_t h = n2 / 2;
  const int64_t threads = h * h + n * h;
  const double tl = std::max(1e-15, 2.2e-16 * (double)n);
  int sw = 0;
  bool conv = false;
  for (; sw <= kMaxSweeps; ++sw) {
    hipLaunchKernelGGL(k_offnorm, dim3(1), dim3(1024), 0, s, (int)n, (const cplx*)A0, dstat);
    e = hipMemcpyAsync(host_scratch, dstat, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (host_scratch[0] <= tl * tl * host_scratch[1]) {
      conv = true;
      break;
    }
    if (sw == kMaxSweeps) break;
    for (int r = 0; r < n2 - 1; ++r) {
      hipLaunchKernelGGL(k_jacobi_round, dim3(nblocks(threads, 256)), dim3(256), 0, s, (int)n, r,
                         (const cplx*)A0, A1, V);
      std::swap(A0, A1);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_eig_rank, dim3(nblocks(n, 256)), dim3(256), 0, s, (int)n, (const cplx*)A0,
                     dev_int);
  hipLaunchKernelGGL(k_eig_scatter, dim3(nblocks(n * n, 256)), dim3(256), 0, s, (int)n,
                     (const cplx*)A0, (const cplx*)V, (const int*)dev_int, w, q, ldq);
  *sweeps_done = conv ? sw : -1;
  return hipGetLastError();
}
