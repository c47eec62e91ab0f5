// Two more iterative eigensolvers of section 5, built on the library's H*psi
// and subspace kernels:
//
//  pw_lobpcg    section 5.1: the band-block LOBPCG (locally optimal block
//               preconditioned conjugate gradient) the paper measures beside
//               Chebyshev filtering, with its block count (nblock_lobpcg) and
//               line count (nline);
//  pw_rmm_diis  section 5.4: RMM-DIIS (residual minimisation, direct
//               inversion in the iterative subspace): band updates with no
//               orthogonalisation, then one full-band Cholesky
//               orthonormalisation and one subspace rotation per call.
//
// The paper names the solvers without their steps; these are the published
// algorithms (Knyazev's LOBPCG in blocks of bands, each kept orthogonal to
// the blocks below it; Kresse and Furthmuller's RMM-DIIS) with the
// Teter-Payne-Allan kinetic-energy preconditioner of plane-wave codes.  H is
// applied only to new directions: H X and H P ride every rotation, so the
// projections P^H X and P^H P are never formed again (the reduction of
// non-local work that section 5.2 reports for its stored projections).
#include "pw_handles.h"

#include <algorithm>
#include <cmath>

namespace {

__device__ __forceinline__ cplx zmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx zconj(cplx a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ cplx zadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx zsub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx zscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double zabs2(cplx a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ cplx zdiv(cplx a, cplx b) {
  const double d = zabs2(b);
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

constexpr int kRed = 256;        // threads of the per-band reduction workgroups (4 wavefronts)
constexpr int kMaxDots = 12;     // complex dot products per band in one k_band_dots launch
constexpr int kMaxDiis = 8;      // longest RMM-DIIS history (ndiis)
constexpr int kMaxPencil = kMaxDiis + 1;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup sums (kRed threads) of nv values per thread in a fixed order;
// every thread receives the totals.  part: 4 * nv doubles of LDS.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = wave_sum(v[k]);
    if (lane == 0) part[wave * NV + k] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = ((part[k] + part[NV + k]) + part[2 * NV + k]) + part[3 * NV + k];
  __syncthreads();
}

// Teter, Payne and Allan's preconditioner factor of x = T_g / E_kin:
// (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4).
__device__ __forceinline__ double teter(double x) {
  const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
  const double x2 = x * x;
  return num / (num + 16.0 * x2 * x2);
}

// ek[b] = sum_g T_g |x_gb|^2 / sum_g |x_gb|^2 (one workgroup per band).
__global__ void __launch_bounds__(kRed) k_band_kinetic(int64_t npw, const cplx* __restrict__ X,
                                                       int64_t ldx, const double* __restrict__ kin,
                                                       double* __restrict__ ek) {
  __shared__ double part[4 * 2];
  const cplx* x = X + (int64_t)blockIdx.x * ldx;
  double v[2] = {0.0, 0.0};
  for (int64_t g = threadIdx.x; g < npw; g += kRed) {
    const double a = zabs2(x[g]);
    v[0] += kin[g] * a;
    v[1] += a;
  }
  wg_sum<2>(v, part);
  if (threadIdx.x == 0) ek[blockIdx.x] = v[0] / v[1];
}

// W[g, b] = K(T_g / ek_b) (HX[g, b] - lam_b X[g, b]) (K = 1 when !precond).
__global__ void k_precond_resid(int64_t npw, const cplx* __restrict__ X, int64_t ldx,
                                const cplx* __restrict__ HX, int64_t ldhx,
                                const double* __restrict__ lam, const double* __restrict__ kin,
                                const double* __restrict__ ek, int precond, cplx* __restrict__ W,
                                int64_t ldw) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int b = blockIdx.y;
  const cplx r = zsub(HX[g + b * ldhx], zscale(X[g + b * ldx], lam[b]));
  W[g + b * ldw] = precond ? zscale(r, teter(kin[g] / ek[b])) : r;
}

// D[g, b] = K(T_g / ek_b) R[g, b]
__global__ void k_precond(int64_t npw, const cplx* __restrict__ R, int64_t ldr,
                          const double* __restrict__ kin, const double* __restrict__ ek,
                          cplx* __restrict__ D, int64_t ldd) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int b = blockIdx.y;
  D[g + b * ldd] = zscale(R[g + b * ldr], teter(kin[g] / ek[b]));
}

// Column b of B (and of HB and of the nc-row block CB, if given) divided by ||B_b||.
__global__ void __launch_bounds__(kRed) k_normalize_cols(int64_t npw, cplx* __restrict__ B,
                                                         int64_t ldb, cplx* __restrict__ HB,
                                                         int64_t ldhb, int64_t nc,
                                                         cplx* __restrict__ CB, int64_t ldcb) {
  __shared__ double part[4];
  cplx* x = B + (int64_t)blockIdx.x * ldb;
  double v[1] = {0.0};
  for (int64_t g = threadIdx.x; g < npw; g += kRed) v[0] += zabs2(x[g]);
  wg_sum<1>(v, part);
  const double s = 1.0 / sqrt(v[0]);
  for (int64_t g = threadIdx.x; g < npw; g += kRed) x[g] = zscale(x[g], s);
  if (HB) {
    cplx* hx = HB + (int64_t)blockIdx.x * ldhb;
    for (int64_t g = threadIdx.x; g < npw; g += kRed) hx[g] = zscale(hx[g], s);
  }
  if (CB) {
    cplx* cx = CB + (int64_t)blockIdx.x * ldcb;
    for (int64_t g = threadIdx.x; g < nc; g += kRed) cx[g] = zscale(cx[g], s);
  }
}

// Per band: e = Re<psi|H psi> / <psi|psi>, R = H psi - e psi, and
// bres = ||R|| / ||psi|| (bres may be null).  One workgroup per band.
__global__ void __launch_bounds__(kRed) k_rq_resid(int64_t npw, const cplx* __restrict__ P,
                                                   int64_t ldp, const cplx* __restrict__ HP,
                                                   int64_t ldhp, cplx* __restrict__ R, int64_t ldr,
                                                   double* __restrict__ bres) {
  __shared__ double part[4 * 2];
  const int b = blockIdx.x;
  const cplx* p = P + (int64_t)b * ldp;
  const cplx* hp = HP + (int64_t)b * ldhp;
  cplx* r = R + (int64_t)b * ldr;
  double v[2] = {0.0, 0.0};
  for (int64_t g = threadIdx.x; g < npw; g += kRed) {
    const cplx a = p[g], h = hp[g];
    v[0] += a.x * h.x + a.y * h.y;   // Re(conj(psi) H psi)
    v[1] += zabs2(a);
  }
  wg_sum<2>(v, part);
  const double e = v[0] / v[1], pp = v[1];
  double w[1] = {0.0};
  for (int64_t g = threadIdx.x; g < npw; g += kRed) {
    const cplx x = zsub(hp[g], zscale(p[g], e));
    r[g] = x;
    w[0] += zabs2(x);
  }
  wg_sum<1>(w, part);
  if (threadIdx.x == 0 && bres) bres[b] = sqrt(w[0]) / sqrt(pp);
}

// out[b * nu * nw + i * nw + j] = sum_g conj(U_i[g, b]) W_j[g, b]: the
// nu x nw inner products of band b (one workgroup per band; every block
// has leading dimension ld).  NU, NW: compile-time bounds of nu, nw.
struct DotArgs {
  const cplx* u[kMaxDots];
  const cplx* w[4];
  int nu, nw;
  int64_t ld;
};
template <int NU, int NW>
__global__ void __launch_bounds__(kRed) k_band_dots(int64_t npw, DotArgs a, cplx* __restrict__ out) {
  static_assert(NU * NW <= kMaxDots && NU <= kMaxDots && NW <= 4, "dot count");
  __shared__ double part[4 * 2 * NU * NW];
  const int b = blockIdx.x;
  const int64_t off = (int64_t)b * a.ld;
  double acc[2 * NU * NW];
#pragma unroll
  for (int k = 0; k < 2 * NU * NW; ++k) acc[k] = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += kRed) {
    cplx wv[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) wv[j] = j < a.nw ? a.w[j][off + g] : make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      if (i < a.nu) {
        const cplx u = a.u[i][off + g];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          acc[2 * (i * NW + j)] += u.x * wv[j].x + u.y * wv[j].y;
          acc[2 * (i * NW + j) + 1] += u.x * wv[j].y - u.y * wv[j].x;
        }
      }
    }
  }
  wg_sum<2 * NU * NW>(acc, part);
#pragma unroll
  for (int i = 0; i < NU; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j)
      if (threadIdx.x == 0 && i < a.nu && j < a.nw)
        out[(int64_t)b * a.nu * a.nw + i * a.nw + j] =
            make_double2(acc[2 * (i * NW + j)], acc[2 * (i * NW + j) + 1]);
}

// ---------------------------------------------------------------------------
// Small Hermitian problems, one thread per band (n <= kMaxPencil)
// ---------------------------------------------------------------------------
// Cyclic Jacobi on a (n x n, column-major, Hermitian): a -> diag(w), v the
// eigenvectors; w ascending with v's columns in the same order.
__device__ void small_heev(int n, cplx* a, cplx* v, double* w) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) v[i + j * n] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double m2 = zabs2(a[i + j * n]);
        tot += m2;
        if (i != j) off += m2;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cplx apq = a[p + q * n];
        const double g = sqrt(zabs2(apq));
        if (g == 0.0) continue;
        const cplx ph = zscale(apq, 1.0 / g);
        const double app = a[p + p * n].x, aqq = a[q + q * n].x;
        const double tau = (aqq - app) / (2.0 * g);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        // G on (p, q): [[c, s], [-s conj(ph), c conj(ph)]]; a <- G^H a G, v <- v G
        const cplx gpp = make_double2(c, 0.0), gpq = make_double2(s, 0.0);
        const cplx gqp = zscale(zconj(ph), -s), gqq = zscale(zconj(ph), c);
        for (int k = 0; k < n; ++k) {   // columns
          const cplx x = a[k + p * n], y = a[k + q * n];
          a[k + p * n] = zadd(zmul(x, gpp), zmul(y, gqp));
          a[k + q * n] = zadd(zmul(x, gpq), zmul(y, gqq));
          const cplx vx = v[k + p * n], vy = v[k + q * n];
          v[k + p * n] = zadd(zmul(vx, gpp), zmul(vy, gqp));
          v[k + q * n] = zadd(zmul(vx, gpq), zmul(vy, gqq));
        }
        for (int k = 0; k < n; ++k) {   // rows
          const cplx x = a[p + k * n], y = a[q + k * n];
          a[p + k * n] = zadd(zmul(zconj(gpp), x), zmul(zconj(gqp), y));
          a[q + k * n] = zadd(zmul(zconj(gpq), x), zmul(zconj(gqq), y));
        }
        a[p + q * n] = make_double2(0.0, 0.0);
        a[q + p * n] = make_double2(0.0, 0.0);
        a[p + p * n].y = 0.0;
        a[q + q * n].y = 0.0;
      }
  }
  for (int i = 0; i < n; ++i) w[i] = a[i + i * n].x;
  // ascending order (selection sort on values and columns)
  for (int i = 0; i < n - 1; ++i) {
    int k = i;
    for (int j = i + 1; j < n; ++j)
      if (w[j] < w[k]) k = j;
    if (k != i) {
      const double t = w[i];
      w[i] = w[k];
      w[k] = t;
      for (int r = 0; r < n; ++r) {
        const cplx x = v[r + i * n];
        v[r + i * n] = v[r + k * n];
        v[r + k * n] = x;
      }
    }
  }
}

// Lowest eigenvector of the pencil A x = e B x (n x n, column-major): the
// Hermitian parts of both; B = U diag(s) U^H with the directions s <=
// rtol max(s) dropped; the reduced standard problem C = Uk^H A Uk, Uk =
// U_kept diag(s_kept)^-1/2; x = Uk z for z the lowest eigenvector of C,
// rotated so that sum_i x_i is real and non-negative.
__device__ void lowest_pencil(int n, const cplx* A, const cplx* B, double rtol, cplx* x) {
  cplx bh[kMaxPencil * kMaxPencil], u[kMaxPencil * kMaxPencil], uk[kMaxPencil * kMaxPencil];
  cplx ch[kMaxPencil * kMaxPencil], z[kMaxPencil * kMaxPencil];
  double s[kMaxPencil], th[kMaxPencil];
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      bh[i + j * n] = zscale(zadd(B[i + j * n], zconj(B[j + i * n])), 0.5);
  small_heev(n, bh, u, s);
  int nk = 0;
  for (int j = 0; j < n; ++j) {
    if (!(s[j] > rtol * s[n - 1])) continue;
    const double f = 1.0 / sqrt(s[j]);
    for (int i = 0; i < n; ++i) uk[i + nk * n] = zscale(u[i + j * n], f);
    ++nk;
  }
  // C = Uk^H Ah Uk, Ah = (A + A^H) / 2
  for (int q = 0; q < nk; ++q)
    for (int p = 0; p < nk; ++p) {
      cplx acc = make_double2(0.0, 0.0);
      for (int j = 0; j < n; ++j) {
        cplx t = make_double2(0.0, 0.0);
        for (int i = 0; i < n; ++i) {
          const cplx ah = zscale(zadd(A[i + j * n], zconj(A[j + i * n])), 0.5);
          t = zadd(t, zmul(zconj(uk[i + p * n]), ah));
        }
        acc = zadd(acc, zmul(t, uk[j + q * n]));
      }
      ch[p + q * nk] = acc;
    }
  for (int q = 0; q < nk; ++q)
    for (int p = 0; p < nk; ++p)
      if (p < q) {
        const cplx m = zscale(zadd(ch[p + q * nk], zconj(ch[q + p * nk])), 0.5);
        ch[p + q * nk] = m;
        ch[q + p * nk] = zconj(m);
      }
  for (int p = 0; p < nk; ++p) ch[p + p * nk].y = 0.0;
  small_heev(nk, ch, z, th);
  cplx tsum = make_double2(0.0, 0.0);
  for (int i = 0; i < n; ++i) {
    cplx acc = make_double2(0.0, 0.0);
    for (int p = 0; p < nk; ++p) acc = zadd(acc, zmul(uk[i + p * n], z[p]));
    x[i] = acc;
    tsum = zadd(tsum, acc);
  }
  const double ta = sqrt(zabs2(tsum));
  if (ta > 0.0) {
    const cplx ph = zscale(zconj(tsum), 1.0 / ta);
    for (int i = 0; i < n; ++i) x[i] = zmul(x[i], ph);
  }
}

// RMM-DIIS first step: per band the line-minimisation step lam of psi + lam
// d over span{psi, d}, from dots = <[psi, d] | [psi, d, H psi, H d]>
// (8 per band, as k_band_dots lays them out); lam = 0 when the overlap
// matrix of {psi, d} has an eigenvalue at or below rtol times its largest.
__global__ void k_line_step(int nb, const cplx* __restrict__ dots, double rtol,
                            cplx* __restrict__ lam) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const cplx* d = dots + (int64_t)b * 8;
  // column-major 2 x 2: B = V^H V, A = V^H H V
  const cplx B[4] = {d[0], d[4], d[1], d[5]};
  const cplx A[4] = {d[2], d[6], d[3], d[7]};
  cplx bh[4], u[4];
  double s[2];
  for (int j = 0; j < 2; ++j)
    for (int i = 0; i < 2; ++i) bh[i + 2 * j] = zscale(zadd(B[i + 2 * j], zconj(B[j + 2 * i])), 0.5);
  small_heev(2, bh, u, s);
  if (!(s[0] > rtol * s[1])) {
    lam[b] = make_double2(0.0, 0.0);
    return;
  }
  cplx c[2];
  lowest_pencil(2, A, B, rtol, c);
  lam[b] = zdiv(c[1], c[0]);
}

// Overlaps of the history: the new row / column M of the (ndiis+1)^2 matrix
// of band b from dots[b * (M + 1) + i] = <V^i_b | V^M_b>.
__global__ void k_hist_store(int nb, int M, int dim, const cplx* __restrict__ dots,
                             cplx* __restrict__ mats) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  cplx* m = mats + (int64_t)b * dim * dim;
  for (int i = 0; i <= M; ++i) {
    const cplx v = dots[(int64_t)b * (M + 1) + i];
    m[i + M * dim] = v;
    m[M + i * dim] = zconj(v);
  }
}

// DIIS coefficients of band b over history 0..M: the lowest vector of the
// pencil <R^i|R^j> a = e <psi^i|psi^j> a.
__global__ void k_diis_pencil(int nb, int M, int dim, const cplx* __restrict__ Ar,
                              const cplx* __restrict__ Bp, double rtol, cplx* __restrict__ coef) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int n = M + 1;
  cplx A[kMaxPencil * kMaxPencil], B[kMaxPencil * kMaxPencil], x[kMaxPencil];
  const cplx* ar = Ar + (int64_t)b * dim * dim;
  const cplx* bp = Bp + (int64_t)b * dim * dim;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      A[i + j * n] = ar[i + j * dim];
      B[i + j * n] = bp[i + j * dim];
    }
  lowest_pencil(n, A, B, rtol, x);
  for (int i = 0; i < n; ++i) coef[(int64_t)b * dim + i] = x[i];
}

// out[g, b] = sum_i a_i psi^i + lam_b K(T_g / ek_b) sum_i a_i R^i, i <= M.
__global__ void k_diis_update(int64_t npw, int M, int dim, const cplx* __restrict__ psi,
                              const cplx* __restrict__ R, int64_t hstride, int64_t ld,
                              const cplx* __restrict__ coef, const cplx* __restrict__ lam,
                              const double* __restrict__ kin, const double* __restrict__ ek,
                              cplx* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int b = blockIdx.y;
  const int64_t o = g + (int64_t)b * ld;
  cplx ps = make_double2(0.0, 0.0), rs = make_double2(0.0, 0.0);
  for (int i = 0; i <= M; ++i) {
    const cplx a = coef[(int64_t)b * dim + i];
    ps = zadd(ps, zmul(a, psi[i * hstride + o]));
    rs = zadd(rs, zmul(a, R[i * hstride + o]));
  }
  out[o] = zadd(ps, zmul(lam[b], zscale(rs, teter(kin[g] / ek[b]))));
}

// out[g, b] = X[g, b] + lam_b D[g, b] (out may alias X)
__global__ void k_axpy_band(int64_t npw, const cplx* X, int64_t ldx, const cplx* __restrict__ D,
                            int64_t ldd, const cplx* __restrict__ lam, cplx* out, int64_t ldo) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int b = blockIdx.y;
  out[g + b * ldo] = zadd(X[g + b * ldx], zmul(lam[b], D[g + b * ldd]));
}

inline dim3 band_grid(int64_t npw, int64_t nb) {
  return dim3((unsigned)((npw + 255) / 256), (unsigned)nb);
}

}  // namespace

using namespace pwi;

namespace {

// B <- B - X (X^H B) and, if HB, HB <- HB - HX (X^H B): X has kx
// orthonormal columns (ld ldx), B and HB m columns with ld npw.  With CB and
// CX (projections of B and X, nproj rows): CB <- CB - CX (X^H B).
pw_status remove_span(pw_ham* h, int64_t m, cplx* B, cplx* HB, int64_t kx, const cplx* X,
                      int64_t ldx, const cplx* HX, int64_t ldhx, cplx* cbuf, cplx* work,
                      cplx* CB = nullptr, const cplx* CX = nullptr) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  const int64_t npw = h->npw;
  if (kx <= 0 || m <= 0) return PW_OK;
  HIPCHK(c, launch_gemm_cn(kx, m, npw, 1.0, X, ldx, B, npw, cbuf, kx, nullptr, work, s));
  HIPCHK(c, launch_gemm_nn(npw, m, kx, -1.0, X, ldx, cbuf, kx, 1.0, B, npw, s, h->nn_tile));
  if (HB) HIPCHK(c, launch_gemm_nn(npw, m, kx, -1.0, HX, ldhx, cbuf, kx, 1.0, HB, npw, s, h->nn_tile));
  if (CB && CX && h->nproj > 0)
    HIPCHK(c, launch_gemm_nn(h->nproj, m, kx, -1.0, CX, h->nproj, cbuf, kx, 1.0, CB, h->nproj, s, 0));
  return PW_OK;
}

hipError_t normalize_cols(int64_t npw, int64_t m, cplx* B, cplx* HB, hipStream_t s,
                          int64_t nc = 0, cplx* CB = nullptr) {
  hipLaunchKernelGGL(k_normalize_cols, dim3((unsigned)m), dim3(kRed), 0, s, npw, B, npw, HB, npw,
                     nc, CB, nc);
  return hipGetLastError();
}

pw_status lobpcg_workspace(pw_ham* h, int64_t nb, int64_t m) {
  LobpcgWork& w = h->lob;
  if (w.m >= m && w.nb >= nb) return PW_OK;
  for (void* p : w.mem) dfree(h, p);
  w = LobpcgWork{};
  const int64_t npw = h->npw, k = 3 * m;
  pw_status st;
  for (int i = 0; i < 2; ++i) {
    if ((st = dalloc(h, &w.v[i], (size_t)(npw * k))) != PW_OK) return st;
    if ((st = dalloc(h, &w.hv[i], (size_t)(npw * k))) != PW_OK) return st;
    w.mem.push_back(w.v[i]);
    w.mem.push_back(w.hv[i]);
  }
  size_t wk = 1;
  for (int64_t kx = 1; kx <= nb; ++kx) wk = std::max(wk, gemm_cn_work_elems(kx, m, npw));
  wk = std::max(wk, gemm_cn_work_elems(k, k, npw));
  wk = std::max(wk, gemm_cn_work_elems(2 * m, 2 * m, npw));
  char* hw = nullptr;
  if ((st = dalloc(h, &w.s, (size_t)(k * k))) != PW_OK ||
      (st = dalloc(h, &w.z, (size_t)(k * k))) != PW_OK ||
      (st = dalloc(h, &w.c, (size_t)(std::max(nb, k) * m))) != PW_OK ||
      (st = dalloc(h, &w.work, wk)) != PW_OK || (st = dalloc(h, &w.theta, (size_t)k)) != PW_OK ||
      (st = dalloc(h, &w.lam, (size_t)m)) != PW_OK || (st = dalloc(h, &w.ek, (size_t)m)) != PW_OK ||
      (st = dalloc(h, &hw, heev_work_bytes(k))) != PW_OK)
    return st;
  w.heev = hw;
  for (void* p : {(void*)w.s, (void*)w.z, (void*)w.c, (void*)w.work, (void*)w.theta, (void*)w.lam,
                  (void*)w.ek, (void*)hw})
    w.mem.push_back(p);
  if (h->nproj > 0)
    for (int i = 0; i < 2; ++i) {
      if ((st = dalloc(h, &w.cv[i], (size_t)(h->nproj * k))) != PW_OK) return st;
      w.mem.push_back(w.cv[i]);
    }
  w.m = m;
  w.nb = nb;
  return PW_OK;
}

pw_status rmm_workspace(pw_ham* h, int64_t nb, int ndiis) {
  RmmWork& w = h->rmm;
  if (w.nb >= nb && w.ndiis >= ndiis) return PW_OK;
  for (void* p : w.mem) dfree(h, p);
  w = RmmWork{};
  const int64_t npw = h->npw, blk = npw * nb;
  const int dim = ndiis + 1;
  pw_status st;
  if ((st = dalloc(h, &w.psi, (size_t)(dim * blk))) != PW_OK ||
      (st = dalloc(h, &w.r, (size_t)(dim * blk))) != PW_OK ||
      (st = dalloc(h, &w.hcur, (size_t)blk)) != PW_OK || (st = dalloc(h, &w.d, (size_t)blk)) != PW_OK ||
      (st = dalloc(h, &w.hd, (size_t)blk)) != PW_OK ||
      (st = dalloc(h, &w.amat, (size_t)(nb * dim * dim))) != PW_OK ||
      (st = dalloc(h, &w.bmat, (size_t)(nb * dim * dim))) != PW_OK ||
      (st = dalloc(h, &w.coef, (size_t)(nb * dim))) != PW_OK ||
      (st = dalloc(h, &w.dots, (size_t)(nb * kMaxDots))) != PW_OK ||
      (st = dalloc(h, &w.lam, (size_t)nb)) != PW_OK || (st = dalloc(h, &w.ek, (size_t)nb)) != PW_OK)
    return st;
  for (void* p : {(void*)w.psi, (void*)w.r, (void*)w.hcur, (void*)w.d, (void*)w.hd, (void*)w.amat,
                  (void*)w.bmat, (void*)w.coef, (void*)w.dots, (void*)w.lam, (void*)w.ek})
    w.mem.push_back(p);
  if (h->nproj > 0) {
    if ((st = dalloc(h, &w.c0, (size_t)(h->nproj * nb))) != PW_OK ||
        (st = dalloc(h, &w.cd, (size_t)(h->nproj * nb))) != PW_OK)
      return st;
    w.mem.push_back(w.c0);
    w.mem.push_back(w.cd);
  }
  w.nb = nb;
  w.ndiis = ndiis;
  return PW_OK;
}

hipError_t band_dots(int64_t npw, int64_t nb, const std::vector<const cplx*>& u,
                     const std::vector<const cplx*>& wv, int64_t ld, cplx* out, hipStream_t s) {
  DotArgs a{};
  a.nu = (int)u.size();
  a.nw = (int)wv.size();
  if (a.nu > kMaxDots || a.nw > 4 || a.nu * a.nw > kMaxDots) return hipErrorInvalidValue;
  for (int i = 0; i < a.nu; ++i) a.u[i] = u[i];
  for (int j = 0; j < a.nw; ++j) a.w[j] = wv[j];
  a.ld = ld;
  if (a.nw == 1)
    hipLaunchKernelGGL((k_band_dots<kMaxDots, 1>), dim3((unsigned)nb), dim3(kRed), 0, s, npw, a, out);
  else if (a.nu <= 2)
    hipLaunchKernelGGL((k_band_dots<2, 4>), dim3((unsigned)nb), dim3(kRed), 0, s, npw, a, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

extern "C" {

pw_status pw_lobpcg(pw_ham* h, int64_t nb, int32_t nblock, int32_t nline, void* yv, int64_t ld,
                    void* hyv, int64_t ldhy, double* eig, double* resid, double* hist) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_status st;
  if ((st = check_hot(h, PW_FP64, nb)) != PW_OK) return st;
  if ((st = check_block(h, yv, ld, "y")) != PW_OK) return st;
  if ((st = check_block(h, hyv, ldhy, "hy")) != PW_OK) return st;
  if (!eig) return fail(h->ctx, PW_ERR_INVALID_ARG, "eig_dev is NULL");
  if (nblock < 1 || nblock > nb)
    return fail(h->ctx, PW_ERR_INVALID_ARG, "nblock must be in [1, nb]");
  if (nline < 1 || nline > 1000) return fail(h->ctx, PW_ERR_INVALID_ARG, "nline must be in [1, 1000]");
  if (ranges_overlap(yv, ld, hyv, ldhy, h->npw, nb))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "y and hy overlap");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const int64_t npw = h->npw;
  const int64_t q = nb / nblock, rem = nb % nblock;
  const int64_t mmax = q + (rem ? 1 : 0);
  if ((st = lobpcg_workspace(h, nb, mmax)) != PW_OK) return st;
  LobpcgWork& w = h->lob;
  cplx* y = static_cast<cplx*>(yv);
  cplx* hy = static_cast<cplx*>(hyv);
  const int64_t np = h->nproj;
  h->cprj_nb = 0;
  // X <- the orthonormalised start block
  if ((st = ortho_block(h, nb, y, ld, nullptr, 0, kOpLobpcg)) != PW_OK) return st;
  int64_t lo = 0;
  for (int j = 0; j < nblock; ++j) {
    const int64_t m = q + (j < rem ? 1 : 0);
    cplx* V = w.v[0];
    cplx* HV = w.hv[0];
    cplx* V2 = w.v[1];
    cplx* HV2 = w.hv[1];
    // projections P^H [X, W, P] (null without projectors): formed by the H
    // applications, then carried through every later step of the block
    cplx* CV = w.cv[0];
    cplx* CV2 = w.cv[1];
    // X_j: orthogonal to the (updated) blocks below, orthonormal, Rayleigh-Ritz
    {
      StageScope sc(c, PW_STAGE_MISC);
      HIPCHK(c, launch_copy_block(npw, m, y + lo * ld, ld, V, npw, s));
    }
    if (lo > 0) {
      StageScope sc(c, PW_STAGE_ROTATE);
      if ((st = remove_span(h, m, V, nullptr, lo, y, ld, nullptr, 0, w.c, w.work)) != PW_OK) return st;
    }
    if ((st = ortho_block(h, m, V, npw, nullptr, 0, kOpLobpcg)) != PW_OK) return st;
    if ((st = ham_apply(h, m, V, npw, HV, npw, 1.0, 0.0, 0.0, nullptr, 0, nullptr, CV)) != PW_OK)
      return st;
    if ((st = subspace_rr(h, m, V, npw, HV, npw, w.lam, nullptr, kOpLobpcg, CV)) != PW_OK) return st;
    if (hist) HIPCHK(c, launch_scale_copy(m, w.lam, 1.0, hist + lo, s));
    bool have_p = false;
    for (int line = 0; line < nline; ++line) {
      cplx* X = V;
      cplx* HX = HV;
      cplx* W = V + m * npw;
      cplx* HW = HV + m * npw;
      cplx* P = V + 2 * m * npw;
      cplx* HP = HV + 2 * m * npw;
      cplx* CX = CV;
      cplx* CW = CV ? CV + m * np : nullptr;
      cplx* CP = CV ? CV + 2 * m * np : nullptr;
      {
        StageScope sc(c, PW_STAGE_MISC);
        hipLaunchKernelGGL(k_band_kinetic, dim3((unsigned)m), dim3(kRed), 0, s, npw, (const cplx*)X,
                           npw, (const double*)h->kin, w.ek);
        hipLaunchKernelGGL(k_precond_resid, band_grid(npw, m), dim3(256), 0, s, npw, (const cplx*)X,
                           npw, (const cplx*)HX, npw, (const double*)w.lam, (const double*)h->kin,
                           (const double*)w.ek, 1, W, npw);
        HIPCHK(c, hipGetLastError());
      }
      {
        StageScope sc(c, PW_STAGE_ROTATE);
        if (lo > 0 &&
            (st = remove_span(h, m, W, nullptr, lo, y, ld, nullptr, 0, w.c, w.work)) != PW_OK)
          return st;
        if ((st = remove_span(h, m, W, nullptr, m, X, npw, nullptr, 0, w.c, w.work)) != PW_OK)
          return st;
        HIPCHK(c, normalize_cols(npw, m, W, nullptr, s));
      }
      if ((st = ortho_block(h, m, W, npw, nullptr, 0, kOpLobpcg)) != PW_OK) return st;
      if ((st = ham_apply(h, m, W, npw, HW, npw, 1.0, 0.0, 0.0, nullptr, 0, nullptr, CW)) != PW_OK)
        return st;
      if (have_p) {
        {
          StageScope sc(c, PW_STAGE_ROTATE);
          if ((st = remove_span(h, m, P, HP, m, X, npw, HX, npw, w.c, w.work, CP, CX)) != PW_OK)
            return st;
          if ((st = remove_span(h, m, P, HP, m, W, npw, HW, npw, w.c, w.work, CP, CW)) != PW_OK)
            return st;
          HIPCHK(c, normalize_cols(npw, m, P, HP, s, np, CP));
        }
        if ((st = ortho_block(h, m, P, npw, HP, npw, kOpLobpcg, PW_FP64, CP)) != PW_OK) return st;
      }
      const int64_t k = have_p ? 3 * m : 2 * m;
      {
        StageScope sc(c, PW_STAGE_GRAM);
        HIPCHK(c, launch_gemm_cn(k, k, npw, 1.0, V, npw, HV, npw, w.s, k, nullptr, w.work, s, 0.0,
                                 nullptr, 2048, 1));
        HIPCHK(c, launch_hermitize(k, w.s, k, s));
      }
      {
        StageScope sc(c, PW_STAGE_EIGH);
        HIPCHK(c, launch_heev_async(k, w.s, k, w.theta, w.z, k, w.heev, sweeps_slot(c),
                                    c->max_sweeps, s));
        HIPCHK(c, launch_status_record(nullptr, sweeps_slot(c), kOpLobpcg, c->rec_dev, s));
      }
      {
        // X' = V Z[:, :m], P' = V[:, m:] Z[m:, :m]; H X', H P' alike
        StageScope sc(c, PW_STAGE_ROTATE);
        HIPCHK(c, launch_gemm_nn(npw, m, k, 1.0, V, npw, w.z, k, 0.0, V2, npw, s, h->nn_tile));
        HIPCHK(c, launch_gemm_nn(npw, m, k, 1.0, HV, npw, w.z, k, 0.0, HV2, npw, s, h->nn_tile));
        HIPCHK(c, launch_gemm_nn(npw, m, k - m, 1.0, V + m * npw, npw, w.z + m, k, 0.0,
                                 V2 + 2 * m * npw, npw, s, h->nn_tile));
        HIPCHK(c, launch_gemm_nn(npw, m, k - m, 1.0, HV + m * npw, npw, w.z + m, k, 0.0,
                                 HV2 + 2 * m * npw, npw, s, h->nn_tile));
        if (CV) {   // the same rotations of the projections, nproj rows
          HIPCHK(c, launch_gemm_nn(np, m, k, 1.0, CV, np, w.z, k, 0.0, CV2, np, s, 0));
          HIPCHK(c, launch_gemm_nn(np, m, k - m, 1.0, CV + m * np, np, w.z + m, k, 0.0,
                                   CV2 + 2 * m * np, np, s, 0));
        }
        HIPCHK(c, launch_scale_copy(m, w.theta, 1.0, w.lam, s));
      }
      std::swap(V, V2);
      std::swap(HV, HV2);
      std::swap(CV, CV2);
      have_p = true;
      if (hist) HIPCHK(c, launch_scale_copy(m, w.lam, 1.0, hist + (int64_t)(line + 1) * nb + lo, s));
    }
    {
      StageScope sc(c, PW_STAGE_MISC);
      HIPCHK(c, launch_copy_block(npw, m, V, npw, y + lo * ld, ld, s));
      HIPCHK(c, launch_copy_block(npw, m, HV, npw, hy + lo * ldhy, ldhy, s));
      if (CV) HIPCHK(c, launch_copy_block(np, m, CV, np, h->cprj_y + lo * np, np, s));
    }
    lo += m;
  }
  // one Rayleigh-Ritz over all bands with the carried H X (and P^H X)
  if ((st = subspace_rr(h, nb, y, ld, hy, ldhy, eig, resid, kOpLobpcg, np > 0 ? h->cprj_y : nullptr)) !=
      PW_OK)
    return st;
  h->cprj_nb = nb;
  return PW_OK;
}

pw_status pw_rmm_diis(pw_ham* h, int64_t nb, int32_t ndiis, void* yv, int64_t ld, void* hyv,
                      int64_t ldhy, int32_t hy_valid, double* eig, double* resid,
                      double* band_resid) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_status st;
  if ((st = check_hot(h, PW_FP64, nb)) != PW_OK) return st;
  if ((st = check_block(h, yv, ld, "y")) != PW_OK) return st;
  if ((st = check_block(h, hyv, ldhy, "hy")) != PW_OK) return st;
  if (!eig) return fail(h->ctx, PW_ERR_INVALID_ARG, "eig_dev is NULL");
  if (ndiis < 1 || ndiis > kMaxDiis)
    return fail(h->ctx, PW_ERR_INVALID_ARG, "ndiis must be in [1, " + std::to_string(kMaxDiis) + "]");
  if (hy_valid != 0 && hy_valid != 1) return fail(h->ctx, PW_ERR_INVALID_ARG, "hy_valid must be 0 or 1");
  if (ranges_overlap(yv, ld, hyv, ldhy, h->npw, nb))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "y and hy overlap");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  if ((st = rmm_workspace(h, nb, ndiis)) != PW_OK) return st;
  RmmWork& w = h->rmm;
  const int64_t npw = h->npw, blk = npw * nb;
  const int dim = w.ndiis + 1;
  const double rtol = 1e-12;
  cplx* y = static_cast<cplx*>(yv);
  cplx* hy = static_cast<cplx*>(hyv);
  auto P = [&](int i) { return w.psi + i * blk; };
  auto R = [&](int i) { return w.r + i * blk; };
  auto bres = [&](int i) { return band_resid ? band_resid + (int64_t)i * nb : nullptr; };
  const dim3 grid = band_grid(npw, nb);
  const unsigned nbg = (unsigned)((nb + 63) / 64);
  // history rows of the overlap matrices: <psi^i|psi^M> and <R^i|R^M>
  auto store_row = [&](int M) -> pw_status {
    std::vector<const cplx*> up, ur;
    for (int i = 0; i <= M; ++i) {
      up.push_back(P(i));
      ur.push_back(R(i));
    }
    HIPCHK(c, band_dots(npw, nb, up, {P(M)}, npw, w.dots, s));
    hipLaunchKernelGGL(k_hist_store, dim3(nbg), dim3(64), 0, s, (int)nb, M, dim,
                       (const cplx*)w.dots, w.bmat);
    HIPCHK(c, band_dots(npw, nb, ur, {R(M)}, npw, w.dots, s));
    hipLaunchKernelGGL(k_hist_store, dim3(nbg), dim3(64), 0, s, (int)nb, M, dim,
                       (const cplx*)w.dots, w.amat);
    HIPCHK(c, hipGetLastError());
    return PW_OK;
  };
  {
    StageScope sc(c, PW_STAGE_MISC);
    HIPCHK(c, launch_copy_block(npw, nb, y, ld, P(0), npw, s));
    if (hy_valid) HIPCHK(c, launch_copy_block(npw, nb, hy, ldhy, w.hcur, npw, s));
  }
  const int64_t np = h->nproj;
  h->cprj_nb = 0;
  // projections of psi^0 (needed only when the pass ends on the line step)
  if (!hy_valid &&
      (st = ham_apply(h, nb, P(0), npw, w.hcur, npw, 1.0, 0.0, 0.0, nullptr, 0, nullptr, w.c0)) != PW_OK)
    return st;
  if (hy_valid && ndiis == 1 && np > 0) {
    StageScope sc(c, PW_STAGE_PROJ);
    HIPCHK(c, launch_gemm_cn(np, nb, npw, 1.0, h->proj, npw, P(0), npw, w.c0, np, nullptr,
                             h->gemm_work, s, 0.0, nullptr, h->gemm_target));
  }
  {
    StageScope sc(c, PW_STAGE_MISC);
    hipLaunchKernelGGL(k_band_kinetic, dim3((unsigned)nb), dim3(kRed), 0, s, npw,
                       (const cplx*)P(0), npw, (const double*)h->kin, w.ek);
    hipLaunchKernelGGL(k_rq_resid, dim3((unsigned)nb), dim3(kRed), 0, s, npw, (const cplx*)P(0), npw,
                       (const cplx*)w.hcur, npw, R(0), npw, bres(0));
    hipLaunchKernelGGL(k_precond, grid, dim3(256), 0, s, npw, (const cplx*)R(0), npw,
                       (const double*)h->kin, (const double*)w.ek, w.d, npw);
    HIPCHK(c, hipGetLastError());
    if ((st = store_row(0)) != PW_OK) return st;
  }
  if ((st = ham_apply(h, nb, w.d, npw, w.hd, npw, 1.0, 0.0, 0.0, nullptr, 0, nullptr, w.cd)) != PW_OK)
    return st;
  {
    StageScope sc(c, PW_STAGE_MISC);
    HIPCHK(c, band_dots(npw, nb, {P(0), w.d}, {P(0), w.d, w.hcur, w.hd}, npw, w.dots, s));
    hipLaunchKernelGGL(k_line_step, dim3(nbg), dim3(64), 0, s, (int)nb, (const cplx*)w.dots, rtol,
                       w.lam);
    hipLaunchKernelGGL(k_axpy_band, grid, dim3(256), 0, s, npw, (const cplx*)P(0), npw,
                       (const cplx*)w.d, npw, (const cplx*)w.lam, P(1), npw);
    hipLaunchKernelGGL(k_axpy_band, grid, dim3(256), 0, s, npw, (const cplx*)w.hcur, npw,
                       (const cplx*)w.hd, npw, (const cplx*)w.lam, w.hcur, npw);
    hipLaunchKernelGGL(k_rq_resid, dim3((unsigned)nb), dim3(kRed), 0, s, npw, (const cplx*)P(1), npw,
                       (const cplx*)w.hcur, npw, R(1), npw, bres(1));
    if (ndiis == 1 && np > 0)   // P^H psi^1 = P^H psi^0 + lam P^H d
      hipLaunchKernelGGL(k_axpy_band, band_grid(np, nb), dim3(256), 0, s, np, (const cplx*)w.c0, np,
                         (const cplx*)w.cd, np, (const cplx*)w.lam, h->cprj_y, np);
    HIPCHK(c, hipGetLastError());
    if (ndiis > 1 && (st = store_row(1)) != PW_OK) return st;
  }
  for (int M = 1; M < ndiis; ++M) {
    {
      StageScope sc(c, PW_STAGE_MISC);
      hipLaunchKernelGGL(k_diis_pencil, dim3(nbg), dim3(64), 0, s, (int)nb, M, dim,
                         (const cplx*)w.amat, (const cplx*)w.bmat, rtol, w.coef);
      hipLaunchKernelGGL(k_diis_update, grid, dim3(256), 0, s, npw, M, dim, (const cplx*)w.psi,
                         (const cplx*)w.r, blk, npw, (const cplx*)w.coef, (const cplx*)w.lam,
                         (const double*)h->kin, (const double*)w.ek, P(M + 1));
      HIPCHK(c, hipGetLastError());
    }
    if ((st = ham_apply(h, nb, P(M + 1), npw, w.hcur, npw, 1.0, 0.0, 0.0, nullptr, 0, nullptr,
                        M + 1 == ndiis && np > 0 ? h->cprj_y : nullptr)) != PW_OK)
      return st;
    {
      StageScope sc(c, PW_STAGE_MISC);
      hipLaunchKernelGGL(k_rq_resid, dim3((unsigned)nb), dim3(kRed), 0, s, npw,
                         (const cplx*)P(M + 1), npw, (const cplx*)w.hcur, npw, R(M + 1), npw,
                         bres(M + 1));
      HIPCHK(c, hipGetLastError());
      if (M + 1 < ndiis && (st = store_row(M + 1)) != PW_OK) return st;
    }
  }
  {
    StageScope sc(c, PW_STAGE_MISC);
    HIPCHK(c, launch_copy_block(npw, nb, P(ndiis), npw, y, ld, s));
    HIPCHK(c, launch_copy_block(npw, nb, w.hcur, npw, hy, ldhy, s));
  }
  cplx* cp = np > 0 ? h->cprj_y : nullptr;
  if ((st = ortho_block(h, nb, y, ld, hy, ldhy, kOpRmmDiis, PW_FP64, cp)) != PW_OK) return st;
  if ((st = subspace_rr(h, nb, y, ld, hy, ldhy, eig, resid, kOpRmmDiis, cp)) != PW_OK) return st;
  h->cprj_nb = nb;
  return PW_OK;
}

}  // extern "C"
