// Pruned, batched 3D FFT route of the local potential (section 5.1: many
// transforms of a wavefunction block at once) for gfx950.
//
// The box is never materialised.  With columns = distinct (m1, m2) of the
// sphere points (lines along N3) and the extent = distinct m1:
//   col_inv  : per (band, tile of columns): scatter the sphere coefficients of
//              each column into LDS, backward transform along N3, write
//              T[b][j3][c] (one contiguous run of columns per plane).
//   plane    : per (band, plane j3): place the plane's column values in an
//              LDS array E[e][m2] (xr x N2), backward along N2, then row by
//              row (j2): backward along N1, multiply by V/N_box, forward
//              along N1, keep the extent outputs; forward along N2; write
//              back the column outputs.
//   col_fwd  : per (band, tile of columns): forward along N3, gather to the
//              sphere, add the kinetic term and the filter's recurrence
//              epilogue.
// HBM traffic per band: 2 npw + 4 ncols*N3 complex elements (plus V, which
// stays in the last-level cache across bands).
//
// Every 1D transform is a sequence of in-place Stockham radix passes in LDS
// (radices 2, 3, 4, 5, 8), each pass a register-staged read / barrier /
// write so that no second buffer is needed.
#include "pw_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
// (S i) z for S = +1 / -1
template <int S>
__device__ __forceinline__ cplx mul_si(cplx z) {
  return S > 0 ? make_double2(-z.y, z.x) : make_double2(z.y, -z.x);
}

// Small DFTs y_k = sum_n x_n exp(S 2 pi i n k / R), in registers.
template <int S>
__device__ __forceinline__ void dft2(cplx* v) {
  cplx a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <int S>
__device__ __forceinline__ void dft3(cplx* v) {
  const double h = 0.86602540378443864676;  // sin(2 pi / 3)
  cplx s = cadd(v[1], v[2]);
  cplx d = csub(v[1], v[2]);
  cplx t = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
  cplx r = mul_si<S>(cscale(d, h));
  v[0] = cadd(v[0], s);
  v[1] = cadd(t, r);
  v[2] = csub(t, r);
}
template <int S>
__device__ __forceinline__ void dft4(cplx* v) {
  cplx a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  cplx c = cadd(v[1], v[3]), d = mul_si<S>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <int S>
__device__ __forceinline__ void dft5(cplx* v) {
  const double c1 = 0.30901699437494742410;   // cos(2 pi/5)
  const double c2 = -0.80901699437494742410;  // cos(4 pi/5)
  const double s1 = 0.95105651629515357212;   // sin(2 pi/5)
  const double s2 = 0.58778525229247312917;   // sin(4 pi/5)
  cplx a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  cplx a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  cplx x0 = v[0];
  cplx p1 = make_double2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
  cplx p2 = make_double2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
  cplx q1 = mul_si<S>(make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
  cplx q2 = mul_si<S>(make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
  v[0] = make_double2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  v[1] = cadd(p1, q1);
  v[4] = csub(p1, q1);
  v[2] = cadd(p2, q2);
  v[3] = csub(p2, q2);
}
template <int S>
__device__ __forceinline__ void dft8(cplx* v) {
  const double h = 0.70710678118654752440;  // sqrt(2)/2
  cplx e[4] = {v[0], v[2], v[4], v[6]};
  cplx o[4] = {v[1], v[3], v[5], v[7]};
  dft4<S>(e);
  dft4<S>(o);
  // w8^k = exp(S 2 pi i k / 8)
  cplx o1 = make_double2(h * (o[1].x - S * o[1].y), h * (o[1].y + S * o[1].x));
  cplx o2 = mul_si<S>(o[2]);
  cplx o3 = make_double2(h * (-o[3].x - S * o[3].y), h * (-o[3].y + S * o[3].x));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}
template <int R, int S>
__device__ __forceinline__ void dft(cplx* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 5) dft5<S>(v);
  else dft8<S>(v);
}

// One Stockham radix-R pass over `ntr` transforms of length n stored at
// buf[t*trs + i], in place.  ns = product of the radices already applied.
// Stockham step: butterfly j reads x[j + r*n/R], twiddles by
// exp(S 2 pi i r (j mod ns) / (ns R)), and writes y[(j - j mod ns) R + j mod ns + r ns].
template <int R, int S>
__device__ void stockham_pass(cplx* buf, int ntr, int trs, int n, int ns,
                              const cplx* __restrict__ tw) {
  const int nbf = n / R;            // butterflies per transform
  const int rest = nbf / ns;        // n / (ns R)
  const int group = blockDim.x / nbf;
  for (int t0 = 0; t0 < ntr; t0 += group) {
    const int cnt = min(group, ntr - t0);
    const int u = threadIdx.x;
    const bool act = u < cnt * nbf;
    cplx v[R];
    int t = 0, j = 0, k = 0;
    if (act) {
      t = t0 + u / nbf;
      j = u - (u / nbf) * nbf;
      k = j % ns;
      const cplx* b = buf + (size_t)t * trs;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cplx x = b[j + r * nbf];
        if (r > 0 && k > 0) {
          cplx w = tw[r * k * rest];          // r k rest < n: no reduction needed
          if (S > 0) w.y = -w.y;
          x = cmul(x, w);
        }
        v[r] = x;
      }
      dft<R, S>(v);
    }
    __syncthreads();
    if (act) {
      cplx* b = buf + (size_t)t * trs;
      const int idxd = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) b[idxd + r * ns] = v[r];
    }
    __syncthreads();
  }
}

template <int S>
__device__ void fft_lds(cplx* buf, int ntr, int trs, const FftAxis& ax) {
  int ns = 1;
  for (int p = 0; p < ax.npass; ++p) {
    switch (ax.radix[p]) {
      case 2: stockham_pass<2, S>(buf, ntr, trs, ax.n, ns, ax.tw); break;
      case 3: stockham_pass<3, S>(buf, ntr, trs, ax.n, ns, ax.tw); break;
      case 4: stockham_pass<4, S>(buf, ntr, trs, ax.n, ns, ax.tw); break;
      case 5: stockham_pass<5, S>(buf, ntr, trs, ax.n, ns, ax.tw); break;
      default: stockham_pass<8, S>(buf, ntr, trs, ax.n, ns, ax.tw); break;
    }
    ns *= ax.radix[p];
  }
}

struct PlanArgs {            // BoxPlan fields passed by value to kernels
  int n1, n2, n3, ncols, xr;
  const int* col_start;
  const int* col_e;
  const int* col_m2;
  const int* pt_perm;
  const int* pt_col;
  const int* pt_m3;
  const int* ext_m1;
  FftAxis ax1, ax2, ax3;
};

PlanArgs plan_args(const BoxPlan& p) {
  PlanArgs a;
  a.n1 = p.n1; a.n2 = p.n2; a.n3 = p.n3; a.ncols = p.ncols; a.xr = p.xr;
  a.col_start = p.col_start; a.col_e = p.col_e; a.col_m2 = p.col_m2;
  a.pt_perm = p.pt_perm; a.pt_col = p.pt_col; a.pt_m3 = p.pt_m3; a.ext_m1 = p.ext_m1;
  a.ax1 = p.ax1; a.ax2 = p.ax2; a.ax3 = p.ax3;
  return a;
}

__global__ void __launch_bounds__(kThreads)
k_col_inv(PlanArgs P, int ct, const cplx* __restrict__ psi, int64_t ldpsi, cplx* __restrict__ T) {
  extern __shared__ cplx lds[];
  const int c0 = blockIdx.x * ct;
  const int b = blockIdx.y;
  const int ncl = min(ct, P.ncols - c0);
  const int trs = P.n3 + 1;
  for (int i = threadIdx.x; i < ncl * trs; i += blockDim.x) lds[i] = make_double2(0.0, 0.0);
  __syncthreads();
  const int k0 = P.col_start[c0], k1 = P.col_start[c0 + ncl];
  const cplx* src = psi + (size_t)b * ldpsi;
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x)
    lds[(P.pt_col[k] - c0) * trs + P.pt_m3[k]] = src[P.pt_perm[k]];
  __syncthreads();
  fft_lds<+1>(lds, ncl, trs, P.ax3);
  cplx* dst = T + (size_t)b * P.n3 * P.ncols + c0;
  for (int i = threadIdx.x; i < ncl * P.n3; i += blockDim.x) {
    const int j3 = i / ncl, lc = i - j3 * ncl;
    dst[(size_t)j3 * P.ncols + lc] = lds[lc * trs + j3];
  }
}

__global__ void __launch_bounds__(kThreads)
k_plane(PlanArgs P, int rb, const double* __restrict__ v, cplx* __restrict__ T) {
  extern __shared__ cplx lds[];
  const int trse = P.n2 + 1;
  const int trsr = P.n1 + 1;
  cplx* E = lds;
  cplx* Rw = lds + P.xr * trse;
  const int j3 = blockIdx.x;
  const int b = blockIdx.y;
  cplx* tp = T + (size_t)b * P.n3 * P.ncols + (size_t)j3 * P.ncols;
  for (int i = threadIdx.x; i < P.xr * trse; i += blockDim.x) E[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int c = threadIdx.x; c < P.ncols; c += blockDim.x) E[P.col_e[c] * trse + P.col_m2[c]] = tp[c];
  __syncthreads();
  fft_lds<+1>(E, P.xr, trse, P.ax2);
  const double* vp = v + (size_t)j3 * P.n2 * P.n1;
  for (int r0 = 0; r0 < P.n2; r0 += rb) {
    const int nr = min(rb, P.n2 - r0);
    for (int i = threadIdx.x; i < nr * trsr; i += blockDim.x) Rw[i] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int i = threadIdx.x; i < nr * P.xr; i += blockDim.x) {
      const int r = i / P.xr, e = i - r * P.xr;
      Rw[r * trsr + P.ext_m1[e]] = E[e * trse + r0 + r];
    }
    __syncthreads();
    fft_lds<+1>(Rw, nr, trsr, P.ax1);
    for (int i = threadIdx.x; i < nr * P.n1; i += blockDim.x) {
      const int r = i / P.n1, j1 = i - r * P.n1;
      const double s = vp[(size_t)(r0 + r) * P.n1 + j1];
      cplx x = Rw[r * trsr + j1];
      Rw[r * trsr + j1] = make_double2(x.x * s, x.y * s);
    }
    __syncthreads();
    fft_lds<-1>(Rw, nr, trsr, P.ax1);
    for (int i = threadIdx.x; i < nr * P.xr; i += blockDim.x) {
      const int r = i / P.xr, e = i - r * P.xr;
      E[e * trse + r0 + r] = Rw[r * trsr + P.ext_m1[e]];
    }
    __syncthreads();
  }
  fft_lds<-1>(E, P.xr, trse, P.ax2);
  for (int c = threadIdx.x; c < P.ncols; c += blockDim.x) tp[c] = E[P.col_e[c] * trse + P.col_m2[c]];
}

__global__ void __launch_bounds__(kThreads)
k_col_fwd(PlanArgs P, int ct, const cplx* __restrict__ T, const double* __restrict__ kin,
          const cplx* in, int64_t ldin, const cplx* prev, int64_t ldprev, cplx* out,
          int64_t ldout, double alpha, double beta, double gamma) {
  extern __shared__ cplx lds[];
  const int c0 = blockIdx.x * ct;
  const int b = blockIdx.y;
  const int ncl = min(ct, P.ncols - c0);
  const int trs = P.n3 + 1;
  const cplx* srcT = T + (size_t)b * P.n3 * P.ncols + c0;
  for (int i = threadIdx.x; i < ncl * P.n3; i += blockDim.x) {
    const int j3 = i / ncl, lc = i - j3 * ncl;
    lds[lc * trs + j3] = srcT[(size_t)j3 * P.ncols + lc];
  }
  __syncthreads();
  fft_lds<-1>(lds, ncl, trs, P.ax3);
  const int k0 = P.col_start[c0], k1 = P.col_start[c0 + ncl];
  const cplx* inb = in + (size_t)b * ldin;
  cplx* outb = out + (size_t)b * ldout;
  const cplx* prevb = prev ? prev + (size_t)b * ldprev : nullptr;
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const int g = P.pt_perm[k];
    const cplx loc = lds[(P.pt_col[k] - c0) * trs + P.pt_m3[k]];
    const cplx x = inb[g];
    const double t = kin[g];
    cplx val = make_double2(alpha * (loc.x + t * x.x) + beta * x.x,
                            alpha * (loc.y + t * x.y) + beta * x.y);
    if (gamma != 0.0) {
      const cplx p = prevb[g];
      val.x += gamma * p.x;
      val.y += gamma * p.y;
    }
    outb[g] = val;
  }
}

int max_butterflies(const FftAxis& ax) {
  int m = 0;
  for (int p = 0; p < ax.npass; ++p) m = std::max(m, ax.n / ax.radix[p]);
  return m;
}

// (cos, sin) of 2 pi num/den, with the fraction reduced to the first octant
// in exact integer arithmetic before a long-double evaluation.
void sincos_2pi_frac(long long num, long long den, double* c, double* s) {
  num %= den;
  if (num < 0) num += den;
  // angle = 2 pi num/den in [0, 2 pi).  Work with x = 8 num / den in [0, 8).
  const long long e8 = 8 * num;               // octant index = e8 / den
  const long long oct = e8 / den;
  const long long rem = e8 - oct * den;       // position inside the octant, [0, den)
  const long double pi_l = 3.141592653589793238462643383279502884L;
  // theta in [0, pi/4]: the angle measured from the octant's even boundary
  const bool odd = (oct & 1) != 0;
  const long double frac = odd ? (long double)(den - rem) / (long double)den
                               : (long double)rem / (long double)den;
  const long double th = frac * pi_l / 4.0L;
  const long double ct = cosl(th), st = sinl(th);
  // angle = oct*pi/4 + (odd ? pi/4 - th : th)
  long double cc, ss;
  switch (oct) {
    case 0: cc = ct; ss = st; break;             // th
    case 1: cc = st; ss = ct; break;             // pi/2 - th
    case 2: cc = -st; ss = ct; break;            // pi/2 + th
    case 3: cc = -ct; ss = st; break;            // pi - th
    case 4: cc = -ct; ss = -st; break;           // pi + th
    case 5: cc = -st; ss = -ct; break;           // 3pi/2 - th
    case 6: cc = st; ss = -ct; break;            // 3pi/2 + th
    default: cc = ct; ss = -st; break;           // 2pi - th
  }
  *c = (double)cc;
  *s = (double)ss;
}

}  // namespace

bool fft_factor(int n, FftAxis* ax) {
  ax->n = n;
  ax->npass = 0;
  ax->tw = nullptr;
  if (n < 1) return false;
  int m = n;
  const int order[5] = {8, 4, 2, 3, 5};
  for (int r : order) {
    while (m % r == 0) {
      if (ax->npass >= kMaxPasses) return false;
      ax->radix[ax->npass++] = r;
      m /= r;
    }
  }
  if (m != 1) return false;
  // every pass must fit one transform's butterflies in a workgroup
  return max_butterflies(*ax) <= kThreads || n == 1;
}

void fft_host_twiddles(int n, std::vector<cplx>* out) {
  out->resize(n);
  for (int t = 0; t < n; ++t) {
    double c, s;
    sincos_2pi_frac(t, n, &c, &s);
    (*out)[t] = make_double2(c, -s);   // exp(-2 pi i t / n)
  }
}

bool fft_choose_config(const BoxPlan& p, size_t lds_limit, FftLaunchCfg* cfg) {
  const int mb3 = std::max(1, max_butterflies(p.ax3));
  int ct = std::max(1, std::min(32, kThreads / mb3));
  size_t col_lds = (size_t)ct * (p.n3 + 1) * sizeof(cplx);
  while (ct > 1 && col_lds > lds_limit) {
    --ct;
    col_lds = (size_t)ct * (p.n3 + 1) * sizeof(cplx);
  }
  if (col_lds > lds_limit) return false;
  const int mb1 = std::max(1, max_butterflies(p.ax1));
  int rb = std::max(1, std::min(p.n2, kThreads / mb1));
  auto plane_bytes = [&](int r) {
    return ((size_t)p.xr * (p.n2 + 1) + (size_t)r * (p.n1 + 1)) * sizeof(cplx);
  };
  while (rb > 1 && plane_bytes(rb) > lds_limit) --rb;
  if (plane_bytes(rb) > lds_limit) return false;
  cfg->col_tile = ct;
  cfg->col_lds = col_lds;
  cfg->plane_rows = rb;
  cfg->plane_lds = plane_bytes(rb);
  cfg->reg_col = fft_reg_col_supported(p.n3);
  cfg->reg_plane = fft_reg_plane_supported(p, lds_limit);
  cfg->plane_variant = 0;
  return true;
}

hipError_t launch_fft_col_inv(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const cplx* psi,
                              int64_t ldpsi, cplx* T, hipStream_t s) {
  if (cfg.reg_col) return launch_fft_col_inv_reg(p, nb, psi, ldpsi, T, s);
  dim3 grid((p.ncols + cfg.col_tile - 1) / cfg.col_tile, nb);
  hipLaunchKernelGGL(k_col_inv, grid, dim3(kThreads), cfg.col_lds, s, plan_args(p), cfg.col_tile,
                     psi, ldpsi, T);
  return hipGetLastError();
}

hipError_t launch_fft_plane(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const double* vscaled,
                            cplx* T, hipStream_t s) {
  if (cfg.reg_plane) return launch_fft_plane_reg(p, cfg.plane_variant, nb, vscaled, T, s);
  dim3 grid(p.n3, nb);
  hipLaunchKernelGGL(k_plane, grid, dim3(kThreads), cfg.plane_lds, s, plan_args(p), cfg.plane_rows,
                     vscaled, T);
  return hipGetLastError();
}

hipError_t launch_fft_col_fwd(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const cplx* T,
                              const double* kin, const cplx* in, int64_t ldin, const cplx* prev,
                              int64_t ldprev, cplx* out, int64_t ldout, double alpha, double beta,
                              double gamma, hipStream_t s) {
  if (cfg.reg_col)
    return launch_fft_col_fwd_reg(p, nb, T, kin, in, ldin, prev, ldprev, out, ldout, alpha, beta,
                                  gamma, s);
  dim3 grid((p.ncols + cfg.col_tile - 1) / cfg.col_tile, nb);
  hipLaunchKernelGGL(k_col_fwd, grid, dim3(kThreads), cfg.col_lds, s, plan_args(p), cfg.col_tile, T,
                     kin, in, ldin, prev, ldprev, out, ldout, alpha, beta, gamma);
  return hipGetLastError();
}

// Dynamic LDS above the default limit must be opted into per kernel.
hipError_t fft_set_lds_limits(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_col_inv,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_plane, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_col_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}
