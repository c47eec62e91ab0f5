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
#include "fft_common.h"

#include <algorithm>
#include <cmath>

using namespace pwfft;

namespace {

constexpr int kThreads = 256;

// One Stockham radix-R pass over `ntr` transforms of length n stored at
// buf[t*trs + i], in place.  ns = product of the radices already applied.
// Stockham step: butterfly j reads x[j + r*n/R], twiddles by
// exp(S 2 pi i r (j mod ns) / (ns R)), and writes y[(j - j mod ns) R + j mod ns + r ns].
template <int R, int S, class C>
__device__ void stockham_pass(C* buf, int ntr, int trs, int n, int ns, const C* __restrict__ tw) {
  const int nbf = n / R;            // butterflies per transform
  const int rest = nbf / ns;        // n / (ns R)
  const int group = blockDim.x / nbf;
  for (int t0 = 0; t0 < ntr; t0 += group) {
    const int cnt = min(group, ntr - t0);
    const int u = threadIdx.x;
    const bool act = u < cnt * nbf;
    C v[R];
    int t = 0, j = 0, k = 0;
    if (act) {
      t = t0 + u / nbf;
      j = u - (u / nbf) * nbf;
      k = j % ns;
      const C* b = buf + (size_t)t * trs;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C x = b[j + r * nbf];
        if (r > 0 && k > 0) {
          C w = tw[r * k * rest];          // r k rest < n: no reduction needed
          if (S > 0) w.y = -w.y;
          x = cmul(x, w);
        }
        v[r] = x;
      }
      dft_base<R, S>(v);
    }
    __syncthreads();
    if (act) {
      C* b = buf + (size_t)t * trs;
      const int idxd = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) b[idxd + r * ns] = v[r];
    }
    __syncthreads();
  }
}

template <class C>
__device__ __forceinline__ const C* ax_tw(const FftAxis& ax);
template <>
__device__ __forceinline__ const double2* ax_tw<double2>(const FftAxis& ax) { return ax.tw; }
template <>
__device__ __forceinline__ const float2* ax_tw<float2>(const FftAxis& ax) { return ax.tw32; }

template <int S, class C>
__device__ void fft_lds(C* buf, int ntr, int trs, const FftAxis& ax) {
  int ns = 1;
  const C* tw = ax_tw<C>(ax);
  for (int p = 0; p < ax.npass; ++p) {
    switch (ax.radix[p]) {
      case 2: stockham_pass<2, S>(buf, ntr, trs, ax.n, ns, tw); break;
      case 3: stockham_pass<3, S>(buf, ntr, trs, ax.n, ns, tw); break;
      case 4: stockham_pass<4, S>(buf, ntr, trs, ax.n, ns, tw); break;
      case 5: stockham_pass<5, S>(buf, ntr, trs, ax.n, ns, tw); break;
      default: stockham_pass<8, S>(buf, ntr, trs, ax.n, ns, tw); break;
    }
    ns *= ax.radix[p];
  }
}

struct PlanArgs {            // BoxPlan fields passed by value to kernels
  int n1, n2, n3, ncols, ldt, xr;
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
  a.n1 = p.n1; a.n2 = p.n2; a.n3 = p.n3; a.ncols = p.ncols; a.ldt = p.ldt; a.xr = p.xr;
  a.col_start = p.col_start; a.col_e = p.col_e; a.col_m2 = p.col_m2;
  a.pt_perm = p.pt_perm; a.pt_col = p.pt_col; a.pt_m3 = p.pt_m3; a.ext_m1 = p.ext_m1;
  a.ax1 = p.ax1; a.ax2 = p.ax2; a.ax3 = p.ax3;
  return a;
}

template <class C, class PL>
__device__ __forceinline__ void col_inv_body(const PL& P, int ct, const C* __restrict__ psi,
                                             int64_t ldpsi, C* __restrict__ T, int cb, int b) {
  extern __shared__ __align__(16) char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const int c0 = cb * ct;
  const int ncl = min(ct, P.ncols - c0);
  const int trs = P.n3 + 1;
  for (int i = threadIdx.x; i < ncl * trs; i += blockDim.x) lds[i] = czero<C>();
  __syncthreads();
  const int k0 = P.col_start[c0], k1 = P.col_start[c0 + ncl];
  const C* src = psi + (size_t)b * ldpsi;
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x)
    lds[(P.pt_col[k] - c0) * trs + P.pt_m3[k]] = src[P.pt_perm[k]];
  __syncthreads();
  fft_lds<+1>(lds, ncl, trs, P.ax3);
  C* dst = T + (size_t)b * P.n3 * P.ldt + c0;
  for (int i = threadIdx.x; i < ncl * P.n3; i += blockDim.x) {
    const int j3 = i / ncl, lc = i - j3 * ncl;
    dst[(size_t)j3 * P.ldt + lc] = lds[lc * trs + j3];
  }
}

template <class C>
__global__ void __launch_bounds__(kThreads)
k_col_inv(PlanArgs P, int ct, const C* __restrict__ psi, int64_t ldpsi, C* __restrict__ T) {
  col_inv_body<C>(P, ct, psi, ldpsi, T, blockIdx.x, blockIdx.y);
}

template <class C, class PL>
__device__ __forceinline__ void plane_body(const PL& P, int rb, const real_t<C>* __restrict__ v,
                                           C* __restrict__ T, int j3, int b) {
  extern __shared__ __align__(16) char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const int trse = P.n2 + 1;
  const int trsr = P.n1 + 1;
  C* E = lds;
  C* Rw = lds + P.xr * trse;
  C* tp = T + (size_t)b * P.n3 * P.ldt + (size_t)j3 * P.ldt;
  for (int i = threadIdx.x; i < P.xr * trse; i += blockDim.x) E[i] = czero<C>();
  __syncthreads();
  for (int c = threadIdx.x; c < P.ncols; c += blockDim.x) E[P.col_e[c] * trse + P.col_m2[c]] = tp[c];
  __syncthreads();
  fft_lds<+1>(E, P.xr, trse, P.ax2);
  const real_t<C>* vp = v + (size_t)j3 * P.n2 * P.n1;
  for (int r0 = 0; r0 < P.n2; r0 += rb) {
    const int nr = min(rb, P.n2 - r0);
    for (int i = threadIdx.x; i < nr * trsr; i += blockDim.x) Rw[i] = czero<C>();
    __syncthreads();
    for (int i = threadIdx.x; i < nr * P.xr; i += blockDim.x) {
      const int r = i / P.xr, e = i - r * P.xr;
      Rw[r * trsr + P.ext_m1[e]] = E[e * trse + r0 + r];
    }
    __syncthreads();
    fft_lds<+1>(Rw, nr, trsr, P.ax1);
    for (int i = threadIdx.x; i < nr * P.n1; i += blockDim.x) {
      const int r = i / P.n1, j1 = i - r * P.n1;
      Rw[r * trsr + j1] = cscale(Rw[r * trsr + j1], vp[(size_t)(r0 + r) * P.n1 + j1]);
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

template <class C>
__global__ void __launch_bounds__(kThreads)
k_plane(PlanArgs P, int rb, const real_t<C>* __restrict__ v, C* __restrict__ T) {
  plane_body<C>(P, rb, v, T, blockIdx.x, blockIdx.y);
}

// Electron density, any box (section 2.4, Eq. nandtau): for z-plane j3 and
// band group g, the backward N2 and N1 transforms of the chunk's bands
// b = g, g + ngroup, ... as in plane_body, w_b |.|^2 added to the group's
// partial array part[g][j3][j2][j1].  Element i of a row batch belongs to
// thread i mod blockDim for every band, so each element has one writer.
__global__ void __launch_bounds__(kThreads)
k_density_plane(PlanArgs P, int rb, const double2* __restrict__ T, int nbc,
                const double* __restrict__ w, int ngroup, double* __restrict__ part, int add) {
  extern __shared__ __align__(16) char lds_raw[];
  double2* E = reinterpret_cast<double2*>(lds_raw);
  const int trse = P.n2 + 1, trsr = P.n1 + 1;
  double2* Rw = E + P.xr * trse;
  const int j3 = blockIdx.x, g = blockIdx.y;
  double* pp = part + ((size_t)g * P.n3 + j3) * P.n2 * P.n1;
  if (g >= nbc && !add) {   // a group without bands in the first chunk starts from zero
    for (int i = threadIdx.x; i < P.n2 * P.n1; i += blockDim.x) pp[i] = 0.0;
    return;
  }
  bool fresh = !add;
  for (int b = g; b < nbc; b += ngroup) {
    const double2* tp = T + ((size_t)b * P.n3 + j3) * P.ldt;
    __syncthreads();
    for (int i = threadIdx.x; i < P.xr * trse; i += blockDim.x) E[i] = czero<double2>();
    __syncthreads();
    for (int c = threadIdx.x; c < P.ncols; c += blockDim.x)
      E[P.col_e[c] * trse + P.col_m2[c]] = tp[c];
    __syncthreads();
    fft_lds<+1>(E, P.xr, trse, P.ax2);
    const double wb = w[b];
    for (int r0 = 0; r0 < P.n2; r0 += rb) {
      const int nr = min(rb, P.n2 - r0);
      for (int i = threadIdx.x; i < nr * trsr; i += blockDim.x) Rw[i] = czero<double2>();
      __syncthreads();
      for (int i = threadIdx.x; i < nr * P.xr; i += blockDim.x) {
        const int r = i / P.xr, e = i - r * P.xr;
        Rw[r * trsr + P.ext_m1[e]] = E[e * trse + r0 + r];
      }
      __syncthreads();
      fft_lds<+1>(Rw, nr, trsr, P.ax1);
      for (int i = threadIdx.x; i < nr * P.n1; i += blockDim.x) {
        const int r = i / P.n1, j1 = i - r * P.n1;
        const double2 v = Rw[r * trsr + j1];
        double* d = pp + (size_t)(r0 + r) * P.n1 + j1;
        *d = (fresh ? 0.0 : *d) + wb * (v.x * v.x + v.y * v.y);
      }
      __syncthreads();
    }
    fresh = false;
  }
}

template <class C, class PL>
__device__ __forceinline__ void col_fwd_body(const PL& P, int ct, const C* __restrict__ T,
                                             const real_t<C>* __restrict__ kin, const C* in,
                                             int64_t ldin, const C* prev, int64_t ldprev, C* out,
                                             int64_t ldout, double alpha_d, double beta_d,
                                             double gamma_d, const double* __restrict__ coef,
                                             int cb, int b) {
  using Rl = real_t<C>;
  extern __shared__ __align__(16) char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  if (coef) {
    alpha_d = coef[0];
    beta_d = coef[1];
    gamma_d = coef[2];
  }
  const Rl alpha = (Rl)alpha_d, beta = (Rl)beta_d, gamma = (Rl)gamma_d;
  const int c0 = cb * ct;
  const int ncl = min(ct, P.ncols - c0);
  const int trs = P.n3 + 1;
  const C* srcT = T + (size_t)b * P.n3 * P.ldt + c0;
  for (int i = threadIdx.x; i < ncl * P.n3; i += blockDim.x) {
    const int j3 = i / ncl, lc = i - j3 * ncl;
    lds[lc * trs + j3] = srcT[(size_t)j3 * P.ldt + lc];
  }
  __syncthreads();
  fft_lds<-1>(lds, ncl, trs, P.ax3);
  const int k0 = P.col_start[c0], k1 = P.col_start[c0 + ncl];
  const C* inb = in + (size_t)b * ldin;
  C* outb = out + (size_t)b * ldout;
  const C* prevb = prev ? prev + (size_t)b * ldprev : nullptr;
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const int g = P.pt_perm[k];
    const C loc = lds[(P.pt_col[k] - c0) * trs + P.pt_m3[k]];
    const C x = inb[g];
    const Rl t = kin[g];
    C val;
    val.x = alpha * (loc.x + t * x.x) + beta * x.x;
    val.y = alpha * (loc.y + t * x.y) + beta * x.y;
    if (prevb) {
      const C p = prevb[g];
      val.x += gamma * p.x;
      val.y += gamma * p.y;
    }
    outb[g] = val;
  }
}

template <class C>
__global__ void __launch_bounds__(kThreads)
k_col_fwd(PlanArgs P, int ct, const C* __restrict__ T, const real_t<C>* __restrict__ kin,
          const C* in, int64_t ldin, const C* prev, int64_t ldprev, C* out, int64_t ldout,
          double alpha_d, double beta_d, double gamma_d, const double* __restrict__ coef) {
  col_fwd_body<C>(P, ct, T, kin, in, ldin, prev, ldprev, out, ldout, alpha_d, beta_d, gamma_d,
                  coef, blockIdx.x, blockIdx.y);
}

// ---- fused-batch variants (item = blockIdx.z; tiles from the item's descriptor)
template <class C>
__device__ __forceinline__ C* gen_block(const ItemDev& d, int sel);
template <>
__device__ __forceinline__ double2* gen_block<double2>(const ItemDev& d, int sel) {
  return item_blk64(d, sel);
}
template <>
__device__ __forceinline__ float2* gen_block<float2>(const ItemDev& d, int sel) {
  return item_blk32(d, sel);
}
template <class C>
__device__ __forceinline__ C* gen_T(const ItemDev& d);
template <>
__device__ __forceinline__ double2* gen_T<double2>(const ItemDev& d) { return d.T; }
template <>
__device__ __forceinline__ float2* gen_T<float2>(const ItemDev& d) { return d.T32; }

template <class C>
__global__ void __launch_bounds__(kThreads)
kb_col_inv(const ItemDev* __restrict__ D, int sel_in) {
  const ItemDev& d = D[blockIdx.z];
  if ((int)blockIdx.y >= d.nb || (int)blockIdx.x * d.col_tile >= d.plan.ncols) return;
  col_inv_body<C>(d.plan, d.col_tile, gen_block<C>(d, sel_in), d.npw, gen_T<C>(d), blockIdx.x,
                  blockIdx.y);
}

template <class C>
__global__ void __launch_bounds__(kThreads)
kb_plane(const ItemDev* __restrict__ D) {
  const ItemDev& d = D[blockIdx.z];
  if ((int)blockIdx.y >= d.nb || (int)blockIdx.x >= d.plan.n3) return;
  if constexpr (sizeof(C) == sizeof(double2))
    plane_body<C>(d.plan, d.plane_rows, d.vs, gen_T<C>(d), blockIdx.x, blockIdx.y);
  else
    plane_body<C>(d.plan, d.plane_rows, d.vs32, gen_T<C>(d), blockIdx.x, blockIdx.y);
}

template <class C>
__global__ void __launch_bounds__(kThreads)
kb_col_fwd(const ItemDev* __restrict__ D, int sel_in, int sel_out, int sel_prev, double alpha,
           double beta, double gamma, int coef_step) {
  const ItemDev& d = D[blockIdx.z];
  if ((int)blockIdx.y >= d.nb || (int)blockIdx.x * d.col_tile >= d.plan.ncols) return;
  const double* coef = coef_step >= 0 ? d.coef + 3 * coef_step : nullptr;
  if constexpr (sizeof(C) == sizeof(double2))
    col_fwd_body<C>(d.plan, d.col_tile, gen_T<C>(d), d.kin, gen_block<C>(d, sel_in), d.npw,
                    gen_block<C>(d, sel_prev), d.npw, gen_block<C>(d, sel_out), d.npw, alpha, beta,
                    gamma, coef, blockIdx.x, blockIdx.y);
  else
    col_fwd_body<C>(d.plan, d.col_tile, gen_T<C>(d), d.kin32, gen_block<C>(d, sel_in), d.npw,
                    gen_block<C>(d, sel_prev), d.npw, gen_block<C>(d, sel_out), d.npw, alpha, beta,
                    gamma, coef, blockIdx.x, blockIdx.y);
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
  cfg->plane_variant32 = 0;
  return true;
}

namespace {

template <class C>
hipError_t col_inv_generic(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const C* psi,
                           int64_t ldpsi, C* T, hipStream_t s) {
  dim3 grid((p.ncols + cfg.col_tile - 1) / cfg.col_tile, nb);
  hipLaunchKernelGGL(k_col_inv<C>, grid, dim3(kThreads), cfg.col_lds, s, plan_args(p), cfg.col_tile,
                     psi, ldpsi, T);
  return hipGetLastError();
}

template <class C>
hipError_t plane_generic(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const real_t<C>* vs, C* T,
                         hipStream_t s) {
  dim3 grid(p.n3, nb);
  hipLaunchKernelGGL(k_plane<C>, grid, dim3(kThreads), cfg.plane_lds, s, plan_args(p),
                     cfg.plane_rows, vs, T);
  return hipGetLastError();
}

template <class C>
hipError_t col_fwd_generic(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const C* T,
                           const real_t<C>* kin, const C* in, int64_t ldin, const C* prev,
                           int64_t ldprev, C* out, int64_t ldout, const Epilogue& ep, hipStream_t s) {
  dim3 grid((p.ncols + cfg.col_tile - 1) / cfg.col_tile, nb);
  hipLaunchKernelGGL(k_col_fwd<C>, grid, dim3(kThreads), cfg.col_lds, s, plan_args(p), cfg.col_tile,
                     T, kin, in, ldin, prev, ldprev, out, ldout, ep.alpha, ep.beta, ep.gamma,
                     ep.coef);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_density_planes_gen(const BoxPlan& p, const FftLaunchCfg& cfg, int nbc,
                                     const cplx* T, const double* w, int ngroup, double* part,
                                     int add, hipStream_t s) {
  hipLaunchKernelGGL(k_density_plane, dim3(p.n3, ngroup), dim3(kThreads), cfg.plane_lds, s,
                     plan_args(p), cfg.plane_rows, T, nbc, w, ngroup, part, add);
  return hipGetLastError();
}

hipError_t launch_fft_col_inv(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const cplx* psi,
                              int64_t ldpsi, cplx* T, hipStream_t s) {
  if (cfg.reg_col) return launch_fft_col_inv_reg(p, nb, psi, ldpsi, T, s);
  return col_inv_generic<double2>(p, cfg, nb, psi, ldpsi, T, s);
}
hipError_t launch_fft_col_inv32(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const float2* psi,
                                int64_t ldpsi, float2* T, hipStream_t s) {
  if (cfg.reg_col) return launch_fft_col_inv_reg32(p, nb, psi, ldpsi, T, s);
  return col_inv_generic<float2>(p, cfg, nb, psi, ldpsi, T, s);
}

hipError_t launch_fft_plane(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const double* vscaled,
                            cplx* T, hipStream_t s) {
  if (cfg.reg_plane) return launch_fft_plane_reg(p, cfg.plane_variant, nb, vscaled, T, s);
  return plane_generic<double2>(p, cfg, nb, vscaled, T, s);
}
hipError_t launch_fft_plane32(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const float* vscaled,
                              float2* T, hipStream_t s) {
  if (cfg.reg_plane && cfg.plane_variant32 == 2) return launch_fft_plane_ls32(p, nb, vscaled, T, s);
  if (cfg.reg_plane) return launch_fft_plane_reg32(p, cfg.plane_variant32, nb, vscaled, T, s);
  return plane_generic<float2>(p, cfg, nb, vscaled, T, s);
}

hipError_t launch_fft_col_fwd(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const cplx* T,
                              const double* kin, const cplx* in, int64_t ldin, const cplx* prev,
                              int64_t ldprev, cplx* out, int64_t ldout, const Epilogue& ep,
                              hipStream_t s) {
  if (cfg.reg_col)
    return launch_fft_col_fwd_reg(p, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
  return col_fwd_generic<double2>(p, cfg, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
}
hipError_t launch_fft_col_fwd32(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const float2* T,
                                const float* kin, const float2* in, int64_t ldin, const float2* prev,
                                int64_t ldprev, float2* out, int64_t ldout, const Epilogue& ep,
                                hipStream_t s) {
  if (cfg.reg_col)
    return launch_fft_col_fwd_reg32(p, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
  return col_fwd_generic<float2>(p, cfg, nb, T, kin, in, ldin, prev, ldprev, out, ldout, ep, s);
}

hipError_t launch_fused_col_inv(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                hipStream_t s) {
  if (f.reg_col) return launch_fused_col_inv_reg(f, fp32, D, sel_in, s);
  dim3 grid(f.col_blocks, f.nb_max, f.nitems);
  if (fp32)
    hipLaunchKernelGGL(kb_col_inv<float2>, grid, dim3(kThreads), f.col_lds, s, D, sel_in);
  else
    hipLaunchKernelGGL(kb_col_inv<double2>, grid, dim3(kThreads), f.col_lds, s, D, sel_in);
  return hipGetLastError();
}

hipError_t launch_fused_plane(const FusedFft& f, bool fp32, const ItemDev* D, hipStream_t s) {
  if (f.reg_plane) return launch_fused_plane_reg(f, fp32, D, s);
  dim3 grid(f.n3_max, f.nb_max, f.nitems);
  if (fp32)
    hipLaunchKernelGGL(kb_plane<float2>, grid, dim3(kThreads), f.plane_lds, s, D);
  else
    hipLaunchKernelGGL(kb_plane<double2>, grid, dim3(kThreads), f.plane_lds, s, D);
  return hipGetLastError();
}

hipError_t launch_fused_col_fwd(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                int sel_out, int sel_prev, double alpha, double beta, double gamma,
                                int coef_step, hipStream_t s) {
  if (f.reg_col)
    return launch_fused_col_fwd_reg(f, fp32, D, sel_in, sel_out, sel_prev, alpha, beta, gamma,
                                    coef_step, s);
  dim3 grid(f.col_blocks, f.nb_max, f.nitems);
  if (fp32)
    hipLaunchKernelGGL(kb_col_fwd<float2>, grid, dim3(kThreads), f.col_lds, s, D, sel_in, sel_out,
                       sel_prev, alpha, beta, gamma, coef_step);
  else
    hipLaunchKernelGGL(kb_col_fwd<double2>, grid, dim3(kThreads), f.col_lds, s, D, sel_in, sel_out,
                       sel_prev, alpha, beta, gamma, coef_step);
  return hipGetLastError();
}

// Dynamic LDS above the default limit must be opted into per kernel.
hipError_t fft_set_lds_limits(size_t bytes) {
  const void* fns[13] = {(const void*)k_col_inv<double2>, (const void*)k_plane<double2>,
                         (const void*)k_col_fwd<double2>, (const void*)k_col_inv<float2>,
                         (const void*)k_plane<float2>, (const void*)k_col_fwd<float2>,
                         (const void*)kb_col_inv<double2>, (const void*)kb_plane<double2>,
                         (const void*)kb_col_fwd<double2>, (const void*)kb_col_inv<float2>,
                         (const void*)kb_plane<float2>, (const void*)kb_col_fwd<float2>,
                         (const void*)k_density_plane};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
