// Device-side building blocks of the FFT kernels, generic over the complex
// type (double2 for the FP64 path, float2 for the FP32 filter path):
// complex helpers, small DFTs in registers (radix 2, 3, 4, 5, 8 and their
// products), compile-time twiddles, and transforms spread over a group of G
// lanes of one wavefront.
#pragma once

#include "pw_internal.h"

namespace pwfft {

template <class C>
struct RealOf;
template <>
struct RealOf<double2> {
  using type = double;
};
template <>
struct RealOf<float2> {
  using type = float;
};
template <class C>
using real_t = typename RealOf<C>::type;

template <class C>
__device__ __forceinline__ C mkc(double re, double im) {
  C r;
  r.x = (real_t<C>)re;
  r.y = (real_t<C>)im;
  return r;
}
template <class C>
__device__ __forceinline__ C czero() {
  C r;
  r.x = 0;
  r.y = 0;
  return r;
}
template <class C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class C>
__device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <class C>
__device__ __forceinline__ C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <class C, class S>
__device__ __forceinline__ C cscale(C a, S s) {
  C r;
  r.x = a.x * (real_t<C>)s;
  r.y = a.y * (real_t<C>)s;
  return r;
}
// (S i) z for S = +1 / -1
template <int S, class C>
__device__ __forceinline__ C mul_si(C z) {
  C r;
  if (S > 0) {
    r.x = -z.y;
    r.y = z.x;
  } else {
    r.x = z.y;
    r.y = -z.x;
  }
  return r;
}
template <class C>
__device__ __forceinline__ C conj_mul(C a, C w) {   // a * conj(w)
  C r;
  r.x = a.x * w.x + a.y * w.y;
  r.y = a.y * w.x - a.x * w.y;
  return r;
}

// ---------------------------------------------------------------------------
// Compile-time exp(-2 pi i t / n): octant reduction in exact integer
// arithmetic, then Taylor series on [0, pi/4].
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

constexpr double cx_sin_poly(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / (double)((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos_poly(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / (double)((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
struct CW {
  double re, im;
};
// exp(-2 pi i t / n)
constexpr CW cx_tw(long t, long n) {
  t %= n;
  if (t < 0) t += n;
  const long e8 = 8 * t;
  const long oct = e8 / n;
  const long rem = e8 - oct * n;
  const bool odd = (oct & 1) != 0;
  const double frac = odd ? (double)(n - rem) / (double)n : (double)rem / (double)n;
  const double th = frac * kPi / 4.0;
  const double ct = cx_cos_poly(th), st = cx_sin_poly(th);
  double c = 0.0, s = 0.0;
  switch (oct) {
    case 0: c = ct; s = st; break;
    case 1: c = st; s = ct; break;
    case 2: c = -st; s = ct; break;
    case 3: c = -ct; s = st; break;
    case 4: c = -ct; s = -st; break;
    case 5: c = -st; s = -ct; break;
    case 6: c = st; s = -ct; break;
    default: c = ct; s = -st; break;
  }
  return CW{c, -s};
}

// ---------------------------------------------------------------------------
// Small DFTs y_k = sum_n x_n exp(S 2 pi i n k / R) in registers.
// ---------------------------------------------------------------------------
template <int S, class C>
__device__ __forceinline__ void dft2(C* v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <int S, class C>
__device__ __forceinline__ void dft3(C* v) {
  using Rl = real_t<C>;
  const Rl h = (Rl)0.86602540378443864676;  // sin(2 pi / 3)
  C s = cadd(v[1], v[2]);
  C d = csub(v[1], v[2]);
  C t;
  t.x = v[0].x - (Rl)0.5 * s.x;
  t.y = v[0].y - (Rl)0.5 * s.y;
  C r = mul_si<S>(cscale(d, h));
  v[0] = cadd(v[0], s);
  v[1] = cadd(t, r);
  v[2] = csub(t, r);
}
template <int S, class C>
__device__ __forceinline__ void dft4(C* v) {
  C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  C c = cadd(v[1], v[3]), d = mul_si<S>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <int S, class C>
__device__ __forceinline__ void dft5(C* v) {
  using Rl = real_t<C>;
  const Rl c1 = (Rl)0.30901699437494742410;   // cos(2 pi/5)
  const Rl c2 = (Rl)-0.80901699437494742410;  // cos(4 pi/5)
  const Rl s1 = (Rl)0.95105651629515357212;   // sin(2 pi/5)
  const Rl s2 = (Rl)0.58778525229247312917;   // sin(4 pi/5)
  C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  C x0 = v[0];
  C p1, p2, z;
  p1.x = x0.x + c1 * a1.x + c2 * a2.x;
  p1.y = x0.y + c1 * a1.y + c2 * a2.y;
  p2.x = x0.x + c2 * a1.x + c1 * a2.x;
  p2.y = x0.y + c2 * a1.y + c1 * a2.y;
  z.x = s1 * b1.x + s2 * b2.x;
  z.y = s1 * b1.y + s2 * b2.y;
  const C q1 = mul_si<S>(z);
  z.x = s2 * b1.x - s1 * b2.x;
  z.y = s2 * b1.y - s1 * b2.y;
  const C q2 = mul_si<S>(z);
  v[0].x = x0.x + a1.x + a2.x;
  v[0].y = x0.y + a1.y + a2.y;
  v[1] = cadd(p1, q1);
  v[4] = csub(p1, q1);
  v[2] = cadd(p2, q2);
  v[3] = csub(p2, q2);
}
template <int S, class C>
__device__ __forceinline__ void dft8(C* v) {
  using Rl = real_t<C>;
  const Rl h = (Rl)0.70710678118654752440;  // sqrt(2)/2
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<S>(e);
  dft4<S>(o);
  C o1, o3;
  o1.x = h * (o[1].x - (Rl)S * o[1].y);
  o1.y = h * (o[1].y + (Rl)S * o[1].x);
  const C o2 = mul_si<S>(o[2]);
  o3.x = h * (-o[3].x - (Rl)S * o[3].y);
  o3.y = h * (-o[3].y + (Rl)S * o[3].x);
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}
template <int R, int S, class C>
__device__ __forceinline__ void dft_base(C* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 5) dft5<S>(v);
  else dft8<S>(v);
}

template <int R>
struct Split {
  static constexpr int P = (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : (R % 3 == 0) ? 3 : 5;
  static constexpr int Q = R / P;
};

constexpr int gcd_ce(int a, int b) { return b == 0 ? a : gcd_ce(b, a % b); }
// x with (a x) mod m == 1, for gcd(a, m) == 1 and m >= 2
constexpr int inv_mod_ce(int a, int m) {
  int x = 1;
  while ((a * x) % m != 1) ++x;
  return x;
}

// R-point DFT in registers for R a product of 2, 3, 5.  R = P Q with
// coprime factors: Good-Thomas prime-factor mapping, no twiddles --
// input n = (Q a + P b) mod R, a P-point DFT over a for each b, then a
// Q-point DFT over b for each k1, output k = (Q q' k1 + P p' k2) mod R with
// q' = Q^-1 mod P, p' = P^-1 mod Q (W_R^{nk} = W_P^{a k1} W_Q^{b k2}).
// Otherwise mixed-radix Cooley-Tukey, n = Q a + b, k = k1 + P k2, with
// compile-time twiddles.
template <int R, int S, class C>
__device__ __forceinline__ void dft_reg(C* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2 || R == 3 || R == 4 || R == 5 || R == 8) {
    dft_base<R, S>(v);
  } else if constexpr (gcd_ce(Split<R>::P, Split<R>::Q) == 1) {
    constexpr int P = Split<R>::P, Q = Split<R>::Q;
    constexpr int qi = inv_mod_ce(Q % P, P), pi = inv_mod_ce(P % Q, Q);
    C y[Q][P];
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      C u[P];
#pragma unroll
      for (int a = 0; a < P; ++a) u[a] = v[(Q * a + P * b) % R];
      dft_reg<P, S>(u);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) y[b][k1] = u[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      C w[Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) w[b] = y[b][k1];
      dft_reg<Q, S>(w);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) v[(Q * qi * k1 + P * pi * k2) % R] = w[k2];
    }
  } else {
    constexpr int P = Split<R>::P, Q = Split<R>::Q;
    C y[Q][P];
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      C u[P];
#pragma unroll
      for (int a = 0; a < P; ++a) u[a] = v[Q * a + b];
      dft_reg<P, S>(u);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) {
        if (b * k1 == 0) {
          y[b][k1] = u[k1];
        } else {
          const CW w = cx_tw(b * k1, R);           // exp(-2 pi i b k1 / R)
          y[b][k1] = cmul(u[k1], mkc<C>(w.re, S > 0 ? -w.im : w.im));
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      C w[Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) w[b] = y[b][k1];
      dft_reg<Q, S>(w);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = w[k2];
    }
  }
}

// Exchange with lane (lane ^ M) inside a 16-lane DPP row, on the VALU:
//   M = 1, 2 : quad_perm [1,0,3,2] / [2,3,0,1]
//   M = 4    : row_half_mirror (i -> 7-i) then quad_perm [3,2,1,0]  (7 - (i^3) = i^4)
//   M = 8    : row_ror:8
// Every lane's source lies inside its own row for these patterns, so the
// "old" operand is never used (bound_ctrl set: no initialising move).
// Larger masks fall back to ds_bpermute.
template <int M>
__device__ __forceinline__ int xor_lane_i32(int v) {
  if constexpr (M == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
  } else if constexpr (M == 4) {
    const int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);
    return __builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, true);
  } else if constexpr (M == 8) {
    return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);
  } else {
    return __shfl_xor(v, M);
  }
}

template <int M>
__device__ __forceinline__ double xor_lane(double x) {
  const long long bits = __double_as_longlong(x);
  const int lo = xor_lane_i32<M>((int)(bits & 0xffffffffLL));
  const int hi = xor_lane_i32<M>((int)(bits >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int M>
__device__ __forceinline__ float xor_lane(float x) {
  return __int_as_float(xor_lane_i32<M>(__float_as_int(x)));
}

template <int M, class C>
__device__ __forceinline__ C xor_lane(C v) {
  C r;
  r.x = xor_lane<M>(v.x);
  r.y = xor_lane<M>(v.y);
  return r;
}

// Bit reversal of b in log2(G) bits.
template <int G>
__device__ __forceinline__ int brev(int b) {
  if constexpr (G == 1) {
    return 0;
  } else {
    constexpr int bits = __builtin_ctz(G);
    return (int)(__brev((unsigned)b) >> (32 - bits));
  }
}

// Per-lane twiddles of a length-N = G R transform for lane b of its group,
// loaded once and shared by both directions (all exp(-2 pi i t/N) values):
//   k[q-1] = exp(-2 pi i b q / N), q = 1..R-1      (between registers and lanes)
//   w[s]   = exp(-2 pi i (b mod h) / (2h)) on the upper lane of a stage-s pair
//            (b & h set, h = 2^s) and exactly 1 on the lower lane
//   sg[s]  = -1 on the upper lane, +1 on the lower lane
// so that both lanes of a pair run the same instructions (no divergence).
template <int R, int G, class C>
struct LaneTw {
  static constexpr int kStages = (G > 1) ? __builtin_ctz(G) : 1;
  C k[R > 1 ? R - 1 : 1];
  C w[kStages];
  real_t<C> sg[kStages];
  __device__ __forceinline__ void load(int b, const C* __restrict__ tw) {
    constexpr int N = R * G;
    if constexpr (G > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) k[q - 1] = tw[b * q];
#pragma unroll
      for (int s = 0; s < kStages; ++s) {
        const int h = 1 << s;
        const bool up = (b & h) != 0;
        w[s] = up ? tw[(b & (h - 1)) * (N / (2 * h))] : mkc<C>(1.0, 0.0);
        sg[s] = up ? (real_t<C>)-1 : (real_t<C>)1;
      }
    }
  }
};

// Transform of length N = G R spread over a group of G lanes (lane b, local
// index in its group), R values per lane.
//
// backward (+):  in : v[a]  = x[G a + b]
//                out: v[k1] = X[k1 + R brev(b)]
// forward  (-):  in : v[k1] = Z[k1 + R brev(b)]    (the backward's layout)
//                out: v[a]  = X'[G a + b]
// The forward is the exact adjoint of the backward, stage by stage.
//
// Decimation-in-frequency stage of span h (backward), pair (lo, up):
//   lo <- lo + up,   up <- (lo - up) conj(w)
// each lane forms p + sg v from its own value v and its partner's p, then
// multiplies by conj(w) (exactly 1 on the lower lane).
template <int R, int G, int SI, class C>
__device__ __forceinline__ void dif_stages(C* v, int b, const LaneTw<R, G, C>& t) {
  if constexpr (SI >= 0) {
    constexpr int h = 1 << SI;
    const real_t<C> sg = t.sg[SI];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const C p = xor_lane<h>(v[r]);
      C u;
      u.x = p.x + sg * v[r].x;
      u.y = p.y + sg * v[r].y;
      v[r] = conj_mul(u, t.w[SI]);
    }
    dif_stages<R, G, SI - 1>(v, b, t);
  }
}

// Decimation-in-time stage of span h (forward), pair (lo, up):
//   lo <- lo + w up,   up <- lo - w up
// each lane scales its own value by w (1 on the lower lane), exchanges, and
// forms p + sg x.
template <int R, int G, int SI, class C>
__device__ __forceinline__ void dit_stages(C* v, int b, const LaneTw<R, G, C>& t) {
  if constexpr (SI < LaneTw<R, G, C>::kStages) {
    constexpr int h = 1 << SI;
    const real_t<C> sg = t.sg[SI];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const C x = cmul(t.w[SI], v[r]);
      const C p = xor_lane<h>(x);
      v[r].x = p.x + sg * x.x;
      v[r].y = p.y + sg * x.y;
    }
    dit_stages<R, G, SI + 1>(v, b, t);
  }
}

template <int R, int G, class C>
__device__ __forceinline__ void lane_fft_bwd(C* v, int b, const LaneTw<R, G, C>& t) {
  dft_reg<R, +1>(v);
  if constexpr (G > 1) {
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) v[k1] = conj_mul(v[k1], t.k[k1 - 1]);   // exp(+2 pi i b k1/N)
    dif_stages<R, G, LaneTw<R, G, C>::kStages - 1>(v, b, t);
  }
}

template <int R, int G, class C>
__device__ __forceinline__ void lane_fft_fwd(C* v, int b, const LaneTw<R, G, C>& t) {
  if constexpr (G > 1) {
    dit_stages<R, G, 0>(v, b, t);
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) v[k1] = cmul(v[k1], t.k[k1 - 1]);       // exp(-2 pi i b k1/N)
  }
  dft_reg<R, -1>(v);
}

// Lane-group shape used for a length-N transform: G a power of two <= gmax
// (<= 16, one DPP row), as large as possible with R = N / G >= 3.
constexpr int lane_group(int n, int gmax = 16) {
  int g = 1;
  while (g < gmax && n % (2 * g) == 0 && n / (2 * g) >= 3) g *= 2;
  return g;
}

}  // namespace pwfft
