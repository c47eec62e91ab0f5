// Internal declarations of libpwdft (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pw.h"

typedef double2 cplx;   // interleaved (re, im), 16 bytes

// A complex value stored as an interleaved pair of bfloat16 bit patterns
// (the BF16 storage of pw_apply_h / pw_cheb_filter blocks; arithmetic
// widens to FP32, stores round to nearest even).
struct __attribute__((aligned(4))) bf16c {
  uint16_t re, im;
};

// Loads and stores of block elements whose storage type may differ from the
// arithmetic type: identity for complex128 / complex64, widening from and
// rounding (to nearest even) to bf16 pairs.
__device__ __forceinline__ double2 ld_c(const double2& v) { return v; }
__device__ __forceinline__ float2 ld_c(const float2& v) { return v; }
__device__ __forceinline__ float2 ld_c(const bf16c& v) {
  return make_float2(__uint_as_float((uint32_t)v.re << 16), __uint_as_float((uint32_t)v.im << 16));
}
template <class S, class C>
__device__ __forceinline__ S st_c(const C& v) {
  return v;
}
template <>
__device__ __forceinline__ bf16c st_c<bf16c, float2>(const float2& v) {
  bf16c r;
  r.re = __builtin_bit_cast(uint16_t, (__bf16)v.x);
  r.im = __builtin_bit_cast(uint16_t, (__bf16)v.y);
  return r;
}
template <>
__device__ __forceinline__ bf16c st_c<bf16c, double2>(const double2& v) {   // one rounding
  bf16c r;
  r.re = __builtin_bit_cast(uint16_t, (__bf16)v.x);
  r.im = __builtin_bit_cast(uint16_t, (__bf16)v.y);
  return r;
}


// ---------------------------------------------------------------------------
// FFT plan along one axis: N = product of radices, each in {2, 3, 4, 5, 8}.
// ---------------------------------------------------------------------------
constexpr int kMaxPasses = 8;
struct FftAxis {
  int n;                    // transform length
  int npass;                // number of radix passes
  int radix[kMaxPasses];    // radix of each pass, first pass first
  const cplx* tw;           // device table, tw[t] = exp(-2 pi i t / n), t < n
  const float2* tw32;       // the same table rounded to FP32
};

// Sphere <-> box maps, all device arrays, built once per pw_ham.
struct BoxPlan {
  int n1, n2, n3;
  int64_t npw;
  int ncols;                // distinct (m1, m2) among sphere points ("columns" along N3)
  // row stride, in columns, of the column intermediate T[b][j3][c]: ncols
  // rounded up to a multiple of 16, so that every 16-column slice of a row
  // the column kernels store or load covers whole 128-byte lines
  int ldt;
  int xr;                   // distinct m1 among sphere points (extent along N1)
  // columns ordered by (n1, n2) of the Miller indices; column c holds the
  // points perm[col_start[c] .. col_start[c+1]) (indices into the caller's order)
  int* col_start;           // ncols + 1
  int* col_e;               // extent slot e in [0, xr) of the column's m1
  int* col_m2;              // box index m2 of the column
  int* pt_perm;             // npw: caller index of the k-th point in column order
  int* pt_col;              // npw: column of the k-th point (column order)
  int* pt_m3;               // npw: box index m3 of the k-th point (column order)
  int* ext_m1;              // xr: box index m1 of extent slot e
  int quarter12;            // 1: every point's centred m1 and m2 lie in [-N/4, N/4)
  // 1: the caller's order is the column order (pt_perm is the identity); a
  // column's points then hold consecutive centred m3 from col_m3lo[c] up
  // (the sphere is convex along N3), so the column kernels need no per-point
  // index arrays
  int runs;
  int* col_m3lo;            // ncols: centred m3 of the column's first point
  FftAxis ax1, ax2, ax3;
};

// ---------------------------------------------------------------------------
// Fused batches: one launch per stage covers every item; each item's sizes,
// plan and buffers are read from an array of ItemDev in device memory
// (indexed by the launch's item coordinate).  Block buffers have ld = npw.
// ---------------------------------------------------------------------------
struct ItemDev {
  BoxPlan plan;
  int npw, nb, nproj, gemm_target;
  int col_tile, plane_rows;            // generic FFT kernels' tiles of this item's box
  cplx* y;                             // complex128 blocks
  cplx* hy;
  cplx* blk;
  float2* b32[2];                      // complex64 blocks of the low-precision filter
  cplx* T;                             // FFT intermediates (all nb bands)
  float2* T32;
  const double* kin;
  const double* vs;                    // V / N_box
  const float* kin32;
  const float* vs32;
  const cplx* proj;
  const float2* proj32;
  const uint16_t* proj3;               // stored three-term copies of proj32 (launch_split3):
  const uint16_t* proj3c;              //   rows = plane waves / rows = projectors
  uint16_t* cprj3;                     // three-term copy of cprj32^T (rows = bands)
  const double* ekb;
  cplx* cprj;
  float2* cprj32;
  cplx* gemm_work;
  float2* work32;
  cplx* sub0;                          // nb x nb, ld nb
  cplx* sub1;
  cplx* dinv;
  double* dtol;
  int* status;
  double* eig;
  double* resid;
  double* coef;                        // 3 per filter step
  double* upper;
  int* flags;
  int* sweeps;
};

// Matrix products of the fused launches (FP64 unless noted):
//   GOP_PROJ     cprj = alpha diag(E_KB) P^H X        (X = block sel_b; FP32 variant: cprj32)
//   GOP_GRAM     sub0 = Y^H X                         (X = block sel_b)
//   GOP_NONLOCAL X += P cprj                          (X = block sel_c; FP32 variant: cprj32)
//   GOP_TRSM     blk = Y dinv                         (one diagonal block: nb <= 64)
//   GOP_ROT      blk = X sub1                         (X = block sel_a)
enum GemmOp : int { GOP_PROJ = 0, GOP_GRAM = 1, GOP_NONLOCAL = 2, GOP_TRSM = 3, GOP_ROT = 4 };

// Block selectors of the fused launches.
enum BlockSel : int { SEL_Y = 0, SEL_HY = 1, SEL_BLK = 2, SEL_B32A = 3, SEL_B32B = 4, SEL_NONE = 5 };

__device__ __forceinline__ cplx* item_blk64(const ItemDev& d, int s) {
  return s == SEL_Y ? d.y : s == SEL_HY ? d.hy : s == SEL_BLK ? d.blk : nullptr;
}
__device__ __forceinline__ float2* item_blk32(const ItemDev& d, int s) {
  return s == SEL_B32A ? d.b32[0] : s == SEL_B32B ? d.b32[1] : nullptr;
}

// Host-side launch shape of one fused group.  Items of a group share the FFT
// kernel family: register column kernels need one N3, the register plane
// kernel one N1 = N2; the generic kernels take every length from the item.
struct FusedFft {
  int n1, n2, n3;                      // the shared lengths (register kernels)
  int n3_max;                          // plane grid
  int nitems, nb_max, ncols_max, xr_max;
  bool reg_col, reg_plane;
  int plane_variant, plane_variant32;
  int col_blocks;                      // generic column grid: max over items of ceil(ncols / tile)
  size_t col_lds, plane_lds;           // generic kernels, largest item
};

// ---------------------------------------------------------------------------
// Launch helpers (defined in the .hip files), all enqueue on `s`.
// ---------------------------------------------------------------------------
struct FftLaunchCfg {
  int col_tile;             // columns per workgroup of the N3 kernels (generic path)
  int plane_rows;           // rows per batch in the plane kernel (generic path)
  size_t col_lds, plane_lds;
  bool reg_col;             // register-resident column kernels available for N3
  bool reg_plane;           // register-resident plane kernel available for (N1, N2)
  int plane_variant;        // FP64 register plane kernel: 0 = lane groups <= 16, 1 = <= 8
  int plane_variant32;      // FP32: 0 / 1 as above, 2 = LDS-exchange kernel (fft_ls.hip)
};

// Host-side choice of tiles and LDS sizes; returns false if this GPU's LDS
// cannot hold the plane kernel's working set.
bool fft_choose_config(const BoxPlan& p, size_t lds_limit, FftLaunchCfg* cfg);
// Build the twiddle table of an axis on the host (exact angle reduction).
void fft_host_twiddles(int n, std::vector<cplx>* out);
// Factor n into passes; false if unsupported.
bool fft_factor(int n, FftAxis* ax);

// Coefficients of the gather epilogue out = alpha (loc + kin in) + beta in + gamma prev.
// If coef is non-null the kernel reads (alpha, beta, gamma) = coef[0..2] from
// device memory (graph-replayable filter steps); prev is read iff non-null.
struct Epilogue {
  double alpha, beta, gamma;
  const double* coef;
};

// psi block (nb bands from band0) -> T[b][j3][c], backward along N3.
hipError_t launch_fft_col_inv(const BoxPlan& p, const FftLaunchCfg& cfg, int nb,
                              const cplx* psi, int64_t ldpsi, cplx* T, hipStream_t s);
// per (band, plane): N2 backward, N1 backward, x V, N1 forward, N2 forward, in place on T.
hipError_t launch_fft_plane(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const double* vscaled,
                            cplx* T, hipStream_t s);
// forward along N3 and gather, with the epilogue (prev may alias out)
hipError_t launch_fft_col_fwd(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const cplx* T,
                              const double* kin, const cplx* in, int64_t ldin, const cplx* prev,
                              int64_t ldprev, cplx* out, int64_t ldout, const Epilogue& ep,
                              hipStream_t s);
// FP32 versions (complex64 blocks, FP32 tables): register kernels when the box allows, else generic
hipError_t launch_fft_col_inv32(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const float2* psi,
                                int64_t ldpsi, float2* T, hipStream_t s);
hipError_t launch_fft_plane32(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const float* vscaled,
                              float2* T, hipStream_t s);
hipError_t launch_fft_col_fwd32(const BoxPlan& p, const FftLaunchCfg& cfg, int nb, const float2* T,
                                const float* kin, const float2* in, int64_t ldin, const float2* prev,
                                int64_t ldprev, float2* out, int64_t ldout, const Epilogue& ep,
                                hipStream_t s);

// Fused-batch FFT stages over the items D[0 .. f.nitems) (block selectors as in BlockSel;
// coef_step >= 0 reads the epilogue coefficients from item.coef + 3 coef_step).
hipError_t launch_fused_col_inv(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                hipStream_t s);
hipError_t launch_fused_plane(const FusedFft& f, bool fp32, const ItemDev* D, hipStream_t s);
hipError_t launch_fused_col_fwd(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                int sel_out, int sel_prev, double alpha, double beta, double gamma,
                                int coef_step, hipStream_t s);
hipError_t launch_fused_col_inv_reg(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                    hipStream_t s);
hipError_t launch_fused_plane_reg(const FusedFft& f, bool fp32, const ItemDev* D, hipStream_t s);
hipError_t launch_fused_col_fwd_reg(const FusedFft& f, bool fp32, const ItemDev* D, int sel_in,
                                    int sel_out, int sel_prev, double alpha, double beta,
                                    double gamma, int coef_step, hipStream_t s);

// Fused-batch products over items D[0 .. nitems) (see GemmOp).  m_max / n_max
// bound the output tiles of any item; nsplit_max the split count of any item.
hipError_t launch_fused_gemm_cn(int nitems, int64_t m_max, int64_t n_max, int nsplit_max,
                                const ItemDev* D, int op, int sel_b, double alpha, int coef_step,
                                hipStream_t s);
hipError_t launch_fused_gemm_nn(int nitems, int64_t m_max, int64_t n_max, const ItemDev* D, int op,
                                int sel_a, int sel_c, hipStream_t s);
// the split count the fused GOP_PROJ / GOP_GRAM product uses for one item
int fused_cn_nsplit(int op, int64_t npw, int64_t nb, int64_t nproj, int target);
hipError_t launch_fused_gemm_cn32(int bf16, int nitems, int64_t m_max, int64_t n_max,
                                  int nsplit_max, const ItemDev* D, int sel_b, double alpha,
                                  int coef_step, hipStream_t s);
hipError_t launch_fused_gemm_nn32(int bf16, int nitems, int64_t m_max, int64_t n_max,
                                  const ItemDev* D, int sel_c, hipStream_t s);
int fused_cn32_nsplit(int bf16, int64_t npw, int64_t nb, int64_t nproj, int target);

// Fused-batch subspace and filter steps (one launch over all items):
//   FS_CHEB_COEF (arg0 = degree), FS_FILTER_FIRST (arg0 = 1: FP32 b32[1], 0: FP64 blk),
//   FS_TO_F32 (y -> b32[0]), FS_TO_F64 (b32[arg0 - SEL_B32A] -> y), FS_COPY (arg0 -> arg1),
//   FS_HERMITIZE (sub0), FS_CHOL_INIT / FS_CHOL_DIAG (sub0 -> U, dinv; nb <= 64),
//   FS_JACOBI (sub0 -> eig, sub1; nb <= 64), FS_RESIDUALS, FS_FLAGS.
enum FusedStep : int {
  FS_CHEB_COEF, FS_FILTER_FIRST, FS_TO_F32, FS_TO_F64, FS_COPY, FS_HERMITIZE, FS_CHOL_INIT,
  FS_CHOL_DIAG, FS_JACOBI, FS_RESIDUALS, FS_FLAGS
};
hipError_t launch_fused_dense(FusedStep step, int nitems, int64_t npw_nb_max, int nb_max,
                              const ItemDev* D, int arg0, int arg1, hipStream_t s);

// Allow `bytes` of dynamic LDS for the FFT kernels (above the default cap).
hipError_t fft_set_lds_limits(size_t bytes);

// Register-resident variants (fft_reg.hip) for the box lengths they are built for.
bool fft_reg_col_supported(int n3);
bool fft_reg_plane_supported(const BoxPlan& p, size_t lds_limit);
bool fft_reg_plane_narrow(const BoxPlan& p, bool fp32);   // an 8-lane plane variant exists
hipError_t fft_reg_set_lds_limits(size_t bytes);
// FP32 plane kernel with LDS exchanges for N1 = N2 = 144 (fft_ls.hip).
size_t fft_plane_ls_lds(const BoxPlan& p);
bool fft_plane_ls_supported(const BoxPlan& p, size_t lds_limit);
hipError_t launch_fft_plane_ls32(const BoxPlan& p, int nb, const float* vscaled, float2* T,
                                 hipStream_t s);
hipError_t fft_ls_set_lds_limit(size_t bytes);

// Electron density (density.hip; generic form in fft_kernels.hip)
hipError_t launch_density_planes_reg(const BoxPlan& p, int nbc, const cplx* T, const double* w,
                                     int ngroup, double* part, int add, hipStream_t s);
hipError_t launch_density_planes_gen(const BoxPlan& p, const FftLaunchCfg& cfg, int nbc,
                                     const cplx* T, const double* w, int ngroup, double* part,
                                     int add, hipStream_t s);
hipError_t launch_density_reduce(int64_t nbox, int ngroup, const double* part, double scale,
                                 double* rho, int accumulate, hipStream_t s);
bool density_reg_supported(const BoxPlan& p, size_t lds_limit);
int density_row_parts(const BoxPlan& p);   // workgroups per (plane, band group), register kernel
hipError_t density_set_lds_limit(size_t bytes);
hipError_t launch_fft_col_inv_reg(const BoxPlan& p, int nb, const cplx* psi, int64_t ldpsi, cplx* T,
                                  hipStream_t s);
hipError_t launch_fft_plane_reg(const BoxPlan& p, int variant, int nb, const double* vscaled,
                                cplx* T, hipStream_t s);
hipError_t launch_fft_col_fwd_reg(const BoxPlan& p, int nb, const cplx* T, const double* kin,
                                  const cplx* in, int64_t ldin, const cplx* prev, int64_t ldprev,
                                  cplx* out, int64_t ldout, const Epilogue& ep, hipStream_t s);
// FP32 (complex64 blocks, FP32 V/N_box and kinetic tables) variants
hipError_t launch_fft_col_inv_reg32(const BoxPlan& p, int nb, const float2* psi, int64_t ldpsi,
                                    float2* T, hipStream_t s);
hipError_t launch_fft_plane_reg32(const BoxPlan& p, int variant, int nb, const float* vscaled,
                                  float2* T, hipStream_t s);
hipError_t launch_fft_col_fwd_reg32(const BoxPlan& p, int nb, const float2* T, const float* kin,
                                    const float2* in, int64_t ldin, const float2* prev,
                                    int64_t ldprev, float2* out, int64_t ldout, const Epilogue& ep,
                                    hipStream_t s);
// The same with the blocks (psi, in, prev, out) stored as bf16 pairs; FP32
// arithmetic and FP32 column intermediate T.
hipError_t launch_fft_col_inv_reg16(const BoxPlan& p, int nb, const bf16c* psi, int64_t ldpsi,
                                    float2* T, hipStream_t s);
hipError_t launch_fft_col_fwd_reg16(const BoxPlan& p, int nb, const float2* T, const float* kin,
                                    const bf16c* in, int64_t ldin, const bf16c* prev,
                                    int64_t ldprev, bf16c* out, int64_t ldout, const Epilogue& ep,
                                    hipStream_t s);

// Split-K C = alpha diag(rowscale) A^H B + beta C (see pw_gemm_cn).  `work`
// holds splits*m*n cplx (gemm_cn_work_elems); with work == null the product
// is not split.  rowscale (m doubles on device) may be null.
size_t gemm_cn_work_elems(int64_t m, int64_t n, int64_t k);
// alpha_dev (may be null): device scalar read in place of alpha.
hipError_t launch_gemm_cn(int64_t m, int64_t n, int64_t k, double alpha, const cplx* A, int64_t lda,
                          const cplx* B, int64_t ldb, cplx* C, int64_t ldc, const double* rowscale,
                          cplx* work, hipStream_t s, double beta = 0.0,
                          const double* alpha_dev = nullptr, int target_blocks = 2048,
                          int upper = 0,    // 1 (m == n, Hermitian result): only the 64 x 64
                                            // tiles on and above the diagonal are formed
                          cplx* craw = nullptr, int64_t ldraw = 0);  // also alpha A^H B without
                                                                     // rowscale (beta = 0 only)
// tile 0: 64 x 64 workgroup tiles; 1: 128 x 64 (tall products)
hipError_t launch_gemm_nn(int64_t m, int64_t n, int64_t k, double alpha, const cplx* A, int64_t lda,
                          const cplx* B, int64_t ldb, double beta, cplx* C, int64_t ldc,
                          hipStream_t s, int tile = 0);

// Low-precision products (gemm32_kernels.hip): complex64 operands, FP32
// accumulation; bf16 != 0 rounds the MFMA operands to bfloat16.
size_t gemm_cn32_work_elems(int64_t m, int64_t n, int64_t k, int bf16);
hipError_t launch_gemm_cn32(int bf16, int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                            int64_t lda, const float2* B, int64_t ldb, float2* C, int64_t ldc,
                            const double* rowscale, float2* work, hipStream_t s,
                            const double* alpha_dev = nullptr, int target_blocks = 2048);
// FP32 (bf16 = 0) with a3 and b3 given: A B from the stored three-term
// copies a3 of A (rows m, contraction k) and b3 of B^T (rows n, contraction
// k); A and B are then not read and tile has no effect.
hipError_t launch_gemm_nn32(int bf16, int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                            int64_t lda, const float2* B, int64_t ldb, double beta, float2* C,
                            int64_t ldc, hipStream_t s, int tile = 0, const uint16_t* a3 = nullptr,
                            const uint16_t* b3 = nullptr);
// As launch_gemm_cn32 with bf16 = 0, A given as the stored three-term copy a3
// of A^T (rows m, contraction k); with c3, the reduction also stores the
// three-term copy of C^T (rows n, contraction m) for launch_gemm_nn32.
hipError_t launch_gemm_cn32_s3(int64_t m, int64_t n, int64_t k, double alpha, const uint16_t* a3,
                               const float2* B, int64_t ldb, float2* C, int64_t ldc,
                               const double* rowscale, float2* work, hipStream_t s,
                               const double* alpha_dev, int target_blocks, uint16_t* c3);
// bf16 operands with the block operand stored as bf16 pairs: A^H B with B a
// bf16-pair block (split-K partials and result complex64, as launch_gemm_cn32
// with bf16 = 1), and C (bf16 pairs) = alpha A B + beta C with A, B complex64.
hipError_t launch_gemm_cn32_s16(int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                                int64_t lda, const bf16c* B, int64_t ldb, float2* C, int64_t ldc,
                                const double* rowscale, float2* work, hipStream_t s,
                                const double* alpha_dev = nullptr, int target_blocks = 2048);
hipError_t launch_gemm_nn32_s16(int64_t m, int64_t n, int64_t k, double alpha, const float2* A,
                                int64_t lda, const float2* B, int64_t ldb, double beta, bf16c* C,
                                int64_t ldc, hipStream_t s, int tile = 0);
// Stored three-term copies: X3 holds X (rows x k; element (r, c) at
// X[r sr + c sk]) split exactly into three bf16 terms per real part, in
// chunks of 32 contraction values (six planes of 32 bf16 per chunk, a row's
// chunks consecutive), rows padded to a multiple of 64 and k to 32, with
// zeros; split3_elems gives its size in bf16.
size_t split3_elems(int64_t rows, int64_t k);
hipError_t launch_split3(int64_t rows, int64_t k, const float2* X, int64_t sr, int64_t sk,
                         uint16_t* X3, hipStream_t s);

// Precision conversions
hipError_t launch_block_to_f32(int64_t rows, int64_t cols, const cplx* x, int64_t ldx, float2* y,
                               int64_t ldy, hipStream_t s);
hipError_t launch_block_to_f64(int64_t rows, int64_t cols, const float2* x, int64_t ldx, cplx* y,
                               int64_t ldy, hipStream_t s);
hipError_t launch_axpby_to_f32(int64_t rows, int64_t cols, double a, const cplx* x, int64_t ldx,
                               double b, const cplx* y, int64_t ldy, float2* out, int64_t ldo,
                               hipStream_t s, const double* coef = nullptr);
hipError_t launch_real_to_f32(int64_t n, const double* src, double scale, float* dst, hipStream_t s);
// complex128 <-> bf16-pair blocks (one rounding to nearest even; widening is exact)
hipError_t launch_block_to_b16(int64_t rows, int64_t cols, const cplx* x, int64_t ldx, bf16c* y,
                               int64_t ldy, hipStream_t s);
hipError_t launch_block_b16_to_f64(int64_t rows, int64_t cols, const bf16c* x, int64_t ldx, cplx* y,
                                   int64_t ldy, hipStream_t s);
// out = a x + b y rounded to bf16 pairs (x, y complex128); coef overrides a, b
hipError_t launch_axpby_to_b16(int64_t rows, int64_t cols, double a, const cplx* x, int64_t ldx,
                               double b, const cplx* y, int64_t ldy, bf16c* out, int64_t ldo,
                               hipStream_t s, const double* coef = nullptr);
hipError_t launch_tw_to_f32(int n, const cplx* src, float2* dst, hipStream_t s);

// Dense kernels (dense_kernels.hip)
// kin[g] = 1/2 |(n_g + k) B|^2 from device Miller indices; recip9/k3 are host values.
hipError_t launch_kinetic(int64_t npw, const int* miller, const double* recip9, const double* k3,
                          double* kin, hipStream_t s);
hipError_t launch_scale_copy(int64_t n, const double* src, double scale, double* dst, hipStream_t s);
hipError_t launch_max_reduce(int64_t n, const double* x, double* out1, hipStream_t s);
// a <- its upper triangle mirrored: a[j][i] = conj(a[i][j]) for i < j, Im a[i][i] = 0
hipError_t launch_hermitize(int64_t n, cplx* a, int64_t lda, hipStream_t s);
hipError_t launch_copy_block(int64_t rows, int64_t cols, const cplx* src, int64_t lds, cplx* dst,
                             int64_t ldd, hipStream_t s);
hipError_t launch_scale_rows_cols(int64_t n, const double* d, cplx* a, int64_t lda, hipStream_t s);
// out = a*x + b*y for npw x nb blocks (out may alias y); coef (device, may be null) overrides a, b
hipError_t launch_axpby_block(int64_t npw, int64_t nb, double a, const cplx* x, int64_t ldx, double b,
                              const cplx* y, int64_t ldy, cplx* out, int64_t ldo, hipStream_t s,
                              const double* coef = nullptr);
// Sticky failure flags of one batch item (chol_status may be null).
hipError_t launch_batch_flags(const int* chol_status, const int* sweeps, int* flags, hipStream_t s);
// Filter coefficients (3 per step) on the device from eig (ascending) and upper[0].
hipError_t launch_cheb_coef(const double* eig, int nb, const double* upper, int degree, double* coef,
                            int* flag, hipStream_t s);
// status: 0 if every element finite, else 1
hipError_t launch_check_finite(int64_t n, const double* x, int* flag, hipStream_t s);
// Blocked Cholesky pieces: tol = n eps max diag, status = -1; per diagonal
// block (kb <= 64) factor + inverse of the factor in LDS.  The status word:
// -1 no failure, p >= 0 the first pivot at or below tol, kCholNonFinite - j
// diagonal entry j is NaN or infinite (column j of the block is not finite;
// set by the init step, never overwritten by a pivot).
constexpr int kCholBlock = 64;
constexpr int kCholNonFinite = -2;
hipError_t launch_chol_init(int64_t n, const cplx* a, int64_t lda, double* tol, int* status,
                            hipStream_t s);
hipError_t launch_chol_diag(int kb, int k0, cplx* a, int64_t lda, cplx* dinv, const double* tol,
                            int* status, hipStream_t s);
hipError_t launch_zero_lower(int64_t n, cplx* a, int64_t lda, hipStream_t s);
hipError_t launch_identity(int64_t n, cplx* a, int64_t lda, hipStream_t s);
// Cyclic Jacobi eigensolver of a Hermitian n x n matrix (n > 64: block
// Jacobi over blocks of 16, one LDS sweep per block pair and round): w
// ascending, q = eigenvectors; a is read only.  work: heev_work_bytes(n)
// device bytes.  launch_heev_async issues at most max_sweeps outer sweeps
// (in [1, 40]) with the convergence test on the device and reads nothing
// back: sweeps_dev[0] = sweeps used, or -1 if the limit was reached.
size_t heev_work_bytes(int64_t n);
// n <= 64 only: the whole solve in one workgroup, no host synchronisation;
// sweeps_dev[0] = sweeps used or -1.
hipError_t launch_heev_small_async(int64_t n, const cplx* a, int64_t lda, double* w, cplx* q,
                                   int64_t ldq, int* sweeps_dev, hipStream_t s);
hipError_t heev_set_lds_limit(size_t bytes);
hipError_t launch_heev_async(int64_t n, const cplx* a, int64_t lda, double* w, cplx* q,
                             int64_t ldq, void* work, int* sweeps_dev, int max_sweeps,
                             hipStream_t s);
// The same with the largest sweep limit, then waits for the stream and
// returns the sweep count (or -1) in *sweeps_done (host_scratch: one int of
// pinned host memory).
hipError_t launch_heev(int64_t n, const cplx* a, int64_t lda, double* w, cplx* q, int64_t ldq,
                       void* work, int* sweeps_dev, int* host_scratch, int* sweeps_done,
                       hipStream_t s);
constexpr int kHeevMaxSweeps = 40;
// Deferred status: rec = {status, op, info}; the first failure since the
// last clear is kept (chol_status[0] >= 0: NOT_POSDEF at that pivot;
// sweeps[0] < 0: NO_CONVERGENCE).  Either pointer may be null.
hipError_t launch_status_record(const int* chol_status, const int* sweeps, int op, int* rec,
                                hipStream_t s);
hipError_t launch_fill_int(int n, int v, int* p, hipStream_t s);
hipError_t launch_residuals(int64_t npw, int64_t nb, const cplx* W, int64_t ldw, const cplx* Y,
                            int64_t ldy, const double* lam, double* resid, hipStream_t s);
