// libpwdft host side: contexts, Hamiltonian handles (plans + workspaces) and
// the orchestration of the hot path on one HIP stream.
//
//   pw_apply_h        section 5.1 (apply H to a block) + section 5.2 Eq. (ham-nl)
//   pw_cheb_filter    section 5.1 (Chebyshev filtering, textbook scaled recurrence)
//   pw_orthonormalize section 5.4 (full-band Cholesky orthogonalisation)
//   pw_rayleigh_ritz  section 5.1 (Rayleigh-Ritz subspace diagonalisation)
#include "plan_host.h"
#include "pw_handles.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_set>
#include <vector>

#define PW_VERSION "0.1.0"

struct BatchItem {
  pw_ham* h = nullptr;
  int64_t nb = 0;
  cplx* y = nullptr;
  cplx* hy = nullptr;
  double* eig = nullptr;
  double* resid = nullptr;
  double* coef = nullptr;    // 3 * degree filter coefficients (device)
  double* upper = nullptr;   // spectral upper bound (device)
  int* flags = nullptr;      // 4 sticky failure flags (device)
  int* sweeps = nullptr;     // sweeps of the last eigensolve (device)
  int stream = 0;
};

struct pw_batch {
  pw_ctx* ctx = nullptr;
  int degree = 0;
  pw_prec prec = PW_FP64;
  std::vector<BatchItem> items;
  std::vector<hipStream_t> streams;
  hipStream_t s0 = nullptr;         // graph launch / fork-join stream
  std::vector<hipEvent_t> ev;       // [0] ctx->s0, [1] s0->ctx, [2] fork, [3 + k] join of stream k
  hipGraph_t graph = nullptr;        // mode 1: one graph, a branch per stream
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraph_t> sgraph;    // mode 2: one graph per stream
  std::vector<hipGraphExec_t> sexec;
  struct Group {                     // mode 3: items fused per box, one launch per stage
    FusedFft f{};
    ItemDev* D = nullptr;            // device descriptors of the group's items
    int nitems = 0, nb_max = 0, nproj_max = 0;
    int64_t npw_max = 0, npw_nb_max = 0;
    int nsplit_proj = 1, nsplit_gram = 1, nsplit_proj32 = 1;
  };
  std::vector<Group> groups;
  hipGraph_t fgraph = nullptr;
  hipGraphExec_t fexec = nullptr;
  std::vector<void*> allocs;
  int* flags_dev = nullptr;         // 4 per item
  int* flags_host = nullptr;        // pinned copy
  int max_sweeps = 0;
};

// Workspace of pw_heev_noalloc: one static device array per GPU, large
// enough for the block-Jacobi work of a 512 x 512 problem.  Host code never
// uses the symbol itself (on the host it is only a stand-in): pw_ctx_create
// resolves each device's own address of it once, with that device current,
// and every later use goes through that address.
constexpr size_t kScratchBytes = (size_t)13 << 20;
constexpr int kScratchHeevMax = 512;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace pwi {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved once per device).
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

thread_local std::string g_err;

pw_status fail(pw_ctx* c, pw_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_err = msg;
  return s;
}

void dfree(pw_ham* h, void* p) {
  auto it = std::find(h->allocs.begin(), h->allocs.end(), p);
  if (it == h->allocs.end()) return;
  (void)hipFree(p);
  h->allocs.erase(it);
}

void free_ham(pw_ham* h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

bool ranges_overlap(const void* a, int64_t lda, const void* b, int64_t ldb, int64_t rows,
                    int64_t cols, int64_t elem) {
  const char* a0 = static_cast<const char*>(a);
  const char* a1 = a0 + ((cols - 1) * lda + rows) * elem;
  const char* b0 = static_cast<const char*>(b);
  const char* b1 = b0 + ((cols - 1) * ldb + rows) * elem;
  return a0 < b1 && b0 < a1;
}

// byte spans [a, a + abytes) and [b, b + bbytes) intersect
bool spans_overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
  const char* a0 = static_cast<const char*>(a);
  const char* b0 = static_cast<const char*>(b);
  return abytes > 0 && bbytes > 0 && a0 < b0 + bbytes && b0 < a0 + abytes;
}

pw_status check_block(pw_ham* h, const void* p, int64_t ld, const char* name) {
  if (!p) return fail(h->ctx, PW_ERR_INVALID_ARG, std::string(name) + " is NULL");
  if (ld < h->npw)
    return fail(h->ctx, PW_ERR_INVALID_ARG,
                std::string("leading dimension of ") + name + " (" + std::to_string(ld) +
                    ") < npw (" + std::to_string(h->npw) + ")");
  return PW_OK;
}

pw_status check_hot(pw_ham* h, pw_prec prec, int64_t nb) {
  if (prec != PW_FP64 && prec != PW_FP32 && prec != PW_BF16)
    return fail(h->ctx, PW_ERR_INVALID_ARG, "unknown precision");
  if (prec != PW_FP64 && !h->low_prec)
    return fail(h->ctx, PW_ERR_UNSUPPORTED,
                "FP32/BF16 need a handle created with low_prec = 1");
  if (nb < 1 || nb > h->nb_max)
    return fail(h->ctx, PW_ERR_INVALID_ARG,
                "nb = " + std::to_string(nb) + " outside [1, nb_max = " + std::to_string(h->nb_max) +
                    "]");
  return PW_OK;
}

// out = alpha (H in) + beta in + gamma prev (prev may alias out).  coef (device,
// may be null) holds {alpha, beta, gamma} and then overrides the host scalars;
// prev is read whenever it is non-null.
pw_status ham_apply(pw_ham* h, int64_t nb, const cplx* in, int64_t ldin, cplx* out, int64_t ldout,
                    double alpha, double beta, double gamma, const cplx* prev, int64_t ldprev,
                    const double* coef, cplx* craw) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  const bool fork = h->nproj > 0 && c->overlap && c->stream == c->home;
  if (h->nproj > 0) {
    // P^H psi on the second stream, concurrent with the FFT route below
    hipStream_t ps = fork ? c->aux : s;
    if (fork) {
      HIPCHK(c, hipEventRecord(c->ev_fork, s));
      HIPCHK(c, hipStreamWaitEvent(ps, c->ev_fork, 0));
    }
    StageScope sc(c, PW_STAGE_PROJ, ps);
    HIPCHK(c, launch_gemm_cn(h->nproj, nb, h->npw, alpha, h->proj, h->npw, in, ldin, h->cprj,
                             h->nproj, h->ekb_dev, h->gemm_work, ps, 0.0, coef, h->gemm_target, 0,
                             craw, h->nproj));
  }
  if (fork) HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
  const Epilogue ep{alpha, beta, gamma, coef};
  for (int64_t c0 = 0; c0 < nb; c0 += h->chunk) {
    const int nc = (int)std::min<int64_t>(h->chunk, nb - c0);
    {
      StageScope sc(c, PW_STAGE_FFT_COL_INV);
      HIPCHK(c, launch_fft_col_inv(h->plan, h->cfg, nc, in + c0 * ldin, ldin, h->T, s));
    }
    {
      StageScope sc(c, PW_STAGE_FFT_PLANE);
      HIPCHK(c, launch_fft_plane(h->plan, h->cfg, nc, h->vscaled, h->T, s));
    }
    {
      StageScope sc(c, PW_STAGE_FFT_COL_FWD);
      HIPCHK(c, launch_fft_col_fwd(h->plan, h->cfg, nc, h->T, h->kin, in + c0 * ldin, ldin,
                                   prev ? prev + c0 * ldprev : nullptr, ldprev, out + c0 * ldout,
                                   ldout, ep, s));
    }
  }
  if (fork) HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
  if (h->nproj > 0) {
    StageScope sc(c, PW_STAGE_NONLOCAL);
    HIPCHK(c, launch_gemm_nn(h->npw, nb, h->nproj, 1.0, h->proj, h->npw, h->cprj, h->nproj, 1.0,
                             out, ldout, s, h->nn_tile));
  }
  return PW_OK;
}

// Low-precision H application on complex64 blocks (FFT route in FP32; the
// projector products in FP32 or, with bf16, bfloat16 operands; FP32
// accumulation): out = alpha (H in) + beta in + gamma prev, coef as above.
pw_status ham_apply32(pw_ham* h, int bf16, int64_t nb, const float2* in, int64_t ldin, float2* out,
                      int64_t ldout, double alpha, double beta, double gamma, const float2* prev,
                      int64_t ldprev, const double* coef = nullptr) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  const bool fork = h->nproj > 0 && c->overlap && c->stream == c->home;
  if (h->nproj > 0) {
    // P^H psi on the second stream, concurrent with the FFT route below
    hipStream_t ps = fork ? c->aux : s;
    if (fork) {
      HIPCHK(c, hipEventRecord(c->ev_fork, s));
      HIPCHK(c, hipStreamWaitEvent(ps, c->ev_fork, 0));
    }
    StageScope sc(c, PW_STAGE_PROJ_LP, ps);
    if (bf16)
      HIPCHK(c, launch_gemm_cn32(1, h->nproj, nb, h->npw, alpha, h->proj32, h->npw, in, ldin,
                                 h->cprj32, h->nproj, h->ekb_dev, h->work32, ps, coef,
                                 h->gemm_target));
    else
      HIPCHK(c, launch_gemm_cn32_s3(h->nproj, nb, h->npw, alpha, h->proj3c, in, ldin, h->cprj32,
                                    h->nproj, h->ekb_dev, h->work32, ps, coef, h->gemm_target,
                                    h->cprj3));
  }
  if (fork) HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
  const Epilogue ep{alpha, beta, gamma, coef};
  for (int64_t c0 = 0; c0 < nb; c0 += h->chunk) {
    const int nc = (int)std::min<int64_t>(h->chunk, nb - c0);
    {
      StageScope sc(c, PW_STAGE_FFT_COL_INV_LP);
      HIPCHK(c, launch_fft_col_inv32(h->plan, h->cfg, nc, in + c0 * ldin, ldin, h->T32, s));
    }
    {
      StageScope sc(c, PW_STAGE_FFT_PLANE_LP);
      HIPCHK(c, launch_fft_plane32(h->plan, h->cfg, nc, h->vs32, h->T32, s));
    }
    {
      StageScope sc(c, PW_STAGE_FFT_COL_FWD_LP);
      HIPCHK(c, launch_fft_col_fwd32(h->plan, h->cfg, nc, h->T32, h->kin32, in + c0 * ldin, ldin,
                                     prev ? prev + c0 * ldprev : nullptr, ldprev, out + c0 * ldout,
                                     ldout, ep, s));
    }
  }
  if (fork) HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
  if (h->nproj > 0) {
    StageScope sc(c, PW_STAGE_NONLOCAL_LP);
    HIPCHK(c, launch_gemm_nn32(bf16, h->npw, nb, h->nproj, 1.0, h->proj32, h->npw, h->cprj32,
                               h->nproj, 1.0, out, ldout, s, h->nn_tile32, h->proj3, h->cprj3));
  }
  return PW_OK;
}

// H application on bf16-pair blocks: the register column kernels read and
// write bf16 pairs (FP32 arithmetic, FP32 column intermediate), the
// projector products take the block operand straight from bf16 storage
// (bf16 MFMA operands, FP32 accumulation, complex64 cprj):
// out = alpha (H in) + beta in + gamma prev, coef as in ham_apply.
pw_status ham_apply16(pw_ham* h, int64_t nb, const bf16c* in, int64_t ldin, bf16c* out,
                      int64_t ldout, double alpha, double beta, double gamma, const bf16c* prev,
                      int64_t ldprev, const double* coef = nullptr) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  if (!h->reg_col_ok)
    return fail(c, PW_ERR_UNSUPPORTED, "BF16 block storage needs the register column kernels");
  if (h->nproj > 0) {
    StageScope sc(c, PW_STAGE_PROJ_LP);
    HIPCHK(c, launch_gemm_cn32_s16(h->nproj, nb, h->npw, alpha, h->proj32, h->npw, in, ldin,
                                   h->cprj32, h->nproj, h->ekb_dev, h->work32, s, coef,
                                   h->gemm_target));
  }
  const Epilogue ep{alpha, beta, gamma, coef};
  for (int64_t c0 = 0; c0 < nb; c0 += h->chunk) {
    const int nc = (int)std::min<int64_t>(h->chunk, nb - c0);
    {
      StageScope sc(c, PW_STAGE_FFT_COL_INV_LP);
      HIPCHK(c, launch_fft_col_inv_reg16(h->plan, nc, in + c0 * ldin, ldin, h->T32, s));
    }
    {
      StageScope sc(c, PW_STAGE_FFT_PLANE_LP);
      HIPCHK(c, launch_fft_plane32(h->plan, h->cfg, nc, h->vs32, h->T32, s));
    }
    {
      StageScope sc(c, PW_STAGE_FFT_COL_FWD_LP);
      HIPCHK(c, launch_fft_col_fwd_reg16(h->plan, nc, h->T32, h->kin32, in + c0 * ldin, ldin,
                                         prev ? prev + c0 * ldprev : nullptr, ldprev,
                                         out + c0 * ldout, ldout, ep, s));
    }
  }
  if (h->nproj > 0) {
    StageScope sc(c, PW_STAGE_NONLOCAL_LP);
    HIPCHK(c, launch_gemm_nn32_s16(h->npw, nb, h->nproj, 1.0, h->proj32, h->npw, h->cprj32,
                                   h->nproj, 1.0, out, ldout, s, h->nn_tile32));
  }
  return PW_OK;
}

// In-place right multiplication of a block by the nb x nb matrix m (ld nb), via blk.
pw_status rotate_block(pw_ham* h, int64_t nb, cplx* y, int64_t ld, const cplx* m) {
  pw_ctx* c = h->ctx;
  StageScope sc(c, PW_STAGE_ROTATE);
  HIPCHK(c, launch_gemm_nn(h->npw, nb, nb, 1.0, y, ld, m, nb, 0.0, h->blk, h->npw, c->stream,
                           h->nn_tile));
  HIPCHK(c, launch_copy_block(h->npw, nb, h->blk, h->npw, y, ld, c->stream));
  return PW_OK;
}

pw_status heev_status(pw_ctx* c, int sweeps) {
  if (sweeps < 0)
    return fail(c, PW_ERR_NO_CONVERGENCE, "Jacobi eigensolver did not converge in its sweep limit");
  return PW_OK;
}

const char* op_name(int op) {
  switch (op) {
    case kOpOrtho: return "pw_orthonormalize";
    case kOpRayleighRitz: return "pw_rayleigh_ritz";
    case kOpLobpcg: return "pw_lobpcg";
    case kOpRmmDiis: return "pw_rmm_diis";
    case kOpHeev: return "pw_heev_noalloc";
  }
  return "a hot call";
}

// Blocked upper Cholesky a = U^H U in place (upper triangle read; blocks
// below the diagonal are left with scratch values).  dinv receives the
// inverse of diagonal block j at dinv + j*kb*kb (ld = that block's size);
// panel holds kb x n; status[0] = -1 or the failing pivot.
hipError_t chol_blocked(int64_t n, cplx* a, int64_t lda, cplx* dinv, cplx* panel, double* tol,
                        int* status, hipStream_t s) {
  const int kb = kCholBlock;
  hipError_t e = launch_chol_init(n, a, lda, tol, status, s);
  for (int64_t k0 = 0; k0 < n && e == hipSuccess; k0 += kb) {
    const int kbk = (int)std::min<int64_t>(kb, n - k0);
    const int64_t m = n - k0 - kbk;
    cplx* dk = dinv + (k0 / kb) * kb * kb;
    e = launch_chol_diag(kbk, (int)k0, a, lda, dk, tol, status, s);
    if (e != hipSuccess || m == 0) break;
    cplx* row = a + k0 + (k0 + kbk) * lda;                       // U[k, k+1:]
    // row <- U_kk^{-H} A[k, k+1:]  (no workspace: the product is not split)
    e = launch_gemm_cn(kbk, m, kbk, 1.0, dk, kbk, row, lda, panel, kbk, nullptr, nullptr, s);
    if (e == hipSuccess) e = launch_copy_block(kbk, m, panel, kbk, row, lda, s);
    // A[k+1:, k+1:] -= row^H row
    if (e == hipSuccess)
      e = launch_gemm_cn(m, m, kbk, -1.0, row, lda, row, lda, a + (k0 + kbk) + (k0 + kbk) * lda, lda,
                         nullptr, nullptr, s, 1.0);
  }
  return e;
}

// y <- y U^{-1} for a rows x n block (ld), by column blocks J:
// y[:, J] = (y[:, J] - y[:, <J] U[<J, J]) U_JJ^{-1}.  tmp: rows x kb.
hipError_t trsm_right(int64_t rows, int64_t n, cplx* y, int64_t ld, const cplx* u, int64_t ldu,
                      const cplx* dinv, cplx* tmp, hipStream_t s, int tile) {
  const int kb = kCholBlock;
  hipError_t e = hipSuccess;
  for (int64_t j0 = 0; j0 < n && e == hipSuccess; j0 += kb) {
    const int kbj = (int)std::min<int64_t>(kb, n - j0);
    if (j0 > 0)
      e = launch_gemm_nn(rows, kbj, j0, -1.0, y, ld, u + j0 * ldu, ldu, 1.0, y + j0 * ld, ld, s,
                         tile);
    if (e == hipSuccess)
      e = launch_gemm_nn(rows, kbj, kbj, 1.0, y + j0 * ld, ld, dinv + (j0 / kb) * kb * kb, kbj, 0.0,
                         tmp, rows, s, tile);
    if (e == hipSuccess) e = launch_copy_block(rows, kbj, tmp, rows, y + j0 * ld, ld, s);
  }
  return e;
}

// Blocked Cholesky of the Gram matrix in sub0 (S = U^H U), its failing
// pivot recorded under op, then Y <- Y U^{-1} and, if hy is given,
// HY <- HY U^{-1}.
pw_status chol_and_solve(pw_ham* h, int64_t nb, cplx* y, int64_t ld, cplx* hy, int64_t ldhy, int op,
                         cplx* cp) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  {
    StageScope sc(c, PW_STAGE_CHOL);
    HIPCHK(c, chol_blocked(nb, h->sub0, nb, h->dinv, h->panel, h->dtol, h->status_dev, s));
    HIPCHK(c, launch_status_record(h->status_dev, nullptr, op, c->rec_dev, s));
  }
  {
    StageScope sc(c, PW_STAGE_ROTATE);
    HIPCHK(c, trsm_right(h->npw, nb, y, ld, h->sub0, nb, h->dinv, h->blk, s, h->nn_tile));
    if (hy)
      HIPCHK(c, trsm_right(h->npw, nb, hy, ldhy, h->sub0, nb, h->dinv, h->blk, s, h->nn_tile));
    // projections kept in memory: (P^H Y) U^{-1} = P^H (Y U^{-1}); h->cprj is free scratch here
    if (cp && h->nproj > 0)
      HIPCHK(c, trsm_right(h->nproj, nb, cp, h->nproj, h->sub0, nb, h->dinv, h->cprj, s, 0));
  }
  return PW_OK;
}

// Cholesky orthonormalisation of a block: Gram in FP64, blocked Cholesky,
// Y <- Y U^{-1} (and HY alike); a failing pivot goes to the context's
// deferred status under op.  gram_prec FP32 / BF16: a first pass whose Gram
// matrix is formed from a complex64 copy of Y on the bf16 matrix cores
// (FP32: three-term split operands, FP32-accurate products; BF16: bf16
// operands), factored in FP64 and applied in FP64, then the FP64 pass on
// the nearly orthonormal result (Cholesky QR twice), so the low-precision
// Gram matrix never decides the final orthonormality.  No host
// synchronisation.
pw_status ortho_block(pw_ham* h, int64_t nb, cplx* y, int64_t ld, cplx* hy, int64_t ldhy, int op,
                      pw_prec gram_prec, cplx* cp) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  pw_status st;
  if (gram_prec != PW_FP64) {
    {
      StageScope sc(c, PW_STAGE_GRAM);
      HIPCHK(c, launch_block_to_f32(h->npw, nb, y, ld, h->blk32[0], h->npw, s));
      HIPCHK(c, launch_gemm_cn32(gram_prec == PW_BF16, nb, nb, h->npw, 1.0, h->blk32[0], h->npw,
                                 h->blk32[0], h->npw, h->gram32, nb, nullptr, h->work32, s, nullptr,
                                 h->gemm_target));
      HIPCHK(c, launch_block_to_f64(nb, nb, h->gram32, nb, h->sub0, nb, s));
      HIPCHK(c, launch_hermitize(nb, h->sub0, nb, s));
    }
    if ((st = chol_and_solve(h, nb, y, ld, hy, ldhy, op, cp)) != PW_OK) return st;
  }
  {
    StageScope sc(c, PW_STAGE_GRAM);
    // Hermitian: the tiles on and above the diagonal, then mirrored
    HIPCHK(c, launch_gemm_cn(nb, nb, h->npw, 1.0, y, ld, y, ld, h->sub0, nb, nullptr, h->gemm_work, s,
                             0.0, nullptr, 2048, 1));
    HIPCHK(c, launch_hermitize(nb, h->sub0, nb, s));
  }
  return chol_and_solve(h, nb, y, ld, hy, ldhy, op, cp);
}

// The subspace part of Rayleigh-Ritz for Y orthonormal and W = H Y given:
// Hs = Y^H W (Hermitian part), Hs = Q diag(eig) Q^H, Y <- Y Q, W <- W Q,
// resid_b = ||W_b - eig_b Y_b|| (if resid); eigensolver status deferred.
pw_status subspace_rr(pw_ham* h, int64_t nb, cplx* y, int64_t ld, cplx* hy, int64_t ldhy, double* eig,
                      double* resid, int op, cplx* cp) {
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  {
    StageScope sc(c, PW_STAGE_GRAM);
    HIPCHK(c, launch_gemm_cn(nb, nb, h->npw, 1.0, y, ld, hy, ldhy, h->sub0, nb, nullptr,
                             h->gemm_work, s, 0.0, nullptr, 2048, 1));
    HIPCHK(c, launch_hermitize(nb, h->sub0, nb, s));
  }
  {
    StageScope sc(c, PW_STAGE_EIGH);
    HIPCHK(c, launch_heev_async(nb, h->sub0, nb, eig, h->sub1, nb, h->heev_work, sweeps_slot(c),
                                c->max_sweeps, s));
    HIPCHK(c, launch_status_record(nullptr, sweeps_slot(c), op, c->rec_dev, s));
  }
  if (cp && h->nproj > 0) {
    // projections kept in memory: (P^H Y) Q = P^H (Y Q), an nproj x nb x nb product
    StageScope sc(c, PW_STAGE_ROTATE);
    HIPCHK(c, launch_gemm_nn(h->nproj, nb, nb, 1.0, cp, h->nproj, h->sub1, nb, 0.0, h->cprj, h->nproj,
                             s, 0));
    HIPCHK(c, launch_copy_block(h->nproj, nb, h->cprj, h->nproj, cp, h->nproj, s));
  }
  pw_status st;
  if ((st = rotate_block(h, nb, y, ld, h->sub1)) != PW_OK) return st;
  if ((st = rotate_block(h, nb, hy, ldhy, h->sub1)) != PW_OK) return st;
  if (resid) {
    StageScope sc(c, PW_STAGE_MISC);
    HIPCHK(c, launch_residuals(h->npw, nb, hy, ldhy, y, ld, eig, resid, s));
  }
  return PW_OK;
}

// Runs the hot-path helpers of one context on another stream (untimed while
// a graph is being captured).
struct StreamSwap {
  pw_ctx* c;
  hipStream_t old;
  bool timing;
  StreamSwap(pw_ctx* ctx, hipStream_t s, bool untimed)
      : c(ctx), old(ctx->stream), timing(ctx->timing) {
    c->stream = s;
    if (untimed) c->timing = false;
  }
  ~StreamSwap() {
    c->stream = old;
    c->timing = timing;
  }
};

// Chebyshev filter of one batch item with coefficients formed on the device
// from its Ritz values; the first product reuses W = H Y.
pw_status batch_filter(pw_batch* b, BatchItem& it) {
  pw_ham* h = it.h;
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  const int64_t nb = it.nb, npw = h->npw;
  const int m = b->degree;
  HIPCHK(c, launch_cheb_coef(it.eig, (int)nb, it.upper, m, it.coef, it.flags + 2, s));
  pw_status st;
  if (b->prec != PW_FP64) {
    const int bf16 = b->prec == PW_BF16;
    float2* buf[2] = {h->blk32[0], h->blk32[1]};
    HIPCHK(c, launch_block_to_f32(npw, nb, it.y, npw, buf[0], npw, s));
    HIPCHK(c, launch_axpby_to_f32(npw, nb, 0.0, it.hy, npw, 0.0, it.y, npw, buf[1], npw, s, it.coef));
    for (int i = 2; i <= m; ++i) {
      const int cur = (i - 1) & 1, nxt = i & 1;
      if ((st = ham_apply32(h, bf16, nb, buf[cur], npw, buf[nxt], npw, 0.0, 0.0, 0.0, buf[nxt], npw,
                            it.coef + 3 * (i - 1))) != PW_OK)
        return st;
    }
    HIPCHK(c, launch_block_to_f64(npw, nb, buf[m & 1], npw, it.y, npw, s));
    return PW_OK;
  }
  cplx* buf[2] = {it.y, h->blk};
  HIPCHK(c, launch_axpby_block(npw, nb, 0.0, it.hy, npw, 0.0, it.y, npw, h->blk, npw, s, it.coef));
  for (int i = 2; i <= m; ++i) {
    const int cur = (i - 1) & 1, nxt = i & 1;
    if ((st = ham_apply(h, nb, buf[cur], npw, buf[nxt], npw, 0.0, 0.0, 0.0, buf[nxt], npw,
                        it.coef + 3 * (i - 1))) != PW_OK)
      return st;
  }
  if (m & 1) HIPCHK(c, launch_copy_block(npw, nb, h->blk, npw, it.y, npw, s));
  return PW_OK;
}

// Cholesky orthonormalisation then Rayleigh-Ritz of one batch item, with no
// host synchronisation (one-workgroup eigensolve, failures go to its flags).
pw_status batch_ortho_rr(BatchItem& it) {
  pw_ham* h = it.h;
  pw_ctx* c = h->ctx;
  hipStream_t s = c->stream;
  const int64_t nb = it.nb, npw = h->npw;
  HIPCHK(c, launch_gemm_cn(nb, nb, npw, 1.0, it.y, npw, it.y, npw, h->sub0, nb, nullptr,
                           h->gemm_work, s, 0.0, nullptr, 2048, 1));
  HIPCHK(c, launch_hermitize(nb, h->sub0, nb, s));
  HIPCHK(c, chol_blocked(nb, h->sub0, nb, h->dinv, h->panel, h->dtol, h->status_dev, s));
  HIPCHK(c, trsm_right(npw, nb, it.y, npw, h->sub0, nb, h->dinv, h->blk, s));
  pw_status st = ham_apply(h, nb, it.y, npw, it.hy, npw, 1.0, 0.0, 0.0, nullptr, 0);
  if (st != PW_OK) return st;
  HIPCHK(c, launch_gemm_cn(nb, nb, npw, 1.0, it.y, npw, it.hy, npw, h->sub0, nb, nullptr,
                           h->gemm_work, s, 0.0, nullptr, 2048, 1));
  HIPCHK(c, launch_hermitize(nb, h->sub0, nb, s));
  HIPCHK(c, launch_heev_small_async(nb, h->sub0, nb, it.eig, h->sub1, nb, it.sweeps, s));
  if ((st = rotate_block(h, nb, it.y, npw, h->sub1)) != PW_OK) return st;
  if ((st = rotate_block(h, nb, it.hy, npw, h->sub1)) != PW_OK) return st;
  HIPCHK(c, launch_residuals(npw, nb, it.hy, npw, it.y, npw, it.eig, it.resid, s));
  HIPCHK(c, launch_batch_flags(h->status_dev, it.sweeps, it.flags, s));
  return PW_OK;
}

// One iteration of every item, forked from s0 over the batch streams and
// joined back (also the body of the captured graph).
// The items of branch stream k, one after another, on that stream.
pw_status batch_issue_stream(pw_batch* b, size_t k, bool filter, bool capturing) {
  pw_ctx* c = b->ctx;
  for (BatchItem& it : b->items) {
    if ((size_t)it.stream != k) continue;
    StreamSwap sw(c, b->streams[k], capturing);
    pw_status st;
    if (filter && (st = batch_filter(b, it)) != PW_OK) return st;
    if ((st = batch_ortho_rr(it)) != PW_OK) return st;
  }
  return PW_OK;
}

pw_status batch_fork(pw_batch* b) {
  pw_ctx* c = b->ctx;
  HIPCHK(c, hipEventRecord(b->ev[2], b->s0));
  for (hipStream_t st : b->streams) HIPCHK(c, hipStreamWaitEvent(st, b->ev[2], 0));
  return PW_OK;
}

pw_status batch_join(pw_batch* b) {
  pw_ctx* c = b->ctx;
  for (size_t k = 0; k < b->streams.size(); ++k) {
    HIPCHK(c, hipEventRecord(b->ev[3 + k], b->streams[k]));
    HIPCHK(c, hipStreamWaitEvent(b->s0, b->ev[3 + k], 0));
  }
  return PW_OK;
}

// One iteration of every item, forked from s0 over the batch streams and
// joined back (also the body of the single captured graph).
pw_status batch_issue(pw_batch* b, bool filter, bool capturing) {
  pw_status st;
  if ((st = batch_fork(b)) != PW_OK) return st;
  for (size_t k = 0; k < b->streams.size(); ++k)
    if ((st = batch_issue_stream(b, k, filter, capturing)) != PW_OK) return st;
  return batch_join(b);
}

// ---- fused mode: items grouped by box, every stage one launch per group ----
// Builds the groups and their device descriptors (once).
pw_status fused_setup(pw_batch* b) {
  pw_ctx* c = b->ctx;
  if (!b->groups.empty()) return PW_OK;
  std::map<std::vector<int>, std::vector<int>> bybox;
  for (size_t i = 0; i < b->items.size(); ++i) {
    const pw_ham* h = b->items[i].h;
    if (h->chunk_alloc < b->items[i].nb)
      return fail(c, PW_ERR_UNSUPPORTED,
                  "fused batch: item " + std::to_string(i) + " FFT buffer holds fewer than nb bands");
    // items share a group when they use the same FFT kernels (register
    // kernels are compiled per length; the generic ones take any box)
    const bool rc = h->reg_col_ok, rp = h->reg_plane_ok;
    bybox[{rc ? h->plan.n3 : -1, rp ? h->plan.n1 : -1, rp ? h->plan.n2 : -1}].push_back((int)i);
  }
  for (auto& kv : bybox) {
    pw_batch::Group g;
    const std::vector<int>& ids = kv.second;
    const pw_ham* h0 = b->items[ids[0]].h;
    FusedFft& f = g.f;
    f.n1 = h0->plan.n1;
    f.n2 = h0->plan.n2;
    f.n3 = h0->plan.n3;
    f.nitems = (int)ids.size();
    f.reg_col = h0->reg_col_ok;
    f.reg_plane = h0->reg_plane_ok;
    f.plane_variant = 0;
    f.plane_variant32 = 0;
    f.col_lds = 0;
    f.plane_lds = 0;
    f.col_blocks = 0;
    f.nb_max = f.ncols_max = f.xr_max = f.n3_max = 0;
    for (int i : ids) {
      const pw_ham* h = b->items[i].h;
      f.nb_max = std::max<int>(f.nb_max, (int)b->items[i].nb);
      f.ncols_max = std::max(f.ncols_max, h->plan.ncols);
      f.xr_max = std::max(f.xr_max, h->plan.xr);
      f.n3_max = std::max(f.n3_max, h->plan.n3);
      f.col_blocks = std::max(f.col_blocks, (h->plan.ncols + h->cfg.col_tile - 1) / h->cfg.col_tile);
      f.col_lds = std::max(f.col_lds, h->cfg.col_lds);
      f.plane_lds = std::max(f.plane_lds, h->cfg.plane_lds);
      g.nproj_max = std::max<int>(g.nproj_max, (int)h->nproj);
      g.npw_max = std::max(g.npw_max, h->npw);
      g.npw_nb_max = std::max(g.npw_nb_max, h->npw * b->items[i].nb);
      g.nsplit_proj = std::max(g.nsplit_proj,
                               fused_cn_nsplit(GOP_PROJ, h->npw, b->items[i].nb, h->nproj,
                                               h->gemm_target));
      g.nsplit_gram = std::max(g.nsplit_gram,
                               fused_cn_nsplit(GOP_GRAM, h->npw, b->items[i].nb, h->nproj,
                                               h->gemm_target));
      if (b->prec != PW_FP64)
        g.nsplit_proj32 = std::max(g.nsplit_proj32,
                                   fused_cn32_nsplit(b->prec == PW_BF16, h->npw, b->items[i].nb,
                                                     h->nproj, h->gemm_target));
    }
    g.nitems = f.nitems;
    g.nb_max = f.nb_max;
    std::vector<ItemDev> host(ids.size());
    for (size_t q = 0; q < ids.size(); ++q) {
      const BatchItem& it = b->items[ids[q]];
      const pw_ham* h = it.h;
      ItemDev& d = host[q];
      d.plan = h->plan;
      d.npw = (int)h->npw;
      d.nb = (int)it.nb;
      d.nproj = (int)h->nproj;
      d.gemm_target = h->gemm_target;
      d.col_tile = h->cfg.col_tile;
      d.plane_rows = h->cfg.plane_rows;
      d.y = it.y;
      d.hy = it.hy;
      d.blk = h->blk;
      d.b32[0] = h->blk32[0];
      d.b32[1] = h->blk32[1];
      d.T = h->T;
      d.T32 = h->T32;
      d.kin = h->kin;
      d.vs = h->vscaled;
      d.kin32 = h->kin32;
      d.vs32 = h->vs32;
      d.proj = h->proj;
      d.proj32 = h->proj32;
      d.proj3 = h->proj3;
      d.proj3c = h->proj3c;
      d.cprj3 = h->cprj3;
      d.ekb = h->ekb_dev;
      d.cprj = h->cprj;
      d.cprj32 = h->cprj32;
      d.gemm_work = h->gemm_work;
      d.work32 = h->work32;
      d.sub0 = h->sub0;
      d.sub1 = h->sub1;
      d.dinv = h->dinv;
      d.dtol = h->dtol;
      d.status = h->status_dev;
      d.eig = it.eig;
      d.resid = it.resid;
      d.coef = it.coef;
      d.upper = it.upper;
      d.flags = it.flags;
      d.sweeps = it.sweeps;
    }
    void* dev = nullptr;
    hipError_t e = hipMalloc(&dev, host.size() * sizeof(ItemDev));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, PW_ERR_OOM, "fused batch: descriptor allocation failed");
    }
    b->allocs.push_back(dev);
    HIPCHK(c, hipMemcpy(dev, host.data(), host.size() * sizeof(ItemDev), hipMemcpyHostToDevice));
    g.D = static_cast<ItemDev*>(dev);
    b->groups.push_back(g);
  }
  return PW_OK;
}

// One fused H application: out = alpha (H in) + beta in + gamma prev.
pw_status fused_apply(pw_ctx* c, const pw_batch::Group& g, int prec, int in, int out, int prev,
                      double alpha, double beta, double gamma, int coef_step, hipStream_t s) {
  const bool lp = prec != PW_FP64;
  const int bf16 = prec == PW_BF16;
  const int lps = lp ? PW_STAGE_FFT_COL_INV_LP - PW_STAGE_FFT_COL_INV : 0;
  if (g.nproj_max > 0) {
    StageScope sc(c, PW_STAGE_PROJ + lps);
    if (lp)
      HIPCHK(c, launch_fused_gemm_cn32(bf16, g.nitems, g.nproj_max, g.nb_max, g.nsplit_proj32, g.D,
                                       in, alpha, coef_step, s));
    else
      HIPCHK(c, launch_fused_gemm_cn(g.nitems, g.nproj_max, g.nb_max, g.nsplit_proj, g.D, GOP_PROJ,
                                     in, alpha, coef_step, s));
  }
  {
    StageScope sc(c, PW_STAGE_FFT_COL_INV + lps);
    HIPCHK(c, launch_fused_col_inv(g.f, lp, g.D, in, s));
  }
  {
    StageScope sc(c, PW_STAGE_FFT_PLANE + lps);
    HIPCHK(c, launch_fused_plane(g.f, lp, g.D, s));
  }
  {
    StageScope sc(c, PW_STAGE_FFT_COL_FWD + lps);
    HIPCHK(c, launch_fused_col_fwd(g.f, lp, g.D, in, out, prev, alpha, beta, gamma, coef_step, s));
  }
  if (g.nproj_max > 0) {
    StageScope sc(c, PW_STAGE_NONLOCAL + lps);
    if (lp) HIPCHK(c, launch_fused_gemm_nn32(bf16, g.nitems, g.npw_max, g.nb_max, g.D, out, s));
    else HIPCHK(c, launch_fused_gemm_nn(g.nitems, g.npw_max, g.nb_max, g.D, GOP_NONLOCAL, 0, out, s));
  }
  return PW_OK;
}

// One iteration (filter, Cholesky, Rayleigh-Ritz) of every item of a group.
pw_status fused_iteration(pw_batch* b, const pw_batch::Group& g, hipStream_t s) {
  pw_ctx* c = b->ctx;
  const int m = b->degree;
  const int64_t ew = g.npw_nb_max;
  pw_status st;
  HIPCHK(c, launch_fused_dense(FS_CHEB_COEF, g.nitems, ew, g.nb_max, g.D, m, 0, s));
  if (b->prec == PW_FP64) {
    const int buf[2] = {SEL_Y, SEL_BLK};
    HIPCHK(c, launch_fused_dense(FS_FILTER_FIRST, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
    for (int i = 2; i <= m; ++i) {
      const int cur = buf[(i - 1) & 1], nxt = buf[i & 1];
      if ((st = fused_apply(c, g, PW_FP64, cur, nxt, nxt, 0.0, 0.0, 0.0, i - 1, s)) != PW_OK)
        return st;
    }
    if (m & 1) HIPCHK(c, launch_fused_dense(FS_COPY, g.nitems, ew, g.nb_max, g.D, SEL_BLK, SEL_Y, s));
  } else {
    const int buf[2] = {SEL_B32A, SEL_B32B};
    HIPCHK(c, launch_fused_dense(FS_TO_F32, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
    HIPCHK(c, launch_fused_dense(FS_FILTER_FIRST, g.nitems, ew, g.nb_max, g.D, 1, 0, s));
    for (int i = 2; i <= m; ++i) {
      const int cur = buf[(i - 1) & 1], nxt = buf[i & 1];
      if ((st = fused_apply(c, g, b->prec, cur, nxt, nxt, 0.0, 0.0, 0.0, i - 1, s)) != PW_OK)
        return st;
    }
    HIPCHK(c, launch_fused_dense(FS_TO_F64, g.nitems, ew, g.nb_max, g.D, buf[m & 1], 0, s));
  }
  // Cholesky orthonormalisation (one diagonal block: nb <= 64)
  {
    StageScope sc(c, PW_STAGE_GRAM);
    HIPCHK(c, launch_fused_gemm_cn(g.nitems, g.nb_max, g.nb_max, g.nsplit_gram, g.D, GOP_GRAM, SEL_Y,
                                   1.0, -1, s));
    HIPCHK(c, launch_fused_dense(FS_HERMITIZE, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
  }
  {
    StageScope sc(c, PW_STAGE_CHOL);
    HIPCHK(c, launch_fused_dense(FS_CHOL_INIT, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
    HIPCHK(c, launch_fused_dense(FS_CHOL_DIAG, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
  }
  {
    StageScope sc(c, PW_STAGE_ROTATE);
    HIPCHK(c, launch_fused_gemm_nn(g.nitems, g.npw_max, g.nb_max, g.D, GOP_TRSM, 0, 0, s));
    HIPCHK(c, launch_fused_dense(FS_COPY, g.nitems, ew, g.nb_max, g.D, SEL_BLK, SEL_Y, s));
  }
  // Rayleigh-Ritz, FP64
  if ((st = fused_apply(c, g, PW_FP64, SEL_Y, SEL_HY, SEL_NONE, 1.0, 0.0, 0.0, -1, s)) != PW_OK)
    return st;
  {
    StageScope sc(c, PW_STAGE_GRAM);
    HIPCHK(c, launch_fused_gemm_cn(g.nitems, g.nb_max, g.nb_max, g.nsplit_gram, g.D, GOP_GRAM, SEL_HY,
                                   1.0, -1, s));
    HIPCHK(c, launch_fused_dense(FS_HERMITIZE, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
  }
  {
    StageScope sc(c, PW_STAGE_EIGH);
    HIPCHK(c, launch_fused_dense(FS_JACOBI, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
  }
  {
    StageScope sc(c, PW_STAGE_ROTATE);
    HIPCHK(c, launch_fused_gemm_nn(g.nitems, g.npw_max, g.nb_max, g.D, GOP_ROT, SEL_Y, 0, s));
    HIPCHK(c, launch_fused_dense(FS_COPY, g.nitems, ew, g.nb_max, g.D, SEL_BLK, SEL_Y, s));
    HIPCHK(c, launch_fused_gemm_nn(g.nitems, g.npw_max, g.nb_max, g.D, GOP_ROT, SEL_HY, 0, s));
    HIPCHK(c, launch_fused_dense(FS_COPY, g.nitems, ew, g.nb_max, g.D, SEL_BLK, SEL_HY, s));
  }
  {
    StageScope sc(c, PW_STAGE_MISC);
    HIPCHK(c, launch_fused_dense(FS_RESIDUALS, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
    HIPCHK(c, launch_fused_dense(FS_FLAGS, g.nitems, ew, g.nb_max, g.D, 0, 0, s));
  }
  return PW_OK;
}

// All groups, forked over the batch streams and joined back.
// With stage timing on and not capturing, every stage is bracketed by HIP
// events on its group's stream.
pw_status fused_issue(pw_batch* b, bool capturing) {
  pw_status st;
  if ((st = batch_fork(b)) != PW_OK) return st;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    hipStream_t gs = b->streams[gi % b->streams.size()];
    StreamSwap sw(b->ctx, gs, capturing);
    if ((st = fused_iteration(b, b->groups[gi], gs)) != PW_OK) return st;
  }
  return batch_join(b);
}

// Reads the flags of all items (synchronises s0) and reports the first failure.
pw_status batch_check(pw_batch* b) {
  pw_ctx* c = b->ctx;
  const size_t bytes = 4 * b->items.size() * sizeof(int);
  HIPCHK(c, hipMemcpyAsync(b->flags_host, b->flags_dev, bytes, hipMemcpyDeviceToHost, b->s0));
  HIPCHK(c, hipStreamSynchronize(b->s0));
  b->max_sweeps = 0;
  for (size_t i = 0; i < b->items.size(); ++i) {
    const int* f = b->flags_host + 4 * i;
    b->max_sweeps = std::max(b->max_sweeps, f[3]);
    const std::string who = "batch item " + std::to_string(i) + ": ";
    if (f[0] > 0)
      return fail(c, PW_ERR_NOT_POSDEF,
                  who + "Gram matrix not positive definite at pivot " + std::to_string(f[0] - 1));
    if (f[0] < 0)
      return fail(c, PW_ERR_NONFINITE,
                  who + "column " + std::to_string(-f[0] - 1) + " of the block is NaN or infinite");
    if (f[1]) return fail(c, PW_ERR_NO_CONVERGENCE, who + "Jacobi eigensolver hit its sweep limit");
    if (f[2])
      return fail(c, PW_ERR_INVALID_ARG,
                  who + "Ritz values outside a0 < a < b; the filter was skipped");
  }
  return PW_OK;
}

// Orders s0 after the context stream and clears the flags.
pw_status batch_enter(pw_batch* b) {
  pw_ctx* c = b->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipEventRecord(b->ev[0], c->stream));
  HIPCHK(c, hipStreamWaitEvent(b->s0, b->ev[0], 0));
  HIPCHK(c, hipMemsetAsync(b->flags_dev, 0, 4 * b->items.size() * sizeof(int), b->s0));
  return PW_OK;
}
// Orders the context stream after s0 and checks the flags.
pw_status batch_leave(pw_batch* b) {
  pw_ctx* c = b->ctx;
  HIPCHK(c, hipEventRecord(b->ev[1], b->s0));
  HIPCHK(c, hipStreamWaitEvent(c->stream, b->ev[1], 0));
  return batch_check(b);
}
struct EventGuard {
  hipEvent_t e = nullptr;
  ~EventGuard() {
    if (e) (void)hipEventDestroy(e);
  }
};

// Median time of one H application of nb bands under the handle's current
// tuning (one untimed warm-up).
// Relative margin by which an autotuning candidate must beat the current choice.
constexpr double kTuneMargin = 0.01;

pw_status time_apply(pw_ham* h, pw_prec prec, int64_t nb, void* in, void* out, int reps, double* ms) {
  pw_ctx* c = h->ctx;
  EventGuard a, b;
  HIPCHK(c, hipEventCreate(&a.e));
  HIPCHK(c, hipEventCreate(&b.e));
  std::vector<double> v;
  for (int r = -1; r < reps; ++r) {
    HIPCHK(c, hipEventRecord(a.e, c->stream));
    pw_status st =
        prec == PW_FP64
            ? ham_apply(h, nb, static_cast<const cplx*>(in), h->npw, static_cast<cplx*>(out), h->npw,
                        1.0, 0.0, 0.0, nullptr, 0)
        : prec == PW_BF16
            ? ham_apply16(h, nb, static_cast<const bf16c*>(in), h->npw, static_cast<bf16c*>(out),
                          h->npw, 1.0, 0.0, 0.0, nullptr, 0)
            : ham_apply32(h, 0, nb, static_cast<const float2*>(in), h->npw,
                          static_cast<float2*>(out), h->npw, 1.0, 0.0, 0.0, nullptr, 0);
    if (st != PW_OK) return st;
    HIPCHK(c, hipEventRecord(b.e, c->stream));
    HIPCHK(c, hipEventSynchronize(b.e));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, a.e, b.e));
    if (r >= 0) v.push_back(t);
  }
  std::sort(v.begin(), v.end());
  *ms = v[v.size() / 2];
  return PW_OK;
}
}  // namespace pwi
using namespace pwi;

extern "C" {

const char* pw_status_string(pw_status s) {
  switch (s) {
    case PW_OK: return "PW_OK";
    case PW_ERR_INVALID_ARG: return "PW_ERR_INVALID_ARG";
    case PW_ERR_UNSUPPORTED: return "PW_ERR_UNSUPPORTED";
    case PW_ERR_HIP: return "PW_ERR_HIP";
    case PW_ERR_OOM: return "PW_ERR_OOM";
    case PW_ERR_NOT_POSDEF: return "PW_ERR_NOT_POSDEF";
    case PW_ERR_NONFINITE: return "PW_ERR_NONFINITE";
    case PW_ERR_NO_CONVERGENCE: return "PW_ERR_NO_CONVERGENCE";
  }
  return "PW_ERR_UNKNOWN";
}

const char* pw_version(void) { return PW_VERSION; }

const char* pw_last_error(const pw_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

pw_status pw_ctx_create(int device, void* hip_stream, pw_ctx** out) {
  if (!out) return fail(nullptr, PW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (device < 0) return fail(nullptr, PW_ERR_INVALID_ARG, "device < 0");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device >= ndev)
    return fail(nullptr, PW_ERR_HIP,
                "no HIP device " + std::to_string(device) + " (" + hipGetErrorString(e) + ")");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, PW_ERR_HIP, hipGetErrorString(e));
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  if (e != hipSuccess) return fail(nullptr, PW_ERR_HIP, hipGetErrorString(e));
  pw_ctx* c = new pw_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->lds_limit = (size_t)lds;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cus > 0)
      c->cus = cus;
  }
  void* pin = nullptr;
  e = hipHostMalloc(&pin, 64 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, PW_ERR_OOM, "pinned host scratch allocation failed");
  }
  c->pinned = static_cast<double*>(pin);
  void* rec = nullptr;
  e = hipMalloc(&rec, 8 * sizeof(int));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(pin);
    delete c;
    return fail(nullptr, PW_ERR_OOM, "status word allocation failed");
  }
  c->rec_dev = static_cast<int*>(rec);
  c->home = c->stream;
  e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = scratch_address(device, &c->scratch);
  if (e == hipSuccess && heev_work_bytes(kScratchHeevMax) > kScratchBytes) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = launch_fill_int(8, 0, c->rec_dev, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = fft_set_lds_limits(c->lds_limit);
  if (e == hipSuccess) e = fft_reg_set_lds_limits(c->lds_limit);
  if (e == hipSuccess) e = heev_set_lds_limit(c->lds_limit);
  if (e == hipSuccess) e = fft_ls_set_lds_limit(c->lds_limit);
  if (e == hipSuccess) e = density_set_lds_limit(c->lds_limit);
  if (e != hipSuccess) {
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    (void)hipFree(rec);
    (void)hipHostFree(pin);
    delete c;
    return fail(nullptr, PW_ERR_HIP, std::string("context set-up: ") + hipGetErrorString(e));
  }
  *out = c;
  return PW_OK;
}

namespace {
// Frees the context once the caller's handle and every ham / batch made on
// it are gone, whatever order they are destroyed in.
void ctx_release(pw_ctx* ctx) {
  if (--ctx->refs > 0) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->rec_dev) (void)hipFree(ctx->rec_dev);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  delete ctx;
}
}  // namespace

pw_status pw_ctx_destroy(pw_ctx* ctx) {
  if (!ctx) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  ctx_release(ctx);
  return PW_OK;
}

pw_status pw_ham_create(pw_ctx* ctx, const pw_ham_desc* d, pw_ham** out) {
  if (!ctx) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (!d || !out) return fail(ctx, PW_ERR_INVALID_ARG, "desc or out is NULL");
  *out = nullptr;
  if (d->npw <= 0 || d->npw > (int64_t)INT32_MAX)
    return fail(ctx, PW_ERR_INVALID_ARG, "npw must be in [1, 2^31)");
  if (!d->miller) return fail(ctx, PW_ERR_INVALID_ARG, "miller is NULL");
  if (!d->vloc_dev) return fail(ctx, PW_ERR_INVALID_ARG, "vloc_dev is NULL");
  if (d->nproj < 0) return fail(ctx, PW_ERR_INVALID_ARG, "nproj < 0");
  if (d->nproj > 0 && (!d->proj_dev || !d->ekb))
    return fail(ctx, PW_ERR_INVALID_ARG, "nproj > 0 needs proj_dev and ekb");
  if (d->nb_max < 1 || d->nb_max > 4096)
    return fail(ctx, PW_ERR_INVALID_ARG, "nb_max must be in [1, 4096]");
  for (int i = 0; i < 3; ++i)
    if (d->n[i] < 1 || d->n[i] > 4096)
      return fail(ctx, PW_ERR_INVALID_ARG, "box dimensions must be in [1, 4096]");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(d->recip[i])) return fail(ctx, PW_ERR_INVALID_ARG, "recip not finite");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(d->kpt[i])) return fail(ctx, PW_ERR_INVALID_ARG, "kpt not finite");
  for (int64_t j = 0; j < d->nproj; ++j)
    if (!std::isfinite(d->ekb[j])) return fail(ctx, PW_ERR_INVALID_ARG, "ekb not finite");
  HIPCHK(ctx, hipSetDevice(ctx->device));

  pw_ham* h = new pw_ham();
  h->ctx = ctx;
  h->npw = d->npw;
  h->nproj = d->nproj;
  h->nb_max = d->nb_max;
  BoxPlan& P = h->plan;
  P.n1 = d->n[0];
  P.n2 = d->n[1];
  P.n3 = d->n[2];
  P.npw = d->npw;
  if (!fft_factor(P.n1, &P.ax1) || !fft_factor(P.n2, &P.ax2) || !fft_factor(P.n3, &P.ax3)) {
    delete h;
    return fail(ctx, PW_ERR_UNSUPPORTED,
                "box sizes must factor into radices 2, 3, 4, 5, 8 with n/radix <= 256");
  }
  // ---- sphere -> box maps (host) ----
  const int64_t npw = d->npw;
  pwplan::HostPlan hp;
  int64_t bad_point = -1;
  const int prc = pwplan::build_host_plan(d->miller, d->npw, P.n1, P.n2, P.n3, &hp, &bad_point);
  if (prc != 0) {
    delete h;
    if (prc == 1)
      return fail(ctx, PW_ERR_INVALID_ARG,
                  "two sphere points fall in the same box cell (box too small), point " +
                      std::to_string(bad_point));
    return fail(ctx, PW_ERR_INVALID_ARG, "sphere -> box map arguments out of range");
  }
  P.ncols = hp.ncols;
  P.ldt = hp.ldt;
  P.xr = hp.xr;
  P.quarter12 = hp.quarter12;
  P.runs = hp.runs;

  pw_status st = PW_OK;
  auto upload_int = [&](int** dst, const std::vector<int>& v) -> pw_status {
    pw_status s2 = dalloc(h, dst, v.size());
    if (s2 != PW_OK) return s2;
    hipError_t e = hipMemcpy(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(ctx, PW_ERR_HIP, hipGetErrorString(e));
    return PW_OK;
  };
#define TRY(x)         \
  do {                 \
    st = (x);          \
    if (st != PW_OK) { \
      free_ham(h);     \
      delete h;        \
      return st;       \
    }                  \
  } while (0)
  TRY(upload_int(&P.col_start, hp.col_start));
  TRY(upload_int(&P.col_e, hp.col_e));
  TRY(upload_int(&P.col_m2, hp.col_m2));
  TRY(upload_int(&P.pt_perm, hp.pt_perm));
  TRY(upload_int(&P.pt_col, hp.pt_col));
  TRY(upload_int(&P.pt_m3, hp.pt_m3));
  TRY(upload_int(&P.col_m3lo, hp.col_m3lo));
  TRY(upload_int(&P.ext_m1, hp.ext_m1));
  // twiddles
  FftAxis* axes[3] = {&P.ax1, &P.ax2, &P.ax3};
  for (FftAxis* ax : axes) {
    std::vector<cplx> tw;
    fft_host_twiddles(ax->n, &tw);
    cplx* dtw = nullptr;
    TRY(dalloc(h, &dtw, tw.size()));
    if (hipMemcpy(dtw, tw.data(), tw.size() * sizeof(cplx), hipMemcpyHostToDevice) != hipSuccess)
      TRY(fail(ctx, PW_ERR_HIP, "twiddle upload failed"));
    ax->tw = dtw;
  }
  if (!fft_choose_config(P, ctx->lds_limit, &h->cfg)) {
    free_ham(h);
    delete h;
    return fail(ctx, PW_ERR_UNSUPPORTED,
                "the plane working set (extent x N2) does not fit this GPU's LDS");
  }
  hipStream_t s = ctx->stream;
  // kinetic energies from the Miller indices
  {
    int* dm = nullptr;
    std::vector<int> mil(d->miller, d->miller + 3 * npw);
    TRY(upload_int(&dm, mil));
    TRY(dalloc(h, &h->kin, (size_t)npw));
    HIPCHK(ctx, launch_kinetic(npw, dm, d->recip, d->kpt, h->kin, s));
  }
  {
    const double* B = d->recip;
    const double det = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
                       B[2] * (B[3] * B[7] - B[4] * B[6]);
    const double two_pi = 6.283185307179586476925286766559;
    h->omega = det != 0.0 ? two_pi * two_pi * two_pi / std::fabs(det) : 0.0;
  }
  // V scaled by 1/N_box; maxima for the spectral bound
  const int64_t nbox = (int64_t)P.n1 * P.n2 * P.n3;
  TRY(dalloc(h, &h->vscaled, (size_t)nbox));
  double* dmax = nullptr;
  TRY(dalloc(h, &dmax, 2));
  HIPCHK(ctx, launch_max_reduce(nbox, d->vloc_dev, dmax, s));
  HIPCHK(ctx, launch_max_reduce(npw, h->kin, dmax + 1, s));
  HIPCHK(ctx, launch_scale_copy(nbox, d->vloc_dev, 1.0 / (double)nbox, h->vscaled, s));
  {
    int* flag = nullptr;
    TRY(dalloc(h, &flag, 1));
    HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int), s));
    HIPCHK(ctx, launch_check_finite(nbox, d->vloc_dev, flag, s));
    int hflag = 0;
    HIPCHK(ctx, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    double hm[2];
    HIPCHK(ctx, hipMemcpyAsync(hm, dmax, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (hflag) TRY(fail(ctx, PW_ERR_NONFINITE, "vloc contains NaN or Inf"));
    h->vmax = hm[0];
    h->kmax = hm[1];
  }
  // projectors
  h->proj = static_cast<const cplx*>(d->proj_dev);
  if (h->nproj > 0) {
    h->ekb.assign(d->ekb, d->ekb + h->nproj);
    TRY(dalloc(h, &h->ekb_dev, (size_t)h->nproj));
    HIPCHK(ctx, hipMemcpy(h->ekb_dev, h->ekb.data(), h->nproj * sizeof(double),
                          hipMemcpyHostToDevice));
  }
  // workspaces
  const size_t per_band = (size_t)P.n3 * P.ldt;
  const size_t budget = (size_t)512 << 20;
  h->chunk = std::max<int64_t>(1, std::min<int64_t>(h->nb_max, budget / (per_band * sizeof(cplx))));
  h->chunk_alloc = h->chunk;
  h->reg_col_ok = h->cfg.reg_col;
  h->reg_plane_ok = h->cfg.reg_plane;
  h->narrow_ok = h->cfg.reg_plane && fft_reg_plane_narrow(P, false);
  h->narrow32_ok = h->cfg.reg_plane && fft_reg_plane_narrow(P, true);
  h->ls32_ok = h->cfg.reg_plane && fft_plane_ls_supported(P, ctx->lds_limit);
  if (h->ls32_ok) h->cfg.plane_variant32 = 2;   // the faster FP32 plane kernel where it applies
  TRY(dalloc(h, &h->T, per_band * h->chunk));
  if (h->nproj > 0) {
    TRY(dalloc(h, &h->cprj, (size_t)(h->nproj * h->nb_max)));
    TRY(dalloc(h, &h->cprj_y, (size_t)(h->nproj * h->nb_max)));
  }
  size_t wmax = 0;
  for (int64_t nb = 1; nb <= h->nb_max; ++nb) {
    if (h->nproj > 0) wmax = std::max(wmax, gemm_cn_work_elems(h->nproj, nb, npw));
    wmax = std::max(wmax, gemm_cn_work_elems(nb, nb, npw));
  }
  TRY(dalloc(h, &h->gemm_work, std::max<size_t>(wmax, 1)));
  TRY(dalloc(h, &h->blk, (size_t)(npw * h->nb_max)));
  TRY(dalloc(h, &h->sub0, (size_t)(h->nb_max * h->nb_max)));
  TRY(dalloc(h, &h->sub1, (size_t)(h->nb_max * h->nb_max)));
  {
    char* hw = nullptr;
    TRY(dalloc(h, &hw, heev_work_bytes(h->nb_max)));
    h->heev_work = hw;
  }
  TRY(dalloc(h, &h->status_dev, 16));
  TRY(dalloc(h, &h->dinv, (size_t)((h->nb_max + kCholBlock) * kCholBlock)));
  TRY(dalloc(h, &h->panel, (size_t)(kCholBlock * h->nb_max)));
  TRY(dalloc(h, &h->dtol, 2));
  // FP32 twiddle tables (all axes)
  for (FftAxis* ax : axes) {
    float2* t32 = nullptr;
    TRY(dalloc(h, &t32, (size_t)ax->n));
    HIPCHK(ctx, launch_tw_to_f32(ax->n, ax->tw, t32, s));
    ax->tw32 = t32;
  }
  if (d->low_prec) {
    h->low_prec = true;
    TRY(dalloc(h, &h->kin32, (size_t)npw));
    TRY(dalloc(h, &h->vs32, (size_t)nbox));
    HIPCHK(ctx, launch_real_to_f32(npw, h->kin, 1.0, h->kin32, s));
    HIPCHK(ctx, launch_real_to_f32(nbox, h->vscaled, 1.0, h->vs32, s));
    if (h->nproj > 0) {
      TRY(dalloc(h, &h->proj32, (size_t)(npw * h->nproj)));
      HIPCHK(ctx, launch_block_to_f32(npw, h->nproj, h->proj, npw, h->proj32, npw, s));
      TRY(dalloc(h, &h->proj3, split3_elems(npw, h->nproj)));
      HIPCHK(ctx, launch_split3(npw, h->nproj, h->proj32, 1, npw, h->proj3, s));
      TRY(dalloc(h, &h->proj3c, split3_elems(h->nproj, npw)));
      HIPCHK(ctx, launch_split3(h->nproj, npw, h->proj32, npw, 1, h->proj3c, s));
      TRY(dalloc(h, &h->cprj32, (size_t)(h->nproj * h->nb_max)));
      // the reduction writes the entries of the nb bands it forms: the
      // projector padding stays zero, and rows of bands past a call's nb
      // (zero, or an earlier call's values) reach only columns not stored
      const size_t n3 = split3_elems(h->nb_max, h->nproj);
      TRY(dalloc(h, &h->cprj3, n3));
      HIPCHK(ctx, hipMemsetAsync(h->cprj3, 0, n3 * sizeof(uint16_t), s));
    }
    {
      // split-K partials of the FP32 / BF16 projections and Gram matrices
      size_t w32 = 1;
      for (int64_t nb = 1; nb <= h->nb_max; ++nb)
        for (int bf = 0; bf < 2; ++bf) {
          if (h->nproj > 0) w32 = std::max(w32, gemm_cn32_work_elems(h->nproj, nb, npw, bf));
          w32 = std::max(w32, gemm_cn32_work_elems(nb, nb, npw, bf));
        }
      TRY(dalloc(h, &h->work32, w32));
      TRY(dalloc(h, &h->gram32, (size_t)(h->nb_max * h->nb_max)));
    }
    const size_t per_band32 = (size_t)P.n3 * P.ldt;
    TRY(dalloc(h, &h->T32, per_band32 * h->chunk_alloc));
    TRY(dalloc(h, &h->blk32[0], (size_t)(npw * h->nb_max)));
    TRY(dalloc(h, &h->blk32[1], (size_t)(npw * h->nb_max)));
  }
  HIPCHK(ctx, hipStreamSynchronize(s));
#undef TRY
  ++ctx->refs;
  *out = h;
  return PW_OK;
}

pw_status pw_ham_destroy(pw_ham* h) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_ctx* c = h->ctx;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_ham(h);
  delete h;
  ctx_release(c);
  return PW_OK;
}

pw_status pw_ham_info(const pw_ham* h, int64_t* npw, int64_t* nproj, int64_t* nb_max,
                      int64_t* ncolumns, int64_t* extent1) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  if (npw) *npw = h->npw;
  if (nproj) *nproj = h->nproj;
  if (nb_max) *nb_max = h->nb_max;
  if (ncolumns) *ncolumns = h->plan.ncols;
  if (extent1) *extent1 = h->plan.xr;
  return PW_OK;
}

pw_status pw_apply_h(pw_ham* h, pw_prec prec, int64_t nb, const void* psi, int64_t ldpsi,
                     void* hpsi, int64_t ldh) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_status st;
  if ((st = check_hot(h, prec, nb)) != PW_OK) return st;
  if ((st = check_block(h, psi, ldpsi, "psi")) != PW_OK) return st;
  if ((st = check_block(h, hpsi, ldh, "hpsi")) != PW_OK) return st;
  const int64_t elem = prec == PW_FP64 ? (int64_t)sizeof(cplx)
                     : prec == PW_FP32 ? (int64_t)sizeof(float2)
                                       : (int64_t)sizeof(bf16c);
  if (ranges_overlap(psi, ldpsi, hpsi, ldh, h->npw, nb, elem))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "psi and hpsi overlap");
  HIPCHK(h->ctx, hipSetDevice(h->ctx->device));
  if (prec == PW_BF16)
    return ham_apply16(h, nb, static_cast<const bf16c*>(psi), ldpsi, static_cast<bf16c*>(hpsi), ldh,
                       1.0, 0.0, 0.0, nullptr, 0);
  if (prec == PW_FP32)
    return ham_apply32(h, 0, nb, static_cast<const float2*>(psi), ldpsi,
                       static_cast<float2*>(hpsi), ldh, 1.0, 0.0, 0.0, nullptr, 0);
  return ham_apply(h, nb, static_cast<const cplx*>(psi), ldpsi, static_cast<cplx*>(hpsi), ldh, 1.0,
                   0.0, 0.0, nullptr, 0);
}

pw_status pw_density(pw_ham* h, int64_t nb, const void* psi, int64_t ldpsi, const double* w,
                     double* rho, int32_t accumulate) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_ctx* c = h->ctx;
  if (nb < 0 || nb > h->nb_max)
    return fail(c, PW_ERR_INVALID_ARG,
                "nb = " + std::to_string(nb) + " outside [0, nb_max = " + std::to_string(h->nb_max) +
                    "]");
  if (!rho) return fail(c, PW_ERR_INVALID_ARG, "rho is NULL");
  if (accumulate != 0 && accumulate != 1)
    return fail(c, PW_ERR_INVALID_ARG, "accumulate must be 0 or 1");
  pw_status st;
  if (nb > 0) {
    if ((st = check_block(h, psi, ldpsi, "psi")) != PW_OK) return st;
    if (!w) return fail(c, PW_ERR_INVALID_ARG, "w is NULL");
  }
  if (!(h->omega > 0.0) || !std::isfinite(h->omega))
    return fail(c, PW_ERR_INVALID_ARG, "the reciprocal lattice is singular");
  const BoxPlan& P = h->plan;
  const int64_t nbox = (int64_t)P.n1 * P.n2 * P.n3;
  const int64_t rho_bytes = nbox * (int64_t)sizeof(double);
  if (nb > 0) {
    const int64_t psi_bytes = ((nb - 1) * ldpsi + h->npw) * (int64_t)sizeof(cplx);
    if (spans_overlap(rho, rho_bytes, psi, psi_bytes))
      return fail(c, PW_ERR_INVALID_ARG, "rho and psi overlap");
    if (spans_overlap(rho, rho_bytes, w, nb * (int64_t)sizeof(double)))
      return fail(c, PW_ERR_INVALID_ARG, "rho and w overlap");
  }
  HIPCHK(c, hipSetDevice(c->device));
  const bool reg = density_reg_supported(P, c->lds_limit);
  if (!h->rho_part) {
    // about four workgroups per compute unit over the z-planes (and row
    // parts), at least one band per group and chunk
    const int64_t per = (int64_t)P.n3 * (reg ? density_row_parts(P) : 1);
    const int64_t want = (4 * (int64_t)c->cus + per - 1) / per;
    const int groups = (int)std::max<int64_t>(1, std::min<int64_t>({want, 64, h->chunk_alloc}));
    if ((st = dalloc(h, &h->rho_part, (size_t)groups * nbox)) != PW_OK) return st;
    h->rho_groups = groups;
  }
  hipStream_t s = c->stream;
  const cplx* in = static_cast<const cplx*>(psi);
  for (int64_t c0 = 0; c0 < nb; c0 += h->chunk_alloc) {
    const int nc = (int)std::min<int64_t>(h->chunk_alloc, nb - c0);
    {
      StageScope sc(c, PW_STAGE_FFT_COL_INV);
      HIPCHK(c, launch_fft_col_inv(P, h->cfg, nc, in + c0 * ldpsi, ldpsi, h->T, s));
    }
    StageScope sc(c, PW_STAGE_DENSITY);
    HIPCHK(c, reg ? launch_density_planes_reg(P, nc, h->T, w + c0, h->rho_groups, h->rho_part,
                                              c0 > 0, s)
                  : launch_density_planes_gen(P, h->cfg, nc, h->T, w + c0, h->rho_groups,
                                              h->rho_part, c0 > 0, s));
  }
  StageScope sc(c, PW_STAGE_MISC);
  HIPCHK(c, launch_density_reduce(nbox, nb > 0 ? h->rho_groups : 0, h->rho_part, 1.0 / h->omega,
                                  rho, accumulate, s));
  return PW_OK;
}

pw_status pw_cheb_filter(pw_ham* h, pw_prec prec, int32_t degree, double a, double b, double a0,
                         int64_t nb, void* yv, int64_t ld, const void* hxv, int64_t ldhx) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_status st;
  if ((st = check_hot(h, prec, nb)) != PW_OK) return st;
  if ((st = check_block(h, yv, ld, "y")) != PW_OK) return st;
  if (hxv && (st = check_block(h, hxv, ldhx, "hx")) != PW_OK) return st;
  if (degree < 1) return fail(h->ctx, PW_ERR_INVALID_ARG, "degree must be >= 1");
  if (!(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0)) || !(a0 < a && a < b))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "filter bounds must satisfy a0 < a < b (finite)");
  HIPCHK(h->ctx, hipSetDevice(h->ctx->device));
  cplx* y = static_cast<cplx*>(yv);
  const cplx* hx = static_cast<const cplx*>(hxv);
  const double e = 0.5 * (b - a), c = 0.5 * (b + a);
  double sigma = e / (a0 - c);
  const double tau = 2.0 / sigma;
  if (prec == PW_BF16) {
    // the block enters and leaves in FP64; the recurrence runs on bf16-pair
    // copies (in the memory of the complex64 work blocks)
    bf16c* buf[2] = {reinterpret_cast<bf16c*>(h->blk32[0]), reinterpret_cast<bf16c*>(h->blk32[1])};
    const int64_t l16 = h->npw;
    hipStream_t s = h->ctx->stream;
    {
      StageScope sc(h->ctx, PW_STAGE_MISC);
      HIPCHK(h->ctx, launch_block_to_b16(h->npw, nb, y, ld, buf[0], l16, s));
      if (hx)
        HIPCHK(h->ctx, launch_axpby_to_b16(h->npw, nb, sigma / e, hx, ldhx, -sigma * c / e, y, ld,
                                           buf[1], l16, s));
    }
    if (!hx && (st = ham_apply16(h, nb, buf[0], l16, buf[1], l16, sigma / e, -sigma * c / e, 0.0,
                                 nullptr, 0)) != PW_OK)
      return st;
    for (int i = 2; i <= degree; ++i) {
      const double sn = 1.0 / (tau - sigma);
      const int cur = (i - 1) & 1, nxt = i & 1;
      const double al = 2.0 * sn / e;
      if ((st = ham_apply16(h, nb, buf[cur], l16, buf[nxt], l16, al, -al * c, -sigma * sn, buf[nxt],
                            l16)) != PW_OK)
        return st;
      sigma = sn;
    }
    StageScope sc(h->ctx, PW_STAGE_MISC);
    HIPCHK(h->ctx, launch_block_b16_to_f64(h->npw, nb, buf[degree & 1], l16, y, ld, s));
    return PW_OK;
  }
  if (prec != PW_FP64) {
    // the block enters and leaves in FP64; the recurrence runs on complex64 copies
    const int bf16 = prec == PW_BF16;
    float2* buf[2] = {h->blk32[0], h->blk32[1]};
    const int64_t l32 = h->npw;
    hipStream_t s = h->ctx->stream;
    {
      StageScope sc(h->ctx, PW_STAGE_MISC);
      HIPCHK(h->ctx, launch_block_to_f32(h->npw, nb, y, ld, buf[0], l32, s));
      if (hx)
        HIPCHK(h->ctx, launch_axpby_to_f32(h->npw, nb, sigma / e, hx, ldhx, -sigma * c / e, y, ld,
                                           buf[1], l32, s));
    }
    if (!hx &&
        (st = ham_apply32(h, bf16, nb, buf[0], l32, buf[1], l32, sigma / e, -sigma * c / e, 0.0,
                          nullptr, 0)) != PW_OK)
      return st;
    for (int i = 2; i <= degree; ++i) {
      const double sn = 1.0 / (tau - sigma);
      const int cur = (i - 1) & 1, nxt = i & 1;
      const double al = 2.0 * sn / e;
      if ((st = ham_apply32(h, bf16, nb, buf[cur], l32, buf[nxt], l32, al, -al * c, -sigma * sn,
                            buf[nxt], l32)) != PW_OK)
        return st;
      sigma = sn;
    }
    StageScope sc(h->ctx, PW_STAGE_MISC);
    HIPCHK(h->ctx, launch_block_to_f64(h->npw, nb, buf[degree & 1], l32, y, ld, s));
    return PW_OK;
  }
  // Y0 lives in y, Y1 in blk; Y_i overwrites Y_{i-2} (y for even i, blk for odd i).
  cplx* buf[2] = {y, h->blk};
  int64_t lds[2] = {ld, h->npw};
  if (hx) {
    StageScope sc(h->ctx, PW_STAGE_MISC);
    HIPCHK(h->ctx, launch_axpby_block(h->npw, nb, sigma / e, hx, ldhx, -sigma * c / e, y, ld, h->blk,
                                      h->npw, h->ctx->stream));
  } else {
    if ((st = ham_apply(h, nb, y, ld, h->blk, h->npw, sigma / e, -sigma * c / e, 0.0, nullptr, 0)) !=
        PW_OK)
      return st;
  }
  for (int i = 2; i <= degree; ++i) {
    const double sn = 1.0 / (tau - sigma);
    const int cur = (i - 1) & 1, nxt = i & 1;
    const double al = 2.0 * sn / e;
    if ((st = ham_apply(h, nb, buf[cur], lds[cur], buf[nxt], lds[nxt], al, -al * c, -sigma * sn,
                        buf[nxt], lds[nxt])) != PW_OK)
      return st;
    sigma = sn;
  }
  if (degree & 1) {
    StageScope sc(h->ctx, PW_STAGE_MISC);
    HIPCHK(h->ctx, launch_copy_block(h->npw, nb, h->blk, h->npw, y, ld, h->ctx->stream));
  }
  return PW_OK;
}

pw_status pw_orthonormalize(pw_ham* h, pw_prec gram_prec, int64_t nb, void* yv, int64_t ld,
                            void* hyv, int64_t ldhy) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_status st;
  if ((st = check_hot(h, gram_prec, nb)) != PW_OK) return st;
  if ((st = check_block(h, yv, ld, "y")) != PW_OK) return st;
  if (hyv && (st = check_block(h, hyv, ldhy, "hy")) != PW_OK) return st;
  if (hyv && ranges_overlap(yv, ld, hyv, ldhy, h->npw, nb))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "y and hy overlap");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  return ortho_block(h, nb, static_cast<cplx*>(yv), ld, static_cast<cplx*>(hyv), ldhy, kOpOrtho,
                     gram_prec);
}

pw_status pw_rayleigh_ritz(pw_ham* h, int64_t nb, void* yv, int64_t ld, void* hyv, int64_t ldhy,
                           double* eig, double* resid) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  pw_status st;
  if ((st = check_hot(h, PW_FP64, nb)) != PW_OK) return st;
  if ((st = check_block(h, yv, ld, "y")) != PW_OK) return st;
  if ((st = check_block(h, hyv, ldhy, "hy")) != PW_OK) return st;
  if (!eig) return fail(h->ctx, PW_ERR_INVALID_ARG, "eig_dev is NULL");
  if (ranges_overlap(yv, ld, hyv, ldhy, h->npw, nb))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "y and hy overlap");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  cplx* y = static_cast<cplx*>(yv);
  cplx* hy = static_cast<cplx*>(hyv);
  h->cprj_nb = 0;
  if ((st = ham_apply(h, nb, y, ld, hy, ldhy, 1.0, 0.0, 0.0, nullptr, 0, nullptr, h->cprj_y)) != PW_OK)
    return st;
  if ((st = subspace_rr(h, nb, y, ld, hy, ldhy, eig, resid, kOpRayleighRitz, h->cprj_y)) != PW_OK)
    return st;
  h->cprj_nb = nb;
  return PW_OK;
}

pw_status pw_ham_cprj(pw_ham* h, int64_t nb, void* out, int64_t ldc) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  if (nb < 0 || nb > h->cprj_nb)
    return fail(h->ctx, PW_ERR_INVALID_ARG,
                "the handle holds the projections of " + std::to_string(h->cprj_nb) +
                    " Ritz vectors, not " + std::to_string(nb));
  if (h->nproj == 0 || nb == 0) return PW_OK;
  if (!out || ldc < h->nproj) return fail(h->ctx, PW_ERR_INVALID_ARG, "out is NULL or ldc < nproj");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_copy_block(h->nproj, nb, h->cprj_y, h->nproj, static_cast<cplx*>(out), ldc,
                              c->stream));
  return PW_OK;
}

pw_status pw_upper_bound(pw_ham* h, double* b_host) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  if (!b_host) return fail(h->ctx, PW_ERR_INVALID_ARG, "b_host is NULL");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  double b = h->kmax + h->vmax;
  if (h->nproj > 0) {
    const int64_t m = h->nproj;
    pw_ham tmp;   // scratch owner for the allocations of this call
    tmp.ctx = c;
    cplx* M = nullptr;
    cplx* Q = nullptr;
    cplx* work = nullptr;
    double* w = nullptr;
    double* sq = nullptr;
    char* hw = nullptr;
    pw_status st = PW_OK;
    if ((st = dalloc(&tmp, &M, (size_t)(m * m))) != PW_OK ||
        (st = dalloc(&tmp, &Q, (size_t)(m * m))) != PW_OK ||
        (st = dalloc(&tmp, &work, std::max<size_t>(1, gemm_cn_work_elems(m, m, h->npw)))) != PW_OK ||
        (st = dalloc(&tmp, &w, (size_t)m)) != PW_OK || (st = dalloc(&tmp, &sq, (size_t)m)) != PW_OK ||
        (st = dalloc(&tmp, &hw, heev_work_bytes(m))) != PW_OK) {
      free_ham(&tmp);
      return st;
    }
    std::vector<double> sqh(m);
    for (int64_t j = 0; j < m; ++j) sqh[j] = std::sqrt(std::max(h->ekb[j], 0.0));
    hipStream_t s = c->stream;
    hipError_t e = hipMemcpy(sq, sqh.data(), m * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_gemm_cn(m, m, h->npw, 1.0, h->proj, h->npw, h->proj, h->npw, M, m, nullptr, work, s);
    if (e == hipSuccess) e = launch_scale_rows_cols(m, sq, M, m, s);
    if (e == hipSuccess) e = launch_hermitize(m, M, m, s);
    int sweeps = 0;
    if (e == hipSuccess)
      e = launch_heev(m, M, m, w, Q, m, hw, sweeps_slot(c), reinterpret_cast<int*>(c->pinned),
                      &sweeps, s);
    double wmax = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&wmax, w + (m - 1), sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    free_ham(&tmp);
    if (e != hipSuccess) return fail(c, PW_ERR_HIP, hipGetErrorString(e));
    if ((st = heev_status(c, sweeps)) != PW_OK) return st;
    b += std::max(wmax, 0.0);
  }
  *b_host = b;
  return PW_OK;
}

// ---------------------------------------------------------------------------
// autotuning of the H*psi launch shapes
// ---------------------------------------------------------------------------
pw_status pw_ham_get_tuning(const pw_ham* h, pw_tuning* t) {
  if (!h || !t) return fail(nullptr, PW_ERR_INVALID_ARG, "ham or tuning is NULL");
  t->reg_col = h->cfg.reg_col ? 1 : 0;
  t->reg_plane = h->cfg.reg_plane ? 1 : 0;
  t->plane_variant = h->cfg.plane_variant;
  t->plane_variant32 = h->cfg.plane_variant32;
  t->chunk = (int32_t)h->chunk;
  t->gemm_blocks = h->gemm_target;
  t->nn_tile = h->nn_tile;
  t->nn_tile32 = h->nn_tile32;
  t->ms = 0.0;
  return PW_OK;
}

pw_status pw_ham_set_tuning(pw_ham* h, const pw_tuning* t) {
  if (!h || !t) return fail(nullptr, PW_ERR_INVALID_ARG, "ham or tuning is NULL");
  if ((t->reg_col != 0 && t->reg_col != 1) || (t->reg_plane != 0 && t->reg_plane != 1) ||
      (t->plane_variant != 0 && t->plane_variant != 1) ||
      (t->plane_variant32 < 0 || t->plane_variant32 > 2))
    return fail(h->ctx, PW_ERR_INVALID_ARG,
                "reg_col, reg_plane and plane_variant are 0 or 1, plane_variant32 0, 1 or 2");
  if (t->reg_col && !h->reg_col_ok)
    return fail(h->ctx, PW_ERR_UNSUPPORTED, "no register column kernel for this N3");
  if (t->reg_plane && !h->reg_plane_ok)
    return fail(h->ctx, PW_ERR_UNSUPPORTED, "no register plane kernel for this (N1, N2)");
  if (t->plane_variant == 1 && (!t->reg_plane || !h->narrow_ok))
    return fail(h->ctx, PW_ERR_UNSUPPORTED, "no 8-lane FP64 plane variant for this (N1, N2)");
  if (t->plane_variant32 == 1 && (!t->reg_plane || !h->narrow32_ok))
    return fail(h->ctx, PW_ERR_UNSUPPORTED, "no 8-lane FP32 plane variant for this (N1, N2)");
  if (t->plane_variant32 == 2 && (!t->reg_plane || !h->ls32_ok))
    return fail(h->ctx, PW_ERR_UNSUPPORTED, "no LDS-exchange FP32 plane kernel for this (N1, N2)");
  if (t->chunk < 1 || t->chunk > h->chunk_alloc)
    return fail(h->ctx, PW_ERR_INVALID_ARG,
                "chunk outside [1, " + std::to_string(h->chunk_alloc) + "]");
  if (t->gemm_blocks < 1 || t->gemm_blocks > 4096)
    return fail(h->ctx, PW_ERR_INVALID_ARG, "gemm_blocks outside [1, 4096]");
  if ((t->nn_tile != 0 && t->nn_tile != 1) || (t->nn_tile32 != 0 && t->nn_tile32 != 1))
    return fail(h->ctx, PW_ERR_INVALID_ARG, "nn_tile and nn_tile32 are 0 or 1");
  h->cfg.reg_col = t->reg_col != 0;
  h->cfg.reg_plane = t->reg_plane != 0;
  h->cfg.plane_variant = t->plane_variant;
  h->cfg.plane_variant32 = t->plane_variant32;
  h->chunk = t->chunk;
  h->gemm_target = t->gemm_blocks;
  h->nn_tile = t->nn_tile;
  h->nn_tile32 = t->nn_tile32;
  return PW_OK;
}


pw_status pw_ham_autotune(pw_ham* h, pw_prec prec, int64_t nb, int32_t reps, pw_tuning* best,
                          pw_tuning* initial) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  if (!best) return fail(h->ctx, PW_ERR_INVALID_ARG, "best is NULL");
  pw_status st;
  if ((st = check_hot(h, prec, nb)) != PW_OK) return st;
  if (reps < 1 || reps > 100) return fail(h->ctx, PW_ERR_INVALID_ARG, "reps outside [1, 100]");
  pw_ctx* c = h->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  const bool timing = c->timing;
  c->timing = false;
  struct Restore {
    pw_ctx* c;
    bool t;
    ~Restore() { c->timing = t; }
  } restore{c, timing};
  // operands: zero input, scratch output
  pw_ham scratch;
  scratch.ctx = c;
  void* in = nullptr;
  void* out = nullptr;
  const size_t elem = prec == PW_FP64 ? sizeof(cplx) : sizeof(float2);
  if (prec == PW_FP64) {
    in = h->blk;
    cplx* o = nullptr;
    if ((st = dalloc(&scratch, &o, (size_t)(h->npw * nb))) != PW_OK) return st;
    out = o;
  } else {
    in = h->blk32[0];
    out = h->blk32[1];
  }
  struct FreeScratch {
    pw_ham* s;
    ~FreeScratch() { free_ham(s); }
  } free_scratch{&scratch};
  HIPCHK(c, hipMemsetAsync(in, 0, (size_t)(h->npw * nb) * elem, c->stream));

  pw_tuning cur;
  pw_ham_get_tuning(h, &cur);
  double cur_ms = 0.0;
  if ((st = time_apply(h, prec, nb, in, out, reps, &cur_ms)) != PW_OK) return st;
  if (initial) {
    *initial = cur;
    initial->ms = cur_ms;
  }
  auto try_one = [&](pw_tuning t) -> pw_status {
    pw_status s2 = pw_ham_set_tuning(h, &t);
    if (s2 != PW_OK) return s2;
    double ms = 0.0;
    if ((s2 = time_apply(h, prec, nb, in, out, reps, &ms)) != PW_OK) return s2;
    // a change must win by more than the spread of repeated timings (about 1%)
    if (ms < (1.0 - kTuneMargin) * cur_ms) {
      cur = t;
      cur_ms = ms;
    }
    return pw_ham_set_tuning(h, &cur);
  };
  // 1) FFT kernel families (the plane variant of the precision being tuned)
  const bool lp = prec != PW_FP64;
  const bool nok = lp ? h->narrow32_ok : h->narrow_ok;
  const bool lsok = lp && h->ls32_ok;
  for (int rc = 0; rc <= (h->reg_col_ok ? 1 : 0); ++rc)
    for (int rp = 0; rp <= (h->reg_plane_ok ? 1 : 0); ++rp)
      for (int pv = 0; pv <= (rp ? 2 : 0); ++pv) {
        if ((pv == 1 && !nok) || (pv == 2 && !lsok)) continue;
        pw_tuning t = cur;
        t.reg_col = rc;
        t.reg_plane = rp;
        if (lp) t.plane_variant32 = pv;
        else t.plane_variant = pv;
        if (!rp) t.plane_variant = t.plane_variant32 = 0;
        if (t.reg_col == cur.reg_col && t.reg_plane == cur.reg_plane &&
            t.plane_variant == cur.plane_variant && t.plane_variant32 == cur.plane_variant32)
          continue;
        if ((st = try_one(t)) != PW_OK) return st;
      }
  // 2) bands per FFT launch
  const int64_t cmax = std::min<int64_t>(h->chunk_alloc, nb);
  for (int64_t ch = cmax; ch >= 1 && ch >= cmax / 8; ch /= 2) {
    if (ch == cur.chunk) continue;
    pw_tuning t = cur;
    t.chunk = (int32_t)ch;
    if ((st = try_one(t)) != PW_OK) return st;
  }
  // 3) split-K parallelism of the projector product
  if (h->nproj > 0)
    for (int g : {4096, 2048, 1024, 512, 256, 64, 1}) {
      if (g == cur.gemm_blocks) continue;
      pw_tuning t = cur;
      t.gemm_blocks = g;
      if ((st = try_one(t)) != PW_OK) return st;
    }
  // 4) workgroup tile of the tall product P C of the precision being tuned
  if (h->nproj > 0) {
    pw_tuning t = cur;
    if (lp)
      t.nn_tile32 = 1 - cur.nn_tile32;
    else
      t.nn_tile = 1 - cur.nn_tile;
    if ((st = try_one(t)) != PW_OK) return st;
  }
  *best = cur;
  best->ms = cur_ms;
  return PW_OK;
}

pw_status pw_autotune(pw_ham* h, pw_prec prec, int64_t nb, int32_t reps, const char* cache_path,
                      pw_tuning* best, pw_tuning* initial, int32_t* cached) {
  if (!h) return fail(nullptr, PW_ERR_INVALID_ARG, "ham is NULL");
  if (!best) return fail(h->ctx, PW_ERR_INVALID_ARG, "best is NULL");
  pw_status st;
  if ((st = check_hot(h, prec, nb)) != PW_OK) return st;
  // shape key: box, sphere columns and extent, npw, nproj, nb, precision
  const BoxPlan& P = h->plan;
  std::ostringstream ks;
  ks << P.n1 << "x" << P.n2 << "x" << P.n3 << "/cols" << P.ncols << "/xr" << P.xr << "/npw"
     << h->npw << "/proj" << h->nproj << "/nb" << nb << "/" << (int)prec;
  const std::string key = ks.str();
  static const char* names[8] = {"reg_col", "reg_plane", "plane_variant", "plane_variant32",
                                 "chunk", "gemm_blocks", "nn_tile", "nn_tile32"};
  auto fields = [](pw_tuning& t) {
    int32_t* f[8] = {&t.reg_col, &t.reg_plane, &t.plane_variant, &t.plane_variant32,
                     &t.chunk, &t.gemm_blocks, &t.nn_tile, &t.nn_tile32};
    return std::vector<int32_t*>(f, f + 8);
  };
  std::vector<std::string> keep;
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream is(line);
      std::string k;
      if (!(is >> k)) continue;
      if (k != key) {
        keep.push_back(line);
        continue;
      }
      pw_tuning t{};
      pw_ham_get_tuning(h, &t);
      int found = 0;
      std::string tok;
      while (is >> tok) {
        const size_t eq = tok.find('=');
        if (eq == std::string::npos) continue;
        const std::string n = tok.substr(0, eq), v = tok.substr(eq + 1);
        if (n == "ms") {
          t.ms = std::atof(v.c_str());
          continue;
        }
        auto f = fields(t);
        for (int i = 0; i < 8; ++i)
          if (n == names[i]) {
            *f[i] = (int32_t)std::atoi(v.c_str());
            ++found;
          }
      }
      if (found == 8 && pw_ham_set_tuning(h, &t) == PW_OK) {
        if (initial) {
          *initial = t;
          initial->ms = 0.0;
        }
        *best = t;
        if (cached) *cached = 1;
        return PW_OK;
      }
    }
  }
  if ((st = pw_ham_autotune(h, prec, nb, reps, best, initial)) != PW_OK) return st;
  if (cached) *cached = 0;
  if (cache_path && *cache_path) {
    std::ostringstream line;
    line << key;
    pw_tuning t = *best;
    auto f = fields(t);
    for (int i = 0; i < 8; ++i) line << " " << names[i] << "=" << *f[i];
    line << " ms=" << best->ms;
    keep.push_back(line.str());
    const std::string tmp = std::string(cache_path) + ".tmp";
    {
      std::ofstream out(tmp, std::ios::trunc);
      for (const std::string& l : keep) out << l << "\n";
      if (!out) return fail(h->ctx, PW_ERR_INVALID_ARG, "cannot write the tuning cache " + tmp);
    }
    if (std::rename(tmp.c_str(), cache_path) != 0)
      return fail(h->ctx, PW_ERR_INVALID_ARG, std::string("cannot replace ") + cache_path);
  }
  return PW_OK;
}

// ---------------------------------------------------------------------------
// batched subspace iteration
// ---------------------------------------------------------------------------
pw_status pw_batch_destroy(pw_batch* b) {
  if (!b) return fail(nullptr, PW_ERR_INVALID_ARG, "batch is NULL");
  (void)hipSetDevice(b->ctx->device);
  if (b->s0) (void)hipStreamSynchronize(b->s0);
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->fexec) (void)hipGraphExecDestroy(b->fexec);
  if (b->fgraph) (void)hipGraphDestroy(b->fgraph);
  for (hipGraphExec_t e : b->sexec)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipGraph_t g : b->sgraph)
    if (g) (void)hipGraphDestroy(g);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  if (b->s0) (void)hipStreamDestroy(b->s0);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->flags_host) (void)hipHostFree(b->flags_host);
  pw_ctx* c = b->ctx;
  delete b;
  ctx_release(c);
  return PW_OK;
}

pw_status pw_batch_create(pw_ctx* ctx, int32_t n, pw_ham* const* hams, const int64_t* nb,
                          void* const* y, void* const* hy, double* const* eig,
                          double* const* resid, int32_t degree, pw_prec prec, int32_t nstreams,
                          pw_batch** out) {
  if (!ctx) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(ctx, PW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(ctx, PW_ERR_INVALID_ARG, "batch needs n >= 1 items");
  if (!hams || !nb || !y || !hy || !eig || !resid)
    return fail(ctx, PW_ERR_INVALID_ARG, "NULL item array");
  if (degree < 1) return fail(ctx, PW_ERR_INVALID_ARG, "degree must be >= 1");
  if (prec != PW_FP64 && prec != PW_FP32 && prec != PW_BF16)
    return fail(ctx, PW_ERR_INVALID_ARG, "unknown precision");
  if (nstreams < 1 || nstreams > 64) return fail(ctx, PW_ERR_INVALID_ARG, "nstreams outside [1, 64]");
  std::unordered_set<const pw_ham*> seen;
  for (int32_t i = 0; i < n; ++i) {
    const std::string who = "item " + std::to_string(i) + ": ";
    pw_ham* h = hams[i];
    if (!h || h->ctx != ctx) return fail(ctx, PW_ERR_INVALID_ARG, who + "ham NULL or of another ctx");
    if (!seen.insert(h).second) return fail(ctx, PW_ERR_INVALID_ARG, who + "ham used twice");
    if (nb[i] < 1 || nb[i] > 64 || nb[i] > h->nb_max)
      return fail(ctx, PW_ERR_INVALID_ARG, who + "nb outside [1, min(64, nb_max)]");
    if (prec != PW_FP64 && !h->low_prec)
      return fail(ctx, PW_ERR_UNSUPPORTED, who + "FP32/BF16 filter needs a low_prec handle");
    if (!y[i] || !hy[i] || !eig[i] || !resid[i])
      return fail(ctx, PW_ERR_INVALID_ARG, who + "NULL buffer");
    if (ranges_overlap(y[i], h->npw, hy[i], h->npw, h->npw, nb[i]))
      return fail(ctx, PW_ERR_INVALID_ARG, who + "y and hy overlap");
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<double> upper(n);
  for (int32_t i = 0; i < n; ++i) {
    pw_status st = pw_upper_bound(hams[i], &upper[i]);
    if (st != PW_OK) return st;
  }
  pw_batch* b = new pw_batch();
  b->ctx = ctx;
  ++ctx->refs;   // released by pw_batch_destroy, also on the failure paths below
  b->degree = degree;
  b->prec = prec;
  const int ns = std::min<int32_t>(nstreams, n);
  auto bail_hip = [&](hipError_t e, const char* what) {
    (void)hipGetLastError();
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    pw_batch_destroy(b);
    return fail(ctx, e == hipErrorOutOfMemory ? PW_ERR_OOM : PW_ERR_HIP, msg);
  };
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&b->s0, hipStreamNonBlocking)) != hipSuccess)
    return bail_hip(e, "hipStreamCreateWithFlags");
  for (int k = 0; k < ns; ++k) {
    hipStream_t st = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
      return bail_hip(e, "hipStreamCreateWithFlags");
    b->streams.push_back(st);
  }
  for (int k = 0; k < 3 + ns; ++k) {
    hipEvent_t ev = nullptr;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return bail_hip(e, "hipEventCreateWithFlags");
    b->ev.push_back(ev);
  }
  const size_t per_item = (size_t)3 * degree + 1;
  double* dbl = nullptr;
  int* ints = nullptr;
  if ((e = hipMalloc(&dbl, per_item * n * sizeof(double))) != hipSuccess)
    return bail_hip(e, "hipMalloc");
  b->allocs.push_back(dbl);
  if ((e = hipMalloc(&ints, (size_t)5 * n * sizeof(int))) != hipSuccess) return bail_hip(e, "hipMalloc");
  b->allocs.push_back(ints);
  void* pin = nullptr;
  if ((e = hipHostMalloc(&pin, (size_t)4 * n * sizeof(int), hipHostMallocDefault)) != hipSuccess)
    return bail_hip(e, "hipHostMalloc");
  b->flags_host = static_cast<int*>(pin);
  b->flags_dev = ints;
  // items go to the least-loaded stream, largest first
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int p, int q) {
    return hams[p]->npw * nb[p] > hams[q]->npw * nb[q];
  });
  std::vector<double> load(ns, 0.0);
  b->items.resize(n);
  for (int i = 0; i < n; ++i) {
    BatchItem& it = b->items[i];
    it.h = hams[i];
    it.nb = nb[i];
    it.y = static_cast<cplx*>(y[i]);
    it.hy = static_cast<cplx*>(hy[i]);
    it.eig = eig[i];
    it.resid = resid[i];
    it.coef = dbl + per_item * i;
    it.upper = it.coef + 3 * degree;
    it.flags = ints + 4 * i;
    it.sweeps = ints + 4 * n + i;
  }
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->items[i].stream = k;
    load[k] += (double)hams[i]->npw * nb[i];
  }
  for (int i = 0; i < n; ++i)
    if ((e = hipMemcpyAsync(b->items[i].upper, &upper[i], sizeof(double), hipMemcpyHostToDevice,
                            b->s0)) != hipSuccess)
      return bail_hip(e, "hipMemcpyAsync");
  if ((e = hipMemsetAsync(ints, 0, (size_t)5 * n * sizeof(int), b->s0)) != hipSuccess)
    return bail_hip(e, "hipMemsetAsync");
  if ((e = hipStreamSynchronize(b->s0)) != hipSuccess) return bail_hip(e, "hipStreamSynchronize");
  *out = b;
  return PW_OK;
}


pw_status pw_batch_start(pw_batch* b) {
  if (!b) return fail(nullptr, PW_ERR_INVALID_ARG, "batch is NULL");
  pw_status st;
  if ((st = batch_enter(b)) != PW_OK) return st;
  if ((st = batch_issue(b, false, false)) != PW_OK) return st;
  return batch_leave(b);
}

pw_status pw_batch_iterate(pw_batch* b, int32_t iters, int32_t use_graph) {
  if (!b) return fail(nullptr, PW_ERR_INVALID_ARG, "batch is NULL");
  if (iters < 0) return fail(b->ctx, PW_ERR_INVALID_ARG, "iters < 0");
  if (use_graph < 0 || use_graph > 4)
    return fail(b->ctx, PW_ERR_INVALID_ARG, "use_graph must be in [0, 4]");
  pw_ctx* c = b->ctx;
  pw_status st;
  if ((st = batch_enter(b)) != PW_OK) return st;
  if (use_graph == 1 && !b->exec) {
    HIPCHK(c, hipStreamBeginCapture(b->s0, hipStreamCaptureModeThreadLocal));
    st = batch_issue(b, true, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->s0, &g);
    if (st != PW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, PW_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    b->graph = g;
    HIPCHK(c, hipGraphInstantiateWithFlags(&b->exec, b->graph, 0));
  }
  if (use_graph == 2 && b->sexec.empty()) {
    const size_t ns = b->streams.size();
    b->sgraph.assign(ns, nullptr);
    b->sexec.assign(ns, nullptr);
    for (size_t k = 0; k < ns; ++k) {
      HIPCHK(c, hipStreamBeginCapture(b->streams[k], hipStreamCaptureModeThreadLocal));
      st = batch_issue_stream(b, k, true, true);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(b->streams[k], &g);
      b->sgraph[k] = g;
      if (st != PW_OK) return st;
      if (e != hipSuccess)
        return fail(c, PW_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      HIPCHK(c, hipGraphInstantiateWithFlags(&b->sexec[k], g, 0));
    }
  }
  if (use_graph >= 3 && b->groups.empty() && (st = fused_setup(b)) != PW_OK) return st;
  if (use_graph == 3 && !b->fexec) {
    HIPCHK(c, hipStreamBeginCapture(b->s0, hipStreamCaptureModeThreadLocal));
    st = fused_issue(b, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->s0, &g);
    if (st != PW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, PW_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    b->fgraph = g;
    HIPCHK(c, hipGraphInstantiateWithFlags(&b->fexec, b->fgraph, 0));
  }
  for (int32_t t = 0; t < iters; ++t) {
    if (use_graph == 3) {
      HIPCHK(c, hipGraphLaunch(b->fexec, b->s0));
    } else if (use_graph == 4) {
      if ((st = fused_issue(b, false)) != PW_OK) return st;
    } else if (use_graph == 1) {
      HIPCHK(c, hipGraphLaunch(b->exec, b->s0));
    } else if (use_graph == 2) {
      if ((st = batch_fork(b)) != PW_OK) return st;
      for (size_t k = 0; k < b->streams.size(); ++k)
        HIPCHK(c, hipGraphLaunch(b->sexec[k], b->streams[k]));
      if ((st = batch_join(b)) != PW_OK) return st;
    } else if ((st = batch_issue(b, true, false)) != PW_OK) {
      return st;
    }
  }
  return batch_leave(b);
}

pw_status pw_batch_chfsi(pw_batch* b, int32_t iters, int32_t use_graph) {
  if (!b) return fail(nullptr, PW_ERR_INVALID_ARG, "batch is NULL");
  pw_status st;
  if ((st = pw_batch_start(b)) != PW_OK) return st;
  return pw_batch_iterate(b, iters, use_graph);
}

pw_status pw_batch_max_sweeps(const pw_batch* b, int32_t* sweeps) {
  if (!b || !sweeps) return fail(nullptr, PW_ERR_INVALID_ARG, "batch or sweeps is NULL");
  *sweeps = b->max_sweeps;
  return PW_OK;
}

// ---------------------------------------------------------------------------
// dense building blocks
// ---------------------------------------------------------------------------
pw_status pw_gemm_cn(pw_ctx* c, int64_t m, int64_t n, int64_t k, double alpha, const void* a,
                     int64_t lda, const void* bm, int64_t ldb, void* cm, int64_t ldc) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (m < 0 || n < 0 || k < 0 || !a || !bm || !cm || lda < std::max<int64_t>(k, 1) ||
      ldb < std::max<int64_t>(k, 1) || ldc < std::max<int64_t>(m, 1))
    return fail(c, PW_ERR_INVALID_ARG, "pw_gemm_cn: bad sizes or pointers");
  HIPCHK(c, hipSetDevice(c->device));
  pw_ham tmp;
  tmp.ctx = c;
  cplx* work = nullptr;
  pw_status st = dalloc(&tmp, &work, std::max<size_t>(1, gemm_cn_work_elems(m, n, k)));
  if (st != PW_OK) return st;
  hipError_t e = launch_gemm_cn(m, n, k, alpha, static_cast<const cplx*>(a), lda,
                                static_cast<const cplx*>(bm), ldb, static_cast<cplx*>(cm), ldc,
                                nullptr, work, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  free_ham(&tmp);
  if (e != hipSuccess) return fail(c, PW_ERR_HIP, hipGetErrorString(e));
  return PW_OK;
}

pw_status pw_gemm_nn(pw_ctx* c, int64_t m, int64_t n, int64_t k, double alpha, const void* a,
                     int64_t lda, const void* bm, int64_t ldb, double beta, void* cm, int64_t ldc) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (m < 0 || n < 0 || k < 0 || !a || !bm || !cm || lda < std::max<int64_t>(m, 1) ||
      ldb < std::max<int64_t>(k, 1) || ldc < std::max<int64_t>(m, 1))
    return fail(c, PW_ERR_INVALID_ARG, "pw_gemm_nn: bad sizes or pointers");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_gemm_nn(m, n, k, alpha, static_cast<const cplx*>(a), lda,
                           static_cast<const cplx*>(bm), ldb, beta, static_cast<cplx*>(cm), ldc,
                           c->stream));
  return PW_OK;
}

pw_status pw_heev(pw_ctx* c, int64_t n, void* a, int64_t lda, double* w, void* q, int64_t ldq) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 1 || n > 4096 || !a || !w || !q || lda < n || ldq < n)
    return fail(c, PW_ERR_INVALID_ARG, "pw_heev: bad sizes or pointers");
  HIPCHK(c, hipSetDevice(c->device));
  pw_ham tmp;
  tmp.ctx = c;
  char* hw = nullptr;
  pw_status st = dalloc(&tmp, &hw, heev_work_bytes(n));
  if (st != PW_OK) return st;
  int sweeps = 0;
  hipError_t e = launch_heev(n, static_cast<const cplx*>(a), lda, w, static_cast<cplx*>(q), ldq, hw,
                             sweeps_slot(c), reinterpret_cast<int*>(c->pinned), &sweeps, c->stream);
  free_ham(&tmp);
  if (e != hipSuccess) return fail(c, PW_ERR_HIP, hipGetErrorString(e));
  return heev_status(c, sweeps);
}

pw_status pw_heev_noalloc(pw_ctx* c, int64_t n, const void* a, int64_t lda, double* w, void* q,
                          int64_t ldq) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 1 || !a || !w || !q || lda < n || ldq < n)
    return fail(c, PW_ERR_INVALID_ARG, "pw_heev_noalloc: bad sizes or pointers");
  if (n > kScratchHeevMax || heev_work_bytes(n) > kScratchBytes)
    return fail(c, PW_ERR_INVALID_ARG,
                "pw_heev_noalloc: n = " + std::to_string(n) + " exceeds its static workspace (n <= " +
                    std::to_string(kScratchHeevMax) + ")");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  {
    StageScope sc(c, PW_STAGE_EIGH);
    HIPCHK(c, launch_heev_async(n, static_cast<const cplx*>(a), lda, w, static_cast<cplx*>(q), ldq,
                                c->scratch, sweeps_slot(c), kHeevMaxSweeps, s));
    HIPCHK(c, launch_status_record(nullptr, sweeps_slot(c), kOpHeev, c->rec_dev, s));
  }
  return PW_OK;
}

pw_status pw_potrf_inv(pw_ctx* c, int64_t n, void* a, int64_t lda, void* ainv, int64_t ldi) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 1 || n > 4096 || !a || !ainv || lda < n || ldi < n)
    return fail(c, PW_ERR_INVALID_ARG, "pw_potrf_inv: bad sizes or pointers");
  HIPCHK(c, hipSetDevice(c->device));
  pw_ham tmp;
  tmp.ctx = c;
  int* stat = nullptr;
  double* tol = nullptr;
  cplx* dinv = nullptr;
  cplx* panel = nullptr;
  cplx* ytmp = nullptr;
  pw_status st = PW_OK;
  if ((st = dalloc(&tmp, &stat, 1)) != PW_OK || (st = dalloc(&tmp, &tol, 1)) != PW_OK ||
      (st = dalloc(&tmp, &dinv, (size_t)((n + kCholBlock) * kCholBlock))) != PW_OK ||
      (st = dalloc(&tmp, &panel, (size_t)(kCholBlock * n))) != PW_OK ||
      (st = dalloc(&tmp, &ytmp, (size_t)(kCholBlock * n))) != PW_OK) {
    free_ham(&tmp);
    return st;
  }
  cplx* A = static_cast<cplx*>(a);
  cplx* X = static_cast<cplx*>(ainv);
  hipStream_t s = c->stream;
  hipError_t e = chol_blocked(n, A, lda, dinv, panel, tol, stat, s);
  int hs = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, stat, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && hs == -1) {
    e = launch_zero_lower(n, A, lda, s);
    if (e == hipSuccess) e = launch_identity(n, X, ldi, s);
    if (e == hipSuccess) e = trsm_right(n, n, X, ldi, A, lda, dinv, ytmp, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  free_ham(&tmp);
  if (e != hipSuccess) return fail(c, PW_ERR_HIP, hipGetErrorString(e));
  if (hs >= 0) return fail(c, PW_ERR_NOT_POSDEF, "matrix not positive definite at pivot " + std::to_string(hs));
  if (hs <= kCholNonFinite)
    return fail(c, PW_ERR_NONFINITE,
                "diagonal entry " + std::to_string(kCholNonFinite - hs) + " is NaN or infinite");
  return PW_OK;
}

// ---------------------------------------------------------------------------
// stage timing
// ---------------------------------------------------------------------------
pw_status pw_ctx_set_timing(pw_ctx* c, int enable) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = enable != 0;
  return PW_OK;
}

static pw_status resolve_timing(pw_ctx* c) {
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->acc_ms[p.stage] += ms;
      c->launches[p.stage] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  return PW_OK;
}

pw_status pw_ctx_stage_time(pw_ctx* c, int stage, double* total_ms, int64_t* launches) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (stage < 0 || stage >= PW_STAGE_COUNT) return fail(c, PW_ERR_INVALID_ARG, "bad stage");
  pw_status st = resolve_timing(c);
  if (st != PW_OK) return st;
  if (total_ms) *total_ms = c->acc_ms[stage];
  if (launches) *launches = c->launches[stage];
  return PW_OK;
}

pw_status pw_ctx_last_sweeps(const pw_ctx* c, int* sweeps) {
  if (!c || !sweeps) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx or sweeps is NULL");
  pw_ctx* m = const_cast<pw_ctx*>(c);
  HIPCHK(m, hipSetDevice(m->device));
  int* hs = reinterpret_cast<int*>(m->pinned) + 8;
  HIPCHK(m, hipMemcpyAsync(hs, sweeps_slot(m), sizeof(int), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(m, hipStreamSynchronize(m->stream));
  *sweeps = hs[0];
  return PW_OK;
}

pw_status pw_ctx_set_sweep_limit(pw_ctx* c, int32_t max_sweeps) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (max_sweeps < 1 || max_sweeps > kHeevMaxSweeps)
    return fail(c, PW_ERR_INVALID_ARG,
                "sweep limit must be in [1, " + std::to_string(kHeevMaxSweeps) + "]");
  c->max_sweeps = max_sweeps;
  return PW_OK;
}

pw_status pw_ctx_set_overlap(pw_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  if (enable != 0 && enable != 1) return fail(c, PW_ERR_INVALID_ARG, "enable must be 0 or 1");
  c->overlap = enable != 0;
  return PW_OK;
}

pw_status pw_ctx_check(pw_ctx* c) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  HIPCHK(c, hipSetDevice(c->device));
  int* hr = reinterpret_cast<int*>(c->pinned) + 16;
  HIPCHK(c, hipMemcpyAsync(hr, c->rec_dev, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int code = hr[0], op = hr[1], info = hr[2];
  if (code == 0) return PW_OK;
  HIPCHK(c, launch_fill_int(4, 0, c->rec_dev, c->stream));
  if (code == PW_ERR_NOT_POSDEF)
    return fail(c, PW_ERR_NOT_POSDEF,
                std::string(op_name(op)) + ": Gram matrix not positive definite at pivot " +
                    std::to_string(info));
  if (code == PW_ERR_NONFINITE)
    return fail(c, PW_ERR_NONFINITE,
                std::string(op_name(op)) + ": column " + std::to_string(info) +
                    " of the block is NaN or infinite (its Gram diagonal entry)");
  if (code == PW_ERR_NO_CONVERGENCE)
    return fail(c, PW_ERR_NO_CONVERGENCE,
                std::string(op_name(op)) + ": Jacobi eigensolver reached its limit of " +
                    std::to_string(c->max_sweeps) + " sweeps");
  return fail(c, (pw_status)code, std::string(op_name(op)) + ": device-side failure");
}

pw_status pw_ctx_reset_timing(pw_ctx* c) {
  if (!c) return fail(nullptr, PW_ERR_INVALID_ARG, "ctx is NULL");
  pw_status st = resolve_timing(c);
  if (st != PW_OK) return st;
  for (int i = 0; i < PW_STAGE_COUNT; ++i) {
    c->acc_ms[i] = 0.0;
    c->launches[i] = 0;
  }
  return PW_OK;
}

}  // extern "C"
