// Handle structures and host helpers shared by the library's host sources
// (pw_api.hip: contexts, Hamiltonian handles, the Chebyshev-filtered path,
// the batch; solvers.hip: LOBPCG and RMM-DIIS).  Not part of the C ABI.
#pragma once

#include "pw_internal.h"

#include <string>
#include <vector>

struct EventPair {
  hipEvent_t a, b;
  int stage;
};

struct pw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // where the library's work goes (the batch swaps it)
  hipStream_t home = nullptr;     // the stream given at creation
  // second stream for the projection product P^H psi, which then overlaps
  // the FFT route of the same H*psi (fork / join by events); off by
  // default: measured slower at C5, the persistent plane kernel and the
  // projection both want whole compute units
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = false;
  std::string err;
  size_t lds_limit = 0;
  int cus = 256;              // compute units of the device
  bool timing = false;
  std::vector<EventPair> pending;
  std::vector<hipEvent_t> pool;
  double acc_ms[PW_STAGE_COUNT] = {0};
  int64_t launches[PW_STAGE_COUNT] = {0};
  double* pinned = nullptr;   // small pinned host scratch (64 doubles)
  // deferred status of the hot calls on the device: [0..2] = {status, op,
  // info} of the first failure since the last pw_ctx_check, [4] = sweeps of
  // the last dense eigensolve (-1: sweep limit reached)
  int* rec_dev = nullptr;
  int max_sweeps = 24;        // sweep limit of the block eigensolver in hot calls
  void* scratch = nullptr;    // this device's address of the static workspace of pw_heev_noalloc
  int refs = 1;               // the caller's handle + one per live ham / batch

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

// Workspace of pw_lobpcg, sized by its largest block (m bands) and nb.
struct LobpcgWork {
  int64_t m = 0, nb = 0;
  cplx* v[2] = {nullptr, nullptr};    // [X, W, P] blocks, npw x 3m each (ping-pong)
  cplx* hv[2] = {nullptr, nullptr};   // H [X, W, P]
  cplx* s = nullptr;                  // subspace matrix (3m)^2
  cplx* z = nullptr;                  // its eigenvectors
  cplx* c = nullptr;                  // projection coefficients, max(nb, 3m) x m
  cplx* work = nullptr;               // split-K partials
  double* theta = nullptr;            // 3m Ritz values
  double* lam = nullptr;              // m current Ritz values of the block
  double* ek = nullptr;               // m band kinetic energies
  void* heev = nullptr;
  cplx* cv[2] = {nullptr, nullptr};   // P^H [X, W, P], nproj x 3m each
  std::vector<void*> mem;
};

// Workspace of pw_rmm_diis, sized by nb and the history length.
struct RmmWork {
  int64_t nb = 0;
  int ndiis = 0;
  cplx* psi = nullptr;                // history psi^0..psi^ndiis, npw x nb each
  cplx* r = nullptr;                  // their residuals
  cplx* hcur = nullptr;               // H psi of the latest step
  cplx* d = nullptr;                  // K R^0
  cplx* hd = nullptr;                 // H K R^0
  cplx* amat = nullptr;               // per band (ndiis+1)^2 <R^i|R^j>
  cplx* bmat = nullptr;               // per band (ndiis+1)^2 <psi^i|psi^j>
  cplx* coef = nullptr;               // per band ndiis+1 DIIS coefficients
  cplx* dots = nullptr;               // per band inner products of one launch
  cplx* lam = nullptr;                // per band trial step
  double* ek = nullptr;               // per band kinetic energy of psi^0
  cplx* c0 = nullptr;                 // P^H psi^0, nproj x nb
  cplx* cd = nullptr;                 // P^H K R^0
  std::vector<void*> mem;
};

struct pw_ham {
  pw_ctx* ctx = nullptr;
  BoxPlan plan{};
  FftLaunchCfg cfg{};
  int64_t npw = 0, nproj = 0, nb_max = 0;
  int64_t chunk = 0;         // bands per FFT launch (tunable, <= chunk_alloc)
  int64_t chunk_alloc = 0;   // bands the FFT work buffer holds
  int gemm_target = 4096;    // split-K target block count of the projector product (tunable;
                             // the FP64 product caps it at 2048)
  int nn_tile = 0;           // workgroup tile of the tall FP64 products P C, Y Q, Y U^-1 (tunable)
  int nn_tile32 = 0;         // the same for the FP32 / BF16 product P C (tunable)
  bool reg_col_ok = false, reg_plane_ok = false, narrow_ok = false, narrow32_ok = false;
  bool ls32_ok = false;      // FP32 plane kernel with LDS exchanges (square P^2 planes)
  std::vector<void*> allocs;
  double* kin = nullptr;
  double* vscaled = nullptr;
  double vmax = 0.0, kmax = 0.0;
  const cplx* proj = nullptr;
  double* ekb_dev = nullptr;
  std::vector<double> ekb;
  cplx* T = nullptr;
  cplx* cprj = nullptr;
  cplx* gemm_work = nullptr;
  cplx* blk = nullptr;
  cplx* sub0 = nullptr;
  cplx* sub1 = nullptr;
  void* heev_work = nullptr;
  int* status_dev = nullptr;
  cplx* dinv = nullptr;     // inverses of the Cholesky diagonal blocks
  cplx* panel = nullptr;    // kb x nb_max row panel
  double* dtol = nullptr;   // pivot threshold
  // low-precision filter path (allocated when desc->low_prec != 0)
  bool low_prec = false;
  float* kin32 = nullptr;
  float* vs32 = nullptr;
  float2* proj32 = nullptr;
  // proj32 split into three bf16 terms (launch_split3 layout) for the FP32
  // products: rows = plane waves (P C) and rows = projectors (P^H psi)
  uint16_t* proj3 = nullptr;
  uint16_t* proj3c = nullptr;
  uint16_t* cprj3 = nullptr;   // cprj32^T in three terms (rows = bands), written by P^H psi
  float2* T32 = nullptr;
  float2* cprj32 = nullptr;
  float2* work32 = nullptr;
  float2* gram32 = nullptr;    // nb_max^2 low-precision Gram matrix
  // projections P^H Y of the Ritz vectors of the last Rayleigh-Ritz-type call
  // (pw_rayleigh_ritz, pw_lobpcg, pw_rmm_diis), nproj x cprj_nb, ld nproj
  cplx* cprj_y = nullptr;
  int64_t cprj_nb = 0;
  float2* blk32[2] = {nullptr, nullptr};
  // electron density (allocated by the first pw_density call)
  double omega = 0.0;        // cell volume (2 pi)^3 / |det B|
  double* rho_part = nullptr;
  int rho_groups = 0;
  // eigensolver workspaces (allocated by the first pw_lobpcg / pw_rmm_diis call)
  LobpcgWork lob;
  RmmWork rmm;
};

namespace pwi {

extern thread_local std::string g_err;

pw_status fail(pw_ctx* c, pw_status s, const std::string& msg);


#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((ctx), PW_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

struct StageScope {
  pw_ctx* c;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageScope(pw_ctx* ctx, int st, hipStream_t on = nullptr)
      : c(ctx), stage(st), s(on ? on : ctx->stream) {
    if (c->timing) {
      a = c->get_event();
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~StageScope() {
    if (c->timing && a) {
      hipEvent_t b = c->get_event();
      if (b) {
        (void)hipEventRecord(b, s);
        c->pending.push_back({a, b, stage});
      } else {
        c->pool.push_back(a);
      }
    }
  }
};

template <class T>
pw_status dalloc(pw_ham* h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return PW_OK;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h->ctx, PW_ERR_OOM,
                "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  h->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return PW_OK;
}


void free_ham(pw_ham* h);
// Frees one allocation made by dalloc on h.
void dfree(pw_ham* h, void* p);
bool ranges_overlap(const void* a, int64_t lda, const void* b, int64_t ldb, int64_t rows,
                    int64_t cols, int64_t elem = (int64_t)sizeof(cplx));
bool spans_overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes);
pw_status check_block(pw_ham* h, const void* p, int64_t ld, const char* name);
pw_status check_hot(pw_ham* h, pw_prec prec, int64_t nb);
// out = alpha (H in) + beta in + gamma prev (FP64 blocks); coef (device,
// may be null) overrides the scalars.
// craw (may be null, nproj x nb, ld nproj) receives alpha P^H in, the
// projections before the KB energies scale them.
pw_status ham_apply(pw_ham* h, int64_t nb, const cplx* in, int64_t ldin, cplx* out, int64_t ldout,
                    double alpha, double beta, double gamma, const cplx* prev, int64_t ldprev,
                    const double* coef = nullptr, cplx* craw = nullptr);
pw_status rotate_block(pw_ham* h, int64_t nb, cplx* y, int64_t ld, const cplx* m);
// Hot calls that record a deferred status (pw_ctx_check names them).
enum DeferredOp { kOpOrtho = 1, kOpRayleighRitz = 2, kOpLobpcg = 3, kOpRmmDiis = 4, kOpHeev = 5 };
const char* op_name(int op);
inline int* sweeps_slot(pw_ctx* c) { return c->rec_dev + 4; }
hipError_t chol_blocked(int64_t n, cplx* a, int64_t lda, cplx* dinv, cplx* panel, double* tol,
                        int* status, hipStream_t s);
hipError_t trsm_right(int64_t rows, int64_t n, cplx* y, int64_t ld, const cplx* u, int64_t ldu,
                      const cplx* dinv, cplx* tmp, hipStream_t s, int tile = 0);
// cp (may be null, nproj x nb, ld nproj): projections P^H Y carried along,
// updated by the same triangular solves / rotation as Y (no product with P).
pw_status ortho_block(pw_ham* h, int64_t nb, cplx* y, int64_t ld, cplx* hy, int64_t ldhy, int op,
                      pw_prec gram_prec = PW_FP64, cplx* cp = nullptr);
pw_status subspace_rr(pw_ham* h, int64_t nb, cplx* y, int64_t ld, cplx* hy, int64_t ldhy, double* eig,
                      double* resid, int op, cplx* cp = nullptr);

}  // namespace pwi
