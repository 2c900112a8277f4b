// Host side of the C ABI (include/mrcqr.h): argument checks, plans and
// workspace layout, and the launch sequence of Algorithm 2.
#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"
#include "mrcqr.h"

namespace mrcqr {
hipError_t launch_regime_reset(Ctrl* ctrl, hipStream_t st);
hipError_t launch_draw(uint64_t seed, int m, int s, int32_t* S, int8_t* D, hipStream_t st, Ctrl* ctrl = nullptr,
                       int prec = 0, int auto_mode = 0);
hipError_t launch_sketch(int prec, const double* A, int64_t lda, int m, int n, const int32_t* S, int s,
                         uint64_t seed, void* Ypart, double* Y, int64_t ldy, const Ctrl* ctrl, int phase,
                         hipStream_t st);
size_t sketch_partial_bytes(int64_t m, int64_t n, int64_t s, int prec);
hipError_t launch_sketch_qr(bool f64, const double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                            double* kappa, Ctrl* ctrl, int slot, int phase, hipStream_t st);
bool qr_supported(int s, int n);
hipError_t launch_condest(const double* R, int n, int64_t ldr, double* kappa, hipStream_t st);
hipError_t launch_trsm(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr,
                       double* X, int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st);
size_t trsm_workspace_bytes(int n);
hipError_t launch_gram(const double* B, int m, int n, int64_t ldb, double* Gpart, double* G, int64_t ldg,
                       const Ctrl* ctrl, int phase, hipStream_t st);
size_t gram_partial_bytes(int64_t m, int64_t n);
hipError_t launch_cholesky(const double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                           double* kappa, Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_trmm(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int n, double* R,
                       int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_trinv(const double* R, int n, int64_t ldr, double* X, int64_t ldx, const Ctrl* ctrl, int phase,
                        hipStream_t st);
hipError_t launch_rc_tail(const double* Rc, int n, int64_t ldc, const double* Rs, int64_t ldrs, double* X, int64_t ldx,
                          double* R, int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_qform(const double* B, int m, int n, int64_t ldb, const double* X, int64_t ldx, double* Q,
                        int64_t ldq, const Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_ctrl_finalize(const Ctrl* ctrl, void* info, hipStream_t st);
}  // namespace mrcqr

using namespace mrcqr;

namespace {

constexpr int64_t NMAX = 128;
constexpr int64_t SMAX = 2048;
constexpr int64_t MMAX = (int64_t)1 << 28;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_prec(int p, bool allow_auto) {
  return (allow_auto && (p == MRCQR_PREC_AUTO || p == MRCQR_PREC_AUTO_CARRY)) || p == MRCQR_PREC_FP64 || p == MRCQR_PREC_FP32 ||
         p == MRCQR_PREC_FP16 || p == MRCQR_PREC_BF16;
}

// 0 = ok, else a status code
int check_shape(int64_t m, int64_t n, int64_t s) {
  if (n < 1 || m < n || s < n || s > m) return MRCQR_ERR_ARG;
  if (n > NMAX || s > SMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!qr_supported((int)s, (int)n)) return MRCQR_ERR_UNSUPPORTED;
  return MRCQR_OK;
}

hipStream_t as_stream(void* p) { return reinterpret_cast<hipStream_t>(p); }

int hip_status(hipError_t e) { return e == hipSuccess ? MRCQR_OK : MRCQR_ERR_DEVICE; }

}  // namespace

struct mrcqr_plan {
  int64_t m, n, s;
  size_t off_ctrl, off_S, off_Ypart, off_Y, off_Rs, off_Gpart, off_G, off_Rc, off_Rci, off_Tw, off_B, total;
};

static void plan_layout(mrcqr_plan* p) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  const size_t m = (size_t)p->m, n = (size_t)p->n, s = (size_t)p->s;
  p->off_ctrl = take(sizeof(Ctrl));
  p->off_S = take(s * sizeof(int32_t));
  p->off_Ypart = take(sketch_partial_bytes(p->m, p->n, p->s, P_FP64));
  p->off_Y = take(s * n * sizeof(double));
  p->off_Rs = take(n * n * sizeof(double));
  p->off_Gpart = take(gram_partial_bytes(p->m, p->n));
  p->off_G = take(n * n * sizeof(double));
  p->off_Rc = take(n * n * sizeof(double));
  p->off_Rci = take(n * n * sizeof(double));
  p->off_Tw = take(trsm_workspace_bytes((int)n));
  p->off_B = take(m * n * sizeof(double));
  p->total = o;
}

static int execute(const mrcqr_plan* p, char* ws, const double* A, int64_t lda, int prec, uint64_t seed,
                   double* Q, int64_t ldq, double* R, int64_t ldr, hipStream_t st, mrcqr_info* info) {
  const int m = (int)p->m, n = (int)p->n, s = (int)p->s;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + p->off_ctrl);
  int32_t* S = reinterpret_cast<int32_t*>(ws + p->off_S);
  void* Ypart = ws + p->off_Ypart;
  double* Y = reinterpret_cast<double*>(ws + p->off_Y);
  double* Rs = reinterpret_cast<double*>(ws + p->off_Rs);
  double* Gpart = reinterpret_cast<double*>(ws + p->off_Gpart);
  double* G = reinterpret_cast<double*>(ws + p->off_G);
  double* Rc = reinterpret_cast<double*>(ws + p->off_Rc);
  double* Rci = reinterpret_cast<double*>(ws + p->off_Rci);
  double* B = reinterpret_cast<double*>(ws + p->off_B);
  void* Tw = ws + p->off_Tw;
  const int64_t ldb = p->m;
  hipError_t e;
  const bool automode = prec == MRCQR_PREC_AUTO || prec == MRCQR_PREC_AUTO_CARRY;
  const int amode = prec == MRCQR_PREC_AUTO_CARRY ? AM_CARRY : automode ? AM_AUTO : AM_FIXED;
  if ((e = launch_draw(seed, m, s, S, nullptr, st, ctrl, automode ? P_FP16 : prec, amode)) != hipSuccess)
    return MRCQR_ERR_DEVICE;
  // The launch sequence is static: in AUTO every attempt is enqueued and
  // the kernels of an attempt whose precision is not the current one (or of
  // a rerun that was not requested) return immediately.
  auto stage1 = [&](int pp, int phase) -> bool {
    return launch_sketch(pp, A, lda, m, n, S, s, seed, Ypart, Y, s, ctrl, phase, st) == hipSuccess &&
           launch_sketch_qr(pp == P_FP64, Y, s, n, s, Rs, n, nullptr, ctrl, pp, phase, st) == hipSuccess;
  };
  auto stage2 = [&](int phase, int tail_phase) -> bool {
    return launch_trsm(A, m, n, lda, Rs, n, B, ldb, Tw, ctrl, phase, st) == hipSuccess &&
           launch_gram(B, m, n, ldb, Gpart, G, n, ctrl, phase, st) == hipSuccess &&
           launch_cholesky(G, n, n, Rc, n, nullptr, nullptr, ctrl, phase, st) == hipSuccess &&
           launch_rc_tail(Rc, n, n, Rs, n, Rci, n, R, ldr, ctrl, tail_phase, st) == hipSuccess &&
           launch_qform(B, m, n, ldb, Rci, n, Q, ldq, ctrl, tail_phase, st) == hipSuccess;
  };
  if (automode) {
    for (int pp : {P_FP16, P_FP32, P_FP64})
      if (!stage1(pp, PH_FIRST)) return MRCQR_ERR_DEVICE;
    if (!stage2(PH_FIRST, PH_FIRST_TAIL)) return MRCQR_ERR_DEVICE;
    // rerun pass, enabled on the device by the posterior check
    for (int pp : {P_FP32, P_FP64})
      if (!stage1(pp, PH_RERUN)) return MRCQR_ERR_DEVICE;
    if (!stage2(PH_RERUN, PH_RERUN)) return MRCQR_ERR_DEVICE;
  } else {
    if (!stage1(prec, PH_FIRST)) return MRCQR_ERR_DEVICE;
    if (!stage2(PH_FIRST, PH_FIRST)) return MRCQR_ERR_DEVICE;
  }
  if (info && (e = launch_ctrl_finalize(ctrl, info, st)) != hipSuccess) return MRCQR_ERR_DEVICE;
  return MRCQR_OK;
}

static int check_factor_args(const double* A, int64_t m, int64_t n, int64_t lda, int prec, int64_t s,
                             const double* Q, int64_t ldq, const double* R, int64_t ldr) {
  if (!A || !Q || !R) return MRCQR_ERR_ARG;
  if (!valid_prec(prec, true)) return MRCQR_ERR_ARG;
  const int c = check_shape(m, n, s);
  if (c) return c;
  if (lda < m || ldq < m || ldr < n) return MRCQR_ERR_ARG;
  if (A == Q) return MRCQR_ERR_ARG;
  return MRCQR_OK;
}

// ---- plan cache for mrcqr_factor ----
namespace {
struct CacheEntry { mrcqr_plan plan; void* ws; };
std::mutex g_mu;
std::map<std::tuple<int, int64_t, int64_t, int64_t>, CacheEntry> g_cache;
}  // namespace

extern "C" {

int mrcqr_plan_create(int64_t m, int64_t n, int64_t s, mrcqr_plan** out) {
  if (!out) return MRCQR_ERR_ARG;
  if (s == 0) s = 2 * n;
  const int c = check_shape(m, n, s);
  if (c) return c;
  mrcqr_plan* p = new mrcqr_plan();
  p->m = m; p->n = n; p->s = s;
  plan_layout(p);
  *out = p;
  return MRCQR_OK;
}

size_t mrcqr_plan_workspace_bytes(const mrcqr_plan* plan) { return plan ? plan->total : 0; }

int mrcqr_plan_destroy(mrcqr_plan* plan) {
  delete plan;
  return MRCQR_OK;
}

int mrcqr_execute(const mrcqr_plan* plan, void* workspace, size_t workspace_bytes, const double* A,
                  int64_t lda, int sketch_precision, uint64_t seed, double* Q, int64_t ldq, double* R,
                  int64_t ldr, void* stream, mrcqr_info* info_dev) {
  if (!plan) return MRCQR_ERR_ARG;
  const int c = check_factor_args(A, plan->m, plan->n, lda, sketch_precision, plan->s, Q, ldq, R, ldr);
  if (c) return c;
  if (!workspace || workspace_bytes < plan->total) return MRCQR_ERR_WORKSPACE;
  return execute(plan, static_cast<char*>(workspace), A, lda, sketch_precision, seed, Q, ldq, R, ldr,
                 as_stream(stream), info_dev);
}

int mrcqr_regime_reset(const mrcqr_plan* plan, void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return MRCQR_ERR_ARG;
  if (!workspace || workspace_bytes < plan->total) return MRCQR_ERR_WORKSPACE;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(static_cast<char*>(workspace) + plan->off_ctrl);
  return hip_status(launch_regime_reset(ctrl, as_stream(stream)));
}

int mrcqr_factor(const double* A, int64_t m, int64_t n, int64_t lda, int sketch_precision, uint64_t seed,
                 int64_t s, double* Q, int64_t ldq, double* R, int64_t ldr, void* stream, mrcqr_info* info_dev) {
  if (s == 0) s = 2 * n;
  const int c = check_factor_args(A, m, n, lda, sketch_precision, s, Q, ldq, R, ldr);
  if (c) return c;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MRCQR_ERR_DEVICE;
  CacheEntry* ent = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(dev, m, n, s);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) {
      CacheEntry ce;
      ce.plan.m = m; ce.plan.n = n; ce.plan.s = s;
      plan_layout(&ce.plan);
      if (hipMalloc(&ce.ws, ce.plan.total) != hipSuccess) return MRCQR_ERR_DEVICE;
      // no AUTO_CARRY record yet: the control block starts as zero bytes
      if (hipMemset(ce.ws, 0, sizeof(Ctrl)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(ce.ws);
        return MRCQR_ERR_DEVICE;
      }
      it = g_cache.emplace(key, ce).first;
    }
    ent = &it->second;
  }
  return execute(&ent->plan, static_cast<char*>(ent->ws), A, lda, sketch_precision, seed, Q, ldq, R, ldr,
                 as_stream(stream), info_dev);
}

int mrcqr_factor_batched(int32_t batch, const double* const* A, const int64_t* m, const int64_t* n,
                         const int64_t* lda, const int32_t* precision, const uint64_t* seeds,
                         double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr,
                         void* stream, mrcqr_info* infos_dev) {
  if (batch < 0 || (batch > 0 && (!A || !m || !n || !lda || !precision || !seeds || !Q || !ldq || !R || !ldr)))
    return MRCQR_ERR_ARG;
  for (int32_t i = 0; i < batch; ++i) {
    const int c = check_factor_args(A[i], m[i], n[i], lda[i], precision[i], 2 * n[i], Q[i], ldq[i], R[i], ldr[i]);
    if (c) return c;
  }
  for (int32_t i = 0; i < batch; ++i) {
    const int c = mrcqr_factor(A[i], m[i], n[i], lda[i], precision[i], seeds[i], 0, Q[i], ldq[i], R[i], ldr[i],
                               stream, infos_dev ? infos_dev + i : nullptr);
    if (c) return c;
  }
  return MRCQR_OK;
}

int mrcqr_draw(uint64_t seed, int64_t m, int64_t s, int32_t* S_dev, int8_t* D_dev, void* stream) {
  if (!S_dev || s < 1 || s > m || s > SMAX || m >= MMAX) return MRCQR_ERR_ARG;
  return hip_status(launch_draw(seed, (int)m, (int)s, S_dev, D_dev, as_stream(stream)));
}

size_t mrcqr_sketch_workspace_bytes(int64_t m, int64_t n, int64_t s, int precision) {
  if (m < 1 || n < 1 || s < 1) return 0;
  return sketch_partial_bytes(m, n, s, precision == MRCQR_PREC_FP64 ? P_FP64 : P_FP32);
}

int mrcqr_sketch(const double* A, int64_t m, int64_t n, int64_t lda, const int32_t* S_dev, int64_t s,
                 uint64_t seed, int precision, double* Y, int64_t ldy, void* workspace, size_t workspace_bytes,
                 void* stream) {
  if (!A || !S_dev || !Y || !valid_prec(precision, false)) return MRCQR_ERR_ARG;
  if (n < 1 || m < 1 || s < 1 || s > m || lda < m || ldy < s) return MRCQR_ERR_ARG;
  if (m >= MMAX || s > SMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < mrcqr_sketch_workspace_bytes(m, n, s, precision)) return MRCQR_ERR_WORKSPACE;
  return hip_status(launch_sketch(precision, A, lda, (int)m, (int)n, S_dev, (int)s, seed, workspace, Y, ldy,
                                  nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_sketch_qr(const double* Y, int64_t s, int64_t n, int64_t ldy, int qr_precision, double* Rs,
                    int64_t ldr, double* kappa_dev, void* stream) {
  if (!Y || !Rs || n < 1 || s < n || ldy < s || ldr < n) return MRCQR_ERR_ARG;
  if (qr_precision != MRCQR_PREC_FP32 && qr_precision != MRCQR_PREC_FP64) return MRCQR_ERR_ARG;
  if (n > NMAX || !qr_supported((int)s, (int)n)) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_sketch_qr(qr_precision == MRCQR_PREC_FP64, Y, (int)s, (int)n, ldy, Rs, ldr, kappa_dev,
                                     nullptr, P_AUTO, PH_FIRST, as_stream(stream)));
}

size_t mrcqr_trsm_workspace_bytes(int64_t n) {
  if (n < 1 || n > NMAX) return 0;
  return trsm_workspace_bytes((int)n);
}

int mrcqr_trsm(const double* A, int64_t m, int64_t n, int64_t lda, const double* R, int64_t ldr, double* X,
               int64_t ldx, void* workspace, size_t workspace_bytes, void* stream) {
  if (!A || !R || !X || m < 1 || n < 1 || lda < m || ldr < n || ldx < m || A == X) return MRCQR_ERR_ARG;
  if (n > NMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < trsm_workspace_bytes((int)n)) return MRCQR_ERR_WORKSPACE;
  return hip_status(launch_trsm(A, (int)m, (int)n, lda, R, ldr, X, ldx, workspace, nullptr, PH_FIRST,
                                as_stream(stream)));
}

size_t mrcqr_gram_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1) return 0;
  return gram_partial_bytes(m, n);
}

int mrcqr_gram(const double* B, int64_t m, int64_t n, int64_t ldb, double* G, int64_t ldg, void* workspace,
               size_t workspace_bytes, void* stream) {
  if (!B || !G || m < 1 || n < 1 || ldb < m || ldg < n) return MRCQR_ERR_ARG;
  if (n > NMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < gram_partial_bytes(m, n)) return MRCQR_ERR_WORKSPACE;
  return hip_status(launch_gram(B, (int)m, (int)n, ldb, static_cast<double*>(workspace), G, ldg, nullptr,
                                PH_FIRST, as_stream(stream)));
}

int mrcqr_cholesky(const double* G, int64_t n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail_dev,
                   double* kappa_dev, void* stream) {
  if (!G || !Rc || n < 1 || ldg < n || ldr < n) return MRCQR_ERR_ARG;
  if (n > NMAX) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_cholesky(G, (int)n, ldg, Rc, ldr, fail_dev, kappa_dev, nullptr, PH_FIRST,
                                    as_stream(stream)));
}

int mrcqr_trmm(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int64_t n, double* R, int64_t ldr,
               void* stream) {
  if (!R2 || !R1 || !R || n < 1 || ld2 < n || ld1 < n || ldr < n) return MRCQR_ERR_ARG;
  if (n > 4096) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_trmm(R2, ld2, R1, ld1, (int)n, R, ldr, nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_tri_inverse(const double* R, int64_t n, int64_t ldr, double* X, int64_t ldx, void* stream) {
  if (!R || !X || n < 1 || ldr < n || ldx < n || R == X) return MRCQR_ERR_ARG;
  if (n > NMAX) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_trinv(R, (int)n, ldr, X, ldx, nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_form_q(const double* B, int64_t m, int64_t n, int64_t ldb, const double* X, int64_t ldx, double* Q,
                 int64_t ldq, void* stream) {
  if (!B || !X || !Q || m < 1 || n < 1 || ldb < m || ldx < n || ldq < m || B == Q) return MRCQR_ERR_ARG;
  if (n > NMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_qform(B, (int)m, (int)n, ldb, X, ldx, Q, ldq, nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_condest(const double* R, int64_t n, int64_t ldr, double* kappa_dev, void* stream) {
  if (!R || !kappa_dev || n < 1 || ldr < n) return MRCQR_ERR_ARG;
  if (n > NMAX) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_condest(R, (int)n, ldr, kappa_dev, as_stream(stream)));
}

const char* mrcqr_status_string(int status) {
  switch (status) {
    case MRCQR_OK: return "ok";
    case MRCQR_ERR_ARG: return "invalid argument";
    case MRCQR_ERR_NONFINITE: return "non-finite value in the sketch";
    case MRCQR_ERR_CHOL_BREAKDOWN: return "Cholesky breakdown (Gram matrix not numerically positive definite)";
    case MRCQR_ERR_SKETCH_SINGULAR: return "sketch factor Rs is singular or not finite";
    case MRCQR_ERR_WORKSPACE: return "workspace missing or too small";
    case MRCQR_ERR_DEVICE: return "HIP runtime error";
    case MRCQR_WARN_POSTERIOR: return "posterior check: kappa(Rc) above bound, sketch precision too low";
    case MRCQR_ERR_UNSUPPORTED: return "shape not supported by this build";
    default: return "unknown status";
  }
}

int mrcqr_version(void) { return 100; }

}  // extern "C"
