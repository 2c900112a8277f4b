// Host side of the C ABI (include/mrcqr.h): argument checks, plans and
// workspace layout, and the launch sequence of Algorithm 2.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <vector>
#include <mutex>
#include <tuple>

#include "batch.hpp"
#include "mrcqr.h"

namespace mrcqr {
hipError_t launch_regime_reset(Ctrl* ctrl, hipStream_t st);
hipError_t launch_draw(uint64_t seed, int m, int s, int32_t* S, int8_t* D, hipStream_t st, Ctrl* ctrl = nullptr,
                       int prec = 0, int auto_mode = 0);
hipError_t launch_sketch(int prec, const double* A, int64_t lda, int m, int n, const int32_t* S, int s,
                         uint64_t seed, void* Ypart, double* Y, int64_t ldy, const Ctrl* ctrl, int phase,
                         hipStream_t st, int xform);
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
hipError_t launch_posterior(const double* Rc, const double* X, int n, int64_t ld, Ctrl* ctrl, int phase,
                            double* kappa_out, hipStream_t st);
hipError_t launch_posterior_grouped(const BatchInst* bi, const int32_t* members, int count, const BatchCall& call,
                                    int phase, hipStream_t st);
hipError_t launch_ctrl_finalize(const Ctrl* ctrl, void* info, hipStream_t st);
hipError_t launch_cholqr2_finalize(const int32_t* fail, void* info, hipStream_t st);
hipError_t launch_onenorm_condest(const double* R, const double* G, int n, int64_t ld, uint64_t seed,
                                  double* kappa, hipStream_t st);
size_t probe_workspace_bytes(int64_t m, int64_t n);
hipError_t launch_cholqr_probe(const double* A, int m, int n, int64_t lda, void* ws, double* kappa,
                               hipStream_t st);
// grouped launches over the members of a batch
hipError_t launch_draw_grouped(const BatchInst* bi, const int32_t* members, int count, int max_s,
                               const BatchCall& call, hipStream_t st);
int sketch_variant(int n, int s);
hipError_t launch_sketch_grouped(int prec, int variant, const BatchInst* bi, const int32_t* members, int count,
                                 int max_chunks, int64_t max_ns, const BatchCall& call, int phase, hipStream_t st);
int qr_group_key(bool f64, int s, int n);
hipError_t launch_sketch_qr_grouped(bool f64, int key, const BatchInst* bi, const int32_t* members, int count,
                                    int max_n, const BatchCall& call, int slot, int phase, hipStream_t st);
int trsm_batch_blocks(int64_t m);
int trsm_prep_elems(int n);
hipError_t launch_trsm_grouped(int nmax, const BatchInst* bi, const int32_t* members, int count, int max_elems,
                               int max_blocks, const BatchCall& call, int phase, hipStream_t st);
int gram_batch_chunks(int64_t m);
int syrk_variant(int n);
hipError_t launch_gram_grouped(int variant, const BatchInst* bi, const int32_t* members, int count, int max_chunks,
                               int max_n, const BatchCall& call, int phase, hipStream_t st);
hipError_t launch_cholesky_grouped(const BatchInst* bi, const int32_t* members, int count, const BatchCall& call,
                                   int phase, hipStream_t st);
hipError_t launch_rc_tail_grouped(const BatchInst* bi, const int32_t* members, int count, int max_n,
                                  const BatchCall& call, int phase, hipStream_t st);
int qform_batch_blocks(int64_t m);
hipError_t launch_qform_grouped(int nb, const BatchInst* bi, const int32_t* members, int count, int max_blocks,
                                const BatchCall& call, int phase, hipStream_t st);
hipError_t launch_finalize_grouped(const BatchInst* bi, const int32_t* members, int count, const BatchCall& call,
                                   hipStream_t st);
struct SketchGeom { int chunks, rows_per_chunk; };
SketchGeom sketch_geometry(int64_t m);
// the column-panel path for 128 < n <= 512 (csrc/wide.hip)
hipError_t launch_sketch_qr_wide(bool f64, double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                                 double* tau, int* flags, double* Rt, double* kappa, Ctrl* ctrl, int slot, int phase,
                                 hipStream_t st);
hipError_t launch_trsm_wide(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr, double* X,
                            int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st);
size_t gram_pair_partial_bytes(int n);
hipError_t launch_gram_wide(const double* B, int m, int n, int64_t ldb, double* Gpart_diag, double* Gpart_pairs,
                            double* G, int64_t ldg, const Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_cholesky_wide(double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                                double* kappa, double* T, int32_t* fails, double* Rt, void* Tw, Ctrl* ctrl, int phase,
                                hipStream_t st);
hipError_t launch_rc_tail_wide(const double* Rc, int n, int64_t ldc, const double* Rs, int64_t lds_, double* X,
                               int64_t ldx, double* R, int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_trinv_wide(const double* R, int n, int64_t ldr, double* X, int64_t ldx, const Ctrl* ctrl, int phase,
                             hipStream_t st);
hipError_t launch_trmm_wide(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int n, double* R,
                            int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_posterior_wide(const double* Rc, const double* X, int n, int64_t ld, double* ws, Ctrl* ctrl,
                                 int phase, double* kappa_out, hipStream_t st);
size_t posterior_wide_ws_bytes();
hipError_t launch_qform_wide(const double* B, int m, int n, int64_t ldb, const double* X, int64_t ldx, double* Q,
                             int64_t ldq, const Ctrl* ctrl, int phase, hipStream_t st);
}  // namespace mrcqr

using namespace mrcqr;

namespace {

constexpr int64_t NMAX = 512;   // whole factorization; 128 < n <= 512 takes the column-panel path
constexpr int64_t NSTEP = 128;  // single-kernel steps (Cholesky, CholQR2, the estimators, batches)
constexpr int64_t SMAX = 2048;
constexpr int64_t SWIDE = 1024; // sketch rows of the column-panel sketch QR
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
  if (n > NSTEP ? s > SWIDE : !qr_supported((int)s, (int)n)) return MRCQR_ERR_UNSUPPORTED;
  return MRCQR_OK;
}

hipStream_t as_stream(void* p) { return reinterpret_cast<hipStream_t>(p); }

int hip_status(hipError_t e) { return e == hipSuccess ? MRCQR_OK : MRCQR_ERR_DEVICE; }

}  // namespace

struct mrcqr_plan {
  int64_t m, n, s;
  int xform = 0;  // 0: DCT-II sketch; 1: real part of the DFT (MRCQR_SKETCH_RFFT)
  size_t off_ctrl, off_S, off_Ypart, off_Y, off_Rs, off_Gpart, off_G, off_Rc, off_Rci, off_Tw, off_B, total;
  // column-panel path (n > 128): Householder tau and flags, the Gram's
  // partials of the blocks above the diagonal, the Cholesky's panel and
  // per-panel pivots
  size_t off_tau = 0, off_flags = 0, off_Gpair = 0, off_T = 0, off_fails = 0;
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
  const bool wide = p->n > NSTEP;
  p->off_Gpart = take(gram_partial_bytes(p->m, wide ? NSTEP : p->n));
  p->off_G = take(n * n * sizeof(double));
  p->off_Rc = take(n * n * sizeof(double));
  p->off_Rci = take(n * n * sizeof(double));
  p->off_Tw = take(trsm_workspace_bytes((int)std::min<int64_t>(p->n, NSTEP)));
  if (wide) {
    p->off_tau = take(n * sizeof(double));
    p->off_flags = take(sizeof(int));
    // also the row-major copies of Rs and Rc for their condition estimates
    p->off_Gpair = take(std::max(gram_pair_partial_bytes((int)n), n * n * sizeof(double)));
    p->off_T = take(n * NSTEP * sizeof(double));
    p->off_fails = take(8 * sizeof(int32_t));
  }
  p->off_B = take(m * n * sizeof(double));
  p->total = o;
}

// A second stream per (device, caller stream) for the posterior check of a
// fixed-precision call with n > 128: there the check (two launches per
// power step over many workgroups) decides nothing that the product
// Q = B Rc^{-1} depends on (no rerun), so it runs beside the product
// (fork after Rc^{-1}, join before the info is written). Created on the
// first call from a stream that is not being captured and kept for the
// process; calls under capture without one take the serial sequence.
struct SideStream {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
static std::mutex g_side_mu;
static std::map<std::pair<int, hipStream_t>, SideStream> g_side;

static const SideStream* side_stream_for(hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_side_mu);
  auto key = std::make_pair(dev, st);
  auto it = g_side.find(key);
  if (it != g_side.end()) return &it->second;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  SideStream ss;
  if (hipStreamCreateWithFlags(&ss.side, hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) != hipSuccess) {
    if (ss.fork) (void)hipEventDestroy(ss.fork);
    (void)hipStreamDestroy(ss.side);
    return nullptr;
  }
  return &g_side.emplace(key, ss).first->second;
}

static int execute(const mrcqr_plan* p, char* ws, const double* A, int64_t lda, int prec, uint64_t seed,
                   double* Q, int64_t ldq, double* R, int64_t ldr, hipStream_t st, mrcqr_info* info,
                   bool allow_fork = true) {
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
  // the DFT variant samples the floor(m/2) + 1 distinct bins of a real signal
  const int mdraw = p->xform ? m / 2 + 1 : m;
  if ((e = launch_draw(seed, mdraw, s, S, nullptr, st, ctrl, automode ? P_FP16 : prec, amode)) != hipSuccess)
    return MRCQR_ERR_DEVICE;
  // The launch sequence is static: in AUTO every attempt is enqueued and
  // the kernels of an attempt whose precision is not the current one (or of
  // a rerun that was not requested) return immediately.
  auto stage1 = [&](int pp, int phase) -> bool {
    if (launch_sketch(pp, A, lda, m, n, S, s, seed, Ypart, Y, s, ctrl, phase, st, p->xform) != hipSuccess)
      return false;
    if (n > NSTEP)
      // the Gram's pair partials are free until the Gram: Rs's row-major copy
      return launch_sketch_qr_wide(pp == P_FP64, Y, s, n, s, Rs, n, reinterpret_cast<double*>(ws + p->off_tau),
                                   reinterpret_cast<int*>(ws + p->off_flags),
                                   reinterpret_cast<double*>(ws + p->off_Gpair), nullptr, ctrl, pp, phase,
                                   st) == hipSuccess;
    return launch_sketch_qr(pp == P_FP64, Y, s, n, s, Rs, n, nullptr, ctrl, pp, phase, st) == hipSuccess;
  };
  // Stage 2 and 3 of one pass; Q is formed in the pass's tail phase, which
  // is skipped when the posterior check asks for a rerun
  // side: the posterior check runs there beside Q (fixed precision only)
  auto stage2 = [&](int phase, int tail_phase, const SideStream* side = nullptr) -> bool {
    const hipStream_t pst = side ? side->side : st;
    auto fork = [&]() -> bool {
      return !side || (hipEventRecord(side->fork, st) == hipSuccess && hipStreamWaitEvent(pst, side->fork, 0) == hipSuccess);
    };
    auto join = [&]() -> bool {
      return !side || (hipEventRecord(side->join, pst) == hipSuccess && hipStreamWaitEvent(st, side->join, 0) == hipSuccess);
    };
    if (n > NSTEP)
      return launch_trsm_wide(A, m, n, lda, Rs, n, B, ldb, Tw, ctrl, phase, st) == hipSuccess &&
             launch_gram_wide(B, m, n, ldb, Gpart, reinterpret_cast<double*>(ws + p->off_Gpair), G, n, ctrl, phase,
                              st) == hipSuccess &&
             launch_cholesky_wide(G, n, n, Rc, n, nullptr, nullptr, reinterpret_cast<double*>(ws + p->off_T),
                                  reinterpret_cast<int32_t*>(ws + p->off_fails),
                                  reinterpret_cast<double*>(ws + p->off_Gpair), Tw, ctrl, phase, st) == hipSuccess &&
             launch_rc_tail_wide(Rc, n, n, Rs, n, Rci, n, R, ldr, ctrl, phase, st) == hipSuccess && fork() &&
             launch_posterior_wide(Rc, Rci, n, n, reinterpret_cast<double*>(ws + p->off_T), ctrl, phase, nullptr,
                                   pst) == hipSuccess &&
             launch_qform_wide(B, m, n, ldb, Rci, n, Q, ldq, ctrl, tail_phase, st) == hipSuccess && join();
    return launch_trsm(A, m, n, lda, Rs, n, B, ldb, Tw, ctrl, phase, st) == hipSuccess &&
           launch_gram(B, m, n, ldb, Gpart, G, n, ctrl, phase, st) == hipSuccess &&
           launch_cholesky(G, n, n, Rc, n, nullptr, nullptr, ctrl, phase, st) == hipSuccess &&
           launch_rc_tail(Rc, n, n, Rs, n, Rci, n, R, ldr, ctrl, phase, st) == hipSuccess && fork() &&
           launch_posterior(Rc, Rci, n, n, ctrl, phase, nullptr, pst) == hipSuccess &&
           launch_qform(B, m, n, ldb, Rci, n, Q, ldq, ctrl, tail_phase, st) == hipSuccess && join();
  };
  if (automode) {
    for (int pp : {P_FP16, P_FP32, P_FP64})
      if (!stage1(pp, PH_FIRST)) return MRCQR_ERR_DEVICE;
    if (!stage2(PH_FIRST, PH_FIRST_TAIL)) return MRCQR_ERR_DEVICE;
    // rerun passes, enabled on the device by the posterior check (at most
    // two: FP16 -> FP32 -> FP64)
    for (int pp : {P_FP32, P_FP64})
      if (!stage1(pp, PH_RERUN)) return MRCQR_ERR_DEVICE;
    if (!stage2(PH_RERUN, PH_RERUN_TAIL)) return MRCQR_ERR_DEVICE;
    if (!stage1(P_FP64, PH_RERUN2)) return MRCQR_ERR_DEVICE;
    if (!stage2(PH_RERUN2, PH_RERUN2)) return MRCQR_ERR_DEVICE;
  } else {
    if (!stage1(prec, PH_FIRST)) return MRCQR_ERR_DEVICE;
    // n <= 128: the check is one workgroup and the product fills every
    // compute unit, so the fork gains nothing there (measured)
    if (!stage2(PH_FIRST, PH_FIRST, allow_fork && n > NSTEP ? side_stream_for(st) : nullptr))
      return MRCQR_ERR_DEVICE;
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

// ---- batches: grouped launches (one per step and kernel configuration) ----
struct BatchGroup {
  int off = 0, count = 0, key = 0, max_a = 0, max_b = 0;
};

struct mrcqr_batch_plan {
  int32_t batch = 0;
  size_t total = 0;
  BatchInst* d_inst = nullptr;
  int32_t* d_members = nullptr;
  BatchGroup all;
  std::vector<BatchGroup> qr32, qr64, trsm, qform, sketch, gram;
  int max_s = 0, max_n = 0;
};

static void batch_plan_free(mrcqr_batch_plan* p) {
  if (!p) return;
  if (p->d_inst) (void)hipFree(p->d_inst);
  if (p->d_members) (void)hipFree(p->d_members);
  delete p;
}

static int batch_plan_build(int32_t batch, const int64_t* m, const int64_t* n, mrcqr_batch_plan** out) {
  if (!out || batch < 1 || !m || !n) return MRCQR_ERR_ARG;
  if (batch > 65535) return MRCQR_ERR_UNSUPPORTED;  // members index grid.y
  std::vector<BatchInst> inst(batch);
  std::vector<int32_t> members;
  std::map<int, std::vector<int32_t>> g32, g64, gtr, gqf, gsk, ggr;
  mrcqr_batch_plan* p = new mrcqr_batch_plan();
  p->batch = batch;
  size_t o = 0;
  for (int32_t i = 0; i < batch; ++i) {
    const int64_t s = 2 * n[i];
    int c = check_shape(m[i], n[i], s);
    if (!c && n[i] > NSTEP) c = MRCQR_ERR_UNSUPPORTED;  // batches run the single-kernel steps
    if (c) { batch_plan_free(p); return c; }
    mrcqr_plan pl;
    pl.m = m[i]; pl.n = n[i]; pl.s = s;
    plan_layout(&pl);
    BatchInst& d = inst[i];
    d.m = (int32_t)m[i]; d.n = (int32_t)n[i]; d.s = (int32_t)s;
    const SketchGeom gg = sketch_geometry(m[i]);
    d.sk_chunks = gg.chunks; d.sk_rows = gg.rows_per_chunk;
    d.gram_chunks = gram_batch_chunks(m[i]);
    d.trsm_blocks = trsm_batch_blocks(m[i]);
    d.qform_blocks = qform_batch_blocks(m[i]);
    d.ws = o;
    d.off_ctrl = pl.off_ctrl; d.off_S = pl.off_S; d.off_Ypart = pl.off_Ypart; d.off_Y = pl.off_Y;
    d.off_Rs = pl.off_Rs; d.off_Gpart = pl.off_Gpart; d.off_G = pl.off_G; d.off_Rc = pl.off_Rc;
    d.off_Rci = pl.off_Rci; d.off_Tw = pl.off_Tw; d.off_B = pl.off_B;
    o = align_up(o + pl.total);
    const int k32 = qr_group_key(false, d.s, d.n), k64 = qr_group_key(true, d.s, d.n);
    if (k32 < 0 || k64 < 0) { batch_plan_free(p); return MRCQR_ERR_UNSUPPORTED; }
    g32[k32].push_back(i);
    g64[k64].push_back(i);
    gtr[d.n <= 32 ? 32 : (d.n <= 64 ? 64 : 128)].push_back(i);
    gqf[(d.n + 15) / 16].push_back(i);
    gsk[sketch_variant(d.n, d.s)].push_back(i);
    ggr[syrk_variant(d.n)].push_back(i);
    p->max_s = std::max(p->max_s, d.s);
    p->max_n = std::max(p->max_n, d.n);
  }
  p->total = o;
  p->all.off = 0;
  p->all.count = batch;
  for (int32_t i = 0; i < batch; ++i) members.push_back(i);
  auto add_groups = [&](std::map<int, std::vector<int32_t>>& g, std::vector<BatchGroup>& dst, int kind) {
    for (auto& kv : g) {
      BatchGroup bg;
      bg.off = (int)members.size();
      bg.count = (int)kv.second.size();
      bg.key = kv.first;
      for (int32_t i : kv.second) {
        members.push_back(i);
        const BatchInst& d = inst[i];
        if (kind == 0) bg.max_a = std::max(bg.max_a, d.n);                   // sketch QR: LDS for the largest n
        if (kind == 1) { bg.max_a = std::max(bg.max_a, trsm_prep_elems(d.n)); bg.max_b = std::max(bg.max_b, d.trsm_blocks); }
        if (kind == 2) bg.max_b = std::max(bg.max_b, d.qform_blocks);
        if (kind == 3) { bg.max_a = std::max(bg.max_a, d.sk_chunks); bg.max_b = std::max(bg.max_b, d.n * d.s); }
        if (kind == 4) { bg.max_a = std::max(bg.max_a, d.gram_chunks); bg.max_b = std::max(bg.max_b, d.n); }
      }
      dst.push_back(bg);
    }
  };
  add_groups(g32, p->qr32, 0);
  add_groups(g64, p->qr64, 0);
  add_groups(gtr, p->trsm, 1);
  add_groups(gqf, p->qform, 2);
  add_groups(gsk, p->sketch, 3);
  add_groups(ggr, p->gram, 4);
  if (hipMalloc(&p->d_inst, inst.size() * sizeof(BatchInst)) != hipSuccess ||
      hipMalloc(&p->d_members, members.size() * sizeof(int32_t)) != hipSuccess ||
      hipMemcpy(p->d_inst, inst.data(), inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_members, members.data(), members.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
    batch_plan_free(p);
    return MRCQR_ERR_DEVICE;
  }
  *out = p;
  return MRCQR_OK;
}

// The static launch sequence of the single factorization, each step as one
// grouped launch per kernel configuration; every member follows its own
// control block (precision, escalation, rerun) on the device.
static int batch_execute(const mrcqr_batch_plan* p, const BatchCall& call, hipStream_t st) {
  const BatchInst* bi = p->d_inst;
  const int32_t* all = p->d_members + p->all.off;
  const int nb = p->batch;
  bool ok = launch_draw_grouped(bi, all, nb, p->max_s, call, st) == hipSuccess;
  auto stage1 = [&](int pp, int phase) {
    for (const BatchGroup& g : p->sketch)
      ok = ok && launch_sketch_grouped(pp, g.key, bi, p->d_members + g.off, g.count, g.max_a, g.max_b, call, phase,
                                       st) == hipSuccess;
    for (const BatchGroup& g : (pp == P_FP64 ? p->qr64 : p->qr32))
      ok = ok && launch_sketch_qr_grouped(pp == P_FP64, g.key, bi, p->d_members + g.off, g.count, g.max_a, call, pp,
                                          phase, st) == hipSuccess;
  };
  auto stage2 = [&](int phase, int tail) {
    for (const BatchGroup& g : p->trsm)
      ok = ok && launch_trsm_grouped(g.key, bi, p->d_members + g.off, g.count, g.max_a, g.max_b, call, phase, st) ==
                     hipSuccess;
    for (const BatchGroup& g : p->gram)
      ok = ok && launch_gram_grouped(g.key, bi, p->d_members + g.off, g.count, g.max_a, g.max_b, call, phase, st) ==
                     hipSuccess;
    ok = ok && launch_cholesky_grouped(bi, all, nb, call, phase, st) == hipSuccess;
    ok = ok && launch_rc_tail_grouped(bi, all, nb, p->max_n, call, phase, st) == hipSuccess;
    ok = ok && launch_posterior_grouped(bi, all, nb, call, phase, st) == hipSuccess;
    for (const BatchGroup& g : p->qform)
      ok = ok && launch_qform_grouped(g.key, bi, p->d_members + g.off, g.count, g.max_b, call, tail, st) == hipSuccess;
  };
  for (int pp : {P_FP16, P_BF16, P_FP32, P_FP64}) stage1(pp, PH_FIRST);
  stage2(PH_FIRST, PH_FIRST_TAIL);
  for (int pp : {P_FP32, P_FP64}) stage1(pp, PH_RERUN);
  stage2(PH_RERUN, PH_RERUN_TAIL);
  stage1(P_FP64, PH_RERUN2);
  stage2(PH_RERUN2, PH_RERUN2);
  if (call.info) ok = ok && launch_finalize_grouped(bi, all, nb, call, st) == hipSuccess;
  return ok ? MRCQR_OK : MRCQR_ERR_DEVICE;
}

// ---- plan cache for mrcqr_factor ----
// One workspace per (device, m, n, s). Calls of one shape are serialized on
// the device: each call's stream waits for the previous call's completion
// event on that workspace before its first kernel (no host wait), so calls
// from different streams or host threads never overlap on it. The entries
// live until mrcqr_release_cache().
namespace {
struct CacheEntry {
  mrcqr_plan plan;
  void* ws = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
  std::mutex mu;
};
std::mutex g_mu;
std::map<std::tuple<int, int64_t, int64_t, int64_t>, std::unique_ptr<CacheEntry>> g_cache;
// mrcqr_factor_batched: plan, workspace and per-call argument arrays per
// (device, shape list)
struct BatchEntry {
  mrcqr_batch_plan* plan = nullptr;
  void* ws = nullptr;
  void* params = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
};
std::mutex g_batch_mu;
std::map<std::vector<int64_t>, BatchEntry> g_batch_cache;

// Workspace of mrcqr_factor_noalloc: a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends. Host code
// never uses the array's name as an address: the first call on a device
// looks up that device's copy with hipGetSymbolAddress and keeps it.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The calling thread's current device's copy of `scratch` (nullptr on error).
void* scratch_for_device(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}
}  // namespace

extern "C" {

int mrcqr_plan_create_ex(int64_t m, int64_t n, int64_t s, int flags, mrcqr_plan** out) {
  if (!out || (flags & ~MRCQR_SKETCH_RFFT) != 0) return MRCQR_ERR_ARG;
  const bool rfft = (flags & MRCQR_SKETCH_RFFT) != 0;
  if (s == 0) s = rfft ? 3 * n : 2 * n;
  const int c = check_shape(m, n, s);
  if (c) return c;
  if (rfft && s > m / 2 + 1) return MRCQR_ERR_ARG;  // distinct bins of a real signal
  mrcqr_plan* p = new mrcqr_plan();
  p->m = m; p->n = n; p->s = s;
  p->xform = rfft ? 1 : 0;
  plan_layout(p);
  *out = p;
  return MRCQR_OK;
}

int mrcqr_plan_create(int64_t m, int64_t n, int64_t s, mrcqr_plan** out) {
  return mrcqr_plan_create_ex(m, n, s, 0, out);
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
  // the carried precision needs a workspace owned by the caller (plan API)
  if (sketch_precision == MRCQR_PREC_AUTO_CARRY) return MRCQR_ERR_ARG;
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
      std::unique_ptr<CacheEntry> ce(new CacheEntry());
      ce->plan.m = m; ce->plan.n = n; ce->plan.s = s;
      plan_layout(&ce->plan);
      if (hipMalloc(&ce->ws, ce->plan.total) != hipSuccess) return MRCQR_ERR_DEVICE;
      if (hipEventCreateWithFlags(&ce->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(ce->ws);
        return MRCQR_ERR_DEVICE;
      }
      it = g_cache.emplace(key, std::move(ce)).first;
    }
    ent = it->second.get();
  }
  const hipStream_t st = as_stream(stream);
  std::lock_guard<std::mutex> lk(ent->mu);
  // Under stream capture the event edges are left out (an event recorded
  // outside the capture cannot be waited on inside it); a captured call
  // shares the workspace with every other call of its shape.
  const bool capturing = stream_capturing(st);
  if (ent->used && !capturing && hipStreamWaitEvent(st, ent->done, 0) != hipSuccess) return MRCQR_ERR_DEVICE;
  const int r = execute(&ent->plan, static_cast<char*>(ent->ws), A, lda, sketch_precision, seed, Q, ldq, R, ldr,
                        st, info_dev);
  if (!capturing) {
    // recorded even after a failed launch: kernels enqueued before it may
    // still use the workspace
    if (hipEventRecord(ent->done, st) != hipSuccess) return MRCQR_ERR_DEVICE;
    ent->used = true;
  }
  return r;
}

int mrcqr_factor_noalloc(const double* A, int64_t m, int64_t n, int64_t lda, int sketch_precision, uint64_t seed,
                         int64_t s, double* Q, int64_t ldq, double* R, int64_t ldr, void* stream,
                         mrcqr_info* info_dev) {
  if (s == 0) s = 2 * n;
  // the carried precision needs a workspace owned by the caller (plan API)
  if (sketch_precision == MRCQR_PREC_AUTO_CARRY) return MRCQR_ERR_ARG;
  const int c = check_factor_args(A, m, n, lda, sketch_precision, s, Q, ldq, R, ldr);
  if (c) return c;
  mrcqr_plan plan;
  plan.m = m; plan.n = n; plan.s = s;
  plan_layout(&plan);
  if (plan.total > NOALLOC_SCRATCH_BYTES) return MRCQR_ERR_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MRCQR_ERR_DEVICE;
  void* ws = scratch_for_device(dev);
  if (!ws) return MRCQR_ERR_DEVICE;
  // Nothing in the workspace has to start at zero: the draw kernel resets
  // the control block, and every partial sum is written before it is read.
  // the serial sequence: no side stream or events are created here
  return execute(&plan, static_cast<char*>(ws), A, lda, sketch_precision, seed, Q, ldq, R, ldr, as_stream(stream),
                 info_dev, false);
}

size_t mrcqr_factor_noalloc_max_workspace_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int mrcqr_release_cache(void) {
  int rc = MRCQR_OK;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_cache) {
      CacheEntry& e = *kv.second;
      std::lock_guard<std::mutex> lk2(e.mu);
      if (e.used && hipEventSynchronize(e.done) != hipSuccess) rc = MRCQR_ERR_DEVICE;
      if (hipEventDestroy(e.done) != hipSuccess || hipFree(e.ws) != hipSuccess) rc = MRCQR_ERR_DEVICE;
    }
    g_cache.clear();
  }
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto& kv : g_batch_cache) {
      BatchEntry& e = kv.second;
      if (e.used && hipEventSynchronize(e.done) != hipSuccess) rc = MRCQR_ERR_DEVICE;
      if (hipEventDestroy(e.done) != hipSuccess || hipFree(e.ws) != hipSuccess || hipFree(e.params) != hipSuccess)
        rc = MRCQR_ERR_DEVICE;
      batch_plan_free(e.plan);
    }
    g_batch_cache.clear();
  }
  return rc;
}

int mrcqr_batch_plan_create(int32_t batch, const int64_t* m, const int64_t* n, mrcqr_batch_plan** out) {
  return batch_plan_build(batch, m, n, out);
}

size_t mrcqr_batch_plan_workspace_bytes(const mrcqr_batch_plan* plan) { return plan ? plan->total : 0; }

int mrcqr_batch_plan_destroy(mrcqr_batch_plan* plan) {
  batch_plan_free(plan);
  return MRCQR_OK;
}

int mrcqr_batch_execute(const mrcqr_batch_plan* plan, void* workspace, size_t workspace_bytes,
                        const double* const* A, const int64_t* lda, const int32_t* precision, const uint64_t* seeds,
                        double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr, void* stream,
                        mrcqr_info* infos_dev) {
  if (!plan || !A || !lda || !precision || !seeds || !Q || !ldq || !R || !ldr) return MRCQR_ERR_ARG;
  if (!workspace || workspace_bytes < plan->total) return MRCQR_ERR_WORKSPACE;
  BatchCall call{static_cast<char*>(workspace), A, lda, Q, ldq, R, ldr, precision, seeds, infos_dev};
  return batch_execute(plan, call, as_stream(stream));
}

int mrcqr_factor_batched(int32_t batch, const double* const* A, const int64_t* m, const int64_t* n,
                         const int64_t* lda, const int32_t* precision, const uint64_t* seeds,
                         double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr,
                         void* stream, mrcqr_info* infos_dev) {
  if (batch < 0 || (batch > 0 && (!A || !m || !n || !lda || !precision || !seeds || !Q || !ldq || !R || !ldr)))
    return MRCQR_ERR_ARG;
  if (batch == 0) return MRCQR_OK;
  for (int32_t i = 0; i < batch; ++i) {
    if (precision[i] == MRCQR_PREC_AUTO_CARRY) return MRCQR_ERR_ARG;  // needs a caller-owned workspace
    const int c = check_factor_args(A[i], m[i], n[i], lda[i], precision[i], 2 * n[i], Q[i], ldq[i], R[i], ldr[i]);
    if (c) return c;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MRCQR_ERR_DEVICE;
  std::vector<int64_t> key{dev};
  for (int32_t i = 0; i < batch; ++i) { key.push_back(m[i]); key.push_back(n[i]); }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto it = g_batch_cache.find(key);
  if (it == g_batch_cache.end()) {
    BatchEntry be;
    const int c = batch_plan_build(batch, m, n, &be.plan);
    if (c) return c;
    const size_t pbytes = (size_t)batch * (6 * sizeof(int64_t) + sizeof(int32_t) + sizeof(uint64_t)) + 256;
    if (hipMalloc(&be.ws, be.plan->total) != hipSuccess || hipMalloc(&be.params, pbytes) != hipSuccess ||
        hipEventCreateWithFlags(&be.done, hipEventDisableTiming) != hipSuccess) {
      batch_plan_free(be.plan);
      return MRCQR_ERR_DEVICE;
    }
    it = g_batch_cache.emplace(key, be).first;
  }
  BatchEntry& be = it->second;
  // the per-call arrays go to device memory; the previous call on this
  // entry must be done reading them
  if (be.used && hipEventSynchronize(be.done) != hipSuccess) return MRCQR_ERR_DEVICE;
  std::vector<unsigned char> host((size_t)batch * (6 * sizeof(int64_t) + sizeof(int32_t) + sizeof(uint64_t)));
  unsigned char* h = host.data();
  const size_t b8 = (size_t)batch * 8;
  std::memcpy(h, A, b8);
  std::memcpy(h + b8, lda, b8);
  std::memcpy(h + 2 * b8, Q, b8);
  std::memcpy(h + 3 * b8, ldq, b8);
  std::memcpy(h + 4 * b8, R, b8);
  std::memcpy(h + 5 * b8, ldr, b8);
  std::memcpy(h + 6 * b8, seeds, b8);
  std::memcpy(h + 7 * b8, precision, (size_t)batch * sizeof(int32_t));
  if (hipMemcpy(be.params, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) return MRCQR_ERR_DEVICE;
  unsigned char* d = static_cast<unsigned char*>(be.params);
  BatchCall call{static_cast<char*>(be.ws),
                 reinterpret_cast<const double* const*>(d), reinterpret_cast<const int64_t*>(d + b8),
                 reinterpret_cast<double* const*>(d + 2 * b8), reinterpret_cast<const int64_t*>(d + 3 * b8),
                 reinterpret_cast<double* const*>(d + 4 * b8), reinterpret_cast<const int64_t*>(d + 5 * b8),
                 reinterpret_cast<const int32_t*>(d + 7 * b8), reinterpret_cast<const uint64_t*>(d + 6 * b8),
                 infos_dev};
  const int c = batch_execute(be.plan, call, as_stream(stream));
  // recorded even after a failed launch: the kernels enqueued before it may
  // still read the argument arrays, and the next call waits for them
  const bool recorded = hipEventRecord(be.done, as_stream(stream)) == hipSuccess;
  be.used = recorded;
  if (c) return c;
  return recorded ? MRCQR_OK : MRCQR_ERR_DEVICE;
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
  return mrcqr_sketch_ex(A, m, n, lda, S_dev, s, seed, precision, 0, Y, ldy, workspace, workspace_bytes, stream);
}

int mrcqr_sketch_ex(const double* A, int64_t m, int64_t n, int64_t lda, const int32_t* S_dev, int64_t s,
                    uint64_t seed, int precision, int flags, double* Y, int64_t ldy, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (!A || !S_dev || !Y || !valid_prec(precision, false)) return MRCQR_ERR_ARG;
  if ((flags & ~MRCQR_SKETCH_RFFT) != 0) return MRCQR_ERR_ARG;
  if ((flags & MRCQR_SKETCH_RFFT) && s > m / 2 + 1) return MRCQR_ERR_ARG;
  if (n < 1 || m < 1 || s < 1 || s > m || lda < m || ldy < s) return MRCQR_ERR_ARG;
  if (m >= MMAX || s > SMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < mrcqr_sketch_workspace_bytes(m, n, s, precision)) return MRCQR_ERR_WORKSPACE;
  return hip_status(launch_sketch(precision, A, lda, (int)m, (int)n, S_dev, (int)s, seed, workspace, Y, ldy,
                                  nullptr, PH_FIRST, as_stream(stream), (flags & MRCQR_SKETCH_RFFT) ? 1 : 0));
}

int mrcqr_sketch_qr(const double* Y, int64_t s, int64_t n, int64_t ldy, int qr_precision, double* Rs,
                    int64_t ldr, double* kappa_dev, void* stream) {
  if (!Y || !Rs || n < 1 || s < n || ldy < s || ldr < n) return MRCQR_ERR_ARG;
  if (qr_precision != MRCQR_PREC_FP32 && qr_precision != MRCQR_PREC_FP64) return MRCQR_ERR_ARG;
  if (n > NSTEP || !qr_supported((int)s, (int)n)) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_sketch_qr(qr_precision == MRCQR_PREC_FP64, Y, (int)s, (int)n, ldy, Rs, ldr, kappa_dev,
                                     nullptr, P_AUTO, PH_FIRST, as_stream(stream)));
}

size_t mrcqr_trsm_workspace_bytes(int64_t n) {
  if (n < 1 || n > NMAX) return 0;
  return trsm_workspace_bytes((int)std::min<int64_t>(n, NSTEP));
}

int mrcqr_trsm(const double* A, int64_t m, int64_t n, int64_t lda, const double* R, int64_t ldr, double* X,
               int64_t ldx, void* workspace, size_t workspace_bytes, void* stream) {
  if (!A || !R || !X || m < 1 || n < 1 || lda < m || ldr < n || ldx < m || A == X) return MRCQR_ERR_ARG;
  if (n > NMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < mrcqr_trsm_workspace_bytes(n)) return MRCQR_ERR_WORKSPACE;
  if (n > NSTEP)
    return hip_status(launch_trsm_wide(A, (int)m, (int)n, lda, R, ldr, X, ldx, workspace, nullptr, PH_FIRST,
                                       as_stream(stream)));
  return hip_status(launch_trsm(A, (int)m, (int)n, lda, R, ldr, X, ldx, workspace, nullptr, PH_FIRST,
                                as_stream(stream)));
}

size_t mrcqr_gram_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1 || n > NMAX) return 0;
  if (n > NSTEP) return align_up(gram_partial_bytes(m, NSTEP)) + gram_pair_partial_bytes((int)n);
  return gram_partial_bytes(m, n);
}

int mrcqr_gram(const double* B, int64_t m, int64_t n, int64_t ldb, double* G, int64_t ldg, void* workspace,
               size_t workspace_bytes, void* stream) {
  if (!B || !G || m < 1 || n < 1 || ldb < m || ldg < n) return MRCQR_ERR_ARG;
  if (n > NMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < mrcqr_gram_workspace_bytes(m, n)) return MRCQR_ERR_WORKSPACE;
  if (n > NSTEP) {
    double* diag = static_cast<double*>(workspace);
    double* pairs = reinterpret_cast<double*>(static_cast<char*>(workspace) + align_up(gram_partial_bytes(m, NSTEP)));
    return hip_status(launch_gram_wide(B, (int)m, (int)n, ldb, diag, pairs, G, ldg, nullptr, PH_FIRST,
                                       as_stream(stream)));
  }
  return hip_status(launch_gram(B, (int)m, (int)n, ldb, static_cast<double*>(workspace), G, ldg, nullptr,
                                PH_FIRST, as_stream(stream)));
}

int mrcqr_cholesky(const double* G, int64_t n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail_dev,
                   double* kappa_dev, void* stream) {
  if (!G || !Rc || n < 1 || ldg < n || ldr < n) return MRCQR_ERR_ARG;
  if (n > NSTEP) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_cholesky(G, (int)n, ldg, Rc, ldr, fail_dev, kappa_dev, nullptr, PH_FIRST,
                                    as_stream(stream)));
}

int mrcqr_trmm(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int64_t n, double* R, int64_t ldr,
               void* stream) {
  if (!R2 || !R1 || !R || n < 1 || ld2 < n || ld1 < n || ldr < n) return MRCQR_ERR_ARG;
  if (n > NMAX) return MRCQR_ERR_UNSUPPORTED;
  if (n > NSTEP)
    return hip_status(launch_trmm_wide(R2, ld2, R1, ld1, (int)n, R, ldr, nullptr, PH_FIRST, as_stream(stream)));
  return hip_status(launch_trmm(R2, ld2, R1, ld1, (int)n, R, ldr, nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_tri_inverse(const double* R, int64_t n, int64_t ldr, double* X, int64_t ldx, void* stream) {
  if (!R || !X || n < 1 || ldr < n || ldx < n || R == X) return MRCQR_ERR_ARG;
  if (n > NMAX) return MRCQR_ERR_UNSUPPORTED;
  if (n > NSTEP)
    return hip_status(launch_trinv_wide(R, (int)n, ldr, X, ldx, nullptr, PH_FIRST, as_stream(stream)));
  return hip_status(launch_trinv(R, (int)n, ldr, X, ldx, nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_form_q(const double* B, int64_t m, int64_t n, int64_t ldb, const double* X, int64_t ldx, double* Q,
                 int64_t ldq, void* stream) {
  if (!B || !X || !Q || m < 1 || n < 1 || ldb < m || ldx < n || ldq < m || B == Q) return MRCQR_ERR_ARG;
  if (n > NMAX || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (n > NSTEP)
    return hip_status(launch_qform_wide(B, (int)m, (int)n, ldb, X, ldx, Q, ldq, nullptr, PH_FIRST, as_stream(stream)));
  return hip_status(launch_qform(B, (int)m, (int)n, ldb, X, ldx, Q, ldq, nullptr, PH_FIRST, as_stream(stream)));
}

int mrcqr_condest(const double* R, int64_t n, int64_t ldr, double* kappa_dev, void* stream) {
  if (!R || !kappa_dev || n < 1 || ldr < n) return MRCQR_ERR_ARG;
  if (n > NSTEP) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_condest(R, (int)n, ldr, kappa_dev, as_stream(stream)));
}

size_t mrcqr_posterior_workspace_bytes(int64_t n) {
  return n > NSTEP && n <= NMAX ? posterior_wide_ws_bytes() : 0;
}

int mrcqr_posterior_kappa(const double* R, const double* X, int64_t n, int64_t ld, double* kappa_dev,
                          void* workspace, void* stream) {
  if (!R || !X || !kappa_dev || n < 1 || ld < n) return MRCQR_ERR_ARG;
  if (n > NMAX) return MRCQR_ERR_UNSUPPORTED;
  if (n > NSTEP) {
    if (!workspace) return MRCQR_ERR_WORKSPACE;
    return hip_status(launch_posterior_wide(R, X, (int)n, ld, static_cast<double*>(workspace), nullptr, PH_FIRST,
                                            kappa_dev, as_stream(stream)));
  }
  return hip_status(launch_posterior(R, X, (int)n, ld, nullptr, PH_FIRST, kappa_dev, as_stream(stream)));
}

// CholQR2 (Algorithm 1 twice): workspace = G, R1, R2 (n x n each), the
// Gram partials, the solve's operand staging, two breakdown indices, Q1.
struct Cholqr2Layout {
  size_t G, R1, R2, Gpart, Tw, fail, Q1, total;
};
static Cholqr2Layout cholqr2_layout(int64_t m, int64_t n) {
  Cholqr2Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  L.G = take((size_t)n * n * sizeof(double));
  L.R1 = take((size_t)n * n * sizeof(double));
  L.R2 = take((size_t)n * n * sizeof(double));
  L.Gpart = take(gram_partial_bytes(m, n));
  L.Tw = take(trsm_workspace_bytes((int)n));
  L.fail = take(2 * sizeof(int32_t));
  L.Q1 = take((size_t)m * n * sizeof(double));
  L.total = o;
  return L;
}

size_t mrcqr_cholqr2_workspace_bytes(int64_t m, int64_t n) {
  if (n < 1 || m < n || n > NSTEP || m >= MMAX) return 0;
  return cholqr2_layout(m, n).total;
}

int mrcqr_cholqr2(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq, double* R,
                  int64_t ldr, void* workspace, size_t workspace_bytes, void* stream, mrcqr_info* info_dev) {
  if (!A || !Q || !R || n < 1 || m < n || lda < m || ldq < m || ldr < n || A == Q) return MRCQR_ERR_ARG;
  if (n > NSTEP || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  const Cholqr2Layout L = cholqr2_layout(m, n);
  if (!workspace || workspace_bytes < L.total) return MRCQR_ERR_WORKSPACE;
  char* ws = static_cast<char*>(workspace);
  double* G = reinterpret_cast<double*>(ws + L.G);
  double* R1 = reinterpret_cast<double*>(ws + L.R1);
  double* R2 = reinterpret_cast<double*>(ws + L.R2);
  double* Gpart = reinterpret_cast<double*>(ws + L.Gpart);
  int32_t* fail = reinterpret_cast<int32_t*>(ws + L.fail);
  double* Q1 = reinterpret_cast<double*>(ws + L.Q1);
  const hipStream_t st = as_stream(stream);
  const int mi = (int)m, ni = (int)n;
  // pass 1: [Q1, R1] = CholQR(A); pass 2: [Q, R2] = CholQR(Q1); R = R2 R1
  const bool ok =
      launch_gram(A, mi, ni, lda, Gpart, G, n, nullptr, PH_FIRST, st) == hipSuccess &&
      launch_cholesky(G, ni, n, R1, n, fail, nullptr, nullptr, PH_FIRST, st) == hipSuccess &&
      launch_trsm(A, mi, ni, lda, R1, n, Q1, m, ws + L.Tw, nullptr, PH_FIRST, st) == hipSuccess &&
      launch_gram(Q1, mi, ni, m, Gpart, G, n, nullptr, PH_FIRST, st) == hipSuccess &&
      launch_cholesky(G, ni, n, R2, n, fail + 1, nullptr, nullptr, PH_FIRST, st) == hipSuccess &&
      launch_trsm(Q1, mi, ni, m, R2, n, Q, ldq, ws + L.Tw, nullptr, PH_FIRST, st) == hipSuccess &&
      launch_trmm(R2, n, R1, n, ni, R, ldr, nullptr, PH_FIRST, st) == hipSuccess &&
      (!info_dev || launch_cholqr2_finalize(fail, info_dev, st) == hipSuccess);
  return ok ? MRCQR_OK : MRCQR_ERR_DEVICE;
}

int mrcqr_condest_1norm(const double* R, const double* G, int64_t n, int64_t ld, uint64_t seed, double* kappa_dev,
                        void* stream) {
  if (!R || !kappa_dev || n < 1 || ld < n) return MRCQR_ERR_ARG;
  if (n > NSTEP) return MRCQR_ERR_UNSUPPORTED;
  return hip_status(launch_onenorm_condest(R, G, (int)n, ld, seed, kappa_dev, as_stream(stream)));
}

size_t mrcqr_cholqr_probe_workspace_bytes(int64_t m, int64_t n) {
  if (n < 1 || m < n || n > NSTEP || m >= MMAX) return 0;
  return probe_workspace_bytes(m, n);
}

int mrcqr_cholqr_probe(const double* A, int64_t m, int64_t n, int64_t lda, void* workspace, size_t workspace_bytes,
                       double* kappa_dev, void* stream) {
  if (!A || !kappa_dev || n < 1 || m < n || lda < m) return MRCQR_ERR_ARG;
  if (n > NSTEP || m >= MMAX) return MRCQR_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < probe_workspace_bytes(m, n)) return MRCQR_ERR_WORKSPACE;
  return hip_status(launch_cholqr_probe(A, (int)m, (int)n, lda, workspace, kappa_dev, as_stream(stream)));
}

const char* mrcqr_status_string(int status) {
  switch (status) {
    case MRCQR_OK: return "ok";
    case MRCQR_ERR_ARG: return "invalid argument";
    case MRCQR_ERR_NONFINITE: return "non-finite value in the sketch (non-finite input, or input out of the precision's range)";
    case MRCQR_ERR_CHOL_BREAKDOWN: return "Cholesky breakdown (Gram matrix not numerically positive definite)";
    case MRCQR_ERR_SKETCH_SINGULAR: return "sketch factor Rs is singular or not finite";
    case MRCQR_ERR_WORKSPACE: return "workspace missing or too small";
    case MRCQR_ERR_DEVICE: return "HIP runtime error";
    case MRCQR_WARN_POSTERIOR: return "posterior check: kappa(Rc) above bound, sketch precision too low";
    case MRCQR_ERR_UNSUPPORTED: return "shape not supported by this library";
    default: return "unknown status";
  }
}

int mrcqr_version(void) { return 100; }

}  // extern "C"
