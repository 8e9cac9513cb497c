// C-ABI host layer: handle construction, validation, workspace, and the
// host-driven CG loop (convergence is decided on the device; the host reads
// the decision every `check_every` iterations).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ppcg.h"
#include "ppcg_handle.h"
#include "ppcg_kernels.h"
#include "ppcg_panels.h"

using namespace ppcg;

namespace {

// Row pass: u = omega .* (X x), as panel partials (omega applied by the pass
// when the rows fit one panel, else by the consumer).
template <typename T>
hipError_t row_pass(ppcg_matrix* X, const Combine<T>& x, const T* omega, const int32_t* done,
                    hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                    const DirIn<T>* dir = nullptr, int parity = 0) {
  Orient& o = X->rows[prec_index<T>()];
  return launch_panel_pass<T>(o.pass, x, reinterpret_cast<T*>(o.part),
                              reinterpret_cast<T*>(o.piece), rows_direct(o) ? omega : nullptr,
                              done, st, ev0, ev1, dir, nullptr, parity);
}

// The column pass's view of u.
template <typename T>
Combine<T> u_view(ppcg_matrix* X, const T* omega) {
  const Orient& o = X->rows[prec_index<T>()];
  return comb_out<T>(o, rows_direct(o) ? nullptr : omega);
}

// Column pass: segment sums of X^T u, u from the row pass (or y if given).
template <typename T>
hipError_t col_pass(ppcg_matrix* X, const T* omega, const Combine<T>* y, const int32_t* done,
                    hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                    const DotOut<T>* dot = nullptr, int parity = 0) {
  Orient& o = X->cols[prec_index<T>()];
  const Combine<T> u = y ? *y : u_view<T>(X, omega);
  return launch_panel_pass<T>(o.pass, u, reinterpret_cast<T*>(o.part),
                              reinterpret_cast<T*>(o.piece), nullptr, done, st, ev0, ev1,
                              nullptr, dot, parity);
}

// FP64 product part qx64 = X^T (omega .* (X x)).
int fp64_phi_parts(ppcg_matrix* X, const double* x, const double* omega64, hipStream_t st) {
  PPCG_TRY_HIP(row_pass<double>(X, comb_vec<double>(x), omega64, nullptr, st));
  PPCG_TRY_HIP(col_pass<double>(X, omega64, nullptr, nullptr, st));
  PPCG_TRY_HIP(launch_combine<double, double>(comb_out<double>(X->cols[0], nullptr), X->p,
                                              X->qx64, st));
  return PPCG_OK;
}

template <typename T>
struct Bufs;
template <>
struct Bufs<double> {
  static double* s(ppcg_matrix* X) { return X->s64; }  // two buffers of p
};
template <>
struct Bufs<float> {
  static float* s(ppcg_matrix* X) { return X->s32; }
};

int sync_scal(ppcg_matrix* X, hipStream_t st) {
  PPCG_TRY_HIP(hipMemcpyAsync(X->h_sc, X->sc, sizeof(DevScal), hipMemcpyDeviceToHost, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return PPCG_OK;
}

// Runs CG iterations until the device reports done; returns via h_sc[0].
// The host checks the device's flag after each batch of check_every
// iterations (fewer near the predicted end, see below).  The next batch is
// normally already queued when the host waits for a batch's flag (read
// back into the other pinned slot), so the device does not idle while the
// host checks.  `phase` (0: first solve from zero, 1: first solve from a
// caller's start vector, 2: refinement restart) selects the iteration count
// of the handle's previous phase of that kind, which sizes the first batch
// (see below).
template <typename T>
int run_loop(ppcg_matrix* X, const T* omegaT, const ppcg_options& o, int phase,
             hipStream_t st) {
  const int ti = prec_index<T>();
  T* s = Bufs<T>::s(X);
  const int32_t* done = &X->sc->done;
  const VecWork w = vw(X);
  const Combine<T> none{};
  const Combine<T> qsrc = comb_out<T>(X->cols[ti], nullptr);
  DirIn<T> dir{};
  dir.z = X->z64;
  dir.s = s;
  dir.sstride = X->p;
  dir.d = X->d;
  dir.sc = X->sc;
  dir.scstride = 0;
  dir.p1 = X->p1[ti];
  dir.sp = w.part;  // the row pass finishes each step (pass_finish below)
  dir.nsb = vec_blocks(X->p);
  DotOut<T> dot{};
  dot.s = s;
  dot.sstride = X->p;
  dot.p2 = X->p2[ti];
  const int32_t n1 = X->rows[ti].pass.nwg, n2 = X->cols[ti].pass.nwg;
  const bool prof = X->profile != 0;
  // Profiling times both passes of one iteration (check_every / 2 into the
  // batch) in every kProfileEvery-th batch longer than that, the first
  // included: event-stamped dispatches leave the device idle for several
  // microseconds each, so few iterations carry them.
  constexpr int kProfileEvery = 4;
  const int sample = o.check_every / 2;
  while (prof && X->ev.size() < 8) {
    hipEvent_t e;
    PPCG_TRY_HIP(hipEventCreate(&e));
    X->ev.push_back(e);
  }
  int parity = 0;
  int32_t it = 0;  // iteration of this phase (the start kernel left iteration 0's scalars)
  int64_t batch = 0;
  int32_t start[2] = {0, 0}, size[2] = {0, 0};
  bool stamped[2] = {false, false};
  auto enqueue = [&](int slot, int nb) -> int {
    start[slot] = it;
    size[slot] = nb;
    stamped[slot] = prof && batch % kProfileEvery == 0 && nb > sample;
    for (int i = 0; i < nb; ++i, parity ^= 1, ++it) {
      hipEvent_t* e = (stamped[slot] && i == sample) ? &X->ev[4 * slot] : nullptr;
      // row pass: finishes the previous step, forms s (buffer 1 - parity)
      // from z and the old s
      dir.it = it;
      PPCG_TRY_HIP(row_pass<T>(X, none, omegaT, done, st, e ? e[0] : nullptr,
                               e ? e[1] : nullptr, &dir, parity));
      PPCG_TRY_HIP(col_pass<T>(X, omegaT, nullptr, done, st, e ? e[2] : nullptr,
                               e ? e[3] : nullptr, &dot, parity));
      // the batch's last step also writes the scalars into the readback slot
      PPCG_TRY_HIP(launch_cg_step<T>(w, s, X->p, parity, true, qsrc, X->d, X->m, X->beta64,
                                     X->r64, X->z64, X->p1[ti], n1, X->p2[ti], n2, X->p, st,
                                     i + 1 == nb ? &X->h_sc[slot] : nullptr));
    }
    PPCG_TRY_HIP(hipEventRecord(X->chk[slot], st));
    ++batch;
    return PPCG_OK;
  };
  // Waits for a batch's flag; true once the device reported done.
  auto check = [&](int slot, bool& is_done) -> int {
    PPCG_TRY_HIP(hipEventSynchronize(X->chk[slot]));
    const DevScal& h = X->h_sc[slot];
    // The sampled iteration counts only if its passes ran: once the rule
    // holds, the row pass of iteration iters and all later ones return early.
    if (stamped[slot] && (!h.done || start[slot] + sample < h.iters)) {
      float a = 0.f, b = 0.f;
      PPCG_TRY_HIP(hipEventElapsedTime(&a, X->ev[4 * slot], X->ev[4 * slot + 1]));
      PPCG_TRY_HIP(hipEventElapsedTime(&b, X->ev[4 * slot + 2], X->ev[4 * slot + 3]));
      X->pass_ms[0] += a;
      X->pass_ms[1] += b;
      X->pass_cnt[0] += 1;
      X->pass_cnt[1] += 1;
    }
    is_done = h.done != 0;
    return PPCG_OK;
  };
  // The decay of the rule measure over the checked batch predicts how many
  // iterations after it the solve needs (-1: no prediction, the measure has
  // not fallen since the start).  A batch queued ahead is skipped when the running batch is
  // predicted to finish the solve (it would only run launches that exit
  // early), and is given the predicted remainder plus one iteration, not the
  // full period, when that is shorter: then few launches run after the stop.
  // (The measure's decay is irregular, so a wider margin saves nothing: a
  // replay of the rule on FP64 convergence histories at n = 1e5, p = 2e4
  // gave 12 iterations after the stop per draw against 16 with full batches
  // and 14 with 1.25 times the remainder plus two.)  The first prediction
  // compares the first batch's end with the measure the start left (slot 2).
  auto ratio = [&](int slot) {
    const DevScal& h = X->h_sc[slot];
    return h.loop2 > 0.0 ? h.meas / h.loop2 : 0.0;
  };
  const int full = o.check_every;
  // (CG's measure is not monotone: over a short batch it can rise, and the
  // prediction then falls back to its mean decay since the start, m_start
  // at iteration 0.)
  double m_start = 0.0;
  auto predict = [&](double m, double m_prev, int nb, int done_its) {
    if (m <= 1.0) return 0.0;
    if (m_prev > 0.0 && m < m_prev) return nb * std::log(m) / std::log(m_prev / m);
    if (m_start > 0.0 && m < m_start && done_its > 0)
      return done_its * std::log(m) / std::log(m_start / m);
    return -1.0;
  };
  auto size_for = [&](double left, int most) {
    if (left < 0.0 || left >= most) return most;
    const int nb = (int)std::ceil(left) + 1;
    return nb < most ? nb : most;
  };
  // A sequence of draws on one handle (a Gibbs sampler's) repeats its
  // iteration counts closely, so the first batch runs to kHintShort short
  // of the previous phase's count, with a batch of kHintTail queued behind
  // it: the first check then comes near the end and the device keeps
  // working while the host makes it.  Near the end the measure swings by
  // orders of magnitude from one iteration to the next, so until a quarter
  // past the previous count the batches stay at most kHintStep long and
  // one is always queued ahead (a replay of the rule on six FP64 draws at
  // n = 1e5, p = 2e4: 3.0 launches after the stop per draw against 6.0
  // with predicted batches).  Without a count the first batch is one
  // period, checked with nothing queued behind it (a short solve then runs
  // no launches after its stop).
  constexpr int kHintShort = 2, kHintTail = 3, kHintStep = 2;
  const int32_t hint = X->iter_hint[phase][ti];
  int first = full;
  if (hint > 0) first = std::max(1, std::min(hint - kHintShort, o.max_iter));
  bool fin = false;
  int rc = enqueue(0, first);
  if (rc) return rc;
  double m_prev = ratio(2);
  m_start = m_prev;
  int cur = 0;
  bool ahead = hint > 0;
  int next = kHintTail;
  for (;;) {
    if (ahead && (rc = enqueue(cur ^ 1, next))) return rc;
    if ((rc = check(cur, fin))) return rc;
    if (fin) {
      // a batch queued ahead exits launch by launch; the scalars no longer change
      if (ahead) PPCG_TRY_HIP(hipStreamSynchronize(st));
      if (cur != 0) X->h_sc[0] = X->h_sc[cur];
      // (a run that hit its cap or broke down predicts nothing)
      X->iter_hint[phase][ti] = X->h_sc[0].status == PPCG_OK ? X->h_sc[0].iters : 0;
      return PPCG_OK;
    }
    const int its = start[cur] + size[cur];  // iterations after batch cur
    const bool near = hint > 0 && its < hint + hint / 4;
    const int most = near ? kHintStep : full;
    const double m = ratio(cur);
    const double left = predict(m, m_prev, size[cur], its);
    m_prev = m;
    if (!ahead && (rc = enqueue(cur ^ 1, size_for(left, most)))) return rc;
    // batch cur ^ 1 runs next; what the one after it would have to do
    const double after = left < 0.0 ? -1.0 : left - size[cur ^ 1];
    ahead = near || !(left >= 0.0 && after <= 0.0);
    next = size_for(after, most);
    cur ^= 1;
  }
}

// CG from the state prepared in b64 (and beta64 when have_beta0), then the
// optional FP64 true residual and refinement restart.
template <typename T>
int solve_core(ppcg_matrix* X, const T* omegaT, const double* omega64, bool have_beta0,
               const ppcg_options& o, ppcg_info* info, hipStream_t st) {
  const VecWork w = vw(X);
  const double* qx0 = nullptr;
  if (have_beta0) {
    int rc = fp64_phi_parts(X, X->beta64, omega64, st);
    if (rc) return rc;
    qx0 = X->qx64;
  }
  // The FP32 form runs its recursion to half the tolerance: its recursive
  // residual drifts from the true one by about the FP32 rounding of the
  // products, and the margin lets the FP64 check pass without a replacement.
  const double loop_factor =
      o.loop_factor > 0.0 ? o.loop_factor : ((sizeof(T) == 4) ? 0.5 : 1.0);
  PPCG_TRY_HIP(launch_cg_start(w, 0, X->b64, qx0, X->d, X->m, X->beta64, X->r64, X->z64, X->p,
                             o.tol, o.criterion, o.max_iter, loop_factor, st, &X->h_sc[2]));
  int rc = run_loop<T>(X, omegaT, o, have_beta0 ? 1 : 0, st);
  if (rc) return rc;
  ppcg_info inf{};
  inf.status = X->h_sc->status;
  inf.iters = X->h_sc->iters;
  inf.resid_rec = ratio(X->h_sc->meas, X->h_sc->thresh2);
  inf.resid_true = -1.0;
  inf.resid_true_first = -1.0;
  inf.bnorm_precond = std::sqrt(X->h_sc->bm2);
  inf.rms_precond = -1.0;
  if (o.true_resid || o.refine) {
    rc = fp64_phi_parts(X, X->beta64, omega64, st);
    if (rc) return rc;
    PPCG_TRY_HIP(launch_cg_start(w, 2, X->b64, X->qx64, X->d, X->m, X->beta64, X->r64, X->z64,
                             X->p, o.tol, o.criterion, o.max_iter, loop_factor, st));
    rc = sync_scal(X, st);
    if (rc) return rc;
    inf.resid_true = ratio(X->h_sc->true_meas, X->h_sc->thresh2);
    inf.resid_true_first = inf.resid_true;
    inf.rms_precond = std::sqrt(X->h_sc->true_rm / (double)X->p);
    if (o.refine && inf.status == PPCG_OK && X->h_sc->true_meas > X->h_sc->thresh2) {
      // One refinement: restart CG from the FP64 true residual
      // b - Phi beta (qx64 holds the product part of the current beta).
      PPCG_TRY_HIP(launch_cg_start(w, 1, X->b64, X->qx64, X->d, X->m, X->beta64, X->r64, X->z64,
                             X->p, o.tol, o.criterion, o.max_iter, loop_factor, st,
                             &X->h_sc[2]));
      rc = run_loop<T>(X, omegaT, o, 2, st);
      if (rc) return rc;
      inf.refined = 1;
      inf.refine_iters = X->h_sc->iters;
      inf.status = X->h_sc->status;
      inf.resid_rec = ratio(X->h_sc->meas, X->h_sc->thresh2);
      rc = fp64_phi_parts(X, X->beta64, omega64, st);
      if (rc) return rc;
      PPCG_TRY_HIP(launch_cg_start(w, 2, X->b64, X->qx64, X->d, X->m, X->beta64, X->r64, X->z64,
                             X->p, o.tol, o.criterion, o.max_iter, loop_factor, st));
      rc = sync_scal(X, st);
      if (rc) return rc;
      inf.resid_true = ratio(X->h_sc->true_meas, X->h_sc->thresh2);
      inf.rms_precond = std::sqrt(X->h_sc->true_rm / (double)X->p);
    }
  }
  if (info) *info = inf;
  return inf.status;
}

// omega pointers for the two precisions: the caller's array when its dtype
// matches, else the handle's FP64 copy filled by launch_prep.
const double* omega_f64(ppcg_matrix* X, const void* omega, int dtype) {
  return dtype == PPCG_F64 ? reinterpret_cast<const double*>(omega) : X->omega64;
}

int prepare(ppcg_matrix* X, const void* omega, const void* lambda, double tau, int dtype,
            hipStream_t st) {
  PPCG_TRY_HIP(launch_prep(lambda, omega, dtype, tau, X->n, X->p, X->d, X->m,
                           dtype == PPCG_F64 ? nullptr : X->omega64, st));
  return PPCG_OK;
}

int dispatch_solve(ppcg_matrix* X, const void* omega, int dtype, bool have_beta0,
                   const ppcg_options& o, ppcg_info* info, hipStream_t st) {
  const double* om64 = omega_f64(X, omega, dtype);
  if (dtype == PPCG_F64)
    return solve_core<double>(X, reinterpret_cast<const double*>(omega), om64, have_beta0, o,
                              info, st);
  return solve_core<float>(X, reinterpret_cast<const float*>(omega), om64, have_beta0, o, info,
                           st);
}

}  // namespace

// The handle from both orientations' index arrays (validated, on the host).
static int build_handle(ppcg_matrix** out, int64_t n, int64_t p, int64_t nnz,
                        const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                        const std::vector<int64_t>& cp, const std::vector<int32_t>& ri) {
  ppcg_matrix* X = new (std::nothrow) ppcg_matrix();
  if (!X) return PPCG_ENOMEM;
  auto fail = [&](int rc) {
    X->mem.release();
    for (hipEvent_t e : X->chk)
      if (e) (void)hipEventDestroy(e);
    if (X->h_sc) (void)hipHostFree(X->h_sc);
    delete X;
    return rc;
  };
  X->n = n;
  X->p = p;
  X->nnz = nnz;
  if (hipGetDevice(&X->device) != hipSuccess) return fail(PPCG_EHIP);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, X->device) !=
          hipSuccess || ncu < 1)
    ncu = 256;
  X->ncu = ncu;
  if (setup_pass_kernels() != hipSuccess) return fail(PPCG_EHIP);

  // Panel-blocked index-only tables of both orientations, for FP64 and
  // FP32 gathered values (the panel width depends on the value size),
  // built on four host threads, then uploaded.
  {
    PanelBuild Bt[4];
    auto job = [&](int q) {
      const int elem = (q / 2) == 0 ? 8 : 4;
      if (q % 2 == 0)
        build_panels(rp, ci, n, p, elem, ncu, Bt[q], /*compact=*/true);
      else
        build_panels(cp, ri, p, n, elem, ncu, Bt[q], /*compact=*/true);
    };
    bool threaded = true;
    std::vector<std::thread> th;
    try {
      for (int q = 1; q < 4; ++q) th.emplace_back(job, q);
    } catch (...) {
      threaded = false;
    }
    job(0);
    for (auto& t : th) t.join();
    if (!threaded)
      for (int q = 1 + (int)th.size(); q < 4; ++q) job(q);
    for (int q = 0; q < 4; ++q) {
      Orient& o = (q % 2 == 0) ? X->rows[q / 2] : X->cols[q / 2];
      int rc = upload_orient(X->mem, Bt[q], (q / 2) == 0 ? 8 : 4, 1, o);
      if (rc) return fail(rc);
      Bt[q] = PanelBuild();
    }
  }

  const size_t N = (size_t)n, P = (size_t)p;
  bool ok = X->mem.alloc(&X->qx64, P) == hipSuccess && X->mem.alloc(&X->y64, N) == hipSuccess &&
            X->mem.alloc(&X->omega64, N) == hipSuccess &&
            X->mem.alloc(&X->d, P) == hipSuccess && X->mem.alloc(&X->m, P) == hipSuccess &&
            X->mem.alloc(&X->b64, P) == hipSuccess && X->mem.alloc(&X->beta64, P) == hipSuccess &&
            X->mem.alloc(&X->r64, P) == hipSuccess && X->mem.alloc(&X->s64, 2 * P) == hipSuccess &&
            X->mem.alloc(&X->qx32, P) == hipSuccess && X->mem.alloc(&X->s32, 2 * P) == hipSuccess &&
            X->mem.alloc(&X->z64, P) == hipSuccess &&
            X->mem.alloc(&X->p1[0], (size_t)X->rows[0].pass.nwg) == hipSuccess &&
            X->mem.alloc(&X->p2[0], (size_t)X->cols[0].pass.nwg) == hipSuccess &&
            X->mem.alloc(&X->p1[1], (size_t)X->rows[1].pass.nwg) == hipSuccess &&
            X->mem.alloc(&X->p2[1], (size_t)X->cols[1].pass.nwg) == hipSuccess &&
            X->mem.alloc(&X->part, (size_t)kMaxRedBlocks * 4) == hipSuccess &&
            X->mem.alloc(&X->sc, 1) == hipSuccess;
  if (!ok) return fail(PPCG_ENOMEM);
  if (hipMemset(X->sc, 0, sizeof(DevScal)) != hipSuccess) return fail(PPCG_EHIP);
  if (hipHostMalloc(reinterpret_cast<void**>(&X->h_sc), 3 * sizeof(DevScal), 0) != hipSuccess) {
    X->h_sc = nullptr;
    return fail(PPCG_ENOMEM);
  }
  std::memset(X->h_sc, 0, 3 * sizeof(DevScal));
  for (hipEvent_t& e : X->chk)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(PPCG_EHIP);
  if (hipDeviceSynchronize() != hipSuccess) return fail(PPCG_EHIP);
  *out = X;
  return PPCG_OK;
}

extern "C" {

void ppcg_options_default(ppcg_options* opt, int32_t dtype) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->dtype = dtype;
  opt->criterion = PPCG_REL_PRECOND;
  opt->max_iter = 0;
  opt->refine = -1;
  opt->tol = 1e-6;
  opt->true_resid = 1;
  opt->check_every = 0;
}

const char* ppcg_status_string(int status) {
  switch (status) {
    case PPCG_OK: return "ok";
    case PPCG_EINVAL: return "invalid argument";
    case PPCG_ENOMEM: return "out of memory";
    case PPCG_EHIP: return "HIP runtime error";
    case PPCG_ENOTCONV: return "not converged within max_iter";
    case PPCG_EBREAKDOWN: return "CG breakdown (<s, Phi s> <= 0 or non-finite)";
    case PPCG_ENODEV: return "no HIP device";
    case PPCG_ETOOBIG: return "needs more scratch than the fixed array of the entry point that allocates nothing";
    default: return "unknown status";
  }
}

const char* ppcg_version(void) { return "ppcg-mi355x 0.1 (gfx950)"; }

int ppcg_matrix_create(ppcg_matrix** out, int64_t n, int64_t p, int64_t nnz,
                       const int64_t* row_ptr, const int32_t* col_idx, const void* values,
                       int32_t mem, hipStream_t stream) {
  try {
    if (!out) return PPCG_EINVAL;
    *out = nullptr;
    if (n < 1 || p < 1 || nnz < 0 || values != nullptr || !row_ptr) return PPCG_EINVAL;
    if (nnz > 0 && !col_idx) return PPCG_EINVAL;
    if (n >= INT32_MAX || p >= INT32_MAX || nnz >= ((int64_t)INT32_MAX) * 1024) return PPCG_EINVAL;
    if (mem != PPCG_MEM_HOST && mem != PPCG_MEM_DEVICE) return PPCG_EINVAL;

    std::vector<int64_t> rp, cp;
    std::vector<int32_t> ci, ri;
    const int rc = read_binary_csr(n, p, nnz, row_ptr, col_idx, mem, stream, rp, ci, cp, ri);
    if (rc) return rc;
    return build_handle(out, n, p, nnz, rp, ci, cp, ri);
  } catch (const std::bad_alloc&) {
    return PPCG_ENOMEM;
  } catch (...) {
    return PPCG_EINVAL;
  }
}

int ppcg_matrix_create_csc(ppcg_matrix** out, int64_t n, int64_t p, int64_t nnz,
                           const int64_t* col_ptr, const int32_t* row_idx, const void* values,
                           int32_t mem, hipStream_t stream) {
  try {
    if (!out) return PPCG_EINVAL;
    *out = nullptr;
    if (n < 1 || p < 1 || nnz < 0 || values != nullptr || !col_ptr) return PPCG_EINVAL;
    if (nnz > 0 && !row_idx) return PPCG_EINVAL;
    if (n >= INT32_MAX || p >= INT32_MAX || nnz >= ((int64_t)INT32_MAX) * 1024) return PPCG_EINVAL;
    if (mem != PPCG_MEM_HOST && mem != PPCG_MEM_DEVICE) return PPCG_EINVAL;
    // The CSC of X is the CSR of X^T: the same reader validates it and builds
    // the other orientation by its counting sort.
    std::vector<int64_t> rp, cp;
    std::vector<int32_t> ci, ri;
    const int rc = read_binary_csr(p, n, nnz, col_ptr, row_idx, mem, stream, cp, ri, rp, ci);
    if (rc) return rc;
    return build_handle(out, n, p, nnz, rp, ci, cp, ri);
  } catch (const std::bad_alloc&) {
    return PPCG_ENOMEM;
  } catch (...) {
    return PPCG_EINVAL;
  }
}

int ppcg_matrix_profile(ppcg_matrix* X, int32_t enable) {
  if (!X) return PPCG_EINVAL;
  X->profile = enable ? 1 : 0;
  if (enable) {
    X->pass_ms[0] = X->pass_ms[1] = 0.0;
    X->pass_cnt[0] = X->pass_cnt[1] = 0;
  }
  return PPCG_OK;
}

int ppcg_matrix_stats(const ppcg_matrix* X, double* csr_ms, int64_t* csr_launches,
                      double* csc_ms, int64_t* csc_launches) {
  if (!X) return PPCG_EINVAL;
  if (csr_ms) *csr_ms = X->pass_ms[0];
  if (csr_launches) *csr_launches = X->pass_cnt[0];
  if (csc_ms) *csc_ms = X->pass_ms[1];
  if (csc_launches) *csc_launches = X->pass_cnt[1];
  return PPCG_OK;
}

int ppcg_matrix_pass_bytes(const ppcg_matrix* X, int32_t dtype, int64_t* row_pass_bytes,
                           int64_t* col_pass_bytes) {
  if (!X || !valid_dtype(dtype)) return PPCG_EINVAL;
  const int pi = dtype == PPCG_F64 ? 0 : 1;
  if (row_pass_bytes) *row_pass_bytes = X->rows[pi].pass_bytes;
  if (col_pass_bytes) *col_pass_bytes = X->cols[pi].pass_bytes;
  return PPCG_OK;
}

int ppcg_matrix_destroy(ppcg_matrix* X) {
  if (!X) return PPCG_OK;
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : X->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : X->chk)
    if (e) (void)hipEventDestroy(e);
  X->mem.release();
  if (X->h_sc) (void)hipHostFree(X->h_sc);
  delete X;
  return PPCG_OK;
}

int ppcg_matrix_shape(const ppcg_matrix* X, int64_t* n, int64_t* p, int64_t* nnz) {
  if (!X) return PPCG_EINVAL;
  if (n) *n = X->n;
  if (p) *p = X->p;
  if (nnz) *nnz = X->nnz;
  return PPCG_OK;
}

int ppcg_phi_matvec(const ppcg_matrix* Xc, const void* omega, const void* lambda, double tau,
                    const void* v, void* out, int32_t dtype, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !lambda || !v || !out || !valid_dtype(dtype) || bad_tau(tau))
    return PPCG_EINVAL;
  int rc = prepare(X, omega, lambda, tau, dtype, st);
  if (rc) return rc;
  if (dtype == PPCG_F64) {
    const double* om = reinterpret_cast<const double*>(omega);
    const double* vv = reinterpret_cast<const double*>(v);
    PPCG_TRY_HIP(row_pass<double>(X, comb_vec<double>(vv), om, nullptr, st));
    PPCG_TRY_HIP(col_pass<double>(X, om, nullptr, nullptr, st));
    PPCG_TRY_HIP(launch_combine<double, double>(comb_out<double>(X->cols[0], nullptr), X->p,
                                                X->qx64, st));
    PPCG_TRY_HIP(launch_phi_finish<double>(X->qx64, X->d, vv, X->p,
                                           reinterpret_cast<double*>(out), st));
  } else {
    const float* om = reinterpret_cast<const float*>(omega);
    const float* vv = reinterpret_cast<const float*>(v);
    PPCG_TRY_HIP(row_pass<float>(X, comb_vec<float>(vv), om, nullptr, st));
    PPCG_TRY_HIP(col_pass<float>(X, om, nullptr, nullptr, st));
    PPCG_TRY_HIP(launch_combine<float, float>(comb_out<float>(X->cols[1], nullptr), X->p,
                                              X->qx32, st));
    PPCG_TRY_HIP(launch_phi_finish<float>(X->qx32, X->d, vv, X->p,
                                          reinterpret_cast<float*>(out), st));
  }
  return PPCG_OK;
}

int ppcg_normals(uint64_t seed, uint64_t stream_id, uint64_t chain, uint64_t draw_index,
                 int64_t count, double* out, hipStream_t st) {
  if (count < 0 || (count > 0 && !out)) return PPCG_EINVAL;
  PPCG_TRY_HIP(launch_normals(seed, stream_id, chain, draw_index, count, out, st));
  return PPCG_OK;
}

static int form_rhs(ppcg_matrix* X, const void* omega, const void* z, const void* lambda,
                    double tau, uint64_t seed, uint64_t chain, uint64_t draw, int dtype,
                    double* b_out, hipStream_t st) {
  int rc = prepare(X, omega, lambda, tau, dtype, st);
  if (rc) return rc;
  const double* om64 = omega_f64(X, omega, dtype);
  PPCG_TRY_HIP(launch_y_draw(om64, z, dtype, seed, chain, draw, X->n, X->y64, st));
  const Combine<double> y = comb_vec<double>(X->y64);
  PPCG_TRY_HIP(col_pass<double>(X, nullptr, &y, nullptr, st));
  PPCG_TRY_HIP(launch_combine<double, double>(comb_out<double>(X->cols[0], nullptr), X->p,
                                              X->qx64, st));
  PPCG_TRY_HIP(launch_rhs_fin(X->qx64, lambda, dtype, tau, seed, chain, draw, X->p, b_out, st));
  return PPCG_OK;
}

int ppcg_rhs(const ppcg_matrix* Xc, const void* omega, const void* z, const void* lambda,
             double tau, uint64_t seed, uint64_t chain, uint64_t draw_index, int32_t dtype,
             double* b_out, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !z || !lambda || !b_out || !valid_dtype(dtype) || bad_tau(tau))
    return PPCG_EINVAL;
  return form_rhs(X, omega, z, lambda, tau, seed, chain, draw_index, dtype, b_out, st);
}

int ppcg_solve(const ppcg_matrix* Xc, const void* omega, const void* lambda, double tau,
               const void* b, const void* beta0, const ppcg_options* opt, void* beta_out,
               ppcg_info* info, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !lambda || !b || !beta_out || bad_tau(tau)) return PPCG_EINVAL;
  const ppcg_options o = resolve(opt, X->p);
  if (check_opts(o)) return PPCG_EINVAL;
  int rc = prepare(X, omega, lambda, tau, o.dtype, st);
  if (rc) return rc;
  PPCG_TRY_HIP(launch_convert_to_f64(b, o.dtype, X->p, X->b64, st));
  if (beta0) PPCG_TRY_HIP(launch_convert_to_f64(beta0, o.dtype, X->p, X->beta64, st));
  const int status = dispatch_solve(X, omega, o.dtype, beta0 != nullptr, o, info, st);
  if (status == PPCG_EINVAL || status == PPCG_ENOMEM || status == PPCG_EHIP) return status;
  PPCG_TRY_HIP(launch_convert_from_f64(X->beta64, o.dtype, X->p, beta_out, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return status;
}

int ppcg_draw(const ppcg_matrix* Xc, const void* omega, const void* z, const void* lambda,
              double tau, uint64_t seed, uint64_t chain, uint64_t draw_index,
              const ppcg_options* opt, void* beta_out, ppcg_info* info, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !z || !lambda || !beta_out || bad_tau(tau)) return PPCG_EINVAL;
  const ppcg_options o = resolve(opt, X->p);
  if (check_opts(o)) return PPCG_EINVAL;
  int rc = form_rhs(X, omega, z, lambda, tau, seed, chain, draw_index, o.dtype, X->b64, st);
  if (rc) return rc;
  const int status = dispatch_solve(X, omega, o.dtype, false, o, info, st);
  if (status == PPCG_EINVAL || status == PPCG_ENOMEM || status == PPCG_EHIP) return status;
  PPCG_TRY_HIP(launch_convert_from_f64(X->beta64, o.dtype, X->p, beta_out, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return status;
}

// ---- Polya-Gamma omega update (Supplement S1, step 3) ----
int ppcg_pg_update(const ppcg_matrix* Xc, const void* beta, const uint8_t* y, uint64_t seed,
                   uint64_t chain, uint64_t draw_index, int32_t dtype, void* omega_out,
                   void* z_out, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !beta || !y || !omega_out || !z_out || !valid_dtype(dtype)) return PPCG_EINVAL;
  // psi = X beta in FP64 (the FP32 form converts beta first), into the
  // n-sized workspace, then one thread per row draws omega and forms z.
  const double* b64 = reinterpret_cast<const double*>(beta);
  if (dtype == PPCG_F32) {
    PPCG_TRY_HIP(launch_convert_to_f64(beta, dtype, X->p, X->beta64, st));
    b64 = X->beta64;
  }
  PPCG_TRY_HIP(row_pass<double>(X, comb_vec<double>(b64), nullptr, nullptr, st));
  PPCG_TRY_HIP(launch_combine<double, double>(comb_out<double>(X->rows[0], nullptr), X->n,
                                              X->y64, st));
  PPCG_TRY_HIP(launch_pg_omega(X->y64, y, X->n, seed, chain, draw_index, dtype, omega_out, z_out,
                               st));
  return PPCG_OK;
}

// ---- general diagonal prior and preconditioner (Supplement S4.3) ----
static int prepare_general(ppcg_matrix* X, const void* omega, const double* prior_prec,
                           const double* precond_inv, int dtype, hipStream_t st) {
  PPCG_TRY_HIP(launch_prep_general(prior_prec, precond_inv, omega, dtype, X->n, X->p, X->d, X->m,
                                   dtype == PPCG_F64 ? nullptr : X->omega64, st));
  return PPCG_OK;
}

int ppcg_solve_general(const ppcg_matrix* Xc, const void* omega, const double* prior_prec,
                       const double* precond_inv, const void* b, const void* beta0,
                       const ppcg_options* opt, void* beta_out, ppcg_info* info,
                       hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !prior_prec || !b || !beta_out) return PPCG_EINVAL;
  const ppcg_options o = resolve(opt, X->p);
  if (check_opts(o)) return PPCG_EINVAL;
  int rc = prepare_general(X, omega, prior_prec, precond_inv, o.dtype, st);
  if (rc) return rc;
  PPCG_TRY_HIP(launch_convert_to_f64(b, o.dtype, X->p, X->b64, st));
  if (beta0) PPCG_TRY_HIP(launch_convert_to_f64(beta0, o.dtype, X->p, X->beta64, st));
  const int status = dispatch_solve(X, omega, o.dtype, beta0 != nullptr, o, info, st);
  if (status == PPCG_EINVAL || status == PPCG_ENOMEM || status == PPCG_EHIP) return status;
  PPCG_TRY_HIP(launch_convert_from_f64(X->beta64, o.dtype, X->p, beta_out, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return status;
}

int ppcg_draw_general(const ppcg_matrix* Xc, const void* omega, const void* z,
                      const double* prior_prec, const double* precond_inv, const void* beta0,
                      uint64_t seed, uint64_t chain, uint64_t draw_index,
                      const ppcg_options* opt, void* beta_out, ppcg_info* info,
                      hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !z || !prior_prec || !beta_out) return PPCG_EINVAL;
  const ppcg_options o = resolve(opt, X->p);
  if (check_opts(o)) return PPCG_EINVAL;
  int rc = prepare_general(X, omega, prior_prec, precond_inv, o.dtype, st);
  if (rc) return rc;
  const double* om64 = omega_f64(X, omega, o.dtype);
  PPCG_TRY_HIP(launch_y_draw(om64, z, o.dtype, seed, chain, draw_index, X->n, X->y64, st));
  const Combine<double> y = comb_vec<double>(X->y64);
  PPCG_TRY_HIP(col_pass<double>(X, nullptr, &y, nullptr, st));
  PPCG_TRY_HIP(launch_combine<double, double>(comb_out<double>(X->cols[0], nullptr), X->p,
                                              X->qx64, st));
  PPCG_TRY_HIP(
      launch_rhs_fin_general(X->qx64, X->d, seed, chain, draw_index, X->p, X->b64, st));
  if (beta0) PPCG_TRY_HIP(launch_convert_to_f64(beta0, o.dtype, X->p, X->beta64, st));
  const int status = dispatch_solve(X, omega, o.dtype, beta0 != nullptr, o, info, st);
  if (status == PPCG_EINVAL || status == PPCG_ENOMEM || status == PPCG_EHIP) return status;
  PPCG_TRY_HIP(launch_convert_from_f64(X->beta64, o.dtype, X->p, beta_out, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return status;
}

int ppcg_phi_diag(const ppcg_matrix* Xc, const void* omega, int32_t dtype,
                  const double* prior_prec, double* diag_out, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !prior_prec || !diag_out || !valid_dtype(dtype)) return PPCG_EINVAL;
  if (dtype != PPCG_F64)
    PPCG_TRY_HIP(launch_convert_to_f64(omega, dtype, X->n, X->omega64, st));
  const double* om64 = omega_f64(X, omega, dtype);
  const Combine<double> w = comb_vec<double>(om64);
  PPCG_TRY_HIP(col_pass<double>(X, nullptr, &w, nullptr, st));
  PPCG_TRY_HIP(
      launch_phi_diag(comb_out<double>(X->cols[0], nullptr), prior_prec, X->p, diag_out, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return PPCG_OK;
}

int ppcg_solve_backward(const ppcg_matrix* Xc, const void* omega, const void* lambda,
                        double tau, const void* beta, const void* grad_beta,
                        const ppcg_options* opt, void* grad_b, void* grad_loglambda,
                        double* grad_logtau, ppcg_info* info, hipStream_t st) {
  ppcg_matrix* X = const_cast<ppcg_matrix*>(Xc);
  if (!X || !omega || !lambda || !beta || !grad_beta || !grad_b || !grad_loglambda ||
      !grad_logtau || bad_tau(tau))
    return PPCG_EINVAL;
  const ppcg_options o = resolve(opt, X->p);
  if (check_opts(o)) return PPCG_EINVAL;
  int rc = prepare(X, omega, lambda, tau, o.dtype, st);
  if (rc) return rc;
  PPCG_TRY_HIP(launch_convert_to_f64(grad_beta, o.dtype, X->p, X->b64, st));
  const int status = dispatch_solve(X, omega, o.dtype, false, o, info, st);
  if (status == PPCG_EINVAL || status == PPCG_ENOMEM || status == PPCG_EHIP) return status;
  PPCG_TRY_HIP(launch_adjoint_epilogue(vw(X), X->beta64, beta, o.dtype, X->d, X->p, grad_b,
                                       grad_loglambda, grad_logtau, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return status;
}

}  // extern "C"
