// C-ABI batches: many chains, each with its own X handle and workspace, whose
// per-iteration phases run as one launch per phase for all chains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ppcg.h"
#include "ppcg_handle.h"
#include "ppcg_kernels.h"

using namespace ppcg;

namespace {

// One chain's device workspace (allocated by the batch).
struct ChainBufs {
  const ppcg_matrix* X = nullptr;
  int64_t n = 0, p = 0;
  double *y64 = nullptr, *omega64 = nullptr, *d = nullptr, *m = nullptr, *b64 = nullptr,
         *beta64 = nullptr, *r64 = nullptr, *qx64 = nullptr, *red = nullptr;
  void *omegaT = nullptr, *s = nullptr, *qx = nullptr;  // the batch's dtype (s: 2 x p)
  double* z = nullptr;                                  // M^-1 r for the next row pass
  double *p1 = nullptr, *p2 = nullptr;                  // the passes' workgroup partials
  void *rpart[2] = {}, *rpiece[2] = {}, *cpart[2] = {}, *cpiece[2] = {};  // per table precision
};

// The consumer's view of an orientation's pass output held in a chain's own
// buffers (optionally scaled).
template <typename T>
Combine<T> comb_buf(const Orient& o, const void* part, const void* piece, const T* scale) {
  Combine<T> c{};
  c.es = 1;
  c.part = reinterpret_cast<const T*>(part);
  c.stride = o.out_dim;
  c.nparts = o.npanels;
  c.scale = scale;
  c.sp_off = o.sp_off;
  c.sp_c0 = o.sp_c0;
  c.sp_c1 = o.sp_c1;
  c.piece = reinterpret_cast<const T*>(piece);
  return c;
}

// Vector c's view of a K-wide orientation's pass output ([panel][dim][K]);
// scale, when given, is [dim][K] too.
template <typename T>
Combine<T> comb_k(const Orient& o, int K, int c, const T* scale) {
  Combine<T> x{};
  x.part = reinterpret_cast<const T*>(o.part) + c;
  x.stride = o.out_dim * K;
  x.nparts = o.npanels;
  x.es = K;
  x.scale = scale ? scale + c : nullptr;
  x.sp_off = o.sp_off;
  x.sp_c0 = o.sp_c0;
  x.sp_c1 = o.sp_c1;
  x.piece = reinterpret_cast<const T*>(o.piece) + c;
  return x;
}

// All K interleaved vectors of a [dim][K] array as a pass input.
template <typename T>
Combine<T> comb_all(const T* v, int K) {
  Combine<T> x{};
  x.part = v;
  x.stride = 0;
  x.nparts = 1;
  x.es = K;
  return x;
}

enum { kJobRow = 0, kJobCol, kJobRow64, kJobCol64, kJobRhs64, kNumJobs };

}  // namespace

struct ppcg_batch {
  int device = 0;
  int32_t dtype = 0;
  int32_t nch = 0;
  std::vector<ChainBufs> ch;
  ppcg::DevBuf mem;
  ppcg::DevScal* sc = nullptr;    // [nch]
  ppcg::DevScal* h_sc = nullptr;  // pinned mirror
  void* jobs[kNumJobs] = {};
  int32_t* wg_job[kNumJobs] = {};  // workgroup maps (every chain)
  int32_t* wg_local[kNumJobs] = {};
  int32_t nwg[kNumJobs] = {};
  void* vjobs = nullptr;  // VecJob<T>[nch]
  int32_t* blk_job = nullptr;  // block maps of the p-vector phases (every chain)
  int32_t* blk_local = nullptr;
  int32_t nblk = 0;
  // maps of the CG loop restricted to the chains still iterating, rebuilt
  // when that set changes (between launches, with the stream idle)
  int32_t *lp_wg_job[2] = {}, *lp_wg_local[2] = {}, *lp_blk_job = nullptr,
          *lp_blk_local = nullptr;
  int32_t lp_nwg[2] = {}, lp_nblk = 0;
  std::vector<char> lp_active;
  int64_t lp_version = 0;  // bumped whenever the loop maps change
  std::vector<int32_t> chain_nwg[2], chain_nblk;
  // the CG loop's check batch captured as a HIP graph, one per loop parity at
  // the batch start, valid for (lp_version, check_every, element size)
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2] = {};
  int64_t g_version = -1;
  int32_t g_every = 0, g_elem = 0;
  // shared form: every chain on one design, K interleaved vectors per pass,
  // in G groups of K vector slots (slot s is position s % K of group s / K;
  // chain c sits in slot slot_of[c]); each group's arrays follow the
  // previous group's, and the groups' passes run one after the other
  // through the same tables and partial buffers
  bool shared = false;
  int32_t K = 1, G = 1;
  int64_t n = 0, p = 0;
  ppcg::Orient srows[2], scols[2];  // K-wide tables: [0] FP64, [1] FP32
  double *y_K = nullptr, *om64_K = nullptr, *beta_K = nullptr;  // [G][dim][K]
  double *z_K = nullptr, *d_K = nullptr;                         // [G][p][K]
  double *p1_K = nullptr, *p2_K = nullptr;                       // [G][nwg][K]
  void *omT_K = nullptr, *s_K = nullptr;                         // [G][dim][K] / [G][2][p][K]
  void* q_K = nullptr;  // [G][p][K], dtype: X^T u of the loop's column pass, summed over panels
  // vector slot of each chain and chain of each slot (slots [0, nch) hold the
  // chains), and each chain's CG iterations in the last call: with two
  // groups the chains are dealt to slots by falling count, so that the
  // chains that iterate longest share a group
  std::vector<int32_t> slot_of, chain_at, last_iters;
};

namespace {

template <typename V>
int upload(ppcg_batch* B, const std::vector<V>& h, V** out) {
  V* d = nullptr;
  PPCG_TRY_ALLOC(B->mem.alloc(&d, h.size()));
  if (!h.empty())
    PPCG_TRY_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  *out = d;
  return PPCG_OK;
}

// Pass job tables of one kind for every chain, with their workgroup maps.
template <typename T>
int build_pass_jobs(ppcg_batch* B, int kind) {
  std::vector<PanelJob<T>> jobs(B->nch);
  std::vector<int32_t> wj, wl;
  for (int32_t c = 0; c < B->nch; ++c) {
    const ChainBufs& C = B->ch[c];
    const ppcg_matrix* X = C.X;
    PanelJob<T>& J = jobs[c];
    J = PanelJob<T>{};
    const int ti = (kind == kJobRow || kind == kJobCol) ? prec_index<T>() : 0;
    const Orient& ro = X->rows[ti];
    const Orient& co = X->cols[ti];
    const T* om = (kind == kJobRow || kind == kJobCol) ? reinterpret_cast<const T*>(C.omegaT)
                                                       : reinterpret_cast<const T*>(C.omega64);
    switch (kind) {
      case kJobRow:
      case kJobRow64:
        J.t = ro.pass;
        J.x = comb_vec<T>(kind == kJobRow ? reinterpret_cast<const T*>(C.s)
                                          : reinterpret_cast<const T*>(C.beta64));
        J.part_out = reinterpret_cast<T*>(C.rpart[ti]);
        J.piece_out = reinterpret_cast<T*>(C.rpiece[ti]);
        J.out_scale = rows_direct(ro) ? om : nullptr;
        break;
      case kJobCol:
      case kJobCol64:
        J.t = co.pass;
        J.x = comb_buf<T>(ro, C.rpart[ti], C.rpiece[ti], rows_direct(ro) ? nullptr : om);
        J.part_out = reinterpret_cast<T*>(C.cpart[ti]);
        J.piece_out = reinterpret_cast<T*>(C.cpiece[ti]);
        break;
      default:  // kJobRhs64
        J.t = co.pass;
        J.x = comb_vec<T>(reinterpret_cast<const T*>(C.y64));
        J.part_out = reinterpret_cast<T*>(C.cpart[ti]);
        J.piece_out = reinterpret_cast<T*>(C.cpiece[ti]);
        break;
    }
    J.done = (kind == kJobRow || kind == kJobCol) ? &B->sc[c].done : nullptr;
    // what the loop's passes read besides the plain pass
    if (J.t.nwg > 0 && (J.t.wg_s0 == nullptr || J.t.wg_s1 == nullptr || J.t.out_dim <= 0 ||
                        J.t.seg_out == nullptr || J.t.no_slot < 0))
      return PPCG_EHIP;
    if (kind == kJobRow) {
      // the loop's row pass forms the direction s from z (DirIn)
      J.x = Combine<T>{};
      J.dir.z = C.z;
      J.dir.s = reinterpret_cast<T*>(C.s);
      J.dir.sstride = C.p;
      J.dir.d = C.d;
      J.dir.sc = &B->sc[c];
      J.dir.p1 = C.p1;
    } else if (kind == kJobCol) {
      J.dot.s = reinterpret_cast<const T*>(C.s);
      J.dot.sstride = C.p;
      J.dot.p2 = C.p2;
    }
    for (int32_t w = 0; w < J.t.nwg; ++w) {
      wj.push_back(c);
      wl.push_back(w);
    }
  }
  PanelJob<T>* dj = nullptr;
  int rc = upload(B, jobs, &dj);
  if (rc) return rc;
  B->jobs[kind] = dj;
  if ((rc = upload(B, wj, &B->wg_job[kind]))) return rc;
  if ((rc = upload(B, wl, &B->wg_local[kind]))) return rc;
  B->nwg[kind] = (int32_t)wj.size();
  if (kind == kJobRow || kind == kJobCol) {
    B->chain_nwg[kind].resize(B->nch);
    for (int32_t c = 0; c < B->nch; ++c) B->chain_nwg[kind][c] = jobs[c].t.nwg;
    if ((rc = upload(B, wj, &B->lp_wg_job[kind]))) return rc;
    if ((rc = upload(B, wl, &B->lp_wg_local[kind]))) return rc;
    B->lp_nwg[kind] = B->nwg[kind];
  }
  return PPCG_OK;
}

// Slot of chain c (the chain itself unless the shared form reassigned it).
int32_t slot(const ppcg_batch* B, int32_t c) { return B->slot_of.empty() ? c : B->slot_of[c]; }

template <typename T>
std::vector<VecJob<T>> vec_jobs(ppcg_batch* B) {
  std::vector<VecJob<T>> jobs(B->nch);
  const int ti = prec_index<T>();
  for (int32_t c = 0; c < B->nch; ++c) {
    const ChainBufs& C = B->ch[c];
    VecJob<T>& J = jobs[c];
    J = VecJob<T>{};
    J.w = VecWork{C.red, &B->sc[slot(B, c)]};
    J.s = reinterpret_cast<T*>(C.s);
    J.sstride = C.p;
    J.z = C.z;
    J.zes = 1;
    J.p1 = C.p1;
    J.p2 = C.p2;
    J.pstride = 1;
    if (!B->shared) {
      J.qsrc = comb_buf<T>(C.X->cols[ti], C.cpart[ti], C.cpiece[ti], nullptr);
      J.n1 = C.X->rows[ti].pass.nwg;
      J.n2 = C.X->cols[ti].pass.nwg;
    }
    J.qx = reinterpret_cast<T*>(C.qx);
    J.b = C.b64;
    J.qx64 = C.qx64;
    J.d = C.d;
    J.m = C.m;
    J.beta = C.beta64;
    J.r = C.r64;
    J.p = C.p;
    J.max_iter = (int32_t)std::min<int64_t>(C.p, INT32_MAX);
    J.nblk = vec_blocks(C.p);
    J.es = 1;
    if (B->shared) {
      // s, z and the pass partials interleaved over the chains; q from the
      // K-wide column pass
      const int64_t g = slot(B, c) / B->K, r = slot(B, c) % B->K, pK = B->p * B->K;
      J.n1 = B->srows[ti].pass.nwg;
      J.n2 = B->scols[ti].pass.nwg;
      J.s = reinterpret_cast<T*>(B->s_K) + g * 2 * pK + r;
      J.sstride = pK;
      J.es = B->K;
      J.z = B->z_K + g * pK + r;
      J.zes = B->K;
      J.p1 = B->p1_K + g * J.n1 * B->K + r;
      J.p2 = B->p2_K + g * J.n2 * B->K + r;
      J.pstride = B->K;
      J.qsrc = comb_all<T>(reinterpret_cast<const T*>(B->q_K) + g * pK + r, B->K);
    }
  }
  return jobs;
}

template <typename T>
int build_vec_jobs(ppcg_batch* B) {
  const std::vector<VecJob<T>> jobs = vec_jobs<T>(B);
  std::vector<int32_t> bj, bl;
  for (int32_t c = 0; c < B->nch; ++c)
    for (int32_t b = 0; b < jobs[c].nblk; ++b) {
      bj.push_back(c);
      bl.push_back(b);
    }
  VecJob<T>* dj = nullptr;
  int rc = upload(B, jobs, &dj);
  if (rc) return rc;
  B->vjobs = dj;
  if ((rc = upload(B, bj, &B->blk_job))) return rc;
  if ((rc = upload(B, bl, &B->blk_local))) return rc;
  if ((rc = upload(B, bj, &B->lp_blk_job))) return rc;
  if ((rc = upload(B, bl, &B->lp_blk_local))) return rc;
  B->nblk = B->lp_nblk = (int32_t)bj.size();
  B->chain_nblk.resize(B->nch);
  for (int32_t c = 0; c < B->nch; ++c) B->chain_nblk[c] = jobs[c].nblk;
  B->lp_active.assign(B->nch, 1);
  return PPCG_OK;
}

int alloc_chain(ppcg_batch* B, ChainBufs& C) {
  const size_t N = (size_t)C.n, P = (size_t)C.p;
  const size_t ts = B->dtype == PPCG_F64 ? 8 : 4;
  unsigned char *om = nullptr, *s = nullptr, *qx = nullptr;
  PPCG_TRY_ALLOC(B->mem.alloc(&C.y64, N));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.omega64, N));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.d, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.m, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.b64, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.beta64, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.r64, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.qx64, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.red, (size_t)kMaxRedBlocks * 4));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.z, P));
  PPCG_TRY_ALLOC(B->mem.alloc(&qx, P * ts));
  C.qx = qx;
  if (B->shared) {
    C.omegaT = C.omega64;  // FP64 copy; the K-wide passes read omT_K
    return PPCG_OK;
  }
  PPCG_TRY_ALLOC(B->mem.alloc(&s, 2 * P * ts));
  PPCG_TRY_HIP(hipMemset(s, 0, 2 * P * ts));
  C.s = s;
  const int ti = B->dtype == PPCG_F64 ? 0 : 1;
  PPCG_TRY_ALLOC(B->mem.alloc(&C.p1, (size_t)C.X->rows[ti].pass.nwg));
  PPCG_TRY_ALLOC(B->mem.alloc(&C.p2, (size_t)C.X->cols[ti].pass.nwg));
  if (B->dtype == PPCG_F64) {
    C.omegaT = C.omega64;
  } else {
    PPCG_TRY_ALLOC(B->mem.alloc(&om, N * ts));
    C.omegaT = om;
  }
  // pass outputs: FP64 tables always (right-hand side, true residual), FP32
  // tables for the FP32 form's iteration
  for (int ti = 0; ti < 2; ++ti) {
    if (ti == 1 && B->dtype == PPCG_F64) continue;
    const size_t es = ti == 0 ? 8 : 4;
    const Orient& ro = C.X->rows[ti];
    const Orient& co = C.X->cols[ti];
    unsigned char *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
    const size_t ra = (size_t)ro.npanels * (size_t)ro.out_dim * es;
    const size_t ca = (size_t)co.npanels * (size_t)co.out_dim * es;
    PPCG_TRY_ALLOC(B->mem.alloc(&a, ra));
    PPCG_TRY_ALLOC(B->mem.alloc(&b, (size_t)std::max<int32_t>(ro.pass.npieces, 1) * es));
    PPCG_TRY_ALLOC(B->mem.alloc(&c, ca));
    PPCG_TRY_ALLOC(B->mem.alloc(&d, (size_t)std::max<int32_t>(co.pass.npieces, 1) * es));
    // (segment, panel) pairs with no elements are never written: they stay zero.
    PPCG_TRY_HIP(hipMemset(a, 0, std::max<size_t>(ra, 1)));
    PPCG_TRY_HIP(hipMemset(c, 0, std::max<size_t>(ca, 1)));
    C.rpart[ti] = a;
    C.rpiece[ti] = b;
    C.cpart[ti] = c;
    C.cpiece[ti] = d;
  }
  return PPCG_OK;
}

// Restricts the CG loop's launch maps to the chains in `act` (the stream
// must be idle: the maps are overwritten in place).
int set_loop_chains(ppcg_batch* B, const std::vector<char>& act) {
  if (act == B->lp_active) return PPCG_OK;
  for (int kind = 0; kind < 2 && !B->shared; ++kind) {
    std::vector<int32_t> wj, wl;
    for (int32_t c = 0; c < B->nch; ++c) {
      if (!act[c]) continue;
      for (int32_t w = 0; w < B->chain_nwg[kind][c]; ++w) {
        wj.push_back(c);
        wl.push_back(w);
      }
    }
    if (!wj.empty()) {
      PPCG_TRY_HIP(hipMemcpy(B->lp_wg_job[kind], wj.data(), wj.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice));
      PPCG_TRY_HIP(hipMemcpy(B->lp_wg_local[kind], wl.data(), wl.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice));
    }
    B->lp_nwg[kind] = (int32_t)wj.size();
  }
  std::vector<int32_t> bj, bl;
  for (int32_t c = 0; c < B->nch; ++c) {
    if (!act[c]) continue;
    for (int32_t b = 0; b < B->chain_nblk[c]; ++b) {
      bj.push_back(c);
      bl.push_back(b);
    }
  }
  if (!bj.empty()) {
    PPCG_TRY_HIP(hipMemcpy(B->lp_blk_job, bj.data(), bj.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice));
    PPCG_TRY_HIP(hipMemcpy(B->lp_blk_local, bl.data(), bl.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice));
  }
  B->lp_nblk = (int32_t)bj.size();
  B->lp_active = act;
  ++B->lp_version;
  return PPCG_OK;
}

// Shared form: row pass u = omega .* (X s) and column pass X^T u for the K
// interleaved vectors of the loop's dtype, group by group, each group's
// launches skipped once all its chains are done.
template <typename T>
int shared_loop_passes(ppcg_batch* B, int parity, hipStream_t st) {
  const int ti = prec_index<T>();
  const Orient& ro = B->srows[ti];
  const Orient& co = B->scols[ti];
  const int dstride = (int)(sizeof(DevScal) / sizeof(int32_t));
  const int64_t K = B->K, pK = B->p * K;
  const int64_t n1 = ro.pass.nwg, n2 = co.pass.nwg;
  for (int64_t g = 0; g < B->G; ++g) {
    const T* om = reinterpret_cast<const T*>(B->omT_K) + g * B->n * K;
    T* sg = reinterpret_cast<T*>(B->s_K) + g * 2 * pK;
    const int32_t* done = &B->sc[g * K].done;
    DirIn<T> dir{};
    dir.z = B->z_K + g * pK;
    dir.s = sg;
    dir.sstride = pK;
    dir.d = B->d_K + g * pK;
    dir.sc = B->sc + g * K;
    dir.scstride = 1;
    dir.p1 = B->p1_K + g * n1 * K;
    DotOut<T> dot{};
    dot.s = sg;
    dot.sstride = pK;
    dot.p2 = B->p2_K + g * n2 * K;
    PPCG_TRY_HIP(launch_panel_pass_k<T>(B->K, ro.pass, Combine<T>{},
                                        reinterpret_cast<T*>(ro.part),
                                        reinterpret_cast<T*>(ro.piece),
                                        rows_direct(ro) ? om : nullptr, done, dstride, st, &dir,
                                        nullptr, parity));
    PPCG_TRY_HIP(launch_panel_pass_k<T>(B->K, co.pass,
                                        comb_k<T>(ro, B->K, 0, rows_direct(ro) ? nullptr : om),
                                        reinterpret_cast<T*>(co.part),
                                        reinterpret_cast<T*>(co.piece), nullptr, done, dstride,
                                        st, nullptr, &dot, parity));
    // q for the group's chains at once, read whole lines (the per-chain step
    // reads it back with stride K from one array instead of from every
    // panel's)
    PPCG_TRY_HIP(launch_combine_k<T>(comb_k<T>(co, B->K, 0, nullptr), B->K, B->p,
                                     reinterpret_cast<T*>(B->q_K) + g * pK, done, dstride, st));
  }
  return PPCG_OK;
}

// Shared form: src_c (FP64, one per chain) interleaved into dst [G][dim][K].
template <typename T>
int interleave(ppcg_batch* B, double* const* src_of_chain, int64_t dim, T* dst,
               hipStream_t st) {
  for (int32_t g = 0; g < B->G; ++g) {
    VecPtrs v{};
    const int32_t c0 = g * B->K, nc = std::min(B->K, B->nch - c0);
    for (int32_t r = 0; r < nc; ++r) v.p[r] = src_of_chain[B->chain_at[c0 + r]];
    PPCG_TRY_HIP(launch_interleave<T>(v, nc, B->K, dim, dst + (int64_t)g * dim * B->K, st));
  }
  return PPCG_OK;
}

// One check batch of CG iterations (row pass, column pass, step each) for
// the chains of the current loop maps; parity alternates per iteration.
template <typename T>
int enqueue_batch(ppcg_batch* B, int every, int parity, hipStream_t st) {
  for (int i = 0; i < every; ++i, parity ^= 1) {
    if (B->shared) {
      const int rc = shared_loop_passes<T>(B, parity, st);
      if (rc) return rc;
    } else {
      PPCG_TRY_HIP(launch_panel_pass_batched<T>(
          reinterpret_cast<const PanelJob<T>*>(B->jobs[kJobRow]), B->lp_wg_job[kJobRow],
          B->lp_wg_local[kJobRow], B->lp_nwg[kJobRow], kPassDir, parity, st));
      PPCG_TRY_HIP(launch_panel_pass_batched<T>(
          reinterpret_cast<const PanelJob<T>*>(B->jobs[kJobCol]), B->lp_wg_job[kJobCol],
          B->lp_wg_local[kJobCol], B->lp_nwg[kJobCol], kPassDot, parity, st));
    }
    PPCG_TRY_HIP(launch_cg_step_batched<T>(reinterpret_cast<const VecJob<T>*>(B->vjobs),
                                           B->lp_blk_job, B->lp_blk_local, B->lp_nblk, parity,
                                           st));
  }
  return PPCG_OK;
}

void drop_graphs(ppcg_batch* B) {
  for (hipGraphExec_t& g : B->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

// The check batch as a graph: captured on the batch's own stream (the
// caller's may be the legacy default stream, which cannot be captured) the
// first time a (maps, batch length, element size, start parity) combination
// is used, then replayed on the caller's stream.  Kernel arguments are
// fixed for that combination: the maps live in device buffers rewritten
// only between batches, and the kernels' own arrival counters reset
// themselves.  Nothing but kernel launches is captured.
template <typename T>
int launch_batch_graph(ppcg_batch* B, int every, int parity, hipStream_t st) {
  if (B->g_version != B->lp_version || B->g_every != every || B->g_elem != (int32_t)sizeof(T)) {
    drop_graphs(B);
    B->g_version = B->lp_version;
    B->g_every = every;
    B->g_elem = (int32_t)sizeof(T);
  }
  if (!B->cap) PPCG_TRY_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  hipGraphExec_t& exec = B->gexec[parity & 1];
  if (!exec) {
    PPCG_TRY_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch<T>(B, every, parity, B->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    PPCG_TRY_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      exec = nullptr;
      return PPCG_EHIP;
    }
  }
  PPCG_TRY_HIP(hipGraphLaunch(exec, st));
  return PPCG_OK;
}

// CG iterations of every chain until all report done; the launches cover
// only the chains still iterating at the last check.  Each check batch is a
// replay of its captured graph unless the options ask for direct launches.
template <typename T>
int run_loop_batched(ppcg_batch* B, const ppcg_options& o, hipStream_t st) {
  std::vector<char> act(B->nch);
  int parity = 0;
  for (;;) {
    PPCG_TRY_HIP(hipMemcpyAsync(B->h_sc, B->sc, sizeof(DevScal) * B->nch,
                                hipMemcpyDeviceToHost, st));
    PPCG_TRY_HIP(hipStreamSynchronize(st));
    bool any = false;
    for (int32_t c = 0; c < B->nch; ++c) {
      act[c] = B->h_sc[slot(B, c)].done ? 0 : 1;
      any = any || act[c];
    }
    if (!any) return PPCG_OK;
    int rc = set_loop_chains(B, act);
    if (rc) return rc;
    rc = o.no_graph ? enqueue_batch<T>(B, o.check_every, parity, st)
                    : launch_batch_graph<T>(B, o.check_every, parity, st);
    if (rc) return rc;
    parity ^= o.check_every & 1;
  }
}

// FP64 product parts qx64_c = X_c^T (omega_c .* (X_c beta64_c)) of every chain.
int fp64_parts_batched(ppcg_batch* B, hipStream_t st) {
  if (B->shared) {
    std::vector<double*> src(B->nch);
    for (int32_t c = 0; c < B->nch; ++c) src[c] = B->ch[c].beta64;
    int rc = interleave<double>(B, src.data(), B->p, B->beta_K, st);
    if (rc) return rc;
    const Orient& ro = B->srows[0];
    const Orient& co = B->scols[0];
    for (int32_t g = 0; g < B->G; ++g) {
      const double* bg = B->beta_K + (int64_t)g * B->p * B->K;
      const double* om = B->om64_K + (int64_t)g * B->n * B->K;
      PPCG_TRY_HIP(launch_panel_pass_k<double>(B->K, ro.pass, comb_all<double>(bg, B->K),
                                               reinterpret_cast<double*>(ro.part),
                                               reinterpret_cast<double*>(ro.piece),
                                               rows_direct(ro) ? om : nullptr, nullptr, 0, st));
      PPCG_TRY_HIP(launch_panel_pass_k<double>(
          B->K, co.pass, comb_k<double>(ro, B->K, 0, rows_direct(ro) ? nullptr : om),
          reinterpret_cast<double*>(co.part), reinterpret_cast<double*>(co.piece), nullptr,
          nullptr, 0, st));
      for (int32_t sl = g * B->K; sl < std::min(B->nch, (g + 1) * B->K); ++sl)
        PPCG_TRY_HIP(launch_combine<double, double>(comb_k<double>(co, B->K, sl % B->K, nullptr),
                                                    B->p, B->ch[B->chain_at[sl]].qx64, st));
    }
    return PPCG_OK;
  }
  PPCG_TRY_HIP(launch_panel_pass_batched<double>(
      reinterpret_cast<const PanelJob<double>*>(B->jobs[kJobRow64]), B->wg_job[kJobRow64],
      B->wg_local[kJobRow64], B->nwg[kJobRow64], kPassPlain, 0, st));
  PPCG_TRY_HIP(launch_panel_pass_batched<double>(
      reinterpret_cast<const PanelJob<double>*>(B->jobs[kJobCol64]), B->wg_job[kJobCol64],
      B->wg_local[kJobCol64], B->nwg[kJobCol64], kPassPlain, 0, st));
  for (const ChainBufs& C : B->ch)
    PPCG_TRY_HIP(launch_combine<double, double>(
        comb_buf<double>(C.X->cols[0], C.cpart[0], C.cpiece[0], nullptr), C.p, C.qx64, st));
  return PPCG_OK;
}

int sync_all(ppcg_batch* B, hipStream_t st) {
  PPCG_TRY_HIP(hipMemcpyAsync(B->h_sc, B->sc, sizeof(DevScal) * B->nch, hipMemcpyDeviceToHost,
                              st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  return PPCG_OK;
}

// Shared form with two groups: chains dealt to slots by falling iteration
// count of the last call (ties by chain), so that the longest-iterating
// chains share a group and the other group stops early.  A new assignment
// rewrites the step's job table in place (ordered on the caller's stream
// after the work that read it) and drops the captured graphs.  The slot does not change a chain's
// arithmetic: every slot of a group is summed the same way.
template <typename T>
int assign_slots(ppcg_batch* B, hipStream_t st) {
  if (!B->shared || B->G < 2) return PPCG_OK;
  std::vector<int32_t> order(B->nch);
  for (int32_t c = 0; c < B->nch; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return B->last_iters[a] > B->last_iters[b];
  });
  if (order == B->chain_at) return PPCG_OK;
  B->chain_at = order;
  for (int32_t sl = 0; sl < B->nch; ++sl) B->slot_of[order[sl]] = sl;
  const std::vector<VecJob<T>> jobs = vec_jobs<T>(B);
  // on the caller's stream, after the work that read the old table; the
  // host copy lives until the stream has taken it
  PPCG_TRY_HIP(hipMemcpyAsync(B->vjobs, jobs.data(), jobs.size() * sizeof(VecJob<T>),
                              hipMemcpyHostToDevice, st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  drop_graphs(B);
  ++B->lp_version;
  return PPCG_OK;
}

template <typename T>
int batch_solve(ppcg_batch* B, const ppcg_chain* chains, const ppcg_options& o,
                ppcg_info* infos, bool draw, hipStream_t st) {
  const int dt = B->dtype;
  {
    const int rc = assign_slots<T>(B, st);
    if (rc) return rc;
  }
  // per-chain preparation: d, m, FP64 omega (and its FP32 copy), b
  for (int32_t c = 0; c < B->nch; ++c) {
    const ChainBufs& C = B->ch[c];
    const ppcg_chain& A = chains[c];
    PPCG_TRY_HIP(launch_prep(A.lambda, A.omega, dt, A.tau, C.n, C.p, C.d, C.m, C.omega64, st));
    if (dt == PPCG_F32 && !B->shared)
      PPCG_TRY_HIP(hipMemcpyAsync(C.omegaT, A.omega, (size_t)C.n * sizeof(float),
                                  hipMemcpyDeviceToDevice, st));
    if (draw) {
      PPCG_TRY_HIP(launch_y_draw(C.omega64, A.z, dt, A.seed, A.chain, A.draw_index, C.n, C.y64,
                                 st));
    } else {
      PPCG_TRY_HIP(launch_convert_to_f64(A.b, dt, C.p, C.b64, st));
    }
  }
  int rc = 0;
  if (B->shared) {
    std::vector<double*> om(B->nch), y(B->nch);
    for (int32_t c = 0; c < B->nch; ++c) {
      om[c] = B->ch[c].omega64;
      y[c] = B->ch[c].y64;
    }
    if ((rc = interleave<double>(B, om.data(), B->n, B->om64_K, st))) return rc;
    std::vector<double*> dd(B->nch);
    for (int32_t c = 0; c < B->nch; ++c) dd[c] = B->ch[c].d;
    if ((rc = interleave<double>(B, dd.data(), B->p, B->d_K, st))) return rc;
    if (dt == PPCG_F32 &&
        (rc = interleave<float>(B, om.data(), B->n, reinterpret_cast<float*>(B->omT_K), st)))
      return rc;
    if (draw) {
      if ((rc = interleave<double>(B, y.data(), B->n, B->y_K, st))) return rc;
      const Orient& co = B->scols[0];
      for (int32_t g = 0; g < B->G; ++g) {
        PPCG_TRY_HIP(launch_panel_pass_k<double>(
            B->K, co.pass, comb_all<double>(B->y_K + (int64_t)g * B->n * B->K, B->K),
            reinterpret_cast<double*>(co.part), reinterpret_cast<double*>(co.piece), nullptr,
            nullptr, 0, st));
        for (int32_t sl = g * B->K; sl < std::min(B->nch, (g + 1) * B->K); ++sl) {
          const ChainBufs& C = B->ch[B->chain_at[sl]];
          const ppcg_chain& A = chains[B->chain_at[sl]];
          PPCG_TRY_HIP(launch_combine<double, double>(
              comb_k<double>(co, B->K, sl % B->K, nullptr), C.p, C.qx64, st));
          PPCG_TRY_HIP(launch_rhs_fin(C.qx64, A.lambda, dt, A.tau, A.seed, A.chain,
                                      A.draw_index, C.p, C.b64, st));
        }
      }
    }
  } else if (draw) {
    PPCG_TRY_HIP(launch_panel_pass_batched<double>(
        reinterpret_cast<const PanelJob<double>*>(B->jobs[kJobRhs64]), B->wg_job[kJobRhs64],
        B->wg_local[kJobRhs64], B->nwg[kJobRhs64], kPassPlain, 0, st));
    for (int32_t c = 0; c < B->nch; ++c) {
      const ChainBufs& C = B->ch[c];
      const ppcg_chain& A = chains[c];
      PPCG_TRY_HIP(launch_combine<double, double>(
          comb_buf<double>(C.X->cols[0], C.cpart[0], C.cpiece[0], nullptr), C.p, C.qx64, st));
      PPCG_TRY_HIP(launch_rhs_fin(C.qx64, A.lambda, dt, A.tau, A.seed, A.chain, A.draw_index,
                                  C.p, C.b64, st));
    }
  }
  const VecJob<T>* vj = reinterpret_cast<const VecJob<T>*>(B->vjobs);
  const double loop_factor =
      o.loop_factor > 0.0 ? o.loop_factor : ((sizeof(T) == 4) ? 0.5 : 1.0);
  // o.max_iter <= 0: each chain's own cap (its p)
  PPCG_TRY_HIP(launch_cg_start_batched<T>(vj, B->blk_job, B->blk_local, B->nblk, 0,
                                            o.tol, o.criterion, o.max_iter, loop_factor,
                                            st));
  if ((rc = run_loop_batched<T>(B, o, st))) return rc;
  std::vector<ppcg_info> inf(B->nch);
  for (int32_t c = 0; c < B->nch; ++c) {
    const DevScal& S = B->h_sc[slot(B, c)];
    ppcg_info& I = inf[c];
    I = ppcg_info{};
    I.status = S.status;
    I.iters = S.iters;
    I.resid_rec = ratio(S.meas, S.thresh2);
    I.resid_true = -1.0;
    I.resid_true_first = -1.0;
    I.rms_precond = -1.0;
    I.bnorm_precond = std::sqrt(S.bm2);
  }
  if (o.true_resid || o.refine) {
    if ((rc = fp64_parts_batched(B, st))) return rc;
    PPCG_TRY_HIP(launch_cg_start_batched<T>(vj, B->blk_job, B->blk_local, B->nblk, 2,
                                            o.tol, o.criterion, o.max_iter, loop_factor,
                                            st));
    if ((rc = sync_all(B, st))) return rc;
    bool any = false;
    for (int32_t c = 0; c < B->nch; ++c) {
      const DevScal& S = B->h_sc[slot(B, c)];
      inf[c].resid_true = inf[c].resid_true_first = ratio(S.true_meas, S.thresh2);
      inf[c].rms_precond = std::sqrt(S.true_rm / (double)B->ch[c].p);
      any = any || (S.status == PPCG_OK && S.true_meas > S.thresh2);
    }
    if (o.refine && any) {
      // One refinement for the chains whose FP64 true residual misses the
      // rule: CG restarts from it (the start kernel leaves the others done).
      PPCG_TRY_HIP(launch_cg_start_batched<T>(vj, B->blk_job, B->blk_local, B->nblk, 1,
                                            o.tol, o.criterion, o.max_iter, loop_factor,
                                            st));
      if ((rc = run_loop_batched<T>(B, o, st))) return rc;
      std::vector<int32_t> refined(B->nch);
      for (int32_t c = 0; c < B->nch; ++c) {
        const DevScal& S = B->h_sc[slot(B, c)];
        refined[c] = S.refined;
        if (S.refined) {
          inf[c].refined = 1;
          inf[c].refine_iters = S.iters;
          inf[c].status = S.status;
          inf[c].resid_rec = ratio(S.meas, S.thresh2);
        }
      }
      if ((rc = fp64_parts_batched(B, st))) return rc;
      PPCG_TRY_HIP(launch_cg_start_batched<T>(vj, B->blk_job, B->blk_local, B->nblk, 2,
                                            o.tol, o.criterion, o.max_iter, loop_factor,
                                            st));
      if ((rc = sync_all(B, st))) return rc;
      for (int32_t c = 0; c < B->nch; ++c) {
        if (!refined[c]) continue;
        const DevScal& S = B->h_sc[slot(B, c)];
        inf[c].resid_true = ratio(S.true_meas, S.thresh2);
        inf[c].rms_precond = std::sqrt(S.true_rm / (double)B->ch[c].p);
      }
    }
  }
  for (int32_t c = 0; c < B->nch; ++c)
    PPCG_TRY_HIP(launch_convert_from_f64(B->ch[c].beta64, dt, B->ch[c].p, chains[c].beta_out,
                                         st));
  PPCG_TRY_HIP(hipStreamSynchronize(st));
  if (!B->last_iters.empty())
    for (int32_t c = 0; c < B->nch; ++c) B->last_iters[c] = inf[c].iters + inf[c].refine_iters;
  int status = PPCG_OK;
  for (int32_t c = 0; c < B->nch; ++c) {
    if (infos) infos[c] = inf[c];
    if (status == PPCG_OK && inf[c].status != PPCG_OK) status = inf[c].status;
  }
  return status;
}

int batched_entry(ppcg_batch* B, const ppcg_chain* chains, const ppcg_options* opt,
                  ppcg_info* infos, bool draw, hipStream_t st) {
  if (!B || !chains) return PPCG_EINVAL;
  ppcg_options o = resolve(opt, 1);
  o.max_iter = (opt && opt->max_iter > 0) ? opt->max_iter : 0;  // 0: each chain's p
  if (check_opts(o) || o.dtype != B->dtype) return PPCG_EINVAL;
  for (int32_t c = 0; c < B->nch; ++c) {
    const ppcg_chain& A = chains[c];
    if (!A.omega || !A.lambda || !A.beta_out || bad_tau(A.tau)) return PPCG_EINVAL;
    if (draw ? !A.z : !A.b) return PPCG_EINVAL;
  }
  if (B->dtype == PPCG_F64) return batch_solve<double>(B, chains, o, infos, draw, st);
  return batch_solve<float>(B, chains, o, infos, draw, st);
}

}  // namespace

extern "C" {

int ppcg_batch_create(ppcg_batch** out, int32_t nchains, const ppcg_matrix* const* X,
                      int32_t dtype, hipStream_t stream) {
  (void)stream;
  try {
    if (!out) return PPCG_EINVAL;
    *out = nullptr;
    if (nchains < 1 || !X || !valid_dtype(dtype)) return PPCG_EINVAL;
    for (int32_t c = 0; c < nchains; ++c)
      if (!X[c]) return PPCG_EINVAL;
    ppcg_batch* B = new (std::nothrow) ppcg_batch();
    if (!B) return PPCG_ENOMEM;
    auto fail = [&](int rc) {
      B->mem.release();
      if (B->h_sc) (void)hipHostFree(B->h_sc);
      delete B;
      return rc;
    };
    B->dtype = dtype;
    B->nch = nchains;
    if (hipGetDevice(&B->device) != hipSuccess) return fail(PPCG_EHIP);
    B->ch.resize(nchains);
    for (int32_t c = 0; c < nchains; ++c) {
      B->ch[c].X = X[c];
      B->ch[c].n = X[c]->n;
      B->ch[c].p = X[c]->p;
      const int rc = alloc_chain(B, B->ch[c]);
      if (rc) return fail(rc);
    }
    if (B->mem.alloc(&B->sc, (size_t)nchains) != hipSuccess) return fail(PPCG_ENOMEM);
    if (hipMemset(B->sc, 0, sizeof(DevScal) * nchains) != hipSuccess) return fail(PPCG_EHIP);
    if (hipHostMalloc(reinterpret_cast<void**>(&B->h_sc), sizeof(DevScal) * nchains, 0) !=
        hipSuccess) {
      B->h_sc = nullptr;
      return fail(PPCG_ENOMEM);
    }
    std::memset(B->h_sc, 0, sizeof(DevScal) * nchains);
    int rc = 0;
    if (dtype == PPCG_F64) {
      if ((rc = build_pass_jobs<double>(B, kJobRow)) || (rc = build_pass_jobs<double>(B, kJobCol)) ||
          (rc = build_vec_jobs<double>(B)))
        return fail(rc);
    } else {
      if ((rc = build_pass_jobs<float>(B, kJobRow)) || (rc = build_pass_jobs<float>(B, kJobCol)) ||
          (rc = build_vec_jobs<float>(B)))
        return fail(rc);
    }
    if ((rc = build_pass_jobs<double>(B, kJobRow64)) || (rc = build_pass_jobs<double>(B, kJobCol64)) ||
        (rc = build_pass_jobs<double>(B, kJobRhs64)))
      return fail(rc);
    if (hipDeviceSynchronize() != hipSuccess) return fail(PPCG_EHIP);
    *out = B;
    return PPCG_OK;
  } catch (const std::bad_alloc&) {
    return PPCG_ENOMEM;
  } catch (...) {
    return PPCG_EINVAL;
  }
}

int ppcg_batch_create_shared(ppcg_batch** out, int32_t nchains, int64_t n, int64_t p,
                             int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                             int32_t mem, int32_t dtype, hipStream_t stream) {
  try {
    if (!out) return PPCG_EINVAL;
    *out = nullptr;
    if (nchains < 1 || nchains > 8 || !valid_dtype(dtype)) return PPCG_EINVAL;
    if (n < 1 || p < 1 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx)) return PPCG_EINVAL;
    if (n >= INT32_MAX || p >= INT32_MAX || nnz >= ((int64_t)INT32_MAX) * 1024) return PPCG_EINVAL;
    if (mem != PPCG_MEM_HOST && mem != PPCG_MEM_DEVICE) return PPCG_EINVAL;
    std::vector<int64_t> rp, cp;
    std::vector<int32_t> ci, ri;
    {
      const int rc = read_binary_csr(n, p, nnz, row_ptr, col_idx, mem, stream, rp, ci, cp, ri);
      if (rc) return rc;
    }
    ppcg_batch* B = new (std::nothrow) ppcg_batch();
    if (!B) return PPCG_ENOMEM;
    auto fail = [&](int rc) {
      B->mem.release();
      if (B->h_sc) (void)hipHostFree(B->h_sc);
      delete B;
      return rc;
    };
    B->shared = true;
    B->dtype = dtype;
    B->nch = nchains;
    // Groups of at most four chains: a pass over eight FP64 vectors needs
    // more registers than a 1024-thread workgroup leaves a lane (two
    // four-vector passes measured faster than one with the spills), and
    // with two groups the chains that iterate longest share one
    B->K = nchains <= 2 ? 2 : 4;
    B->G = (nchains + B->K - 1) / B->K;
    B->n = n;
    B->p = p;
    const int K = B->K;
    const size_t KG = (size_t)K * B->G;  // vector slots
    if (hipGetDevice(&B->device) != hipSuccess) return fail(PPCG_EHIP);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, B->device) !=
            hipSuccess || ncu < 1)
      ncu = 256;
    if (setup_pass_kernels() != hipSuccess) return fail(PPCG_EHIP);
    // K-wide tables (the panel holds K values per entry): FP64 always, FP32
    // for the FP32 form; built on host threads, then uploaded.
    {
      const int nt = dtype == PPCG_F64 ? 2 : 4;
      PanelBuild Bt[4];
      auto job = [&](int q) {
        const int elem = (q / 2) == 0 ? 8 : 4;
        if (q % 2 == 0)
          build_panels(rp, ci, n, p, elem * K, ncu, Bt[q]);
        else
          build_panels(cp, ri, p, n, elem * K, ncu, Bt[q]);
      };
      std::vector<std::thread> th;
      int started = 1;
      try {
        for (int q = 1; q < nt; ++q, ++started) th.emplace_back(job, q);
      } catch (...) {
      }
      job(0);
      for (auto& t : th) t.join();
      for (int q = started; q < nt; ++q) job(q);
      for (int q = 0; q < nt; ++q) {
        Orient& o = (q % 2 == 0) ? B->srows[q / 2] : B->scols[q / 2];
        const int rc = upload_orient(B->mem, Bt[q], (q / 2) == 0 ? 8 : 4, K, o);
        if (rc) return fail(rc);
        Bt[q] = PanelBuild();
      }
    }
    B->ch.resize(nchains);
    for (int32_t c = 0; c < nchains; ++c) {
      B->ch[c].n = n;
      B->ch[c].p = p;
      const int rc = alloc_chain(B, B->ch[c]);
      if (rc) return fail(rc);
    }
    const size_t ts = dtype == PPCG_F64 ? 8 : 4;
    unsigned char *omT = nullptr, *sK = nullptr, *qK = nullptr;
    const int tl = dtype == PPCG_F64 ? 0 : 1;
    if (B->mem.alloc(&B->y_K, (size_t)n * KG) != hipSuccess ||
        B->mem.alloc(&B->om64_K, (size_t)n * KG) != hipSuccess ||
        B->mem.alloc(&B->beta_K, (size_t)p * KG) != hipSuccess ||
        B->mem.alloc(&B->z_K, (size_t)p * KG) != hipSuccess ||
        B->mem.alloc(&B->d_K, (size_t)p * KG) != hipSuccess ||
        B->mem.alloc(&B->p1_K, (size_t)B->srows[tl].pass.nwg * KG) != hipSuccess ||
        B->mem.alloc(&B->p2_K, (size_t)B->scols[tl].pass.nwg * KG) != hipSuccess ||
        B->mem.alloc(&sK, 2 * (size_t)p * KG * ts) != hipSuccess ||
        B->mem.alloc(&qK, (size_t)p * KG * ts) != hipSuccess)
      return fail(PPCG_ENOMEM);
    B->q_K = qK;
    if (dtype == PPCG_F32) {
      if (B->mem.alloc(&omT, (size_t)n * KG * ts) != hipSuccess) return fail(PPCG_ENOMEM);
      B->omT_K = omT;
    } else {
      B->omT_K = B->om64_K;
    }
    B->s_K = sK;
    // vector slots beyond the chains stay zero (their products are ignored)
    if (hipMemset(B->y_K, 0, (size_t)n * KG * 8) != hipSuccess ||
        hipMemset(B->om64_K, 0, (size_t)n * KG * 8) != hipSuccess ||
        hipMemset(B->beta_K, 0, (size_t)p * KG * 8) != hipSuccess ||
        hipMemset(B->z_K, 0, (size_t)p * KG * 8) != hipSuccess ||
        hipMemset(B->d_K, 0, (size_t)p * KG * 8) != hipSuccess ||
        hipMemset(sK, 0, 2 * (size_t)p * KG * ts) != hipSuccess ||
        (omT && hipMemset(omT, 0, (size_t)n * KG * ts) != hipSuccess))
      return fail(PPCG_EHIP);
    // one scalar block per vector slot; slots beyond the chains stay done
    if (B->mem.alloc(&B->sc, KG) != hipSuccess) return fail(PPCG_ENOMEM);
    {
      std::vector<DevScal> init(KG);
      std::memset(init.data(), 0, sizeof(DevScal) * KG);
      for (size_t c = (size_t)nchains; c < KG; ++c) init[c].done = 1;
      if (hipMemcpy(B->sc, init.data(), sizeof(DevScal) * KG, hipMemcpyHostToDevice) !=
          hipSuccess)
        return fail(PPCG_EHIP);
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&B->h_sc), sizeof(DevScal) * KG, 0) !=
        hipSuccess) {
      B->h_sc = nullptr;
      return fail(PPCG_ENOMEM);
    }
    std::memset(B->h_sc, 0, sizeof(DevScal) * KG);
    B->slot_of.resize(nchains);
    B->chain_at.resize(nchains);
    B->last_iters.assign(nchains, 0);
    for (int32_t c = 0; c < nchains; ++c) B->slot_of[c] = B->chain_at[c] = c;
    const int rc = dtype == PPCG_F64 ? build_vec_jobs<double>(B) : build_vec_jobs<float>(B);
    if (rc) return fail(rc);
    if (hipDeviceSynchronize() != hipSuccess) return fail(PPCG_EHIP);
    *out = B;
    return PPCG_OK;
  } catch (const std::bad_alloc&) {
    return PPCG_ENOMEM;
  } catch (...) {
    return PPCG_EINVAL;
  }
}

int ppcg_batch_destroy(ppcg_batch* B) {
  if (!B) return PPCG_OK;
  (void)hipDeviceSynchronize();
  drop_graphs(B);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  B->mem.release();
  if (B->h_sc) (void)hipHostFree(B->h_sc);
  delete B;
  return PPCG_OK;
}

int ppcg_draw_batched(ppcg_batch* B, const ppcg_chain* chains, const ppcg_options* opt,
                      ppcg_info* infos, hipStream_t stream) {
  return batched_entry(B, chains, opt, infos, true, stream);
}

int ppcg_solve_batched(ppcg_batch* B, const ppcg_chain* chains, const ppcg_options* opt,
                       ppcg_info* infos, hipStream_t stream) {
  return batched_entry(B, chains, opt, infos, false, stream);
}

}  // extern "C"
