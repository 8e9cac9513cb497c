// Internal interface between the C-ABI host layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppcg_layout.h"

namespace ppcg {

constexpr int kWG = 256;            // threads per workgroup (4 wavefronts of 64)
// Variants of the X pass: plain, the CG loop's row pass (DirIn), the CG
// loop's column pass (DotOut).
enum { kPassPlain = 0, kPassDir = 1, kPassDot = 2 };
constexpr int kMaxRedBlocks = 1024; // max workgroups of a p-vector phase

// ---- X passes ----
// One orientation of X (rows of CSR for v -> X v, columns of CSC for
// w -> X^T w) in a panel-blocked, index-only layout.  The gathered
// dimension is cut into panels of at most W entries so that a panel of the
// gathered vector fits in LDS; the elements of each (segment, panel) pair are
// stored as indices local to the panel, in 16-byte groups (ppcg_layout.h:
// compact or wide groups for one vector, kPV 16-bit indices padded with the
// index W, an LDS zero, for K interleaved vectors).  Chunks (ChunkDesc, ppcg_layout.h) are the units
// a wavefront reads: packed chunks give each of their segments a lane range
// for up to kPR windows, long chunks run one segment over up to kPLongWin
// windows, and pieces are parts of a longer segment whose sums the consumer
// adds.  Workgroup w serves panel wg_panel[w]; its wavefront q runs the
// chunks [wave_c[kPWaves w + q], wave_c[kPWaves w + q + 1]) in order.
struct PanelPass {
  const uint16_t* idx;      // [stream] 16-bit words of the index groups
  const ChunkDesc* chunks;  // [nchunks]
  const int32_t* seg_out;   // [entries + 1] output slot = panel * out_dim + segment id;
                            // entry no_slot (the last) is -1: no output
  const int32_t* wg_panel;  // [nwg]
  const int32_t* wave_c;    // [kPWaves * nwg + 1]
  const int32_t* wg_s0;     // [nwg] gathered entries [s0, s1) the workgroup owns
  const int32_t* wg_s1;
  int64_t gdim;             // gathered dimension (p for rows, n for columns)
  int64_t out_dim;          // outputs per panel
  int32_t W;                // panel width
  int32_t nwg;
  int32_t nchunks;
  int32_t npieces;
  int32_t no_slot;          // index of seg_out's trailing -1 entry
};

// value(i) = scale[i es] * (sum_k part[k * stride + i es] + sum of the pieces
// of i): the input a pass gathers, or the consumer's view of a pass output.
// es is 1 for one vector; K when K vectors are interleaved ([dim][K], with
// the pointers offset to the vector wanted).
template <typename T>
struct Combine {
  const T* part;
  int64_t stride;
  int32_t nparts;
  int32_t es;
  const T* scale;         // may be null
  const int32_t* sp_off;  // [dim + 1] pieces of element i (null: none)
  const int32_t* sp_c0;   // piece id ranges [c0, c1]
  const int32_t* sp_c1;
  const T* piece;         // [npieces] piece sums
};

// Scalars of one CG run, in device memory.
struct DevScal {
  double rho;      // <r, M^-1 r> = ||r~||^2
  double alpha;    // step length
  double betacg;   // direction update ratio
  double sq;       // <s, Phi s>
  double thresh2;  // squared threshold of the stopping rule
  double loop2;    // squared threshold the recursive residual is run to
  double rho_prev; // rho of the previous iteration
  double bm2;      // <b, M^-1 b>
  double bb;       // <b, b>
  double rr;       // <r, r>
  double meas;     // current rule measure (squared)
  double true_meas;// rule measure of the FP64 true residual (squared)
  double true_rm;  // <r_t, M^-1 r_t> of the true residual
  double grad_sum; // reduction output of the adjoint epilogue
  double rho_par[2]; // rho by iteration parity (row passes that finish the step)
  int32_t iters;
  int32_t done;
  int32_t status;
  int32_t max_iter;
  int32_t criterion;
  int32_t refined;  // set by a mode-1 restart
  uint32_t arrive[8]; // last-arriver counters of the reduction phases
};

struct VecWork {
  double* part;   // [kMaxRedBlocks * 4] per-block partial sums
  DevScal* sc;
};

// Row pass of the CG loop: the panel being gathered is the new direction
// s = z + (rho'/rho) s_old (z = M^-1 r, the ratio from each vector's scalars),
// formed while the panel is assembled; the workgroup writes its entries
// [wg_s0, wg_s1) of s and its part of <s, d s> (p1[w K + r]).  The two s
// buffers are s and s + sstride (old / new by the launch's parity).  All
// vectors are [dim][K] (K = 1: plain vectors).
//
// With sp set (one vector), the row pass also finishes the step before it:
// the step kernel left per-block partials of <r, M^-1 r> and <r, r> (nsb
// blocks, at sp + (1 - parity) * 2 * kMaxRedBlocks); every wavefront totals
// them in the order of the step's own reduction, forms the ratio and applies
// the stopping rule, and workgroup 0 records the scalars (iteration it of the
// phase; it = 0: the start kernel left them, s = z).
template <typename T>
struct DirIn {
  const double* z;
  T* s;
  int64_t sstride;
  const double* d;
  DevScal* sc;  // vector r's scalars at sc + r * scstride
  int32_t scstride;
  int32_t pad;
  double* p1;
  const double* sp;
  int32_t nsb;
  int32_t it;
};

// Column pass of the CG loop: each workgroup also sums s_j times every
// output (segment sum) it writes for column j, per vector (p2[w K + r]);
// s is the new direction (the buffer the row pass wrote).
template <typename T>
struct DotOut {
  const T* s;
  int64_t sstride;
  double* p2;
};

// ---- many chains in one launch ----
// One chain's X pass in a batched launch.
template <typename T>
struct PanelJob {
  PanelPass t;
  Combine<T> x;
  T* part_out;
  T* piece_out;
  const T* out_scale;
  const int32_t* done;
  DirIn<T> dir;
  DotOut<T> dot;
};

// One chain's p-vector state in a batched launch (nblk blocks).
template <typename T>
struct VecJob {
  VecWork w;
  T* s;              // direction buffers s and s + sstride
  int64_t sstride;
  double* z;         // M^-1 r for the next row pass ([p] with stride zes)
  const double* p1;  // the passes' workgroup partials of <s, d s> and <s, X^T u>
  const double* p2;  //   (stride pstride)
  int32_t n1, n2, pstride, zes;
  Combine<T> qsrc;   // the column pass's view of q
  T* qx;
  const double* b;
  const double* qx64;  // FP64 product part (restart and true-residual modes)
  const double* d;
  const double* m;
  double* beta;
  double* r;
  int64_t p;
  int32_t max_iter;    // the chain's iteration cap when the call gives none
  int32_t nblk;
  int32_t es;          // element stride of s (K when the chains' s are interleaved)
  int32_t pad;
};

// ---- launchers (all asynchronous on `st`) ----
// One X pass: gathers value(x, .) panel by panel and writes the segment sums
// of panel k to part_out[k * out_dim + id] (times out_scale[id] when given:
// only for a single-panel table without pieces), piece sums to piece_out.
// With ev0/ev1 the dispatch records the kernel's start and end in them.
template <typename T>
hipError_t launch_panel_pass(const PanelPass& t, const Combine<T>& x, T* part_out,
                             T* piece_out, const T* out_scale, const int32_t* done,
                             hipStream_t st, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr, const DirIn<T>* dir = nullptr,
                             const DotOut<T>* dot = nullptr, int parity = 0);

// out[i] = value(c, i) for i < dim.
template <typename T, typename U>
hipError_t launch_combine(const Combine<T>& c, int64_t dim, U* out, hipStream_t st);

// out[j * K + r] = value(c, j, r) for j < dim, r < K (c.es == K); a no-op
// launch once all K flags done[r * dstride] are set.
template <typename T>
hipError_t launch_combine_k(const Combine<T>& c, int K, int64_t dim, T* out,
                            const int32_t* done, int dstride, hipStream_t st);

// Maximum dynamic LDS the pass kernels may use (call once per device).
hipError_t setup_pass_kernels();

hipError_t launch_prep(const void* lambda, const void* omega, int dtype, double tau,
                       int64_t n, int64_t p, double* d, double* m, double* omega64,
                       hipStream_t st);

// General diagonal prior (Supplement S4.3): d = prior_prec, m = precond_inv
// (NULL: 1 / prior_prec), omega64 as launch_prep.
hipError_t launch_prep_general(const double* prior_prec, const double* precond_inv,
                               const void* omega, int dtype, int64_t n, int64_t p, double* d,
                               double* m, double* omega64, hipStream_t st);

hipError_t launch_y_draw(const double* omega64, const void* z, int dtype, uint64_t seed,
                         uint64_t chain, uint64_t draw, int64_t n, double* y, hipStream_t st);

hipError_t launch_rhs_fin(const double* bx, const void* lambda, int dtype, double tau,
                          uint64_t seed, uint64_t chain, uint64_t draw, int64_t p,
                          double* b, hipStream_t st);

// b = bx + sqrt(d) .* delta (Prop 2.1 with the prior precision diag(d)).
hipError_t launch_rhs_fin_general(const double* bx, const double* d, uint64_t seed,
                                  uint64_t chain, uint64_t draw, int64_t p, double* b,
                                  hipStream_t st);

// out[j] = value(c, j) + d[j] (diag(Phi) from the column pass of omega).
hipError_t launch_phi_diag(const Combine<double>& c, const double* d, int64_t p, double* out,
                           hipStream_t st);

hipError_t launch_normals(uint64_t seed, uint64_t stream_id, uint64_t chain, uint64_t draw,
                          int64_t count, double* out, hipStream_t st);

// omega_i ~ PG(1, psi_i) (and, with y, z_i = (y_i - 1/2) / omega_i) in `dtype`.
hipError_t launch_pg_omega(const double* psi, const uint8_t* y, int64_t n, uint64_t seed,
                           uint64_t chain, uint64_t draw, int dtype, void* omega_out, void* z_out,
                           hipStream_t st);
hipError_t launch_convert_to_f64(const void* in, int dtype, int64_t count, double* out,
                                 hipStream_t st);
hipError_t launch_convert_from_f64(const double* in, int dtype, int64_t count, void* out,
                                   hipStream_t st);

// Up to eight FP64 source vectors (kernel argument).
struct VecPtrs {
  const double* p[8];
};
// dst[i K + r] = (T) src[r][i] for r < nsrc, i < dim.
template <typename T>
hipError_t launch_interleave(const VecPtrs& src, int nsrc, int K, int64_t dim, T* dst,
                             hipStream_t st);

// out = qx + d .* v  (dtype T in and out).
template <typename T>
hipError_t launch_phi_finish(const T* qx, const double* d, const T* v, int64_t p, T* out,
                             hipStream_t st);

// CG start and restart.  If qx64 != NULL, r = b - qx64 - d .* beta, else
// r = b (beta must then be zero).  z = M^-1 r (the first row pass forms s = z
// from it: the direction ratio is zero after a start).
// mode 0: fresh start: also computes <b,Mb>, <b,b> and the thresholds (the
//         recursion runs to loop_factor * tol);
// mode 1: restart from the FP64 true residual of the current beta (keeps the
//         thresholds);
// mode 2: true-residual check only (no state change; writes true_meas, true_rm).
// Modes 0 and 1 also copy the new scalars to `snap` when it is not null (a
// pinned host slot: the host's first convergence check reads the starting
// rule measure there).
hipError_t launch_cg_start(VecWork w, int mode, const double* b, const double* qx64,
                           const double* d, const double* m, double* beta, double* r,
                           double* z, int64_t p, double tol, int criterion, int max_iter,
                           double loop_factor, hipStream_t st, DevScal* snap = nullptr);

// After the column pass: <s, Phi s> from the passes' workgroup partials
// (fixed order), alpha = rho / <s, Phi s>; q = qx + d .* s with qx from the
// column pass's panel partials; beta += alpha s; r -= alpha q; z = M^-1 r;
// rho' = <r, z> and the stopping rule.  s is the new direction (buffer
// 1 - parity of s).  With pass_finish the kernel stops at the per-block
// partials of rho' and <r, r> (in w.part + parity * 2 * kMaxRedBlocks) and the
// next row pass finishes the step (DirIn.sp); otherwise its last block does.
// With pass_finish and snap set, the kernel also copies the scalars to snap
// (host memory mapped for the device, e.g. a pinned readback slot) once they
// are final for this launch, in place of a copy operation after it.
template <typename T>
hipError_t launch_cg_step(VecWork w, const T* s, int64_t sstride, int parity, bool pass_finish,
                          const Combine<T>& qsrc, const double* d, const double* m,
                          double* beta, double* r, double* z, const double* p1, int32_t n1,
                          const double* p2, int32_t n2, int64_t p, hipStream_t st,
                          DevScal* snap = nullptr);

// One X pass over K in {2, 4} interleaved vectors ([dim][K] inputs and
// outputs; part_out[(k * out_dim + id) * K + r]); skipped when the K flags
// done[i * dstride] are all set (done may be null).  dir / dot as for
// launch_panel_pass, over the K vectors.
template <typename T>
hipError_t launch_panel_pass_k(int K, const PanelPass& t, const Combine<T>& x, T* part_out,
                               T* piece_out, const T* out_scale, const int32_t* done,
                               int dstride, hipStream_t st, const DirIn<T>* dir = nullptr,
                               const DotOut<T>* dot = nullptr, int parity = 0);

// Blocks of one chain's p-vector phases.
int32_t vec_blocks(int64_t p);

// Workgroup g of a batched pass runs workgroup wg_local[g] of job wg_job[g].
template <typename T>
hipError_t launch_panel_pass_batched(const PanelJob<T>* jobs, const int32_t* wg_job,
                                     const int32_t* wg_local, int32_t nwg, int mode, int parity,
                                     hipStream_t st);
// Block g runs block blk_local[g] of chain blk_job[g] (nblk blocks in all);
// max_iter <= 0 takes each chain's own cap.
template <typename T>
hipError_t launch_cg_start_batched(const VecJob<T>* jobs, const int32_t* blk_job,
                                   const int32_t* blk_local, int32_t nblk, int mode, double tol,
                                   int criterion, int max_iter, double loop_factor,
                                   hipStream_t st);
// The step kernel (launch_cg_step) of the chains listed in blk_job.
template <typename T>
hipError_t launch_cg_step_batched(const VecJob<T>* jobs, const int32_t* blk_job,
                                  const int32_t* blk_local, int32_t nblk, int parity,
                                  hipStream_t st);

// Adjoint epilogue: grad_b = a, grad_loglambda = 2 d a beta, grad_logtau = sum.
hipError_t launch_adjoint_epilogue(VecWork w, const double* a, const void* beta, int dtype,
                                   const double* d, int64_t p, void* grad_b,
                                   void* grad_loglambda, double* grad_logtau,
                                   hipStream_t st);

}  // namespace ppcg
