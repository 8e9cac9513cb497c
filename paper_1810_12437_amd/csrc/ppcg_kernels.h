// Internal interface between the C-ABI host layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppcg {

constexpr int kWG = 256;            // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxRedBlocks = 1024; // max workgroups of a p-vector phase

// Chunked segment table: the non-empty segments (rows of CSR or columns of
// CSC) of one orientation of X, cut into chunks of at most C - 3 elements
// (C = kWG * V) along segment boundaries.  A chunk either packs whole
// segments (cnseg > 0) or is one piece of a segment longer than a chunk
// (cnseg == 0); the pieces of such a split segment are summed, in chunk
// order, by a follow-up kernel.  A chunk is processed from the 16-byte
// aligned element start & ~3, so its index loads are aligned.
struct SegTable {
  const int64_t* ptr;    // [nseg + 1] offsets of the non-empty segments
  const int32_t* sid;    // [nseg] original row / column id of each segment
  const int32_t* idx;    // [nnz] gathered index of each element
  const int64_t* cstart; // [nchunks + 1] first element of each chunk; last = nnz
  const int32_t* cseg;   // [nchunks] first (or split) segment of the chunk
  const int32_t* cnseg;  // [nchunks] whole segments in the chunk; 0 for a piece
  void* part;            // [nchunks] piece sums (T)
  const int32_t* split_seg; // [nsplit] segments longer than a chunk
  const int32_t* split_c0;  // [nsplit] their first piece chunk
  const int32_t* split_c1;  // [nsplit] their last piece chunk
  int64_t nnz;
  int32_t nseg;
  int32_t nchunks;
  int32_t nsplit;
  int32_t chunk;         // C
};

// Scalars of one CG run, in device memory.
struct DevScal {
  double rho;      // <r, M^-1 r> = ||r~||^2
  double alpha;    // step length
  double betacg;   // direction update ratio
  double sq;       // <s, Phi s>
  double thresh2;  // squared threshold of the stopping rule
  double bm2;      // <b, M^-1 b>
  double bb;       // <b, b>
  double rr;       // <r, r>
  double meas;     // current rule measure (squared)
  double true_meas;// rule measure of the FP64 true residual (squared)
  double true_rm;  // <r_t, M^-1 r_t> of the true residual
  double grad_sum; // reduction output of the adjoint epilogue
  int32_t iters;
  int32_t done;
  int32_t status;
  int32_t max_iter;
  int32_t criterion;
  int32_t pad0;
  uint32_t arrive[8]; // last-arriver counters of the reduction phases
};

struct VecWork {
  double* part;   // [kMaxRedBlocks * 4] per-block partial sums
  DevScal* sc;
};

// ---- launchers (all asynchronous on `st`) ----
// out = scale .* (X-orientation sum of x): a segmented gather-sum pass.
template <typename T>
hipError_t launch_segsum(const SegTable& t, const T* x, const T* scale, T* out,
                         const int32_t* done, hipStream_t st);

hipError_t launch_prep(const void* lambda, const void* omega, int dtype, double tau,
                       int64_t n, int64_t p, double* d, double* m, double* omega64,
                       hipStream_t st);

hipError_t launch_y_draw(const double* omega64, const void* z, int dtype, uint64_t seed,
                         uint64_t chain, uint64_t draw, int64_t n, double* y, hipStream_t st);

hipError_t launch_rhs_fin(const double* bx, const void* lambda, int dtype, double tau,
                          uint64_t seed, uint64_t chain, uint64_t draw, int64_t p,
                          double* b, hipStream_t st);

hipError_t launch_normals(uint64_t seed, uint64_t stream_id, uint64_t chain, uint64_t draw,
                          int64_t count, double* out, hipStream_t st);

hipError_t launch_convert_to_f64(const void* in, int dtype, int64_t count, double* out,
                                 hipStream_t st);
hipError_t launch_convert_from_f64(const double* in, int dtype, int64_t count, void* out,
                                   hipStream_t st);

// out = qx + d .* v  (dtype T in and out).
template <typename T>
hipError_t launch_phi_finish(const T* qx, const double* d, const T* v, int64_t p, T* out,
                             hipStream_t st);

// CG start / restart.  If qx64 != NULL, r = b - qx64 - d .* beta, else r = b
// (beta must then be zero).  z = m .* r, s = z.  mode 0: fresh start (computes
// <b,Mb>, <b,b>, threshold); mode 1: restart (keeps the threshold); mode 2:
// true-residual check only (no state change, writes true_meas / true_rm).
template <typename T>
hipError_t launch_cg_start(VecWork w, int mode, const double* b, const double* qx64,
                           const double* d, const double* m, double* beta, double* r,
                           T* s, int64_t p, double tol, int criterion, int max_iter,
                           hipStream_t st);

// One CG iteration's vector phases after the matvec q = qx + d .* s.
template <typename T>
hipError_t launch_cg_dot(VecWork w, const T* s, const T* qx, const double* d, int64_t p,
                         hipStream_t st);
template <typename T>
hipError_t launch_cg_update(VecWork w, const T* s, const T* qx, const double* d,
                            const double* m, double* beta, double* r, int64_t p,
                            hipStream_t st);
template <typename T>
hipError_t launch_cg_direction(VecWork w, const double* m, const double* r, T* s,
                               int64_t p, hipStream_t st);

// Adjoint epilogue: grad_b = a, grad_loglambda = 2 d a beta, grad_logtau = sum.
hipError_t launch_adjoint_epilogue(VecWork w, const double* a, const void* beta, int dtype,
                                   const double* d, int64_t p, void* grad_b,
                                   void* grad_loglambda, double* grad_logtau,
                                   hipStream_t st);

}  // namespace ppcg
