// Internal state of the C-ABI handles (matrix and batch) shared by the host
// sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "../../include/ppcg.h"
#include "ppcg_kernels.h"
#include "ppcg_panels.h"

namespace ppcg {

struct DevBuf {
  std::vector<void*> ptrs;
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    *out = reinterpret_cast<T*>(p);
    return hipSuccess;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

// One orientation of X at one precision on the device.
struct Orient {
  PanelPass pass{};
  void* part = nullptr;   // [npanels][out_dim] segment sums (zero where absent)
  void* piece = nullptr;  // [npieces] piece sums
  const int32_t* sp_off = nullptr;
  const int32_t* sp_c0 = nullptr;
  const int32_t* sp_c1 = nullptr;
  int32_t npanels = 0;
  int64_t out_dim = 0;
  int64_t dev_bytes = 0;
  int64_t pass_bytes = 0;  // algorithmic bytes of one launch (inputs counted once)
};

}  // namespace ppcg

struct ppcg_matrix {
  int64_t n = 0, p = 0, nnz = 0;
  int device = 0;
  int ncu = 256;
  ppcg::DevBuf mem;
  ppcg::Orient rows[2], cols[2];  // [0]: FP64 tables, [1]: FP32 tables
  // workspace
  double *qx64 = nullptr, *y64 = nullptr, *omega64 = nullptr;
  double *d = nullptr, *m = nullptr, *b64 = nullptr, *beta64 = nullptr, *r64 = nullptr,
         *s64 = nullptr;
  float *qx32 = nullptr, *s32 = nullptr;  // s64, s32: two direction buffers of p each
  double* z64 = nullptr;                  // M^-1 r for the next row pass
  double *p1[2] = {}, *p2[2] = {};        // workgroup partials of the passes, per table
  double* part = nullptr;
  ppcg::DevScal* sc = nullptr;
  ppcg::DevScal* h_sc = nullptr;  // pinned host mirror: [0] the result, [0..1] check slots,
                                  // [2] the scalars a start left
  hipEvent_t chk[2] = {};         // one per check slot: that batch's flags are on the host
  // CG iterations of the last converged solve phase, [phase: 0 first from zero, 1 first
  // from a caller's beta0, 2 refinement][table]: the first check batch of the next such
  // phase is sized from it (0: none)
  int32_t iter_hint[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  // pass timing (ppcg_matrix_profile)
  int profile = 0;
  std::vector<hipEvent_t> ev;  // 4 per iteration of a check batch
  double pass_ms[2] = {0.0, 0.0};
  int64_t pass_cnt[2] = {0, 0};
};

#define PPCG_TRY_HIP(...)                     \
  do {                                        \
    hipError_t _e = (__VA_ARGS__);            \
    if (_e != hipSuccess) return PPCG_EHIP;   \
  } while (0)

#define PPCG_TRY_ALLOC(...)                                                \
  do {                                                                     \
    hipError_t _e = (__VA_ARGS__);                                         \
    if (_e == hipErrorOutOfMemory || _e == hipErrorMemoryAllocation)       \
      return PPCG_ENOMEM;                                                  \
    if (_e != hipSuccess) return PPCG_EHIP;                                \
  } while (0)


namespace ppcg {

// ---- helpers shared by the entry points ----
inline bool valid_dtype(int32_t d) { return d == PPCG_F64 || d == PPCG_F32; }

inline ppcg_options resolve(const ppcg_options* o, int64_t p) {
  ppcg_options r;
  if (o) {
    r = *o;
  } else {
    ppcg_options_default(&r, PPCG_F64);
  }
  if (r.max_iter <= 0) r.max_iter = (int32_t)std::min<int64_t>(p, INT32_MAX);
  if (r.refine < 0) r.refine = (r.dtype == PPCG_F32) ? 1 : 0;
  if (r.check_every <= 0) r.check_every = 16;
  return r;
}

inline int check_opts(const ppcg_options& o) {
  if (!valid_dtype(o.dtype)) return PPCG_EINVAL;
  if (o.criterion < 0 || o.criterion > 2) return PPCG_EINVAL;
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return PPCG_EINVAL;
  if (!(o.loop_factor >= 0.0) || !(o.loop_factor <= 1.0)) return PPCG_EINVAL;
  return PPCG_OK;
}

inline VecWork vw(ppcg_matrix* X) { return VecWork{X->part, X->sc}; }

template <typename T>
constexpr int prec_index() {
  return sizeof(T) == 8 ? 0 : 1;
}

template <typename T>
inline Combine<T> comb_vec(const T* v) {
  Combine<T> c{};
  c.es = 1;
  c.part = v;
  c.stride = 0;
  c.nparts = 1;
  return c;
}

// The consumer's view of an orientation's pass output (optionally scaled).
template <typename T>
inline Combine<T> comb_out(const Orient& o, const T* scale) {
  Combine<T> c{};
  c.es = 1;
  c.part = reinterpret_cast<const T*>(o.part);
  c.stride = o.out_dim;
  c.nparts = o.npanels;
  c.scale = scale;
  c.sp_off = o.sp_off;
  c.sp_c0 = o.sp_c0;
  c.sp_c1 = o.sp_c1;
  c.piece = reinterpret_cast<const T*>(o.piece);
  return c;
}

// Whether the row pass can apply omega itself: one panel and no pieces, so
// each row's sum is complete when the pass writes it.
inline bool rows_direct(const Orient& o) { return o.npanels == 1 && o.sp_off == nullptr; }

inline double ratio(double meas, double thresh2) {
  if (thresh2 > 0.0) return std::sqrt(meas / thresh2);
  return meas > 0.0 ? std::numeric_limits<double>::infinity() : 0.0;
}

inline bool bad_tau(double tau) { return !(tau > 0.0) || !std::isfinite(tau); }

// Uploads a host table to device memory owned by `mem`.
template <typename V>
int upload_vec(DevBuf& mem, const std::vector<V>& h, const V** out, int64_t* bytes) {
  V* d = nullptr;
  PPCG_TRY_ALLOC(mem.alloc(&d, h.size()));
  if (!h.empty())
    PPCG_TRY_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  *out = d;
  *bytes += (int64_t)(h.size() * sizeof(V));
  return PPCG_OK;
}

// Uploads one orientation's tables and allocates its outputs for K
// interleaved vectors of `elem`-byte values (K = 1: one vector).
int upload_orient(DevBuf& mem, const PanelBuild& B, int elem, int K, Orient& o);

// Reads (host or device), validates and sorts out a binary CSR: rp, ci as
// given, cp, ri the CSC twin.  PPCG_EINVAL on malformed input, PPCG_ENODEV
// without a device.
int read_binary_csr(int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                    const int32_t* col_idx, int32_t mem, hipStream_t stream,
                    std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                    std::vector<int64_t>& cp, std::vector<int32_t>& ri);

}  // namespace ppcg
