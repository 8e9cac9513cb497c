// Phi v without any device allocation: the entry point for callers that
// cannot allocate (code under HIP graph capture, tight serving loops).
//
// ppcg_phi_matvec runs its two X passes into output buffers of the handle
// and forms d = tau^-2 lambda^-2 and the combined X^T u in handle workspace.
// This variant runs the same kernels with all of that scratch carved out of
// one file-scope device array of fixed size, so the call allocates nothing
// and leaves the handle's workspace untouched.  Each device holds its own
// copy of the array; its address is looked up once per device and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ppcg.h"
#include "ppcg_handle.h"
#include "ppcg_kernels.h"

using namespace ppcg;

namespace {

static __device__ __align__(256) unsigned char scratch[PPCG_NOALLOC_SCRATCH_BYTES];

// Device addresses of `scratch`, one per device (the host-side name is only
// a stand-in and must never reach a kernel).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

int scratch_on(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return PPCG_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return PPCG_EHIP;
    g_scratch[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[device];
  return PPCG_OK;
}

// Consecutive 256-byte aligned regions of the scratch array.
struct Carve {
  size_t end = 0;
  size_t take(size_t bytes) {
    const size_t at = end;
    end += (bytes + 255) & ~(size_t)255;
    return at;
  }
};

// Zero-fills `words` 8-byte words (a kernel rather than a memset node, so
// that a captured graph replays it like any other launch).
__global__ __launch_bounds__(256) void k_zero_words(uint64_t* p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

hipError_t zero_region(unsigned char* at, size_t bytes, hipStream_t st) {
  const int64_t words = (int64_t)(((bytes + 255) & ~(size_t)255) / 8);
  if (words == 0) return hipSuccess;
  int64_t blocks = (words + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, st,
                     reinterpret_cast<uint64_t*>(at), words);
  return hipGetLastError();
}

template <typename T>
int phi_matvec_scratch(const ppcg_matrix* X, const void* omega, const void* lambda, double tau,
                       const T* v, T* out, int32_t dtype, hipStream_t st) {
  const int ti = prec_index<T>();
  Orient r = X->rows[ti], c = X->cols[ti];  // copies: the outputs go to scratch
  Carve cv;
  const size_t d_at = cv.take(sizeof(double) * (size_t)X->p);
  const size_t m_at = cv.take(sizeof(double) * (size_t)X->p);
  const size_t rpart_bytes = sizeof(T) * (size_t)r.npanels * (size_t)r.out_dim;
  const size_t cpart_bytes = sizeof(T) * (size_t)c.npanels * (size_t)c.out_dim;
  const size_t rpart_at = cv.take(rpart_bytes);
  const size_t rpiece_at = cv.take(sizeof(T) * (size_t)(r.pass.npieces > 0 ? r.pass.npieces : 1));
  const size_t cpart_at = cv.take(cpart_bytes);
  const size_t cpiece_at = cv.take(sizeof(T) * (size_t)(c.pass.npieces > 0 ? c.pass.npieces : 1));
  const size_t qx_at = cv.take(sizeof(T) * (size_t)X->p);
  if (cv.end > (size_t)PPCG_NOALLOC_SCRATCH_BYTES) return PPCG_ETOOBIG;

  unsigned char* base = nullptr;
  int rc = scratch_on(X->device, &base);
  if (rc) return rc;
  double* d = reinterpret_cast<double*>(base + d_at);
  double* m = reinterpret_cast<double*>(base + m_at);
  r.part = base + rpart_at;
  r.piece = base + rpiece_at;
  c.part = base + cpart_at;
  c.piece = base + cpiece_at;
  T* qx = reinterpret_cast<T*>(base + qx_at);

  // A pass writes only the (segment, panel) slots that hold elements; the
  // consumer reads every slot, so the rest must be zero, whatever an earlier
  // call left in the array.
  PPCG_TRY_HIP(zero_region(base + rpart_at, rpart_bytes, st));
  PPCG_TRY_HIP(zero_region(base + cpart_at, cpart_bytes, st));
  PPCG_TRY_HIP(launch_prep(lambda, omega, dtype, tau, X->n, X->p, d, m, nullptr, st));
  const T* om = reinterpret_cast<const T*>(omega);
  const bool direct = rows_direct(r);
  PPCG_TRY_HIP(launch_panel_pass<T>(r.pass, comb_vec<T>(v), reinterpret_cast<T*>(r.part),
                                    reinterpret_cast<T*>(r.piece), direct ? om : nullptr,
                                    nullptr, st));
  PPCG_TRY_HIP(launch_panel_pass<T>(c.pass, comb_out<T>(r, direct ? nullptr : om),
                                    reinterpret_cast<T*>(c.part), reinterpret_cast<T*>(c.piece),
                                    nullptr, nullptr, st));
  PPCG_TRY_HIP(launch_combine<T, T>(comb_out<T>(c, nullptr), X->p, qx, st));
  PPCG_TRY_HIP(launch_phi_finish<T>(qx, d, v, X->p, out, st));
  return PPCG_OK;
}

}  // namespace

int ppcg_phi_matvec_noalloc(const ppcg_matrix* X, const void* omega, const void* lambda,
                            double tau, const void* v, void* out, int32_t dtype,
                            hipStream_t stream) {
  if (!X || !omega || !lambda || !v || !out || !valid_dtype(dtype) || bad_tau(tau))
    return PPCG_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PPCG_EHIP;
  if (dev != X->device) return PPCG_EINVAL;  // the tables and the scratch are per device
  if (dtype == PPCG_F64)
    return phi_matvec_scratch<double>(X, omega, lambda, tau, reinterpret_cast<const double*>(v),
                                      reinterpret_cast<double*>(out), dtype, stream);
  return phi_matvec_scratch<float>(X, omega, lambda, tau, reinterpret_cast<const float*>(v),
                                   reinterpret_cast<float*>(out), dtype, stream);
}
