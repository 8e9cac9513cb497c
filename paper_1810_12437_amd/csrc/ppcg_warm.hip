// Initial vector of the CG sampler (Supplement S4.1, choice of initial vector):
// a running sum of the draws rescaled by the shrinkage scales they were drawn
// under, and the next start beta0 = tau lambda * (sum / count).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/ppcg.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double load_as_f64(const void* p, int32_t dtype, int64_t i) {
  return dtype == PPCG_F64 ? static_cast<const double*>(p)[i]
                           : (double)static_cast<const float*>(p)[i];
}

__global__ __launch_bounds__(kBlock) void k_warm_accumulate(double* acc, const void* beta,
                                                            const void* lambda_prev,
                                                            double tau_prev, int32_t dtype,
                                                            int64_t p) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < p)
    acc[j] += load_as_f64(beta, dtype, j) / (tau_prev * load_as_f64(lambda_prev, dtype, j));
}

__global__ __launch_bounds__(kBlock) void k_warm_vector(void* beta0, const double* acc,
                                                        double count, const void* lambda,
                                                        double tau, int32_t dtype, int64_t p) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= p) return;
  const double v = tau * load_as_f64(lambda, dtype, j) * (acc[j] / count);
  if (dtype == PPCG_F64)
    static_cast<double*>(beta0)[j] = v;
  else
    static_cast<float*>(beta0)[j] = (float)v;
}

bool bad_scale(double v) { return !(v > 0.0) || v != v || v > 1.7976931348623157e308; }

}  // namespace

extern "C" {

int ppcg_warm_start_accumulate(double* acc, const void* beta, const void* lambda_prev,
                               double tau_prev, int32_t dtype, int64_t p, hipStream_t stream) {
  if (!acc || !beta || !lambda_prev || p < 1 || bad_scale(tau_prev) ||
      (dtype != PPCG_F64 && dtype != PPCG_F32))
    return PPCG_EINVAL;
  hipLaunchKernelGGL(k_warm_accumulate, dim3((unsigned)((p + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, stream, acc, beta, lambda_prev, tau_prev, dtype, p);
  return hipGetLastError() == hipSuccess ? PPCG_OK : PPCG_EHIP;
}

int ppcg_warm_start_vector(void* beta0, const double* acc, double count, const void* lambda,
                           double tau, int32_t dtype, int64_t p, hipStream_t stream) {
  if (!beta0 || !acc || !lambda || p < 1 || bad_scale(tau) || bad_scale(count) ||
      (dtype != PPCG_F64 && dtype != PPCG_F32))
    return PPCG_EINVAL;
  hipLaunchKernelGGL(k_warm_vector, dim3((unsigned)((p + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     stream, beta0, acc, count, lambda, tau, dtype, p);
  return hipGetLastError() == hipSuccess ? PPCG_OK : PPCG_EHIP;
}

}  // extern "C"
