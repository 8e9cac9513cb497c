// Gibbs-level companions of the CG draw:
//  - the initial vector from the rescaled running mean of earlier draws
//    (Supplement S4.1, choice of initial vector);
//  - prior precision and preconditioner scales when some coefficients are
//    not shrunk, gamma_j = c eta_hat_j from the spread of earlier draws
//    (Supplement S4.3);
//  - the Jacobi preconditioner M = diag(Phi) and the adaptive choice between
//    it and the prior preconditioner (Section 3.3, Supplement S5.3).
// Everything here is elementwise over p or calls the library's own entry
// points; the X passes stay in the pass kernels.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <new>

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

// Welford's update of the running mean and sum of squared deviations with
// the count-th draw.
__global__ __launch_bounds__(kBlock) void k_moments_update(double* mean, double* m2,
                                                           const void* beta, int32_t dtype,
                                                           double count, int64_t q1) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= q1) return;
  const double x = load_as_f64(beta, dtype, j);
  const double dev = x - mean[j];
  const double mu = mean[j] + dev / count;
  mean[j] = mu;
  m2[j] += dev * (x - mu);
}

// d_j and m_j: the unshrunk block [0, q1) from sigma_j^-2 and c^2 times the
// sample variance m2_j / (count - 1) (NaN for a variance that is not
// positive, so a solve with it reports breakdown); the rest from tau lambda_j.
__global__ __launch_bounds__(kBlock) void k_unshrunk_setup(double* d, double* m,
                                                           const double* sigma_inv2,
                                                           const double* m2, double count,
                                                           double c2, const void* lambda,
                                                           double tau, int32_t dtype, int64_t q1,
                                                           int64_t p) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= p) return;
  double dj, mj;
  if (j < q1) {
    dj = sigma_inv2[j];
    const double var = m2[j] / (count - 1.0);
    mj = var > 0.0 ? c2 * var : __builtin_nan("");
  } else {
    const double s = tau * load_as_f64(lambda, dtype, j);
    dj = 1.0 / (s * s);
    mj = s * s;
  }
  d[j] = dj;
  if (m) m[j] = mj;
}

__global__ __launch_bounds__(kBlock) void k_reciprocal(double* v, int64_t p) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < p) v[j] = 1.0 / v[j];
}

bool bad_scale(double v) { return !(v > 0.0) || v != v || v > 1.7976931348623157e308; }
bool bad_dtype(int32_t dtype) { return dtype != PPCG_F64 && dtype != PPCG_F32; }
dim3 grid_for(int64_t count) { return dim3((unsigned)((count + kBlock - 1) / kBlock)); }
int launched() { return hipGetLastError() == hipSuccess ? PPCG_OK : PPCG_EHIP; }

}  // namespace

struct ppcg_switch {
  int64_t p = 0;
  int32_t period = 0;
  int32_t choice = PPCG_PRECOND_PRIOR;
  int64_t draws = 0;
  int32_t trial_iters[2] = {-1, -1};  // prior, Jacobi at the last trial
  double* m_jacobi = nullptr;         // p
  void* beta_alt = nullptr;           // p doubles (either dtype fits)
};

extern "C" {

int ppcg_warm_start_accumulate(double* acc, const void* beta, const void* lambda_prev,
                               double tau_prev, int32_t dtype, int64_t p, hipStream_t stream) {
  if (!acc || !beta || !lambda_prev || p < 1 || bad_scale(tau_prev) || bad_dtype(dtype))
    return PPCG_EINVAL;
  hipLaunchKernelGGL(k_warm_accumulate, grid_for(p), dim3(kBlock), 0, stream, acc, beta,
                     lambda_prev, tau_prev, dtype, p);
  return launched();
}

int ppcg_warm_start_vector(void* beta0, const double* acc, double count, const void* lambda,
                           double tau, int32_t dtype, int64_t p, hipStream_t stream) {
  if (!beta0 || !acc || !lambda || p < 1 || bad_scale(tau) || bad_scale(count) ||
      bad_dtype(dtype))
    return PPCG_EINVAL;
  hipLaunchKernelGGL(k_warm_vector, grid_for(p), dim3(kBlock), 0, stream, beta0, acc, count,
                     lambda, tau, dtype, p);
  return launched();
}

int ppcg_moments_update(double* mean, double* m2, const void* beta, int32_t dtype, int64_t q1,
                        int64_t count, hipStream_t stream) {
  if (!mean || !m2 || !beta || q1 < 1 || count < 1 || bad_dtype(dtype)) return PPCG_EINVAL;
  hipLaunchKernelGGL(k_moments_update, grid_for(q1), dim3(kBlock), 0, stream, mean, m2, beta,
                     dtype, (double)count, q1);
  return launched();
}

int ppcg_unshrunk_setup(double* prior_prec, double* precond_inv, const double* sigma_inv2,
                        const double* m2, int64_t count, double c, const void* lambda, double tau,
                        int32_t dtype, int64_t q1, int64_t p, hipStream_t stream) {
  if (!prior_prec || !lambda || p < 1 || q1 < 0 || q1 > p || bad_scale(tau) || bad_dtype(dtype))
    return PPCG_EINVAL;
  if (q1 > 0 && (!sigma_inv2 || (precond_inv && (!m2 || count < 2 || bad_scale(c)))))
    return PPCG_EINVAL;
  hipLaunchKernelGGL(k_unshrunk_setup, grid_for(p), dim3(kBlock), 0, stream, prior_prec,
                     precond_inv, sigma_inv2, m2, (double)count, c * c, lambda, tau, dtype, q1,
                     p);
  return launched();
}

int ppcg_jacobi_precond(const ppcg_matrix* X, const void* omega, int32_t dtype,
                        const double* prior_prec, double* precond_inv, hipStream_t stream) {
  int64_t n = 0, p = 0, nnz = 0;
  if (!X || !precond_inv || ppcg_matrix_shape(X, &n, &p, &nnz) != PPCG_OK) return PPCG_EINVAL;
  const int rc = ppcg_phi_diag(X, omega, dtype, prior_prec, precond_inv, stream);
  if (rc != PPCG_OK) return rc;
  hipLaunchKernelGGL(k_reciprocal, grid_for(p), dim3(kBlock), 0, stream, precond_inv, p);
  return launched();
}

int ppcg_switch_create(ppcg_switch** out, int64_t p, int32_t period) {
  if (!out || p < 1 || period < 1) return PPCG_EINVAL;
  *out = nullptr;
  ppcg_switch* S = new (std::nothrow) ppcg_switch;
  if (!S) return PPCG_ENOMEM;
  S->p = p;
  S->period = period;
  if (hipMalloc(&S->m_jacobi, sizeof(double) * p) != hipSuccess ||
      hipMalloc(&S->beta_alt, sizeof(double) * p) != hipSuccess) {
    (void)hipGetLastError();
    if (S->m_jacobi) (void)hipFree(S->m_jacobi);
    delete S;
    return PPCG_ENOMEM;
  }
  *out = S;
  return PPCG_OK;
}

int ppcg_switch_destroy(ppcg_switch* S) {
  if (!S) return PPCG_EINVAL;
  (void)hipFree(S->m_jacobi);
  (void)hipFree(S->beta_alt);
  delete S;
  return PPCG_OK;
}

int ppcg_switch_state(const ppcg_switch* S, int32_t* choice, int64_t* draws,
                      int32_t* iters_prior, int32_t* iters_jacobi) {
  if (!S) return PPCG_EINVAL;
  if (choice) *choice = S->choice;
  if (draws) *draws = S->draws;
  if (iters_prior) *iters_prior = S->trial_iters[0];
  if (iters_jacobi) *iters_jacobi = S->trial_iters[1];
  return PPCG_OK;
}

int ppcg_draw_switch(ppcg_switch* S, const ppcg_matrix* X, const void* omega, const void* z,
                     const double* prior_prec, const double* precond_inv, const void* beta0,
                     uint64_t seed, uint64_t chain, uint64_t draw_index, const ppcg_options* opt,
                     void* beta_out, ppcg_info* info, hipStream_t stream) {
  int64_t n = 0, p = 0, nnz = 0;
  if (!S || !X || ppcg_matrix_shape(X, &n, &p, &nnz) != PPCG_OK || p != S->p) return PPCG_EINVAL;
  const int32_t dtype = opt ? opt->dtype : PPCG_F64;
  if (bad_dtype(dtype)) return PPCG_EINVAL;
  ppcg_info local[2];
  const bool trial = S->draws % S->period == 0;
  int rc;
  if (trial || S->choice == PPCG_PRECOND_JACOBI) {
    rc = ppcg_jacobi_precond(X, omega, dtype, prior_prec, S->m_jacobi, stream);
    if (rc != PPCG_OK) return rc;
  }
  if (!trial) {
    const double* m = S->choice == PPCG_PRECOND_JACOBI ? S->m_jacobi : precond_inv;
    rc = ppcg_draw_general(X, omega, z, prior_prec, m, beta0, seed, chain, draw_index, opt,
                           beta_out, info, stream);
    if (rc == PPCG_EINVAL || rc == PPCG_ENOMEM || rc == PPCG_EHIP) return rc;
    ++S->draws;
    return rc;
  }
  // Trial: the same draw (same b, same start) under both preconditioners,
  // Jacobi first; the prior solve is then stopped at the Jacobi count, since
  // it can win only within it (an unbounded prior solve can run to p
  // iterations where it does not converge).
  const int rj = ppcg_draw_general(X, omega, z, prior_prec, S->m_jacobi, beta0, seed, chain,
                                   draw_index, opt, S->beta_alt, &local[1], stream);
  if (rj == PPCG_EINVAL || rj == PPCG_ENOMEM || rj == PPCG_EHIP) return rj;
  const int32_t ij = local[1].iters + local[1].refine_iters;
  ppcg_options capped;
  if (opt)
    capped = *opt;
  else
    ppcg_options_default(&capped, PPCG_F64);
  if (rj == PPCG_OK) capped.max_iter = ij > 0 ? ij : 1;
  const int rp = ppcg_draw_general(X, omega, z, prior_prec, precond_inv, beta0, seed, chain,
                                   draw_index, &capped, beta_out, &local[0], stream);
  if (rp == PPCG_EINVAL || rp == PPCG_ENOMEM || rp == PPCG_EHIP) return rp;
  const int32_t ip = local[0].iters + local[0].refine_iters;
  S->trial_iters[0] = ip;
  S->trial_iters[1] = ij;
  // Fewer iterations to the same stopping rule wins; a tie keeps the prior
  // preconditioner, and so does a Jacobi solve that did not converge when
  // the prior one did.
  const bool jacobi = rj == PPCG_OK ? !(rp == PPCG_OK && ip <= ij) : false;
  S->choice = jacobi ? PPCG_PRECOND_JACOBI : PPCG_PRECOND_PRIOR;
  if (jacobi) {
    const size_t bytes = (size_t)p * (dtype == PPCG_F64 ? sizeof(double) : sizeof(float));
    if (hipMemcpyAsync(beta_out, S->beta_alt, bytes, hipMemcpyDeviceToDevice, stream) !=
        hipSuccess)
      return PPCG_EHIP;
  }
  if (info) *info = local[jacobi ? 1 : 0];
  ++S->draws;
  return jacobi ? rj : rp;
}

}  // extern "C"
