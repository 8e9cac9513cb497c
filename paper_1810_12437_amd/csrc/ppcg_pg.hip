// Polya-Gamma omega update of the Gibbs cycle (Supplement S1, step 3):
// omega_i ~ PG(1, psi_i) with psi = X beta, and the pseudo-response
// z_i = (y_i - 1/2) / omega_i (eq. pg_augmented_likelihood).
//
// PG(1, c) = J*(1, |c|/2) / 4, drawn by Devroye's exact alternating-series
// sampler (as described by Polson, Scott & Windle 2013, Section 4): a proposal
// mixing an exponential on (t, inf) and an inverse Gaussian truncated to
// (0, t], t = 0.64, accepted against the partial sums of the J* density's
// series (both divided by its leading term).  One thread per element;
// element i draws its uniforms from its own Philox4x64-10 stream (counter (i, 2 | (k / 4) << 8, chain, draw), key
// (seed, 0), word k % 4 as ((w >> 11) + 1/2) 2^-53), so every element is a
// pure function of (seed, chain, draw, i, psi_i).  Every loop is capped at 64
// rounds (reached with probability far below 1e-100): each wave exits.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "../../include/ppcg.h"
#include "ppcg_kernels.h"
#include "ppcg_philox.h"

namespace ppcg {
namespace {

constexpr int kBlock = 256;
constexpr int kCap = 64;
constexpr double kT = 0.64;                 // split point of the two series forms
constexpr double kPi = 3.141592653589793;   // pi rounded to double
constexpr double kTwoPi = 6.283185307179586;
constexpr uint64_t kStreamPG = 2;

struct PgUniforms {
  uint64_t seed, chain, draw, i;
  uint32_t k;
  U64x4 w;

  __device__ double operator()() {
    const uint32_t q = k & 3u;
    if (q == 0)
      w = philox4x64_10(U64x4{i, kStreamPG | ((uint64_t)(k >> 2) << 8), chain, draw}, seed, 0ull);
    ++k;
    const uint64_t word = q == 0 ? w.x0 : q == 1 ? w.x1 : q == 2 ? w.x2 : w.x3;
    return ((double)(word >> 11) + 0.5) * 0x1p-53;
  }
};

// Term n of the alternating series of the J*(1, 0) density divided by its
// leading term: (2n + 1) exp(-2 n (n + 1) / x) up to t, (2n + 1)
// exp(-n (n + 1) pi^2 x / 2) beyond.  The acceptance test divided by a_0 > 0
// takes the same decisions and stays defined where a_0 underflows.
__device__ double series_ratio(int n, double x) {
  const double k = (double)(n * (n + 1));
  if (x <= kT) return (2 * n + 1) * exp(-2.0 * k / x);
  return (2 * n + 1) * exp(-k * (kPi * kPi) * x / 2.0);
}

// p / (p + q), the chance of the exponential part of the proposal, from the
// masses' logarithms (both underflow at large z): p = pi/(2K) exp(-K t),
// q = exp(-z) erfc((1 - z t)/sqrt(2t)) + erfcx((1 + z t)/sqrt(2t))
// exp(-z^2 t/2 - 1/(2t)).
__device__ double right_probability(double z, double K) {
  const double lp = log(kPi / (2.0 * K)) - K * kT;
  const double r = sqrt(2.0 * kT);
  const double l1 = -z + log(erfc((1.0 - z * kT) / r));
  const double l2 = log(erfcx((1.0 + z * kT) / r)) - z * z * kT / 2.0 - 1.0 / (2.0 * kT);
  const double hi = l1 >= l2 ? l1 : l2, lo = l1 >= l2 ? l2 : l1;
  const double d = hi + log1p(exp(lo - hi)) - lp;
  return d > 700.0 ? 0.0 : 1.0 / (1.0 + exp(d));
}

// IG(1/z, 1) restricted to (0, t]; z < 1/t (z = 0 included) through the
// truncated Levy law and a tilt acceptance, else by the Michael-Schucany-Haas
// transform repeated until the draw falls below t.
__device__ double truncated_ig(double z, PgUniforms& u) {
  double x = kT;
  if (z < 1.0 / kT) {
    for (int a = 0; a < kCap; ++a) {
      double e1 = 0.0;
      for (int b = 0; b < kCap; ++b) {
        e1 = -log(u());
        const double e2 = -log(u());
        if (e1 * e1 <= 2.0 * e2 / kT) break;
      }
      x = kT / ((1.0 + kT * e1) * (1.0 + kT * e1));
      if (u() <= exp(-z * z * x / 2.0)) break;
    }
    return x;
  }
  const double mu = 1.0 / z;
  for (int a = 0; a < kCap; ++a) {
    const double u1 = u(), u2 = u();
    const double cs = cos(kTwoPi * u2);
    const double y = -2.0 * log(u1) * cs * cs;
    x = mu + 0.5 * mu * mu * y - 0.5 * mu * sqrt(4.0 * mu * y + (mu * y) * (mu * y));
    if (u() > mu / (mu + x)) x = mu * mu / x;
    if (x <= kT) break;
  }
  return x;
}

__device__ double pg1(double c, PgUniforms& u) {
  const double z = 0.5 * fabs(c);
  const double K = kPi * kPi / 8.0 + z * z / 2.0;
  const double right = right_probability(z, K);
  double x = kT;
  for (int a = 0; a < kCap; ++a) {
    if (u() < right)
      x = kT - log(u()) / K;
    else
      x = truncated_ig(z, u);
    double s = 1.0;  // partial sums over a_0(x)
    const double y = u();
    bool accepted = false;
    for (int n = 1; n < kCap; ++n) {
      if (n & 1) {
        s -= series_ratio(n, x);
        if (y < s) {
          accepted = true;
          break;
        }
      } else {
        s += series_ratio(n, x);
        if (y > s) break;
      }
    }
    if (accepted) break;
  }
  return 0.25 * x;
}

// omega_i ~ PG(1, psi_i); with y given, also z_i = (y_i - 1/2) / omega_i.
// Outputs in `dtype` (PPCG_F64 or PPCG_F32).
__global__ __launch_bounds__(kBlock) void k_pg_omega(const double* psi, const uint8_t* y,
                                                     int64_t n, uint64_t seed, uint64_t chain,
                                                     uint64_t draw, int dtype, void* omega_out,
                                                     void* z_out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  PgUniforms u{seed, chain, draw, (uint64_t)i, 0u, U64x4{0, 0, 0, 0}};
  const double w = pg1(psi[i], u);
  const double zi = y ? ((double)y[i] - 0.5) / w : 0.0;
  if (dtype == PPCG_F64) {
    static_cast<double*>(omega_out)[i] = w;
    if (y) static_cast<double*>(z_out)[i] = zi;
  } else {
    static_cast<float*>(omega_out)[i] = (float)w;
    if (y) static_cast<float*>(z_out)[i] = (float)zi;
  }
}

}  // namespace

hipError_t launch_pg_omega(const double* psi, const uint8_t* y, int64_t n, uint64_t seed,
                           uint64_t chain, uint64_t draw, int dtype, void* omega_out, void* z_out,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pg_omega, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     psi, y, n, seed, chain, draw, dtype, omega_out, z_out);
  return hipGetLastError();
}

}  // namespace ppcg

extern "C" int ppcg_pg_sample(const double* c, int64_t n, uint64_t seed, uint64_t chain,
                              uint64_t draw_index, double* omega_out, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!c || !omega_out))) return PPCG_EINVAL;
  return ppcg::launch_pg_omega(c, nullptr, n, seed, chain, draw_index, PPCG_F64, omega_out,
                               nullptr, stream) == hipSuccess
             ? PPCG_OK
             : PPCG_EHIP;
}
