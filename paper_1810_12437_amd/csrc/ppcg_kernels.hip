// HIP kernels (CDNA4 / gfx950) of the prior-preconditioned CG sampler.
//
// Hot path of one CG iteration (Supplement S2 with the prior preconditioner
// of Section 2.4):
//   pass 1 (CSR): u = omega .* (X s)        -- v -> X v, then Omega
//   pass 2 (CSC): q = X^T u                  -- w -> X^T w
//   phase A     : <s, q + d .* s>  ->  alpha
//   phase B     : beta += alpha s, r -= alpha (q + d s), z = M^-1 r, rho'
//   phase C     : s = z + (rho'/rho) s
// X is binary, so both passes are segmented gather-sums over int32 index
// streams with no value array.  The passes split the index stream into
// equal chunks of C = 256 * V elements per workgroup, so column lengths that
// span three orders of magnitude stay load balanced; segments (rows or
// columns) that cross a chunk boundary are finished by the last chunk to
// arrive, summing the chunk partials in chunk order, so every result is
// bitwise reproducible.  Reductions of the p-vector phases are fixed-order
// too.
#include "ppcg_kernels.h"

#include <math.h>

namespace ppcg {

typedef int int4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Fixed-order sum of NV values over the workgroup; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[kWG / 64][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wid][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double a = red[0][i];
      for (int w = 1; w < kWG / 64; ++w) a += red[w][i];
      v[i] = a;
    }
  }
}

// Writes this block's NV partials and reports whether it is the last block
// of the grid to arrive (then the whole grid's partials are visible to it).
// Must be called by every thread of the block after block_sum.
template <int NV>
__device__ __forceinline__ bool publish_and_arrive(double (&v)[NV], double* part,
                                                   uint32_t* ctr) {
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) st_agent(&part[blockIdx.x * NV + i], v[i]);
    __threadfence();
    uint32_t old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (old == gridDim.x - 1);
  }
  __syncthreads();
  return is_last != 0;
}

// In the last block: fixed-order total of every block's partials (valid in
// lane 0 of wave 0).  Resets the arrival counter for the next launch.
template <int NV>
__device__ __forceinline__ void gather_totals(const double* part, uint32_t* ctr,
                                              double (&tot)[NV]) {
  if (threadIdx.x < 64) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double a = 0.0;
      for (int b = threadIdx.x; b < (int)gridDim.x; b += 64) a += ld_agent(&part[b * NV + i]);
      tot[i] = wave_sum(a);
    }
    if (threadIdx.x == 0) st_agent(ctr, 0u);
  }
}

// ------------------------------------------------------------------------
// segmented gather-sum pass: out[sid[g]] = scale[sid[g]] * sum_{e in g} x[idx[e]]
// ------------------------------------------------------------------------
template <typename T, int V>
__global__ __launch_bounds__(kWG) void k_segsum(SegTable t, const T* __restrict__ x,
                                                const T* __restrict__ scale,
                                                T* __restrict__ out,
                                                const int32_t* __restrict__ done) {
  if (done != nullptr && *done) return;
  constexpr int C = kWG * V;
  __shared__ int32_t lptr[C + 2];
  __shared__ int32_t wkey[kWG / 64];
  __shared__ T wval[kWG / 64];

  const int c = blockIdx.x;
  const int64_t cs = t.cstart[c], ce = t.cstart[c + 1];
  const int64_t base = cs & ~(int64_t)3;  // aligned start; [base, cs) is masked
  const int lo = (int)(cs - base);
  const int len = (int)(ce - base);  // <= C
  const int sf = t.cseg[c];
  const int nsg = t.cnseg[c];

  for (int k = threadIdx.x; k <= nsg; k += kWG) lptr[k] = (int32_t)(t.ptr[sf + k] - base);

  // Stream this thread's V indices (non-temporal: read once per pass) and
  // gather x; the gathered vector stays in cache.
  const int e0 = threadIdx.x * V;
  T xv[V];
  if (e0 + V <= len) {
    const int4v* ip = reinterpret_cast<const int4v*>(t.idx + base + e0);
    int32_t ix[V];
#pragma unroll
    for (int q = 0; q < V / 4; ++q) {
      int4v w4 = __builtin_nontemporal_load(ip + q);
      ix[4 * q + 0] = w4.x;
      ix[4 * q + 1] = w4.y;
      ix[4 * q + 2] = w4.z;
      ix[4 * q + 3] = w4.w;
    }
#pragma unroll
    for (int j = 0; j < V; ++j) xv[j] = x[ix[j]];
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) xv[j] = (e0 + j < len) ? x[t.idx[base + e0 + j]] : T(0);
  }
#pragma unroll
  for (int j = 0; j < V; ++j)
    if (e0 + j < lo) xv[j] = T(0);  // elements of the previous chunk

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (nsg == 0) {
    // One piece of a long segment: fixed-order sum over the workgroup.
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < V; ++j) acc += xv[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) wval[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      T tot = wval[0];
      for (int w = 1; w < kWG / 64; ++w) tot += wval[w];
      reinterpret_cast<T*>(t.part)[c] = tot;
    }
    return;
  }
  __syncthreads();

  auto emit = [&](int k, T v) {
    const int o = t.sid[sf + k];
    out[o] = scale ? v * scale[o] : v;
  };

  // Walk this thread's elements; every segment of a packed chunk ends inside
  // the chunk, so each is finished by the thread holding its last element.
  int k = nsg, first_k = nsg;
  T acc = T(0), first_val = T(0);
  bool first_closed = false, closes_at_end = false;
  const int eb = max(e0, lo);
  const int eend = min(e0 + V, len);
  if (eb < eend) {
    int a = 0, b = nsg - 1;
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (lptr[mid] <= eb) a = mid; else b = mid - 1;
    }
    k = first_k = a;
    int nxt = lptr[k + 1];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int e = e0 + j;
      if (e >= eb && e < eend) {
        while (e >= nxt) {  // segment k ended before element e
          if (!first_closed) {
            first_val = acc;
            first_closed = true;
          } else {
            emit(k, acc);  // started and ended inside this thread
          }
          acc = T(0);
          ++k;
          nxt = lptr[k + 1];
        }
        acc += xv[j];
      }
    }
    closes_at_end = (nxt == eend);
  }

  // Segmented inclusive scan of (segment, partial) over the workgroup gives
  // each thread the sum of the earlier threads' share of its first segment.
  int key = k;
  T val = acc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int ku = __shfl_up(key, d, 64);
    const T vu = __shfl_up(val, d, 64);
    if (lane >= d && ku == key) val += vu;
  }
  if (lane == 63) {
    wkey[wid] = key;
    wval[wid] = val;
  }
  __syncthreads();
  int pk = -1;
  T pv = T(0);
  for (int w = 0; w < wid; ++w) {
    pv = wval[w] + (wkey[w] == pk ? pv : T(0));
    pk = wkey[w];
  }
  const T incl = val + (pk == key ? pv : T(0));
  int ek = __shfl_up(key, 1, 64);
  T ev = __shfl_up(incl, 1, 64);
  if (lane == 0) {
    ek = pk;
    ev = pv;
  }
  const T carry_in = (ek == first_k) ? ev : T(0);

  if (eb < eend) {
    if (first_closed) {
      emit(first_k, carry_in + first_val);
      if (closes_at_end) emit(k, acc);
    } else if (closes_at_end) {
      emit(k, carry_in + acc);
    }
  }
}

// Sums the pieces of each split segment in chunk order.
template <typename T>
__global__ __launch_bounds__(kWG) void k_split_sum(SegTable t, const T* __restrict__ scale,
                                                   T* __restrict__ out,
                                                   const int32_t* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i >= t.nsplit) return;
  const T* part = reinterpret_cast<const T*>(t.part);
  const int c0 = t.split_c0[i], c1 = t.split_c1[i];
  T tot = part[c0];
  for (int cc = c0 + 1; cc <= c1; ++cc) tot += part[cc];
  const int o = t.sid[t.split_seg[i]];
  out[o] = scale ? tot * scale[o] : tot;
}

template <typename T>
hipError_t launch_segsum(const SegTable& t, const T* x, const T* scale, T* out,
                         const int32_t* done, hipStream_t st) {
  if (t.nchunks == 0) return hipSuccess;
  const dim3 grid(t.nchunks), block(kWG);
  switch (t.chunk / kWG) {
    case 4:
      hipLaunchKernelGGL((k_segsum<T, 4>), grid, block, 0, st, t, x, scale, out, done);
      break;
    case 8:
      hipLaunchKernelGGL((k_segsum<T, 8>), grid, block, 0, st, t, x, scale, out, done);
      break;
    case 16:
      hipLaunchKernelGGL((k_segsum<T, 16>), grid, block, 0, st, t, x, scale, out, done);
      break;
    default:
      return hipErrorInvalidValue;
  }
  if (t.nsplit > 0)
    hipLaunchKernelGGL((k_split_sum<T>), dim3((t.nsplit + kWG - 1) / kWG), block, 0, st, t,
                       scale, out, done);
  return hipGetLastError();
}

template hipError_t launch_segsum<float>(const SegTable&, const float*, const float*, float*,
                                         const int32_t*, hipStream_t);
template hipError_t launch_segsum<double>(const SegTable&, const double*, const double*,
                                          double*, const int32_t*, hipStream_t);

// ------------------------------------------------------------------------
// Philox4x64-10 and Box-Muller normals
// ------------------------------------------------------------------------
struct U64x4 {
  uint64_t x0, x1, x2, x3;
};

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c.x0), lo0 = M0 * c.x0;
    const uint64_t hi1 = __umul64hi(M1, c.x2), lo1 = M1 * c.x2;
    c = U64x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
  }
  return c;
}

// Four N(0,1) values of counter block i of stream `stream_id`.
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t stream_id, uint64_t chain,
                                         uint64_t draw, uint64_t i, double g[4]) {
  const U64x4 w = philox4x64_10(U64x4{i, stream_id, chain, draw}, seed, 0ull);
  constexpr double kTwoPi = 6.283185307179586;  // 2 * pi rounded to double
  const double ua0 = ((double)(w.x0 >> 12) + 0.5) * 0x1p-52;
  const double ub0 = (double)(w.x1 >> 11) * 0x1p-53;
  const double ua1 = ((double)(w.x2 >> 12) + 0.5) * 0x1p-52;
  const double ub1 = (double)(w.x3 >> 11) * 0x1p-53;
  const double r0 = sqrt(-2.0 * log(ua0)), r1 = sqrt(-2.0 * log(ua1));
  const double a0 = kTwoPi * ub0, a1 = kTwoPi * ub1;
  g[0] = r0 * cos(a0);
  g[1] = r0 * sin(a0);
  g[2] = r1 * cos(a1);
  g[3] = r1 * sin(a1);
}

__global__ __launch_bounds__(kWG) void k_normals(uint64_t seed, uint64_t sid, uint64_t chain,
                                                 uint64_t draw, int64_t count, double* out) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (4 * i >= count) return;
  double g[4];
  normals4(seed, sid, chain, draw, (uint64_t)i, g);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * i + q < count) out[4 * i + q] = g[q];
}

hipError_t launch_normals(uint64_t seed, uint64_t stream_id, uint64_t chain, uint64_t draw,
                          int64_t count, double* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t nb = (count + 3) / 4;
  hipLaunchKernelGGL(k_normals, dim3((unsigned)((nb + kWG - 1) / kWG)), dim3(kWG), 0, st, seed,
                     stream_id, chain, draw, count, out);
  return hipGetLastError();
}

template <typename T>
__device__ __forceinline__ double ldv(const void* p, int64_t i) {
  return (double)reinterpret_cast<const T*>(p)[i];
}
__device__ __forceinline__ double ld_dtype(const void* p, int dtype, int64_t i) {
  return dtype == 0 ? ldv<double>(p, i) : ldv<float>(p, i);
}

// y = omega .* z + sqrt(omega) .* eta  (the n-vector X^T is applied to in Prop 2.1).
__global__ __launch_bounds__(kWG) void k_y_draw(const double* omega64, const void* z, int dtype,
                                                uint64_t seed, uint64_t chain, uint64_t draw,
                                                int64_t n, double* y) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (4 * i >= n) return;
  double g[4];
  normals4(seed, 0ull, chain, draw, (uint64_t)i, g);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = 4 * i + q;
    if (e < n) {
      const double om = omega64[e];
      y[e] = om * ld_dtype(z, dtype, e) + sqrt(om) * g[q];
    }
  }
}

hipError_t launch_y_draw(const double* omega64, const void* z, int dtype, uint64_t seed,
                         uint64_t chain, uint64_t draw, int64_t n, double* y, hipStream_t st) {
  const int64_t nb = (n + 3) / 4;
  hipLaunchKernelGGL(k_y_draw, dim3((unsigned)((nb + kWG - 1) / kWG)), dim3(kWG), 0, st,
                     omega64, z, dtype, seed, chain, draw, n, y);
  return hipGetLastError();
}

// b = X^T y + delta / (tau lambda)
__global__ __launch_bounds__(kWG) void k_rhs_fin(const double* bx, const void* lambda, int dtype,
                                                 double tau, uint64_t seed, uint64_t chain,
                                                 uint64_t draw, int64_t p, double* b) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (4 * i >= p) return;
  double g[4];
  normals4(seed, 1ull, chain, draw, (uint64_t)i, g);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t j = 4 * i + q;
    if (j < p) b[j] = bx[j] + g[q] / (tau * ld_dtype(lambda, dtype, j));
  }
}

hipError_t launch_rhs_fin(const double* bx, const void* lambda, int dtype, double tau,
                          uint64_t seed, uint64_t chain, uint64_t draw, int64_t p, double* b,
                          hipStream_t st) {
  const int64_t nb = (p + 3) / 4;
  hipLaunchKernelGGL(k_rhs_fin, dim3((unsigned)((nb + kWG - 1) / kWG)), dim3(kWG), 0, st, bx,
                     lambda, dtype, tau, seed, chain, draw, p, b);
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// elementwise preparation
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_prep(const void* lambda, const void* omega, int dtype,
                                              double tau, int64_t n, int64_t p, double* d,
                                              double* m, double* omega64) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < p) {
    const double c = tau * ld_dtype(lambda, dtype, i);
    m[i] = c * c;          // M^-1 = (tau lambda)^2
    d[i] = 1.0 / (c * c);  // tau^-2 lambda^-2
  }
  if (omega64 != nullptr && i < n) omega64[i] = ld_dtype(omega, dtype, i);
}

hipError_t launch_prep(const void* lambda, const void* omega, int dtype, double tau, int64_t n,
                       int64_t p, double* d, double* m, double* omega64, hipStream_t st) {
  const int64_t cnt = n > p ? n : p;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)((cnt + kWG - 1) / kWG)), dim3(kWG), 0, st, lambda,
                     omega, dtype, tau, n, p, d, m, omega64);
  return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_to_f64(const void* in, int dtype, int64_t cnt,
                                                double* out) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < cnt) out[i] = ld_dtype(in, dtype, i);
}
__global__ __launch_bounds__(kWG) void k_from_f64(const double* in, int dtype, int64_t cnt,
                                                  void* out) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= cnt) return;
  if (dtype == 0)
    reinterpret_cast<double*>(out)[i] = in[i];
  else
    reinterpret_cast<float*>(out)[i] = (float)in[i];
}

hipError_t launch_convert_to_f64(const void* in, int dtype, int64_t cnt, double* out,
                                 hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((cnt + kWG - 1) / kWG)), dim3(kWG), 0, st, in,
                     dtype, cnt, out);
  return hipGetLastError();
}
hipError_t launch_convert_from_f64(const double* in, int dtype, int64_t cnt, void* out,
                                   hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_from_f64, dim3((unsigned)((cnt + kWG - 1) / kWG)), dim3(kWG), 0, st, in,
                     dtype, cnt, out);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_phi_finish(const T* qx, const double* d, const T* v,
                                                    int64_t p, T* out) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < p) out[i] = (T)((double)qx[i] + d[i] * (double)v[i]);
}

template <typename T>
hipError_t launch_phi_finish(const T* qx, const double* d, const T* v, int64_t p, T* out,
                             hipStream_t st) {
  hipLaunchKernelGGL((k_phi_finish<T>), dim3((unsigned)((p + kWG - 1) / kWG)), dim3(kWG), 0, st,
                     qx, d, v, p, out);
  return hipGetLastError();
}
template hipError_t launch_phi_finish<float>(const float*, const double*, const float*, int64_t,
                                             float*, hipStream_t);
template hipError_t launch_phi_finish<double>(const double*, const double*, const double*,
                                              int64_t, double*, hipStream_t);

// ------------------------------------------------------------------------
// CG vector phases (p-vectors; FP64 state and reductions)
// ------------------------------------------------------------------------
static inline unsigned red_grid(int64_t p) {
  int64_t g = (p + kWG * 4 - 1) / (kWG * 4);
  if (g < 1) g = 1;
  if (g > kMaxRedBlocks) g = kMaxRedBlocks;
  return (unsigned)g;
}

enum { kCritRelPrecond = 0, kCritRmsAbs = 1, kCritRelPlain = 2 };
enum { kStatOK = 0, kStatNotConv = 4, kStatBreakdown = 5 };

template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_start(VecWork w, int mode, const double* b,
                                                  const double* qx64, const double* d,
                                                  const double* m, double* beta, double* r,
                                                  T* s, int64_t p, double tol, int criterion,
                                                  int max_iter) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // <r,Mr>, <r,r>, <b,Mb>, <b,b>
  for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < p;
       j += (int64_t)gridDim.x * kWG) {
    const double bj = b[j];
    const double rj = qx64 ? bj - qx64[j] - d[j] * beta[j] : bj;
    const double zj = m[j] * rj;
    v[0] += rj * zj;
    v[1] += rj * rj;
    if (mode == 0) {
      v[2] += bj * m[j] * bj;
      v[3] += bj * bj;
    }
    if (mode != 2) {
      r[j] = rj;
      s[j] = (T)zj;
      if (mode == 0 && qx64 == nullptr) beta[j] = 0.0;
    }
  }
  block_sum<4>(v);
  if (!publish_and_arrive<4>(v, w.part, &w.sc->arrive[1])) return;
  double tot[4];
  gather_totals<4>(w.part, &w.sc->arrive[1], tot);
  if (threadIdx.x == 0) {
    DevScal* sc = w.sc;
    const int crit = (mode == 0) ? criterion : sc->criterion;
    const double meas = (crit == kCritRelPlain) ? tot[1] : tot[0];
    if (mode == 2) {
      sc->true_rm = tot[0];
      sc->true_meas = meas;
      return;
    }
    if (mode == 0) {
      sc->criterion = criterion;
      sc->max_iter = max_iter;
      sc->bm2 = tot[2];
      sc->bb = tot[3];
      const double t2 = tol * tol;
      sc->thresh2 = criterion == kCritRelPrecond ? t2 * tot[2]
                  : criterion == kCritRmsAbs     ? t2 * (double)p
                                                 : t2 * tot[3];
    }
    sc->rho = tot[0];
    sc->rr = tot[1];
    sc->meas = meas;
    sc->iters = 0;
    sc->status = kStatOK;
    sc->alpha = 0.0;
    sc->betacg = 0.0;
    sc->done = (meas <= sc->thresh2) ? 1 : 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      sc->status = kStatBreakdown;
      sc->done = 1;
    }
  }
}

template <typename T>
hipError_t launch_cg_start(VecWork w, int mode, const double* b, const double* qx64,
                           const double* d, const double* m, double* beta, double* r, T* s,
                           int64_t p, double tol, int criterion, int max_iter, hipStream_t st) {
  hipLaunchKernelGGL((k_cg_start<T>), dim3(red_grid(p)), dim3(kWG), 0, st, w, mode, b, qx64, d,
                     m, beta, r, s, p, tol, criterion, max_iter);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_dot(VecWork w, const T* s, const T* qx,
                                                const double* d, int64_t p) {
  if (w.sc->done) return;
  double v[1] = {0.0};
  for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < p;
       j += (int64_t)gridDim.x * kWG) {
    const double sj = (double)s[j];
    v[0] += sj * ((double)qx[j] + d[j] * sj);
  }
  block_sum<1>(v);
  if (!publish_and_arrive<1>(v, w.part, &w.sc->arrive[2])) return;
  double tot[1];
  gather_totals<1>(w.part, &w.sc->arrive[2], tot);
  if (threadIdx.x == 0) {
    DevScal* sc = w.sc;
    sc->sq = tot[0];
    if (!(tot[0] > 0.0) || !isfinite(tot[0])) {
      sc->status = kStatBreakdown;
      sc->done = 1;
      sc->alpha = 0.0;
    } else {
      sc->alpha = sc->rho / tot[0];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_update(VecWork w, const T* s, const T* qx,
                                                   const double* d, const double* m,
                                                   double* beta, double* r, int64_t p) {
  if (w.sc->done) return;
  const double alpha = w.sc->alpha;
  double v[2] = {0.0, 0.0};  // <r, M^-1 r>, <r, r>
  for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < p;
       j += (int64_t)gridDim.x * kWG) {
    const double sj = (double)s[j];
    const double qj = (double)qx[j] + d[j] * sj;
    beta[j] += alpha * sj;
    const double rj = r[j] - alpha * qj;
    r[j] = rj;
    v[0] += rj * (m[j] * rj);
    v[1] += rj * rj;
  }
  block_sum<2>(v);
  if (!publish_and_arrive<2>(v, w.part, &w.sc->arrive[3])) return;
  double tot[2];
  gather_totals<2>(w.part, &w.sc->arrive[3], tot);
  if (threadIdx.x == 0) {
    DevScal* sc = w.sc;
    const double rho_new = tot[0];
    sc->iters += 1;
    sc->rr = tot[1];
    const double meas = (sc->criterion == kCritRelPlain) ? tot[1] : rho_new;
    sc->meas = meas;
    sc->betacg = rho_new / sc->rho;
    sc->rho = rho_new;
    if (!isfinite(rho_new)) {
      sc->status = kStatBreakdown;
      sc->done = 1;
    } else if (meas <= sc->thresh2) {
      sc->done = 1;
    } else if (sc->iters >= sc->max_iter) {
      sc->status = kStatNotConv;
      sc->done = 1;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_direction(VecWork w, const double* m,
                                                      const double* r, T* s, int64_t p) {
  if (w.sc->done) return;
  const double bc = w.sc->betacg;
  for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < p;
       j += (int64_t)gridDim.x * kWG)
    s[j] = (T)(m[j] * r[j] + bc * (double)s[j]);
}

template <typename T>
hipError_t launch_cg_dot(VecWork w, const T* s, const T* qx, const double* d, int64_t p,
                         hipStream_t st) {
  hipLaunchKernelGGL((k_cg_dot<T>), dim3(red_grid(p)), dim3(kWG), 0, st, w, s, qx, d, p);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_cg_update(VecWork w, const T* s, const T* qx, const double* d,
                            const double* m, double* beta, double* r, int64_t p,
                            hipStream_t st) {
  hipLaunchKernelGGL((k_cg_update<T>), dim3(red_grid(p)), dim3(kWG), 0, st, w, s, qx, d, m, beta,
                     r, p);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_cg_direction(VecWork w, const double* m, const double* r, T* s, int64_t p,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_cg_direction<T>), dim3(red_grid(p)), dim3(kWG), 0, st, w, m, r, s, p);
  return hipGetLastError();
}

#define PPCG_INST(T)                                                                         \
  template hipError_t launch_cg_start<T>(VecWork, int, const double*, const double*,         \
                                         const double*, const double*, double*, double*, T*, \
                                         int64_t, double, int, int, hipStream_t);            \
  template hipError_t launch_cg_dot<T>(VecWork, const T*, const T*, const double*, int64_t,  \
                                       hipStream_t);                                         \
  template hipError_t launch_cg_update<T>(VecWork, const T*, const T*, const double*,        \
                                          const double*, double*, double*, int64_t,          \
                                          hipStream_t);                                      \
  template hipError_t launch_cg_direction<T>(VecWork, const double*, const double*, T*,      \
                                             int64_t, hipStream_t);
PPCG_INST(float)
PPCG_INST(double)
#undef PPCG_INST

// ------------------------------------------------------------------------
// adjoint epilogue
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_adjoint(VecWork w, const double* a, const void* beta,
                                                 int dtype, const double* d, int64_t p,
                                                 void* grad_b, void* grad_ll,
                                                 double* grad_lt) {
  double v[1] = {0.0};
  for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < p;
       j += (int64_t)gridDim.x * kWG) {
    const double aj = a[j];
    const double gl = 2.0 * d[j] * aj * ld_dtype(beta, dtype, j);
    v[0] += gl;
    if (dtype == 0) {
      reinterpret_cast<double*>(grad_b)[j] = aj;
      reinterpret_cast<double*>(grad_ll)[j] = gl;
    } else {
      reinterpret_cast<float*>(grad_b)[j] = (float)aj;
      reinterpret_cast<float*>(grad_ll)[j] = (float)gl;
    }
  }
  block_sum<1>(v);
  if (!publish_and_arrive<1>(v, w.part, &w.sc->arrive[4])) return;
  double tot[1];
  gather_totals<1>(w.part, &w.sc->arrive[4], tot);
  if (threadIdx.x == 0) {
    w.sc->grad_sum = tot[0];
    *grad_lt = tot[0];
  }
}

hipError_t launch_adjoint_epilogue(VecWork w, const double* a, const void* beta, int dtype,
                                   const double* d, int64_t p, void* grad_b,
                                   void* grad_loglambda, double* grad_logtau, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint, dim3(red_grid(p)), dim3(kWG), 0, st, w, a, beta, dtype, d, p,
                     grad_b, grad_loglambda, grad_logtau);
  return hipGetLastError();
}

}  // namespace ppcg
