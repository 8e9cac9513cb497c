// HIP kernels (CDNA4 / gfx950) of the prior-preconditioned CG sampler.
//
// Hot path of one CG iteration (Supplement S2 with the prior preconditioner
// of Section 2.4):
//   row pass    : u = omega .* (X s)        -- v -> X v, then Omega
//   column pass : q = X^T u                  -- w -> X^T w
//   dot phase   : <s, q + d .* s>  ->  alpha
//   update      : beta += alpha s, r -= alpha (q + d s), rho' = <r, M^-1 r>
//   direction   : s = M^-1 r + (rho'/rho) s
// X is binary, so both passes are segmented gather-sums over panel-local
// index streams with no value array (16-byte groups of byte or 16-bit
// differences for one vector, 16-bit indices for K interleaved vectors;
// ppcg_layout.h): a workgroup holds one panel
// of the gathered vector in LDS, each wavefront runs its own list of chunks,
// every lane of a chunk sums groups of one segment across the chunk's
// windows, and one DPP segmented scan per chunk combines the lanes of each
// segment.  Every output has one writer and every sum has a fixed order, so
// results are bitwise reproducible.  Reductions of the p-vector phases are
// fixed-order too.
#include "ppcg_kernels.h"
#include "ppcg_philox.h"

#include <hip/hip_ext.h>

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

// stopping rules and statuses (the values of ppcg.h)
enum { kCritRelPrecond = 0, kCritRmsAbs = 1, kCritRelPlain = 2 };
enum { kStatOK = 0, kStatNotConv = 4, kStatBreakdown = 5 };

// wave_sum's total in every lane.
__device__ __forceinline__ double wave_total(double v) { return __shfl(wave_sum(v), 0, 64); }

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

// Block bid of a (possibly virtual) grid of nblk blocks: a batched launch runs
// the grids of several chains side by side.
struct VGrid {
  int bid, nblk;
};
__device__ __forceinline__ VGrid own_grid() { return VGrid{(int)blockIdx.x, (int)gridDim.x}; }

// Writes this block's NV partials and reports whether it is the last block
// of the grid to arrive (then the whole grid's partials are visible to it).
// Must be called by every thread of the block after block_sum.
template <int NV>
__device__ __forceinline__ bool publish_and_arrive(double (&v)[NV], double* part,
                                                   uint32_t* ctr, VGrid g) {
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) st_agent(&part[g.bid * NV + i], v[i]);
    __threadfence();
    uint32_t old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (old == (uint32_t)g.nblk - 1u);
  }
  __syncthreads();
  return is_last != 0;
}

// In the last block: fixed-order total of every block's partials (valid in
// lane 0 of wave 0).  Resets the arrival counter for the next launch.
template <int NV>
__device__ __forceinline__ void gather_totals(const double* part, uint32_t* ctr,
                                              double (&tot)[NV], VGrid g) {
  if (threadIdx.x < 64) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double a = 0.0;
      for (int b = threadIdx.x; b < g.nblk; b += 64) a += ld_agent(&part[b * NV + i]);
      tot[i] = wave_sum(a);
    }
    if (threadIdx.x == 0) st_agent(ctr, 0u);
  }
}

// ------------------------------------------------------------------------
// X pass: panel-resident gathers, one wavefront per chunk
// ------------------------------------------------------------------------
// value(i) of vector r of an interleaved set (r = 0 for one vector).
template <typename T>
__device__ __forceinline__ T combine_at(const Combine<T>& c, int64_t i, int r = 0) {
  const int64_t e = i * c.es + r;
  // Issue up to eight partial loads before adding them (fixed order).
  T pv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) pv[k] = (k < c.nparts) ? c.part[(int64_t)k * c.stride + e] : T(0);
  T v = pv[0];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (k < c.nparts) v += pv[k];
  for (int k = 8; k < c.nparts; ++k) v += c.part[(int64_t)k * c.stride + e];
  if (c.sp_off != nullptr) {
    const int q1 = c.sp_off[i + 1];
    for (int q = c.sp_off[i]; q < q1; ++q) {
      const int c1 = c.sp_c1[q];
      for (int cc = c.sp_c0[q]; cc <= c1; ++cc) v += c.piece[(int64_t)cc * c.es + r];
    }
  }
  return c.scale ? v * c.scale[e] : v;
}

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

typedef __attribute__((address_space(3))) unsigned char lds_u8;
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(size_t)(const lds_u8*)p;
}
template <typename T>
__device__ __forceinline__ T lds_load(uint32_t addr) {
  return *(const __attribute__((address_space(3))) T*)(size_t)addr;
}

__device__ __forceinline__ int ck_windows(int32_t info) { return info & 0xff; }
__device__ __forceinline__ int ck_kind(int32_t info) { return (info >> 8) & 3; }

// Number of set bits of m below this lane.
__device__ __forceinline__ int bits_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// DPP move of x from another lane (0 where the source is outside the row or
// the row is not selected by RM).
template <int CTRL, int RM>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, RM, 0xf, true));
}
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, RM, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, RM, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
constexpr int kDppRowShr = 0x110;   // row_shr:n = 0x110 + n (within 16-lane rows)
constexpr int kDppBcast15 = 0x142;  // lane 15 of each row to the next row
constexpr int kDppBcast31 = 0x143;  // lane 31 to rows 2 and 3

// Chunk descriptors are read-only for the whole pass: read them through the
// constant address space, so that the uniform reads are scalar loads even
// after the pass has written outputs.
__device__ __forceinline__ ChunkDesc read_desc(const ChunkDesc* p, int c) {
  typedef const __attribute__((address_space(4))) ChunkDesc ConstDesc;
  ConstDesc* q = (ConstDesc*)p + c;
  ChunkDesc D;
  D.base = q->base;
#pragma unroll
  for (int s = 0; s < kPR; ++s) D.vm[s] = q->vm[s];
  D.sm = q->sm;
  D.first = q->first;
  D.info = q->info;
  D.seg = q->seg;
  return D;
}

// A pointer that may have been read from memory (a batched job) is generic
// to the compiler; these views address global memory explicitly, so that
// its loads are global (vector memory only) or, for read-only workgroup-
// uniform tables, scalar.
template <typename V>
__device__ __forceinline__ const __attribute__((address_space(1))) V* gview(const V* p) {
  return (const __attribute__((address_space(1))) V*)p;
}
template <typename V>
__device__ __forceinline__ __attribute__((address_space(1))) V* gview_mut(V* p) {
  return (__attribute__((address_space(1))) V*)p;
}
__device__ __forceinline__ int32_t read_table(const int32_t* p, int64_t i) {
  typedef const __attribute__((address_space(4))) int32_t ConstI32;
  return ((ConstI32*)p)[i];
}

// Load cursor of a wavefront's index stream: window k of chunk c.  Every
// step issues the same three loads (the window's two halves and the output
// slot of its chunk for this lane), with in-bounds stand-ins for lanes that
// have no group in the window and for steps past the wavefront's last
// window, so that the wait before a window's sums covers its own loads only.
struct StreamLoad {
  int32_t c, k, pre, windows, kind;
  int32_t sidx;        // this lane's seg_out entry for chunk c (no_slot: none)
  int64_t base, clen, last_base;
  uint64_t vm0, vm1, vm2, vm3;
};

__device__ __forceinline__ void stream_open(const PanelPass& t, const ChunkDesc& D, int c,
                                            int lane, StreamLoad& L) {
  L.c = c;
  L.k = 0;
  L.pre = 0;
  L.windows = ck_windows(D.info);
  L.kind = ck_kind(D.info);
  L.base = D.base;
  L.last_base = D.base;
  L.clen = (int64_t)D.vm[0];
  L.vm0 = D.vm[0];
  L.vm1 = D.vm[1];
  L.vm2 = D.vm[2];
  L.vm3 = D.vm[3];
  if (L.kind == kChunkLong) {
    L.sidx = D.first;
  } else if (L.kind == kChunkPiece) {
    L.sidx = t.no_slot;
  } else {
    // packed: the last lane of each segment's slice writes that segment
    const uint64_t sm = D.sm;
    const bool last = lane == 63 || ((sm >> (lane + 1)) & 1ull);
    const int si = bits_below(sm) + (int)((sm >> lane) & 1ull) - 1;
    L.sidx = (last && si < (D.info >> 24)) ? D.first + si : t.no_slot;
  }
}

// Issues the loads of the cursor's window into one ring slot and advances.
// Bit `bit` of `have` tells whether this lane has a group in that window.
// CMP: compact groups (ppcg_layout.h), one 16-byte load per lane (b unused);
// otherwise a group's two halves.
template <bool CMP>
__device__ __forceinline__ void stream_issue(const PanelPass& t, int c_end, int lane,
                                             StreamLoad& L, u16x8& a, u16x8& b, int32_t& slot,
                                             uint32_t& have, int bit) {
  constexpr int H = kPV / 2;
  constexpr int GW = CMP ? H : kPV;  // words per group in the stream
  int64_t ea = L.last_base, eb = L.last_base;
  int32_t si = t.no_slot;
  bool h = false, first = false;
  if (L.c < c_end) {
    // window start w0, its ng groups, this lane's rank r among them
    int64_t w0;
    int ng, r;
    if (L.kind == kChunkPacked) {
      const uint64_t m = L.k == 0 ? L.vm0 : L.k == 1 ? L.vm1 : L.k == 2 ? L.vm2 : L.vm3;
      h = ((m >> lane) & 1ull) != 0;
      w0 = L.base + (int64_t)L.pre * GW;
      ng = __popcll(m);
      r = bits_below(m);
      L.pre += ng;
    } else {
      w0 = L.base + (int64_t)L.k * 64 * GW;
      const int64_t left = (L.clen - (int64_t)L.k * kPC) / kPV;
      ng = left < 64 ? (int)left : 64;
      r = lane;
      h = lane < ng;
    }
    ea = h ? w0 + (int64_t)r * H : w0;
    eb = (h && !CMP) ? w0 + (int64_t)(ng + r) * H : w0;
    si = L.sidx;
    first = L.k == 0;
    if (++L.k == L.windows && ++L.c < c_end) stream_open(t, read_desc(t.chunks, L.c), L.c, lane, L);
  }
  a = __builtin_nontemporal_load(gview(reinterpret_cast<const u16x8*>(t.idx + ea)));
  if constexpr (!CMP) b = __builtin_nontemporal_load(gview(reinterpret_cast<const u16x8*>(t.idx + eb)));
  (void)eb;
  // the chunk's output slot rides with its first window only
  if (first) slot = gview(t.seg_out)[si];
  have = (have & ~(1u << bit)) | ((h ? 1u : 0u) << bit);
}

// K values of one panel entry (the K vectors of an interleaved set).
template <typename T, int K>
struct alignas(sizeof(T) * K) PanelEntry {
  T v[K];
};

// Adds this lane's group of kPV elements to acc (per vector, K > 1
// interleaved vectors), in element order.
template <typename T, int K>
__device__ __forceinline__ void gather_add16(const T* xl, const u16x8& a, const u16x8& b,
                                             T (&acc)[K]) {
  static_assert(K > 1, "one vector reads compact groups (gather_cmp, gather_wide)");
  const PanelEntry<T, K>* xp = reinterpret_cast<const PanelEntry<T, K>*>(xl);
  T s[K];
  {
    const PanelEntry<T, K> u = xp[a[0]];
#pragma unroll
    for (int r = 0; r < K; ++r) s[r] = u.v[r];
  }
#pragma unroll
  for (int j = 1; j < kPV; ++j) {
    const PanelEntry<T, K> u = xp[j < 8 ? a[j] : b[j - 8]];
#pragma unroll
    for (int r = 0; r < K; ++r) s[r] += u.v[r];
  }
#pragma unroll
  for (int r = 0; r < K; ++r) acc[r] += s[r];
}

// Adds this lane's compact group (ppcg_layout.h) to acc: its first index
// and the running sums of its byte differences give its kCGroup panel-local
// indices, their gathers are all in flight before a pairwise sum, and the c
// pads (copies of the last entry) are taken off again with one fused
// multiply-add.
template <typename T>
__device__ __forceinline__ void gather_cmp(const T* xl, const u16x8& a, T& acc) {
  const u32x4 d = __builtin_bit_cast(u32x4, a);
  uint32_t e[kCGroup];
  e[0] = d[0] & 0xffffu;
  const uint32_t pads = (d[0] >> 16) & 0xffu;
  e[1] = e[0] + (d[0] >> 24);
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    e[4 * w - 2] = e[4 * w - 3] + (d[w] & 0xffu);
    e[4 * w - 1] = e[4 * w - 2] + ((d[w] >> 8) & 0xffu);
    e[4 * w] = e[4 * w - 1] + ((d[w] >> 16) & 0xffu);
    e[4 * w + 1] = e[4 * w] + (d[w] >> 24);
  }
  const uint32_t l0 = __builtin_amdgcn_readfirstlane(lds_addr(xl));
  T v[16];
#pragma unroll
  for (int k = 0; k < kCGroup; ++k) v[k] = lds_load<T>(e[k] * (uint32_t)sizeof(T) + l0);
  const T last = v[kCGroup - 1];
#pragma unroll
  for (int w = 1; w < 8; w *= 2)
#pragma unroll
    for (int j = 0; j + w < kCGroup; j += 2 * w) v[j] += v[j + w];
  // v[0]: entries 0..7, v[8]: entries 8..13
  if constexpr (sizeof(T) == 8)
    acc += __builtin_fma(-(double)pads, last, v[0] + v[8]);
  else
    acc += __builtin_fmaf(-(float)pads, last, v[0] + v[8]);
}

// The same for a wide group (ppcg_layout.h): its first index and the
// running sums of six 16-bit differences give kWGroup indices.
template <typename T>
__device__ __forceinline__ void gather_wide(const T* xl, const u16x8& a, T& acc) {
  const u32x4 d = __builtin_bit_cast(u32x4, a);
  uint32_t e[kWGroup];
  e[0] = d[0] & 0xffffu;
  const uint32_t pads = (d[0] >> 16) & 0xffu;
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    e[2 * w - 1] = e[2 * w - 2] + (d[w] & 0xffffu);
    e[2 * w] = e[2 * w - 1] + (d[w] >> 16);
  }
  const uint32_t l0 = __builtin_amdgcn_readfirstlane(lds_addr(xl));
  T v[kWGroup];
#pragma unroll
  for (int k = 0; k < kWGroup; ++k) v[k] = lds_load<T>(e[k] * (uint32_t)sizeof(T) + l0);
  const T last = v[kWGroup - 1];
  const T s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + v[6]);
  if constexpr (sizeof(T) == 8)
    acc += __builtin_fma(-(double)pads, last, s);
  else
    acc += __builtin_fmaf(-(float)pads, last, s);
}

// acc[r] += (cond ? DPP move of acc[r] : 0) for every vector.
template <int CTRL, int RM, typename T, int K>
__device__ __forceinline__ void dpp_add(T (&acc)[K], bool cond) {
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const T v = dpp_move<CTRL, RM>(acc[r]);
    if (cond) acc[r] += v;
  }
}

// Sum of each slice of chunk D at the slice's last lane (packed), or of the
// whole wavefront at lane 63 (long), then the write (K values per slot).
// Fixed order.
// With `dotting`, every written sum also adds s_j * sum to p2acc (sd: s_j of
// the lane's output column, per vector).
template <typename T, int K, bool dotting>
__device__ __forceinline__ void finish_chunk(int32_t info, uint64_t sm, T (&acc)[K],
                                             int32_t slot, const T (&scl)[K], int32_t piece,
                                             int lane, T* __restrict__ part_out,
                                             T* __restrict__ piece_out,
                                             const T* __restrict__ out_scale,
                                             const T (&sd)[K], double (&p2acc)[K]) {
  const int kind = ck_kind(info);
  if (kind == kChunkPacked) {
    // Segmented inclusive scan over the slices: row-local shifts, then the
    // row-to-row broadcasts, each taken only from lanes of the same slice.
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int off = lane - (63 - __clzll(sm & upto));
    const int nrow = (info >> 12) & 7;
    if (nrow > 0) dpp_add<kDppRowShr + 1, 0xf>(acc, off >= 1);
    if (nrow > 1) dpp_add<kDppRowShr + 2, 0xf>(acc, off >= 2);
    if (nrow > 2) dpp_add<kDppRowShr + 4, 0xf>(acc, off >= 4);
    if (nrow > 3) dpp_add<kDppRowShr + 8, 0xf>(acc, off >= 8);
    if ((info >> 16) & 1) dpp_add<kDppBcast15, 0xa>(acc, off > (lane & 15));
    if ((info >> 17) & 1) dpp_add<kDppBcast31, 0xc>(acc, off >= lane - 31);
    if (slot >= 0) {
#pragma unroll
      for (int r = 0; r < K; ++r) {
        gview_mut(part_out)[(int64_t)slot * K + r] = out_scale ? acc[r] * scl[r] : acc[r];
        if constexpr (dotting) p2acc[r] += (double)sd[r] * (double)acc[r];
      }
    }
    return;
  }
  dpp_add<kDppRowShr + 1, 0xf>(acc, true);
  dpp_add<kDppRowShr + 2, 0xf>(acc, true);
  dpp_add<kDppRowShr + 4, 0xf>(acc, true);
  dpp_add<kDppRowShr + 8, 0xf>(acc, true);
  dpp_add<kDppBcast15, 0xa>(acc, true);
  dpp_add<kDppBcast31, 0xc>(acc, true);
  if (lane == 63) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
      if (kind == kChunkLong)
        gview_mut(part_out)[(int64_t)slot * K + r] = out_scale ? acc[r] * scl[r] : acc[r];
      else
        gview_mut(piece_out)[(int64_t)piece * K + r] = acc[r];
      if constexpr (dotting) p2acc[r] += (double)sd[r] * (double)acc[r];
    }
  }
}

// ---- panel assembly, FP64 single-vector fast paths ----
template <typename T, int K>
constexpr bool kFastPanel = sizeof(T) == 8 && K == 1;
// the direction panel's fast path: one vector, FP64 or FP32 values
template <typename T, int K>
constexpr bool kFastDir = K == 1;
constexpr int kAsmPairs = 10;  // 16-byte loads per thread: kPThreads * 2 * 10 >= W

__device__ __forceinline__ bool aligned16(const void* p) {
  return ((uintptr_t)p & 15u) == 0;
}
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Pair2;
template <> struct Pair2<double> { typedef f64x2 type; };
template <> struct Pair2<float> { typedef f32x2 type; };

// Pair u of thread tid of a panel assembly: pair tid + b kPThreads of block
// b = (u + w) mod nb (nb blocks of kPThreads pairs), so that the workgroups
// of one XCD start on different blocks; -1 past the end.
__device__ __forceinline__ int asm_pair(int u, int tid, int rb, int nb, int npairs) {
  int b = u + rb;
  b = b >= nb ? b - nb : b;
  const int pl = tid + b * kPThreads;
  return (u < nb && pl < npairs) ? pl : -1;
}

// The loads of the direction panel (z in FP64, the old direction in the
// pass's type), held in registers so that they are in flight while the pass
// finishes the previous step (the ratio bc is not needed until the stores).
// False when the panel is not aligned for pair loads, is shorter than two
// entries or holds more pairs than kAsmPairs per thread (FP32 panels beyond
// 20,480 entries); the same loads are issued then too, all from the first
// 16 bytes of `safe` (16 readable bytes on a 16-byte boundary), so that no
// branch joins paths with different numbers of loads in flight: the waits
// for the loads issued before these (the step's partials) then count them
// exactly, instead of waiting for the whole panel.
template <typename T>
struct DirFast {
  f64x2 zv[kAsmPairs];
  typename Pair2<T>::type sv[kAsmPairs];
  int pi[kAsmPairs];
  double zt;
  T st;
};
template <typename T>
__device__ __forceinline__ bool dir_fast_load(DirFast<T>& L, const double* zp, const T* sp,
                                              int wlen, int w, const void* safe) {
  const int npairs = wlen >> 1;
  const int nbp = (npairs + kPThreads - 1) / kPThreads;
  const bool ok = npairs >= 1 && aligned16(zp) && ((uintptr_t)sp & (2 * sizeof(T) - 1)) == 0 &&
                  nbp <= kAsmPairs;
  const int nb = ok ? nbp : 1;
  const double* zb = ok ? zp : reinterpret_cast<const double*>(safe);
  const T* sb = ok ? sp : reinterpret_cast<const T*>(safe);
  const int rb = w % nb;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kAsmPairs; ++u) {
    L.pi[u] = ok ? asm_pair(u, tid, rb, nb, npairs) : -1;
    const int at = L.pi[u] >= 0 ? 2 * L.pi[u] : 0;
    L.zv[u] = *gview(reinterpret_cast<const f64x2*>(zb + at));
    L.sv[u] = *gview(reinterpret_cast<const typename Pair2<T>::type*>(sb + at));
  }
  // The odd entry, when wlen is odd (thread 0 stores it): a per-lane address
  // (entry 0 elsewhere), so that these are vector loads in flight with the
  // pairs rather than scalar loads waited for at once.
  const int last = (ok && tid == 0) ? wlen - 1 : 0;
  L.zt = gview(zb)[last];
  L.st = gview(sb)[last];
  return ok;
}

// s = z + bc s_old from the loaded pairs into the panel: the first half's
// entries go to LDS, the ring is primed, then the second half; an odd last
// entry is stored by thread 0.  (The workgroup's own entries go to s_new
// after the pass, from LDS.)
template <typename T, typename PRIME>
__device__ __forceinline__ void dir_fast_store(const DirFast<T>& L, double bc, int wlen, T* xl,
                                               PRIME& prime) {
  const int tid = threadIdx.x;
  const int last = wlen - 1;
  auto form = [&](double z, T so) { return (T)(bc == 0.0 ? z : z + bc * (double)so); };
#pragma unroll
  for (int u = 0; u < kAsmPairs / 2; ++u) {
    if (L.pi[u] >= 0) {
      xl[2 * L.pi[u]] = form(L.zv[u].x, L.sv[u].x);
      xl[2 * L.pi[u] + 1] = form(L.zv[u].y, L.sv[u].y);
    }
  }
  prime();
#pragma unroll
  for (int u = kAsmPairs / 2; u < kAsmPairs; ++u) {
    if (L.pi[u] >= 0) {
      xl[2 * L.pi[u]] = form(L.zv[u].x, L.sv[u].x);
      xl[2 * L.pi[u] + 1] = form(L.zv[u].y, L.sv[u].y);
    }
  }
  if ((wlen & 1) && tid == 0) xl[last] = form(L.zt, L.st);
}

// Panel copied from src (FP64, one vector), the same way.
template <typename PRIME>
__device__ __forceinline__ bool assemble_copy_fast(const double* src, int wlen, int w, double* xl,
                                                   PRIME& prime) {
  const int npairs = wlen >> 1;
  if (npairs < 1 || !aligned16(src)) return false;
  const int nb = (npairs + kPThreads - 1) / kPThreads;
  const int rb = w % nb;
  const int tid = threadIdx.x;
  f64x2 v[kAsmPairs];
  int pi[kAsmPairs];
#pragma unroll
  for (int u = 0; u < kAsmPairs; ++u) {
    pi[u] = asm_pair(u, tid, rb, nb, npairs);
    v[u] = *gview(reinterpret_cast<const f64x2*>(src + (pi[u] >= 0 ? 2 * pi[u] : 0)));
  }
  const int last = wlen - 1;
  const double vt = gview(src)[last];
  prime();
#pragma unroll
  for (int u = 0; u < kAsmPairs; ++u)
    if (pi[u] >= 0) *reinterpret_cast<f64x2*>(xl + 2 * pi[u]) = v[u];
  if ((wlen & 1) && tid == 0) xl[last] = vt;
  return true;
}

// Workgroup w of one X pass over K interleaved vectors (K = 1: one vector).
// The pass is skipped when all K flags done[i * dstride] are set.  With
// dir.z set the gathered panel is the new CG direction (DirIn); with dot.s
// set the workgroup also sums its outputs against s (DotOut).
template <typename T, int K, int MODE>
__device__ __forceinline__ void panel_body(const PanelPass& t, const Combine<T>& xin,
                                           T* __restrict__ part_out, T* __restrict__ piece_out,
                                           const T* __restrict__ out_scale,
                                           const int32_t* __restrict__ done,
                                           int dstride, const DirIn<T>& dir,
                                           const DotOut<T>& dot, int parity, int w) {
  constexpr bool dotting = MODE == kPassDot;
  extern __shared__ __align__(16) unsigned char smem[];
  T* xl = reinterpret_cast<T*>(smem);

  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  // What the start needs, requested together: this wavefront's chunk range,
  // the panel, the stop flag(s) and the direction's ratio; then the loads
  // that depend on them.  The stop flags are tested only once every load of
  // the start is in flight (each of them is in bounds either way), so that
  // no load of a launch that runs waits behind the test.
  int c = read_table(t.wave_c, kPWaves * w + wave);
  const int c_end = read_table(t.wave_c, kPWaves * w + wave + 1);
  const int panel = read_table(t.wg_panel, w);
  // (loads without branches, so that none is waited for before the
  // descriptor's; no flags: the table stands in, read at offset 0)
  const int32_t* fp = done != nullptr ? done : t.wave_c;
  const int64_t fs = done != nullptr ? dstride : 0;
  int32_t flag[K];
#pragma unroll
  for (int i = 0; i < K; ++i) flag[i] = gview(fp)[(int64_t)i * fs];
  // direction ratio per vector (a vector whose chain has stopped keeps s = z:
  // its sums are unused), formed once the flags are tested
  int32_t sdone[K];
  double sbc[K], bc[K];
  if constexpr (MODE == kPassDir) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const auto& S = gview(dir.sc)[(int64_t)r * dir.scstride];
      sdone[r] = S.done;
      sbc[r] = S.betacg;
    }
  }
  // The previous step's partials (pass-side finish), requested now and
  // summed after the panel's loads are issued: up to kFinRegs pairs per lane
  // in registers (clamped in-bounds reads, zeros past the end), more by a
  // loop.  Either way each lane adds its pairs in index order.
  constexpr int kFinRegs = 4;
  double fa[kFinRegs], fb[kFinRegs];
  double fin_a = 0.0, fin_b = 0.0;
  bool fin_regs = false;
  if constexpr (MODE == kPassDir) {
    if (K == 1 && dir.sp != nullptr && dir.it > 0) {
      const auto* P = gview(dir.sp + (int64_t)(1 - parity) * 2 * kMaxRedBlocks);
      if (dir.nsb <= 64 * kFinRegs) {
        fin_regs = true;
#pragma unroll
        for (int i = 0; i < kFinRegs; ++i) {
          const int q = lane + 64 * i;
          const int qc = q < dir.nsb ? q : dir.nsb - 1;
          fa[i] = P[2 * qc];  // (the stand-ins past the end are dropped in the sum)
          fb[i] = P[2 * qc + 1];
        }
      } else {
        for (int q = lane; q < dir.nsb; q += 64) {
          fin_a += P[2 * q];
          fin_b += P[2 * q + 1];
        }
      }
    }
  }
  const int64_t g0 = (int64_t)panel * t.W;
  const int64_t rem = t.gdim - g0;
  const int wlen = (int)(rem < t.W ? rem : t.W);
  DirFast<T> dfl;
  bool dfl_ok = false;
  if constexpr (MODE == kPassDir && kFastDir<T, K>) {
    const T* s_old = dir.s + (int64_t)parity * dir.sstride;
    dfl_ok = dir_fast_load(dfl, dir.z + g0, s_old + g0, wlen, w, t.idx);
  }
  ChunkDesc D0{};
  if (c < c_end) D0 = read_desc(t.chunks, c);
  if (done != nullptr) {
    bool all = true;
#pragma unroll
    for (int i = 0; i < K; ++i) all = all && flag[i] != 0;
    if (all) return;
  }
  if constexpr (MODE == kPassDir) {
#pragma unroll
    for (int r = 0; r < K; ++r) bc[r] = sdone[r] ? 0.0 : sbc[r];
  }
  if (fin_regs) {
#pragma unroll
    for (int i = 0; i < kFinRegs; ++i) {
      const bool in = lane + 64 * i < dir.nsb;
      fin_a += in ? fa[i] : 0.0;
      fin_b += in ? fb[i] : 0.0;
    }
  }
  if constexpr (MODE == kPassDir && K == 1) {
    if (dir.sp != nullptr) {
      if (dir.it == 0) {
        bc[0] = 0.0;  // the start kernel's scalars: s = z
      } else {
        // totals in the order of the step kernel's own reduction
        const double rho_new = wave_total(fin_a), rr = wave_total(fin_b);
        auto* sc = gview_mut(dir.sc);
        const double rho_old = sc->rho_par[1 - parity];
        bc[0] = rho_new / rho_old;
        const double meas = sc->criterion == kCritRelPlain ? rr : rho_new;
        int stop = 0, status = kStatOK;
        if (!isfinite(rho_new)) {
          stop = 1;
          status = kStatBreakdown;
        } else if (meas <= sc->loop2) {
          stop = 1;
        } else if (dir.it >= sc->max_iter) {
          stop = 1;
          status = kStatNotConv;
        }
        if (w == 0 && threadIdx.x == 0) {
          sc->iters = dir.it;
          sc->rr = rr;
          sc->meas = meas;
          sc->betacg = bc[0];
          sc->rho_prev = rho_old;
          sc->rho = rho_new;
          sc->rho_par[parity] = rho_new;
          if (stop) {
            sc->status = status;
            sc->done = 1;
          }
        }
        if (stop) return;
      }
    }
  }
  const double bc0 = bc[0];

  // The wavefront's chunks as one stream of windows with kRing in flight:
  // ring slot q % kRing holds window q.  The first kRing are requested while
  // the panel is assembled, after the panel's own loads (the waits count in
  // issue order), always kRing of them (stand-ins when the wavefront has no
  // chunk: the index stream has at least kPV entries).
  StreamLoad ld{};
  u16x8 ra[kRing], rb[kRing];
  int32_t rs[kRing];
  uint32_t rh = 0;
  auto prime = [&]() {
    if (c < c_end) {
      stream_open(t, D0, c, lane, ld);
    } else {
      ld.c = c_end;
      ld.last_base = 0;
    }
#pragma unroll
    for (int q = 0; q < kRing; ++q)
      stream_issue<K == 1>(t, c_end, lane, ld, ra[q], rb[q], rs[q], rh, q);
  };

  // The panel of the gathered vector(s), assembled once per workgroup; entry
  // W holds the zeros the padding indices point to.  Eight loads in flight
  // per thread before the LDS stores.  Every workgroup reads the same
  // entries: each starts at its own offset, so that at any moment the
  // workgroups of one XCD touch different lines and later reads hit in L2.
  const int64_t span = (int64_t)wlen * K;
  const int rot = span > 0 ? (int)(((int64_t)w * 7919) % span) : 0;
  constexpr int U = 8;
  double p1acc[K], p2acc[K];
#pragma unroll
  for (int r = 0; r < K; ++r) p1acc[r] = p2acc[r] = 0.0;
  const T* sdot = dotting ? dot.s + (int64_t)(1 - parity) * dot.sstride : nullptr;
  const int64_t pofs = (int64_t)panel * t.out_dim;
  bool assembled = false;
  if constexpr (MODE == kPassDir && kFastDir<T, K>) {
    // one vector: every thread's pair loads issued at once, then the ring's
    // first windows, then the LDS stores
    if (dfl_ok) {
      dir_fast_store(dfl, bc0, wlen, xl, prime);
      assembled = true;
    }
  } else if constexpr (MODE != kPassDir && kFastPanel<T, K>) {
    // FP64, one vector: the same for a copied panel
    if (xin.nparts == 1 && xin.scale == nullptr && xin.sp_off == nullptr && xin.es == 1)
      assembled = assemble_copy_fast(xin.part + g0, wlen, w, xl, prime);
  }
  if (assembled) {
    // panel done (the ring is primed)
  } else if constexpr (MODE == kPassDir) {
    prime();
    // s = z + bc s_old per vector (s = z right after a start: bc = 0), into
    // the panel; the workgroup's own entries also go to s_new and <s, d s>.
    const T* s_old = dir.s + (int64_t)parity * dir.sstride;
    T* s_new = dir.s + (int64_t)(1 - parity) * dir.sstride;
    const int64_t o0 = t.wg_s0[w], o1 = t.wg_s1[w];
    constexpr int UE = K >= 4 ? 1 : 8 / K;
    const int rotj = rot / K;
    for (int j0 = threadIdx.x; j0 < wlen; j0 += kPThreads * UE) {
      T v[UE][K];
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const int jl = j0 + u * kPThreads;
        const int j = jl + rotj < wlen ? jl + rotj : jl + rotj - wlen;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          v[u][r] = T(0);
          if (jl < wlen) {
            const int64_t e = (g0 + j) * K + r;
            v[u][r] = bc[r] == 0.0 ? (T)dir.z[e] : (T)(dir.z[e] + bc[r] * (double)s_old[e]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const int jl = j0 + u * kPThreads;
        const int j = jl + rotj < wlen ? jl + rotj : jl + rotj - wlen;
        if (jl < wlen) {
          const bool own = g0 + j >= o0 && g0 + j < o1;
#pragma unroll
          for (int r = 0; r < K; ++r) {
            const int64_t e = (g0 + j) * K + r;
            xl[(int64_t)j * K + r] = v[u][r];
            if (own) {
              s_new[e] = v[u][r];
              p1acc[r] += dir.d[e] * (double)v[u][r] * (double)v[u][r];
            }
          }
        }
      }
    }
  } else if (xin.nparts == 1 && xin.scale == nullptr && xin.sp_off == nullptr && xin.es == K) {
    prime();
    const T* src = xin.part + g0 * K;
    const int cnt = wlen * K;
    for (int j0 = threadIdx.x; j0 < cnt; j0 += kPThreads * U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jl = j0 + u * kPThreads;
        const int j = jl + rot < cnt ? jl + rot : jl + rot - cnt;
        v[u] = (jl < cnt) ? src[j] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jl = j0 + u * kPThreads;
        const int j = jl + rot < cnt ? jl + rot : jl + rot - cnt;
        if (jl < cnt) xl[j] = v[u];
      }
    }
  } else {
    prime();
    constexpr int UC = 2;  // (each value already has up to eight partial loads in flight)
    const int cnt = wlen * K;
    for (int j0 = threadIdx.x; j0 < cnt; j0 += kPThreads * UC) {
      T v[UC];
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int jl = j0 + u * kPThreads;
        const int j = jl + rot < cnt ? jl + rot : jl + rot - cnt;
        v[u] = (jl < cnt) ? combine_at(xin, g0 + j / K, j % K) : T(0);
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int jl = j0 + u * kPThreads;
        const int j = jl + rot < cnt ? jl + rot : jl + rot - cnt;
        if (jl < cnt) xl[j] = v[u];
      }
    }
  }
  if (threadIdx.x < K) xl[(int64_t)t.W * K + threadIdx.x] = T(0);
  __syncthreads();

  // Compute cursor: window k of chunk c, in ring slot q; each step sums its
  // window, refills the slot with the window kRing ahead and, after a chunk's
  // last window, writes the chunk's sums.
  int32_t cinfo = 0, cfirst = 0, slot = -1;
  int64_t cseg = -1;
  uint64_t csm = 0;
  int k = 0;
  T acc[K], scl[K], sd[K];
#pragma unroll
  for (int r = 0; r < K; ++r) acc[r] = scl[r] = sd[r] = T(0);
  if (c < c_end) {
    const ChunkDesc D = read_desc(t.chunks, c);
    cinfo = D.info;
    cfirst = D.first;
    cseg = D.seg;
    csm = D.sm;
  }
  // Every step refills its slot, also past the last window, so that between
  // a slot's refill and its next use the other kRing - 1 slots are always
  // refilled too: the wait before a window's sums then leaves the loads of
  // the windows after it in flight.
  while (c < c_end) {
#pragma unroll
    for (int q = 0; q < kRing; ++q) {
      const bool live = c < c_end;
      if (live) {
        if (k == 0) {
          // chunk start: its output slot (from the ring), scale and dot factor
          slot = rs[q];
#pragma unroll
          for (int r = 0; r < K; ++r) {
            scl[r] = (out_scale != nullptr && slot >= 0) ? gview(out_scale)[(int64_t)slot * K + r]
                                                         : T(1);
            sd[r] = T(0);
          }
          if constexpr (dotting) {
            const int64_t jd =
                ck_kind(cinfo) == kChunkPiece ? cseg : (slot >= 0 ? slot - pofs : -1);
            if (jd >= 0) {
#pragma unroll
              for (int r = 0; r < K; ++r) sd[r] = gview(sdot)[jd * K + r];
            }
          }
        }
        if ((rh >> q) & 1u) {
          if constexpr (K == 1) {
            if (cinfo & kChunkWide)
              gather_wide<T>(xl, ra[q], acc[0]);
            else
              gather_cmp<T>(xl, ra[q], acc[0]);
          } else {
            gather_add16<T, K>(xl, ra[q], rb[q], acc);
          }
        }
      }
      stream_issue<K == 1>(t, c_end, lane, ld, ra[q], rb[q], rs[q], rh, q);
      if (live && ++k == ck_windows(cinfo)) {
        finish_chunk<T, K, dotting>(cinfo, csm, acc, slot, scl, cfirst, lane, part_out, piece_out,
                                    out_scale, sd, p2acc);
#pragma unroll
        for (int r = 0; r < K; ++r) acc[r] = T(0);
        k = 0;
        if (++c < c_end) {
          const ChunkDesc D = read_desc(t.chunks, c);
          cinfo = D.info;
          cfirst = D.first;
          cseg = D.seg;
          csm = D.sm;
        }
      }
    }
  }
  if constexpr (MODE == kPassDir && kFastDir<T, K>) {
    if (assembled) {
      // the workgroup's own entries of the new direction, from the panel
      const int64_t o0 = read_table(t.wg_s0, w), o1 = read_table(t.wg_s1, w);
      T* s_new = dir.s + (int64_t)(1 - parity) * dir.sstride;
      for (int64_t j = o0 + threadIdx.x; j < o1; j += kPThreads) {
        const double v = xl[j - g0];
        gview_mut(s_new)[j] = v;
        p1acc[0] += gview(dir.d)[j] * v * v;
      }
    }
  }
  if constexpr (MODE != kPassPlain) {
    // The workgroup's partials, in a fixed order: lanes, then wavefronts
    // (the panel's LDS is free once every wavefront is done).
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const double a = wave_sum(p1acc[r]);
      const double b = wave_sum(p2acc[r]);
      if (lane == 0) {
        red[(wave * K + r) * 2 + 0] = a;
        red[(wave * K + r) * 2 + 1] = b;
      }
    }
    __syncthreads();
    if (threadIdx.x < K) {
      const int r = threadIdx.x;
      double a = 0.0, b = 0.0;
      for (int q = 0; q < kPWaves; ++q) {
        a += red[(q * K + r) * 2 + 0];
        b += red[(q * K + r) * 2 + 1];
      }
      if constexpr (MODE == kPassDir) gview_mut(dir.p1)[(int64_t)w * K + r] = a;
      if constexpr (dotting) gview_mut(dot.p2)[(int64_t)w * K + r] = b;
    }
  }
}

// The dispatcher deals workgroups to the eight XCDs in turn (block b runs on
// XCD b % 8), while logical workgroups are numbered panel by panel: giving
// each XCD a contiguous run of logical workgroups keeps each XCD's L2 on one
// or two panels of the gathered vector instead of all of them.  A bijection
// when the grid is a multiple of 8 (else the identity).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_logical_wg() {
  const int b = (int)blockIdx.x, nwg = (int)gridDim.x;
  if (nwg % kXcds) return b;
  return (b % kXcds) * (nwg / kXcds) + b / kXcds;
}

template <typename T, int MODE>
__global__ __launch_bounds__(kPThreads) void k_panel(PanelPass t, Combine<T> xin,
                                                     T* __restrict__ part_out,
                                                     T* __restrict__ piece_out,
                                                     const T* __restrict__ out_scale,
                                                     const int32_t* __restrict__ done,
                                                     DirIn<T> dir, DotOut<T> dot, int parity) {
  panel_body<T, 1, MODE>(t, xin, part_out, piece_out, out_scale, done, 0, dir, dot, parity,
                         xcd_logical_wg());
}

template <typename T, int MODE>
__global__ __launch_bounds__(kPThreads) void k_panel_b(const PanelJob<T>* __restrict__ jobs,
                                                       const int32_t* __restrict__ wg_job,
                                                       const int32_t* __restrict__ wg_local,
                                                       int parity) {
  const PanelJob<T>& J = jobs[wg_job[blockIdx.x]];
  panel_body<T, 1, MODE>(J.t, J.x, J.part_out, J.piece_out, J.out_scale, J.done, 0, J.dir,
                         J.dot, parity, wg_local[blockIdx.x]);
}

// One X pass over K interleaved vectors; skipped when the done flags of all
// K chains are set.
template <typename T, int K, int MODE>
__global__ __launch_bounds__(kPThreads) void k_panel_k(PanelPass t, Combine<T> xin,
                                                       T* __restrict__ part_out,
                                                       T* __restrict__ piece_out,
                                                       const T* __restrict__ out_scale,
                                                       const int32_t* __restrict__ done,
                                                       int dstride, DirIn<T> dir, DotOut<T> dot,
                                                       int parity) {
  panel_body<T, K, MODE>(t, xin, part_out, piece_out, out_scale, done, dstride, dir, dot,
                         parity, xcd_logical_wg());
}

static size_t pass_lds_bytes() { return (size_t)kPanelBytes; }

// The pass variant: a direction (row pass of the CG loop), a dot output
// (column pass of the CG loop), or neither; -1 for both.
template <typename T>
static int pass_mode(const DirIn<T>* dir, const DotOut<T>* dot) {
  const bool a = dir != nullptr && dir->z != nullptr;
  const bool b = dot != nullptr && dot->s != nullptr;
  if (a && b) return -1;
  return a ? kPassDir : (b ? kPassDot : kPassPlain);
}

// Host-side check of what a pass with a direction or a dot output reads
// besides the plain pass: the workgroup slices and the output dimension.
template <typename T>
static bool pass_args_ok(const PanelPass& t, const DirIn<T>* dir, const DotOut<T>* dot) {
  if (t.idx == nullptr || t.chunks == nullptr || t.wave_c == nullptr || t.wg_panel == nullptr ||
      t.seg_out == nullptr || t.no_slot < 0)
    return false;
  if (dir != nullptr && dir->z != nullptr &&
      (t.wg_s0 == nullptr || t.wg_s1 == nullptr || dir->s == nullptr || dir->d == nullptr ||
       dir->sc == nullptr || dir->p1 == nullptr))
    return false;
  if (dot != nullptr && dot->s != nullptr && (t.out_dim <= 0 || dot->p2 == nullptr))
    return false;
  return true;
}

template <typename T, int MODE>
static hipError_t set_lds(int bytes) {
  const void* fns[] = {reinterpret_cast<const void*>(&k_panel<T, MODE>),
                       reinterpret_cast<const void*>(&k_panel_b<T, MODE>),
                       reinterpret_cast<const void*>(&k_panel_k<T, 2, MODE>),
                       reinterpret_cast<const void*>(&k_panel_k<T, 4, MODE>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t setup_pass_kernels() {
  const int bytes = (int)pass_lds_bytes();
  hipError_t e;
  if ((e = set_lds<float, kPassPlain>(bytes)) != hipSuccess) return e;
  if ((e = set_lds<float, kPassDir>(bytes)) != hipSuccess) return e;
  if ((e = set_lds<float, kPassDot>(bytes)) != hipSuccess) return e;
  if ((e = set_lds<double, kPassPlain>(bytes)) != hipSuccess) return e;
  if ((e = set_lds<double, kPassDir>(bytes)) != hipSuccess) return e;
  return set_lds<double, kPassDot>(bytes);
}

template <typename T>
hipError_t launch_panel_pass_batched(const PanelJob<T>* jobs, const int32_t* wg_job,
                                     const int32_t* wg_local, int32_t nwg, int mode, int parity,
                                     hipStream_t st) {
  if (nwg <= 0) return hipSuccess;
  const dim3 g(nwg), b(kPThreads);
  const size_t lds = pass_lds_bytes();
  if (mode == kPassDir)
    hipLaunchKernelGGL((k_panel_b<T, kPassDir>), g, b, lds, st, jobs, wg_job, wg_local, parity);
  else if (mode == kPassDot)
    hipLaunchKernelGGL((k_panel_b<T, kPassDot>), g, b, lds, st, jobs, wg_job, wg_local, parity);
  else if (mode == kPassPlain)
    hipLaunchKernelGGL((k_panel_b<T, kPassPlain>), g, b, lds, st, jobs, wg_job, wg_local,
                       parity);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template <typename T>
hipError_t launch_panel_pass_k(int K, const PanelPass& t, const Combine<T>& x, T* part_out,
                               T* piece_out, const T* out_scale, const int32_t* done,
                               int dstride, hipStream_t st, const DirIn<T>* dir,
                               const DotOut<T>* dot, int parity) {
  if (t.nwg == 0) return hipSuccess;
  if (!pass_args_ok(t, dir, dot)) return hipErrorInvalidValue;
  const dim3 g(t.nwg), b(kPThreads);
  const size_t lds = pass_lds_bytes();
  const DirIn<T> di = dir ? *dir : DirIn<T>{};
  const DotOut<T> dd = dot ? *dot : DotOut<T>{};
  const int mode = pass_mode(dir, dot);
  if (mode < 0) return hipErrorInvalidValue;
#define PPCG_LAUNCH_K(KK, M)                                                                   \
  hipLaunchKernelGGL((k_panel_k<T, KK, M>), g, b, lds, st, t, x, part_out, piece_out,          \
                     out_scale, done, dstride, di, dd, parity)
#define PPCG_LAUNCH_M(KK)        \
  if (mode == kPassDir)          \
    PPCG_LAUNCH_K(KK, kPassDir); \
  else if (mode == kPassDot)     \
    PPCG_LAUNCH_K(KK, kPassDot); \
  else                           \
    PPCG_LAUNCH_K(KK, kPassPlain);
  switch (K) {
    case 2:
      PPCG_LAUNCH_M(2)
      break;
    case 4:
      PPCG_LAUNCH_M(4)
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef PPCG_LAUNCH_M
#undef PPCG_LAUNCH_K
  return hipGetLastError();
}
template hipError_t launch_panel_pass_k<float>(int, const PanelPass&, const Combine<float>&,
                                               float*, float*, const float*, const int32_t*, int,
                                               hipStream_t, const DirIn<float>*,
                                               const DotOut<float>*, int);
template hipError_t launch_panel_pass_k<double>(int, const PanelPass&, const Combine<double>&,
                                                double*, double*, const double*, const int32_t*,
                                                int, hipStream_t, const DirIn<double>*,
                                                const DotOut<double>*, int);
template hipError_t launch_panel_pass_batched<float>(const PanelJob<float>*, const int32_t*,
                                                     const int32_t*, int32_t, int, int,
                                                     hipStream_t);
template hipError_t launch_panel_pass_batched<double>(const PanelJob<double>*, const int32_t*,
                                                      const int32_t*, int32_t, int, int,
                                                      hipStream_t);

template <typename T>
hipError_t launch_panel_pass(const PanelPass& t, const Combine<T>& x, T* part_out,
                             T* piece_out, const T* out_scale, const int32_t* done,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                             const DirIn<T>* dir, const DotOut<T>* dot, int parity) {
  if (t.nwg == 0) return hipSuccess;
  if (!pass_args_ok(t, dir, dot)) return hipErrorInvalidValue;
  const DirIn<T> di = dir ? *dir : DirIn<T>{};
  const DotOut<T> dd = dot ? *dot : DotOut<T>{};
  const int mode = pass_mode(dir, dot);
  if (mode < 0) return hipErrorInvalidValue;
  const dim3 g(t.nwg), b(kPThreads);
  const size_t lds = pass_lds_bytes();
  // With events, the dispatch itself records them: the kernel's own duration.
#define PPCG_LAUNCH(M)                                                                        \
  if (ev0 != nullptr)                                                                         \
    hipExtLaunchKernelGGL((k_panel<T, M>), g, b, lds, st, ev0, ev1, 0u, t, x, part_out,       \
                          piece_out, out_scale, done, di, dd, parity);                        \
  else                                                                                        \
    hipLaunchKernelGGL((k_panel<T, M>), g, b, lds, st, t, x, part_out, piece_out, out_scale,  \
                       done, di, dd, parity);
  if (mode == kPassDir) {
    PPCG_LAUNCH(kPassDir)
  } else if (mode == kPassDot) {
    PPCG_LAUNCH(kPassDot)
  } else {
    PPCG_LAUNCH(kPassPlain)
  }
#undef PPCG_LAUNCH
  return hipGetLastError();
}

template <typename T, typename U>
__global__ __launch_bounds__(kWG) void k_combine(Combine<T> c, int64_t dim, U* out) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < dim) out[i] = (U)combine_at(c, i);
}

// The panel partials of K interleaved vectors summed into out[dim][K]: one
// thread per element, consecutive threads on consecutive addresses of every
// partial array (a per-vector reader with stride K would fetch each line K
// times).  Returns at once when all K flags done[i * dstride] are set.
template <typename T>
__global__ __launch_bounds__(kWG) void k_combine_k(Combine<T> c, int K, int64_t dim, T* out,
                                                   const int32_t* done, int dstride) {
  int all = 1;
  for (int r = 0; r < K; ++r) all &= gview(done)[(int64_t)r * dstride] != 0 ? 1 : 0;
  if (all) return;
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < dim * K) out[i] = combine_at(c, i / K, (int)(i % K));
}

template <typename T>
hipError_t launch_combine_k(const Combine<T>& c, int K, int64_t dim, T* out,
                            const int32_t* done, int dstride, hipStream_t st) {
  if (dim <= 0) return hipSuccess;
  if (c.es != K || done == nullptr) return hipErrorInvalidValue;
  const int64_t n = dim * K;
  hipLaunchKernelGGL((k_combine_k<T>), dim3((unsigned)((n + kWG - 1) / kWG)), dim3(kWG), 0, st,
                     c, K, dim, out, done, dstride);
  return hipGetLastError();
}
template hipError_t launch_combine_k<float>(const Combine<float>&, int, int64_t, float*,
                                            const int32_t*, int, hipStream_t);
template hipError_t launch_combine_k<double>(const Combine<double>&, int, int64_t, double*,
                                             const int32_t*, int, hipStream_t);

template <typename T, typename U>
hipError_t launch_combine(const Combine<T>& c, int64_t dim, U* out, hipStream_t st) {
  if (dim <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_combine<T, U>), dim3((unsigned)((dim + kWG - 1) / kWG)), dim3(kWG), 0,
                     st, c, dim, out);
  return hipGetLastError();
}

template hipError_t launch_panel_pass<float>(const PanelPass&, const Combine<float>&, float*,
                                             float*, const float*, const int32_t*, hipStream_t,
                                             hipEvent_t, hipEvent_t, const DirIn<float>*,
                                             const DotOut<float>*, int);
template hipError_t launch_panel_pass<double>(const PanelPass&, const Combine<double>&, double*,
                                              double*, const double*, const int32_t*,
                                              hipStream_t, hipEvent_t, hipEvent_t,
                                              const DirIn<double>*, const DotOut<double>*, int);
template hipError_t launch_combine<float, float>(const Combine<float>&, int64_t, float*,
                                                 hipStream_t);
template hipError_t launch_combine<double, double>(const Combine<double>&, int64_t, double*,
                                                   hipStream_t);

// ------------------------------------------------------------------------
// Box-Muller normals from Philox4x64-10 blocks
// ------------------------------------------------------------------------

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

__global__ __launch_bounds__(kWG) void k_rhs_fin_general(const double* bx, const double* d,
                                                         uint64_t seed, uint64_t chain,
                                                         uint64_t draw, int64_t p, double* b) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (4 * i >= p) return;
  double g[4];
  normals4(seed, 1ull, chain, draw, (uint64_t)i, g);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t j = 4 * i + q;
    if (j < p) b[j] = bx[j] + g[q] * sqrt(d[j]);
  }
}

hipError_t launch_rhs_fin_general(const double* bx, const double* d, uint64_t seed,
                                  uint64_t chain, uint64_t draw, int64_t p, double* b,
                                  hipStream_t st) {
  const int64_t nb = (p + 3) / 4;
  hipLaunchKernelGGL(k_rhs_fin_general, dim3((unsigned)((nb + kWG - 1) / kWG)), dim3(kWG), 0,
                     st, bx, d, seed, chain, draw, p, b);
  return hipGetLastError();
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

__global__ __launch_bounds__(kWG) void k_prep_general(const double* prior_prec,
                                                      const double* precond_inv,
                                                      const void* omega, int dtype, int64_t n,
                                                      int64_t p, double* d, double* m,
                                                      double* omega64) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < p) {
    const double pr = prior_prec[i];
    d[i] = pr;
    m[i] = precond_inv != nullptr ? precond_inv[i] : 1.0 / pr;
  }
  if (omega64 != nullptr && i < n) omega64[i] = ld_dtype(omega, dtype, i);
}

hipError_t launch_prep_general(const double* prior_prec, const double* precond_inv,
                               const void* omega, int dtype, int64_t n, int64_t p, double* d,
                               double* m, double* omega64, hipStream_t st) {
  const int64_t cnt = n > p ? n : p;
  hipLaunchKernelGGL(k_prep_general, dim3((unsigned)((cnt + kWG - 1) / kWG)), dim3(kWG), 0, st,
                     prior_prec, precond_inv, omega, dtype, n, p, d, m, omega64);
  return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_phi_diag(Combine<double> c, const double* d, int64_t p,
                                                  double* out) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j < p) out[j] = combine_at(c, j) + d[j];
}

hipError_t launch_phi_diag(const Combine<double>& c, const double* d, int64_t p, double* out,
                           hipStream_t st) {
  if (p <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_phi_diag, dim3((unsigned)((p + kWG - 1) / kWG)), dim3(kWG), 0, st, c, d,
                     p, out);
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

// dst[i K + r] = src[r][i] (r < nsrc; slots r >= nsrc untouched).
template <typename T>
__global__ __launch_bounds__(kWG) void k_interleave(VecPtrs src, int nsrc, int K, int64_t dim,
                                                    T* dst) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= dim) return;
  for (int r = 0; r < nsrc; ++r) dst[i * K + r] = (T)src.p[r][i];
}

template <typename T>
hipError_t launch_interleave(const VecPtrs& src, int nsrc, int K, int64_t dim, T* dst,
                             hipStream_t st) {
  if (dim <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_interleave<T>), dim3((unsigned)((dim + kWG - 1) / kWG)), dim3(kWG), 0,
                     st, src, nsrc, K, dim, dst);
  return hipGetLastError();
}
template hipError_t launch_interleave<float>(const VecPtrs&, int, int, int64_t, float*,
                                             hipStream_t);
template hipError_t launch_interleave<double>(const VecPtrs&, int, int, int64_t, double*,
                                              hipStream_t);

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
  int64_t g = (p + kWG - 1) / kWG;
  if (g < 1) g = 1;
  if (g > kMaxRedBlocks) g = kMaxRedBlocks;
  return (unsigned)g;
}


// The scalars copied word by word to snap by one thread, after that
// thread's own writes to them (so its loads see them): every word is loaded
// before the first store, one round trip (the compiler cannot tell that snap
// and sc do not overlap, and would otherwise wait for each load in turn).
__device__ __forceinline__ void snapshot_scal(const DevScal* sc, DevScal* snap) {
  static_assert(sizeof(DevScal) % 8 == 0, "DevScal is copied in 8-byte words");
  constexpr int kWords = (int)(sizeof(DevScal) / 8);
  const uint64_t* a = reinterpret_cast<const uint64_t*>(sc);
  uint64_t* b = reinterpret_cast<uint64_t*>(snap);
  uint64_t v[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i) v[i] = a[i];
#pragma unroll
  for (int i = 0; i < kWords; ++i) b[i] = v[i];
}

// Mode 1 restarts only a run that ended well but whose FP64 true residual
// misses the rule; any other run is left as it is.
__device__ __forceinline__ bool restart_wanted(const DevScal* sc) {
  return sc->status == kStatOK && sc->true_meas > sc->thresh2;
}

__device__ __forceinline__ void cg_start_body(VecWork w, int mode, const double* b,
                                              const double* qx64, const double* d,
                                              const double* m, double* beta, double* r,
                                              double* z, int64_t p, double tol, int criterion,
                                              int max_iter, double loop_factor, VGrid g,
                                              int zes = 1, DevScal* snap = nullptr) {
  if (mode == 1 && !restart_wanted(w.sc)) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // <r,Mr>, <r,r>, <b,Mb>, <b,b>
  for (int64_t j = (int64_t)g.bid * kWG + threadIdx.x; j < p; j += (int64_t)g.nblk * kWG) {
    const double bj = b[j];
    const double rj = qx64 ? bj - qx64[j] - d[j] * beta[j] : bj;
    const double zj = m[j] * rj;
    v[0] += rj * zj;
    v[1] += rj * rj;
    if (mode == 0) {
      v[2] += bj * m[j] * bj;
      v[3] += bj * bj;
      if (qx64 == nullptr) beta[j] = 0.0;
    }
    if (mode != 2) {
      r[j] = rj;
      z[j * zes] = zj;
    }
  }
  block_sum<4>(v);
  if (!publish_and_arrive<4>(v, w.part, &w.sc->arrive[1], g)) return;
  double tot[4];
  gather_totals<4>(w.part, &w.sc->arrive[1], tot, g);
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
      sc->refined = 0;
      sc->criterion = criterion;
      sc->max_iter = max_iter;
      sc->bm2 = tot[2];
      sc->bb = tot[3];
      const double t2 = tol * tol;
      sc->thresh2 = criterion == kCritRelPrecond ? t2 * tot[2]
                  : criterion == kCritRmsAbs     ? t2 * (double)p
                                                 : t2 * tot[3];
      sc->loop2 = sc->thresh2 * loop_factor * loop_factor;
    }
    sc->betacg = 0.0;  // the first row pass takes s = z
    sc->rho_prev = tot[0];
    sc->rho = tot[0];
    sc->rho_par[0] = tot[0];
    sc->rr = tot[1];
    sc->meas = meas;
    sc->iters = 0;
    sc->status = kStatOK;
    sc->alpha = 0.0;
    sc->done = (meas <= sc->loop2) ? 1 : 0;
    if (mode == 1) sc->refined = 1;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      sc->status = kStatBreakdown;
      sc->done = 1;
    }
    if (snap) snapshot_scal(sc, snap);
  }
}

// One CG step after the two passes (see launch_cg_step).  p1 / p2 hold the
// passes' workgroup partials (n1 and n2 of them, stride ps).
template <typename T, bool PassFinish = false>
__device__ __forceinline__ void cg_step_body(VecWork w, const T* s, int es,
                                             const Combine<T>& qsrc, const double* d,
                                             const double* m, double* beta, double* r,
                                             double* z, int zes, const double* p1, int n1,
                                             const double* p2, int n2, int ps, int64_t p,
                                             VGrid g, int parity = 0, DevScal* snap = nullptr) {
  DevScal* sc = w.sc;
  const bool snapper = PassFinish && snap != nullptr && g.bid == 0 && threadIdx.x == 0;
  // The passes' partials and this thread's first element are requested
  // before the stop flag is tested (every read is in bounds either way) and
  // before the grid total below (the element does not depend on alpha), so
  // that all these loads are in flight together.
  // <s, Phi s> = <s, d s> + <s, X^T u>: the same fixed-order total in every
  // block, all threads loading at once (the partials come from other XCDs);
  // one partial of each pass per thread when they fit, a loop otherwise.
  const bool fit = n1 <= kWG && n2 <= kWG;
  double pa = 0.0, pb = 0.0;
  if (fit) {
    if ((int)threadIdx.x < n1) pa = p1[(int64_t)threadIdx.x * ps];
    if ((int)threadIdx.x < n2) pb = p2[(int64_t)threadIdx.x * ps];
  }
  const int64_t j0 = (int64_t)g.bid * kWG + threadIdx.x;
  double s0 = 0.0, q0 = 0.0, d0 = 0.0, r0 = 0.0, m0 = 0.0;
  if (j0 < p) {
    s0 = (double)s[j0 * es];
    q0 = (double)combine_at(qsrc, j0);
    d0 = d[j0];
    r0 = r[j0];
    m0 = m[j0];
  }
  double a[1] = {0.0};
  if (fit) {
    a[0] += pa;
    a[0] += pb;
  } else {
    for (int q = threadIdx.x; q < n1; q += kWG) a[0] += p1[(int64_t)q * ps];
    for (int q = threadIdx.x; q < n2; q += kWG) a[0] += p2[(int64_t)q * ps];
  }
  if (sc->done) {
    if (snapper) snapshot_scal(sc, snap);
    return;
  }
  const double rho = sc->rho;
  __shared__ double sq_sh;
  {
    block_sum<1>(a);
    if (threadIdx.x == 0) sq_sh = a[0];
  }
  __syncthreads();
  const double sq = sq_sh;
  if (!(sq > 0.0) || !isfinite(sq)) {
    if (g.bid == 0 && threadIdx.x == 0) {
      sc->sq = sq;
      sc->status = kStatBreakdown;
      sc->done = 1;
      sc->alpha = 0.0;
      if (snapper) snapshot_scal(sc, snap);
    }
    return;
  }
  const double alpha = rho / sq;
  double v[2] = {0.0, 0.0};  // <r, M^-1 r>, <r, r>
  for (int64_t j = j0; j < p; j += (int64_t)g.nblk * kWG) {
    const bool first = j == j0;
    const double sj = first ? s0 : (double)s[j * es];
    const double qj = (first ? q0 : (double)combine_at(qsrc, j)) + (first ? d0 : d[j]) * sj;
    beta[j] += alpha * sj;
    const double rj = (first ? r0 : r[j]) - alpha * qj;
    r[j] = rj;
    const double zj = (first ? m0 : m[j]) * rj;
    z[j * zes] = zj;
    v[0] += rj * zj;
    v[1] += rj * rj;
  }
  block_sum<2>(v);
  if constexpr (PassFinish) {
    // the next row pass totals these (see DirIn)
    if (threadIdx.x == 0) {
      double* out = w.part + (int64_t)parity * 2 * kMaxRedBlocks + 2 * g.bid;
      out[0] = v[0];
      out[1] = v[1];
      if (g.bid == 0) {
        sc->sq = sq;
        sc->alpha = alpha;
        if (snapper) snapshot_scal(sc, snap);
      }
    }
    return;
  }
  if (!publish_and_arrive<2>(v, w.part, &w.sc->arrive[3], g)) return;
  double tot[2];
  gather_totals<2>(w.part, &w.sc->arrive[3], tot, g);
  if (threadIdx.x == 0) {
    const double rho_new = tot[0];
    sc->sq = sq;
    sc->alpha = alpha;
    sc->iters += 1;
    sc->rr = tot[1];
    const double meas = (sc->criterion == kCritRelPlain) ? tot[1] : rho_new;
    sc->meas = meas;
    sc->betacg = rho_new / sc->rho;
    sc->rho_prev = sc->rho;
    sc->rho = rho_new;
    if (!isfinite(rho_new)) {
      sc->status = kStatBreakdown;
      sc->done = 1;
    } else if (meas <= sc->loop2) {
      sc->done = 1;
    } else if (sc->iters >= sc->max_iter) {
      sc->status = kStatNotConv;
      sc->done = 1;
    }
  }
}

// ---- one chain ----
__global__ __launch_bounds__(kWG) void k_cg_start(VecWork w, int mode, const double* b,
                                                  const double* qx64, const double* d,
                                                  const double* m, double* beta, double* r,
                                                  double* z, int64_t p, double tol,
                                                  int criterion, int max_iter,
                                                  double loop_factor, DevScal* snap) {
  cg_start_body(w, mode, b, qx64, d, m, beta, r, z, p, tol, criterion, max_iter, loop_factor,
                own_grid(), 1, snap);
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_step(VecWork w, const T* s, Combine<T> qsrc,
                                                 const double* d, const double* m, double* beta,
                                                 double* r, double* z, const double* p1,
                                                 int n1, const double* p2, int n2, int64_t p) {
  cg_step_body<T>(w, s, 1, qsrc, d, m, beta, r, z, 1, p1, n1, p2, n2, 1, p, own_grid());
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_step_pf(VecWork w, const T* s, Combine<T> qsrc,
                                                    const double* d, const double* m,
                                                    double* beta, double* r, double* z,
                                                    const double* p1, int n1, const double* p2,
                                                    int n2, int64_t p, int parity,
                                                    DevScal* snap) {
  cg_step_body<T, true>(w, s, 1, qsrc, d, m, beta, r, z, 1, p1, n1, p2, n2, 1, p, own_grid(),
                        parity, snap);
}

hipError_t launch_cg_start(VecWork w, int mode, const double* b, const double* qx64,
                           const double* d, const double* m, double* beta, double* r,
                           double* z, int64_t p, double tol, int criterion, int max_iter,
                           double loop_factor, hipStream_t st, DevScal* snap) {
  hipLaunchKernelGGL(k_cg_start, dim3(red_grid(p)), dim3(kWG), 0, st, w, mode, b, qx64, d, m,
                     beta, r, z, p, tol, criterion, max_iter, loop_factor, snap);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_cg_step(VecWork w, const T* s, int64_t sstride, int parity, bool pass_finish,
                          const Combine<T>& qsrc, const double* d, const double* m,
                          double* beta, double* r, double* z, const double* p1, int32_t n1,
                          const double* p2, int32_t n2, int64_t p, hipStream_t st,
                          DevScal* snap) {
  const T* sn = s + (int64_t)(1 - parity) * sstride;
  if (pass_finish)
    hipLaunchKernelGGL((k_cg_step_pf<T>), dim3(red_grid(p)), dim3(kWG), 0, st, w, sn, qsrc, d, m,
                       beta, r, z, p1, n1, p2, n2, p, parity, snap);
  else
    hipLaunchKernelGGL((k_cg_step<T>), dim3(red_grid(p)), dim3(kWG), 0, st, w, sn, qsrc, d, m,
                       beta, r, z, p1, n1, p2, n2, p);
  return hipGetLastError();
}

// ---- many chains: block g runs block blk_local[g] of chain blk_job[g] ----
template <typename T>
__device__ __forceinline__ const VecJob<T>& vec_job(const VecJob<T>* jobs,
                                                    const int32_t* blk_job,
                                                    const int32_t* blk_local, VGrid& g) {
  const VecJob<T>& J = jobs[blk_job[blockIdx.x]];
  g = VGrid{blk_local[blockIdx.x], J.nblk};
  return J;
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_start_b(const VecJob<T>* jobs,
                                                    const int32_t* blk_job,
                                                    const int32_t* blk_local, int mode,
                                                    double tol, int criterion, int max_iter,
                                                    double loop_factor) {
  VGrid g;
  const VecJob<T>& J = vec_job(jobs, blk_job, blk_local, g);
  cg_start_body(J.w, mode, J.b, mode == 0 ? nullptr : J.qx64, J.d, J.m, J.beta, J.r, J.z, J.p,
                tol, criterion, max_iter > 0 ? max_iter : J.max_iter, loop_factor, g, J.zes);
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_cg_step_b(const VecJob<T>* jobs, const int32_t* blk_job,
                                                   const int32_t* blk_local, int parity) {
  VGrid g;
  const VecJob<T>& J = vec_job(jobs, blk_job, blk_local, g);
  cg_step_body<T>(J.w, J.s + (int64_t)(1 - parity) * J.sstride, J.es, J.qsrc, J.d, J.m, J.beta,
                  J.r, J.z, J.zes, J.p1, J.n1, J.p2, J.n2, J.pstride, J.p, g);
}

int32_t vec_blocks(int64_t p) { return (int32_t)red_grid(p); }

template <typename T>
hipError_t launch_cg_start_batched(const VecJob<T>* jobs, const int32_t* blk_job,
                                   const int32_t* blk_local, int32_t nblk, int mode, double tol,
                                   int criterion, int max_iter, double loop_factor,
                                   hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cg_start_b<T>), dim3(nblk), dim3(kWG), 0, st, jobs, blk_job, blk_local,
                     mode, tol, criterion, max_iter, loop_factor);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_cg_step_batched(const VecJob<T>* jobs, const int32_t* blk_job,
                                  const int32_t* blk_local, int32_t nblk, int parity,
                                  hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cg_step_b<T>), dim3(nblk), dim3(kWG), 0, st, jobs, blk_job, blk_local,
                     parity);
  return hipGetLastError();
}

#define PPCG_INST(T)                                                                         \
  template hipError_t launch_cg_step<T>(VecWork, const T*, int64_t, int, bool, const Combine<T>&,  \
                                        const double*, const double*, double*, double*,      \
                                        double*, const double*, int32_t, const double*,      \
                                        int32_t, int64_t, hipStream_t, DevScal*);            \
  template hipError_t launch_cg_start_batched<T>(const VecJob<T>*, const int32_t*,           \
                                                 const int32_t*, int32_t, int, double, int,    \
                                                 int, double, hipStream_t);                    \
  template hipError_t launch_cg_step_batched<T>(const VecJob<T>*, const int32_t*,            \
                                                const int32_t*, int32_t, int, hipStream_t);
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
  const VGrid g = own_grid();
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
  if (!publish_and_arrive<1>(v, w.part, &w.sc->arrive[4], g)) return;
  double tot[1];
  gather_totals<1>(w.part, &w.sc->arrive[4], tot, g);
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
