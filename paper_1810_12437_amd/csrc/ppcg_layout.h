// Layout of the panel-blocked X passes, shared by the kernels and the
// host-side table builder (plain C++, no HIP dependency).
#pragma once

#include <stdint.h>

namespace ppcg {

constexpr int kPWaves = 16;            // wavefronts per pass workgroup
constexpr int kPThreads = kPWaves * 64;
constexpr int kPV = 16;                // elements per lane in one window (one group)
constexpr int kPC = 64 * kPV;          // window: the elements one wavefront reads at once
constexpr int kPR = 4;                 // windows of a packed chunk
constexpr int kRing = 4;               // windows a pass wavefront has in flight
constexpr int kPLongWin = 16;          // most windows of a long chunk
constexpr int kPLongMax = kPLongWin * kPC;  // longest segment one wavefront sums whole
constexpr int kPanelBytes = 160 * 1024 - 64;  // LDS for the gathered panel (+ zero slot)
constexpr int kPLongGroups = kPLongWin * 64;  // most groups one wavefront sums whole
// (after the pass, the same LDS holds the workgroup's partial-sum reduction)

// Relative work of the wavefronts of a pass workgroup by rank.  Wavefront q
// runs on SIMD q % 4 as the (q / 4)-th oldest of its four, and the SIMD's
// arbiter issues the older ones first: given equal shares, the youngest end
// about 40 % after the oldest.  The chunk lists give each rank a share in
// proportion to its issue rate measured with equal shares, so that all
// sixteen end together.
constexpr double kWaveRankWeight[4] = {1.0, 0.91, 0.80, 0.72};
inline double wave_weight(int q) { return kWaveRankWeight[(q % kPWaves) / 4]; }

enum ChunkKind { kChunkPacked = 0, kChunkLong = 1, kChunkPiece = 2 };

// Compact groups (the tables of one gathered vector per pass): a group is
// 16 bytes, read by its lane with one 16-byte load: its first panel-local
// index (bytes 0-1), its pad count c (byte 2) and 13 one-byte differences
// (bytes 3-15) give indices e_0..e_13 of at most kCGroup real entries, any
// two consecutive ones at most 255 apart (a segment's run is cut into as
// many groups as that takes).  The c pads repeat the last real index
// (difference 0), and the summing lane takes c times that entry off again.
constexpr int kCGroup = 14;  // entries per compact group
// Wide groups, for segment entries whose runs the 255 limit would cut into
// mostly padded compact groups (sparse segments): the same 16 bytes hold
// the first index (bytes 0-1), the pad count (byte 2, byte 3 zero) and six
// 16-bit differences (bytes 4-15), so kWGroup entries at any distance
// within the panel.  A chunk holds groups of one kind: wide when bit
// kChunkWide of its info is set.
constexpr int kWGroup = 7;  // entries per wide group
constexpr int32_t kChunkWide = 1 << 18;

// One chunk of an orientation's index stream, read by one wavefront.
//
// Packed chunk: up to 64 lanes x kPR windows.  Each segment of the chunk owns
// a contiguous lane range (a slice) for the whole chunk: its groups go to
// its lanes kPR at a time (group j on lane l0 + j / kPR in window j % kPR),
// so a lane only ever sums elements of one segment.  Bit l of vm[k] is set when lane l has a
// group in window k; the ng groups of window k follow those of the windows
// before it: compact groups in lane order (the lane of rank r reads group r),
// kPV-index groups stored as halves: the first kPV / 2 entries of each group
// in lane order, then the second halves (the lane of rank r reads entries
// r kPV/2 and (ng + r) kPV/2 of the window).  Bit
// l of sm is set when lane l starts a slice (lanes after the last segment
// form one idle slice).
//
// Long chunk: one segment (or, for a piece, a part of one) laid out as
// consecutive windows of 64 groups (the last one fewer), each stored the
// same way; vm[0] holds its group count times kPV.
struct alignas(64) ChunkDesc {
  int64_t base;      // first 16-bit word of the chunk in the index stream
  uint64_t vm[kPR];  // see above
  uint64_t sm;
  int32_t first;     // packed: first seg_out entry; long: its seg_out entry; piece: its id
  int32_t info;      // windows | kind << 8 | row steps << 12 | bcast15 << 16 | bcast31 << 17
                     //   | wide groups << 18 | segments << 24
  int64_t seg;       // piece: the segment (output element) it is part of
};
static_assert(sizeof(ChunkDesc) == 64, "chunk descriptor is one 64-byte scalar load");

constexpr int32_t chunk_info(int windows, int kind, int nrow, int b15, int b31, int nseg,
                             bool wide = false) {
  return windows | (kind << 8) | (nrow << 12) | (b15 << 16) | (b31 << 17) |
         (wide ? kChunkWide : 0) | (nseg << 24);
}

}  // namespace ppcg
