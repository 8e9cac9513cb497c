// Layout constants of the panel-blocked X passes (shared by the kernels and
// the host-side table builder; no HIP dependency).
#pragma once

namespace ppcg {

constexpr int kPWaves = 16;            // wavefronts per pass workgroup
constexpr int kPThreads = kPWaves * 64;
constexpr int kPV = 16;                // elements per lane per chunk
constexpr int kPC = 64 * kPV;          // window: elements one wavefront reads at once
constexpr int kPPad = 16;              // chunks start and end on multiples of this
constexpr int kPSegMax = 256;          // segments per packed chunk
constexpr int kPLongMax = 16 * kPC;    // longest segment a single wavefront sums whole
constexpr int kPanelBytes = 128 * 1024;  // LDS for the gathered panel

}  // namespace ppcg
