// Layout constants of the panel-blocked X passes (shared by the kernels and
// the host-side table builder; no HIP dependency).
#pragma once

namespace ppcg {

constexpr int kPWaves = 16;            // wavefronts per pass workgroup
constexpr int kPThreads = kPWaves * 64;
constexpr int kPV = 16;                // elements per lane (one group)
constexpr int kPC = 64 * kPV;          // window: the elements one wavefront reads at once
constexpr int kPNW = 2;                // windows of a packed chunk
constexpr int kPGroups = 64 * kPNW;    // lane groups of a packed chunk
constexpr int kPLongMax = 16 * kPC;    // longest segment a single wavefront sums whole
constexpr int kPanelBytes = 160 * 1024 - 64;  // LDS for the gathered panel (+ zero slot)

}  // namespace ppcg
