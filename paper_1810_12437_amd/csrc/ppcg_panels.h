// Host-side builder of the panel-blocked, index-only layout of one
// orientation of X (see PanelPass in ppcg_kernels.h).  Plain C++.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <array>
#include <vector>

#include "ppcg_layout.h"

namespace ppcg {

// Host-side build of one orientation of X in the panel-blocked layout of
// PanelPass (see ppcg_kernels.h).
struct PanelBuild {
  std::vector<uint16_t> idx;
  std::vector<int64_t> cstart;
  std::vector<int32_t> cseg, cnseg;
  std::vector<uint64_t> cmask;
  std::vector<int32_t> seg_out;
  std::vector<int32_t> wg_panel, wg_c0, wg_c1;
  std::vector<int32_t> sp_off, sp_c0, sp_c1;
  int64_t gdim = 0, out_dim = 0;
  int32_t W = 1, npanels = 1;
};

// off: segment offsets (out_dim + 1), gidx: gathered index of each element
// (increasing within a segment), gdim: gathered dimension, elem: bytes of
// one gathered value, ncu: compute units to spread the workgroups over.
//
// Every (segment, panel) is padded with the sentinel index W (a zero in the
// LDS panel) to a multiple of kPV elements, so each lane's kPV elements
// belong to one segment.  Chunk kinds (cnseg): > 0 packs whole padded
// segments into up to kPNW windows (kPGroups groups of kPV elements), with
// bit g of the chunk's kPNW mask words set when group g starts a segment; 0
// is one segment longer than that, summed whole by one wavefront; < 0 is a
// piece of a segment longer than kPLongMax (its sum goes to the piece array
// and the consumer adds the pieces).
void build_panels(const std::vector<int64_t>& off, const std::vector<int32_t>& gidx,
                  int64_t out_dim, int64_t gdim, int elem, int ncu, PanelBuild& B) {
  B = PanelBuild();
  B.gdim = gdim;
  B.out_dim = out_dim;
  const int64_t wmax = kPanelBytes / elem - 1;  // one LDS slot holds the zero sentinel
  B.npanels = (int32_t)((gdim + wmax - 1) / wmax);
  if (B.npanels < 1) B.npanels = 1;
  B.W = (int32_t)((gdim + B.npanels - 1) / B.npanels);
  const uint16_t sentinel = (uint16_t)B.W;
  std::vector<int64_t> cur(off.begin(), off.end() - 1);
  std::vector<int32_t> pc0(B.npanels + 1, 0);
  std::vector<std::array<int32_t, 3>> splits;  // (segment id, c0, c1)
  std::vector<int64_t> seg_a, seg_e;           // element range of each (segment, panel)
  auto groups = [&](int64_t len) { return (len + kPV - 1) / kPV; };
  auto append = [&](int64_t a, int64_t e, int64_t glo) {
    for (int64_t q = a; q < e; ++q) B.idx.push_back((uint16_t)(gidx[q] - glo));
    while (B.idx.size() % kPV) B.idx.push_back(sentinel);
  };
  for (int32_t k = 0; k < B.npanels; ++k) {
    const int64_t hi = (int64_t)(k + 1) * B.W;
    const int64_t glo = (int64_t)k * B.W;
    const int64_t seg_first = (int64_t)B.seg_out.size();
    for (int64_t sgm = 0; sgm < out_dim; ++sgm) {
      const int64_t a = cur[sgm];
      int64_t e = a;
      const int64_t end = off[sgm + 1];
      while (e < end && gidx[e] < hi) ++e;
      if (e > a) {
        B.seg_out.push_back((int32_t)((int64_t)k * out_dim + sgm));
        seg_a.push_back(a);
        seg_e.push_back(e);
        cur[sgm] = e;
      }
    }
    const int64_t seg_end = (int64_t)B.seg_out.size();
    pc0[k] = (int32_t)B.cseg.size();
    int64_t g = seg_first;
    while (g < seg_end) {
      const int64_t len = seg_e[g] - seg_a[g];
      if (groups(len) > kPGroups) {
        if (len <= kPLongMax) {
          B.cstart.push_back((int64_t)B.idx.size());
          B.cseg.push_back((int32_t)g);
          B.cnseg.push_back(0);
          for (int q = 0; q < kPNW; ++q) B.cmask.push_back(0);
          append(seg_a[g], seg_e[g], glo);
        } else {
          const int32_t c0 = (int32_t)B.cseg.size();
          for (int64_t o = seg_a[g]; o < seg_e[g]; o += kPLongMax) {
            B.cstart.push_back((int64_t)B.idx.size());
            B.cseg.push_back((int32_t)g);
            B.cnseg.push_back(-1);
            for (int q = 0; q < kPNW; ++q) B.cmask.push_back(0);
            append(o, std::min<int64_t>(o + kPLongMax, seg_e[g]), glo);
          }
          splits.push_back({(int32_t)(B.seg_out[g] % out_dim), c0, (int32_t)B.cseg.size() - 1});
        }
        ++g;
      } else {
        const int64_t first = g;
        int64_t used = 0;  // groups
        uint64_t mask[kPNW] = {};
        B.cstart.push_back((int64_t)B.idx.size());
        while (g < seg_end && used + groups(seg_e[g] - seg_a[g]) <= kPGroups) {
          mask[used / 64] |= 1ull << (used % 64);
          used += groups(seg_e[g] - seg_a[g]);
          append(seg_a[g], seg_e[g], glo);
          ++g;
        }
        B.cseg.push_back((int32_t)first);
        B.cnseg.push_back((int32_t)(g - first));
        for (int q = 0; q < kPNW; ++q) B.cmask.push_back(mask[q]);
      }
    }
  }
  pc0[B.npanels] = (int32_t)B.cseg.size();
  B.cstart.push_back((int64_t)B.idx.size());
  // pieces of segments longer than kPLongMax, grouped by output element
  if (!splits.empty()) {
    std::stable_sort(splits.begin(), splits.end(),
                     [](const std::array<int32_t, 3>& a, const std::array<int32_t, 3>& b) {
                       return a[0] < b[0];
                     });
    B.sp_off.assign(out_dim + 1, 0);
    for (auto& sp : splits) B.sp_off[sp[0] + 1]++;
    for (int64_t i = 0; i < out_dim; ++i) B.sp_off[i + 1] += B.sp_off[i];
    for (auto& sp : splits) {
      B.sp_c0.push_back(sp[1]);
      B.sp_c1.push_back(sp[2]);
    }
  }
  // workgroups: each serves one panel, in proportion to its elements
  const int nwg_total = std::max<int>(ncu, B.npanels);
  std::vector<int64_t> pe(B.npanels, 0);
  for (int32_t k = 0; k < B.npanels; ++k) pe[k] = B.cstart[pc0[k + 1]] - B.cstart[pc0[k]];
  const int64_t tot = std::max<int64_t>(B.cstart.back(), 1);
  std::vector<int> g_k(B.npanels, 0);
  int assigned = 0;
  for (int32_t k = 0; k < B.npanels; ++k) {
    const int64_t ck = pc0[k + 1] - pc0[k];
    if (ck == 0) continue;
    int gk = (int)((int64_t)nwg_total * pe[k] / tot);
    gk = std::max(1, std::min<int>(gk, (int)ck));
    g_k[k] = gk;
    assigned += gk;
  }
  while (assigned < nwg_total) {
    int best = -1;
    double best_load = 0.0;
    for (int32_t k = 0; k < B.npanels; ++k) {
      const int64_t ck = pc0[k + 1] - pc0[k];
      if (ck == 0 || g_k[k] >= ck) continue;
      const double load = (double)pe[k] / g_k[k];
      if (load > best_load) {
        best_load = load;
        best = k;
      }
    }
    if (best < 0) break;
    g_k[best]++;
    assigned++;
  }
  // within a panel, split the chunks into equal-element ranges
  for (int32_t k = 0; k < B.npanels; ++k) {
    if (g_k[k] == 0) continue;
    const int64_t e_lo = B.cstart[pc0[k]];
    int32_t c = pc0[k];
    for (int i = 0; i < g_k[k]; ++i) {
      const int64_t target = e_lo + pe[k] * (i + 1) / g_k[k];
      const int32_t c_begin = c;
      if (i == g_k[k] - 1) {
        c = pc0[k + 1];
      } else {
        while (c < pc0[k + 1] && B.cstart[c + 1] <= target) ++c;
        if (c == c_begin && c < pc0[k + 1]) ++c;  // at least one chunk each
      }
      B.wg_panel.push_back(k);
      B.wg_c0.push_back(c_begin);
      B.wg_c1.push_back(c);
    }
  }
}

}  // namespace ppcg
