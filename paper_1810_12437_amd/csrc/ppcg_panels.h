// Host-side builder of the panel-blocked, index-only layout of one
// orientation of X (see PanelPass in ppcg_kernels.h and ChunkDesc in
// ppcg_layout.h).  Plain C++.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <array>
#include <numeric>
#include <vector>

#include "ppcg_layout.h"

namespace ppcg {

struct PanelBuild {
  std::vector<uint16_t> idx;
  std::vector<ChunkDesc> chunks;  // wave-major: the chunks of wave q of workgroup w are
                                  // [wave_c[16 w + q], wave_c[16 w + q + 1])
  std::vector<int32_t> seg_out;
  std::vector<int32_t> wg_panel, wave_c;
  std::vector<int32_t> wg_s0, wg_s1;  // gathered entries [s0, s1) each workgroup owns
  std::vector<int32_t> sp_off, sp_c0, sp_c1;  // pieces of element i: ids sp_c0..sp_c1
  int64_t gdim = 0, out_dim = 0;
  int64_t nseg = 0;    // (segment, panel) pairs with elements
  int32_t npieces = 0;
  int32_t W = 1, npanels = 1;
};

namespace detail {

inline int ceil_log2(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return s;
}

// Whether the lane range [l0, l0 + w) contains both lane a and lane a + 1.
inline bool crosses(int l0, int w, int a) { return l0 <= a && a + 1 < l0 + w; }

struct Entry {
  int64_t a, e, g;    // element range, groups
  int32_t slot;       // panel * out_dim + segment
  int64_t g0;         // compact tables: the entry's first group in the group starts
  bool wide = false;  // compact tables: wide groups (kWGroup entries, 16-bit differences)
};

// A chunk's share of a wavefront's work, in half windows of compact groups:
// a window of compact groups issues 14 gathers per lane, one of wide groups
// 7 (window_cost).
inline int window_cost(bool wide) { return wide ? 1 : 2; }
inline int chunk_cost(const ChunkDesc& d) {
  const int u = window_cost((d.info & kChunkWide) != 0);
  if (((d.info >> 8) & 3) != kChunkPacked) return (d.info & 0xff) * u;
  int c = 0;
  for (int k = 0; k < kPR; ++k) c += d.vm[k] ? 1 : 0;
  return c * u;
}

// Packed chunks of one panel from its entries sorted by decreasing length:
// each chunk takes entries from the front (longest) while they fit, then
// fills its leftover lanes from the back (shortest).  An entry of g groups
// gets ceil(g / R) lanes, R being the chunk's windows.
struct Packer {
  const std::vector<Entry>* ent;
  std::vector<int32_t> order;  // packed entries, longest first
  size_t lo = 0, hi = 0;

  bool empty() const { return lo >= hi; }
  int lanes(int32_t i, int R) const { return (int)(((*ent)[i].g + R - 1) / R); }
  int min_windows() const {  // windows the shortest entry needs to fit one chunk
    return (int)(((*ent)[order[hi - 1]].g + 63) / 64);
  }

  // Takes the members of the next chunk of R windows (no stream output).
  void take(int R, std::vector<int32_t>& members) {
    members.clear();
    int used = 0;
    while (lo < hi && used + lanes(order[lo], R) <= 64) {
      used += lanes(order[lo], R);
      members.push_back(order[lo++]);
    }
    while (hi > lo && used + lanes(order[hi - 1], R) <= 64) {
      used += lanes(order[hi - 1], R);
      members.push_back(order[--hi]);
    }
  }
};


// LDS banks of a gathered entry: the panel holds elem-byte values, so entry i
// starts at dword i * elem / 4 of 64 four-byte banks; a gather instruction
// reads one entry per lane, and lanes of one half-wavefront that hit the same
// bank at different entries are served one after the other.
inline int entry_bank(int i, int elem) { return (int)(((int64_t)i * (elem / 4)) & 63) >> (elem == 8 ? 1 : 0); }

// Orders the kPV entries of each group of one window (lanes[g] is the lane
// of group g, grp[g] its entries) so that, instruction by instruction, the
// lanes of each half-wavefront read entries of different banks where they
// can: a greedy pass over the positions, each lane taking the remaining
// entry whose bank is least used at that position.  Only the order in which
// a lane sums its group changes.
inline void spread_window(uint16_t* const* grp, const int* lanes, int ngroups, int elem,
                          uint16_t sentinel) {
  const int nb = elem == 8 ? 32 : 64;
  for (int pos = 0; pos < kPV; ++pos) {
    int cnt[2][64] = {};
    int seen_e[2][64];  // one distinct entry per bank counts once per repeat
    for (int h = 0; h < 2; ++h)
      for (int b = 0; b < 64; ++b) seen_e[h][b] = -1;
    for (int g = 0; g < ngroups; ++g) {
      uint16_t* e = grp[g];
      const int h = lanes[g] >> 5;
      int best = pos, best_cost = 1 << 30;
      for (int q = pos; q < kPV; ++q) {
        const int b = entry_bank(e[q], elem) % nb;
        const int cost = (e[q] == sentinel || seen_e[h][b] == (int)e[q]) ? -1 : cnt[h][b];
        if (cost < best_cost) {
          best_cost = cost;
          best = q;
        }
      }
      std::swap(e[pos], e[best]);
      if (e[pos] != sentinel) {
        const int b = entry_bank(e[pos], elem) % nb;
        if (seen_e[h][b] != (int)e[pos]) cnt[h][b]++;
        seen_e[h][b] = e[pos];
      }
    }
  }
}
}  // namespace detail

// off: segment offsets (out_dim + 1), gidx: gathered index of each element
// (increasing within a segment), gdim: gathered dimension, elem: bytes of
// one gathered value, ncu: compute units to spread the workgroups over.
//
// The gathered dimension is cut into panels of W entries (W + 1 values fit
// the LDS budget; slot W holds the zero the padding indices point to).  Each
// non-empty (segment, panel) pair is a segment entry of g = ceil(len / kPV)
// groups, padded with the index W.  Entries of at most 64 kPR groups go to
// packed chunks; longer ones get long chunks of up to kPLongWin windows, and
// one longer than that is cut into pieces whose sums the consumer adds.
// Each panel gets workgroups in proportion to its windows; every wavefront
// of them gets an explicit chunk list: long chunks first (least loaded
// wavefront per unit of weight first), then packed chunks up to its share of
// windows (in proportion to wave_weight), the last chunk of a share built
// with fewer windows (from the shortest entries when the longest do not fit
// in fewer) to end on the share.
//
// With `compact` (tables of one gathered vector) groups are the compact
// 16-byte groups of ppcg_layout.h: up to kCGroup consecutive entries at most
// 255 apart, a segment's run being cut into as many groups as that takes,
// or, for an entry where wide groups of kWGroup entries are fewer (sparse
// segments, whose runs the cuts would leave mostly padding), wide groups;
// packed chunks hold entries of one kind.  Otherwise (K interleaved vectors)
// groups are kPV 16-bit indices padded with the zero index W and stored as
// halves.
inline void build_panels(const std::vector<int64_t>& off, const std::vector<int32_t>& gidx,
                         int64_t out_dim, int64_t gdim, int elem, int ncu, PanelBuild& B,
                         bool compact = false) {
  using detail::Entry;
  B = PanelBuild();
  B.gdim = gdim;
  B.out_dim = out_dim;
  const int64_t wmax = kPanelBytes / elem - 1;
  B.npanels = (int32_t)((gdim + wmax - 1) / wmax);
  if (B.npanels < 1) B.npanels = 1;
  B.W = (int32_t)((gdim + B.npanels - 1) / B.npanels);
  const uint16_t sentinel = (uint16_t)B.W;
  const int64_t packed_max = 64 * kPR;  // groups
  std::vector<int64_t> gstart;  // compact: first element of every group

  auto append_group = [&](int64_t a, int64_t e, int64_t glo) {
    // elements [a, e) (at most kPV) as one padded group
    int64_t q = a;
    for (; q < e; ++q) B.idx.push_back((uint16_t)(gidx[q] - glo));
    for (; q < a + kPV; ++q) B.idx.push_back(sentinel);
  };
  // group j of entry en as one compact group: first index, pad count, the
  // differences (0 for the pads, which repeat the last index); one- or
  // two-byte differences as the entry is narrow or wide
  auto append_cgroup = [&](const Entry& en, int64_t j, int64_t glo) {
    const int64_t a = gstart[en.g0 + j];
    const int64_t e = j + 1 < en.g ? gstart[en.g0 + j + 1] : en.e;
    const int64_t i0 = gidx[a] - glo;
    uint16_t w[8];
    if (en.wide) {
      w[0] = (uint16_t)i0;
      w[1] = (uint16_t)(kWGroup - (e - a));
      for (int k = 1; k < kWGroup; ++k) {
        const int64_t q = a + k;
        w[k + 1] = q < e ? (uint16_t)(gidx[q] - gidx[q - 1]) : 0;
      }
    } else {
      uint8_t by[16];
      by[0] = (uint8_t)(i0 & 0xff);
      by[1] = (uint8_t)(i0 >> 8);
      by[2] = (uint8_t)(kCGroup - (e - a));
      for (int k = 1; k < kCGroup; ++k) {
        const int64_t q = a + k;
        by[k + 2] = q < e ? (uint8_t)(gidx[q] - gidx[q - 1]) : 0;
      }
      for (int q = 0; q < 8; ++q) w[q] = (uint16_t)(by[2 * q] | (by[2 * q + 1] << 8));
    }
    for (int q = 0; q < 8; ++q) B.idx.push_back(w[q]);
  };
  // compact: cuts the run [a, e) into groups
  auto cut_groups = [&](int64_t a, int64_t e) {
    int64_t q = a;
    while (q < e) {
      gstart.push_back(q);
      int n = 1;
      ++q;
      while (q < e && n < kCGroup && gidx[q] - gidx[q - 1] <= 255) {
        ++n;
        ++q;
      }
    }
  };

  // 1. entries of every panel
  std::vector<std::vector<Entry>> ent(B.npanels);
  {
    std::vector<int64_t> cur(off.begin(), off.end() - 1);
    for (int32_t k = 0; k < B.npanels; ++k) {
      const int64_t hi = (int64_t)(k + 1) * B.W;
      for (int64_t sgm = 0; sgm < out_dim; ++sgm) {
        const int64_t a = cur[sgm];
        int64_t e = a;
        const int64_t end = off[sgm + 1];
        while (e < end && gidx[e] < hi) ++e;
        if (e > a) {
          Entry en{a, e, (e - a + kPV - 1) / kPV, (int32_t)((int64_t)k * out_dim + sgm), 0};
          if (compact) {
            en.g0 = (int64_t)gstart.size();
            cut_groups(a, e);
            const int64_t gn = (int64_t)gstart.size() - en.g0;
            const int64_t gw = (e - a + kWGroup - 1) / kWGroup;
            if (gw < gn) {  // panel-local differences always fit 16 bits
              gstart.resize((size_t)en.g0);
              for (int64_t q = a; q < e; q += kWGroup) gstart.push_back(q);
              en.wide = true;
              en.g = gw;
            } else {
              en.g = gn;
            }
          }
          ent[k].push_back(en);
          cur[sgm] = e;
        }
      }
      B.nseg += (int64_t)ent[k].size();
    }
  }

  // 2. estimated windows per panel (packed entries as chunks of kPR windows;
  // narrow and wide entries packed apart)
  std::vector<detail::Packer> pk(B.npanels), pkw(B.npanels);
  std::vector<int64_t> pwin(B.npanels, 0);
  std::vector<std::array<int64_t, 2>> pwin_kind(B.npanels, {0, 0});  // packed: narrow, wide
  std::vector<int32_t> members;
  for (int32_t k = 0; k < B.npanels; ++k) {
    detail::Packer& P = pk[k];
    detail::Packer& Pw = pkw[k];
    P.ent = &ent[k];
    Pw.ent = &ent[k];
    for (int32_t i = 0; i < (int32_t)ent[k].size(); ++i) {
      const Entry& en = ent[k][i];
      if (en.g > packed_max) {
        if (compact) {
          for (int64_t o = 0; o < en.g; o += kPLongGroups)
            pwin[k] += (std::min<int64_t>(o + kPLongGroups, en.g) - o + 63) / 64 *
                       detail::window_cost(en.wide);
        } else {
          const int64_t len = en.e - en.a;
          for (int64_t o = 0; o < len; o += kPLongMax) {
            const int64_t ng = (std::min<int64_t>(o + kPLongMax, len) - o + kPV - 1) / kPV;
            pwin[k] += (ng + 63) / 64 * detail::window_cost(false);
          }
        }
      } else {
        (ent[k][i].wide ? Pw : P).order.push_back(i);
      }
    }
    for (detail::Packer* Q : {&P, &Pw}) {
      std::stable_sort(Q->order.begin(), Q->order.end(),
                       [&](int32_t x, int32_t y) { return ent[k][x].g > ent[k][y].g; });
      detail::Packer T = *Q;
      T.hi = T.order.size();
      while (!T.empty()) {
        T.take(kPR, members);
        int64_t last = 0;  // windows of the chunk: the longest lane's groups
        for (int32_t i : members)
          last = std::max<int64_t>(last, std::min<int64_t>(ent[k][i].g, kPR));
        const int64_t cost = last * detail::window_cost(Q == &Pw);
        pwin[k] += cost;
        pwin_kind[k][Q == &Pw ? 1 : 0] += cost;
      }
      Q->hi = Q->order.size();
    }
  }

  // 3. workgroups per panel, in proportion to its windows
  const int nwg_total = std::max<int>(ncu, B.npanels);
  const int64_t tot = std::max<int64_t>(std::accumulate(pwin.begin(), pwin.end(), (int64_t)0), 1);
  std::vector<int> g_k(B.npanels, 0);
  int assigned = 0;
  // (every panel gets at least one workgroup: its workgroups also own the
  // panel's entries of the gathered vector)
  for (int32_t k = 0; k < B.npanels; ++k) {
    g_k[k] = std::max(1, (int)((int64_t)nwg_total * pwin[k] / tot));
    assigned += g_k[k];
  }
  while (assigned < nwg_total) {
    int best = -1;
    double best_load = 0.0;
    for (int32_t k = 0; k < B.npanels; ++k) {
      if (pwin[k] == 0) continue;
      const double load = (double)pwin[k] / g_k[k];
      if (load > best_load) {
        best_load = load;
        best = k;
      }
    }
    if (best < 0) break;
    g_k[best]++;
    assigned++;
  }

  // 4. chunk lists, wavefront by wavefront
  std::vector<std::array<int32_t, 3>> splits;  // (output element, first piece, last piece)
  B.wave_c.push_back(0);
  for (int32_t k = 0; k < B.npanels; ++k) {
    if (g_k[k] == 0) continue;
    const int64_t glo = (int64_t)k * B.W;
    const int nwv = kPWaves * g_k[k];
    std::vector<std::vector<ChunkDesc>> lists(nwv);
    std::vector<int64_t> load(nwv, 0);
    // shares by rank (wave_weight): cumulative weights, and the wavefront
    // with the least load per unit of weight
    std::vector<double> cumw(nwv + 1, 0.0);
    for (int q = 0; q < nwv; ++q) cumw[q + 1] = cumw[q] + wave_weight(q);
    auto least_loaded = [&]() {
      int best = 0;
      for (int q = 1; q < nwv; ++q)
        if ((double)load[q] / wave_weight(q) < (double)load[best] / wave_weight(best)) best = q;
      return best;
    };
    // long entries: least loaded wavefront first
    for (const Entry& en : ent[k]) {
      if (en.g <= packed_max) continue;
      const int64_t len = compact ? en.g : en.e - en.a;  // groups or elements
      const int64_t step = compact ? kPLongGroups : kPLongMax;
      const bool pieces = len > step;
      if (!pieces) B.seg_out.push_back(en.slot);
      const int32_t p_first = B.npieces;
      for (int64_t o = 0; o < len; o += step) {
        const int64_t oe = std::min<int64_t>(o + step, len);
        ChunkDesc d{};
        d.base = (int64_t)B.idx.size();
        const int64_t ng = compact ? oe - o : (oe - o + kPV - 1) / kPV;
        d.vm[0] = (uint64_t)(ng * kPV);
        const int win = (int)((ng + 63) / 64);
        d.first = pieces ? B.npieces++ : (int32_t)B.seg_out.size() - 1;
        d.seg = en.slot % out_dim;
        d.info = chunk_info(win, pieces ? kChunkPiece : kChunkLong, 0, 0, 0, 1, en.wide);
        if (compact) {
          for (int64_t j = o; j < oe; ++j) append_cgroup(en, j, glo);
        } else {
          for (int64_t q = en.a + o; q < en.a + oe; q += kPV)
            append_group(q, std::min<int64_t>(q + kPV, en.a + oe), glo);
        }
        const int q = least_loaded();
        lists[q].push_back(d);
        load[q] += win * detail::window_cost(en.wide);
      }
      if (pieces) splits.push_back({(int32_t)(en.slot % out_dim), p_first, B.npieces - 1});
    }
    // packed entries: fill each wavefront to its share of the panel's
    // windows; the share starts from the estimate and is rebuilt from the
    // windows the first fill actually used when that fill ends unevenly.
    detail::Packer& P = pk[k];
    detail::Packer& Pw = pkw[k];
    const size_t idx0 = B.idx.size(), seg0 = B.seg_out.size();
    const std::vector<std::vector<ChunkDesc>> lists_long = lists;
    const std::vector<int64_t> load_long = load;
    // narrow and wide chunks interleaved in the proportion of their
    // estimated windows, so that every wavefront's share mixes them (wide
    // chunks hold up to 64 short segments, and their outputs, gathered
    // onto a few wavefronts, made those the pass's last)
    auto all_taken = [&]() { return P.empty() && Pw.empty(); };
    int64_t took[2] = {0, 0};
    auto next_packer = [&]() -> detail::Packer& {
      if (P.empty()) return Pw;
      if (Pw.empty()) return P;
      return took[1] * pwin_kind[k][0] <= took[0] * pwin_kind[k][1] ? Pw : P;
    };
    auto make_packed = [&](detail::Packer& Q, int R) {
      const bool wide = &Q == &Pw;
      Q.take(R, members);
      ChunkDesc d{};
      d.base = (int64_t)B.idx.size();
      d.first = (int32_t)B.seg_out.size();
      std::vector<int> l0s(members.size()), ws(members.size());
      int l = 0, maxw = 1, b15 = 0, b31 = 0;
      for (size_t s = 0; s < members.size(); ++s) {
        const int w = Q.lanes(members[s], R);
        l0s[s] = l;
        ws[s] = w;
        d.sm |= 1ull << l;
        maxw = std::max(maxw, w);
        if (detail::crosses(l, w, 15) || detail::crosses(l, w, 47)) b15 = 1;
        if (detail::crosses(l, w, 31)) b31 = 1;
        l += w;
        B.seg_out.push_back(ent[k][members[s]].slot);
      }
      if (l < 64) d.sm |= 1ull << l;  // idle tail slice
      // window-major stream: window kw holds, lane by lane, group
      // (lane - l0) * R + kw of the lane's entry when it exists
      int nw = 0;
      for (int kw = 0; kw < R; ++kw) {
        for (size_t s = 0; s < members.size(); ++s) {
          const Entry& en = ent[k][members[s]];
          for (int i = 0; i < ws[s]; ++i) {
            const int64_t j = (int64_t)i * R + kw;
            if (j >= en.g) continue;
            d.vm[kw] |= 1ull << (l0s[s] + i);
            if (compact) {
              append_cgroup(en, j, glo);
            } else {
              const int64_t q = en.a + j * kPV;
              append_group(q, std::min<int64_t>(q + kPV, en.e), glo);
            }
          }
        }
        if (d.vm[kw]) nw = kw + 1;
      }
      d.info = chunk_info(nw, kChunkPacked, detail::ceil_log2(std::min(maxw, 16)), b15, b31,
                          (int)members.size(), wide);
      return d;
    };
    int64_t total = pwin[k];
    for (int attempt = 0; attempt < 3; ++attempt) {
      lists = lists_long;
      load = load_long;
      B.idx.resize(idx0);
      B.seg_out.resize(seg0);
      P.lo = 0;
      P.hi = P.order.size();
      Pw.lo = 0;
      Pw.hi = Pw.order.size();
      took[0] = took[1] = 0;
      const double per_w = (double)total / cumw[nwv];
      for (int q = 0; q < nwv && !all_taken(); ++q) {
        const int64_t target =
            (int64_t)std::llround(per_w * cumw[q + 1]) - (int64_t)std::llround(per_w * cumw[q]);
        while (!all_taken() && load[q] < target) {
          detail::Packer& Q = next_packer();
          const int u = detail::window_cost(&Q == &Pw);
          int R = (int)std::min<int64_t>(kPR, (target - load[q] + u - 1) / u);
          R = std::max(R, Q.min_windows());
          const ChunkDesc d = make_packed(Q, R);
          lists[q].push_back(d);
          load[q] += detail::chunk_cost(d);
          took[&Q == &Pw ? 1 : 0] += detail::chunk_cost(d);
        }
      }
      bool leftover = false;
      while (!all_taken()) {  // what the share missed: least loaded wavefront
        leftover = true;
        const int q = least_loaded();
        detail::Packer& Q = next_packer();
        const ChunkDesc d = make_packed(Q, kPR);
        took[&Q == &Pw ? 1 : 0] += detail::chunk_cost(d);
        lists[q].push_back(d);
        load[q] += detail::chunk_cost(d);
      }
      const int64_t used = std::accumulate(load.begin(), load.end(), (int64_t)0);
      double excess = 0.0;  // most windows any wavefront has above its share
      for (int q = 0; q < nwv; ++q)
        excess = std::max(excess, (double)load[q] - (double)used * wave_weight(q) / cumw[nwv]);
      if (!leftover && excess <= 2.0 * detail::window_cost(false)) break;
      total = used;
    }
    const int64_t e0 = glo, e1 = std::min<int64_t>(glo + B.W, gdim);
    for (int g = 0; g < g_k[k]; ++g) {
      B.wg_panel.push_back(k);
      B.wg_s0.push_back((int32_t)(e0 + (e1 - e0) * g / g_k[k]));
      B.wg_s1.push_back((int32_t)(e0 + (e1 - e0) * (g + 1) / g_k[k]));
      for (int q = 0; q < kPWaves; ++q) {
        for (const ChunkDesc& d : lists[g * kPWaves + q]) B.chunks.push_back(d);
        B.wave_c.push_back((int32_t)B.chunks.size());
      }
    }
  }

  // 5. bank-spread order within the groups of every window (the compact
  // groups' order is their positions' order)
  if (!compact) {
    uint16_t* grp[64];
    int lanes[64];
    const uint16_t sentinel = (uint16_t)B.W;
    for (const ChunkDesc& d : B.chunks) {
      const int R = d.info & 0xff;
      if (((d.info >> 8) & 3) == kChunkPacked) {
        int64_t at = d.base;
        for (int kw = 0; kw < R; ++kw) {
          int ng = 0;
          for (int l = 0; l < 64; ++l)
            if ((d.vm[kw] >> l) & 1ull) {
              lanes[ng] = l;
              grp[ng++] = &B.idx[at];
              at += kPV;
            }
          detail::spread_window(grp, lanes, ng, elem, sentinel);
        }
      } else {
        const int64_t groups = (int64_t)d.vm[0] / kPV;
        for (int kw = 0; kw < R; ++kw) {
          int ng = 0;
          for (int l = 0; l < 64 && (int64_t)kw * 64 + l < groups; ++l) {
            lanes[ng] = l;
            grp[ng++] = &B.idx[d.base + ((int64_t)kw * 64 + l) * kPV];
          }
          detail::spread_window(grp, lanes, ng, elem, sentinel);
        }
      }
    }
  }

  // 6. each window's groups stored as halves: the first kPV / 2 entries of
  // every group in lane order, then the second halves (one 16-byte load per
  // lane then reads a contiguous block of the window); compact groups are
  // already one 16-byte block each
  if (!compact) {
    std::vector<uint16_t> tmp;
    auto split = [&](int64_t at, int ng) {
      tmp.assign(B.idx.begin() + at, B.idx.begin() + at + (int64_t)ng * kPV);
      const int h = kPV / 2;
      for (int g = 0; g < ng; ++g)
        for (int j = 0; j < h; ++j) {
          B.idx[at + (int64_t)g * h + j] = tmp[(size_t)g * kPV + j];
          B.idx[at + (int64_t)ng * h + (int64_t)g * h + j] = tmp[(size_t)g * kPV + h + j];
        }
    };
    for (const ChunkDesc& d : B.chunks) {
      const int R = d.info & 0xff;
      if (((d.info >> 8) & 3) == kChunkPacked) {
        int64_t at = d.base;
        for (int kw = 0; kw < R; ++kw) {
          const int ng = __builtin_popcountll(d.vm[kw]);
          split(at, ng);
          at += (int64_t)ng * kPV;
        }
      } else {
        const int64_t groups = (int64_t)d.vm[0] / kPV;
        for (int kw = 0; kw < R; ++kw)
          split(d.base + (int64_t)kw * kPC, (int)std::min<int64_t>(64, groups - (int64_t)kw * 64));
      }
    }
  }

  // pieces of the longest entries, grouped by output element
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
}

}  // namespace ppcg
