// Host-side check of the panel-blocked layout of the X passes (a test
// program, built by tests/test_layout_cpu.py with AddressSanitizer and
// UndefinedBehaviorSanitizer).
//
// For a binary X read from a file it builds the tables of both orientations
// at both value sizes (compact groups, as the library's one-vector tables)
// and at the K-interleaved entry sizes of shared-design batches (16-bit
// indices as halves) exactly as the library does (build_panels), then runs
// a lane-by-lane model of the pass kernel's reads over them: every
// workgroup's panel, every wavefront's chunk list, the loads each lane
// issues for every window (the stand-in loads of lanes without a group and
// of steps past the wavefront's last window included), the segmented lane
// sums of packed chunks with the kernel's own shift and broadcast steps, the
// whole-wavefront sums of long chunks and pieces, and the consumer's total
// over panels and pieces.  With integer values every sum is exact, so the
// model's X v and X^T w must equal the products computed directly from the
// index arrays, element by element.  Every read of a table is checked
// against the table's uploaded length.
//
// Usage: layout_check <file>  (int64 n, p, nnz; int64 row_ptr[n + 1];
// int32 col_idx[nnz]).  Prints one JSON line; exit status 0 when every
// check holds.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <climits>
#include <memory>
#include <string>
#include <vector>

#include "ppcg_panels.h"

using namespace ppcg;

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                        \
  do {                                                          \
    if (!(cond)) {                                              \
      if (g_fail < 20) {                                        \
        fprintf(stderr, "check failed: %s: ", #cond);           \
        fprintf(stderr, __VA_ARGS__);                           \
        fprintf(stderr, "\n");                                  \
      }                                                         \
      ++g_fail;                                                 \
    }                                                           \
  } while (0)

// A table as the device holds it: exactly `n` entries on the heap, so that a
// read past the end is a sanitizer report as well as a failed check.
template <typename V>
struct Table {
  std::unique_ptr<V[]> a;
  int64_t n = 0;
  explicit Table(const std::vector<V>& v, int64_t min_len = 0, V fill = V()) {
    n = std::max<int64_t>((int64_t)v.size(), min_len);
    a.reset(new V[n > 0 ? n : 1]);
    for (int64_t i = 0; i < n; ++i) a[i] = i < (int64_t)v.size() ? v[i] : fill;
  }
  V at(int64_t i, const char* what) const {
    CHECK(i >= 0 && i < n, "%s index %lld of %lld", what, (long long)i, (long long)n);
    return (i >= 0 && i < n) ? a[i] : V();
  }
};

int popc(uint64_t m) { return __builtin_popcountll(m); }
int below(uint64_t m, int lane) {
  return lane == 0 ? 0 : popc(m & ((lane == 64) ? ~0ull : ((1ull << lane) - 1ull)));
}

// The pass kernel's segmented inclusive scan over the lanes (slices start
// at the set bits of sm): row-local shifts by 1, 2, 4, 8 (the first nrow of
// them), each taken only from lanes of the same slice, then the broadcasts
// of lane 15 (to rows 1 and 3, from lanes 15 and 47) and of lane 31 (to rows
// 2 and 3).  A lane reads its source's value from before the step; a source
// outside the lane's row gives zero.
void scan(int64_t (&acc)[64], uint64_t sm, int nrow, int b15, int b31) {
  CHECK((sm & 1ull) != 0, "lane 0 starts no slice");
  int off[64];
  for (int l = 0; l < 64; ++l) {
    int s = l;
    while (s > 0 && !((sm >> s) & 1ull)) --s;
    off[l] = l - s;
  }
  auto step = [&](auto src_of, auto cond_of) {
    int64_t mv[64];
    for (int l = 0; l < 64; ++l) {
      const int s = src_of(l);
      mv[l] = s >= 0 ? acc[s] : 0;
    }
    for (int l = 0; l < 64; ++l)
      if (cond_of(l)) acc[l] += mv[l];
  };
  for (int t = 0; t < 4 && t < nrow; ++t) {
    const int sh = 1 << t;
    step([&](int l) { return (l & 15) >= sh ? l - sh : -1; },
         [&](int l) { return off[l] >= sh; });
  }
  if (b15)
    step([&](int l) { return (l >> 4) == 1 ? 15 : (l >> 4) == 3 ? 47 : -1; },
         [&](int l) { return off[l] > (l & 15); });
  if (b31)
    step([&](int l) { return l >= 32 ? 31 : -1; }, [&](int l) { return off[l] >= l - 31; });
}

struct Stats {
  int64_t packed = 0, longc = 0, piece = 0, segs = 0, pieces = 0, nwg = 0, panels = 0;
  int64_t cgroups = 0;  // compact groups decoded
  int64_t wgroups = 0;  // of which wide
};

// The model of one orientation: gathered vector x (gdim), outputs out_dim.
// Returns the consumer's totals.
std::vector<int64_t> run_pass(const PanelBuild& B, const std::vector<int64_t>& x, Stats& st,
                              bool compact) {
  const int64_t out_dim = B.out_dim;
  // device tables (as uploaded: the index stream at least kPV long, a
  // trailing -1 output slot)
  Table<uint16_t> idx(B.idx, kPV, (uint16_t)B.W);
  Table<ChunkDesc> chunks(B.chunks);
  std::vector<int32_t> so(B.seg_out);
  so.push_back(-1);
  Table<int32_t> seg_out(so);
  const int32_t no_slot = (int32_t)B.seg_out.size();
  Table<int32_t> wg_panel(B.wg_panel), wave_c(B.wave_c), wg_s0(B.wg_s0), wg_s1(B.wg_s1);
  const int nwg = (int)B.wg_panel.size();
  CHECK((int64_t)B.wave_c.size() == (int64_t)kPWaves * nwg + 1, "wave_c size");
  std::vector<int64_t> part((size_t)B.npanels * out_dim, 0);
  std::vector<int> part_writes((size_t)B.npanels * out_dim, 0);
  std::vector<int64_t> piece((size_t)std::max(B.npieces, 1), 0);
  std::vector<int> piece_writes((size_t)std::max(B.npieces, 1), 0);
  std::vector<int> owned((size_t)B.gdim, 0);
  st.nwg += nwg;
  st.panels += B.npanels;
  st.pieces += B.npieces;
  st.segs += B.nseg;

  for (int w = 0; w < nwg; ++w) {
    const int panel = wg_panel.at(w, "wg_panel");
    CHECK(panel >= 0 && panel < B.npanels, "panel %d", panel);
    const int64_t g0 = (int64_t)panel * B.W;
    const int64_t wlen = std::min<int64_t>(B.W, B.gdim - g0);
    // the panel in LDS, entry W zero
    std::vector<int64_t> xl((size_t)B.W + 1, 0);
    for (int64_t j = 0; j < wlen; ++j) xl[j] = x[g0 + j];
    // one compact group read by a lane at word ea: first index, pad count,
    // differences; the sum of its entries less the pads' copies of the last
    auto cgroup = [&](int64_t ea, bool wide) {
      ++st.cgroups;
      if (wide) {
        // wide: first index, pad count (byte 3 zero), six 16-bit differences
        ++st.wgroups;
        uint16_t wv[8];
        for (int e = 0; e < 8; ++e) wv[e] = idx.at(ea + e, "idx");
        const int pads = wv[1] & 0xff;
        CHECK((wv[1] >> 8) == 0, "wide group byte 3 is %d", wv[1] >> 8);
        CHECK(pads < kWGroup, "wide pad count %d", pads);
        int64_t ix = wv[0], sum = 0;
        for (int e = 0; e < kWGroup; ++e) {
          if (e > 0) ix += wv[e + 1];
          CHECK(ix >= 0 && ix < wlen, "index %lld outside the panel's %lld values",
                (long long)ix, (long long)wlen);
          CHECK(e < kWGroup - pads || wv[e + 1] == 0 || e == 0, "pad %d moves the index", e);
          sum += (ix >= 0 && ix <= B.W) ? xl[ix] : 0;
        }
        sum -= (int64_t)pads * ((ix >= 0 && ix <= B.W) ? xl[ix] : 0);
        return sum;
      }
      uint8_t by[16];
      for (int e = 0; e < 8; ++e) {
        const uint16_t wv = idx.at(ea + e, "idx");
        by[2 * e] = (uint8_t)(wv & 0xff);
        by[2 * e + 1] = (uint8_t)(wv >> 8);
      }
      const int pads = by[2];
      CHECK(pads < kCGroup, "pad count %d", pads);
      int64_t ix = by[0] | (by[1] << 8), sum = 0;
      for (int e = 0; e < kCGroup; ++e) {
        if (e > 0) ix += by[e + 2];
        CHECK(ix >= 0 && ix < wlen, "index %lld outside the panel's %lld values", (long long)ix,
              (long long)wlen);
        CHECK(e < kCGroup - pads || by[e + 2] == 0 || e == 0, "pad %d moves the index", e);
        sum += (ix >= 0 && ix <= B.W) ? xl[ix] : 0;
      }
      sum -= (int64_t)pads * ((ix >= 0 && ix <= B.W) ? xl[ix] : 0);
      return sum;
    };
    // ownership of the panel's entries (the direction update's slices)
    const int64_t o0 = wg_s0.at(w, "wg_s0"), o1 = wg_s1.at(w, "wg_s1");
    CHECK(o0 >= g0 && o1 <= g0 + wlen && o0 <= o1, "slice [%lld, %lld) of panel %d",
          (long long)o0, (long long)o1, panel);
    for (int64_t j = o0; j < o1 && j >= 0 && j < B.gdim; ++j) owned[j]++;
    for (int q = 0; q < kPWaves; ++q) {
      const int c0 = wave_c.at((int64_t)kPWaves * w + q, "wave_c");
      const int c1 = wave_c.at((int64_t)kPWaves * w + q + 1, "wave_c");
      CHECK(c0 <= c1, "wave chunk range");
      int64_t last_base = 0;  // the stand-in address of steps past the end
      for (int c = c0; c < c1; ++c) {
        const ChunkDesc D = chunks.at(c, "chunks");
        const int R = D.info & 0xff, kind = (D.info >> 8) & 3;
        const bool wide = (D.info & kChunkWide) != 0;
        CHECK(compact || !wide, "wide groups in a K-interleaved table");
        last_base = D.base;
        CHECK(R >= 1 && R <= kPLongWin, "windows %d", R);
        int64_t acc[64] = {};
        int32_t sidx[64];
        if (kind == kChunkPacked) {
          ++st.packed;
          CHECK(R <= kPR, "packed windows %d", R);
          const int nseg = D.info >> 24;
          for (int l = 0; l < 64; ++l) {
            const bool last = l == 63 || ((D.sm >> (l + 1)) & 1ull);
            const int si = below(D.sm, l + 1) - 1;
            sidx[l] = (last && si < nseg) ? D.first + si : no_slot;
          }
          int64_t pre = 0;
          for (int k = 0; k < R; ++k) {
            const uint64_t m = D.vm[k];
            const int ng = popc(m);
            CHECK(ng > 0, "empty window %d of a packed chunk", k);
            if (compact) {
              const int64_t w0 = D.base + pre * (kPV / 2);
              for (int l = 0; l < 64; ++l) {
                const bool h = (m >> l) & 1ull;
                const int64_t ea = h ? w0 + (int64_t)below(m, l) * (kPV / 2) : w0;
                const int64_t v = cgroup(ea, wide);
                if (h) acc[l] += v;
              }
              pre += ng;
              continue;
            }
            const int64_t w0 = D.base + pre * kPV;
            for (int l = 0; l < 64; ++l) {
              const bool h = (m >> l) & 1ull;
              const int r = below(m, l);
              const int64_t ea = h ? w0 + (int64_t)r * (kPV / 2) : w0;
              const int64_t eb = h ? w0 + (int64_t)(ng + r) * (kPV / 2) : w0;
              for (int e = 0; e < kPV / 2; ++e) {
                const uint16_t ia = idx.at(ea + e, "idx"), ib = idx.at(eb + e, "idx");
                if (h) {
                  CHECK(ia <= B.W && ib <= B.W, "index %d %d beyond W %d", ia, ib, B.W);
                  acc[l] += xl[std::min<int>(ia, B.W)] + xl[std::min<int>(ib, B.W)];
                }
              }
            }
            pre += ng;
          }
          scan(acc, D.sm, (D.info >> 12) & 7, (D.info >> 16) & 1, (D.info >> 17) & 1);
          // each slice's sum, written by its last lane
          for (int l = 0; l < 64; ++l) {
            const int32_t slot = seg_out.at(sidx[l], "seg_out");
            if (slot >= 0) {
              CHECK(slot / out_dim == panel, "slot %d outside panel %d", slot, panel);
              part[slot] = acc[l];
              part_writes[slot]++;
            }
          }
        } else {
          CHECK(kind == kChunkLong || kind == kChunkPiece, "chunk kind %d", kind);
          if (kind == kChunkLong) ++st.longc; else ++st.piece;
          const int64_t clen = (int64_t)D.vm[0];
          CHECK(clen % kPV == 0 && clen > 0 && clen <= kPLongMax, "long length %lld",
                (long long)clen);
          CHECK(R == (int)((clen / kPV + 63) / 64), "long windows");
          for (int k = 0; k < R; ++k) {
            const int64_t left = (clen - (int64_t)k * kPC) / kPV;
            const int ng = left < 64 ? (int)left : 64;
            if (compact) {
              const int64_t w0 = D.base + (int64_t)k * 64 * (kPV / 2);
              for (int l = 0; l < 64; ++l) {
                const bool h = l < ng;
                const int64_t v = cgroup(h ? w0 + (int64_t)l * (kPV / 2) : w0, wide);
                if (h) acc[l] += v;
              }
              continue;
            }
            const int64_t w0 = D.base + (int64_t)k * kPC;
            for (int l = 0; l < 64; ++l) {
              const bool h = l < ng;
              const int64_t ea = h ? w0 + (int64_t)l * (kPV / 2) : w0;
              const int64_t eb = h ? w0 + (int64_t)(ng + l) * (kPV / 2) : w0;
              for (int e = 0; e < kPV / 2; ++e) {
                const uint16_t ia = idx.at(ea + e, "idx"), ib = idx.at(eb + e, "idx");
                if (h) {
                  CHECK(ia <= B.W && ib <= B.W, "index beyond W");
                  acc[l] += xl[std::min<int>(ia, B.W)] + xl[std::min<int>(ib, B.W)];
                }
              }
            }
          }
          // one slice over the whole wavefront, the sum at lane 63
          scan(acc, 1ull, 4, 1, 1);
          const int64_t tot = acc[63];
          if (kind == kChunkLong) {
            const int32_t slot = seg_out.at(D.first, "seg_out");
            CHECK(slot >= 0 && slot / out_dim == panel, "long slot %d", slot);
            if (slot >= 0) {
              part[slot] = tot;
              part_writes[slot]++;
            }
          } else {
            CHECK(D.first >= 0 && D.first < B.npieces, "piece id %d", D.first);
            CHECK(D.seg >= 0 && D.seg < out_dim, "piece segment");
            if (D.first >= 0 && D.first < B.npieces) {
              piece[D.first] = tot;
              piece_writes[D.first]++;
            }
          }
        }
        // every step's output-slot load of the chunk's first window
      }
      // the ring's loads past the wavefront's last window read 16 bytes at
      // the last chunk's base (0 with no chunk)
      for (int e = 0; e < kPV / 2; ++e) (void)idx.at(last_base + e, "idx past end");
    }
  }
  for (int64_t j = 0; j < B.gdim; ++j) CHECK(owned[j] == 1, "entry %lld owned %d times",
                                             (long long)j, owned[j]);
  for (size_t s = 0; s < part_writes.size(); ++s)
    CHECK(part_writes[s] <= 1, "slot %zu written %d times", s, part_writes[s]);
  for (int i = 0; i < B.npieces; ++i) CHECK(piece_writes[i] == 1, "piece %d written %d times", i,
                                            piece_writes[i]);
  // the consumer: panels in order, then the pieces of each element
  std::vector<int64_t> out((size_t)out_dim, 0);
  const bool have_sp = !B.sp_off.empty();
  Table<int32_t> sp_off(B.sp_off), sp_c0(B.sp_c0), sp_c1(B.sp_c1);
  for (int64_t i = 0; i < out_dim; ++i) {
    int64_t v = 0;
    for (int k = 0; k < B.npanels; ++k) v += part[(size_t)k * out_dim + i];
    if (have_sp) {
      const int q1 = sp_off.at(i + 1, "sp_off");
      for (int q = sp_off.at(i, "sp_off"); q < q1; ++q) {
        const int c1 = sp_c1.at(q, "sp_c1");
        for (int cc = sp_c0.at(q, "sp_c0"); cc <= c1; ++cc) {
          CHECK(cc >= 0 && cc < B.npieces, "piece %d", cc);
          if (cc >= 0 && cc < B.npieces) v += piece[cc];
        }
      }
    }
    out[i] = v;
  }
  return out;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: layout_check <file>\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) {
    perror("open");
    return 2;
  }
  int64_t hdr[3];
  if (fread(hdr, sizeof(int64_t), 3, f) != 3) return 2;
  const int64_t n = hdr[0], p = hdr[1], nnz = hdr[2];
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> ci(nnz);
  if (fread(rp.data(), sizeof(int64_t), n + 1, f) != (size_t)(n + 1)) return 2;
  if (nnz && fread(ci.data(), sizeof(int32_t), nnz, f) != (size_t)nnz) return 2;
  fclose(f);
  // column orientation by a counting sort
  std::vector<int64_t> cp(p + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) cp[ci[k] + 1]++;
  for (int64_t j = 0; j < p; ++j) cp[j + 1] += cp[j];
  std::vector<int32_t> ri(nnz);
  {
    std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k) ri[fill[ci[k]]++] = (int32_t)i;
  }
  // integer vectors: every sum is exact in any order
  std::vector<int64_t> v(p), u(n);
  for (int64_t j = 0; j < p; ++j) v[j] = (int64_t)((j * 2654435761ull) % 2001ull) - 1000;
  for (int64_t i = 0; i < n; ++i) u[i] = (int64_t)((i * 40503ull + 7) % 4001ull) - 2000;
  std::vector<int64_t> xv(n, 0), xtu(p, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      xv[i] += v[ci[k]];
      xtu[ci[k]] += u[i];
    }
  Stats st;
  int64_t bad = 0;
  // 8 and 4: one FP64 or FP32 vector; 16 and 32: the K-interleaved tables of
  // shared-design batches (K x value size per panel entry, K = 2 or 4); 64
  // checks the builder beyond the widths the library uses
  for (int elem : {8, 4, 16, 32, 64}) {
    PanelBuild Br, Bc;
    // compact groups in the one-vector tables, as the library builds them
    const bool compact = elem <= 8;
    build_panels(rp, ci, n, p, elem, 256, Br, compact);
    build_panels(cp, ri, p, n, elem, 256, Bc, compact);
    const std::vector<int64_t> a = run_pass(Br, v, st, compact);
    const std::vector<int64_t> b = run_pass(Bc, u, st, compact);
    for (int64_t i = 0; i < n; ++i)
      if (a[i] != xv[i]) {
        if (bad < 10)
          fprintf(stderr, "elem %d: (X v)[%lld] = %lld, want %lld\n", elem, (long long)i,
                  (long long)a[i], (long long)xv[i]);
        ++bad;
      }
    for (int64_t j = 0; j < p; ++j)
      if (b[j] != xtu[j]) {
        if (bad < 10)
          fprintf(stderr, "elem %d: (X^T u)[%lld] = %lld, want %lld\n", elem, (long long)j,
                  (long long)b[j], (long long)xtu[j]);
        ++bad;
      }
  }
  printf("{\"n\": %lld, \"p\": %lld, \"nnz\": %lld, \"packed\": %lld, \"long\": %lld, "
         "\"piece_chunks\": %lld, \"pieces\": %lld, \"segments\": %lld, \"workgroups\": %lld, "
         "\"panels\": %lld, \"compact_groups\": %lld, \"wide_groups\": %lld, "
         "\"mismatches\": %lld, \"failed_checks\": %d}\n",
         (long long)n, (long long)p, (long long)nnz, (long long)st.packed, (long long)st.longc,
         (long long)st.piece, (long long)st.pieces, (long long)st.segs, (long long)st.nwg,
         (long long)st.panels, (long long)st.cgroups, (long long)st.wgroups, (long long)bad,
         g_fail);
  return (bad == 0 && g_fail == 0) ? 0 : 1;
}
