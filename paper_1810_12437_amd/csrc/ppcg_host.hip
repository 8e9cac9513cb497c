// Host-side construction shared by the matrix and batch handles: reading and
// validating a binary CSR, its CSC twin, and uploading panel tables.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "ppcg_handle.h"

namespace ppcg {

int upload_orient(DevBuf& mem, const PanelBuild& B, int elem, int K, Orient& o) {
  int rc;
  int64_t by = 0;
  PanelPass& t = o.pass;
  if (B.idx.size() >= (size_t)kPV) {
    if ((rc = upload_vec(mem, B.idx, &t.idx, &by))) return rc;
  } else {
    // at least one group: a wavefront without chunks reads group 0
    std::vector<uint16_t> ix(B.idx);
    ix.resize(kPV, (uint16_t)B.W);
    if ((rc = upload_vec(mem, ix, &t.idx, &by))) return rc;
  }
  if ((rc = upload_vec(mem, B.chunks, &t.chunks, &by))) return rc;
  {
    // A trailing -1 entry: the slot the index stream reads for lanes and
    // chunks that write no output.
    std::vector<int32_t> so(B.seg_out);
    so.push_back(-1);
    if ((rc = upload_vec(mem, so, &t.seg_out, &by))) return rc;
    t.no_slot = (int32_t)B.seg_out.size();
  }
  if ((rc = upload_vec(mem, B.wg_panel, &t.wg_panel, &by))) return rc;
  if ((rc = upload_vec(mem, B.wave_c, &t.wave_c, &by))) return rc;
  if ((rc = upload_vec(mem, B.wg_s0, &t.wg_s0, &by))) return rc;
  if ((rc = upload_vec(mem, B.wg_s1, &t.wg_s1, &by))) return rc;
  if (!B.sp_off.empty()) {
    if ((rc = upload_vec(mem, B.sp_off, &o.sp_off, &by))) return rc;
    if ((rc = upload_vec(mem, B.sp_c0, &o.sp_c0, &by))) return rc;
    if ((rc = upload_vec(mem, B.sp_c1, &o.sp_c1, &by))) return rc;
  }
  t.gdim = B.gdim;
  t.out_dim = B.out_dim;
  t.W = B.W;
  t.nwg = (int32_t)B.wg_panel.size();
  t.nchunks = (int32_t)B.chunks.size();
  t.npieces = B.npieces;
  o.npanels = B.npanels;
  o.out_dim = B.out_dim;
  const size_t part_bytes = (size_t)B.npanels * (size_t)B.out_dim * (size_t)elem * K;
  unsigned char* part = nullptr;
  unsigned char* piece = nullptr;
  PPCG_TRY_ALLOC(mem.alloc(&part, part_bytes));
  PPCG_TRY_ALLOC(mem.alloc(&piece, (size_t)std::max<int32_t>(t.npieces, 1) * elem * K));
  // (segment, panel) pairs with no elements are never written: they stay zero.
  PPCG_TRY_HIP(hipMemset(part, 0, std::max<size_t>(part_bytes, 1)));
  o.part = part;
  o.piece = piece;
  o.dev_bytes = by + (int64_t)part_bytes + (int64_t)t.npieces * elem * K;
  // Per launch: the padded index stream, the chunk descriptors, the output
  // slots, K sums per (segment, panel) pair, and the gathered vectors once
  // (their panel copies come from cache).
  o.pass_bytes = 2 * (int64_t)B.idx.size() + (int64_t)sizeof(ChunkDesc) * t.nchunks +
                 4 * (int64_t)B.seg_out.size() + (int64_t)elem * K * B.nseg +
                 (int64_t)elem * K * B.gdim;
  return PPCG_OK;
}

int read_binary_csr(int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                    const int32_t* col_idx, int32_t mem, hipStream_t stream,
                    std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                    std::vector<int64_t>& cp, std::vector<int32_t>& ri) {
  rp.assign(n + 1, 0);
  ci.assign(nnz, 0);
  if (mem == PPCG_MEM_HOST) {
    std::memcpy(rp.data(), row_ptr, (n + 1) * sizeof(int64_t));
    if (nnz) std::memcpy(ci.data(), col_idx, nnz * sizeof(int32_t));
  } else {
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd < 1) return PPCG_ENODEV;
    PPCG_TRY_HIP(hipMemcpyAsync(rp.data(), row_ptr, (n + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToHost, stream));
    if (nnz)
      PPCG_TRY_HIP(hipMemcpyAsync(ci.data(), col_idx, nnz * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, stream));
    PPCG_TRY_HIP(hipStreamSynchronize(stream));
  }
  // Validate CSR: offsets monotone from 0 to nnz; columns in range and
  // strictly increasing within a row (binary X has no duplicates).
  if (rp[0] != 0 || rp[n] != nnz) return PPCG_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return PPCG_EINVAL;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t c = ci[k];
      if (c < 0 || c >= p) return PPCG_EINVAL;
      if (k > rp[i] && c <= ci[k - 1]) return PPCG_EINVAL;
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return PPCG_ENODEV;
  // CSC twin by a counting sort over columns (rows stay increasing).
  cp.assign(p + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) cp[ci[k] + 1]++;
  for (int64_t j = 0; j < p; ++j) cp[j + 1] += cp[j];
  ri.assign(nnz, 0);
  std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) ri[fill[ci[k]]++] = (int32_t)i;
  return PPCG_OK;
}

}  // namespace ppcg
