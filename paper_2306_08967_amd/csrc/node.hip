// node.hip -- node change (Sec. 4.2, Theorem 1; Algorithm 2, node branch).
//
// A node joins as one new column of A (its in-edges from the other nodes),
// then one new row (its out-edges, with its self-loop).  With a fixed node
// range the joining node is a slot whose row and column of A are empty, so
// the column step is the edge update of Theorem 2 with B the column's
// indicator and C = e_node (W_C = V_b[node] P_V is zero, which reduces the
// core to Theorem 1's [[Sigma, W_B], [0, R_B]]), and the row step is the same
// with B = e_node.  The event is a handful of entries, so its chunks and edit
// lists are built here on the host and uploaded into the batch workspace;
// graph edits, Steps 1-4 and the statistics then run as for a batch.  A side
// with more than r_max entries is cut into consecutive rank-1 pieces of at
// most r_max rows (the chunk kernels' row limit); the first piece is
// Theorem 1's step, later ones are Theorem 2 updates of the existing column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "damf_internal.h"

namespace damf {

namespace {

void sort_unique(std::vector<int32_t> &v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

// distinct leading keys of a sorted entry list and the start of each run
// (plus a sentinel), as the CSR edit and PPR fix-up kernels expect
void runs(const std::vector<NetEntry> &e, bool by_col, std::vector<int32_t> &keys,
          std::vector<int32_t> &pos) {
  keys.clear();
  pos.clear();
  for (size_t i = 0; i < e.size(); ++i) {
    const int32_t k = by_col ? e[i].col : e[i].row;
    if (keys.empty() || keys.back() != k) {
      keys.push_back(k);
      pos.push_back((int32_t)i);
    }
  }
  pos.push_back((int32_t)e.size());
}

bool meets(const int32_t *a, int na, const int32_t *b, int nb) {
  int i = 0, j = 0;
  while (i < na && j < nb) {
    if (a[i] == b[j]) return true;
    if (a[i] < b[j]) ++i; else ++j;
  }
  return false;
}

}  // namespace

damf_status node_prepare(damf_ctx *c, int32_t node, int64_t k_in, const int32_t *in_nbrs,
                         int64_t k_out, const int32_t *out_nbrs, BatchHeader *h) {
  *h = BatchHeader{};
  if (c->poisoned) return api_fail(c, DAMF_E_STATE, "context poisoned");
  if (k_in < 0 || k_out < 0 || (k_in > 0 && !in_nbrs) || (k_out > 0 && !out_nbrs))
    return api_fail(c, DAMF_E_INVALID_ARG, "bad neighbour lists");
  if (k_in + k_out > kMaxBatch) return api_fail(c, DAMF_E_INVALID_ARG, "node event too large");
  if (!c->cfg.directed && k_out != 0)
    return api_fail(c, DAMF_E_INVALID_ARG, "undirected graph: pass the neighbours as in_nbrs only");
  if (node < 0 || node >= c->n) return api_fail(c, DAMF_E_OUT_OF_RANGE, "node id out of range");
  for (int64_t i = 0; i < k_in; ++i)
    if (in_nbrs[i] < 0 || in_nbrs[i] >= c->n) return api_fail(c, DAMF_E_OUT_OF_RANGE, "neighbour id out of range");
  for (int64_t i = 0; i < k_out; ++i)
    if (out_nbrs[i] < 0 || out_nbrs[i] >= c->n) return api_fail(c, DAMF_E_OUT_OF_RANGE, "neighbour id out of range");
  // the column step takes the in-edges without a self-loop; the row step the
  // out-edges and the self-loop (the row spans the new column too)
  std::vector<int32_t> ins, outs;
  bool self = false;
  try {
    for (int64_t i = 0; i < k_in; ++i) {
      if (in_nbrs[i] == node) self = true;
      else ins.push_back(in_nbrs[i]);
    }
    if (c->cfg.directed) {
      for (int64_t i = 0; i < k_out; ++i) outs.push_back(out_nbrs[i]);
    } else {
      outs = ins;  // A[node, v] = A[v, node]
    }
    if (self) outs.push_back(node);
  } catch (...) {
    return api_fail(c, DAMF_E_OOM, "host memory");
  }
  sort_unique(ins);
  sort_unique(outs);
  // the node must not have edges yet
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  int32_t *lens = reinterpret_cast<int32_t *>(w.counters_host + 13);
  hipError_t e = hipMemcpyAsync(lens, c->out.len + node, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(lens + 1, c->in.len + node, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return api_dev_fail(c, e, "node degree");
  if (lens[0] != 0 || lens[1] != 0)
    return api_fail(c, DAMF_E_INVALID_ARG, "node change needs a node without edges (use damf_update)");
  if (ins.empty() && outs.empty()) return DAMF_OK;

  const int rmax = c->cfg.max_side;
  std::vector<ChunkDesc> chunks;
  std::vector<int32_t> s1l, s2l;
  std::vector<NetEntry> ent, net, nett;
  std::vector<int32_t> rows_out, pos_out, rows_in, pos_in;
  try {
    auto add_piece = [&](const int32_t *ids, int cnt, bool column) {
      ChunkDesc cd{};
      cd.s1_off = (int32_t)s1l.size();
      cd.s2_off = (int32_t)s2l.size();
      cd.e_off = (int32_t)ent.size();
      cd.ne = cnt;
      if (column) {  // S1 = the piece, S2 = {node}
        cd.s1 = cnt;
        cd.s2 = 1;
        s1l.insert(s1l.end(), ids, ids + cnt);
        s2l.push_back(node);
        for (int i = 0; i < cnt; ++i) ent.push_back(NetEntry{ids[i], node, 1, 0});
      } else {  // S1 = {node}, S2 = the piece
        cd.s1 = 1;
        cd.s2 = cnt;
        s1l.push_back(node);
        s2l.insert(s2l.end(), ids, ids + cnt);
        for (int i = 0; i < cnt; ++i) ent.push_back(NetEntry{node, ids[i], 1, 0});
      }
      chunks.push_back(cd);
    };
    for (size_t i = 0; i < ins.size(); i += rmax)
      add_piece(ins.data() + i, (int)std::min<size_t>(rmax, ins.size() - i), true);
    for (size_t i = 0; i < outs.size(); i += rmax)
      add_piece(outs.data() + i, (int)std::min<size_t>(rmax, outs.size() - i), false);
    net = ent;
    std::sort(net.begin(), net.end(), [](const NetEntry &a, const NetEntry &b) {
      return a.row != b.row ? a.row < b.row : a.col < b.col;
    });
    nett = ent;
    std::sort(nett.begin(), nett.end(), [](const NetEntry &a, const NetEntry &b) {
      return a.col != b.col ? a.col < b.col : a.row < b.row;
    });
    // the CSR edit kernels read pad as the number of inserts before the entry
    // in its sorted list (here every entry inserts)
    for (size_t i = 0; i < net.size(); ++i) net[i].pad = (int32_t)i;
    for (size_t i = 0; i < nett.size(); ++i) nett[i].pad = (int32_t)i;
    runs(net, false, rows_out, pos_out);
    runs(nett, true, rows_in, pos_in);
  } catch (...) {
    return api_fail(c, DAMF_E_OOM, "host memory");
  }
  BatchHeader hd{};
  hd.n_net = (int32_t)net.size();
  hd.n_chunks = (int32_t)chunks.size();
  hd.n_rows_out = (int32_t)rows_out.size();
  hd.n_rows_in = (int32_t)rows_in.size();
  hd.s1_total = (int32_t)s1l.size();
  hd.s2_total = (int32_t)s2l.size();
  for (const ChunkDesc &cd : chunks) hd.max_s = std::max(hd.max_s, std::max(cd.s1, cd.s2));
  for (int j = 1; j < hd.n_chunks; ++j) {
    const ChunkDesc &a = chunks[j], &b = chunks[j - 1];
    if (meets(s1l.data() + a.s1_off, a.s1, s1l.data() + b.s1_off, b.s1) ||
        meets(s2l.data() + a.s2_off, a.s2, s2l.data() + b.s2_off, b.s2))
      hd.meets_prev[j >> 6] |= 1ull << (j & 63);
  }
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  up(w.chunks, chunks.data(), chunks.size() * sizeof(ChunkDesc));
  up(w.chunk_s1, s1l.data(), s1l.size() * sizeof(int32_t));
  up(w.chunk_s2, s2l.data(), s2l.size() * sizeof(int32_t));
  up(w.chunk_ent, ent.data(), ent.size() * sizeof(NetEntry));
  up(w.net, net.data(), net.size() * sizeof(NetEntry));
  up(w.net_t, nett.data(), nett.size() * sizeof(NetEntry));
  up(w.rows_out, rows_out.data(), rows_out.size() * sizeof(int32_t));
  up(w.rowpos_out, pos_out.data(), pos_out.size() * sizeof(int32_t));
  up(w.rows_in, rows_in.data(), rows_in.size() * sizeof(int32_t));
  up(w.rowpos_in, pos_in.data(), pos_in.size() * sizeof(int32_t));
  *w.hdr_host = hd;
  up(w.hdr, w.hdr_host, sizeof(BatchHeader));
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return api_dev_fail(c, e, "node event upload");
  *h = hd;
  return DAMF_OK;
}

}  // namespace damf
