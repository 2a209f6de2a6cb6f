// Host plan of the pose-graph solver: nested-dissection ordering of the free
// poses, symbolic block Cholesky, level schedule of the elimination tree, and
// the gather lists the kernels use (no atomics anywhere).
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "pgo_plan.hpp"

namespace ba {

namespace {

// Nested dissection over the nodes in `nodes` (indices into adj): each
// connected part is split by the middle level of a breadth-first search from
// a far node; parts of at most `leaf` nodes are emitted as they are.
void dissect(const std::vector<std::vector<int>>& adj, std::vector<int> nodes, std::vector<int>& in_set,
             int tag, int& next_tag, std::vector<int>& order, int leaf) {
  if ((int)nodes.size() <= leaf) {
    for (int v : nodes) order.push_back(v);
    return;
  }
  // split into connected parts
  std::vector<std::vector<int>> parts;
  {
    for (int s : nodes) {
      if (in_set[s] != tag) continue;
      const int ptag = next_tag++;
      std::vector<int> part{s};
      in_set[s] = ptag;
      for (size_t q = 0; q < part.size(); ++q)
        for (int u : adj[part[q]])
          if (in_set[u] == tag) {
            in_set[u] = ptag;
            part.push_back(u);
          }
      parts.push_back(part);
    }
  }
  if (parts.size() > 1) {
    for (auto& part : parts) {
      const int t = in_set[part[0]];
      dissect(adj, part, in_set, t, next_tag, order, leaf);
    }
    return;
  }
  const std::vector<int>& part = parts[0];
  const int ptag = in_set[part[0]];
  // breadth-first levels from a far node (two sweeps)
  auto bfs = [&](int root, std::vector<std::vector<int>>& lv) {
    lv.clear();
    const int vtag = next_tag++;
    std::vector<int> cur{root};
    std::vector<int> mark_back;
    in_set[root] = vtag;
    mark_back.push_back(root);
    while (!cur.empty()) {
      lv.push_back(cur);
      std::vector<int> nxt;
      for (int v : cur)
        for (int u : adj[v])
          if (in_set[u] == ptag) {
            in_set[u] = vtag;
            mark_back.push_back(u);
            nxt.push_back(u);
          }
      cur.swap(nxt);
    }
    for (int v : mark_back) in_set[v] = ptag;
  };
  std::vector<std::vector<int>> lv;
  bfs(part[0], lv);
  bfs(lv.back()[0], lv);
  if (lv.size() < 3) {
    for (int v : part) order.push_back(v);
    return;
  }
  // separator: the smallest level among the middle third
  size_t best = lv.size() / 2;
  for (size_t k = lv.size() / 3; k <= 2 * lv.size() / 3 && k + 1 < lv.size(); ++k)
    if (k >= 1 && lv[k].size() < lv[best].size()) best = k;
  std::vector<int> a, b;
  for (size_t k = 0; k < lv.size(); ++k) {
    if (k == best) continue;
    for (int v : lv[k]) (k < best ? a : b).push_back(v);
  }
  const int ta = next_tag++, tb = next_tag++;
  for (int v : a) in_set[v] = ta;
  for (int v : b) in_set[v] = tb;
  for (int v : lv[best]) in_set[v] = -1;
  dissect(adj, a, in_set, ta, next_tag, order, leaf);
  dissect(adj, b, in_set, tb, next_tag, order, leaf);
  for (int v : lv[best]) order.push_back(v);
}

// Symbolic factorisation for elimination order `order` (order[p] = node):
// struct[p] = sorted positions of the off-diagonal rows of column p, and the
// parent of p in the elimination tree (-1 for a root).
void symbolic(const std::vector<std::vector<int>>& adj, const std::vector<int>& order,
              std::vector<std::vector<int>>& st, std::vector<int>& parent) {
  const int n = (int)order.size();
  std::vector<int> pos(n);
  for (int p = 0; p < n; ++p) pos[order[p]] = p;
  std::vector<std::set<int>> pending(n);
  st.assign(n, {});
  parent.assign(n, -1);
  for (int p = 0; p < n; ++p) {
    std::set<int> s = std::move(pending[p]);
    for (int u : adj[order[p]])
      if (pos[u] > p) s.insert(pos[u]);
    st[p].assign(s.begin(), s.end());
    if (!s.empty()) {
      const int q = *s.begin();
      parent[p] = q;
      for (int r : s)
        if (r != q) pending[q].insert(r);
    }
  }
}

}  // namespace

std::string build_pgo_plan(int32_t n_poses, int32_t n_edges, const int32_t* edge_i,
                           const int32_t* edge_j, const uint8_t* pose_fixed, PgoPlan& P) {
  if (n_poses < 1) return "n_poses < 1";
  if (n_edges < 0) return "negative edge count";
  if (n_edges > 0 && (!edge_i || !edge_j)) return "edge arrays are NULL";
  P = PgoPlan();
  P.n_poses = n_poses;
  P.n_edges = n_edges;
  std::vector<char> fixed(n_poses, 0);
  if (pose_fixed) {
    for (int i = 0; i < n_poses; ++i) fixed[i] = pose_fixed[i] != 0;
  } else {
    fixed[0] = 1;
  }
  for (int e = 0; e < n_edges; ++e) {
    if (edge_i[e] < 0 || edge_i[e] >= n_poses || edge_j[e] < 0 || edge_j[e] >= n_poses)
      return "edge " + std::to_string(e) + ": pose index out of range";
    if (edge_i[e] == edge_j[e]) return "edge " + std::to_string(e) + " joins a pose to itself";
  }
  P.edge_i.assign(edge_i, edge_i + n_edges);
  P.edge_j.assign(edge_j, edge_j + n_edges);
  // free nodes and their adjacency
  std::vector<int> node_of_pose(n_poses, -1), pose_of_node;
  for (int i = 0; i < n_poses; ++i)
    if (!fixed[i]) {
      node_of_pose[i] = (int)pose_of_node.size();
      pose_of_node.push_back(i);
    }
  const int nf = (int)pose_of_node.size();
  P.n_free = nf;
  if (nf > (1 << 24)) return "too many free poses";
  std::vector<std::vector<int>> adj(nf);
  for (int e = 0; e < n_edges; ++e) {
    const int a = node_of_pose[edge_i[e]], b = node_of_pose[edge_j[e]];
    if (a >= 0 && b >= 0) {
      adj[a].push_back(b);
      adj[b].push_back(a);
    }
  }
  for (auto& l : adj) {
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
  // nested dissection, then the elimination tree and its levels
  std::vector<int> order;
  {
    std::vector<int> all(nf);
    std::iota(all.begin(), all.end(), 0);
    std::vector<int> in_set(nf, 1);
    int next_tag = 2;
    dissect(adj, all, in_set, 1, next_tag, order, 2);
  }
  std::vector<std::vector<int>> st;
  std::vector<int> parent;
  symbolic(adj, order, st, parent);
  std::vector<int> level(nf, 0);
  for (int p = 0; p < nf; ++p)
    if (parent[p] >= 0) level[parent[p]] = std::max(level[parent[p]], level[p] + 1);
  // renumber columns by (level, position): children stay before parents, so
  // the factor's pattern is unchanged; recompute it in the new numbering
  std::vector<int> perm(nf);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return level[x] < level[y]; });
  std::vector<int> order2(nf);
  for (int c = 0; c < nf; ++c) order2[c] = order[perm[c]];
  symbolic(adj, order2, st, parent);
  std::vector<int> lev2(nf, 0);
  for (int c = 0; c < nf; ++c)
    if (parent[c] >= 0) lev2[parent[c]] = std::max(lev2[parent[c]], lev2[c] + 1);
  for (int c = 1; c < nf; ++c)
    if (lev2[c] < lev2[c - 1]) return "internal: level order broken";
  P.n_levels = nf ? lev2[nf - 1] + 1 : 0;
  P.lev_ptr.assign(P.n_levels + 1, 0);
  for (int c = 0; c < nf; ++c) P.lev_ptr[lev2[c] + 1] = c + 1;
  for (int l = 1; l <= P.n_levels; ++l) P.lev_ptr[l] = std::max(P.lev_ptr[l], P.lev_ptr[l - 1]);
  P.col_of_pose.assign(n_poses, -1);
  P.pose_of_col.resize(nf);
  for (int c = 0; c < nf; ++c) {
    P.pose_of_col[c] = pose_of_node[order2[c]];
    P.col_of_pose[P.pose_of_col[c]] = c;
  }
  // blocks
  P.blk_ptr.assign(nf + 1, 0);
  for (int c = 0; c < nf; ++c) P.blk_ptr[c + 1] = P.blk_ptr[c] + 1 + (int)st[c].size();
  P.blk_row.resize(P.blk_ptr[nf]);
  for (int c = 0; c < nf; ++c) {
    P.blk_row[P.blk_ptr[c]] = c;
    for (size_t k = 0; k < st[c].size(); ++k) P.blk_row[P.blk_ptr[c] + 1 + k] = st[c][k];
  }
  auto blk = [&](int r, int c) {   // block (r, c), r >= c, of the pattern
    if (r == c) return P.blk_ptr[c];
    const auto b = P.blk_row.begin() + P.blk_ptr[c] + 1, e = P.blk_row.begin() + P.blk_ptr[c + 1];
    const auto it = std::lower_bound(b, e, r);
    return (it != e && *it == r) ? (int)(it - P.blk_row.begin()) : -1;
  };
  const int nb = P.blk_ptr[nf];
  // updates into (r, c) from every column k with r, c in struct(k)
  std::vector<std::vector<std::pair<int, int>>> upd(nb);
  std::vector<std::vector<std::pair<int, int>>> fwd(nf);
  for (int k = 0; k < nf; ++k) {
    const auto& s = st[k];
    for (size_t q = 0; q < s.size(); ++q) {
      const int c = s[q];
      const int bck = P.blk_ptr[k] + 1 + (int)q;
      fwd[c].push_back({bck, k});
      for (size_t p = q; p < s.size(); ++p) {
        const int r = s[p];
        const int t = blk(r, c);
        if (t < 0) return "internal: fill block missing";
        upd[t].push_back({P.blk_ptr[k] + 1 + (int)p, bck});
      }
    }
  }
  P.upd_ptr.assign(nb + 1, 0);
  for (int t = 0; t < nb; ++t) P.upd_ptr[t + 1] = P.upd_ptr[t] + (int)upd[t].size();
  for (int t = 0; t < nb; ++t)
    for (auto& pr : upd[t]) {
      P.upd_a.push_back(pr.first);
      P.upd_b.push_back(pr.second);
    }
  P.fwd_ptr.assign(nf + 1, 0);
  for (int c = 0; c < nf; ++c) P.fwd_ptr[c + 1] = P.fwd_ptr[c] + (int)fwd[c].size();
  for (int c = 0; c < nf; ++c)
    for (auto& pr : fwd[c]) {
      P.fwd_blk.push_back(pr.first);
      P.fwd_col.push_back(pr.second);
    }
  // edge terms: + w B^T B into both diagonal blocks, - w B^T B into the
  // off-diagonal one; RHS -g: + w B^T r at the i end, - w B^T r at the j end
  std::vector<std::vector<int>> as(nb), rh(nf);
  for (int e = 0; e < n_edges; ++e) {
    const int ci = P.col_of_pose[edge_i[e]], cj = P.col_of_pose[edge_j[e]];
    if (ci >= 0) {
      as[P.blk_ptr[ci]].push_back(2 * e);
      rh[ci].push_back(2 * e);
    }
    if (cj >= 0) {
      as[P.blk_ptr[cj]].push_back(2 * e);
      rh[cj].push_back(2 * e + 1);
    }
    if (ci >= 0 && cj >= 0) {
      const int t = blk(std::max(ci, cj), std::min(ci, cj));
      if (t < 0) return "internal: edge block missing";
      as[t].push_back(2 * e + 1);
    }
  }
  P.asm_ptr.assign(nb + 1, 0);
  for (int t = 0; t < nb; ++t) P.asm_ptr[t + 1] = P.asm_ptr[t] + (int)as[t].size();
  for (int t = 0; t < nb; ++t) P.asm_edge.insert(P.asm_edge.end(), as[t].begin(), as[t].end());
  P.rhs_ptr.assign(nf + 1, 0);
  for (int c = 0; c < nf; ++c) P.rhs_ptr[c + 1] = P.rhs_ptr[c] + (int)rh[c].size();
  for (int c = 0; c < nf; ++c) P.rhs_edge.insert(P.rhs_edge.end(), rh[c].begin(), rh[c].end());
  P.blk_col.resize(nb);
  for (int c = 0; c < nf; ++c)
    for (int b = P.blk_ptr[c]; b < P.blk_ptr[c + 1]; ++b) P.blk_col[b] = c;
  P.chunk_ptr.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    const int n = P.upd_ptr[b + 1] - P.upd_ptr[b];
    P.chunk_ptr[b + 1] = P.chunk_ptr[b] + (n + kPgoChunk - 1) / kPgoChunk;
    for (int q = P.chunk_ptr[b]; q < P.chunk_ptr[b + 1]; ++q) P.chunk_blk.push_back(b);
  }
  P.fchunk_ptr.assign(nf + 1, 0);
  for (int c = 0; c < nf; ++c) {
    const int n = P.fwd_ptr[c + 1] - P.fwd_ptr[c];
    P.fchunk_ptr[c + 1] = P.fchunk_ptr[c] + (n + kPgoChunk - 1) / kPgoChunk;
    for (int q = P.fchunk_ptr[c]; q < P.fchunk_ptr[c + 1]; ++q) P.fchunk_col.push_back(c);
  }
  P.chunk_ab.assign(P.chunk_blk.size() * 2 * kPgoChunk, -1);
  for (int b = 0; b < nb; ++b)
    for (int q = P.chunk_ptr[b]; q < P.chunk_ptr[b + 1]; ++q) {
      const int u0 = P.upd_ptr[b] + kPgoChunk * (q - P.chunk_ptr[b]);
      const int u1 = std::min(u0 + kPgoChunk, P.upd_ptr[b + 1]);
      for (int k = 0; u0 + k < u1; ++k) {
        P.chunk_ab[(size_t)2 * kPgoChunk * q + k] = P.upd_a[u0 + k];
        P.chunk_ab[(size_t)2 * kPgoChunk * q + kPgoChunk + k] = P.upd_b[u0 + k];
      }
    }
  P.fchunk_bc.assign(P.fchunk_col.size() * 2 * kPgoChunk, -1);
  for (int c = 0; c < nf; ++c)
    for (int q = P.fchunk_ptr[c]; q < P.fchunk_ptr[c + 1]; ++q) {
      const int g0 = P.fwd_ptr[c] + kPgoChunk * (q - P.fchunk_ptr[c]);
      const int g1 = std::min(g0 + kPgoChunk, P.fwd_ptr[c + 1]);
      for (int k = 0; g0 + k < g1; ++k) {
        P.fchunk_bc[(size_t)2 * kPgoChunk * q + k] = P.fwd_blk[g0 + k];
        P.fchunk_bc[(size_t)2 * kPgoChunk * q + kPgoChunk + k] = P.fwd_col[g0 + k];
      }
    }
  // leading levels whose update phase has at least 4096 tasks run as
  // launches over the whole GPU
  for (int l = 0; l < P.n_levels; ++l) {
    const int c0 = P.lev_ptr[l], c1 = P.lev_ptr[l + 1];
    const int b0 = P.blk_ptr[c0], b1 = P.blk_ptr[c1];
    const int t1 = (P.chunk_ptr[b1] - P.chunk_ptr[b0]) * 36 + (P.fchunk_ptr[c1] - P.fchunk_ptr[c0]) * 6;
    if (t1 < 4096 && l > 0) break;
    P.wide_tasks.push_back(t1);
    P.wide_tasks.push_back(c1 - c0);
    P.wide_tasks.push_back((b1 - b0) * 6);
    P.n_wide = l + 1;
  }
  return "";
}

size_t pgo_workspace_bytes(const PgoPlan& P) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return 2 * up((size_t)P.n_edges * 28 * 8) + up((size_t)P.n_poses * 12 * 8) +
         up((size_t)P.n_blocks() * 36 * 8) + 2 * up((size_t)P.n_free * 6 * 8) +
         up(((size_t)P.chunk_blk.size() * 36 + P.fchunk_col.size() * 6) * 8) + up(8 * 8) + up(8 * 4);
}

PgoWork pgo_carve(const PgoPlan& P, void* ws) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* p = (char*)ws;
  PgoWork W;
  W.edge[0] = (double*)p;
  p += up((size_t)P.n_edges * 28 * 8);
  W.edge[1] = (double*)p;
  p += up((size_t)P.n_edges * 28 * 8);
  W.cand = (double*)p;
  p += up((size_t)P.n_poses * 12 * 8);
  W.L = (double*)p;
  p += up((size_t)P.n_blocks() * 36 * 8);
  W.y = (double*)p;
  p += up((size_t)P.n_free * 6 * 8);
  W.x = (double*)p;
  p += up((size_t)P.n_free * 6 * 8);
  W.part = (double*)p;
  p += up(((size_t)P.chunk_blk.size() * 36 + P.fchunk_col.size() * 6) * 8);
  W.state = (double*)p;
  p += up(8 * 8);
  W.istate = (int32_t*)p;
  return W;
}

}  // namespace ba
