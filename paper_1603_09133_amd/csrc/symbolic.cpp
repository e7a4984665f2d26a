// Host symbolic analysis of the compress-and-eliminate factorization.
//
// Everything here is integer work on the block graph:
//   * the initial permutation of a tensor grid: patches in Z (Morton) order
//     (Section 2, eq. (init_perm); Section 2.8 on the choice of P);
//   * the close pattern of every level (structural nonzero blocks);
//   * the elimination order (block order, or a distance-2 colouring) and the
//     dependency waves: two steps whose blocks are at graph distance <= 2
//     touch a common block (far blocks join distance-2 pairs, the Schur
//     update joins pairs of close neighbours), so they keep their order;
//     steps at distance >= 3 commute exactly;
//   * the far blocks created by each step (eq. (A_st)): pairs of close
//     neighbours of the eliminated block that are not close to each other;
//     a block whose far row is empty when it is processed is eliminated
//     whole (Section 2.1) and leaves the graph (Section 2.4, node 1);
//   * the coarsening of 2^d Morton siblings into super-blocks (Section 2.5, eq. (bsp));
//   * the work lists of the numeric kernels (slots, views, Schur targets).
#include "symbolic.h"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <unordered_set>

namespace cae {

namespace {

uint64_t morton(const int32_t* c, int ndim) {
  uint64_t key = 0;
  for (int bit = 0; bit < 21; ++bit)
    for (int k = 0; k < ndim; ++k)
      key |= (uint64_t)((c[k] >> bit) & 1) << (bit * ndim + k);
  return key;
}

inline uint64_t pkey(int32_t p, int32_t q) {
  if (p > q) std::swap(p, q);
  return ((uint64_t)(uint32_t)p << 32) | (uint32_t)q;
}

void build_adjacency(int32_t M, const std::vector<int32_t>& pairs,
                     std::vector<int32_t>& ptr, std::vector<int32_t>& adj) {
  ptr.assign(M + 1, 0);
  size_t np = pairs.size() / 2;
  for (size_t k = 0; k < np; ++k) {
    ptr[pairs[2 * k] + 1]++;
    ptr[pairs[2 * k + 1] + 1]++;
  }
  for (int32_t i = 0; i < M; ++i) ptr[i + 1] += ptr[i];
  adj.assign(ptr[M], 0);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (size_t k = 0; k < np; ++k) {
    int32_t p = pairs[2 * k], q = pairs[2 * k + 1];
    adj[fill[p]++] = q;
    adj[fill[q]++] = p;
  }
  for (int32_t i = 0; i < M; ++i) std::sort(adj.begin() + ptr[i], adj.begin() + ptr[i + 1]);
}

// Colouring at distance 2 by a lattice pattern of the block coordinates when
// it is valid on this graph ((x + 2y) mod 5 / (x + 2y + 3z) mod 7, then the
// product of coordinates mod 3), else greedy in block index order.
// Order = (colour, index).
bool valid_colouring(const LevelSym& L, const std::vector<int32_t>& col) {
  for (int32_t i = 0; i < L.M; ++i)
    for (int32_t k = L.cptr[i]; k < L.cptr[i + 1]; ++k) {
      const int32_t c = L.cadj[k];
      if (col[c] == col[i]) return false;
      for (int32_t m = L.cptr[c]; m < L.cptr[c + 1]; ++m) {
        const int32_t d = L.cadj[m];
        if (d != i && col[d] == col[i]) return false;
      }
    }
  return true;
}

bool lattice_colours(const LevelSym& L, int ndim, std::vector<int32_t>& col) {
  if (L.coords.empty() || ndim < 1) return false;
  struct Cand {
    bool lin;
    int a[3];
    int q;
  };
  std::vector<Cand> cands;
  if (ndim == 1) cands = {{true, {1, 0, 0}, 3}};
  if (ndim == 2) cands = {{true, {1, 2, 0}, 5}, {false, {0, 0, 0}, 3}};
  if (ndim == 3) cands = {{true, {1, 2, 3}, 7}, {false, {0, 0, 0}, 3}};
  col.assign(L.M, 0);
  for (const Cand& cd : cands) {
    for (int32_t i = 0; i < L.M; ++i) {
      const int32_t* c = &L.coords[(int64_t)i * ndim];
      int64_t v = 0;
      if (cd.lin) {
        for (int k = 0; k < ndim; ++k) v += (int64_t)cd.a[k] * c[k];
        v %= cd.q;
      } else {
        int64_t mul = 1;
        for (int k = 0; k < ndim; ++k) {
          v += (int64_t)(c[k] % cd.q) * mul;
          mul *= cd.q;
        }
      }
      col[i] = (int32_t)v;
    }
    if (valid_colouring(L, col)) return true;
  }
  return false;
}

void colour_order(LevelSym& L, int ndim) {
  const int32_t M = L.M;
  std::vector<int32_t> colour;
  if (!lattice_colours(L, ndim, colour)) {
    colour.assign(M, -1);
    std::vector<int32_t> stamp;
    for (int32_t i = 0; i < M; ++i) {
      auto mark = [&](int32_t j) {
        if (j < i) {
          int32_t c = colour[j];
          if ((int32_t)stamp.size() <= c) stamp.resize(c + 1, -1);
          stamp[c] = i;
        }
      };
      for (int32_t k = L.cptr[i]; k < L.cptr[i + 1]; ++k) {
        int32_t c = L.cadj[k];
        mark(c);
        for (int32_t m = L.cptr[c]; m < L.cptr[c + 1]; ++m)
          if (L.cadj[m] != i) mark(L.cadj[m]);
      }
      int32_t c = 0;
      while (c < (int32_t)stamp.size() && stamp[c] == i) ++c;
      colour[i] = c;
    }
  }
  L.order.resize(M);
  std::iota(L.order.begin(), L.order.end(), 0);
  std::stable_sort(L.order.begin(), L.order.end(),
                   [&](int32_t a, int32_t b) { return colour[a] < colour[b]; });
}

void compute_waves(LevelSym& L) {
  const int32_t M = L.M;
  L.wave.assign(M, 0);
  int32_t nw = 0;
  for (int32_t s = 0; s < M; ++s) {
    int32_t i = L.order[s];
    int32_t w = 0;
    for (int32_t k = L.cptr[i]; k < L.cptr[i + 1]; ++k) {
      int32_t c = L.cadj[k];
      if (L.pos[c] < s) w = std::max(w, L.wave[c] + 1);
      for (int32_t m = L.cptr[c]; m < L.cptr[c + 1]; ++m) {
        int32_t d = L.cadj[m];
        if (d != i && L.pos[d] < s) w = std::max(w, L.wave[d] + 1);
      }
    }
    L.wave[i] = w;
    nw = std::max(nw, w + 1);
  }
  L.nwaves = M ? nw : 0;
}

// Structural pass in the elimination order: far rows at step time, created
// far pairs, removed blocks.
void simulate(LevelSym& L, std::vector<std::vector<int32_t>>& far_at_step) {
  const int32_t M = L.M;
  std::vector<std::vector<int32_t>> far(M);
  std::unordered_set<uint64_t> farset;
  farset.reserve((size_t)M * 8);
  L.removed.assign(M, 0);
  far_at_step.assign(M, {});
  for (int32_t s = 0; s < M; ++s) {
    int32_t i = L.order[s];
    far_at_step[i] = far[i];
    std::sort(far_at_step[i].begin(), far_at_step[i].end());
    if (far[i].empty()) L.removed[i] = 1;
    for (int32_t ka = L.cptr[i]; ka < L.cptr[i + 1]; ++ka) {
      int32_t a = L.cadj[ka];
      if (L.removed[a]) continue;
      // the candidates c (ascending) against a's sorted close list, walked
      // together instead of searched one by one
      int32_t ma = L.cptr[a];
      const int32_t ea = L.cptr[a + 1];
      for (int32_t kc = ka + 1; kc < L.cptr[i + 1]; ++kc) {
        int32_t c = L.cadj[kc];
        while (ma < ea && L.cadj[ma] < c) ++ma;
        if (L.removed[c]) continue;
        if (ma < ea && L.cadj[ma] == c) continue;   // (a, c) is close
        if (!farset.insert(pkey(a, c)).second) continue;
        far[a].push_back(c);
        far[c].push_back(a);
      }
    }
  }
  L.far_pairs.clear();
  std::vector<uint64_t> keys(farset.begin(), farset.end());
  std::sort(keys.begin(), keys.end());
  for (uint64_t k : keys) {
    L.far_pairs.push_back((int32_t)(k >> 32));
    L.far_pairs.push_back((int32_t)(k & 0xffffffffu));
  }
}

void build_slots(LevelSym& L) {
  const int32_t M = L.M;
  std::vector<uint64_t> keys;
  keys.reserve(L.close_pairs.size() / 2 + L.far_pairs.size() / 2);
  for (size_t k = 0; k < L.close_pairs.size(); k += 2) keys.push_back(pkey(L.close_pairs[k], L.close_pairs[k + 1]));
  for (size_t k = 0; k < L.far_pairs.size(); k += 2) keys.push_back(pkey(L.far_pairs[k], L.far_pairs[k + 1]));
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  L.nslots = M + (int32_t)keys.size();
  L.slot_p.resize(L.nslots);
  L.slot_q.resize(L.nslots);
  for (int32_t i = 0; i < M; ++i) L.slot_p[i] = L.slot_q[i] = i;
  L.up_ptr.assign(M + 1, 0);
  for (size_t k = 0; k < keys.size(); ++k) {
    int32_t p = (int32_t)(keys[k] >> 32), q = (int32_t)(keys[k] & 0xffffffffu);
    L.slot_p[M + k] = p;
    L.slot_q[M + k] = q;
    L.up_ptr[p + 1]++;
  }
  for (int32_t i = 0; i < M; ++i) L.up_ptr[i + 1] += L.up_ptr[i];
  L.up_q.resize(keys.size());
  L.up_slot.resize(keys.size());
  // keys are sorted by (p, q): the run of p is contiguous and in q order
  for (size_t k = 0; k < keys.size(); ++k) {
    L.up_q[k] = L.slot_q[M + k];
    L.up_slot[k] = M + (int32_t)k;
  }
}

void build_items(LevelSym& L, const std::vector<std::vector<int32_t>>& far_at_step) {
  const int32_t M = L.M;
  std::vector<int32_t> by_wave(M);
  std::iota(by_wave.begin(), by_wave.end(), 0);
  // steps sorted by (wave, position in the order)
  std::vector<int32_t> seq(L.order);
  std::stable_sort(seq.begin(), seq.end(), [&](int32_t a, int32_t b) { return L.wave[a] < L.wave[b]; });
  L.steps.clear();
  L.views.clear();
  L.rot.clear();
  L.trsm.clear();
  L.pairs.clear();
  L.wave_ptr.assign(L.nwaves + 1, 0);
  L.rot_ptr.assign(L.nwaves + 1, 0);
  L.trsm_ptr.assign(L.nwaves + 1, 0);
  L.pair_ptr.assign(L.nwaves + 1, 0);
  {
    size_t np = 0;   // Schur targets of every step, at most (nclose + 1)(nclose + 2) / 2
    for (int32_t i = 0; i < L.M; ++i) {
      const size_t c = (size_t)(L.cptr[i + 1] - L.cptr[i]);
      np += (c + 1) * (c + 2) / 2;
    }
    L.pairs.reserve(np);
  }
  int32_t cur_wave = 0;
  auto close_wave = [&](int32_t upto) {
    while (cur_wave < upto) {
      ++cur_wave;
      L.wave_ptr[cur_wave] = (int32_t)L.steps.size();
      L.rot_ptr[cur_wave] = (int32_t)L.rot.size();
      L.trsm_ptr[cur_wave] = (int32_t)L.trsm.size();
      L.pair_ptr[cur_wave] = (int32_t)L.pairs.size();
    }
  };
  for (int32_t i : seq) {
    close_wave(L.wave[i]);
    const int32_t s = (int32_t)L.steps.size();
    const int32_t me = L.pos[i];
    Step st;
    st.blk = i;
    st.nclose = L.cptr[i + 1] - L.cptr[i];
    st.nfar = (int32_t)far_at_step[i].size();
    st.view0 = (int32_t)L.views.size();
    auto add_view = [&](int32_t x) {
      View v;
      v.slot = L.slot_of(i, x);
      v.x = x;
      v.trans = x < i ? 1 : 0;
      v.proc = L.pos[x] < me ? 1 : 0;
      L.views.push_back(v);
    };
    for (int32_t k = L.cptr[i]; k < L.cptr[i + 1]; ++k) add_view(L.cadj[k]);
    for (int32_t x : far_at_step[i]) add_view(x);
    L.steps.push_back(st);
    auto gone = [&](int32_t x) { return L.removed[x] && L.pos[x] < me; };
    if (st.nfar > 0) {
      L.rot.push_back(Item{s, -1});
      for (int32_t v = 0; v < st.nclose + st.nfar; ++v) L.rot.push_back(Item{s, st.view0 + v});
    }
    for (int32_t v = 0; v < st.nclose; ++v)
      if (!gone(L.views[st.view0 + v].x)) L.trsm.push_back(Item{s, st.view0 + v});
    for (int32_t a = 0; a <= st.nclose; ++a) {
      int32_t xa = a ? L.views[st.view0 + a - 1].x : i;
      if (a && gone(xa)) continue;
      // slots (xa, xc) with xc > xa: the close views come in ascending block
      // order, so one walk along xa's sorted upper neighbours finds them all
      int32_t u = a ? L.up_ptr[xa] : 0;
      const int32_t ue = a ? L.up_ptr[xa + 1] : 0;
      for (int32_t c = a; c <= st.nclose; ++c) {
        int32_t xc = c ? L.views[st.view0 + c - 1].x : i;
        if (c && gone(xc)) continue;
        Pair pr;
        pr.step = s;
        pr.a = a;
        pr.c = c;
        pr.slot = -1;
        pr.trans = 0;
        if (a > 0) {
          if (a == c) {
            pr.slot = xa;
          } else if (xc > xa) {
            while (u < ue && L.up_q[u] < xc) ++u;
            pr.slot = (u < ue && L.up_q[u] == xc) ? L.up_slot[u] : -1;
          } else {
            pr.slot = L.slot_of(xa, xc);
            pr.trans = 1;
          }
        }
        L.pairs.push_back(pr);
      }
    }
  }
  close_wave(L.nwaves);
}

}  // namespace

int32_t LevelSym::slot_of(int32_t p, int32_t q) const {
  if (p == q) return p;
  if (p > q) std::swap(p, q);
  auto b = up_q.begin() + up_ptr[p], e = up_q.begin() + up_ptr[p + 1];
  auto it = std::lower_bound(b, e, q);
  if (it == e || *it != q) return -1;
  return up_slot[it - up_q.begin()];
}

std::string graph_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t B,
                        std::vector<int32_t>& perm, std::vector<int32_t>& block_ptr) {
  if (n <= 0 || B <= 0) return "n and B must be positive";
  if (n > INT32_MAX) return "too many unknowns";
  int depth = 0;
  while (((n + ((int64_t)1 << depth) - 1) >> depth) > B && ((int64_t)2 << depth) <= n) ++depth;
  std::vector<int32_t> ord(n), part(n, 0), dist(n, -1), queue;
  for (int64_t v = 0; v < n; ++v) ord[v] = (int32_t)v;
  queue.reserve(n);
  // breadth-first order of ord[b..e) inside the part `id`, from `start`,
  // restarting at the first unvisited vertex for disconnected parts
  auto bfs = [&](int64_t b, int64_t e, int32_t id, int32_t start, std::vector<int32_t>& out) -> int32_t {
    out.clear();
    for (int64_t k = b; k < e; ++k) dist[ord[k]] = -1;
    int32_t last = start;
    int64_t next_seed = b;
    int32_t s = start;
    while ((int64_t)out.size() < e - b) {
      if (dist[s] >= 0) {
        while (next_seed < e && dist[ord[next_seed]] >= 0) ++next_seed;
        s = ord[next_seed];
      }
      size_t head = out.size();
      dist[s] = 0;
      out.push_back(s);
      while (head < out.size()) {
        const int32_t u = out[head++];
        last = u;
        for (int64_t q = row_ptr[u]; q < row_ptr[u + 1]; ++q) {
          const int32_t w = col_idx[q];
          if (w < 0 || w >= n || part[w] != id || dist[w] >= 0) continue;
          dist[w] = dist[u] + 1;
          out.push_back(w);
        }
      }
    }
    return last;
  };
  std::vector<int32_t> tmp;
  std::vector<std::pair<int64_t, int64_t>> level{{0, n}};
  int32_t next_id = 1;
  for (int d = 0; d < depth; ++d) {
    std::vector<std::pair<int64_t, int64_t>> nxt;
    for (auto [b, e] : level) {
      const int32_t id = part[ord[b]];
      // pseudo-peripheral vertex: the last vertex of two breadth-first sweeps
      int32_t v = ord[b];
      for (int64_t k = b + 1; k < e; ++k) v = std::min(v, ord[k]);
      v = bfs(b, e, id, v, tmp);
      v = bfs(b, e, id, v, tmp);
      bfs(b, e, id, v, tmp);
      const int64_t m = e - b, h = (m + 1) / 2;
      const int32_t idl = next_id++, idr = next_id++;
      for (int64_t k = 0; k < m; ++k) {
        ord[b + k] = tmp[k];
        part[tmp[k]] = k < h ? idl : idr;
      }
      nxt.push_back({b, b + h});
      nxt.push_back({b + h, e});
    }
    level.swap(nxt);
  }
  perm.assign(ord.begin(), ord.end());
  block_ptr.clear();
  for (auto [b, e] : level) block_ptr.push_back((int32_t)b);
  block_ptr.push_back((int32_t)n);
  return {};
}

std::string grid_order(int32_t ndim, const int32_t* dims, const int32_t* patch,
                       std::vector<int32_t>& perm, std::vector<int32_t>& block_ptr,
                       std::vector<int32_t>& coords) {
  if (ndim < 1 || ndim > 3) return "ndim must be 1, 2 or 3";
  int64_t n = 1;
  int32_t np[3] = {1, 1, 1}, d[3] = {1, 1, 1}, p[3] = {1, 1, 1};
  for (int k = 0; k < ndim; ++k) {
    if (dims[k] <= 0 || patch[k] <= 0) return "dims and patch must be positive";
    d[k] = dims[k];
    p[k] = patch[k];
    np[k] = (dims[k] + patch[k] - 1) / patch[k];
    n *= dims[k];
  }
  if (n > INT32_MAX) return "grid too large";
  const int64_t npt = (int64_t)np[0] * np[1] * np[2];
  std::vector<std::pair<uint64_t, int64_t>> keyed(npt);
  for (int64_t t = 0; t < npt; ++t) {
    int32_t c[3] = {(int32_t)(t % np[0]), (int32_t)((t / np[0]) % np[1]), (int32_t)(t / ((int64_t)np[0] * np[1]))};
    keyed[t] = {morton(c, ndim), t};
  }
  std::sort(keyed.begin(), keyed.end());
  perm.clear();
  perm.reserve(n);
  block_ptr.assign(1, 0);
  coords.clear();
  for (auto& kt : keyed) {
    int64_t t = kt.second;
    int32_t c[3] = {(int32_t)(t % np[0]), (int32_t)((t / np[0]) % np[1]), (int32_t)(t / ((int64_t)np[0] * np[1]))};
    int32_t lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = c[k] * p[k];
      hi[k] = std::min(lo[k] + p[k], d[k]);
    }
    for (int32_t z = lo[2]; z < hi[2]; ++z)
      for (int32_t y = lo[1]; y < hi[1]; ++y)
        for (int32_t x = lo[0]; x < hi[0]; ++x)
          perm.push_back(x + d[0] * (y + d[1] * z));
    block_ptr.push_back((int32_t)perm.size());
    for (int k = 0; k < ndim; ++k) coords.push_back(c[k]);
  }
  return "";
}

std::string analyze(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                    const int32_t* perm, const int32_t* block_ptr, int32_t nblocks,
                    int32_t B, const int32_t* coords, int32_t ndim, int32_t order_kind,
                    Analysis& A, int32_t coarsen_kind) {
  if (n <= 0 || n > INT32_MAX) return "n out of range";
  if (!row_ptr || !col_idx || !perm) return "row_ptr, col_idx and perm are required";
  if (order_kind != 0 && order_kind != 1) return "unknown elimination order";
  if (ndim < 0 || ndim > 3) return "ndim must be 0..3";
  A.n = n;
  A.ndim = ndim;
  A.order_kind = order_kind;
  if (row_ptr[0] != 0) return "row_ptr[0] must be 0";
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return "row_ptr is not monotone";
  const int64_t nnz = row_ptr[n];
  A.row_ptr.assign(row_ptr, row_ptr + n + 1);
  A.col_idx.assign(col_idx, col_idx + nnz);
  A.diag_pos.assign(n, -1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t j = col_idx[k];
      if (j < 0 || j >= n) return "column index out of range";
      if (j == i) A.diag_pos[i] = k;
    }
  for (int64_t i = 0; i < n; ++i)
    if (A.diag_pos[i] < 0) return "every row needs a diagonal entry";
  A.perm.assign(perm, perm + n);
  A.iperm.assign(n, -1);
  for (int64_t k = 0; k < n; ++k) {
    int32_t o = perm[k];
    if (o < 0 || o >= n || A.iperm[o] != -1) return "perm is not a permutation";
    A.iperm[o] = (int32_t)k;
  }
  if (block_ptr) {
    if (nblocks <= 0 || block_ptr[0] != 0 || block_ptr[nblocks] != n) return "block_ptr must span 0..n";
    A.block_ptr.assign(block_ptr, block_ptr + nblocks + 1);
    for (int32_t b = 0; b < nblocks; ++b)
      if (block_ptr[b + 1] <= block_ptr[b]) return "blocks must be non-empty";
  } else {
    if (B <= 0) return "B must be positive when block_ptr is NULL";
    A.block_ptr.clear();
    for (int64_t s = 0; s < n; s += B) A.block_ptr.push_back((int32_t)s);
    A.block_ptr.push_back((int32_t)n);
    nblocks = (int32_t)A.block_ptr.size() - 1;
    coords = nullptr;
  }
  const int32_t M1 = nblocks;
  std::vector<int32_t> owner(n);
  for (int32_t b = 0; b < M1; ++b)
    for (int32_t k = A.block_ptr[b]; k < A.block_ptr[b + 1]; ++k) owner[k] = b;

  // level-1 close pattern: blocks that hold a structural nonzero of A0
  std::vector<uint64_t> keys;
  for (int64_t i = 0; i < n; ++i) {
    int32_t bi = owner[A.iperm[i]];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t bj = owner[A.iperm[col_idx[k]]];
      if (bi != bj) keys.push_back(pkey(bi, bj));
    }
  }
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  std::vector<int32_t> pairs;
  pairs.reserve(keys.size() * 2);
  for (uint64_t k : keys) {
    pairs.push_back((int32_t)(k >> 32));
    pairs.push_back((int32_t)(k & 0xffffffffu));
  }

  std::vector<int32_t> cur_coords;
  if (coords && ndim > 0) cur_coords.assign(coords, coords + (int64_t)M1 * ndim);
  const int32_t J = ndim > 0 ? (1 << ndim) : 2;
  int32_t M = M1;
  A.levels.clear();
  while (true) {
    A.levels.emplace_back();
    LevelSym& L = A.levels.back();
    L.M = M;
    L.close_pairs = pairs;
    L.coords = cur_coords;
    build_adjacency(M, pairs, L.cptr, L.cadj);
    if (order_kind == 0 || M == 1) {
      L.order.resize(M);
      std::iota(L.order.begin(), L.order.end(), 0);
    } else {
      colour_order(L, cur_coords.empty() ? 0 : ndim);
    }
    L.pos.assign(M, 0);
    for (int32_t s = 0; s < M; ++s) L.pos[L.order[s]] = s;
    std::vector<std::vector<int32_t>> far_at_step;
    simulate(L, far_at_step);
    compute_waves(L);
    build_slots(L);
    build_items(L, far_at_step);
    if (M == 1) {
      L.parent.assign(1, 0);
      L.Mnext = 1;
      break;
    }
    // coarsening: Morton siblings (coordinate >> 1), else groups of J
    L.parent.assign(M, 0);
    std::vector<int32_t> next_coords;
    if (!cur_coords.empty()) {
      // siblings: 2^d blocks sharing coordinate >> 1 on every axis, or (pairs)
      // 2 blocks sharing coordinate >> 1 on axis (level mod d) -- the lowest
      // remaining bit of the Morton key, so the axes alternate
      const int lev = (int)A.levels.size() - 1;
      const int ax = coarsen_kind == 1 ? lev % ndim : -1;
      int32_t P = -1;
      std::vector<int32_t> last(ndim, INT32_MIN);
      for (int32_t i = 0; i < M; ++i) {
        bool same = P >= 0;
        for (int k = 0; k < ndim; ++k) {
          const int sh = (ax < 0 || k == ax) ? 1 : 0;
          same = same && ((cur_coords[(int64_t)i * ndim + k] >> sh) == last[k]);
        }
        if (!same) {
          ++P;
          for (int k = 0; k < ndim; ++k) {
            const int sh = (ax < 0 || k == ax) ? 1 : 0;
            last[k] = cur_coords[(int64_t)i * ndim + k] >> sh;
            next_coords.push_back(last[k]);
          }
        }
        L.parent[i] = P;
      }
      L.Mnext = P + 1;
      // the siblings must be consecutive (Morton order of the blocks)
      if (ax < 0) {
        std::vector<uint64_t> seen;
        for (int32_t P2 = 0; P2 < L.Mnext; ++P2) seen.push_back(morton(&next_coords[(int64_t)P2 * ndim], ndim));
        for (size_t k = 1; k < seen.size(); ++k)
          if (seen[k] <= seen[k - 1]) return "blocks are not in Morton order of their coordinates";
      } else {
        std::vector<uint64_t> seen;
        for (int32_t P2 = 0; P2 < L.Mnext; ++P2) {
          uint64_t key = 0;
          for (int k = 0; k < ndim; ++k) key = key * 2097152u + (uint64_t)(uint32_t)next_coords[(int64_t)P2 * ndim + k];
          seen.push_back(key);
        }
        std::sort(seen.begin(), seen.end());
        for (size_t k = 1; k < seen.size(); ++k)
          if (seen[k] == seen[k - 1]) return "blocks are not in Morton order of their coordinates";
      }
    } else {
      for (int32_t i = 0; i < M; ++i) L.parent[i] = i / J;
      L.Mnext = (M + J - 1) / J;
    }
    // next-level pattern from the pairs that keep unknowns
    std::vector<uint64_t> nk;
    auto add = [&](int32_t p, int32_t q) {
      if (L.removed[p] || L.removed[q]) return;
      int32_t P = L.parent[p], Q = L.parent[q];
      if (P != Q) nk.push_back(pkey(P, Q));
    };
    for (size_t k = 0; k < L.close_pairs.size(); k += 2) add(L.close_pairs[k], L.close_pairs[k + 1]);
    for (size_t k = 0; k < L.far_pairs.size(); k += 2) add(L.far_pairs[k], L.far_pairs[k + 1]);
    std::sort(nk.begin(), nk.end());
    nk.erase(std::unique(nk.begin(), nk.end()), nk.end());
    pairs.clear();
    for (uint64_t k : nk) {
      pairs.push_back((int32_t)(k >> 32));
      pairs.push_back((int32_t)(k & 0xffffffffu));
    }
    cur_coords.swap(next_coords);
    M = L.Mnext;
  }
  // copies of the basis parts into the next level
  for (size_t l = 0; l + 1 < A.levels.size(); ++l) {
    LevelSym& L = A.levels[l];
    const LevelSym& N = A.levels[l + 1];
    L.trans.clear();
    for (int32_t s = 0; s < L.nslots; ++s) {
      int32_t p = L.slot_p[s], q = L.slot_q[s];
      if (L.removed[p] || L.removed[q]) continue;
      Trans t;
      t.src_slot = s;
      t.p = p;
      t.q = q;
      t.dst_slot = N.slot_of(L.parent[p], L.parent[q]);
      if (t.dst_slot < 0) return "internal: missing next-level slot";
      L.trans.push_back(t);
    }
  }
  // level-1 arena positions of the entries of A0 (slots are p <= q)
  const LevelSym& L1 = A.levels[0];
  A.level1_slot_off.assign(L1.nslots + 1, 0);
  for (int32_t s = 0; s < L1.nslots; ++s) {
    int64_t bp = A.block_ptr[L1.slot_p[s] + 1] - A.block_ptr[L1.slot_p[s]];
    int64_t bq = A.block_ptr[L1.slot_q[s] + 1] - A.block_ptr[L1.slot_q[s]];
    A.level1_slot_off[s + 1] = A.level1_slot_off[s] + bp * bq;
  }
  A.a0_dst.assign(nnz, -1);
  for (int64_t i = 0; i < n; ++i) {
    int32_t ni = A.iperm[i], p = owner[ni];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t nj = A.iperm[col_idx[k]], q = owner[nj];
      if (p > q) continue;
      int32_t s = L1.slot_of(p, q);
      if (s < 0) return "internal: missing level-1 slot";
      int64_t bq = A.block_ptr[q + 1] - A.block_ptr[q];
      A.a0_dst[k] = A.level1_slot_off[s] + (int64_t)(ni - A.block_ptr[p]) * bq + (nj - A.block_ptr[q]);
    }
  }
  return "";
}

// ---------------------------------------------------------------- batches ---
namespace {
void batch_offset(int32_t t, int32_t out[3]) {
  out[0] = out[1] = out[2] = 0;
  for (int bit = 0; (t >> bit) != 0; ++bit) out[bit % 3] |= ((t >> bit) & 1) << (bit / 3);
  for (int a = 0; a < 3; ++a) out[a] <<= kBatchCoordBits;
}
}  // namespace

std::string batch_assemble(int32_t nprob, const BatchProblem* probs, std::vector<int64_t>& row_off,
                           std::vector<int64_t>& row_ptr, std::vector<int32_t>& col_idx,
                           std::vector<int32_t>& perm, std::vector<int32_t>& block_ptr,
                           std::vector<int32_t>& coords) {
  if (nprob <= 0 || !probs) return "nprob > 0 problems are required";
  if (nprob > (1 << 21)) return "too many problems for the block-coordinate budget";
  std::vector<int64_t> nz_off(nprob + 1, 0);
  row_off.assign(nprob + 1, 0);
  for (int t = 0; t < nprob; ++t) {
    const BatchProblem& P = probs[t];
    const std::string who = "problem " + std::to_string(t) + ": ";
    if (P.ndim != 2 && P.ndim != 3) return who + "ndim must be 2 or 3";
    int64_t cells = 1;
    for (int a = 0; a < P.ndim; ++a) cells *= P.dims[a] > 0 ? P.dims[a] : 0;
    if (P.n <= 0 || cells != P.n) return who + "n must be the product of dims";
    if (!P.row_ptr || !P.col_idx) return who + "row_ptr and col_idx are required";
    if (P.row_ptr[P.n] < P.row_ptr[0]) return who + "row_ptr is not ascending";
    row_off[t + 1] = row_off[t] + P.n;
    nz_off[t + 1] = nz_off[t] + (P.row_ptr[P.n] - P.row_ptr[0]);
  }
  const int64_t n = row_off[nprob], nnz = nz_off[nprob];
  if (n >= ((int64_t)1 << 31)) return "the joint matrix needs 32-bit column indices";
  row_ptr.assign(n + 1, 0);
  col_idx.assign(nnz, 0);
  perm.assign(n, 0);
  block_ptr.clear();
  coords.clear();
  for (int t = 0; t < nprob; ++t) {
    const BatchProblem& P = probs[t];
    const std::string who = "problem " + std::to_string(t) + ": ";
    const int64_t r0 = row_off[t], z0 = nz_off[t];
    for (int64_t i = 0; i < P.n; ++i) {
      if (P.row_ptr[i + 1] < P.row_ptr[i]) return who + "row_ptr is not ascending";
      row_ptr[r0 + i] = z0 + P.row_ptr[i] - P.row_ptr[0];
    }
    for (int64_t e = 0; e < nz_off[t + 1] - z0; ++e) {
      const int32_t c = P.col_idx[P.row_ptr[0] + e];
      if (c < 0 || c >= P.n) return who + "column index out of range";
      col_idx[z0 + e] = (int32_t)(c + r0);
    }
    int32_t patch[3] = {P.patch[0], P.patch[1], P.patch[2]};
    if (patch[0] == 0 && patch[1] == 0 && patch[2] == 0)
      for (int a = 0; a < P.ndim; ++a) patch[a] = P.ndim == 2 ? 8 : 4;
    std::vector<int32_t> p, bp, co;
    const std::string e = grid_order(P.ndim, P.dims, patch, p, bp, co);
    if (!e.empty()) return who + e;
    int32_t off[3];
    batch_offset(t, off);
    for (int64_t i = 0; i < P.n; ++i) perm[r0 + i] = (int32_t)(p[i] + r0);
    const size_t nb = bp.size() - 1;
    for (size_t k = 0; k < nb; ++k) block_ptr.push_back((int32_t)(bp[k] + r0));
    for (size_t k = 0; k < nb; ++k)
      for (int a = 0; a < 3; ++a) {
        const int32_t c = a < P.ndim ? co[k * P.ndim + a] : 0;
        if (c >= (1 << kBatchCoordBits)) return who + "more than 256 patches along an axis";
        coords.push_back(c + off[a]);
      }
  }
  row_ptr[n] = nnz;
  block_ptr.push_back((int32_t)n);
  return "";
}

}  // namespace cae
