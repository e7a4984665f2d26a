// Host-only driver of the symbolic analysis for the sanitizer build: orders
// and analyses a few grids and a general graph with every option, and checks
// the structural invariants the numeric kernels rely on (slots, views, Schur
// targets, copies into the next level).  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <string>
#include <vector>

#include "symbolic.h"

namespace {

int g_fail = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++g_fail;                                                          \
    }                                                                    \
  } while (0)

// 2D 5-point / 3D 7-point grid graph (both triangles, diagonal present)
void grid_csr(const std::vector<int>& d, std::vector<int64_t>& rp, std::vector<int32_t>& ci) {
  const int nd = (int)d.size();
  int64_t n = 1;
  for (int v : d) n *= v;
  rp.assign(1, 0);
  ci.clear();
  for (int64_t i = 0; i < n; ++i) {
    int c[3] = {0, 0, 0};
    int64_t t = i;
    for (int k = 0; k < nd; ++k) {
      c[k] = (int)(t % d[k]);
      t /= d[k];
    }
    std::vector<int32_t> row;
    int64_t stride = 1;
    for (int k = 0; k < nd; ++k) {
      if (c[k] > 0) row.push_back((int32_t)(i - stride));
      if (c[k] + 1 < d[k]) row.push_back((int32_t)(i + stride));
      stride *= d[k];
    }
    row.push_back((int32_t)i);
    std::sort(row.begin(), row.end());
    ci.insert(ci.end(), row.begin(), row.end());
    rp.push_back((int64_t)ci.size());
  }
}

void check_analysis(const cae::Analysis& A) {
  for (size_t l = 0; l < A.levels.size(); ++l) {
    const cae::LevelSym& L = A.levels[l];
    CHECK((int)L.order.size() == L.M && (int)L.wave.size() == L.M);
    CHECK((int)L.wave_ptr.size() == L.nwaves + 1);
    for (const cae::Step& s : L.steps) {
      CHECK(s.blk >= 0 && s.blk < L.M);
      for (int v = 0; v < s.nclose + s.nfar; ++v) {
        const cae::View& w = L.views[s.view0 + v];
        CHECK(w.slot >= L.M && w.slot < L.nslots);
        CHECK(L.slot_of(s.blk, w.x) == w.slot);
      }
    }
    for (const cae::Pair& p : L.pairs) {
      CHECK(p.step >= 0 && p.step < (int)L.steps.size());
      CHECK(p.a <= p.c);
      CHECK(p.slot >= -1 && p.slot < L.nslots);
    }
    for (const cae::Trans& t : L.trans) {
      CHECK(t.src_slot >= 0 && t.src_slot < L.nslots);
      if (l + 1 < A.levels.size()) CHECK(t.dst_slot >= 0 && t.dst_slot < A.levels[l + 1].nslots);
    }
  }
}

}  // namespace

int main() {
  const std::vector<std::vector<int>> grids = {{16, 16}, {18, 13}, {40, 24}, {8, 8, 8}, {7, 9, 6}, {16, 16, 16}};
  for (const auto& d : grids) {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    grid_csr(d, rp, ci);
    const int nd = (int)d.size();
    std::vector<int32_t> dims(d.begin(), d.end()), patch(nd, nd == 2 ? 4 : 2);
    std::vector<int32_t> perm, bp, co;
    std::string e = cae::grid_order(nd, dims.data(), patch.data(), perm, bp, co);
    CHECK(e.empty());
    for (int order = 0; order < 2; ++order)
      for (int coarsen = 0; coarsen < (nd == 3 ? 2 : 1); ++coarsen) {
        cae::Analysis A;
        e = cae::analyze((int64_t)perm.size(), rp.data(), ci.data(), perm.data(), bp.data(), (int32_t)bp.size() - 1,
                         0, co.data(), nd, order, A, coarsen);
        CHECK(e.empty());
        check_analysis(A);
      }
  }
  {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    grid_csr({30, 22}, rp, ci);
    std::vector<int32_t> perm, bp;
    std::string e = cae::graph_order((int64_t)rp.size() - 1, rp.data(), ci.data(), 16, perm, bp);
    CHECK(e.empty());
    cae::Analysis A;
    e = cae::analyze((int64_t)perm.size(), rp.data(), ci.data(), perm.data(), bp.data(), (int32_t)bp.size() - 1, 0,
                     nullptr, 1, 1, A, 0);
    CHECK(e.empty());
    check_analysis(A);
  }
  // a batch of independent 2D and 3D problems joined into one analysis: the
  // invariants above, and no close or far pair of the first level couples two
  // problems; invalid problems are reported
  {
    const std::vector<std::vector<int>> probs = {{24, 24}, {8, 8, 8}, {17, 9}, {6, 6, 6}};
    std::vector<std::vector<int64_t>> rps(probs.size());
    std::vector<std::vector<int32_t>> cis(probs.size());
    std::vector<cae::BatchProblem> bp(probs.size());
    for (size_t t = 0; t < probs.size(); ++t) {
      grid_csr(probs[t], rps[t], cis[t]);
      bp[t].n = (int64_t)rps[t].size() - 1;
      bp[t].row_ptr = rps[t].data();
      bp[t].col_idx = cis[t].data();
      bp[t].ndim = (int32_t)probs[t].size();
      for (size_t a = 0; a < probs[t].size(); ++a) {
        bp[t].dims[a] = probs[t][a];
        bp[t].patch[a] = probs[t].size() == 2 ? 4 : 2;
      }
    }
    std::vector<int64_t> off, rp;
    std::vector<int32_t> ci, perm, bptr, co;
    std::string e = cae::batch_assemble((int32_t)bp.size(), bp.data(), off, rp, ci, perm, bptr, co);
    CHECK(e.empty());
    cae::Analysis A;
    e = cae::analyze(off.back(), rp.data(), ci.data(), perm.data(), bptr.data(), (int32_t)bptr.size() - 1, 0,
                     co.data(), 3, 1, A, 0);
    CHECK(e.empty());
    check_analysis(A);
    // problem of every level-1 block, from the row its first unknown came from
    std::vector<int> prob(bptr.size() - 1);
    for (size_t k = 0; k + 1 < bptr.size(); ++k) {
      const int64_t row = perm[bptr[k]];
      prob[k] = (int)(std::upper_bound(off.begin(), off.end(), row) - off.begin()) - 1;
    }
    const cae::LevelSym& L0 = A.levels[0];
    for (size_t q = 0; q < L0.close_pairs.size(); q += 2)
      CHECK(prob[L0.close_pairs[q]] == prob[L0.close_pairs[q + 1]]);
    for (size_t q = 0; q < L0.far_pairs.size(); q += 2) CHECK(prob[L0.far_pairs[q]] == prob[L0.far_pairs[q + 1]]);
    cae::BatchProblem bad = bp[1];
    bad.dims[2] = 9;   // n is not the product of dims
    CHECK(!cae::batch_assemble(1, &bad, off, rp, ci, perm, bptr, co).empty());
    std::vector<int32_t> ci_bad = cis[0];
    ci_bad[3] = 1 << 20;   // a column index out of range
    bad = bp[0];
    bad.col_idx = ci_bad.data();
    CHECK(!cae::batch_assemble(1, &bad, off, rp, ci, perm, bptr, co).empty());
    CHECK(!cae::batch_assemble(0, bp.data(), off, rp, ci, perm, bptr, co).empty());
  }
  // invalid inputs are reported, not read out of bounds
  {
    std::vector<int64_t> rp = {0, 1, 2};
    std::vector<int32_t> ci = {0, 5};
    std::vector<int32_t> perm = {0, 1}, bp = {0, 2};
    cae::Analysis A;
    CHECK(!cae::analyze(2, rp.data(), ci.data(), perm.data(), bp.data(), 1, 0, nullptr, 0, 1, A, 0).empty());
  }
  if (g_fail) return 1;
  std::printf("ok\n");
  return 0;
}
