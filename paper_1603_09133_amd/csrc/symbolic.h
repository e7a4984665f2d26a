// Host symbolic analysis of the CE factorization (integers only).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "cae_internal.h"

namespace cae {

struct LevelSym {
  int32_t M = 0;
  std::vector<int32_t> cptr, cadj;          // close adjacency (CSR, sorted)
  std::vector<int32_t> close_pairs;         // 2 * nclose, p < q, sorted
  std::vector<int32_t> order, pos, wave;
  int32_t nwaves = 0;
  std::vector<int32_t> far_pairs;           // 2 * nfar created far pairs, sorted
  std::vector<uint8_t> removed;             // eliminated whole (empty far row)
  std::vector<int32_t> parent;              // next-level block of every block
  int32_t Mnext = 0;
  std::vector<int32_t> coords;              // M * ndim, or empty
  // slots: 0..M-1 diagonal, then the pairs (close U far) in (p, q) order
  int32_t nslots = 0;
  std::vector<int32_t> slot_p, slot_q;
  std::vector<int32_t> up_ptr, up_q, up_slot;   // q > p neighbours of p, sorted
  // step-ordered work lists, grouped by wave
  std::vector<Step> steps;
  std::vector<View> views;
  std::vector<int32_t> wave_ptr;            // nwaves + 1 into steps
  std::vector<Item> rot, trsm;
  std::vector<int32_t> rot_ptr, trsm_ptr;   // nwaves + 1
  std::vector<Pair> pairs;
  std::vector<int32_t> pair_ptr;            // nwaves + 1
  std::vector<Trans> trans;                 // copies into the next level

  int32_t slot_of(int32_t p, int32_t q) const;   // -1 when absent
};

struct Analysis {
  int64_t n = 0;
  int32_t ndim = 0;
  int32_t order_kind = 1;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col_idx;
  std::vector<int32_t> perm, iperm, block_ptr;
  std::vector<LevelSym> levels;             // until one block is left
  std::vector<int64_t> a0_dst;              // per CSR entry: level-1 arena index or -1
  std::vector<int64_t> diag_pos;            // CSR position of A_ii, per row
  std::vector<int64_t> level1_slot_off;     // nslots + 1 (level-1 sizes are known)
};

// Returns an empty string on success, else the error message.
// Nested bisection of a general sparse graph (both triangles, diagonal
// allowed): every part is split into halves by the breadth-first order from a
// pseudo-peripheral vertex of the part, to a uniform depth so that the leaves
// have at most B vertices; leaves in depth-first order are the blocks, and
// the two halves of a part are consecutive, so coarsening by pairs (J = 2)
// follows the bisection tree.
std::string graph_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t B,
                        std::vector<int32_t>& perm, std::vector<int32_t>& block_ptr);
std::string grid_order(int32_t ndim, const int32_t* dims, const int32_t* patch,
                       std::vector<int32_t>& perm, std::vector<int32_t>& block_ptr,
                       std::vector<int32_t>& coords);

std::string analyze(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                    const int32_t* perm, const int32_t* block_ptr, int32_t nblocks,
                    int32_t B, const int32_t* coords, int32_t ndim, int32_t order_kind,
                    Analysis& out, int32_t coarsen_kind = 0);

}  // namespace cae
