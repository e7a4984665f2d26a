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

// One problem of a batch: a matrix on a tensor grid of ndim (2 or 3)
// dimensions, unknowns numbered with the first axis fastest, level-1 blocks
// are patches of the given shape (all zero: 8 x 8 or 4 x 4 x 4).
struct BatchProblem {
  int64_t n = 0;
  const int64_t* row_ptr = nullptr;   // n + 1 (row_ptr[0] may be nonzero)
  const int32_t* col_idx = nullptr;
  int32_t ndim = 0;
  int32_t dims[3] = {0, 0, 0};
  int32_t patch[3] = {0, 0, 0};
};
// The joint block-diagonal problem of a batch: problem t's rows follow those
// of problems 0..t-1 (row_off, nprob + 1 entries), its Morton patch order is
// kept, and its block coordinates (3 per block) are offset by t's binary
// digits dealt to the three axes in turn above kBatchCoordBits bits, so the
// joint Morton order runs problem by problem and the coarsening never joins
// blocks of two problems before each is one block.  Returns an empty string,
// or an error that names the problem.
constexpr int kBatchCoordBits = 8;
std::string batch_assemble(int32_t nprob, const BatchProblem* probs, std::vector<int64_t>& row_off,
                           std::vector<int64_t>& row_ptr, std::vector<int32_t>& col_idx,
                           std::vector<int32_t>& perm, std::vector<int32_t>& block_ptr,
                           std::vector<int32_t>& coords);

}  // namespace cae
