// Internal structures shared by the host runtime and the HIP kernels.
//
// Storage model of one level (the in-place factor layout):
//   * every block pair (p, q) that holds a close block or a far block, and
//     every diagonal block, owns one "slot" of the level arena: a dense
//     row-major b_p x b_q array with p <= q (rows of the lower index);
//     diagonal slots are 0..M-1, pair slots follow in (p, q) order;
//   * the coordinates of block i are rotated by U_i at its step (eq. (q)),
//     its basis is the leading r_i unknowns, the eliminated sub-row S_i the
//     trailing n_i = b_i - r_i (eq. (sm_L));
//   * after the step, the rows n_i of every view (i, c), c close, hold the
//     factor panel L(c, n_i)^T, and the n_i x n_i trailing part of the
//     diagonal slot holds the Cholesky factor of S_ii (lower triangle);
//     later rotations of block c then rotate the stored factor rows of c,
//     as eq. (big_L) requires;
//   * far views lose their rows n_i at the step (E_i dropped).
#pragma once
#include <cstdint>

namespace cae {

// Block (i, x) seen from row block i: a b_i x b_x matrix stored in slot
// `slot`, transposed when the slot is stored with the rows of x.
struct View {
  int32_t slot;
  int32_t x;       // neighbour block
  int32_t trans;   // 1: slot rows are x (view = slot^T)
  int32_t proc;    // x is processed before this step (live width r_x)
};

struct Step {
  int32_t blk;     // block i
  int32_t nclose;  // close views [view0, view0 + nclose)
  int32_t nfar;    // far views [view0 + nclose, view0 + nclose + nfar)
  int32_t view0;
};

// A step-local work item (rotation / triangular solve): view = -1 is the
// diagonal block.
struct Item {
  int32_t step;
  int32_t view;
};

// Schur-complement target of a step: panel indices a <= c, 0 = basis of the
// step's block, k > 0 = close view k-1.  For a, c > 0 the target is slot
// `slot`, stored with the rows of x_c when trans = 1.
struct Pair {
  int32_t step;
  int32_t a;
  int32_t c;
  int32_t slot;
  int32_t trans;
};

// Copy of the basis part of a slot (p, q), p <= q, into the next level.
struct Trans {
  int32_t src_slot;
  int32_t p;
  int32_t q;
  int32_t dst_slot;
};

}  // namespace cae
