// Runtime and C ABI of the compress-and-eliminate preconditioner.
//
// The host drives the levels of Algorithm 1: per level it uploads the sizes
// that depend on the ranks of the previous level (one device-to-host copy of
// the ranks per level is the only synchronisation of the factorization),
// launches the dependency waves of Algorithm 2, and gathers the basis parts of
// 2^d siblings into the next level.  The dense remainder is inverted on the
// device.  Apply, product and PCG run entirely on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cae.h"
#include "kernels.h"
#include "symbolic.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(call)                                         \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) throw HipError{e_, #call};         \
  } while (0)

// Device blocks are cached instead of freed: a factorization allocates its
// level arenas, bases and vectors again every time it runs, and hipMalloc /
// hipFree of hundreds of MB cost milliseconds and synchronise the device.  A
// released block is kept with the stream it was last used on; a later request
// on another stream first waits for that stream.  When hipMalloc fails the
// cache is emptied and the allocation retried.
thread_local hipStream_t g_cur_stream = nullptr;

struct BlockCache {
  struct Blk {
    void* p;
    hipStream_t s;
  };
  std::mutex mu;
  std::multimap<size_t, Blk> free_blocks;
  size_t cached = 0;

  void* get(size_t& bytes) {
    {
      std::lock_guard<std::mutex> g(mu);
      auto it = free_blocks.lower_bound(bytes);
      if (it != free_blocks.end() && it->first <= 2 * bytes + (1u << 20)) {
        Blk b = it->second;
        bytes = it->first;
        cached -= it->first;
        free_blocks.erase(it);
        if (b.s != g_cur_stream) (void)hipStreamSynchronize(b.s);
        return b.p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      HIPCHK(hipMalloc(&p, bytes));
    }
    return p;
  }
  void put(void* p, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    free_blocks.emplace(bytes, Blk{p, g_cur_stream});
    cached += bytes;
  }
  void trim() {
    std::lock_guard<std::mutex> g(mu);
    (void)hipDeviceSynchronize();
    for (auto& kv : free_blocks) (void)hipFree(kv.second.p);
    free_blocks.clear();
    cached = 0;
  }
};

BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();   // lives until the process ends
  return *c;
}

// A caller-provided device arena (cae_options_t.workspace) of one numeric
// factorization: while it is installed on the thread, device buffers are
// carved from it in allocation order (256-byte aligned) instead of taken from
// the block cache, and releasing a carved buffer gives nothing back (the
// arena belongs to the caller).  In counting mode (cae_workspace_query) the
// buffers come from the cache as usual and `used` adds up what the carves
// would have taken, so a factorization of the same values in an arena of that
// size carves exactly the same sequence.
struct Carver {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool counting = false;
};
thread_local Carver* g_carve = nullptr;

struct WorkspaceFull {
  size_t need;
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;   // capacity of the block
  size_t req = 0;     // bytes requested by the last allocation
  bool carved = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), req(o.req), carved(o.carved) {
    o.p = nullptr;
    o.bytes = o.req = 0;
    o.carved = false;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      req = o.req;
      carved = o.carved;
      o.p = nullptr;
      o.bytes = o.req = 0;
      o.carved = false;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p && !carved) block_cache().put(p, bytes);
    p = nullptr;
    bytes = req = 0;
    carved = false;
  }
  void alloc(size_t b) {
    if (b == 0) b = 8;
    // (inside a factorization with an arena, or counting for one, a buffer is
    // reused only up to the size it was requested with, as a carve would be)
    if (p && b <= (g_carve ? req : bytes)) return;
    release();
    const size_t a = (b + 255) & ~(size_t)255;
    if (g_carve && !g_carve->counting) {
      if (g_carve->used + a > g_carve->cap) throw WorkspaceFull{g_carve->used + a};
      p = g_carve->base + g_carve->used;
      g_carve->used += a;
      bytes = req = b;
      carved = true;
      return;
    }
    if (g_carve) g_carve->used += a;
    size_t cap = b;
    p = block_cache().get(cap);
    bytes = cap;
    req = b;
  }
  template <typename U>
  U* as() const {
    return static_cast<U*>(p);
  }
};

// Optional check for reads of memory that no kernel has written (environment
// CAE_DEBUG_POISON=1): floating-point work buffers are filled with all-ones
// bytes (NaN in FP32 and FP64) when they are handed out, so such a read shows
// up as NaN in the results instead of depending on what the block held before.
void poison(DevBuf& d, hipStream_t s) {
  static const bool on = getenv("CAE_DEBUG_POISON") != nullptr;
  if (on && d.p) HIPCHK(hipMemsetAsync(d.p, 0xFF, d.bytes, s));
}

template <typename U>
void upload(DevBuf& d, const std::vector<U>& h, hipStream_t s) {
  d.alloc(h.size() * sizeof(U));
  if (!h.empty()) HIPCHK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(U), hipMemcpyHostToDevice, s));
}

// A pinned host buffer of this thread for the factorization's small
// read-backs (grown on demand; every read-back is waited for before the
// buffer is used again; kept until the process ends, when the runtime that
// would free it may already be gone).
char* pinned_readback(size_t bytes) {
  struct Pinned {
    char* p = nullptr;
    size_t cap = 0;
  };
  static thread_local Pinned pb;
  if (bytes > pb.cap) {
    if (pb.p) HIPCHK(hipHostFree(pb.p));
    pb.p = nullptr;
    pb.cap = 0;
    const size_t cap = std::max<size_t>(bytes, (size_t)1 << 20);
    HIPCHK(hipHostMalloc((void**)&pb.p, cap, hipHostMallocDefault));
    pb.cap = cap;
  }
  return pb.p;
}

void init_device_limits() {
  static bool done = false;
  if (done) return;
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0) {
    // leave room for the static LDS of the kernels
    cae::set_max_lds_bytes((size_t)lds > 8192 ? (size_t)lds - 4096 : (size_t)lds);
  }
  done = true;
}

struct DevLevelSym {
  DevBuf steps, views, rot, trsm, pairs, trans, slot_p, slot_q, parent;
};

}  // namespace

struct cae_analysis_s {
  cae::Analysis a;
  std::vector<int64_t> batch_off;   // first row of every problem of a batch (empty: one problem)
  bool uploaded = false;
  std::vector<DevLevelSym> dlev;
  DevBuf row_ptr, col_idx, perm, a0_dst, diag_pos;
};

namespace {

struct NumLevel {
  int32_t M = 0, bmax = 0;
  int64_t dim = 0;
  std::vector<int32_t> sizes, ranks;
  std::vector<double> drops;   // ||E_i||_F^2 per block
  std::vector<int64_t> slot_off, u_off, dof_off;
  std::vector<int32_t> off_in_parent;
  std::vector<cae::WaveRange> waves;
  DevBuf arena, U, Li, bsz, d_slot_off, d_u_off, d_dof_off, d_off_in_parent, rank, edrop, minpiv;
  DevBuf need_exact;   // learned ranks: steps the exact compression takes
  DevBuf big_fail;     // steps left to a later compression pass
  DevBuf lwidth;       // LEARNED_CAP: the MLP's width of every step
  double end_ms = 0;   // host time since the factorization began when the level's ranks were back
};

}  // namespace

struct cae_factor_s {
  // (declared first, destroyed last: the analysis of a one-call cae_factor)
  std::unique_ptr<cae_analysis_s> owned_an;
  cae_analysis_t an = nullptr;
  int precision = 0;
  size_t esize = 8;
  cae_options_t opt{};
  hipStream_t stream = nullptr;
  std::vector<NumLevel> lev;      // lev[0..K]; lev[K] is the dense remainder
  int32_t K = 0;                  // factored levels
  int64_t coarse_dim = 0;
  DevBuf Ainv, Acopy, vals, theta, err, gscratch, gj_p, gj_w, gj_r, bigbuf;
  double tau = 0, dropped = 0, min_pivot = 0, factor_ms = 0;
  int64_t factor_bytes = 0;
  int32_t compress_launches = 0, compressions = 0, schur_launches = 0;
  double compress_ms = 0, compress_flops = 0, schur_ms = 0;
  double rotate_flops = 0, elim_flops = 0, schur_flops = 0, coarse_flops = 0;
  bool flops_pending = false;   // the flop counts are not yet computed
  // apply / multiply / PCG work vectors
  int32_t vec_nrhs = 0;
  std::vector<DevBuf> ybuf, wbuf, obuf;
  DevBuf ctmp;
  DevBuf apart;   // close-block products of the split backward apply
  int32_t pcg_nrhs = 0;
  DevBuf pr, pz, pp, pq, sc, act, partial;
  // a batch of independent problems: the row tiles of the per-problem PCG
  // reductions (nseg = 0 for one problem)
  DevBuf seg_tiles;
  cae::SegTiles sg{};
  DevBuf mr[7], mst;   // MINRES vectors and per-column scalars
  DevBuf lcount;       // sketches accepted / rejected
  int64_t rec_rows = 0;
  int32_t sketch_acc = 0, sketch_rej = 0;
  int32_t big_count[4] = {0, 0, 0, 0};   // big-block compressions by outcome
  // the preconditioner apply of the iterative solvers, captured once per
  // (right-hand sides, vectors) and replayed every iteration (MINRES
  // alternates two input vectors, hence a few entries)
  struct ApGraph {
    hipGraphExec_t exec = nullptr;
    int32_t uses = 0;   // eager applies with this key so far
    int32_t nrhs = 0;
    const double* r = nullptr;
    double* z = nullptr;
    int64_t ldr = 0, ldz = 0;
  };
  ApGraph ap[4];
  std::string last_err;   // message of the last failing call on this handle
  int32_t ap_next = 0;
  hipStream_t ap_stream = nullptr;   // non-blocking stream the captures run on
  cae::SideStream side;              // the diagonal blocks of big steps during the factorization
  ~cae_factor_s() {
    for (auto& g : ap)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (ap_stream) (void)hipStreamDestroy(ap_stream);
    if (side.fork) (void)hipEventDestroy(side.fork);
    if (side.join) (void)hipEventDestroy(side.join);
    if (side.s) (void)hipStreamDestroy(side.s);
  }
};

namespace {

void upload_symbolic(cae_analysis_s* A, hipStream_t s) {
  if (A->uploaded) return;
  const cae::Analysis& a = A->a;
  A->dlev.clear();
  A->dlev.resize(a.levels.size());
  for (size_t l = 0; l < a.levels.size(); ++l) {
    const cae::LevelSym& L = a.levels[l];
    DevLevelSym& D = A->dlev[l];
    upload(D.steps, L.steps, s);
    upload(D.views, L.views, s);
    upload(D.rot, L.rot, s);
    upload(D.trsm, L.trsm, s);
    upload(D.pairs, L.pairs, s);
    upload(D.trans, L.trans, s);
    upload(D.slot_p, L.slot_p, s);
    upload(D.slot_q, L.slot_q, s);
    upload(D.parent, L.parent, s);
  }
  upload(A->row_ptr, a.row_ptr, s);
  upload(A->col_idx, a.col_idx, s);
  upload(A->perm, a.perm, s);
  upload(A->a0_dst, a.a0_dst, s);
  upload(A->diag_pos, a.diag_pos, s);
  HIPCHK(hipStreamSynchronize(s));
  A->uploaded = true;
}

// Sizes of a level -> slot offsets, U offsets, unknown offsets, wave ranges.
void level_layout(const cae::LevelSym& L, NumLevel& N, size_t esize, hipStream_t s) {
  N.M = L.M;
  N.bmax = 0;
  for (int32_t b : N.sizes) N.bmax = std::max(N.bmax, b);
  N.slot_off.assign(L.nslots + 1, 0);
  for (int32_t k = 0; k < L.nslots; ++k)
    N.slot_off[k + 1] = N.slot_off[k] + (int64_t)N.sizes[L.slot_p[k]] * N.sizes[L.slot_q[k]];
  N.u_off.assign(L.M + 1, 0);
  N.dof_off.assign(L.M + 1, 0);
  for (int32_t i = 0; i < L.M; ++i) {
    N.u_off[i + 1] = N.u_off[i] + (int64_t)N.sizes[i] * N.sizes[i];
    N.dof_off[i + 1] = N.dof_off[i] + N.sizes[i];
  }
  N.dim = N.dof_off[L.M];
  N.waves.resize(L.nwaves);
  for (int32_t w = 0; w < L.nwaves; ++w) {
    int32_t mc = 0;
    for (int32_t k = L.wave_ptr[w]; k < L.wave_ptr[w + 1]; ++k) mc = std::max(mc, L.steps[k].nclose);
    N.waves[w] = cae::WaveRange{L.wave_ptr[w], L.wave_ptr[w + 1], L.rot_ptr[w], L.rot_ptr[w + 1],
                                L.trsm_ptr[w], L.trsm_ptr[w + 1], L.pair_ptr[w], L.pair_ptr[w + 1], mc};
  }
  upload(N.bsz, N.sizes, s);
  upload(N.d_slot_off, N.slot_off, s);
  upload(N.d_u_off, N.u_off, s);
  upload(N.d_dof_off, N.dof_off, s);
  N.arena.alloc((size_t)N.slot_off[L.nslots] * esize);
  HIPCHK(hipMemsetAsync(N.arena.p, 0, (size_t)N.slot_off[L.nslots] * esize, s));
}

template <typename T>
cae::LevelArgs<T> level_args(cae_factor_s* h, int l) {
  const DevLevelSym& D = h->an->dlev[l];
  NumLevel& N = h->lev[l];
  cae::LevelArgs<T> A;
  A.arena = N.arena.as<T>();
  A.slot_off = N.d_slot_off.as<int64_t>();
  A.bsz = N.bsz.as<int32_t>();
  A.U = N.U.as<T>();
  A.u_off = N.d_u_off.as<int64_t>();
  A.Li = N.Li.as<T>();
  A.rank = N.rank.as<int32_t>();
  A.edrop = N.edrop.as<double>();
  A.minpiv = N.minpiv.as<double>();
  A.steps = D.steps.as<cae::Step>();
  A.views = D.views.as<cae::View>();
  A.items = nullptr;
  A.rot = D.rot.as<cae::Item>();
  A.trsm = D.trsm.as<cae::Item>();
  A.pairs = D.pairs.as<cae::Pair>();
  A.err = h->err.as<int32_t>();
  A.theta = h->theta.as<double>();
  A.rank_mode = h->opt.rank_mode;
  A.fixed_rank = h->opt.fixed_rank;
  A.dbg = nullptr;
  A.small_by_wave = 0;
  A.mlp = nullptr;
  A.seed = 0;
  A.level = l;
  A.feat_only = 0;
  A.rec = nullptr;
  A.rec_off = 0;
  A.need_exact = nullptr;
  A.lcount = nullptr;
  A.bf16_schur = h->precision == CAE_FP32_BF16 ? 1 : 0;
  A.compensate = h->opt.compensate ? 1 : 0;
  A.big = nullptr;
  A.big_stride = 0;
  A.big_fail = nullptr;
  A.big_retry = 0;
  A.bg_cap = 128;
  A.bg_count = nullptr;
  A.lwidth = nullptr;
  return A;
}

template <typename T>
cae::ApplyArgs<T> apply_args(cae_factor_s* h, int l, int nrhs) {
  const DevLevelSym& D = h->an->dlev[l];
  NumLevel& N = h->lev[l];
  cae::ApplyArgs<T> A;
  A.arena = N.arena.as<T>();
  A.slot_off = N.d_slot_off.as<int64_t>();
  A.bsz = N.bsz.as<int32_t>();
  A.rank = N.rank.as<int32_t>();
  A.U = N.U.as<T>();
  A.u_off = N.d_u_off.as<int64_t>();
  A.Li = N.Li.as<T>();
  A.dof_off = N.d_dof_off.as<int64_t>();
  A.steps = D.steps.as<cae::Step>();
  A.views = D.views.as<cae::View>();
  A.nrhs = nrhs;
  return A;
}

template <typename T>
int factor_numeric(cae_factor_s* h, const double* vals, double eps) {
  cae_analysis_s* AN = h->an;
  const cae::Analysis& a = AN->a;
  hipStream_t s = h->stream;
  const int64_t nnz = a.row_ptr[a.n];
  auto t0 = std::chrono::steady_clock::now();
  upload_symbolic(AN, s);
  h->vals.alloc(nnz * sizeof(double));
  HIPCHK(hipMemcpyAsync(h->vals.p, vals, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  h->theta.alloc(2 * sizeof(double));
  h->err.alloc(2 * sizeof(int32_t));
  HIPCHK(hipMemsetAsync(h->err.p, 0, 2 * sizeof(int32_t), s));
  h->lcount.alloc(6 * sizeof(int32_t));   // sketches accepted / rejected, big-block outcomes
  HIPCHK(hipMemsetAsync(h->lcount.p, 0, 6 * sizeof(int32_t), s));
  h->rec_rows = 0;
  cae::launch_theta(h->vals.as<double>(), AN->diag_pos.as<int64_t>(), a.n, eps, h->theta.as<double>(), s);

  h->lev.clear();
  h->lev.reserve(a.levels.size());
  h->lev.emplace_back();
  {
    NumLevel& N = h->lev[0];
    N.sizes.resize(a.levels[0].M);
    for (int32_t b = 0; b < a.levels[0].M; ++b) N.sizes[b] = a.block_ptr[b + 1] - a.block_ptr[b];
    level_layout(a.levels[0], N, sizeof(T), s);
    cae::launch_scatter_a0<T>(N.arena.as<T>(), h->vals.as<double>(), AN->a0_dst.as<int64_t>(), nnz, s);
  }
  double dropped = 0.0, minpiv = 1e300;
  int l = 0;
  while (true) {
    const cae::LevelSym& L = a.levels[l];
    NumLevel& N = h->lev[l];
    const bool stop = L.M <= 1 || N.dim <= h->opt.coarse_max_dim ||
                      (h->opt.max_levels > 0 && l >= h->opt.max_levels) || l + 1 >= (int)a.levels.size();
    if (stop) break;
    N.U.alloc((size_t)N.u_off[L.M] * sizeof(T));
    N.Li.alloc((size_t)N.u_off[L.M] * sizeof(T));
    N.rank.alloc((size_t)L.M * sizeof(int32_t));
    N.edrop.alloc((size_t)L.M * sizeof(double));
    poison(N.U, s);
    poison(N.Li, s);
    poison(N.edrop, s);
    N.minpiv.alloc((size_t)L.M * sizeof(double));
    cae::launch_fill(N.minpiv.as<double>(), L.M, 1e300, s);
    // per-workgroup global scratch when a kernel's operands exceed the LDS
    size_t maxitems = 0;
    for (auto& w : N.waves)
      maxitems = std::max({maxitems, (size_t)(w.s1 - w.s0), (size_t)(w.r1 - w.r0), (size_t)(w.t1 - w.t0),
                           (size_t)(w.p1 - w.p0)});
    T* gs = nullptr;
    if (cae::factor_needs_global<T>(N.bmax)) {
      maxitems = std::min(maxitems, (size_t)cae::scratch_group<T>(N.bmax));
      h->gscratch.alloc(maxitems * cae::factor_scratch_elems<T>(N.bmax) * sizeof(T));
      poison(h->gscratch, s);
      gs = h->gscratch.as<T>();
    }
    cae::LevelArgs<T> A = level_args<T>(h, l);
    // steps left to a later compression pass (big blocks, learned caps)
    N.big_fail.alloc((size_t)L.M * sizeof(int32_t));
    HIPCHK(hipMemsetAsync(N.big_fail.p, 0, (size_t)L.M * sizeof(int32_t), s));
    A.big_fail = N.big_fail.as<int32_t>();
    if (N.bmax > 64) {
      // big-block scratch (compression, rotation of the diagonal blocks,
      // elimination): the steps of the largest wave
      size_t wmax = 0;
      for (auto& w : N.waves) wmax = std::max(wmax, (size_t)(w.s1 - w.s0));
      const int64_t stride = cae::bg_stride(std::min(N.bmax, 512));
      h->bigbuf.alloc(wmax * (size_t)stride * sizeof(double));
      A.big = h->bigbuf.as<double>();
      A.big_stride = stride;
      A.bg_cap = h->opt.big_pivot_cap > 0 ? h->opt.big_pivot_cap : 128;
      A.bg_count = h->lcount.as<int32_t>() + 2;
      if (!h->side.s) {
        // (default priority, no implicit synchronization with the null stream)
        HIPCHK(hipStreamCreateWithFlags(&h->side.s, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&h->side.fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->side.join, hipEventDisableTiming));
      }
    }
    if (h->opt.rank_mode == CAE_RANK_LEARNED_CAP) {
      N.lwidth.alloc((size_t)L.M * sizeof(int32_t));
      A.lwidth = N.lwidth.as<int32_t>();
      A.mlp = h->opt.mlp_params;
      A.lcount = h->lcount.as<int32_t>();
      A.rank_mode = 0;   // the kept rank is the threshold rank
    }
    if (h->opt.rank_mode == CAE_RANK_LEARNED || h->opt.record) {
      N.need_exact.alloc((size_t)L.M * sizeof(int32_t));
      A.need_exact = N.need_exact.as<int32_t>();
      A.lcount = h->lcount.as<int32_t>();
      A.seed = h->opt.seed;
      if (h->opt.rank_mode == CAE_RANK_LEARNED) {
        A.mlp = h->opt.mlp_params;
        A.rank_mode = 0;   // the kept rank is the threshold rank of the sketch
      }
      if (h->opt.record) {
        if (h->rec_rows + L.M > h->opt.record_cap) return fail(CAE_EINVAL, "record buffer too small");
        A.rec = h->opt.record;
        A.rec_off = h->rec_rows;
        A.feat_only = h->opt.rank_mode == CAE_RANK_LEARNED ? 0 : 1;
        h->rec_rows += L.M;
      }
    }
    // optional compression counters (environment CAE_DEBUG_COMPRESS=1)
    static const bool dbg_on = getenv("CAE_DEBUG_COMPRESS") != nullptr;
    DevBuf dbgbuf;
    if (dbg_on) {
      dbgbuf.alloc((size_t)72 * L.M * sizeof(int64_t));
      HIPCHK(hipMemsetAsync(dbgbuf.p, 0, (size_t)72 * L.M * sizeof(int64_t), s));
      A.dbg = dbgbuf.as<int64_t>();
    }
    std::vector<hipEvent_t> evs, sevs;
    // (CAE_VERBOSE=2: a progress line every 8 waves, each after the wave has run)
    static const bool wave_verbose = getenv("CAE_VERBOSE") && getenv("CAE_VERBOSE")[0] == '2';
    int wave_no = 0;
    for (auto& w : N.waves) {
      if (h->opt.timing && w.s1 > w.s0) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s));
        cae::launch_wave_compress<T>(A, w, N.bmax, gs, s);
        HIPCHK(hipEventRecord(e1, s));
        evs.push_back(e0);
        evs.push_back(e1);
      } else {
        cae::launch_wave_compress<T>(A, w, N.bmax, gs, s);
      }
      HIPCHK(cae::launch_wave_rest<T>(A, w, N.bmax, gs, s, &h->side));
      if (h->opt.timing && w.p1 > w.p0) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s));
        cae::launch_wave_schur<T>(A, w, N.bmax, gs, s);
        HIPCHK(hipEventRecord(e1, s));
        sevs.push_back(e0);
        sevs.push_back(e1);
      } else {
        cae::launch_wave_schur<T>(A, w, N.bmax, gs, s);
      }
      if (wave_verbose && (++wave_no % 8 == 0 || wave_no == (int)N.waves.size())) {
        HIPCHK(hipStreamSynchronize(s));
        fprintf(stderr, "[cae] level %d: wave %d/%zu done, %.1f ms\n", l + 1, wave_no, N.waves.size(),
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
      }
    }
    HIPCHK(hipGetLastError());
    if (dbg_on) {
      std::vector<int64_t> hd((size_t)72 * L.M);
      HIPCHK(hipMemcpyAsync(hd.data(), dbgbuf.p, hd.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double sum[8] = {0}, mx[8] = {0};
      int cnt = 0;
      int worst = -1;
      double bsum[8] = {0}, bmx[8] = {0}, bs_sum = 0.0;
      int bcnt = 0;
      for (int32_t b2 = 0; b2 < L.M; ++b2) {
        if (hd[72 * b2 + 3] == 0) continue;
        if (hd[72 * b2 + 3] > 128) {
          // big-block compression: ma, truncated (+2 certificate), phase cycles
          ++bcnt;
          for (int k = 0; k < 8; ++k) {
            bsum[k] += (double)hd[72 * b2 + k];
            bmx[k] = std::max(bmx[k], (double)hd[72 * b2 + k]);
          }
          bs_sum += (double)hd[72 * b2 + 8];
          continue;
        }
        ++cnt;
        for (int k = 0; k < 8; ++k) {
          sum[k] += (double)hd[72 * b2 + k];
          mx[k] = std::max(mx[k], (double)hd[72 * b2 + k]);
        }
        if (worst < 0 || hd[72 * b2 + 1] > hd[72 * worst + 1]) worst = b2;
      }
      if (worst >= 0) {
        const double* sv = reinterpret_cast<const double*>(&hd[72 * worst + 8]);
        fprintf(stderr, "[cae] worst block %d: ma %lld sweeps %lld b %lld w %lld sigma:", worst,
                (long long)hd[72 * worst], (long long)hd[72 * worst + 1], (long long)hd[72 * worst + 3],
                (long long)hd[72 * worst + 2]);
        for (int k = 0; k < std::min<int64_t>(hd[72 * worst], 64); ++k) fprintf(stderr, " %.3g", sv[k]);
        fprintf(stderr, "\n");
      }
      if (cnt)
        fprintf(stderr,
                "[cae] level %d: %d compressions | ma %.1f/%.0f sweeps %.1f/%.0f w %.0f/%.0f b %.0f | cycles "
                "qr %.0f/%.0f compact %.0f/%.0f jacobi %.0f/%.0f basis %.0f/%.0f\n",
                l + 1, cnt, sum[0] / cnt, mx[0], sum[1] / cnt, mx[1], sum[2] / cnt, mx[2], sum[3] / cnt,
                sum[4] / cnt, mx[4], sum[5] / cnt, mx[5], sum[6] / cnt, mx[6], sum[7] / cnt, mx[7]);
      if (bcnt)
        fprintf(stderr,
                "[cae] level %d: %d big compressions | ma %.1f/%.0f b %.0f/%.0f sweeps %.1f/%.0f | cycles chol "
                "%.0f/%.0f eig %.0f/%.0f (X X^T %.0f) checks+dirs %.0f/%.0f basis %.0f/%.0f\n",
                l + 1, bcnt, bsum[0] / bcnt, bmx[0], bsum[3] / bcnt, bmx[3], bsum[2] / bcnt, bmx[2], bsum[4] / bcnt,
                bmx[4], bsum[5] / bcnt, bmx[5], bs_sum / bcnt, bsum[6] / bcnt, bmx[6], bsum[7] / bcnt, bmx[7]);
    }
    // the ranks decide the sizes of the next level (read back through pinned
    // memory: a copy into pageable memory costs a staged transfer each)
    N.ranks.resize(L.M);
    int32_t herr[2];
    char* pin = pinned_readback((size_t)L.M * (sizeof(int32_t) + 2 * sizeof(double)) + 2 * sizeof(int32_t));
    double* ed = reinterpret_cast<double*>(pin);
    double* mp = ed + L.M;
    int32_t* hr = reinterpret_cast<int32_t*>(mp + L.M);
    int32_t* he = hr + L.M;
    HIPCHK(hipMemcpyAsync(hr, N.rank.p, L.M * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ed, N.edrop.p, L.M * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(mp, N.minpiv.p, L.M * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(he, h->err.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::copy(hr, hr + L.M, N.ranks.begin());
    for (int32_t i = 0; i < L.M; ++i)
      if (N.ranks[i] < 0 || N.ranks[i] > N.sizes[i]) {
        char buf[160];
        snprintf(buf, sizeof buf, "internal: rank %d of block %d (size %d) at level %d was not computed", N.ranks[i],
                 i, N.sizes[i], l + 1);
        return fail(CAE_EDEVICE, buf);
      }
    herr[0] = he[0];
    herr[1] = he[1];
    if (herr[0]) {
      char buf[160];
      snprintf(buf, sizeof buf, "non-SPD pivot block at level %d, block %d", l + 1, herr[1]);
      return fail(CAE_ENOTSPD, buf);
    }
    N.drops.assign(ed, ed + L.M);
    for (int32_t i = 0; i < L.M; ++i) {
      dropped += ed[i];
      minpiv = std::min(minpiv, mp[i]);
    }
    N.end_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // optional progress report per level (environment CAE_VERBOSE=1)
    static const bool verbose = getenv("CAE_VERBOSE") != nullptr;
    if (verbose) {
      int64_t rs = 0;
      for (int32_t i = 0; i < L.M; ++i) rs += N.ranks[i];
      fprintf(stderr, "[cae] level %d: %d blocks, b max %d, dim %lld -> %lld kept, %d waves, %.1f ms\n", l + 1, L.M,
              N.bmax, (long long)N.dim, (long long)rs, L.nwaves,
              std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    if (h->opt.timing) {
      for (size_t k = 0; k < evs.size(); k += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, evs[k], evs[k + 1]));
        h->compress_ms += ms;
        h->compress_launches += 1;
        (void)hipEventDestroy(evs[k]);
        (void)hipEventDestroy(evs[k + 1]);
      }
      for (size_t k = 0; k < sevs.size(); k += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, sevs[k], sevs[k + 1]));
        h->schur_ms += ms;
        h->schur_launches += 1;
        (void)hipEventDestroy(sevs[k]);
        (void)hipEventDestroy(sevs[k + 1]);
      }
    }
    h->lev.emplace_back();
    NumLevel& Nn = h->lev[l + 1];
    NumLevel& Nc = h->lev[l];
    Nn.sizes.assign(L.Mnext, 0);
    Nc.off_in_parent.assign(L.M, 0);
    for (int32_t c = 0; c < L.M; ++c) {
      Nc.off_in_parent[c] = Nn.sizes[L.parent[c]];
      Nn.sizes[L.parent[c]] += Nc.ranks[c];
    }
    upload(Nc.d_off_in_parent, Nc.off_in_parent, s);
    level_layout(a.levels[l + 1], Nn, sizeof(T), s);
    const DevLevelSym& D = AN->dlev[l];
    cae::launch_gather_next<T>(D.trans.as<cae::Trans>(), (int32_t)L.trans.size(), Nc.arena.as<T>(),
                               Nc.d_slot_off.as<int64_t>(), Nc.bsz.as<int32_t>(), Nc.rank.as<int32_t>(),
                               D.parent.as<int32_t>(), Nc.d_off_in_parent.as<int32_t>(), Nn.arena.as<T>(),
                               Nn.d_slot_off.as<int64_t>(), Nn.bsz.as<int32_t>(), s);
    ++l;
  }
  h->K = l;
  // dense remainder: assemble, keep a copy for the product, invert in place
  NumLevel& N = h->lev[l];
  const cae::LevelSym& L = a.levels[l];
  const int64_t dim = N.dim;
  h->coarse_dim = dim;
  if (dim > 0) {
    h->Ainv.alloc((size_t)dim * dim * sizeof(double));
    h->Acopy.alloc((size_t)dim * dim * sizeof(double));
    HIPCHK(hipMemsetAsync(h->Ainv.p, 0, (size_t)dim * dim * sizeof(double), s));
    const DevLevelSym& D = AN->dlev[l];
    cae::launch_coarse_assemble<T>(D.slot_p.as<int32_t>(), D.slot_q.as<int32_t>(), L.nslots, N.arena.as<T>(),
                                   N.d_slot_off.as<int64_t>(), N.bsz.as<int32_t>(), N.d_dof_off.as<int64_t>(),
                                   h->Ainv.as<double>(), dim, s);
    HIPCHK(hipMemcpyAsync(h->Acopy.p, h->Ainv.p, (size_t)dim * dim * sizeof(double), hipMemcpyDeviceToDevice, s));
    h->gj_p.alloc(2 * 64 * 64 * sizeof(double));   // two pivot inverses (this panel's, the next one's)
    h->gj_w.alloc((size_t)64 * dim * sizeof(double));
    h->gj_r.alloc((size_t)64 * dim * sizeof(double));
    poison(h->gj_p, s);
    poison(h->gj_w, s);
    poison(h->gj_r, s);
    cae::launch_gj_inverse(h->Ainv.as<double>(), dim, h->gj_p.as<double>(), h->gj_w.as<double>(),
                           h->gj_r.as<double>(), h->err.as<int32_t>(), s);
    HIPCHK(hipGetLastError());
  }
  // error flag and threshold through the pinned read-back buffer
  char* pin = pinned_readback(2 * sizeof(double) + 2 * sizeof(int32_t));
  double* th = reinterpret_cast<double*>(pin);
  int32_t* herr = reinterpret_cast<int32_t*>(th + 2);
  HIPCHK(hipMemcpyAsync(herr, h->err.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(th, h->theta.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr[0]) {
    char buf[160];
    snprintf(buf, sizeof buf, "non-SPD pivot in the dense remainder (dimension %lld, flag %d, block %d)",
             (long long)dim, herr[0], herr[1]);
    return fail(CAE_ENOTSPD, buf);
  }
  h->tau = th[1];
  h->dropped = dropped;
  h->min_pivot = minpiv;
  int64_t bytes = 0;
  for (int k = 0; k < h->K; ++k)
    bytes += (h->lev[k].slot_off.back() + h->lev[k].u_off.back()) * (int64_t)sizeof(T);
  bytes += dim * dim * (int64_t)sizeof(double);
  h->factor_bytes = bytes;
  {
    int32_t* lc = reinterpret_cast<int32_t*>(pinned_readback(6 * sizeof(int32_t)));
    HIPCHK(hipMemcpyAsync(lc, h->lcount.p, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->sketch_acc = lc[0];
    h->sketch_rej = lc[1];
    for (int k = 0; k < 4; ++k) h->big_count[k] = lc[2 + k];
  }
  h->factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // (the algorithmic flop counts are computed when the statistics are read,
  // outside the factorization)
  h->flops_pending = true;
  return CAE_OK;
}

// The captured solver applies bake in the addresses of the work vectors:
// whenever those are released and allocated again, every graph is dropped
// (the next solver apply runs eagerly and captures afresh).
void drop_graphs(cae_factor_s* h) {
  for (auto& g : h->ap) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = cae_factor_s::ApGraph{};
  }
  h->ap_next = 0;
}

void ensure_vectors(cae_factor_s* h, int32_t nrhs) {
  if (h->vec_nrhs >= nrhs && (int)h->ybuf.size() == h->K + 1) return;
  drop_graphs(h);
  h->ybuf.clear();
  h->wbuf.clear();
  h->obuf.clear();
  h->ybuf.resize(h->K + 1);
  h->wbuf.resize(h->K + 1);
  h->obuf.resize(h->K + 1);
  for (int l = 0; l <= h->K; ++l) {
    size_t b = (size_t)std::max<int64_t>(h->lev[l].dim, 1) * nrhs * sizeof(double);
    h->ybuf[l].alloc(b);
    h->wbuf[l].alloc(b);
    h->obuf[l].alloc(b);
    poison(h->ybuf[l], g_cur_stream);
    poison(h->wbuf[l], g_cur_stream);
    poison(h->obuf[l], g_cur_stream);
  }
  h->ctmp.alloc((size_t)std::max<int64_t>(h->coarse_dim, 1) * nrhs * sizeof(double));
  size_t part = 0;
  for (int l = 0; l < h->K; ++l)
    for (const auto& w : h->lev[l].waves)
      if (cae::ap_split<double>(w, h->lev[l].bmax, h->opt.apply_split_steps))
        part = std::max(part, cae::ap_part_elems(w, h->lev[l].bmax, nrhs));
  h->apart.release();
  if (part > 0) h->apart.alloc(part * sizeof(double));
  poison(h->ctmp, g_cur_stream);
  poison(h->apart, g_cur_stream);
  h->vec_nrhs = nrhs;
}

// Work vectors of one preconditioner apply: the level vectors y[l]
// (dim_l x nrhs, l = 0..K), the coarse product (coarse_dim x nrhs) and the
// partial products of the split backward pass (ap_part_elems of the largest
// split wave).  Every entry the apply reads has been written by it first.
struct ApplyBufs {
  double* const* y;
  double* ctmp;
  double* apart;
};

template <typename T>
void apply_precond(cae_factor_s* h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz,
                   const ApplyBufs& B, hipStream_t s) {
  const cae::Analysis& a = h->an->a;
  cae::launch_perm_in(a.n, nrhs, h->an->perm.as<int32_t>(), r, ldr, B.y[0], s);
  for (int l = 0; l < h->K; ++l) {
    NumLevel& N = h->lev[l];
    const cae::LevelSym& L = a.levels[l];
    auto A = apply_args<T>(h, l, nrhs);
    double* y = B.y[l];
    cae::launch_ap_rotate<T>(A, L.M, y, 0, N.bmax, s);
    for (auto& w : N.waves) cae::launch_ap_fwd<T>(A, w, y, N.bmax, h->opt.apply_split_steps, s);
    cae::launch_to_next(L.M, N.d_dof_off.as<int64_t>(), N.rank.as<int32_t>(), h->an->dlev[l].parent.as<int32_t>(),
                        N.d_off_in_parent.as<int32_t>(), h->lev[l + 1].d_dof_off.as<int64_t>(), nrhs, y, B.y[l + 1],
                        0, s);
  }
  const int64_t dim = h->coarse_dim;
  if (dim > 0) {
    cae::launch_coarse_apply(h->Ainv.as<double>(), dim, nrhs, B.y[h->K], B.ctmp, s);
    cae::launch_copy_cols(dim * nrhs, 1, B.ctmp, dim * nrhs, B.y[h->K], dim * nrhs, s);
  }
  for (int l = h->K - 1; l >= 0; --l) {
    NumLevel& N = h->lev[l];
    const cae::LevelSym& L = a.levels[l];
    auto A = apply_args<T>(h, l, nrhs);
    double* y = B.y[l];
    cae::launch_to_next(L.M, N.d_dof_off.as<int64_t>(), N.rank.as<int32_t>(), h->an->dlev[l].parent.as<int32_t>(),
                        N.d_off_in_parent.as<int32_t>(), h->lev[l + 1].d_dof_off.as<int64_t>(), nrhs, y, B.y[l + 1],
                        1, s);
    for (int w = (int)N.waves.size() - 1; w >= 0; --w)
      cae::launch_ap_bwd<T>(A, N.waves[w], y, N.bmax, B.apart, h->opt.apply_split_steps, s);
    cae::launch_ap_rotate<T>(A, L.M, y, 1, N.bmax, s);
  }
  cae::launch_perm_out(a.n, nrhs, h->an->perm.as<int32_t>(), B.y[0], z, ldz, s);
  HIPCHK(hipGetLastError());
}

template <typename T>
void apply_factor(cae_factor_s* h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy) {
  hipStream_t s = h->stream;
  const cae::Analysis& a = h->an->a;
  ensure_vectors(h, nrhs);
  cae::launch_perm_in(a.n, nrhs, h->an->perm.as<int32_t>(), x, ldx, h->ybuf[0].as<double>(), s);
  for (int l = 0; l < h->K; ++l) {
    NumLevel& N = h->lev[l];
    const cae::LevelSym& L = a.levels[l];
    auto A = apply_args<T>(h, l, nrhs);
    double* z = h->ybuf[l].as<double>();
    cae::launch_ap_rotate<T>(A, L.M, z, 0, N.bmax, s);
    cae::launch_mul_w<T>(A, L.M, z, h->wbuf[l].as<double>(), N.bmax, s);
    cae::launch_to_next(L.M, N.d_dof_off.as<int64_t>(), N.rank.as<int32_t>(), h->an->dlev[l].parent.as<int32_t>(),
                        N.d_off_in_parent.as<int32_t>(), h->lev[l + 1].d_dof_off.as<int64_t>(), nrhs, z,
                        h->ybuf[l + 1].as<double>(), 0, s);
  }
  const int64_t dim = h->coarse_dim;
  if (dim > 0)
    cae::launch_coarse_mul(h->Acopy.as<double>(), dim, nrhs, h->ybuf[h->K].as<double>(), h->obuf[h->K].as<double>(), s);
  for (int l = h->K - 1; l >= 0; --l) {
    NumLevel& N = h->lev[l];
    const cae::LevelSym& L = a.levels[l];
    auto A = apply_args<T>(h, l, nrhs);
    double* out = h->obuf[l].as<double>();
    cae::launch_fill(out, N.dim * nrhs, 0.0, s);
    cae::launch_to_next(L.M, N.d_dof_off.as<int64_t>(), N.rank.as<int32_t>(), h->an->dlev[l].parent.as<int32_t>(),
                        N.d_off_in_parent.as<int32_t>(), h->lev[l + 1].d_dof_off.as<int64_t>(), nrhs, out,
                        h->obuf[l + 1].as<double>(), 1, s);
    for (auto& w : N.waves) cae::launch_mul_lw<T>(A, w.s0, w.s1, h->wbuf[l].as<double>(), out, N.bmax, s);
    cae::launch_ap_rotate<T>(A, L.M, out, 1, N.bmax, s);
  }
  cae::launch_perm_out(a.n, nrhs, h->an->perm.as<int32_t>(), h->obuf[0].as<double>(), y, ldy, s);
  HIPCHK(hipGetLastError());
}

// The apply with the handle's own work vectors, on the handle's stream.
void do_apply(cae_factor_s* h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz) {
  ensure_vectors(h, nrhs);
  std::vector<double*> y(h->K + 1);
  for (int l = 0; l <= h->K; ++l) y[l] = h->ybuf[l].as<double>();
  const ApplyBufs B{y.data(), h->ctmp.as<double>(), h->apart.as<double>()};
  if (h->precision != CAE_FP64)
    apply_precond<float>(h, nrhs, r, ldr, z, ldz, B, h->stream);
  else
    apply_precond<double>(h, nrhs, r, ldr, z, ldz, B, h->stream);
}

// The apply of an iterative solver: with cae_options_t.graphs, its kernel
// sequence is captured on a stream of its own the first time (work vectors
// allocated before, so the capture holds kernel launches only) and the graph
// is launched on the handle's stream from then on.
void solver_apply(cae_factor_s* h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz) {
  if (!h->opt.graphs) {
    do_apply(h, nrhs, r, ldr, z, ldz);
    return;
  }
  // the first applies of a key run eagerly: capturing and instantiating the
  // graph costs more than a couple of replays save (a factor used for one
  // short solve never captures)
  constexpr int32_t kEagerApplies = 3;
  ensure_vectors(h, nrhs);   // (may drop every graph: before the lookup)
  cae_factor_s::ApGraph* hit = nullptr;
  for (auto& g : h->ap)
    if (g.uses > 0 && g.nrhs == nrhs && g.r == r && g.z == z && g.ldr == ldr && g.ldz == ldz) hit = &g;
  if (!hit) {
    hit = &h->ap[h->ap_next];
    h->ap_next = (h->ap_next + 1) % 4;
    if (hit->exec) {
      HIPCHK(hipGraphExecDestroy(hit->exec));
      hit->exec = nullptr;
    }
    hit->uses = 0;
    hit->nrhs = nrhs;
    hit->r = r;
    hit->z = z;
    hit->ldr = ldr;
    hit->ldz = ldz;
  }
  if (!hit->exec && hit->uses < kEagerApplies) {
    ++hit->uses;
    do_apply(h, nrhs, r, ldr, z, ldz);
    return;
  }
  if (!hit->exec) {
    if (!h->ap_stream) HIPCHK(hipStreamCreateWithFlags(&h->ap_stream, hipStreamNonBlocking));
    hipStream_t keep = h->stream;
    h->stream = h->ap_stream;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(h->ap_stream, hipStreamCaptureModeThreadLocal));
    try {
      do_apply(h, nrhs, r, ldr, z, ldz);
    } catch (...) {
      (void)hipStreamEndCapture(h->ap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      h->stream = keep;
      throw;
    }
    h->stream = keep;
    HIPCHK(hipStreamEndCapture(h->ap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&hit->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
  }
  HIPCHK(hipGraphLaunch(hit->exec, h->stream));
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free apply (cae_apply_precond_noalloc): the level
// vectors, the coarse product and the split backward's partial products of
// one call live in this array instead of the handle's work vectors.  Every
// GPU that loads the library holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name in host code is not a device address).
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxLevels = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current device, looked up once per device.
void* noalloc_scratch() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw HipError{hipErrorInvalidDevice, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[dev] = p;
  }
  return ptr[dev];
}

// Byte layout of the allocation-free apply's work vectors for nrhs columns:
// every vector starts on a 256-byte boundary.  Returns the bytes needed.
size_t noalloc_layout(const cae_factor_s* h, int32_t nrhs, size_t* y_off, size_t* ctmp_off, size_t* part_off) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  for (int l = 0; l <= h->K; ++l) {
    y_off[l] = off;
    off = up(off + (size_t)std::max<int64_t>(h->lev[l].dim, 1) * nrhs * sizeof(double));
  }
  *ctmp_off = off;
  off = up(off + (size_t)std::max<int64_t>(h->coarse_dim, 1) * nrhs * sizeof(double));
  size_t part = 0;
  for (int l = 0; l < h->K; ++l)
    for (const auto& w : h->lev[l].waves)
      if (cae::ap_split<double>(w, h->lev[l].bmax, h->opt.apply_split_steps))
        part = std::max(part, cae::ap_part_elems(w, h->lev[l].bmax, nrhs));
  *part_off = off;
  off = up(off + part * sizeof(double));
  return off;
}

int check_handle(cae_factor_s* h) {
  if (!h) return fail(CAE_EINVAL, "null handle");
  return CAE_OK;
}

// A failing call on a handle also leaves its message with the handle.
int keep_error(cae_factor_s* h, int rc) {
  if (h && rc != CAE_OK) h->last_err = g_err;
  return rc;
}

}  // namespace

extern "C" {

void cae_default_options(cae_options_t* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = sizeof(cae_options_t);
  opt->rank_mode = CAE_RANK_EPS;
  opt->fixed_rank = 0;
  opt->precision = CAE_FP64;
  opt->order = CAE_ORDER_MULTICOLOUR;
  opt->max_levels = 0;
  opt->coarse_max_dim = 2048;
  opt->graphs = 1;
  opt->apply_split_steps = 1024;
  opt->stream = nullptr;
}

const char* cae_last_error(cae_handle_t h) { return h ? h->last_err.c_str() : g_err.c_str(); }

int cae_graph_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t B, int32_t* perm,
                    int32_t* block_ptr, int32_t* nblocks) {
  if (!row_ptr || !col_idx || !nblocks) return fail(CAE_EINVAL, "row_ptr, col_idx and nblocks are required");
  try {
    std::vector<int32_t> p, bp;
    std::string e = cae::graph_order(n, row_ptr, col_idx, B, p, bp);
    if (!e.empty()) return fail(CAE_EINVAL, e);
    *nblocks = (int32_t)bp.size() - 1;
    if (perm) std::memcpy(perm, p.data(), p.size() * sizeof(int32_t));
    if (block_ptr) std::memcpy(block_ptr, bp.data(), bp.size() * sizeof(int32_t));
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

int cae_grid_order(int32_t ndim, const int32_t* dims, const int32_t* patch, int32_t* perm, int32_t* block_ptr,
                   int32_t* coords, int32_t* nblocks) {
  if (!dims || !patch || !nblocks) return fail(CAE_EINVAL, "dims, patch and nblocks are required");
  try {
    std::vector<int32_t> p, bp, co;
    std::string e = cae::grid_order(ndim, dims, patch, p, bp, co);
    if (!e.empty()) return fail(CAE_EINVAL, e);
    *nblocks = (int32_t)bp.size() - 1;
    if (perm) std::memcpy(perm, p.data(), p.size() * sizeof(int32_t));
    if (block_ptr) std::memcpy(block_ptr, bp.data(), bp.size() * sizeof(int32_t));
    if (coords) std::memcpy(coords, co.data(), co.size() * sizeof(int32_t));
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

int cae_analyze(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* perm,
                const int32_t* block_ptr, int32_t nblocks, int32_t B, const int32_t* coords, int32_t ndim,
                const cae_options_t* opt, cae_analysis_t* out) {
  if (!out) return fail(CAE_EINVAL, "out is required");
  *out = nullptr;
  cae_options_t o;
  cae_default_options(&o);
  if (opt) {
    if (opt->struct_size != (int32_t)sizeof(cae_options_t)) return fail(CAE_EINVAL, "options struct_size mismatch");
    o = *opt;
  }
  try {
    std::unique_ptr<cae_analysis_s> A(new cae_analysis_s);
    std::string e = cae::analyze(n, row_ptr, col_idx, perm, block_ptr, nblocks, B, coords, ndim, o.order, A->a,
                                 o.coarsen);
    if (!e.empty()) return fail(CAE_EINVAL, e);
    *out = A.release();
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

int cae_analysis_levels(cae_analysis_t a, int32_t* nlevels) {
  if (!a || !nlevels) return fail(CAE_EINVAL, "null argument");
  *nlevels = (int32_t)a->a.levels.size();
  return CAE_OK;
}

int cae_analysis_level_info(cae_analysis_t a, int32_t level, cae_level_info_t* info) {
  if (!a || !info) return fail(CAE_EINVAL, "null argument");
  if (level < 0 || level >= (int32_t)a->a.levels.size()) return fail(CAE_EINVAL, "level out of range");
  const cae::LevelSym& L = a->a.levels[level];
  info->M = L.M;
  info->nclose = (int32_t)L.close_pairs.size() / 2;
  info->nfar = (int32_t)L.far_pairs.size() / 2;
  int32_t nr = 0;
  for (uint8_t r : L.removed) nr += r;
  info->nremoved = nr;
  info->nwaves = L.nwaves;
  info->Mnext = L.Mnext;
  return CAE_OK;
}

int cae_analysis_level_arrays(cae_analysis_t a, int32_t level, int32_t* order, int32_t* wave, int32_t* close_pairs,
                              int32_t* far_pairs, uint8_t* removed, int32_t* parent) {
  if (!a) return fail(CAE_EINVAL, "null analysis");
  if (level < 0 || level >= (int32_t)a->a.levels.size()) return fail(CAE_EINVAL, "level out of range");
  const cae::LevelSym& L = a->a.levels[level];
  if (order) std::memcpy(order, L.order.data(), L.order.size() * sizeof(int32_t));
  if (wave) std::memcpy(wave, L.wave.data(), L.wave.size() * sizeof(int32_t));
  if (close_pairs) std::memcpy(close_pairs, L.close_pairs.data(), L.close_pairs.size() * sizeof(int32_t));
  if (far_pairs) std::memcpy(far_pairs, L.far_pairs.data(), L.far_pairs.size() * sizeof(int32_t));
  if (removed) std::memcpy(removed, L.removed.data(), L.removed.size());
  if (parent) std::memcpy(parent, L.parent.data(), L.parent.size() * sizeof(int32_t));
  return CAE_OK;
}

int cae_analysis_perm(cae_analysis_t a, int32_t* perm, int32_t* block_ptr) {
  if (!a) return fail(CAE_EINVAL, "null analysis");
  if (perm) std::memcpy(perm, a->a.perm.data(), a->a.perm.size() * sizeof(int32_t));
  if (block_ptr) std::memcpy(block_ptr, a->a.block_ptr.data(), a->a.block_ptr.size() * sizeof(int32_t));
  return CAE_OK;
}

void cae_analysis_destroy(cae_analysis_t a) { delete a; }

}  // extern "C"

namespace {

// Options with defaults, validated against the analysis.
int checked_options(cae_analysis_t an, double eps, const cae_options_t* opt, cae_options_t& o) {
  if (!(eps >= 0.0)) return fail(CAE_EINVAL, "eps must be >= 0");
  cae_default_options(&o);
  if (opt) {
    if (opt->struct_size != (int32_t)sizeof(cae_options_t)) return fail(CAE_EINVAL, "options struct_size mismatch");
    o = *opt;
  }
  if (o.precision != CAE_FP64 && o.precision != CAE_FP32 && o.precision != CAE_FP32_BF16)
    return fail(CAE_EINVAL, "unknown precision");
  if (o.rank_mode != CAE_RANK_EPS && o.rank_mode != CAE_RANK_FIXED && o.rank_mode != CAE_RANK_LEARNED &&
      o.rank_mode != CAE_RANK_LEARNED_CAP)
    return fail(CAE_EINVAL, "unknown rank mode");
  if ((o.rank_mode == CAE_RANK_LEARNED || o.rank_mode == CAE_RANK_LEARNED_CAP) && (!o.mlp_params || !(eps > 0.0)))
    return fail(CAE_EINVAL, "learned ranks need mlp_params and eps > 0");
  if (o.rank_mode == CAE_RANK_LEARNED_CAP && o.record)
    return fail(CAE_EINVAL, "training records come from CE(eps) or LEARNED factorizations");
  if (o.record && (o.record_cap <= 0 || o.rank_mode == CAE_RANK_FIXED))
    return fail(CAE_EINVAL, "record needs record_cap > 0 and a threshold rank mode");
  if (o.rank_mode == CAE_RANK_FIXED && o.fixed_rank < 0) return fail(CAE_EINVAL, "fixed_rank must be >= 0");
  if (o.order != an->a.order_kind) return fail(CAE_EINVAL, "order differs from the analysis");
  if (o.workspace && o.workspace_bytes == 0) return fail(CAE_EINVAL, "workspace given with workspace_bytes = 0");
  if (o.big_pivot_cap < 0 || o.big_pivot_cap > 128) return fail(CAE_EINVAL, "big_pivot_cap must be in 0..128");
  return CAE_OK;
}

// The numeric factorization with validated options; `carve` installs an arena
// (or a counter) for the handle's device buffers.
// Row tiles of the per-problem PCG reductions of a batch, none straddling
// two problems.
void setup_batch(cae_factor_s* h) {
  const std::vector<int64_t>& off = h->an->batch_off;
  const int nprob = (int)off.size() - 1;
  std::vector<int64_t> tb, te;
  std::vector<int32_t> ts, sfirst(nprob + 1, 0);
  for (int t = 0; t < nprob; ++t) {
    sfirst[t] = (int32_t)tb.size();
    for (int64_t r = off[t]; r < off[t + 1]; r += cae::SEG_TILE_ROWS) {
      tb.push_back(r);
      te.push_back(std::min(off[t + 1], r + (int64_t)cae::SEG_TILE_ROWS));
      ts.push_back(t);
    }
  }
  sfirst[nprob] = (int32_t)tb.size();
  const size_t nt = tb.size();
  const size_t o_te = nt * sizeof(int64_t), o_ts = 2 * o_te, o_sf = o_ts + nt * sizeof(int32_t);
  const size_t bytes = o_sf + (nprob + 1) * sizeof(int32_t);
  std::vector<char> host(bytes);
  std::memcpy(host.data(), tb.data(), nt * sizeof(int64_t));
  std::memcpy(host.data() + o_te, te.data(), nt * sizeof(int64_t));
  std::memcpy(host.data() + o_ts, ts.data(), nt * sizeof(int32_t));
  std::memcpy(host.data() + o_sf, sfirst.data(), (nprob + 1) * sizeof(int32_t));
  h->seg_tiles.alloc(bytes);
  HIPCHK(hipMemcpyAsync(h->seg_tiles.p, host.data(), bytes, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const char* base = static_cast<const char*>(h->seg_tiles.p);
  h->sg.tb = reinterpret_cast<const int64_t*>(base);
  h->sg.te = reinterpret_cast<const int64_t*>(base + o_te);
  h->sg.ts = reinterpret_cast<const int32_t*>(base + o_ts);
  h->sg.sfirst = reinterpret_cast<const int32_t*>(base + o_sf);
  h->sg.ntiles = (int32_t)nt;
  h->sg.nseg = nprob;
}

int factor_checked(cae_analysis_t an, const double* vals, double eps, const cae_options_t& o, Carver* carve,
                   cae_handle_t* out) {
  struct Uninstall {
    ~Uninstall() { g_carve = nullptr; }
  } uninstall;
  hipStream_t stream = (hipStream_t)o.stream;
  try {
    init_device_limits();
    g_cur_stream = stream;
    // the analysis' device arrays belong to the analysis, never to an arena
    upload_symbolic(an, stream);
    g_carve = carve;
    std::unique_ptr<cae_factor_s> h(new cae_factor_s);
    h->an = an;
    h->opt = o;
    h->precision = o.precision;
    h->stream = stream;
    int rc = o.precision != CAE_FP64 ? factor_numeric<float>(h.get(), vals, eps)
                                     : factor_numeric<double>(h.get(), vals, eps);
    g_carve = nullptr;
    if (rc != CAE_OK) {
      (void)hipStreamSynchronize(h->stream);
      return rc;
    }
    if (!an->batch_off.empty()) setup_batch(h.get());
    *out = h.release();
  } catch (const WorkspaceFull& e) {
    g_carve = nullptr;
    (void)hipStreamSynchronize(stream);
    char buf[200];
    snprintf(buf, sizeof buf, "workspace of %zu bytes is too small: this factorization needs more than %zu",
             carve ? carve->cap : (size_t)0, e.need);
    return fail(CAE_ENOMEM, buf);
  } catch (const HipError& e) {
    g_carve = nullptr;
    (void)hipStreamSynchronize(stream);
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    g_carve = nullptr;
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

}  // namespace

extern "C" {

int cae_factor_numeric(cae_analysis_t an, const double* vals, double eps, const cae_options_t* opt,
                       cae_handle_t* out) {
  if (!out) return fail(CAE_EINVAL, "out is required");
  *out = nullptr;
  if (!an || !vals) return fail(CAE_EINVAL, "analysis and vals are required");
  cae_options_t o;
  if (int rc = checked_options(an, eps, opt, o)) return rc;
  if (!o.workspace) return factor_checked(an, vals, eps, o, nullptr, out);
  Carver carve;
  carve.base = static_cast<char*>(o.workspace);
  carve.cap = o.workspace_bytes;
  if ((reinterpret_cast<uintptr_t>(carve.base) & 255) != 0) return fail(CAE_EINVAL, "workspace must be 256-byte aligned");
  return factor_checked(an, vals, eps, o, &carve, out);
}

int cae_workspace_query(cae_analysis_t an, const double* vals, double eps, const cae_options_t* opt, size_t* bytes) {
  if (!an || !vals || !bytes) return fail(CAE_EINVAL, "analysis, vals and bytes are required");
  cae_options_t o;
  if (int rc = checked_options(an, eps, opt, o)) return rc;
  o.workspace = nullptr;
  o.workspace_bytes = 0;
  Carver count;
  count.counting = true;
  cae_handle_t h = nullptr;
  if (int rc = factor_checked(an, vals, eps, o, &count, &h)) return rc;
  cae_destroy(h);
  *bytes = count.used;
  return CAE_OK;
}

int cae_factor(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals, const int32_t* perm,
               const int32_t* block_ptr, int32_t nblocks, int32_t B, const int32_t* coords, int32_t ndim, double eps,
               const cae_options_t* opt, cae_handle_t* out) {
  if (!out) return fail(CAE_EINVAL, "out is required");
  *out = nullptr;
  if (!vals || !row_ptr) return fail(CAE_EINVAL, "row_ptr and vals are required");
  cae_analysis_t an = nullptr;
  if (int rc = cae_analyze(n, row_ptr, col_idx, perm, block_ptr, nblocks, B, coords, ndim, opt, &an)) return rc;
  std::unique_ptr<cae_analysis_s> own(an);
  cae_options_t o;
  if (int rc = checked_options(an, eps, opt, o)) return rc;
  try {
    g_cur_stream = (hipStream_t)o.stream;
    const int64_t nnz = row_ptr[n];
    DevBuf dv;
    dv.alloc((size_t)nnz * sizeof(double));
    HIPCHK(hipMemcpyAsync(dv.p, vals, (size_t)nnz * sizeof(double), hipMemcpyHostToDevice, (hipStream_t)o.stream));
    cae_handle_t h = nullptr;
    Carver carve;
    carve.base = static_cast<char*>(o.workspace);
    carve.cap = o.workspace_bytes;
    if (o.workspace && (reinterpret_cast<uintptr_t>(carve.base) & 255) != 0)
      return fail(CAE_EINVAL, "workspace must be 256-byte aligned");
    if (int rc = factor_checked(an, dv.as<double>(), eps, o, o.workspace ? &carve : nullptr, &h)) return rc;
    h->owned_an.reset(own.release());   // the handle owns the analysis it was made with
    *out = h;
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

// ---------------------------------------------------------------- batches ---
// Independent problems in one factorization (the joint block-diagonal
// problem of cae::batch_assemble): every dependency wave of the joint
// analysis holds the independent steps of all problems, one launch per wave
// for the batch.
namespace {
// first row and first stored entry of every problem (after
// cae::batch_assemble has validated them), and their values; CAE_OK or an error
int batch_sizes(int32_t nprob, const cae_problem_t* probs, bool need_vals, std::vector<int64_t>& row_off,
                std::vector<int64_t>& nz_off) {
  if (nprob <= 0 || !probs) return fail(CAE_EINVAL, "nprob > 0 problems are required");
  row_off.assign(nprob + 1, 0);
  nz_off.assign(nprob + 1, 0);
  for (int t = 0; t < nprob; ++t) {
    const cae_problem_t& P = probs[t];
    if (P.n <= 0 || !P.row_ptr || (need_vals && !P.vals))
      return fail(CAE_EINVAL, "problem " + std::to_string(t) + ": n > 0, row_ptr and vals are required");
    row_off[t + 1] = row_off[t] + P.n;
    nz_off[t + 1] = nz_off[t] + (P.row_ptr[P.n] - P.row_ptr[0]);
  }
  return CAE_OK;
}
}  // namespace

int cae_analyze_batched(int32_t nprob, const cae_problem_t* probs, const cae_options_t* opt, cae_analysis_t* out) {
  if (!out) return fail(CAE_EINVAL, "out is required");
  *out = nullptr;
  if (nprob <= 0 || !probs) return fail(CAE_EINVAL, "nprob > 0 problems are required");
  try {
    std::vector<cae::BatchProblem> bp(nprob);
    for (int t = 0; t < nprob; ++t) {
      bp[t].n = probs[t].n;
      bp[t].row_ptr = probs[t].row_ptr;
      bp[t].col_idx = probs[t].col_idx;
      bp[t].ndim = probs[t].ndim;
      for (int a = 0; a < 3; ++a) {
        bp[t].dims[a] = probs[t].dims[a];
        bp[t].patch[a] = probs[t].patch[a];
      }
    }
    std::vector<int64_t> row_off, rp;
    std::vector<int32_t> ci, perm, bptr, coords;
    const std::string e = cae::batch_assemble(nprob, bp.data(), row_off, rp, ci, perm, bptr, coords);
    if (!e.empty()) return fail(CAE_EINVAL, e);
    cae_analysis_t an = nullptr;
    if (int rc = cae_analyze(row_off[nprob], rp.data(), ci.data(), perm.data(), bptr.data(),
                             (int32_t)bptr.size() - 1, 0, coords.data(), 3, opt, &an))
      return rc;
    an->batch_off = row_off;
    *out = an;
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

int cae_analysis_batch_rows(cae_analysis_t a, int32_t* nprob, int64_t* row_off) {
  if (!a || !nprob) return fail(CAE_EINVAL, "analysis and nprob are required");
  if (a->batch_off.empty()) {
    *nprob = 1;
    if (row_off) {
      row_off[0] = 0;
      row_off[1] = a->a.n;
    }
    return CAE_OK;
  }
  *nprob = (int32_t)a->batch_off.size() - 1;
  if (row_off) std::memcpy(row_off, a->batch_off.data(), a->batch_off.size() * sizeof(int64_t));
  return CAE_OK;
}

int cae_factor_batched(int32_t nprob, const cae_problem_t* probs, double eps, const cae_options_t* opt,
                       cae_handle_t* out) {
  if (!out) return fail(CAE_EINVAL, "out is required");
  *out = nullptr;
  try {
    // the analysis validates every problem's structure first
    cae_analysis_t an = nullptr;
    if (int rc = cae_analyze_batched(nprob, probs, opt, &an)) return rc;
    std::unique_ptr<cae_analysis_s> own(an);
    std::vector<int64_t> row_off, nz_off;
    if (int rc = batch_sizes(nprob, probs, true, row_off, nz_off)) return rc;
    cae_options_t o;
    if (int rc = checked_options(an, eps, opt, o)) return rc;
    hipStream_t st = (hipStream_t)o.stream;
    g_cur_stream = st;
    DevBuf dv;
    dv.alloc((size_t)nz_off[nprob] * sizeof(double));
    for (int t = 0; t < nprob; ++t)
      HIPCHK(hipMemcpyAsync(dv.as<double>() + nz_off[t], probs[t].vals, (size_t)(nz_off[t + 1] - nz_off[t]) * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    Carver carve;
    carve.base = static_cast<char*>(o.workspace);
    carve.cap = o.workspace_bytes;
    if (o.workspace && (reinterpret_cast<uintptr_t>(carve.base) & 255) != 0)
      return fail(CAE_EINVAL, "workspace must be 256-byte aligned");
    cae_handle_t h = nullptr;
    if (int rc = factor_checked(an, dv.as<double>(), eps, o, o.workspace ? &carve : nullptr, &h)) return rc;
    h->owned_an.reset(own.release());   // the handle owns the joint analysis
    *out = h;
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

static int cae_apply_precond_impl(cae_handle_t h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz) {
  if (h) g_cur_stream = h->stream;
  if (check_handle(h)) return CAE_EINVAL;
  const int64_t n = h->an->a.n;
  if (nrhs <= 0 || !r || !z || ldr < n || ldz < n) return fail(CAE_EINVAL, "bad vector arguments");
  try {
    do_apply(h, nrhs, r, ldr, z, ldz);
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

static int cae_apply_precond_noalloc_impl(cae_handle_t h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz,
                              void* stream) {
  if (check_handle(h)) return CAE_EINVAL;
  const int64_t n = h->an->a.n;
  if (nrhs <= 0 || !r || !z || ldr < n || ldz < n) return fail(CAE_EINVAL, "bad vector arguments");
  if (h->K + 1 > kNoAllocMaxLevels) return fail(CAE_EINVAL, "too many levels for the allocation-free apply");
  size_t y_off[kNoAllocMaxLevels], ctmp_off = 0, part_off = 0;
  const size_t need = noalloc_layout(h, nrhs, y_off, &ctmp_off, &part_off);
  if (need > kNoAllocScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "the allocation-free apply needs %zu bytes of scratch for %d right-hand sides; its limit is %zu bytes",
             need, nrhs, kNoAllocScratchBytes);
    return fail(CAE_EINVAL, buf);
  }
  try {
    char* base = static_cast<char*>(noalloc_scratch());
    double* y[kNoAllocMaxLevels];
    for (int l = 0; l <= h->K; ++l) y[l] = reinterpret_cast<double*>(base + y_off[l]);
    const ApplyBufs B{y, reinterpret_cast<double*>(base + ctmp_off), reinterpret_cast<double*>(base + part_off)};
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    if (h->precision != CAE_FP64)
      apply_precond<float>(h, nrhs, r, ldr, z, ldz, B, s);
    else
      apply_precond<double>(h, nrhs, r, ldr, z, ldz, B, s);
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

static int cae_apply_factor_impl(cae_handle_t h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy) {
  if (h) g_cur_stream = h->stream;
  if (check_handle(h)) return CAE_EINVAL;
  const int64_t n = h->an->a.n;
  if (nrhs <= 0 || !x || !y || ldx < n || ldy < n) return fail(CAE_EINVAL, "bad vector arguments");
  try {
    if (h->precision != CAE_FP64)
      apply_factor<float>(h, nrhs, x, ldx, y, ldy);
    else
      apply_factor<double>(h, nrhs, x, ldx, y, ldy);
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

// PCG (Algorithm of Hestenes and Stiefel with the preconditioner M^{-1} of
// Proposition 2.2) on independent lanes: every column of every segment (one
// problem of a batch; the whole matrix when sg is null) has its own scalars
// and stopping test; lane = k * nseg + segment.  iters / relres per lane.
static int pcg_lanes(cae_handle_t h, const cae::SegTiles* sg, int32_t nrhs, const double* b, int64_t ldb, double* x,
                     int64_t ldx, double rtol, int32_t maxit, int32_t* iters, double* relres) {
  const int64_t n = h->an->a.n;
  const int nseg = sg ? sg->nseg : 1;
  const int L = nrhs * nseg;
  hipStream_t s = h->stream;
  try {
    const cae_analysis_s* A = h->an;
    const size_t vb = (size_t)n * nrhs * sizeof(double);
    h->pr.alloc(vb);
    h->pz.alloc(vb);
    h->pp.alloc(vb);
    h->pq.alloc(vb);
    poison(h->pr, s);
    poison(h->pz, s);
    poison(h->pp, s);
    poison(h->pq, s);
    h->sc.alloc((size_t)8 * L * sizeof(double));
    h->act.alloc((size_t)L * sizeof(int32_t));
    h->partial.alloc((size_t)nrhs * (sg ? (size_t)sg->ntiles : 1024) * sizeof(double));
    double* r = h->pr.as<double>();
    double* z = h->pz.as<double>();
    double* p = h->pp.as<double>();
    double* q = h->pq.as<double>();
    double* rz = h->sc.as<double>();
    double* rz_new = rz + L;
    double* pq = rz + 2 * L;
    double* rr = rz + 3 * L;
    double* beta = rz + 4 * L;
    double* part = h->partial.as<double>();
    int32_t* active = h->act.as<int32_t>();
    const int64_t* rp = A->row_ptr.as<int64_t>();
    const int32_t* ci = A->col_idx.as<int32_t>();
    const double* av = h->vals.as<double>();
    auto dots = [&](const double* u, int64_t ldu, const double* v, int64_t ldv, double* out) {
      if (sg)
        cae::launch_seg_dots(*sg, nrhs, u, ldu, v, ldv, part, out, s);
      else
        cae::launch_dots(n, nrhs, u, ldu, v, ldv, part, out, s);
    };

    for (int k = 0; k < nrhs; ++k) cae::launch_fill(x + k * ldx, n, 0.0, s);
    cae::launch_copy_cols(n, nrhs, b, ldb, r, n, s);
    std::vector<double> bn(L), hrr(L);
    dots(b, ldb, b, ldb, rr);
    HIPCHK(hipMemcpyAsync(bn.data(), rr, L * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int32_t> hact(L);
    int nact = 0;
    for (int k = 0; k < L; ++k) {
      bn[k] = std::sqrt(bn[k]);
      hact[k] = bn[k] > 0.0 ? 1 : 0;
      nact += hact[k];
      iters[k] = 0;
    }
    HIPCHK(hipMemcpyAsync(active, hact.data(), L * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (nact > 0) {
      solver_apply(h, nrhs, r, n, z, n);
      cae::launch_copy_cols(n, nrhs, z, n, p, n, s);
      dots(r, n, z, n, rz);
    }
    int it = 0;
    while (nact > 0 && it < maxit) {
      cae::launch_spmv(n, rp, ci, av, nrhs, p, n, q, n, s);
      dots(p, n, q, n, pq);
      if (sg)
        cae::launch_seg_pcg_xr(*sg, n, nrhs, rz, pq, active, x, ldx, p, r, q, s);
      else
        cae::launch_pcg_xr(n, nrhs, rz, pq, active, x, ldx, p, r, q, s);
      ++it;
      dots(r, n, r, n, rr);
      HIPCHK(hipMemcpyAsync(hrr.data(), rr, L * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int k = 0; k < L; ++k) {
        if (hact[k] && std::sqrt(hrr[k]) <= rtol * bn[k]) {
          hact[k] = 0;
          iters[k] = it;
          --nact;
        }
      }
      if (nact == 0) break;
      HIPCHK(hipMemcpyAsync(active, hact.data(), L * sizeof(int32_t), hipMemcpyHostToDevice, s));
      solver_apply(h, nrhs, r, n, z, n);
      dots(r, n, z, n, rz_new);
      if (sg)
        cae::launch_seg_pcg_p(*sg, n, nrhs, rz, rz_new, active, z, p, beta, s);
      else
        cae::launch_pcg_p(n, nrhs, rz, rz_new, active, z, p, beta, s);
    }
    for (int k = 0; k < L; ++k)
      if (hact[k]) iters[k] = it;
    // true residual
    cae::launch_spmv(n, rp, ci, av, nrhs, x, ldx, q, n, s);
    cae::launch_residual(n, nrhs, b, ldb, q, s);
    dots(q, n, q, n, rr);
    HIPCHK(hipMemcpyAsync(hrr.data(), rr, L * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < L; ++k) relres[k] = bn[k] > 0 ? std::sqrt(hrr[k]) / bn[k] : 0.0;
    if (nact > 0) return fail(CAE_ENOCONV, "PCG did not converge within maxit");
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return fail(CAE_ENOMEM, "host allocation failed");
  }
  return CAE_OK;
}

static int cae_pcg_solve_impl(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx, double rtol,
                  int32_t maxit, int32_t* iters, double* relres) {
  if (h) g_cur_stream = h->stream;
  if (check_handle(h)) return CAE_EINVAL;
  const int64_t n = h->an->a.n;
  if (nrhs <= 0 || !b || !x || ldb < n || ldx < n || !iters || !relres || maxit < 0 || !(rtol >= 0))
    return fail(CAE_EINVAL, "bad PCG arguments");
  return pcg_lanes(h, nullptr, nrhs, b, ldb, x, ldx, rtol, maxit, iters, relres);
}

static int cae_pcg_solve_batched_impl(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                                      int64_t ldx, double rtol, int32_t maxit, int32_t* iters, double* relres) {
  if (h) g_cur_stream = h->stream;
  if (check_handle(h)) return CAE_EINVAL;
  if (h->sg.nseg == 0) return fail(CAE_EINVAL, "the handle was not made from a batch of problems");
  const int64_t n = h->an->a.n;
  if (nrhs <= 0 || !b || !x || ldb < n || ldx < n || !iters || !relres || maxit < 0 || !(rtol >= 0))
    return fail(CAE_EINVAL, "bad PCG arguments");
  const int nseg = h->sg.nseg;
  if ((int64_t)nrhs * nseg > (int64_t)1 << 26) return fail(CAE_EINVAL, "too many (problem, column) pairs");
  std::vector<int32_t> it((size_t)nrhs * nseg);
  std::vector<double> rel((size_t)nrhs * nseg);
  const int rc = pcg_lanes(h, &h->sg, nrhs, b, ldb, x, ldx, rtol, maxit, it.data(), rel.data());
  if (rc == CAE_OK || rc == CAE_ENOCONV)
    for (int t = 0; t < nseg; ++t)
      for (int k = 0; k < nrhs; ++k) {
        iters[(size_t)t * nrhs + k] = it[(size_t)k * nseg + t];
        relres[(size_t)t * nrhs + k] = rel[(size_t)k * nseg + t];
      }
  return rc;
}

static int cae_minres_solve_impl(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                     double rtol, int32_t maxit, int32_t* iters, double* relres) {
  if (h) g_cur_stream = h->stream;
  if (check_handle(h)) return CAE_EINVAL;
  const int64_t n = h->an->a.n;
  if (nrhs <= 0 || !b || !x || ldb < n || ldx < n || !iters || !relres || maxit < 0 || !(rtol >= 0))
    return fail(CAE_EINVAL, "bad MINRES arguments");
  hipStream_t s = h->stream;
  try {
    const cae_analysis_s* A = h->an;
    const size_t vb = (size_t)n * nrhs * sizeof(double);
    for (auto& m : h->mr) m.alloc(vb);
    h->mst.alloc((size_t)cae::MR_NFIELDS * nrhs * sizeof(double));
    h->act.alloc((size_t)nrhs * sizeof(int32_t));
    h->partial.alloc((size_t)nrhs * 1024 * sizeof(double));
    double* st = h->mst.as<double>();
    double* part = h->partial.as<double>();
    int32_t* active = h->act.as<int32_t>();
    const int64_t* rp = A->row_ptr.as<int64_t>();
    const int32_t* ci = A->col_idx.as<int32_t>();
    const double* av = h->vals.as<double>();
    // rotating buffers: r1, r2, y (three-term Lanczos); w1, w2, w hold w_{k-2},
    // w_{k-1}, w_k after iteration k; and v
    double* r1 = h->mr[0].as<double>();
    double* r2 = h->mr[1].as<double>();
    double* y = h->mr[2].as<double>();
    double* w1 = h->mr[3].as<double>();
    double* w2 = h->mr[4].as<double>();
    double* w = h->mr[5].as<double>();
    double* v = h->mr[6].as<double>();
    auto F = [&](int f) { return st + (int64_t)f * nrhs; };

    for (int k = 0; k < nrhs; ++k) cae::launch_fill(x + k * ldx, n, 0.0, s);
    cae::launch_fill(w, (int64_t)n * nrhs, 0.0, s);
    cae::launch_fill(w2, (int64_t)n * nrhs, 0.0, s);
    cae::launch_fill(w1, (int64_t)n * nrhs, 0.0, s);
    cae::launch_copy_cols(n, nrhs, b, ldb, r1, n, s);
    cae::launch_copy_cols(n, nrhs, b, ldb, r2, n, s);
    std::vector<double> bn(nrhs), hv(nrhs), hb(nrhs);
    cae::launch_dots(n, nrhs, b, ldb, b, ldb, part, F(cae::MR_BSQ), s);
    HIPCHK(hipMemcpyAsync(bn.data(), F(cae::MR_BSQ), nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    solver_apply(h, nrhs, r1, n, y, n);
    cae::launch_dots(n, nrhs, r1, n, y, n, part, F(cae::MR_BSQ), s);
    HIPCHK(hipMemcpyAsync(hv.data(), F(cae::MR_BSQ), nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // initial state: beta = phibar = beta_1, cs = -1, the rest 0
    std::vector<double> init((size_t)cae::MR_NFIELDS * nrhs, 0.0);
    std::vector<double> beta1(nrhs);
    std::vector<int32_t> hact(nrhs);
    int nact = 0;
    for (int k = 0; k < nrhs; ++k) {
      bn[k] = std::sqrt(bn[k]);
      beta1[k] = std::sqrt(std::max(hv[k], 0.0));
      init[cae::MR_BETA * nrhs + k] = beta1[k];
      init[cae::MR_PHIBAR * nrhs + k] = beta1[k];
      init[cae::MR_CS * nrhs + k] = -1.0;
      hact[k] = beta1[k] > 0.0 ? 1 : 0;
      nact += hact[k];
      iters[k] = 0;
    }
    HIPCHK(hipMemcpyAsync(st, init.data(), init.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(active, hact.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    int it = 0;
    while (nact > 0 && it < maxit) {
      cae::launch_mr_v(n, nrhs, active, st, y, v, s);
      cae::launch_spmv(n, rp, ci, av, nrhs, v, n, y, n, s);
      if (it > 0) cae::launch_mr_y(n, nrhs, active, st, r1, y, 0, s);
      cae::launch_dots(n, nrhs, v, n, y, n, part, F(cae::MR_ALPHA), s);
      cae::launch_mr_y(n, nrhs, active, st, r2, y, 1, s);
      // r1 <- r2, r2 <- y; the old r1 takes the next y = M^{-1} r2
      double* t = r1;
      r1 = r2;
      r2 = y;
      y = t;
      solver_apply(h, nrhs, r2, n, y, n);
      cae::launch_dots(n, nrhs, r2, n, y, n, part, F(cae::MR_BSQ), s);
      cae::launch_mr_scalars(nrhs, active, st, s);
      // w_k from w_{k-2} (w2) and w_{k-1} (w); it overwrites w_{k-3} (w1)
      cae::launch_mr_wx(n, nrhs, active, st, v, w2, w, w1, x, ldx, s);
      double* u = w1;
      w1 = w2;
      w2 = w;
      w = u;
      ++it;
      HIPCHK(hipMemcpyAsync(hv.data(), F(cae::MR_PHIBAR), nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(hb.data(), F(cae::MR_BETA), nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bool changed = false;
      for (int k = 0; k < nrhs; ++k) {
        if (hact[k] && (hv[k] <= rtol * beta1[k] || !(hb[k] > 0.0))) {
          hact[k] = 0;
          iters[k] = it;
          --nact;
          changed = true;
        }
      }
      if (changed) HIPCHK(hipMemcpyAsync(active, hact.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    for (int k = 0; k < nrhs; ++k)
      if (hact[k]) iters[k] = it;
    double* q = v;
    cae::launch_spmv(n, rp, ci, av, nrhs, x, ldx, q, n, s);
    cae::launch_residual(n, nrhs, b, ldb, q, s);
    cae::launch_dots(n, nrhs, q, n, q, n, part, F(cae::MR_BSQ), s);
    HIPCHK(hipMemcpyAsync(hv.data(), F(cae::MR_BSQ), nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < nrhs; ++k) relres[k] = bn[k] > 0 ? std::sqrt(hv[k]) / bn[k] : 0.0;
    if (nact > 0) return fail(CAE_ENOCONV, "MINRES did not converge within maxit");
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

// Algorithmic flops of the block operations of every factored level (the
// work the method must do, not what a kernel happens to execute), from the
// recorded sizes and ranks.  Per step with b = b_i, r = r_i, n = b - r, live
// widths s_c of the close views (r_c for processed neighbours, b_c otherwise)
// and far width w (the same rule over the far views):
//   compression  2 w b^2 - 2 b^3 / 3 (QR of the b x w far row; w < b: the
//                transposed count) + 12 b^3 (SVD of the triangular factor)
//   rotation     4 b^3 (U^T D U) + 2 b^2 sum_close b_c (U^T V, stored factor
//                rows included) + 2 r b w (kept rows of the far views)
//   elimination  n^3 / 3 (Cholesky of S_ii) + n^2 (r + sum_close s_c)
//                (triangular solves of the panels)
//   Schur        sum over panel pairs a <= c of 2 n s_a s_c (panel widths r
//                and s_c)
// compression and rotation only for steps with a non-empty far row; the dense
// remainder counts dim^3 / 3 (its Cholesky).
void count_block_flops(cae_factor_s* h) {
  h->compress_flops = h->rotate_flops = h->elim_flops = h->schur_flops = 0;
  h->compressions = 0;
  const cae::Analysis& a = h->an->a;
  for (int l = 0; l < h->K; ++l) {
    const cae::LevelSym& L = a.levels[l];
    const NumLevel& N = h->lev[l];
    std::vector<double> sw;
    for (const cae::Step& stp : L.steps) {
      const double b = N.sizes[stp.blk], r = N.ranks[stp.blk], n = b - r;
      double w = 0, bclose = 0;
      sw.assign(1, r);
      for (int v = 0; v < stp.nclose + stp.nfar; ++v) {
        const cae::View& vw = L.views[stp.view0 + v];
        const double live = vw.proc ? N.ranks[vw.x] : N.sizes[vw.x];
        if (v < stp.nclose) {
          sw.push_back(live);
          bclose += N.sizes[vw.x];
        } else {
          w += live;
        }
      }
      if (stp.nfar > 0) {
        const double qr = w >= b ? 2 * w * b * b - 2 * b * b * b / 3 : 2 * b * w * w - 2 * w * w * w / 3;
        h->compress_flops += qr + 12 * b * b * b;
        h->compressions += 1;
        h->rotate_flops += 4 * b * b * b + 2 * b * b * bclose + 2 * r * b * w;
      }
      if (n > 0) {
        double ssum = 0, pairs = 0, pre = 0;
        for (double x : sw) {
          ssum += x;
          pre += x;
          pairs += x * pre;   // sum over a <= c of s_a s_c
        }
        h->elim_flops += n * n * n / 3 + n * n * ssum;
        h->schur_flops += 2 * n * pairs;
      }
    }
  }
  const double d = (double)h->coarse_dim;
  h->coarse_flops = d * d * d / 3;
  h->flops_pending = false;
}

static int cae_get_stats_impl(cae_handle_t h, cae_stats_t* st) {
  if (check_handle(h) || !st) return fail(CAE_EINVAL, "null argument");
  if (h->flops_pending) count_block_flops(h);
  st->nlevels = h->K;
  st->coarse_dim = h->coarse_dim;
  st->tau = h->tau;
  st->dropped_sq = h->dropped;
  st->min_pivot = h->min_pivot;
  st->factor_bytes = h->factor_bytes;
  st->factor_ms = h->factor_ms;
  st->compress_launches = h->compress_launches;
  st->compress_ms = h->compress_ms;
  st->compress_flops = h->compress_flops;
  st->compressions = h->compressions;
  st->rotate_flops = h->rotate_flops;
  st->elim_flops = h->elim_flops;
  st->schur_flops = h->schur_flops;
  st->coarse_flops = h->coarse_flops;
  st->sketch_accepted = h->sketch_acc;
  st->sketch_rejected = h->sketch_rej;
  st->record_rows = h->rec_rows;
  st->big_untruncated = h->big_count[0];
  st->big_frobenius = h->big_count[1];
  st->big_certified = h->big_count[2];
  st->big_uncapped = h->big_count[3];
  st->schur_launches = h->schur_launches;
  st->schur_ms = h->schur_ms;
  return CAE_OK;
}

int32_t cae_mlp_param_count(void) { return cae::MLP_NPARAM; }

int cae_mlp_train(const float* records, int64_t n, float* params, int32_t epochs, float lr, float* loss,
                  void* stream) {
  if (!records || !params || n <= 0 || epochs < 0 || !(lr > 0.0f)) return fail(CAE_EINVAL, "bad MLP training arguments");
  hipStream_t s = (hipStream_t)stream;
  g_cur_stream = s;
  try {
    DevBuf grad, m, v, lossd, nv;
    grad.alloc(cae::MLP_NPARAM * sizeof(float));
    m.alloc(cae::MLP_NPARAM * sizeof(float));
    v.alloc(cae::MLP_NPARAM * sizeof(float));
    lossd.alloc(sizeof(float));
    nv.alloc(sizeof(int));
    cae::launch_mlp_zero(m.as<float>(), cae::MLP_NPARAM, s);
    cae::launch_mlp_zero(v.as<float>(), cae::MLP_NPARAM, s);
    cae::launch_mlp_stats(records, n, params, nv.as<int>(), s);
    int nvalid = 0;
    HIPCHK(hipMemcpyAsync(&nvalid, nv.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nvalid == 0) return fail(CAE_EINVAL, "no training rows (all labels negative)");
    for (int e = 0; e < epochs; ++e) {
      cae::launch_mlp_grad(params, records, n, 1.0f / (float)nvalid, grad.as<float>(), lossd.as<float>(), s);
      cae::launch_mlp_adam(params, grad.as<float>(), m.as<float>(), v.as<float>(), lr, e + 1, s);
    }
    float hl = 0.0f;
    cae::launch_mlp_grad(params, records, n, 1.0f / (float)nvalid, grad.as<float>(), lossd.as<float>(), s);
    HIPCHK(hipMemcpyAsync(&hl, lossd.p, sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (loss) *loss = hl;
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

int cae_mlp_loss_grad(const float* params, const float* records, int64_t n, float* grad, float* loss, void* stream) {
  if (!records || !params || !grad || n <= 0) return fail(CAE_EINVAL, "bad MLP gradient arguments");
  hipStream_t s = (hipStream_t)stream;
  g_cur_stream = s;
  try {
    // count the valid rows on the device through the statistics kernel (on a copy of the parameters)
    DevBuf tmp, lossd, nv;
    tmp.alloc(cae::MLP_NPARAM * sizeof(float));
    lossd.alloc(sizeof(float));
    nv.alloc(sizeof(int));
    cae::launch_mlp_stats(records, n, tmp.as<float>(), nv.as<int>(), s);
    int nvalid = 0;
    HIPCHK(hipMemcpyAsync(&nvalid, nv.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nvalid == 0) return fail(CAE_EINVAL, "no training rows (all labels negative)");
    cae::launch_mlp_grad(params, records, n, 1.0f / (float)nvalid, grad, lossd.as<float>(), s);
    float hl = 0.0f;
    HIPCHK(hipMemcpyAsync(&hl, lossd.p, sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (loss) *loss = hl;
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

int cae_mlp_predict(const float* params, const float* records, int64_t n, float* z, void* stream) {
  if (!records || !params || !z || n < 0) return fail(CAE_EINVAL, "bad MLP prediction arguments");
  hipStream_t s = (hipStream_t)stream;
  try {
    cae::launch_mlp_predict(params, records, n, z, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  } catch (const HipError& e) {
    return fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return CAE_OK;
}

static int cae_get_ranks_impl(cae_handle_t h, int32_t level, int32_t* ranks) {
  if (check_handle(h) || !ranks) return fail(CAE_EINVAL, "null argument");
  if (level < 0 || level >= h->K) return fail(CAE_EINVAL, "level out of range");
  std::memcpy(ranks, h->lev[level].ranks.data(), h->lev[level].ranks.size() * sizeof(int32_t));
  return CAE_OK;
}

static int cae_get_drops_impl(cae_handle_t h, int32_t level, double* e) {
  if (check_handle(h) || !e) return fail(CAE_EINVAL, "null argument");
  if (level < 0 || level >= h->K) return fail(CAE_EINVAL, "level out of range");
  std::memcpy(e, h->lev[level].drops.data(), h->lev[level].drops.size() * sizeof(double));
  return CAE_OK;
}

static int cae_get_sizes_impl(cae_handle_t h, int32_t level, int32_t* sizes) {
  if (check_handle(h) || !sizes) return fail(CAE_EINVAL, "null argument");
  if (level < 0 || level > h->K) return fail(CAE_EINVAL, "level out of range");
  std::memcpy(sizes, h->lev[level].sizes.data(), h->lev[level].sizes.size() * sizeof(int32_t));
  return CAE_OK;
}

int cae_apply_precond(cae_handle_t h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz) {
  return keep_error(h, cae_apply_precond_impl(h, nrhs, r, ldr, z, ldz));
}

int cae_apply_precond_noalloc(cae_handle_t h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz,
                              void* stream) {
  return keep_error(h, cae_apply_precond_noalloc_impl(h, nrhs, r, ldr, z, ldz, stream));
}

int cae_apply_factor(cae_handle_t h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy) {
  return keep_error(h, cae_apply_factor_impl(h, nrhs, x, ldx, y, ldy));
}

int cae_pcg_solve(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx, double rtol,
                  int32_t maxit, int32_t* iters, double* relres) {
  return keep_error(h, cae_pcg_solve_impl(h, nrhs, b, ldb, x, ldx, rtol, maxit, iters, relres));
}

int cae_pcg_solve_batched(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                          double rtol, int32_t maxit, int32_t* iters, double* relres) {
  return keep_error(h, cae_pcg_solve_batched_impl(h, nrhs, b, ldb, x, ldx, rtol, maxit, iters, relres));
}

int cae_minres_solve(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                     double rtol, int32_t maxit, int32_t* iters, double* relres) {
  return keep_error(h, cae_minres_solve_impl(h, nrhs, b, ldb, x, ldx, rtol, maxit, iters, relres));
}

int cae_get_stats(cae_handle_t h, cae_stats_t* st) {
  return keep_error(h, cae_get_stats_impl(h, st));
}

int cae_get_ranks(cae_handle_t h, int32_t level, int32_t* ranks) {
  return keep_error(h, cae_get_ranks_impl(h, level, ranks));
}

int cae_get_sizes(cae_handle_t h, int32_t level, int32_t* sizes) {
  return keep_error(h, cae_get_sizes_impl(h, level, sizes));
}

int cae_get_drops(cae_handle_t h, int32_t level, double* e) {
  return keep_error(h, cae_get_drops_impl(h, level, e));
}

int cae_get_level_ms(cae_handle_t h, int32_t level, double* ms) {
  if (check_handle(h) || !ms) return fail(CAE_EINVAL, "null argument");
  if (level < 0 || level > h->K) return keep_error(h, fail(CAE_EINVAL, "level out of range"));
  const double start = level > 0 ? h->lev[level - 1].end_ms : 0.0;
  *ms = (level < h->K ? h->lev[level].end_ms : h->factor_ms) - start;
  return CAE_OK;
}

int cae_export_factor(cae_handle_t h, const char* path) {
  if (check_handle(h) || !path) return fail(CAE_EINVAL, "handle and path are required");
  FILE* fp = fopen(path, "wb");
  if (!fp) return keep_error(h, fail(CAE_EINVAL, std::string("cannot open ") + path));
  std::unique_ptr<FILE, int (*)(FILE*)> closer(fp, fclose);
  bool ok = true;
  auto put = [&](const void* p, size_t bytes) { ok = ok && (bytes == 0 || fwrite(p, 1, bytes, fp) == bytes); };
  auto put_vec = [&](const auto& v) { put(v.data(), v.size() * sizeof(v[0])); };
  std::vector<char> host;
  auto put_dev = [&](const DevBuf& d, size_t bytes) {
    host.resize(bytes);
    if (bytes) HIPCHK(hipMemcpy(host.data(), d.p, bytes, hipMemcpyDeviceToHost));
    put(host.data(), bytes);
  };
  try {
    HIPCHK(hipStreamSynchronize(h->stream));
    const cae::Analysis& a = h->an->a;
    const int32_t esize = h->precision == CAE_FP64 ? 8 : 4;
    put("CAEFACT1", 8);
    const int32_t hdr[2] = {esize, h->K};
    put(hdr, sizeof hdr);
    const int64_t dims[2] = {a.n, h->coarse_dim};
    put(dims, sizeof dims);
    put(&h->tau, sizeof(double));
    put_vec(a.perm);
    for (int l = 0; l < h->K; ++l) {
      const cae::LevelSym& L = a.levels[l];
      const NumLevel& N = h->lev[l];
      const int32_t ms[2] = {L.M, L.nslots};
      put(ms, sizeof ms);
      put_vec(N.sizes);
      put_vec(N.ranks);
      put_vec(L.slot_p);
      put_vec(L.slot_q);
      put_vec(N.slot_off);
      put_dev(N.arena, (size_t)N.slot_off.back() * esize);
      put_vec(N.u_off);
      put_dev(N.U, (size_t)N.u_off.back() * esize);
      put_dev(N.Li, (size_t)N.u_off.back() * esize);
      put_vec(L.parent);
      put_vec(N.off_in_parent);
      put_vec(L.order);
    }
    const size_t dd = (size_t)h->coarse_dim * h->coarse_dim * sizeof(double);
    put_dev(h->Acopy, h->coarse_dim > 0 ? dd : 0);
    put_dev(h->Ainv, h->coarse_dim > 0 ? dd : 0);
  } catch (const HipError& e) {
    return keep_error(h, fail(CAE_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e)));
  } catch (const std::bad_alloc&) {
    return keep_error(h, fail(CAE_ENOMEM, "host allocation failed"));
  }
  if (!ok) return keep_error(h, fail(CAE_EINVAL, std::string("write to ") + path + " failed"));
  return CAE_OK;
}

void cae_destroy(cae_handle_t h) {
  if (h) g_cur_stream = h->stream;
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
