// Host side of the EOD-ABE library: C ABI, workspace plan and the enqueue
// logic of Alg. 1 (basis extraction) and Alg. 2 (power iteration,
// projection, closing QRs).  All arithmetic runs in the kernels of
// eodabe_kernels.hpp; the host only validates, carves the caller's
// workspace and enqueues.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/eodabe.h"
#include "eodabe_kernels.hpp"
#include "eodabe_tiles.hpp"
#include "eodabe_mlp.hpp"
#include "eodabe_apps.hpp"

using namespace eodabe;

// Scratch of eodabe_factor_noalloc: a fixed device array in the library's
// code object, one copy per GPU.  Host code must not take this name as a
// device address: its per-device address comes from hipGetSymbolAddress
// (scratch_dev below), fetched once per device at context creation.
static __device__ __align__(256) unsigned char scratch[EODABE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[MAX_DEVICES] = {};
}  // namespace

struct eodabe_ctx {
  eodabe_opts o;
  hipStream_t stream;
  int device;
  int cu_count;
  int last_hip;
  State* host_state;      // pinned host copy of the control block
  State* host_state_dev;  // its device address (null: copied by hipMemcpyAsync only)
  bool barrier_fail = false;  // EODABE_TEST_BARRIER_FAIL set at creation: every grid barrier times out (tests)
  int64_t* host_wlog;     // pinned host copy of the basis-width log
  int64_t host_wlog_cap;
  bool host_only;
  // live timing (eodabe_profile)
  bool prof_on = false;
  struct Mark { hipEvent_t a, b; int kind; int block; double bytes, bytes_per_r; };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Mark> marks;
  double prof_ms[EODABE_PROF_KINDS] = {};
  int64_t prof_n[EODABE_PROF_KINDS] = {};
  double prof_bytes[EODABE_PROF_KINDS] = {};
  // batched tiles: pinned staging of descriptors and results, a private
  // stream for the captured launch, the graph and its key, tuned widths
  void* tile_host = nullptr;
  size_t tile_host_bytes = 0;
  hipStream_t tile_stream = nullptr;
  hipEvent_t tile_ev = nullptr;
  hipGraph_t tile_graph = nullptr;
  hipGraphExec_t tile_exec = nullptr;
  struct { const void* ws; const void* pool; int ntiles, grid; double tol; uint64_t seed; } tile_key{};
  int tile_b[4] = {0, 0, 0, 0};   // block width per tile-size bucket (0: opts.block)
  int tile_graphs = 1;            // capture the launch in a hipGraph
  // learned warm start (eodabe_set_predictor): device parameters of the MLP
  void* scratch = nullptr;        // this device's copy of the static scratch array
  bool cplx_pairs = false;        // set by eodabe_factor_complex around its realified call
  const float* pred_params = nullptr;
  double pred_margin = 0.1;
  struct { int64_t d0 = 0; double y0 = 0, y1 = 0; int used = 0; } pred_last;
};

namespace {

constexpr int BN_MAX = 128;

inline int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline int64_t cdiv(int64_t x, int64_t a) { return (x + a - 1) / a; }
// Workgroups of a Gram kernel of the basis loop (one row panel each up to
// this; the partial buffer holds that many)
constexpr int GRAM_LOOP_WG = 192;
// Workgroups of a k_apply launch (its 64-row blocks taken grid-stride)
constexpr int64_t APPLY_WG = 1024;

// K-chunk (multiple of 16) and the number of non-empty splits actually
// launched for a reduction of length K asked to use `want` splits.  Every
// partial buffer consumer must use this count.
inline int64_t split_chunk(int64_t K, int want) {
  return rup(cdiv(std::max<int64_t>(K, 1), std::max(want, 1)), 16);
}
inline int eff_splits(int64_t K, int want) {
  return (int)std::max<int64_t>(1, cdiv(std::max<int64_t>(K, 1), split_chunk(K, want)));
}

#define HIPCHK(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) {                            \
      ctx->last_hip = (int)e_;                         \
      return EODABE_EHIP;                              \
    }                                                  \
  } while (0)

#define LAUNCHCHK()                                    \
  do {                                                 \
    hipError_t e_ = hipGetLastError();                 \
    if (e_ != hipSuccess) {                            \
      ctx->last_hip = (int)e_;                         \
      return EODABE_EHIP;                              \
    }                                                  \
  } while (0)

#define TRY(x)                                         \
  do {                                                 \
    int s_ = (x);                                      \
    if (s_ < 0) return s_;                             \
  } while (0)

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(int64_t count) {
    off = (size_t)rup((int64_t)off, 256);
    T* p = base ? (T*)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

// Event pair of one timed launch (no-op unless profiling is on); the events
// ride on the kernel dispatch itself (hipExtLaunchKernelGGL), so they time
// the kernel execution without the launch gaps around it.
hipEvent_t prof_event(eodabe_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
int prof_begin(eodabe_ctx* ctx, hipStream_t st) {
  if (!ctx->prof_on) return -1;
  eodabe_ctx::Mark mk{prof_event(ctx), prof_event(ctx), 0, 0, 0.0, 0.0};
  if (!mk.a || !mk.b) return -1;
  (void)st;
  ctx->marks.push_back(mk);
  return (int)ctx->marks.size() - 1;
}
// Marks of closing steps enqueued ahead of the stop flag carry SPEC_BLOCK.
constexpr int SPEC_BLOCK = -2;
void prof_end(eodabe_ctx* ctx, hipStream_t st, int id, int kind, int block, double bytes,
              double bytes_per_r = 0.0) {
  if (id < 0) return;
  auto& mk = ctx->marks[id];
  mk.kind = kind;
  mk.block = block;
  mk.bytes = bytes;
  mk.bytes_per_r = bytes_per_r;
  (void)st;
}
// Attach (or detach, id < 0) the events of mark id to the next timed launch.
template <typename O>
void prof_attach(eodabe_ctx* ctx, O& ops, int id) {
  ops.pe0 = id >= 0 ? ctx->marks[id].a : nullptr;
  ops.pe1 = id >= 0 ? ctx->marks[id].b : nullptr;
}
// After the stream has been synchronised: fold the marks of launches that
// did their work (blocks <= last_block; speculative closing steps only when
// spec_ran) into the totals and recycle the events.  rank sizes the
// rank-dependent bytes.
void prof_collect(eodabe_ctx* ctx, int last_block, bool spec_ran, int64_t rank) {
  for (auto& mk : ctx->marks) {
    const bool ran = mk.block == SPEC_BLOCK ? spec_ran : (mk.block >= 0 && mk.block <= last_block);
    if (ran) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, mk.a, mk.b) == hipSuccess) {
        ctx->prof_ms[mk.kind] += ms;
        ctx->prof_n[mk.kind] += 1;
        ctx->prof_bytes[mk.kind] += mk.bytes + mk.bytes_per_r * (double)rank;
      }
    }
    ctx->ev_pool.push_back(mk.a);
    ctx->ev_pool.push_back(mk.b);
  }
  ctx->marks.clear();
}

// Realified complex input: re-impose the pairing on ncols columns (see
// k_pair_fix); nothing otherwise.
template <typename T>
int pair_fix(eodabe_ctx* ctx, hipStream_t st, bool paired, T* X, int64_t ld, int64_t nn, int64_t ncols,
             const int32_t* stopb = nullptr, int blk = 0) {
  if (!paired || ncols < 2 || nn <= 0) return 0;
  dim3 grid((unsigned)((nn + 255) / 256), (unsigned)(ncols / 2));
  hipLaunchKernelGGL((k_pair_fix<T>), grid, dim3(256), 0, st, X, ld, nn, ncols, stopb, blk);
  LAUNCHCHK();
  return 0;
}

// Problem geometry after the optional transpose (mm >= nn).
struct Geo {
  int64_t mm, nn;       // factored matrix is mm x nn (row-major, ld lda_eff)
  bool transposed;
  bool packed;          // A copied into workspace (transpose or alignment)
  int64_t lda_eff;
  int b, bn;            // block width and padded width (multiple of 16)
  int64_t nblk;         // ceil(nn / b)
  int64_t ldk;          // Omega^T leading dim (>= nn, multiple of 4)
  int64_t ldy;          // Y / Q leading dim (>= mm, multiple of 4)
  int64_t r_cap;        // output capacity (rank bound)
  int s_sketch;         // K-splits of the sketch
  int s_proj;           // K-splits of Q^T Y
  int s_gram;           // K-splits of block Grams
  int s_core;           // K-splits of the r-column products (C = Q^T A etc.)
  size_t elem;
  int lp;               // low-precision sketch: 0 none, 1 FP16, 2 BF16
  int64_t ld_lp;        // leading dimension of the low-precision copy of A (multiple of 8)
  bool wide;            // learned warm start: buffers of the wide sketch
  bool paired;          // realified complex input: test columns and stops in pairs
  bool sk_rows;         // sketch by 16-row tiles straight into Y (k_sketch_rows)
};

// Widest sketch of the learned warm start in one pass over A (columns).
constexpr int WIDE_COLS = 128;
// K-splits of the Gram of blocks wider than 64 columns (partials, then a sum).
constexpr int GRAM_SPLITS_WIDE = 16;
// Waves of a k_sketch_rows workgroup (the K parts of one 16-row tile).
constexpr int SKETCH_ROWS_WAVES = 8;

struct WS {
  State* st;
  int64_t* wlog;
  int32_t* accv;
  int32_t* dead;        // nblk x BN_MAX
  double* diag_log;     // nn
  double* normparts;    // per sketch workgroup: sum of squares
  float* maxparts;      // per sketch workgroup: max |A|
  uint16_t* alp;        // low-precision copy of A (mm x ld_lp), if g.lp
  void* omega;          // bn x ldk
  void* ypart;          // s_sketch x ldy x bn
  void* y;              // ldy x bn
  void* wpart;          // s_proj x ldw x bn
  void* w;              // ldw x bn
  double* gpart;        // Gram partials (max(s_gram, GRAM_LOOP_WG) x bn x bn)
  void* wfp;            // W = Q^T Y partials of the one-launch block Gram-Schmidt
  double* gsum;         // summed block Gram (bn x bn)
  double* r1;           // bn x bn
  double* r2;
  double* r1inv;        // bn x bn: R1^{-1} of the current block
  double* r2inv;        // bn x bn: R2^{-1} of the current block
  void* q;              // ldy x (nn + bn)
  void* apack;          // mm x lda_eff (if packed)
  // closing steps
  void* cbuf;           // r_cap x ldk   (C = Q^T A, then V^T in place)
  void* cpart;          // s_core x r_cap x ldk
  void* ybig;           // ldy x r_cap   (power iteration / U_hat scratch)
  double* gbig;         // Gram partials of the closing QRs
  double* rb1;          // r_cap x r_cap
  double* rb2;
  double* rb3;
  double* rb4;
  double* rb5;
  int32_t* deadbig;     // r_cap
  double* dg;           // r_cap
  void* tbig;           // ldy x r_cap scratch for large-f triangular solves
  double* sq128;        // 7 x 128 x 128: closing QR scratch for ranks 65..128
  uint64_t* cbmask;     // per 64-column panel: pivots that did not eliminate (wide Cholesky)
  // learned warm start (g.wide): wide Omega, sketch partials and sketch, prediction
  void* omega_w;        // WIDE_COLS x ldk
  void* ypart_w;        // s_sketch x ldy x WIDE_COLS
  void* y_w;            // ldy x WIDE_COLS
  MlpPred* pred;
  size_t total;
};

int64_t ldw_of(const Geo& g) { return rup(g.nn + g.bn, 4); }

WS carve(void* base, const Geo& g) {
  Carver c(base);
  WS w{};
  const size_t e = g.elem;
  w.st = c.take<State>(1);
  w.wlog = c.take<int64_t>(g.nblk + 2);
  w.accv = c.take<int32_t>(g.nblk + 1);
  w.dead = c.take<int32_t>((g.nblk + 1) * BN_MAX);
  w.diag_log = c.take<double>(g.nn + BN_MAX);
  const int64_t nparts = std::max<int64_t>((int64_t)g.s_sketch * cdiv(g.mm, 128), cdiv(g.mm, 16));
  w.normparts = c.take<double>(nparts + 64);
  w.maxparts = c.take<float>(nparts + 64);
  w.alp = g.lp ? c.take<uint16_t>(g.mm * g.ld_lp) : nullptr;
  w.omega = c.take<char>((int64_t)g.bn * rup(g.ldk, 16) * e);   // column or tiled layout
  w.ypart = c.take<char>((int64_t)g.s_sketch * g.ldy * g.bn * e);
  w.y = c.take<char>(g.ldy * g.bn * e);
  w.wpart = c.take<char>((int64_t)g.s_proj * ldw_of(g) * g.bn * e);
  w.w = c.take<char>(ldw_of(g) * g.bn * e);
  w.gpart = c.take<double>((int64_t)std::max(g.s_gram, GRAM_LOOP_WG) * g.bn * g.bn);
  w.wfp = c.take<char>((int64_t)CQR2_GMAX * CQR2_PROJ_WMAX * 32 * e);   // W partials of the one-launch BCGS2
  w.gsum = c.take<double>((int64_t)g.bn * g.bn);
  w.r1 = c.take<double>(g.bn * g.bn);
  w.r2 = c.take<double>(g.bn * g.bn);
  w.r1inv = c.take<double>(g.bn * g.bn);
  w.r2inv = c.take<double>(g.bn * g.bn);
  w.q = c.take<char>(g.ldy * (g.nn + g.bn) * e);
  w.apack = g.packed ? c.take<char>(g.mm * g.lda_eff * e) : nullptr;
  const int64_t rc = std::max<int64_t>(g.r_cap, 1);
  w.cbuf = c.take<char>(rc * g.ldk * e);
  w.cpart = c.take<char>((int64_t)g.s_core * rc * g.ldk * e);
  w.ybig = c.take<char>(g.ldy * rc * e);
  const int64_t rb = std::max<int64_t>(rc, g.bn);
  // Gram partials of the closing QRs: 64 of up to 128 x 128 (the K-split
  // partials of a Gram of at most 128 columns and their sum), or
  // GRAM_SPLITS_WIDE + 1 of rb x rb (wider)
  const int64_t rb128 = std::min<int64_t>(rb, 128);
  w.gbig = c.take<double>(std::max<int64_t>(64 * rb128 * rb128, (GRAM_SPLITS_WIDE + 1) * rb * rb));
  w.rb1 = c.take<double>(rb * rb);
  w.rb2 = c.take<double>(rb * rb);
  w.rb3 = c.take<double>(rb * rb);
  w.rb4 = c.take<double>(rb * rb);
  w.rb5 = c.take<double>(rb * rb);
  w.deadbig = c.take<int32_t>(rc + 64);
  w.dg = c.take<double>(std::max<int64_t>(rc, g.bn) + 64);
  w.tbig = c.take<char>(std::max(g.ldy, g.ldk) * rc * std::max<size_t>(e, 8));
  w.sq128 = rb > 64 ? c.take<double>(7 * 128 * 128) : nullptr;
  w.cbmask = c.take<uint64_t>(2 * (cdiv(rb, 64) + 1));   // per panel: nolive, then the dead masks
  if (g.wide) {
    w.omega_w = c.take<char>((int64_t)WIDE_COLS * g.ldk * e);
    w.ypart_w = c.take<char>((int64_t)g.s_sketch * g.ldy * WIDE_COLS * e);
    w.y_w = c.take<char>(g.ldy * WIDE_COLS * e);
    w.pred = c.take<MlpPred>(1);
  }
  w.total = c.off + 256;
  return w;
}

// Whether the sketch of an mm-row matrix runs as k_sketch_rows: its 16-row
// tiles alone fill the chip (one workgroup each), the sketch would otherwise
// be split along K (splits > 1), and the block is at most 32 columns wide
// (wider blocks reuse an LDS-staged Omega slab across 128 rows instead).
bool use_sketch_rows(int64_t mm, int64_t splits, int64_t bn) {
  return splits > 1 && cdiv(mm, 16) >= 256 && bn <= 32;
}

bool plan(const eodabe_ctx* ctx, int64_t m, int64_t n, int64_t lda, const void* A,
          int64_t r_cap, Geo& g) {
  if (m < 0 || n < 0) return false;
  const int dt = ctx->o.a_dtype;
  g.elem = dt == EODABE_F64 ? 8 : 4;
  g.transposed = m < n;
  g.mm = g.transposed ? n : m;
  g.nn = g.transposed ? m : n;
  const int64_t mn = std::min(m, n);
  if (r_cap == 0) r_cap = mn;
  if (r_cap < 0 || r_cap > mn) return false;
  g.r_cap = r_cap;
  const bool aligned = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  g.packed = g.transposed || !aligned;
  g.lda_eff = g.packed ? rup(std::max<int64_t>(g.nn, 1), 4) : lda;
  g.lp = (dt == EODABE_F32) ? ctx->o.sketch_dtype : 0;
  g.ld_lp = rup(std::max<int64_t>(g.nn, 1), 8);
  g.paired = ctx->cplx_pairs;
  if (g.paired) g.lp = 0;
  g.wide = ctx->pred_params != nullptr && g.lp == 0 && g.nn > 64 && ctx->o.block <= 64 && !g.paired;
  // paired: opts.block complex columns per block, i.e. twice as many real ones
  g.b = g.paired ? 2 * std::min(ctx->o.block, 64) : ctx->o.block;
  g.bn = (int)rup(g.b, 16);
  g.nblk = cdiv(g.nn, g.b);
  g.ldk = rup(std::max<int64_t>(g.nn, 1), 4);
  g.ldy = rup(std::max<int64_t>(g.mm, 1), 4);
  // K-splits: aim for ~2048 waves on the sketch, at least 256 K per split.
  const int64_t mt = std::max<int64_t>(cdiv(g.mm, 128), 1);
  int64_t s = cdiv(512, mt);
  s = std::min<int64_t>(s, std::max<int64_t>(g.nn / 256, 1));
  g.s_sketch = (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
  // Matrices whose 16-row tiles alone fill the chip (one workgroup each) and
  // whose sketch would otherwise be split along K: no partials at all.
  g.sk_rows = use_sketch_rows(g.mm, g.s_sketch, g.bn) && !g.paired;
  g.s_proj = (int)std::max<int64_t>(1, std::min<int64_t>(64, g.mm / 256));
  g.s_gram = (int)std::max<int64_t>(1, std::min<int64_t>(64, g.mm / 2048));
  // C = Q^T A: output r x nn is small, the reduction over mm is long.
  const int64_t rc1 = std::max<int64_t>(r_cap, 1);
  const int64_t tiles = cdiv(std::max<int64_t>(g.nn, 1), 256) * cdiv(rc1, 64);
  int64_t sc = std::max<int64_t>(1, std::min<int64_t>(cdiv(2048, tiles), g.mm / 256));
  const int64_t per = rc1 * g.ldk * (int64_t)g.elem;
  while (sc > 1 && sc * per > ((int64_t)1 << 29)) sc /= 2;
  g.s_core = (int)std::min<int64_t>(sc, 1024);
  return true;
}

// ------------------------------------------------------------------------
// Typed enqueue helpers.
// ------------------------------------------------------------------------
template <typename T>
struct Ops {
  eodabe_ctx* ctx;
  hipStream_t st;
  // Timed launches (sketch, projection): when set, the events are attached
  // to the kernel's own dispatch (start and end of its execution).
  hipEvent_t pe0 = nullptr, pe1 = nullptr;

  // out_parts = X (M x K, row-major ldx) * Z (N x K, row-major ldz)^T
  template <typename Tacc>
  int gemm_nt(const T* X, int64_t ldx, const T* Z, int64_t ldz, int64_t M, int64_t N, int64_t K,
              int splits, Tacc* out, int64_t ldo, int64_t part_stride, double* sumsq = nullptr,
              const int64_t* wlog = nullptr, const int32_t* stopb = nullptr, int blk = 0) {
    if (M <= 0 || N <= 0) return 0;
    const int64_t kchunk = split_chunk(K, splits);
    splits = eff_splits(K, splits);
    if (N <= 16) {
      dim3 grid((unsigned)cdiv(M, 128), splits, 1);
      hipLaunchKernelGGL((k_gemm_nt<T, Tacc, 2, 1>), grid, dim3(256), 0, st, X, ldx, Z, ldz, M, N, K,
                         kchunk, out, ldo, part_stride, sumsq, wlog, stopb, blk);
    } else if (N <= 32) {
      dim3 grid((unsigned)cdiv(M, 128), splits, 1);
      hipLaunchKernelGGL((k_gemm_nt<T, Tacc, 2, 2>), grid, dim3(256), 0, st, X, ldx, Z, ldz, M, N, K,
                         kchunk, out, ldo, part_stride, sumsq, wlog, stopb, blk);
    } else {
      dim3 grid((unsigned)cdiv(M, 128), splits, (unsigned)cdiv(N, 64));
      hipLaunchKernelGGL((k_gemm_nt<T, Tacc, 2, 4>), grid, dim3(256), 0, st, X, ldx, Z, ldz, M, N, K,
                         kchunk, out, ldo, part_stride, sumsq, wlog, stopb, blk);
    }
    LAUNCHCHK();
    return 0;
  }

  // Y partials = A Omega^T (bn <= 128 columns), see k_sketch
  // lp_write (1 FP16, 2 BF16; FP32 data only): also store the low-precision
  // copy of A (scaled by lp_st->lp_scale) to lp_out (row-major, ld_lp).
  int sketch(const T* A, int64_t lda, const T* Om, int64_t ldk, int64_t M, int bn, int64_t K,
             int splits, T* out, int64_t ldo, int64_t part_stride, double* sumsq,
             const int32_t* stopb, int blk, float* maxabs = nullptr, int lp_write = 0,
             uint16_t* lp_out = nullptr, int64_t ld_lp = 0, const State* lp_st = nullptr) {
    if (M <= 0 || bn <= 0) return 0;
    const int64_t kchunk = split_chunk(K, splits);
    splits = eff_splits(K, splits);
#define SK_LAUNCH(CC, LW)                                                                             \
  do {                                                                                                \
    dim3 grid((unsigned)cdiv(M, 128), splits, 1);                                                     \
    hipExtLaunchKernelGGL((k_sketch<T, 2, CC, LW>), grid, dim3(256), 0, st, pe0, pe1, 0, A, lda, Om,  \
                          ldk, M, bn, K, kchunk, out, ldo, part_stride, sumsq, maxabs, lp_out, ld_lp, \
                          lp_st, stopb, blk);                                                         \
  } while (0)
#define SK_CASE(CC)                                                                                   \
  do {                                                                                                \
    if constexpr (sizeof(T) == 4) {                                                                   \
      if (lp_write == 1) SK_LAUNCH(CC, 1);                                                            \
      else if (lp_write == 2) SK_LAUNCH(CC, 2);                                                       \
      else SK_LAUNCH(CC, 0);                                                                          \
    } else {                                                                                          \
      if (lp_write) return EODABE_EINVAL;                                                             \
      SK_LAUNCH(CC, 0);                                                                               \
    }                                                                                                 \
  } while (0)
    if (bn <= 16) SK_CASE(1);
    else if (bn <= 32) SK_CASE(2);
    else if (bn <= 48) SK_CASE(3);
    else if (bn <= 64) SK_CASE(4);
    else if (bn <= 96) SK_CASE(6);
    else SK_CASE(8);
#undef SK_CASE
#undef SK_LAUNCH
    LAUNCHCHK();
    return 0;
  }

  // Y = A Omega straight into Y (no K-split partials), see k_sketch_rows;
  // Omt in the tiled layout of k_omega_tiled, bn <= 32; sumsq / maxabs
  // receive one partial per 16-row tile.
  int sketch_rows(const T* A, int64_t lda, const T* Omt, int64_t M, int bn, int64_t K, T* Y, int64_t ldy,
                  double* sumsq, const int32_t* stopb, int blk, float* maxabs = nullptr, int lp_write = 0,
                  uint16_t* lp_out = nullptr, int64_t ld_lp = 0, const State* lp_st = nullptr) {
    if (M <= 0 || bn <= 0) return 0;
    if (bn > 32 || (lp_write && sizeof(T) != 4) || (maxabs && !sumsq)) return EODABE_EINVAL;
    if (cdiv(M, 16) > 0x7fffffff) return EODABE_EINVAL;
#define SR_LAUNCH(CC, LW, SS)                                                                         \
  hipExtLaunchKernelGGL((k_sketch_rows<T, CC, SKETCH_ROWS_WAVES, LW, SS>), dim3((unsigned)cdiv(M, 16)), \
                        dim3(64 * SKETCH_ROWS_WAVES), 0, st, pe0, pe1, 0, A, lda, Omt, M, bn, K, Y, ldy,  \
                        sumsq, maxabs, lp_out, ld_lp, lp_st, stopb, blk)
#define SR_SS(CC, LW)                                  \
  do {                                                 \
    if (!sumsq) SR_LAUNCH(CC, LW, 0);                  \
    else if (!maxabs) SR_LAUNCH(CC, LW, 1);            \
    else SR_LAUNCH(CC, LW, 2);                         \
  } while (0)
#define SR_CASE(CC)                                    \
  do {                                                 \
    if constexpr (sizeof(T) == 4) {                    \
      if (lp_write == 1) SR_SS(CC, 1);                 \
      else if (lp_write == 2) SR_SS(CC, 2);            \
      else SR_SS(CC, 0);                               \
    } else {                                           \
      SR_SS(CC, 0);                                    \
    }                                                  \
  } while (0)
    if (bn <= 16) SR_CASE(1);
    else SR_CASE(2);
#undef SR_CASE
#undef SR_SS
#undef SR_LAUNCH
    LAUNCHCHK();
    return 0;
  }

  // Low-precision sketch partials from the FP16 (lp 1) or BF16 (lp 2) copy of A.
  int sketch_lp(int lp, const uint16_t* Alp, int64_t ld_lp, const float* Om, int64_t ldk, int64_t M,
                int bn, int64_t K, int splits, float* out, int64_t ldo, int64_t part_stride,
                const State* lp_st, const int32_t* stopb, int blk) {
    if (M <= 0 || bn <= 0) return 0;
    const int64_t kchunk = split_chunk(K, splits);
    splits = eff_splits(K, splits);
#define SL_LAUNCH(LP, CC)                                                                             \
  do {                                                                                                \
    dim3 grid((unsigned)cdiv(M, 128), splits, 1);                                                     \
    hipExtLaunchKernelGGL((k_sketch_lp<LP, CC>), grid, dim3(256), 0, st, pe0, pe1, 0, Alp, ld_lp, Om, \
                          ldk, M, bn, K, kchunk, out, ldo, part_stride, lp_st, stopb, blk);           \
  } while (0)
#define SL_CASE(CC)                          \
  do {                                       \
    if (lp == 1) SL_LAUNCH(1, CC);           \
    else SL_LAUNCH(2, CC);                   \
  } while (0)
    if (bn <= 16) SL_CASE(1);
    else if (bn <= 32) SL_CASE(2);
    else if (bn <= 48) SL_CASE(3);
    else if (bn <= 64) SL_CASE(4);
    else if (bn <= 96) SL_CASE(6);
    else SL_CASE(8);
#undef SL_CASE
#undef SL_LAUNCH
    LAUNCHCHK();
    return 0;
  }

  // M_dev: row count read on the device (M is then its host-side bound).
  int gemm_nn(const T* X, int64_t ldx, const T* Z, int64_t ldz, int64_t M, int64_t N, int64_t K,
              int splits, T* out, int64_t ldo, int64_t part_stride, Gate gate = Gate{},
              const int64_t* M_dev = nullptr) {
    if (M <= 0 || N <= 0) return 0;
    if (cdiv(N, 256) > 65535) return EODABE_EINVAL;   // grid y holds the 256-column panels
    const int64_t kchunk = split_chunk(K, splits);
    splits = eff_splits(K, splits);
    // rows of the output per wave: 16*RT with RT = ceil(M/16) up to 4, so a
    // small rank does not spend MFMA cycles on padding rows
    const int rt = (int)std::min<int64_t>(4, cdiv(M, 16));
    dim3 grid((unsigned)splits, (unsigned)cdiv(N, 256), (unsigned)cdiv(M, 16 * rt));
#define NN_CASE(RR)                                                                                   \
  hipExtLaunchKernelGGL((k_gemm_nn<T, RR>), grid, dim3(256), 0, st, pe0, pe1, 0, X, ldx, Z, ldz, M, N, \
                        K, kchunk, out, ldo, part_stride, gate, M_dev)
    if (rt == 1) NN_CASE(1);
    else if (rt == 2) NN_CASE(2);
    else if (rt == 3) NN_CASE(3);
    else NN_CASE(4);
#undef NN_CASE
    LAUNCHCHK();
    return 0;
  }

  // Partials of (Q_lp^T A_lp) / scale (lp 1 FP16, 2 BF16; FP32 data only):
  // X = Q^T row-major (ldx), Z = the low-precision copy of A (ldz), see
  // k_gemm_nn_lp.
  int gemm_nn_lp(int lp, const float* X, int64_t ldx, const uint16_t* Z, int64_t ldz, int64_t M, int64_t N,
                 int64_t K, int splits, float* out, int64_t ldo, int64_t part_stride, const State* lp_st) {
    if (M <= 0 || N <= 0) return 0;
    if (cdiv(N, 256) > 65535) return EODABE_EINVAL;
    const int64_t kchunk = split_chunk(K, splits);
    splits = eff_splits(K, splits);
    const int rt = (int)std::min<int64_t>(4, cdiv(M, 16));
    dim3 grid((unsigned)splits, (unsigned)cdiv(N, 256), (unsigned)cdiv(M, 16 * rt));
#define NL_CASE(LP, RR)                                                                              \
  hipLaunchKernelGGL((k_gemm_nn_lp<LP, RR>), grid, dim3(256), 0, st, X, ldx, Z, ldz, M, N, K, kchunk, out, \
                     ldo, part_stride, lp_st)
#define NL_RT(LP)                    \
  do {                               \
    if (rt == 1) NL_CASE(LP, 1);     \
    else if (rt == 2) NL_CASE(LP, 2); \
    else if (rt == 3) NL_CASE(LP, 3); \
    else NL_CASE(LP, 4);             \
  } while (0)
    if (lp == 1) NL_RT(1);
    else NL_RT(2);
#undef NL_RT
#undef NL_CASE
    LAUNCHCHK();
    return 0;
  }

  template <typename U>
  int reduce(const U* parts, int nparts, int64_t stride, int64_t count, U* out,
             const int32_t* stopb = nullptr, int blk = 0, Gate gate = Gate{}) {
    if (count <= 0) return 0;
    unsigned nb = (unsigned)std::min<int64_t>(cdiv(count, 256), 4096);
    hipLaunchKernelGGL((k_reduce_parts<U>), dim3(nb), dim3(256), 0, st, parts, nparts, stride, count,
                       out, stopb, blk, gate);
    LAUNCHCHK();
    return 0;
  }

  template <typename U>
  int reduce_wide(const U* parts, int nparts, int64_t stride, int64_t count, U* out,
                  const int32_t* stopb = nullptr, int blk = 0, Gate gate = Gate{}) {
    if (count <= 0) return 0;
    if (nparts <= 4) return reduce(parts, nparts, stride, count, out, stopb, blk, gate);
    // many partials over few elements: spread each element group's partials
    // over P threads (few elements: count below 2^17, fewer than 256 workgroups)
    const int P = (count <= (1 << 17) && nparts >= 128) ? 16 : (count <= (1 << 17) && nparts >= 48) ? 4 : 1;
#define FOLD_P(PP)                                                                                       \
  hipLaunchKernelGGL((k_fold_parts<U, PP>), dim3((unsigned)cdiv(count, 512 / PP)), dim3(128), 0, st, parts, \
                     nparts, stride, count, out, stopb, blk, gate)
    if (P == 16) FOLD_P(16);
    else if (P == 4) FOLD_P(4);
    else FOLD_P(1);
#undef FOLD_P
    LAUNCHCHK();
    return 0;
  }

  // Z = X W for blocks of f <= 128 columns (one job, or two in one launch).
  int apply(const ApplyJob& j0, const ApplyJob* j1, int f, const int32_t* stopb = nullptr,
            int blk = 0, Gate gate = Gate{}) {
    if (f <= 0) return 0;
    const int64_t rows = std::max<int64_t>(j0.rows, j1 ? j1->rows : 0);
    if (rows <= 0) return 0;
    dim3 grid((unsigned)cdiv(rows, 64), j1 ? 2 : 1);
    // k_apply takes its 64-row blocks grid-stride: up to 32 columns at most
    // APPLY_WG workgroups, each staging W once; wider, one block each
    const dim3 gs((unsigned)(f <= 32 ? std::min<int64_t>(grid.x, APPLY_WG) : grid.x), grid.y);
    const ApplyJob jb = j1 ? *j1 : j0;
    if (f <= 16)
      hipLaunchKernelGGL((k_apply<T, 16>), gs, dim3(256), 0, st, j0, jb, stopb, blk, gate);
    else if (f <= 32)
      hipLaunchKernelGGL((k_apply<T, 32>), gs, dim3(256), 0, st, j0, jb, stopb, blk, gate);
    else if (f <= 64)
      hipLaunchKernelGGL((k_apply<T, 64>), gs, dim3(256), 0, st, j0, jb, stopb, blk, gate);
    else if (f <= 128 && j0.Z != j0.X && jb.Z != jb.X)   // output columns over four workgroups
      hipLaunchKernelGGL((k_apply_cols<T, 128>), dim3(grid.x, grid.y, 4), dim3(256), 0, st, j0, jb, stopb, blk,
                         gate);
    else if (f <= 128)
      hipLaunchKernelGGL((k_apply<T, 128>), gs, dim3(256), 0, st, j0, jb, stopb, blk, gate);
    else
      return EODABE_EINVAL;
    LAUNCHCHK();
    return 0;
  }

  // Y = Q W with an FP64 W (column-major, ldw); FP64 accumulation.
  int update_d(T* Y, int64_t ldy, const T* Q, int64_t ldq, int64_t m, int64_t w, int f,
               const double* W, int64_t ldw) {
    if (m <= 0 || f <= 0) return 0;
    dim3 grid((unsigned)cdiv(m, 64), (unsigned)cdiv(f, 64));
    hipLaunchKernelGGL((k_update_rows<T, double>), grid, dim3(256), 0, st, Y, ldy, Q, ldq, m, w, f,
                       W, ldw, 0, (const int64_t*)nullptr, (const int32_t*)nullptr, 0);
    LAUNCHCHK();
    return 0;
  }

  int update(T* Y, int64_t ldy, const T* Q, int64_t ldq, int64_t m, int64_t w, int f, const T* W,
             int64_t ldw, int subtract, const int64_t* wlog = nullptr, const int32_t* stopb = nullptr,
             int blk = 0) {
    if (m <= 0 || f <= 0) return 0;
    if (cdiv(m, 16) > 0x7fffffff) return EODABE_EINVAL;
#define UT_LAUNCH(CC)                                                                                 \
  hipLaunchKernelGGL((k_update_tiles<T, CC, 4>), dim3((unsigned)cdiv(m, 16), (unsigned)cdiv(f, 16 * CC)), \
                     dim3(256), 0, st, Y, ldy, Q, ldq, m, w, f, W, ldw, subtract, wlog, stopb, blk)
    if (f <= 16) UT_LAUNCH(1);
    else if (f <= 32) UT_LAUNCH(2);
    else UT_LAUNCH(4);
#undef UT_LAUNCH
    LAUNCHCHK();
    return 0;
  }
};

CholArgs chol_args(const WS& w, double* R, int32_t* dead, int first, int fresh, int count_floors) {
  CholArgs ca{};
  ca.R = R;
  ca.dead = dead;
  ca.first_pass = first;
  ca.fresh = fresh;
  ca.st = w.st;
  ca.count_floors = count_floors;
  return ca;
}

// Panel-blocked Cholesky with inverse of an f x f Gram matrix (k_cb_*; G,
// R, R^{-1} column-major, leading dimension f; G overwritten by the Schur
// complements): one workgroup on each diagonal block, the independent 64 x 64
// block products of a step on separate workgroups, R^{-1} by recursive
// doubling.  dg: f doubles; cbmask: two words per 64-column panel.
void cb_chol(hipStream_t st, double* G, int f, double* R, double* Rinv, double* dg, int32_t* dead,
             uint64_t* cbmask, int first_pass, int fresh, State* state, int count_floors,
             const int32_t* stopb = nullptr, int blk = 0) {
  const int P = (int)cdiv(f, 64);
  const int64_t ff = (int64_t)f * f;
  if (P == 2) {                          // two panels: one workgroup, every block in LDS
    hipLaunchKernelGGL(k_chol2p, dim3(1), dim3(256), 0, st, G, f, f, R, Rinv, dead, first_pass, fresh, state,
                       count_floors, stopb, blk);
    return;
  }
  hipLaunchKernelGGL(k_cb_init, dim3((unsigned)std::min<int64_t>(cdiv(ff, 256), 1024)), dim3(256), 0, st, G, f, f,
                     R, Rinv, dg, dead, fresh, stopb, blk);
  hipLaunchKernelGGL(k_cb_diag, dim3(1), dim3(256), 0, st, G, f, f, 0, R, Rinv, dg, dead, cbmask, first_pass,
                     state, count_floors, stopb, blk);
  uint64_t* deadmask = cbmask + P;        // dead flags found by the steps p >= 1
  for (int p = 0; p + 1 < P; ++p) {
    // R_p. and the trailing update of step p, the diagonal step p+1 on its workgroup 0
    hipLaunchKernelGGL(k_cb_look, dim3((P - p - 1) * (P - p) / 2), dim3(256), 0, st, G, f, f, p, R, Rinv, dg,
                       dead, cbmask, deadmask, first_pass, state, count_floors, stopb, blk);
  }
  for (int L = 1; L < P; L *= 2) {                       // R^{-1} by recursive doubling
    int nb = 0;
    for (int a = 0; a + L < P; a += 2 * L) nb += L * (std::min(a + 2 * L, P) - (a + L));
    if (L == 1) {
      hipLaunchKernelGGL(k_cb_inv, dim3(nb), dim3(256), 0, st, R, Rinv, G, f, f, L, 2, deadmask, dead, stopb, blk);
    } else {
      hipLaunchKernelGGL(k_cb_inv, dim3(nb), dim3(256), 0, st, R, Rinv, G, f, f, L, 0, deadmask, dead, stopb, blk);
      hipLaunchKernelGGL(k_cb_inv, dim3(nb), dim3(256), 0, st, R, Rinv, G, f, f, L, 1, deadmask, dead, stopb, blk);
    }
  }
}

// The one-launch CholeskyQR2 (k_cqr2) takes blocks of at most 32 columns
// whose row panels fit its grid (every workgroup resident at once).
bool cqr2_fits(int64_t rows, int64_t f) {
  return f > 0 && f <= 32 && rows > 0 && cdiv(rows, CQR2_RPW) <= CQR2_GMAX;
}

template <typename T>
int cqr2(eodabe_ctx* ctx, hipStream_t st, const Cqr2Args& a_in, bool proj = false) {
  const int64_t fb = a_in.f;                       // the launch width (the bound of f_dev)
  if (!cqr2_fits(a_in.rows, fb)) return EODABE_EINVAL;
  Cqr2Args a = a_in;
  if (ctx->barrier_fail) {                         // 10 us waits for an arrival that never comes
    a.wait_extra = 1;
    a.wait_ticks = 1000;
  }
  const dim3 grid((unsigned)cdiv(a.rows, CQR2_RPW));
  if (proj) {
    if (fb <= 16) hipLaunchKernelGGL((k_cqr2<T, 16, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_cqr2<T, 32, true>), grid, dim3(256), 0, st, a);
  } else {
    if (fb <= 16) hipLaunchKernelGGL((k_cqr2<T, 16, false>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_cqr2<T, 32, false>), grid, dim3(256), 0, st, a);
  }
  LAUNCHCHK();
  return 0;
}

// G = Z^T Z (FP64) of the rows x f block Z = X (W null) or Z = X W (W f x f
// FP64, element (i,j) at j*f + i, Z rounded to T and written over X), then
// the Cholesky with the floor/kill rules and the epilogues in ca (R,
// R^{-1}, stop test, ||A||_F finish).  f <= 64: one launch (k_gram_rows; its last workgroup runs the
// Cholesky with inverse).  Wider: generic GEMM as K-split partials, then the
// panel-blocked Cholesky with inverse as one kernel per step (k_cb_*, the
// Gram overwritten), separate stop test.  Above 64 columns ca.Rinv is
// required and there is no fused W.
template <typename T>
int gram_chol(eodabe_ctx* ctx, hipStream_t st, const WS& w, T* X, int64_t ld, int64_t rows, int f,
              double* parts, const CholArgs& ca, const int32_t* stopb = nullptr, int blk = 0,
              const double* W = nullptr, int64_t max_wg = 64) {
  if (f <= 0) return 0;
  if (f <= 64) {
    uint32_t* counter = &w.st->counter[0];
    const int64_t cap = max_wg;
#define GRAM_CASE(FF, MM)                                                                            \
  do {                                                                                               \
    const int64_t npan = cdiv(rows, GramCfg<T, FF, MM>::RPW);                                        \
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(npan, cap));              \
    hipLaunchKernelGGL((k_gram_rows<T, FF, MM>), dim3(grid), dim3(256), 0, st, X, ld, rows, f, W,    \
                       parts, counter, stopb, blk, ca);                                              \
  } while (0)
#define GRAM_F(FF)                   \
  do {                               \
    if (W) GRAM_CASE(FF, 1);         \
    else GRAM_CASE(FF, 0);           \
  } while (0)
    if (f <= 16) GRAM_F(16);
    else if (f <= 32) GRAM_F(32);
    else GRAM_F(64);
#undef GRAM_F
#undef GRAM_CASE
    LAUNCHCHK();
    return 0;
  }
  if (W || ca.gate.st || ca.f_dev || !ca.Rinv) return EODABE_EINVAL;   // fused / gated forms only for f <= 64
  Ops<T> ops{ctx, st};
  if (ca.norm_parts)
    hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(256), 0, st, ca.norm_parts, ca.max_parts, ca.n_norm,
                       w.st);
  // G = X^T X as K-split partials summed in fixed order: up to 63 splits of
  // at least 64 rows for f <= 128 (the partial buffers hold 64 such
  // matrices; more splits put more workgroups on the FP64 products),
  // GRAM_SPLITS_WIDE of at least 512 rows above
  const int gs = (int)std::max<int64_t>(
      1, f <= 128 ? std::min<int64_t>(63, rows / 64) : std::min<int64_t>(GRAM_SPLITS_WIDE, rows / 512));
  const int64_t ff = (int64_t)f * f;
  double* gsum = parts + (int64_t)gs * ff;
  TRY(ops.template gemm_nt<double>(X, ld, X, ld, f, f, rows, gs, parts, f, ff, nullptr, nullptr, stopb, blk));
  TRY(ops.reduce_wide(parts, eff_splits(rows, gs), ff, ff, gsum, stopb, blk));
  parts = gsum;
  // panel-blocked, one kernel per step (see k_cb_*); every step returns at
  // once for a speculative block after the stop
  cb_chol(st, parts, f, ca.R, ca.Rinv, w.dg, ca.dead, w.cbmask, ca.first_pass, ca.fresh, w.st, ca.count_floors,
          stopb, blk);
  if (ca.R1)
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, st, ca.R1, ca.R, ca.dead, f, ca.col0, ca.n, w.st,
                       ca.wlog, ca.acc, ca.diag_log, blk);
  LAUNCHCHK();
  return 0;
}

// CholeskyQR2 of X (rows x f, element (i,c) at c*ld + i), first Cholesky
// pass floored.  The orthonormal factor goes to Zout (leading dimension ldz;
// X itself when Zout is null).  Blocks wider than 64 columns also write
// R = R2 R1 (element (i,j) at j*f + i, or its transpose when transpose_R) to
// Rout and optionally R in the data type, row-major, to Dout (ldd), and
// overwrite X.
template <typename T>
int cholqr2(eodabe_ctx* ctx, hipStream_t st, const Geo& g, const WS& w, T* X, int64_t ld,
            int64_t rows, int f, double* Rout, int transpose_R, T* tmp, T* Zout = nullptr,
            int64_t ldz = 0, T* Dout = nullptr, int64_t ldd = 0) {
  (void)g;
  Ops<T> ops{ctx, st};
  if (f <= 0 || rows <= 0) return 0;
  if (!Zout) {
    Zout = X;
    ldz = ld;
  }
  if (f <= 128) {
    // [Gram, Cholesky with inverse] -> R1 (rb1), R1^{-1} (rb3); [X := X R1^{-1},
    // Gram, Cholesky with inverse] -> R2 (rb2), R2^{-1} (rb5); Z = X R2^{-1}.
    // Up to 64 columns the normalisation is fused into the second Gram
    // kernel.  Rout and Dout are not written on this path (the closing
    // steps take R1, R2 from rb1, rb2).
    CholArgs c1 = chol_args(w, w.rb1, w.deadbig, 1, 1, 1);
    c1.Rinv = w.rb3;
    TRY(gram_chol<T>(ctx, st, w, X, ld, rows, f, w.gbig, c1));
    CholArgs c2 = chol_args(w, w.rb2, w.deadbig, 0, 0, 1);
    c2.Rinv = w.rb5;
    if (f <= 64) {
      TRY(gram_chol<T>(ctx, st, w, X, ld, rows, f, w.gbig, c2, nullptr, 0, w.rb3));
    } else {
      const ApplyJob a1{X, ld, X, ld, w.rb3, rows, 0, f, f, nullptr, nullptr, nullptr};
      TRY(ops.apply(a1, nullptr, f));
      TRY(gram_chol<T>(ctx, st, w, X, ld, rows, f, w.gbig, c2));
    }
    const ApplyJob a{X, ld, Zout, ldz, w.rb5, rows, 0, f, f, nullptr, nullptr, nullptr};
    TRY(ops.apply(a, nullptr, f));
    return 0;
  }
  // wider: [Gram, blocked Cholesky with inverse] twice, X := X R^{-1} through
  // scratch after each (explicit inverse, FP64 weights)
  double* Rs[2] = {w.rb1, w.rb2};
  double* Ris[2] = {w.rb3, w.rb5};
  for (int pass = 0; pass < 2; ++pass) {
    CholArgs ca = chol_args(w, Rs[pass], w.deadbig, pass == 0, pass == 0, 1);
    ca.Rinv = Ris[pass];
    TRY(gram_chol<T>(ctx, st, w, X, ld, rows, f, w.gbig, ca));
    TRY(ops.update_d(tmp, ld, X, ld, rows, f, f, Ris[pass], f));
    const int64_t cnt = ld * (int64_t)f;
    hipLaunchKernelGGL((k_copy2d<T, T>), dim3((unsigned)cdiv(cnt, 32), 1), dim3(32, 8), 0, st, tmp,
                       cnt, X, cnt, (int64_t)1, cnt, 0);
    LAUNCHCHK();
  }
  const int64_t ff = (int64_t)f * f;
  hipLaunchKernelGGL(k_trimul, dim3((unsigned)(cdiv(f, 64) * cdiv(f, 64))), dim3(256), 0, st, w.rb2, w.rb1, f,
                     Rout, transpose_R);
  LAUNCHCHK();
  if (Zout != X) {
    dim3 grid((unsigned)cdiv(rows, 32), (unsigned)cdiv(f, 32));
    hipLaunchKernelGGL((k_copy2d<T, T>), grid, dim3(32, 8), 0, st, X, ld, Zout, ldz, (int64_t)f, rows,
                       0);
    LAUNCHCHK();
  }
  if (Dout) {
    if (transpose_R) return EODABE_EINVAL;
    dim3 grid((unsigned)cdiv(f, 32), (unsigned)cdiv(f, 32));
    hipLaunchKernelGGL((k_copy2d<double, T>), grid, dim3(32, 8), 0, st, Rout, (int64_t)f, Dout, ldd,
                       (int64_t)f, (int64_t)f, 1);
    LAUNCHCHK();
  }
  return 0;
}

template <typename T>
int copy2d(eodabe_ctx* ctx, hipStream_t st, const T* src, int64_t lds, T* dst, int64_t ldd,
           int64_t rows, int64_t cols, int transpose) {
  if (rows <= 0 || cols <= 0) return 0;
  dim3 grid((unsigned)cdiv(cols, 32), (unsigned)cdiv(rows, 32));
  hipLaunchKernelGGL((k_copy2d<T, T>), grid, dim3(32, 8), 0, st, src, lds, dst, ldd, rows, cols,
                     transpose);
  LAUNCHCHK();
  return 0;
}

// Alg. 1 on the (already oriented) mm x nn matrix Ae.  On return the basis
// is in w.q (column-major, ld g.ldy) and *rank holds its width.
// after_chunk(jend) is called once the blocks [.., jend) are enqueued and
// before the host reads the stop flag; it returns 1 if it enqueued the
// (gated) closing steps, 2 if those steps also write the control block to
// the context's host copy (no copy needed), 0 if not, < 0 on error.  *spec_ran tells whether
// such closing steps ran to completion for the chunk that ended the loop.
template <typename T, typename Hook>
int run_basis(eodabe_ctx* ctx, hipStream_t st, const Geo& g, const WS& w, const T* Ae, double tol,
              int64_t* rank, int* blocks, double* norm_a, Hook&& after_chunk, bool* spec_ran) {
  *spec_ran = false;
  Ops<T> ops{ctx, st};
  const uint32_t k0 = (uint32_t)(ctx->o.seed & 0xffffffffu), k1 = (uint32_t)(ctx->o.seed >> 32);
  const int nwlog = (int)(g.nblk + 2);
  const bool learned = g.wide && ctx->pred_params != nullptr;
  // The reset of the control block rides on block 0's tiled Omega launch when
  // that is the first launch (ungated), else it is a launch of its own.
  StateInit init{w.st, tol, w.wlog, nwlog, w.dead, (int64_t)(g.nblk + 1) * BN_MAX, w.accv, (int)(g.nblk + 1),
                 g.lp, g.paired ? 1 : 0};
  if (!(g.sk_rows && !learned && g.nn > 0)) {
    hipLaunchKernelGGL(k_init_state, dim3(64), dim3(256), 0, st, init.st, init.tol, init.wlog, init.nwlog,
                       init.dead, init.ndead, init.acc, init.nacc, init.lp_mode, init.paired);
    LAUNCHCHK();
    init.st = nullptr;
  }
  T* omega = (T*)w.omega;
  T* y = (T*)w.y;
  T* q = (T*)w.q;
  T* wbuf = (T*)w.w;
  const int64_t ldw = ldw_of(g);
  const int32_t* stopb = &w.st->stop_block;
  // blocks enqueued before each host check of the stop flag: 1, 2, 4, 4, ...
  // (speculative blocks after the stop return at once from every kernel)
  int per_sync = ctx->o.blocks_per_sync > 0 ? ctx->o.blocks_per_sync : 1;
  int64_t j = 0;
  bool finished = (g.nn == 0);
  int64_t sketch_wgs = cdiv(g.mm, 128);
  // Learned warm start: the blocks covering Omega's first 64 columns run as
  // a probe; if they do not stop, the predictor reads their stopping-test
  // values (device) and returns a width d0; the blocks up to column d0 then
  // take their sketches from one wide pass over A (WIDE_COLS columns at a
  // time) and are orthogonalised as usual; past d0 the plain loop resumes.
  ctx->pred_last = {};
  bool probed = !learned;
  int64_t pred_end = 0;                 // warm-start end column (exclusive)
  int64_t pre_j0 = 0, pre_j1 = 0;       // blocks whose sketch sits in y_w
  while (!finished) {
    int64_t jend = std::min<int64_t>(g.nblk, j + per_sync);
    if (!probed) {
      jend = std::min<int64_t>(g.nblk, cdiv(64, g.b));
    } else if (learned && j * g.b < pred_end) {
      // one wide sketch for the next blocks up to the predicted width
      const int64_t kw = std::min<int64_t>({(int64_t)(WIDE_COLS / g.b), cdiv(pred_end - j * g.b, g.b), g.nblk - j});
      const int64_t col0 = j * g.b;
      const int fw = (int)std::min<int64_t>(kw * g.b, g.nn - col0);
      const int bnw = (int)rup(fw, 16);
      T* omw = (T*)w.omega_w;
      dim3 grid((unsigned)cdiv(cdiv(g.ldk, 4), 256), bnw);
      hipLaunchKernelGGL((k_omega<T>), grid, dim3(256), 0, st, k0, k1, g.nn, col0, fw, g.ldk, omw, stopb, (int)j);
      if (fw < bnw)
        hipLaunchKernelGGL(k_zero<T>, dim3(64), dim3(256), 0, st, omw + (int64_t)fw * g.ldk,
                           (int64_t)(bnw - fw) * g.ldk);
      LAUNCHCHK();
      const int64_t ystride = g.ldy * bnw;
      const int pid = prof_begin(ctx, st);
      prof_attach(ctx, ops, pid);
      TRY(ops.sketch(Ae, g.lda_eff, omw, g.ldk, g.mm, bnw, g.nn, g.s_sketch, (T*)w.ypart_w, g.ldy, ystride,
                     nullptr, stopb, (int)j));
      prof_attach(ctx, ops, -1);
      prof_end(ctx, st, pid, EODABE_PROF_SKETCH, (int)j,
               (double)g.elem * ((double)g.mm * g.nn + (double)g.nn * fw + (double)g.mm * fw));
      TRY(ops.reduce_wide((const T*)w.ypart_w, eff_splits(g.nn, g.s_sketch), ystride, ystride, (T*)w.y_w,
                          stopb, (int)j));
      pre_j0 = j;
      pre_j1 = j + kw;
      jend = pre_j1;
    }
    for (; j < jend; ++j) {
      const int blk = (int)j;
      const int64_t col0 = j * g.b;
      const int f = (int)std::min<int64_t>(g.b, g.nn - col0);
      const bool pre = j >= pre_j0 && j < pre_j1;
      T* y = pre ? (T*)w.y_w + (j - pre_j0) * (int64_t)g.b * g.ldy : (T*)w.y;
      // the sketch of this block runs by 16-row tiles (tiled test matrix)
      const bool rows_blk = g.sk_rows && !(g.lp && j >= 2);
      // a1: Omega_j (bn rows; rows f..bn-1 zero)
      if (!pre) {
        if (rows_blk) {
          dim3 grid((unsigned)cdiv(cdiv(rup(g.nn, 16), 4), 256), g.bn);
          hipLaunchKernelGGL((k_omega_tiled<T>), grid, dim3(256), 0, st, k0, k1, g.nn, col0, f, g.bn / 16,
                             omega, stopb, blk, j == 0 ? init : StateInit{});
        } else if (g.paired) {
          dim3 grid((unsigned)cdiv(g.ldk, 256), f);
          hipLaunchKernelGGL((k_omega_paired<T>), grid, dim3(256), 0, st, k0, k1, g.nn, col0, f, g.ldk, omega,
                             stopb, blk);
        } else {
          dim3 grid((unsigned)cdiv(cdiv(g.ldk, 4), 256), g.bn);
          hipLaunchKernelGGL((k_omega<T>), grid, dim3(256), 0, st, k0, k1, g.nn, col0, f, g.ldk, omega,
                             stopb, blk);
        }
        if (f < g.bn && !rows_blk)
          hipLaunchKernelGGL(k_zero<T>, dim3(64), dim3(256), 0, st, omega + (int64_t)f * g.ldk,
                             (int64_t)(g.bn - f) * g.ldk);
        LAUNCHCHK();
      }
      // a2: sketch Y = A Omega_j (K-split partials folded into Y, or Y written
      // by 16-row tiles directly; block 0 also ||A||_F)
      const int64_t ystride = g.ldy * g.bn;
      const int nsp = eff_splits(g.nn, g.s_sketch);
      // low-precision form: block 1 also writes the FP16/BF16 copy of A
      // (scale from block 0's max |A|), later blocks sketch that copy
      if (!pre) {
      const int pid = prof_begin(ctx, st);
      prof_attach(ctx, ops, pid);
      double abytes = (double)g.elem * g.mm * g.nn;
      if (g.lp && j >= 2) {
        if constexpr (sizeof(T) == 4)
          TRY(ops.sketch_lp(g.lp, w.alp, g.ld_lp, omega, g.ldk, g.mm, g.bn, g.nn, g.s_sketch,
                            (T*)w.ypart, g.ldy, ystride, w.st, stopb, blk));
        abytes = 2.0 * g.mm * g.nn;
      } else if (rows_blk) {
        TRY(ops.sketch_rows(Ae, g.lda_eff, omega, g.mm, g.bn, g.nn, y, g.ldy, j == 0 ? w.normparts : nullptr,
                            stopb, blk, (j == 0 && g.lp) ? w.maxparts : nullptr, (g.lp && j == 1) ? g.lp : 0, w.alp,
                            g.ld_lp, w.st));
        if (g.lp && j == 1) abytes += 2.0 * g.mm * g.nn;
      } else {
        // one K-split: the sketch writes Y itself (no partial to fold)
        TRY(ops.sketch(Ae, g.lda_eff, omega, g.ldk, g.mm, g.bn, g.nn, g.s_sketch, nsp == 1 ? y : (T*)w.ypart, g.ldy,
                       ystride, j == 0 ? w.normparts : nullptr, stopb, blk,
                       (j == 0 && g.lp) ? w.maxparts : nullptr, (g.lp && j == 1) ? g.lp : 0, w.alp, g.ld_lp,
                       w.st));
        if (g.lp && j == 1) abytes += 2.0 * g.mm * g.nn;
      }
      prof_attach(ctx, ops, -1);
      prof_end(ctx, st, pid, EODABE_PROF_SKETCH, blk,
               abytes + (double)g.elem * ((double)g.nn * f + (double)g.mm * f));
      // partials to fold unless the sketch wrote Y itself
      const bool y_direct = rows_blk || (nsp == 1 && !(g.lp && j >= 2));
      if (j > 0 && !y_direct) TRY(ops.reduce_wide((const T*)w.ypart, nsp, ystride, ystride, y, stopb, blk));
      if (j > 0) TRY(pair_fix<T>(ctx, st, g.paired, y, g.ldy, g.mm, f, stopb, blk));
      }
      // a3 + a4: two rounds of [project against the basis so far (width
      // wlog[j] <= j*b), FP64-Gram Cholesky, triangular solve]: block
      // Gram-Schmidt with re-orthogonalisation interleaved with CholeskyQR2
      // (first Cholesky pass floored).  The second Cholesky also runs the
      // stop test (a5); the second solve is the append below.
      int32_t* deadj = w.dead + j * BN_MAX;
      const int64_t wmax = std::min<int64_t>(j * g.b, g.nn);
      const bool small = f <= 64;     // fused Gram + Cholesky-with-inverse kernels
      const bool mid = f <= 128;      // explicit R^{-1} (blocked Cholesky above 64 columns) + apply
      if (j == 0 && !(rows_blk || nsp == 1)) TRY(ops.reduce_wide((const T*)w.ypart, nsp, ystride, ystride, y, stopb, blk));
      if (j == 0) TRY(pair_fix<T>(ctx, st, g.paired, y, g.ldy, g.mm, f, stopb, blk));
      if (j == 0 && cqr2_fits(g.mm, f)) {
        // block 0: both CholeskyQR2 passes, the stop test and the append in
        // one launch (nothing to project against)
        Cqr2Args a{};
        a.X = y;
        a.ldx = g.ldy;
        a.rows = g.mm;
        a.f = f;
        a.parts = w.gpart;
        a.counter = &w.st->counter[1];
        a.stop_block = stopb;
        a.block_id = blk;
        a.st = w.st;
        a.R1 = w.r1;
        a.R1inv = w.r1inv;
        a.R2 = w.r2;
        a.R2inv = w.r2inv;
        a.dead = deadj;
        a.norm_parts = w.normparts;
        a.max_parts = g.lp ? w.maxparts : nullptr;
        a.n_norm = g.sk_rows ? cdiv(g.mm, 16) : sketch_wgs * (int64_t)nsp;
        a.stop_test = 1;
        a.col0 = col0;
        a.n = g.nn;
        a.wlog = w.wlog;
        a.acc = w.accv;
        a.diag_log = w.diag_log;
        a.Q = q;
        a.ldq = g.ldy;
        TRY(cqr2<T>(ctx, st, a));
        continue;
      }
      if (j > 0 && cqr2_fits(g.mm, f) && !g.paired && wmax <= CQR2_PROJ_WMAX) {
        // later blocks while the basis is narrow: both BCGS2 projections,
        // both CholeskyQR2 passes, the stop test and the append in one launch
        Cqr2Args a{};
        a.X = y;
        a.ldx = g.ldy;
        a.rows = g.mm;
        a.f = f;
        a.parts = w.gpart;
        a.counter = &w.st->counter[3];       // shared by these launches, reset by each one's last workgroup
        a.reuse_counter = 1;
        a.stop_block = stopb;
        a.block_id = blk;
        a.st = w.st;
        a.R1 = w.r1;
        a.R1inv = w.r1inv;
        a.R2 = w.r2;
        a.R2inv = w.r2inv;
        a.dead = deadj;
        a.stop_test = 1;
        a.col0 = col0;
        a.n = g.nn;
        a.wlog = w.wlog;
        a.acc = w.accv;
        a.diag_log = w.diag_log;
        a.Q = q;
        a.ldq = g.ldy;
        a.Qb = q;
        a.ldqb = g.ldy;
        a.w_dev = w.wlog + j;
        a.wparts = w.wfp;
        TRY(cqr2<T>(ctx, st, a, true));
        continue;
      }
      for (int pass = 0; pass < 2; ++pass) {
        if (j > 0) {
          TRY(ops.template gemm_nt<T>(q, g.ldy, y, g.ldy, wmax, f, g.mm, g.s_proj, (T*)w.wpart, ldw,
                                      ldw * g.bn, nullptr, w.wlog, stopb, blk));
          hipLaunchKernelGGL((k_reduce_cols<T>), dim3(256), dim3(256), 0, st, (const T*)w.wpart,
                             eff_splits(g.mm, g.s_proj), ldw * g.bn, wmax, (int64_t)f, ldw, wbuf, w.wlog,
                             stopb, blk);
          LAUNCHCHK();
          TRY(ops.update(y, g.ldy, q, g.ldy, g.mm, wmax, f, wbuf, ldw, 1, w.wlog, stopb, blk));
          TRY(pair_fix<T>(ctx, st, g.paired, y, g.ldy, g.mm, f, stopb, blk));
        }
        CholArgs ca = chol_args(w, pass == 0 ? w.r1 : w.r2, deadj, pass == 0, 0, 0);
        if (pass == 0) {
          if (mid) ca.Rinv = w.r1inv;
          if (j == 0) {
            ca.norm_parts = w.normparts;
            ca.max_parts = g.lp ? w.maxparts : nullptr;     // max |A|: the FP16 scale only
            ca.n_norm = g.sk_rows ? cdiv(g.mm, 16) : sketch_wgs * (int64_t)nsp;
          }
        } else {
          if (mid) ca.Rinv = w.r2inv;
          ca.R1 = w.r1;
          ca.col0 = col0;
          ca.n = g.nn;
          ca.wlog = w.wlog;
          ca.acc = w.accv;
          ca.diag_log = w.diag_log;
        }
        // Y := Y R1^{-1} between the passes.  Block 0 (nothing to project
        // against) lets the second Gram kernel form it in place; later blocks
        // normalise first, so that the second projection acts on the
        // normalised block (re-orthogonalisation needs that order).
        const bool fuse = small && j == 0;
        TRY(gram_chol<T>(ctx, st, w, y, g.ldy, g.mm, f, w.gpart, ca, stopb, blk,
                         (fuse && pass == 1) ? w.r1inv : nullptr, GRAM_LOOP_WG));
        if (pass == 0 && mid && !fuse) {
          const ApplyJob a{y, g.ldy, y, g.ldy, w.r1inv, g.mm, 0, f, f, nullptr, nullptr, nullptr};
          TRY(ops.apply(a, nullptr, f, stopb, blk));
        }
        if (pass == 0 && !mid) return EODABE_EINVAL;   // blocks are at most BN_MAX = 128 wide
      }
      // a6: append P = Z R2^{-1} (accepted columns) into Q at column wlog[j]
      if (mid) {
        const ApplyJob a{y, g.ldy, q, g.ldy, w.r2inv, g.mm, 0, f, 0, w.wlog, w.accv, nullptr};
        TRY(ops.apply(a, nullptr, f, stopb, blk));
      } else {
        return EODABE_EINVAL;          // blocks are at most BN_MAX = 128 wide
      }
    }
    const int spec = after_chunk(j);
    if (spec < 0) return spec;
    // host check of the stop flag (one small D2H copy per chunk, unless the
    // closing kernel wrote the control block to host memory itself: spec 2)
    if (spec != 2) HIPCHK(hipMemcpyAsync(ctx->host_state, w.st, sizeof(State), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const State& hs = *ctx->host_state;
    if (hs.sync_fail) return EODABE_ESYNC;
    if (hs.stop_block != 0x7fffffff || j >= g.nblk) finished = true;
    // the gated closing steps ran iff the loop stopped with a finite norm
    // and 0 < rank <= r_cap (the gate of those kernels)
    const bool ran = spec >= 1 && hs.stop_block != 0x7fffffff && !hs.nonfinite && hs.rank > 0 &&
                     hs.rank <= g.r_cap;
    if (ctx->prof_on)
      prof_collect(ctx, hs.stop_block != 0x7fffffff ? hs.stop_block : (int)g.nblk, ran, hs.rank);
    if (hs.nonfinite) return EODABE_ENONFINITE;
    if (finished) *spec_ran = ran;
    if (!probed) {
      probed = true;
      if (!finished) {
        // predictor on the device from the probe's stopping-test values
        hipLaunchKernelGGL(k_mlp_infer1, dim3(1), dim3(256), 0, st, ctx->pred_params, w.diag_log, g.mm, g.nn,
                           (const State*)w.st, g.b, ctx->pred_margin, w.pred);
        LAUNCHCHK();
        MlpPred hp{};
        HIPCHK(hipMemcpyAsync(&hp, w.pred, sizeof(MlpPred), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->pred_last.d0 = hp.d0;
        ctx->pred_last.y0 = hp.y0;
        ctx->pred_last.y1 = hp.y1;
        ctx->pred_last.used = 1;
        pred_end = std::min<int64_t>(hp.d0, g.nn);
      }
      continue;
    }
    if (ctx->o.blocks_per_sync <= 0) per_sync = std::min(per_sync * 2, 4);
  }
  int64_t r = 0;
  int nb = 0;
  if (g.nn > 0) {
    nb = (int)std::min<int64_t>(ctx->host_state->stop_block, g.nblk - 1) + 1;
    r = ctx->host_state->rank;           // set by the stop test of the last block
    *norm_a = std::sqrt(ctx->host_state->normsq);
    // the warm start did not contain the stop: the plain loop went on past d0
    if (ctx->pred_last.used && r >= pred_end && pred_end < g.nn) ctx->pred_last.used = 2;
  } else {
    *norm_a = 0.0;
  }
  *rank = r;
  *blocks = nb;
  return 0;
}

// QR of M^T on one workgroup (f <= 128): M = R2 R1, or M = R2 when R1 is null
// (both column-major f x f FP64).  Q_hat -> Qout (FP64, column-major),
// R_hat -> Dout (type T, row-major ldd); floored pivots counted in st.
// Above 64 the matrices stay in global memory (scr: 7 x 128 x 128 doubles;
// no gated form).
template <typename T>
int small_qr(eodabe_ctx* ctx, hipStream_t st, const double* R1, const double* R2, int f, double* Qout, T* Dout,
             int64_t ldd, State* state, Gate gate = Gate{}, const int64_t* f_dev = nullptr,
             double* scr = nullptr, int32_t* dead_scr = nullptr, double* dg_scr = nullptr,
             uint64_t* mask_scr = nullptr) {
  if (f <= 0) return 0;
  if (f > 64 && f <= 128 && scr && dead_scr && dg_scr && mask_scr && !gate.st && !f_dev) {
    // 64 < f <= 128: the steps of the one-workgroup closing QR as separate
    // launches, so each product runs on (f/32)^2 workgroups: M = R2 R1,
    // G = M M^T, chol -> H1, Z1 = M^T H1^{-1}, G = Z1^T Z1, chol -> H2,
    // Q_hat = Z1 H2^{-1}, R_hat = H2 H1 (all column-major, ld f; the first
    // Cholesky floors, the second kills what stays non-positive; both
    // panel-blocked, cb_chol)
    constexpr int64_t B2 = 128 * 128;
    double* M = scr;
    double* G = scr + B2;
    double* H1 = scr + 2 * B2;
    double* H1i = scr + 3 * B2;
    double* Z1 = scr + 4 * B2;
    double* H2 = scr + 5 * B2;
    double* H2i = scr + 6 * B2;
    const dim3 grid((unsigned)cdiv(f, 32), (unsigned)cdiv(f, 32));
    const double* Mr = R2;
    if (R1) {
      hipLaunchKernelGGL((k_sq_prod<double, true, true, false>), grid, dim3(256), 0, st, R2, R1, f, M, (int64_t)f);
      Mr = M;
    }
    hipLaunchKernelGGL((k_sq_prod<double, true, false, false>), grid, dim3(256), 0, st, Mr, Mr, f, G, (int64_t)f);
    cb_chol(st, G, f, H1, H1i, dg_scr, dead_scr, mask_scr, 1, 1, state, 1);
    hipLaunchKernelGGL((k_sq_prod<double, false, true, false>), grid, dim3(256), 0, st, Mr, H1i, f, Z1, (int64_t)f);
    hipLaunchKernelGGL((k_sq_prod<double, false, true, false>), grid, dim3(256), 0, st, Z1, Z1, f, G, (int64_t)f);
    cb_chol(st, G, f, H2, H2i, dg_scr, dead_scr, mask_scr, 0, 0, state, 1);
    hipLaunchKernelGGL((k_sq_prod<double, true, true, false>), grid, dim3(256), 0, st, Z1, H2i, f, Qout, (int64_t)f);
    hipLaunchKernelGGL((k_sq_prod<T, true, true, true>), grid, dim3(256), 0, st, H2, H1, f, Dout, ldd);
    LAUNCHCHK();
    return 0;
  }
  if (f <= 16)
    hipLaunchKernelGGL((k_small_qr<T, 16>), dim3(1), dim3(256), 0, st, R1, R2, f, Qout, Dout, ldd, state, 1,
                       gate, f_dev);
  else if (f <= 32)
    hipLaunchKernelGGL((k_small_qr<T, 32>), dim3(1), dim3(256), 0, st, R1, R2, f, Qout, Dout, ldd, state, 1,
                       gate, f_dev);
  else if (f <= 64)
    hipLaunchKernelGGL((k_small_qr<T, 64>), dim3(1), dim3(256), 0, st, R1, R2, f, Qout, Dout, ldd, state, 1,
                       gate, f_dev);
  else if (f <= 128 && scr && !gate.st && !f_dev)
    hipLaunchKernelGGL((k_small_qr128<T>), dim3(1), dim3(256), 0, st, R1, R2, f, Qout, Dout, ldd, state, 1,
                       scr);
  else
    return EODABE_EINVAL;
  LAUNCHCHK();
  return 0;
}

// K-splits of the r x nn products over mm rows: about 1024 waves, bounded
// by the partial buffer (planned for r_cap) and by 256 rows per split.
int core_splits(const Geo& g, int64_t r) {
  const int64_t tiles = cdiv(g.nn, 256) * cdiv(r, 16 * std::min<int64_t>(4, cdiv(r, 16)));
  int64_t sc = std::max<int64_t>(1, cdiv(r > 64 ? 512 : 256, tiles));   // more waves when MFMA-bound
  sc = std::min<int64_t>(sc, std::max<int64_t>(1, g.mm / 256));
  sc = std::min<int64_t>(sc, std::max<int64_t>(1, ((int64_t)g.s_core * std::max<int64_t>(g.r_cap, 1)) / r));
  return (int)std::min<int64_t>(sc, 1024);
}

// a9-a11 of Alg. 2 for a rank of at most 128: C = Q^T A; C^T = V R by
// CholeskyQR2 (R = R2 R1 in rb2, rb1; V = (C^T R1^{-1}) R2^{-1}); R^T =
// Q_hat R_hat on one workgroup (Q_hat -> rb4, D_hat = R_hat -> Dout); V and
// U_hat = Q Q_hat in one launch.  r bounds the rank (template widths and
// partial layouts); with r_dev (ranks <= 64 only) the exact rank is read on
// the device and gate holds every kernel until the basis loop has stopped
// (closing steps enqueued before the host has seen the stop flag).
// prof_block tags the timed projection (SPEC_BLOCK for gated launches).
template <typename T>
int close_small(eodabe_ctx* ctx, hipStream_t st, const Geo& g, const WS& w, const T* Ae, int64_t r,
                Gate gate, const int64_t* r_dev, T* Uout, int64_t ldu, T* Vout, int64_t ldv, T* Dout,
                int64_t ldd, int prof_block, bool* state_sent = nullptr) {
  if (r <= 0 || r > 128 || (r > 64 && (gate.st || r_dev))) return EODABE_EINVAL;
  Ops<T> ops{ctx, st};
  T* q = (T*)w.q;
  T* cb = (T*)w.cbuf;
  const int64_t cstride = r * g.ldk;
  const int s_core = core_splits(g, r);
  // a9: C = Q^T A (r x nn, row-major ld ldk)
  const int pid = prof_begin(ctx, st);
  prof_attach(ctx, ops, pid);
  TRY(ops.gemm_nn(q, g.ldy, Ae, g.lda_eff, r, g.nn, g.mm, s_core, (T*)w.cpart, g.ldk, cstride, gate,
                  r_dev));
  prof_attach(ctx, ops, -1);
  // algorithmic bytes: A once, Q (mm x r) and C (r x nn) once
  if (r_dev)
    prof_end(ctx, st, pid, EODABE_PROF_PROJECT, prof_block, (double)g.elem * g.mm * g.nn,
             (double)g.elem * (g.mm + g.nn));
  else
    prof_end(ctx, st, pid, EODABE_PROF_PROJECT, prof_block,
             (double)g.elem * ((double)g.mm * g.nn + (double)g.mm * r + (double)r * g.nn));
  TRY(ops.reduce_wide((const T*)w.cpart, eff_splits(g.mm, s_core), cstride, cstride, cb, nullptr, 0,
                      gate));
  if (!gate.st) TRY(pair_fix<T>(ctx, st, g.paired, cb, g.ldk, g.nn, r));
  if (cqr2_fits(g.nn, r)) {
    // C^T = V R by CholeskyQR2 in one launch, V written straight to Vout
    Cqr2Args a{};
    a.X = cb;
    a.ldx = g.ldk;
    a.rows = g.nn;
    a.f = (int)r;
    a.f_dev = r_dev;
    a.parts = w.gbig;
    a.counter = &w.st->counter[2];
    a.gate = gate;
    a.st = w.st;
    a.R1 = w.rb1;
    a.R1inv = w.rb3;
    a.R2 = w.rb2;
    a.R2inv = w.rb5;
    a.dead = w.deadbig;
    a.fresh = 1;
    a.count_floors = 1;
    a.Q = Vout;
    a.ldq = ldv;
    // and the QR of R^T on every workgroup, U = Q Qh too when the rows of U
    // split into at most 1024 per workgroup
    a.close_qr = 1;
    a.Dout = Dout;
    a.ldd = ldd;
    a.Qh_out = w.rb4;
    const bool u_in = cdiv(g.mm, cdiv(g.nn, CQR2_RPW)) <= 1024;
    if (u_in) {
      a.Uq = q;
      a.ldq_u = g.ldy;
      a.Uout = Uout;
      a.ldu = ldu;
      a.m_u = g.mm;
    }
    // the control block to host memory from the same kernel, once final (no
    // later launch of the chunk changes it): the host needs no copy
    if (state_sent && ctx->host_state_dev) {
      a.state_out = ctx->host_state_dev;
      *state_sent = true;
    }
    TRY(cqr2<T>(ctx, st, a));
    if (!u_in) {
      const ApplyJob ju{q, g.ldy, Uout, ldu, w.rb4, g.mm, 0, (int)r, (int)r, nullptr, nullptr, r_dev};
      TRY(ops.apply(ju, nullptr, (int)r, nullptr, 0, gate));
    }
    return 0;
  }
  CholArgs c1 = chol_args(w, w.rb1, w.deadbig, 1, 1, 1);
  c1.Rinv = w.rb3;
  c1.gate = gate;
  c1.f_dev = r_dev;
  TRY(gram_chol<T>(ctx, st, w, cb, g.ldk, g.nn, (int)r, w.gbig, c1));
  CholArgs c2 = chol_args(w, w.rb2, w.deadbig, 0, 0, 1);
  c2.Rinv = w.rb5;
  c2.gate = gate;
  c2.f_dev = r_dev;
  if (r <= 64) {
    TRY(gram_chol<T>(ctx, st, w, cb, g.ldk, g.nn, (int)r, w.gbig, c2, nullptr, 0, w.rb3));
  } else {
    const ApplyJob a1{cb, g.ldk, cb, g.ldk, w.rb3, g.nn, 0, (int)r, (int)r, nullptr, nullptr, nullptr};
    TRY(ops.apply(a1, nullptr, (int)r));
    TRY(gram_chol<T>(ctx, st, w, cb, g.ldk, g.nn, (int)r, w.gbig, c2));
  }
  TRY(small_qr<T>(ctx, st, w.rb1, w.rb2, (int)r, w.rb4, Dout, ldd, w.st, gate, r_dev, w.sq128, w.deadbig, w.dg,
                  w.cbmask));
  const ApplyJob jv{cb, g.ldk, Vout, ldv, w.rb5, g.nn, 0, (int)r, (int)r, nullptr, nullptr, r_dev};
  const ApplyJob ju{q, g.ldy, Uout, ldu, w.rb4, g.mm, 0, (int)r, (int)r, nullptr, nullptr, r_dev};
  TRY(ops.apply(jv, &ju, (int)r, nullptr, 0, gate));
  return 0;
}

// Alg. 2 after Alg. 1: power iteration, C = Q^T A, QR(C^T), QR(R^T).
// Writes U_hat (column-major mm x r, ld ldu) to Uout, V_hat^T (r x nn,
// row-major ldv) to Vout and D_hat (r x r row-major, ldd) to Dout.
// lp_refine: the low-precision form read its copy of A, so it runs one
// subspace iteration on top of opts.power_iters, and every iteration takes
// its first product A^T Q from the copy (the second, A Q~, and the
// projection C = Q^T A stay in the data type).
template <typename T>
int run_close(eodabe_ctx* ctx, hipStream_t st, const Geo& g, const WS& w, const T* Ae, int64_t r,
              T* Uout, int64_t ldu, T* Vout, int64_t ldv, T* Dout, int64_t ldd, bool lp_refine) {
  if (r <= 0) return 0;
  Ops<T> ops{ctx, st};
  T* q = (T*)w.q;
  T* cb = (T*)w.cbuf;
  const int64_t cstride = r * g.ldk;
  const int s_core = core_splits(g, r);
  const int iters = ctx->o.power_iters + (lp_refine ? 1 : 0);
  for (int it = 0; it < iters; ++it) {
    // Y~^T = Q^T A (r x nn), QR(Y~) -> Q~ (stored as Q~^T = cbuf rows)
    if constexpr (sizeof(T) == 4) {
      if (lp_refine)
        TRY(ops.gemm_nn_lp(g.lp, (const float*)q, g.ldy, w.alp, g.ld_lp, r, g.nn, g.mm, s_core, (float*)w.cpart,
                           g.ldk, cstride, w.st));
      else
        TRY(ops.gemm_nn(q, g.ldy, Ae, g.lda_eff, r, g.nn, g.mm, s_core, (T*)w.cpart, g.ldk, cstride));
    } else {
      TRY(ops.gemm_nn(q, g.ldy, Ae, g.lda_eff, r, g.nn, g.mm, s_core, (T*)w.cpart, g.ldk, cstride));
    }
    TRY(ops.reduce_wide((const T*)w.cpart, eff_splits(g.mm, s_core), cstride, cstride, cb));
    TRY(pair_fix<T>(ctx, st, g.paired, cb, g.ldk, g.nn, r));
    TRY(cholqr2<T>(ctx, st, g, w, cb, g.ldk, g.nn, (int)r, w.rb4, 0, (T*)w.tbig));
    // Y = A Q~ (mm x r), QR(Y) -> Q
    TRY(ops.template gemm_nt<T>(Ae, g.lda_eff, cb, g.ldk, g.mm, r, g.nn, 1, q, g.ldy, g.ldy * r));
    TRY(pair_fix<T>(ctx, st, g.paired, q, g.ldy, g.mm, r));
    TRY(cholqr2<T>(ctx, st, g, w, q, g.ldy, g.mm, (int)r, w.rb4, 0, (T*)w.tbig));
  }
  if (r <= 128)
    return close_small<T>(ctx, st, g, w, Ae, r, Gate{}, nullptr, Uout, ldu, Vout, ldv, Dout, ldd, 0);
  // a9: C = Q^T A (r x nn, row-major ld ldk)
  const int pid = prof_begin(ctx, st);
  prof_attach(ctx, ops, pid);
  TRY(ops.gemm_nn(q, g.ldy, Ae, g.lda_eff, r, g.nn, g.mm, s_core, (T*)w.cpart, g.ldk, cstride));
  prof_attach(ctx, ops, -1);
  prof_end(ctx, st, pid, EODABE_PROF_PROJECT, 0,
           (double)g.elem * ((double)g.mm * g.nn + (double)g.mm * r + (double)r * g.nn));
  TRY(ops.reduce_wide((const T*)w.cpart, eff_splits(g.mm, s_core), cstride, cstride, cb));
  TRY(pair_fix<T>(ctx, st, g.paired, cb, g.ldk, g.nn, r));
  // a10: C^T = V R  (C^T is nn x r with element (j,a) at a*ldk + j = cbuf);
  //      V^T rows go straight to Vout, R^T (row-major R) to rb4 as a
  //      column-major r x r matrix.
  TRY(cholqr2<T>(ctx, st, g, w, cb, g.ldk, g.nn, (int)r, w.rb4, 1, (T*)w.tbig, Vout, ldv));
  // R^T = Q_hat R_hat (FP64, r x r, column-major in rb4); D_hat = R_hat -> Dout
  TRY(cholqr2<double>(ctx, st, g, w, w.rb4, r, r, (int)r, w.rb3, 0, (double*)w.tbig, nullptr, 0,
                      nullptr, 0));
  {
    dim3 grid((unsigned)cdiv(r, 32), (unsigned)cdiv(r, 32));
    hipLaunchKernelGGL((k_copy2d<double, T>), grid, dim3(32, 8), 0, st, w.rb3, r, Dout, ldd, r, r, 1);
    LAUNCHCHK();
  }
  // U_hat = Q Q_hat : (mm x r) (r x r); Q_hat FP64 column-major in rb4.
  TRY(ops.update_d(Uout, ldu, q, g.ldy, g.mm, r, (int)r, w.rb4, r));
  return 0;
}

int check_ctx(const eodabe_ctx* ctx) { return ctx ? 0 : EODABE_EINVAL; }

int check_dev(const eodabe_ctx* ctx) { return ctx->host_only ? EODABE_ENODEVICE : 0; }

}  // namespace

namespace {
struct SketchPlan {
  int64_t bn, ldk, ldyp, s;
};
SketchPlan sketch_plan(int64_t m, int64_t n, int64_t ncols) {
  SketchPlan p;
  p.bn = rup(std::max<int64_t>(ncols, 1), 16);
  p.ldk = rup(std::max<int64_t>(n, 1), 4);
  p.ldyp = rup(std::max<int64_t>(m, 1), 4);
  const int64_t mt = std::max<int64_t>(cdiv(m, 128), 1);
  int64_t s = std::min<int64_t>(cdiv(512, mt), std::max<int64_t>(n / 256, 1));
  p.s = std::max<int64_t>(1, std::min<int64_t>(s, 64));
  return p;
}
struct SketchLp {
  State* st;
  double* normp;
  float* maxp;
  uint16_t* alp;
  int64_t ld_lp;
};
template <typename T>
size_t sketch_carve(void* base, int64_t m, int64_t n, const SketchPlan& p, T** om, T** yp, T** ap,
                    T** yr, SketchLp* lp) {
  Carver c(base);
  *om = c.take<T>(p.bn * rup(p.ldk, 16));
  *yp = c.take<T>(p.s * p.ldyp * p.bn);
  *ap = c.take<T>(m * p.ldk);
  *yr = c.take<T>(p.ldyp * p.bn);
  const int64_t nparts = p.s * std::max<int64_t>(cdiv(m, 128), 1) + 64;
  lp->ld_lp = rup(std::max<int64_t>(n, 1), 8);
  lp->st = c.take<State>(1);
  lp->normp = c.take<double>(nparts);
  lp->maxp = c.take<float>(nparts);
  lp->alp = c.take<uint16_t>(m * lp->ld_lp);
  return c.off + 256;
}
}  // namespace

// ---------------------------------------------------------------------------
// Batched tiles
// ---------------------------------------------------------------------------
namespace {
int tile_bucket(int64_t side) { return side <= 128 ? 0 : (side <= 256 ? 1 : (side <= 512 ? 2 : 3)); }
int tile_slots(const eodabe_ctx* ctx) { return ctx->host_only ? 256 : std::max(ctx->cu_count, 1); }

struct BatchWS {
  TileDesc* descs;
  TileResult* res;
  uint32_t* queue;
  char* slots;
  void* fws;            // workspace of the regular path (tiles above the in-kernel rank cap)
  size_t fws_bytes;
  size_t total;
};
BatchWS batch_carve(void* base, eodabe_ctx* ctx, int ntiles) {
  Carver c(base);
  BatchWS b{};
  b.descs = c.take<TileDesc>(std::max(ntiles, 1));
  b.res = c.take<TileResult>(std::max(ntiles, 1));
  b.queue = c.take<uint32_t>(64);
  b.slots = c.take<char>((int64_t)tile_slots(ctx) * TileSlot::BYTES);
  eodabe_opts o = ctx->o;
  o.a_dtype = EODABE_F32;
  eodabe_ctx tmp{};
  tmp.o = o;
  tmp.host_only = true;
  b.fws_bytes = 0;                      // any tile block width (tile_block: 1 .. TILE_BMAX)
  for (int bw = 1; bw <= TILE_BMAX; ++bw) {
    tmp.o.block = bw;
    b.fws_bytes = std::max(b.fws_bytes, eodabe_workspace_size(&tmp, TILE_MAX, TILE_MAX, TILE_MAX));
  }
  b.fws = c.take<char>((int64_t)b.fws_bytes);
  b.total = c.off + 256;
  return b;
}

int tile_block(const eodabe_ctx* ctx, int64_t h, int64_t w) {
  const int t = ctx->tile_b[tile_bucket(std::max(h, w))];
  const int b = t > 0 ? t : ctx->o.block;
  return std::max(1, std::min(b, TILE_BMAX));
}

// Enqueue the batch on the private stream (descriptor copy, queue reset,
// persistent kernel, result copy), captured once into a hipGraph per key and
// replayed afterwards; the host copies read the pinned staging buffer when
// they execute, so new descriptors need no new capture.
int batch_launch(eodabe_ctx* ctx, const BatchWS& b, int ntiles, int grid, float* pool, double tol,
                 void* ws) {
  hipStream_t st = ctx->tile_stream;
  TileDesc* hd = (TileDesc*)ctx->tile_host;
  TileResult* hr = (TileResult*)((char*)ctx->tile_host + (size_t)ntiles * sizeof(TileDesc));
  const uint32_t k0 = (uint32_t)(ctx->o.seed & 0xffffffffu), k1 = (uint32_t)(ctx->o.seed >> 32);
  auto enqueue = [&]() -> int {
    HIPCHK(hipMemcpyAsync(b.descs, hd, (size_t)ntiles * sizeof(TileDesc), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_zero<uint32_t>, dim3(1), dim3(64), 0, st, b.queue, (int64_t)64);
    hipLaunchKernelGGL(k_tiles, dim3(grid), dim3(256), 0, st, b.descs, ntiles, b.queue, b.slots, pool,
                       b.res, tol, k0, k1);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(hr, b.res, (size_t)ntiles * sizeof(TileResult), hipMemcpyDeviceToHost, st));
    return 0;
  };
  if (!ctx->tile_graphs) {
    TRY(enqueue());
    return 0;
  }
  const bool same = ctx->tile_exec && ctx->tile_key.ws == ws && ctx->tile_key.pool == pool &&
                    ctx->tile_key.ntiles == ntiles && ctx->tile_key.grid == grid &&
                    ctx->tile_key.tol == tol && ctx->tile_key.seed == ctx->o.seed;
  if (!same) {
    if (ctx->tile_exec) (void)hipGraphExecDestroy(ctx->tile_exec);
    if (ctx->tile_graph) (void)hipGraphDestroy(ctx->tile_graph);
    ctx->tile_exec = nullptr;
    ctx->tile_graph = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int e = enqueue();
    hipGraph_t gph = nullptr;
    const hipError_t ce = hipStreamEndCapture(st, &gph);
    TRY(e);
    HIPCHK(ce);
    ctx->tile_graph = gph;
    HIPCHK(hipGraphInstantiate(&ctx->tile_exec, gph, nullptr, nullptr, 0));
    ctx->tile_key.ws = ws;
    ctx->tile_key.pool = pool;
    ctx->tile_key.ntiles = ntiles;
    ctx->tile_key.grid = grid;
    ctx->tile_key.tol = tol;
    ctx->tile_key.seed = ctx->o.seed;
  }
  HIPCHK(hipGraphLaunch(ctx->tile_exec, st));
  return 0;
}
}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

size_t eodabe_batched_workspace_size(eodabe_ctx* ctx, int ntiles) {
  if (!ctx || ntiles < 0) return 0;
  return batch_carve(nullptr, ctx, ntiles).total;
}

int eodabe_factor_batched(eodabe_ctx* ctx, int ntiles, const void* const* A, const int64_t* m,
                          const int64_t* n, const int64_t* lda, double tol, void* ws, size_t ws_bytes,
                          void* out_pool, int64_t pool_len, const int64_t* out_offsets,
                          const int64_t* r_caps, int64_t* ranks, int32_t* status, int32_t* blocks_used) {
  TRY(check_ctx(ctx));
  if (ntiles < 0 || (ntiles > 0 && (!A || !m || !n || !lda || !out_offsets || !r_caps || !ranks || !status)))
    return EODABE_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return EODABE_EINVAL;
  if (ctx->o.a_dtype != EODABE_F32) return EODABE_EINVAL;
  for (int t = 0; t < ntiles; ++t) {
    if (m[t] < 1 || n[t] < 1 || m[t] > TILE_MAX || n[t] > TILE_MAX || lda[t] < n[t] || !A[t]) return EODABE_EINVAL;
    if (r_caps[t] < 0 || r_caps[t] > std::min(m[t], n[t]) || out_offsets[t] < 0) return EODABE_EINVAL;
    const int64_t rc = r_caps[t] ? r_caps[t] : std::min(m[t], n[t]);
    if (out_offsets[t] > pool_len || rc * (m[t] + rc + n[t]) > pool_len - out_offsets[t]) return EODABE_EINVAL;
  }
  if (ntiles == 0) return EODABE_OK;
  const BatchWS b = batch_carve(ws, ctx, ntiles);
  if (!ws || ws_bytes < b.total || !out_pool) return EODABE_EWORKSPACE;
  TRY(check_dev(ctx));
  if (!ctx->tile_stream) {
    HIPCHK(hipStreamCreateWithFlags(&ctx->tile_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->tile_ev, hipEventDisableTiming));
  }
  const size_t hbytes = (size_t)ntiles * (sizeof(TileDesc) + sizeof(TileResult));
  if (ctx->tile_host_bytes < hbytes) {
    if (ctx->tile_host) HIPCHK(hipHostFree(ctx->tile_host));
    ctx->tile_host = nullptr;
    ctx->tile_host_bytes = 0;
    HIPCHK(hipHostMalloc(&ctx->tile_host, hbytes, hipHostMallocDefault));
    ctx->tile_host_bytes = hbytes;
    if (ctx->tile_exec) (void)hipGraphExecDestroy(ctx->tile_exec);   // staging moved
    ctx->tile_exec = nullptr;
  }
  // largest tiles first (longest-processing-time order over the workgroups)
  std::vector<int> order(ntiles);
  for (int t = 0; t < ntiles; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return m[a] * n[a] > m[c] * n[c]; });
  TileDesc* hd = (TileDesc*)ctx->tile_host;
  for (int i = 0; i < ntiles; ++i) {
    const int t = order[i];
    TileDesc d{};
    d.A = (const float*)A[t];
    d.h = m[t];
    d.w = n[t];
    d.lda = lda[t];
    d.out_off = out_offsets[t];
    d.r_cap = r_caps[t] ? r_caps[t] : std::min(m[t], n[t]);
    d.b = tile_block(ctx, m[t], n[t]);
    d.index = t;
    hd[i] = d;
  }
  // inputs are produced on the caller's stream
  HIPCHK(hipEventRecord(ctx->tile_ev, ctx->stream));
  HIPCHK(hipStreamWaitEvent(ctx->tile_stream, ctx->tile_ev, 0));
  const int grid = std::min(ntiles, tile_slots(ctx));
  hipEvent_t pa = ctx->prof_on ? prof_event(ctx) : nullptr, pb = ctx->prof_on ? prof_event(ctx) : nullptr;
  if (pa && pb) HIPCHK(hipEventRecord(pa, ctx->tile_stream));
  TRY(batch_launch(ctx, b, ntiles, grid, (float*)out_pool, tol, ws));
  if (pa && pb) HIPCHK(hipEventRecord(pb, ctx->tile_stream));
  HIPCHK(hipStreamSynchronize(ctx->tile_stream));
  const TileResult* hr = (const TileResult*)((char*)ctx->tile_host + (size_t)ntiles * sizeof(TileDesc));
  int first_err = EODABE_OK;
  double bytes = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    ranks[t] = hr[t].rank;
    status[t] = hr[t].status;
    if (blocks_used) blocks_used[t] = tile_block(ctx, m[t], n[t]);
    const double hw = 4.0 * (double)m[t] * (double)n[t], r = (double)hr[t].rank;
    bytes += status[t] == TS_OK ? hw * (hr[t].blocks + 1) + 4.0 * r * (double)(m[t] + n[t] + hr[t].rank)
                                : hw * hr[t].blocks;
  }
  if (pa && pb) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pa, pb) == hipSuccess) {
      ctx->prof_ms[EODABE_PROF_TILES] += ms;
      ctx->prof_n[EODABE_PROF_TILES] += 1;
      ctx->prof_bytes[EODABE_PROF_TILES] += bytes;
    }
  }
  if (pa) ctx->ev_pool.push_back(pa);
  if (pb) ctx->ev_pool.push_back(pb);
  // tiles whose rank went above the in-kernel cap: the regular path
  eodabe_ctx* sub = nullptr;
  for (int t = 0; t < ntiles; ++t) {
    if (status[t] != TS_RANK) continue;
    if (!sub) {
      eodabe_opts o = ctx->o;
      o.stream = ctx->stream;
      TRY(eodabe_create(&sub, &o));
    }
    sub->o.block = tile_block(ctx, m[t], n[t]);
    const int64_t rc = r_caps[t] ? r_caps[t] : std::min(m[t], n[t]);
    float* Ut = (float*)out_pool + out_offsets[t];
    float* core = Ut + rc * m[t];
    float* Vt = core + rc * rc;
    eodabe_info info{};
    const int e = eodabe_factor(sub, A[t], m[t], n[t], lda[t], tol, b.fws, b.fws_bytes, Ut, core, Vt, rc,
                                &info);
    ranks[t] = info.rank;
    status[t] = e == EODABE_ECAPACITY ? TS_CAPACITY : (e == EODABE_ENONFINITE ? TS_NONFINITE : (e < 0 ? -1 : TS_OK));
    if (e < 0 && e != EODABE_ECAPACITY && e != EODABE_ENONFINITE && first_err == EODABE_OK) first_err = e;
  }
  if (sub) eodabe_destroy(sub);
  return first_err;
}

// Pick the block width per tile-size bucket (sides <= 128, 256, 512, 1024)
// among {16, 32, 64} by timing the whole batch, one bucket at a time; the
// choice is kept in the context for later eodabe_factor_batched calls.
int eodabe_tune_batched(eodabe_ctx* ctx, int ntiles, const void* const* A, const int64_t* m,
                        const int64_t* n, const int64_t* lda, double tol, void* ws, size_t ws_bytes,
                        void* out_pool, int64_t pool_len, const int64_t* out_offsets, const int64_t* r_caps,
                        int32_t* chosen) {
  TRY(check_ctx(ctx));
  TRY(check_dev(ctx));
  if (ntiles <= 0) return EODABE_EINVAL;
  std::vector<int64_t> rk(ntiles);
  std::vector<int32_t> stt(ntiles);
  const int cand[3] = {16, 32, 64};
  for (int k = 0; k < 4; ++k) {
    bool present = false;
    for (int t = 0; t < ntiles; ++t) present = present || tile_bucket(std::max(m[t], n[t])) == k;
    if (!present) continue;
    double best = 1e300;
    int bestb = ctx->tile_b[k];
    for (int c : cand) {
      ctx->tile_b[k] = c;
      double tot = 0.0;
      for (int rep = 0; rep < 2; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        TRY(eodabe_factor_batched(ctx, ntiles, A, m, n, lda, tol, ws, ws_bytes, out_pool, pool_len, out_offsets,
                                  r_caps, rk.data(), stt.data(), nullptr));
        const auto t1 = std::chrono::steady_clock::now();
        if (rep) tot += std::chrono::duration<double>(t1 - t0).count();
      }
      if (tot < best) {
        best = tot;
        bestb = c;
      }
    }
    ctx->tile_b[k] = bestb;
  }
  if (chosen)
    for (int k = 0; k < 4; ++k) chosen[k] = ctx->tile_b[k];
  return EODABE_OK;
}


// ---- learned predictor: training and inference kernels --------------------
}  // extern "C"
namespace {
struct MlpWS {
  float *z1, *h1, *z2, *h2, *z3, *h3, *y, *dy, *g1, *g2;
  double* loss;
  size_t total;
};
MlpWS mlp_carve(void* base, int B) {
  Carver c(base);
  MlpWS w{};
  const int64_t bh = (int64_t)std::max(B, 1) * MLP_H;
  w.z1 = c.take<float>(bh);
  w.h1 = c.take<float>(bh);
  w.z2 = c.take<float>(bh);
  w.h2 = c.take<float>(bh);
  w.z3 = c.take<float>(bh);
  w.h3 = c.take<float>(bh);
  w.y = c.take<float>(2 * (int64_t)std::max(B, 1));
  w.dy = c.take<float>(2 * (int64_t)std::max(B, 1));
  w.g1 = c.take<float>(bh);
  w.g2 = c.take<float>(bh);
  w.loss = c.take<double>(1);
  w.total = c.off + 256;
  return w;
}
template <bool TA, bool TB>
int mlp_gemm(eodabe_ctx* ctx, hipStream_t st, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
             int M, int N, int K, const float* bias) {
  dim3 grid((unsigned)cdiv(N, 64), (unsigned)cdiv(M, 64));
  hipLaunchKernelGGL((k_mlp_gemm<TA, TB>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, bias);
  LAUNCHCHK();
  return 0;
}
int mlp_act(eodabe_ctx* ctx, hipStream_t st, const float* Z, float* H, int64_t cnt) {
  hipLaunchKernelGGL(k_gelu_fwd, dim3((unsigned)std::min<int64_t>(cdiv(cnt, 256), 2048)), dim3(256), 0, st, Z, H,
                     cnt);
  LAUNCHCHK();
  return 0;
}
int mlp_act_grad(eodabe_ctx* ctx, hipStream_t st, float* G, const float* Z, int64_t cnt) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3((unsigned)std::min<int64_t>(cdiv(cnt, 256), 2048)), dim3(256), 0, st, G, Z, G,
                     cnt);
  LAUNCHCHK();
  return 0;
}
int mlp_forward_impl(eodabe_ctx* ctx, hipStream_t st, const float* P, const float* X, int B, const MlpWS& w) {
  TRY((mlp_gemm<false, true>(ctx, st, X, MLP_IN, P + MLP_W1, MLP_IN, w.z1, MLP_H, B, MLP_H, MLP_IN, P + MLP_B1)));
  TRY(mlp_act(ctx, st, w.z1, w.h1, (int64_t)B * MLP_H));
  TRY((mlp_gemm<false, true>(ctx, st, w.h1, MLP_H, P + MLP_W2, MLP_H, w.z2, MLP_H, B, MLP_H, MLP_H, P + MLP_B2)));
  TRY(mlp_act(ctx, st, w.z2, w.h2, (int64_t)B * MLP_H));
  TRY((mlp_gemm<false, true>(ctx, st, w.h2, MLP_H, P + MLP_W3, MLP_H, w.z3, MLP_H, B, MLP_H, MLP_H, P + MLP_B3)));
  TRY(mlp_act(ctx, st, w.z3, w.h3, (int64_t)B * MLP_H));
  TRY((mlp_gemm<false, true>(ctx, st, w.h3, MLP_H, P + MLP_W4, MLP_H, w.y, MLP_OUT, B, MLP_OUT, MLP_H,
                             P + MLP_B4)));
  return 0;
}
// dW = dZ^T H_prev, db = column sums of dZ, dH_prev = dZ W (then times GELU'(Z_prev))
int mlp_layer_grad(eodabe_ctx* ctx, hipStream_t st, const float* dZ, int nout, const float* Hprev, int nin, int B,
                   const float* W, float* dW, float* db, float* dHprev) {
  TRY((mlp_gemm<true, false>(ctx, st, dZ, nout, Hprev, nin, dW, nin, nout, nin, B, nullptr)));
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)cdiv(nout, 256)), dim3(256), 0, st, dZ, B, nout, db);
  LAUNCHCHK();
  if (dHprev) TRY((mlp_gemm<false, false>(ctx, st, dZ, nout, W, nin, dHprev, nin, B, nin, nout, nullptr)));
  return 0;
}
int mlp_backward_impl(eodabe_ctx* ctx, hipStream_t st, const float* P, const float* X, const float* T, int B,
                      float* G, const MlpWS& w) {
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, w.y, T, B, w.dy, w.loss);
  LAUNCHCHK();
  const int64_t bh = (int64_t)B * MLP_H;
  TRY(mlp_layer_grad(ctx, st, w.dy, MLP_OUT, w.h3, MLP_H, B, P + MLP_W4, G + MLP_W4, G + MLP_B4, w.g1));
  TRY(mlp_act_grad(ctx, st, w.g1, w.z3, bh));
  TRY(mlp_layer_grad(ctx, st, w.g1, MLP_H, w.h2, MLP_H, B, P + MLP_W3, G + MLP_W3, G + MLP_B3, w.g2));
  TRY(mlp_act_grad(ctx, st, w.g2, w.z2, bh));
  TRY(mlp_layer_grad(ctx, st, w.g2, MLP_H, w.h1, MLP_H, B, P + MLP_W2, G + MLP_W2, G + MLP_B2, w.g1));
  TRY(mlp_act_grad(ctx, st, w.g1, w.z1, bh));
  TRY(mlp_layer_grad(ctx, st, w.g1, MLP_H, X, MLP_IN, B, P + MLP_W1, G + MLP_W1, G + MLP_B1, nullptr));
  return 0;
}
}  // namespace
extern "C" {

int64_t eodabe_mlp_param_count(void) { return MLP_NPARAM; }

size_t eodabe_mlp_workspace_size(int batch) { return batch < 1 ? 0 : mlp_carve(nullptr, batch).total; }

int eodabe_mlp_forward(eodabe_ctx* ctx, const float* params, const float* X, int batch, float* Y, void* ws,
                       size_t ws_bytes) {
  TRY(check_ctx(ctx));
  if (batch < 1 || !params || !X || !Y) return EODABE_EINVAL;
  const MlpWS w = mlp_carve(ws, batch);
  if (!ws || ws_bytes < w.total) return EODABE_EWORKSPACE;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  TRY(mlp_forward_impl(ctx, st, params, X, batch, w));
  HIPCHK(hipMemcpyAsync(Y, w.y, sizeof(float) * 2 * (size_t)batch, hipMemcpyDeviceToDevice, st));
  return 0;
}

int eodabe_mlp_grad(eodabe_ctx* ctx, const float* params, const float* X, const float* T, int batch, float* grads,
                    void* ws, size_t ws_bytes, double* loss) {
  TRY(check_ctx(ctx));
  if (batch < 1 || !params || !X || !T || !grads) return EODABE_EINVAL;
  const MlpWS w = mlp_carve(ws, batch);
  if (!ws || ws_bytes < w.total) return EODABE_EWORKSPACE;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  TRY(mlp_forward_impl(ctx, st, params, X, batch, w));
  TRY(mlp_backward_impl(ctx, st, params, X, T, batch, grads, w));
  if (loss) {
    HIPCHK(hipMemcpyAsync(loss, w.loss, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return 0;
}

int eodabe_mlp_adam(eodabe_ctx* ctx, float* params, const float* grads, float* m, float* v, float lr, int step) {
  TRY(check_ctx(ctx));
  if (!params || !grads || !m || !v || step < 1 || !(lr > 0.0f)) return EODABE_EINVAL;
  TRY(check_dev(ctx));
  const double b1 = 0.9, b2 = 0.999;
  AdamCoef a;
  a.lr = lr;
  a.b1 = (float)b1;
  a.omb1 = (float)(1.0 - b1);
  a.b2 = (float)b2;
  a.omb2 = (float)(1.0 - b2);
  a.c1 = (float)(1.0 - std::pow(b1, (double)step));
  a.c2 = (float)(1.0 - std::pow(b2, (double)step));
  a.eps = 1e-8f;
  hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, ctx->stream, params, grads, m, v, (int64_t)MLP_NPARAM, a);
  LAUNCHCHK();
  return 0;
}

int eodabe_mlp_features(const double* diag, int64_t m, int64_t n, double eps, float* out) {
  if (!diag || !out || m < 1 || n < 1 || !(eps >= 0.0)) return EODABE_EINVAL;
  for (int c = 0; c < MLP_IN; ++c) out[c] = mlp_feature(diag, c, m, n, eps);
  return 0;
}

int eodabe_set_predictor(eodabe_ctx* ctx, const float* params, double margin) {
  TRY(check_ctx(ctx));
  if (!(margin >= 0.0) || margin > 10.0) return EODABE_EINVAL;
  ctx->pred_params = params;
  ctx->pred_margin = margin;
  return 0;
}

int eodabe_last_prediction(const eodabe_ctx* ctx, int64_t* d0, double* log_rank, double* log_rank_q, int* used) {
  TRY(check_ctx(ctx));
  if (d0) *d0 = ctx->pred_last.d0;
  if (log_rank) *log_rank = ctx->pred_last.y0;
  if (log_rank_q) *log_rank_q = ctx->pred_last.y1;
  if (used) *used = ctx->pred_last.used;
  return 0;
}

void eodabe_default_opts(eodabe_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block = 32;
  o->power_iters = 0;
  o->seed = 0;
  o->a_dtype = EODABE_F32;
  o->sketch_dtype = EODABE_SKETCH_NATIVE;
  o->blocks_per_sync = 0;
  o->stream = nullptr;
}

static int validate_opts(const eodabe_opts* opts) {
  if (opts->block < 1 || opts->block > BN_MAX) return EODABE_EINVAL;
  if (opts->power_iters < 0 || opts->power_iters > 16) return EODABE_EINVAL;
  if (opts->a_dtype != EODABE_F32 && opts->a_dtype != EODABE_F64) return EODABE_EINVAL;
  if (opts->sketch_dtype != EODABE_SKETCH_NATIVE && opts->sketch_dtype != EODABE_SKETCH_F16 &&
      opts->sketch_dtype != EODABE_SKETCH_BF16)
    return EODABE_EINVAL;
  // the low-precision sketch rounds FP32 data; FP64 data keeps the native sketch
  if (opts->sketch_dtype != EODABE_SKETCH_NATIVE && opts->a_dtype != EODABE_F32) return EODABE_EINVAL;
  if (opts->blocks_per_sync < 0) return EODABE_EINVAL;
  return EODABE_OK;
}

int eodabe_create_host(eodabe_ctx** out, const eodabe_opts* opts) {
  if (!out || !opts) return EODABE_EINVAL;
  *out = nullptr;
  TRY(validate_opts(opts));
  eodabe_ctx* c = new (std::nothrow) eodabe_ctx();
  if (!c) return EODABE_EINVAL;
  c->o = *opts;
  c->stream = nullptr;
  c->device = -1;
  c->cu_count = 0;
  c->last_hip = 0;
  c->host_state = nullptr;
  c->host_state_dev = nullptr;
  c->host_wlog = nullptr;
  c->host_wlog_cap = 0;
  c->host_only = true;
  *out = c;
  return EODABE_OK;
}

int eodabe_create(eodabe_ctx** out, const eodabe_opts* opts) {
  if (!out || !opts) return EODABE_EINVAL;
  *out = nullptr;
  TRY(validate_opts(opts));
  int dev = 0, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return EODABE_ENODEVICE;
  if (hipGetDevice(&dev) != hipSuccess) return EODABE_ENODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return EODABE_ENODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return EODABE_ENODEVICE;
  eodabe_ctx* c = new (std::nothrow) eodabe_ctx();
  if (!c) return EODABE_EINVAL;
  c->o = *opts;
  c->stream = (hipStream_t)opts->stream;
  c->device = dev;
  c->cu_count = prop.multiProcessorCount;
  c->last_hip = 0;
  if (hipHostMalloc((void**)&c->host_state, sizeof(State), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return EODABE_EHIP;
  }
  // test of the barrier time-out path (EODABE_ESYNC) without a stuck device
  {
    const char* e = std::getenv("EODABE_TEST_BARRIER_FAIL");
    c->barrier_fail = e && e[0] == '1';
  }
  // the fused closing kernel can then write the control block there itself
  if (hipHostGetDevicePointer((void**)&c->host_state_dev, c->host_state, 0) != hipSuccess) {
    (void)hipGetLastError();
    c->host_state_dev = nullptr;
  }
  // device address of this GPU's copy of the no-allocation scratch, looked up
  // once per device with the device current
  if (dev < MAX_DEVICES) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        (void)hipHostFree(c->host_state);
        delete c;
        return EODABE_EHIP;
      }
      scratch_dev[dev] = p;
    }
    c->scratch = scratch_dev[dev];
  }
  c->host_wlog = nullptr;
  c->host_wlog_cap = 0;
  c->host_only = false;
  *out = c;
  return EODABE_OK;
}

int eodabe_profile(eodabe_ctx* ctx, int enable) {
  TRY(check_ctx(ctx));
  ctx->prof_on = enable != 0 && !ctx->host_only;
  for (int k = 0; k < EODABE_PROF_KINDS; ++k) {
    ctx->prof_ms[k] = 0.0;
    ctx->prof_n[k] = 0;
    ctx->prof_bytes[k] = 0.0;
  }
  return EODABE_OK;
}

int eodabe_profile_read(const eodabe_ctx* ctx, int kind, double* total_ms, int64_t* launches,
                        double* bytes) {
  TRY(check_ctx(ctx));
  if (kind < 0 || kind >= EODABE_PROF_KINDS) return EODABE_EINVAL;
  if (total_ms) *total_ms = ctx->prof_ms[kind];
  if (launches) *launches = ctx->prof_n[kind];
  if (bytes) *bytes = ctx->prof_bytes[kind];
  return EODABE_OK;
}

void eodabe_destroy(eodabe_ctx* ctx) {
  if (!ctx) return;
  for (auto& mk : ctx->marks) {
    (void)hipEventDestroy(mk.a);
    (void)hipEventDestroy(mk.b);
  }
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->host_state) (void)hipHostFree(ctx->host_state);
  if (ctx->tile_exec) (void)hipGraphExecDestroy(ctx->tile_exec);
  if (ctx->tile_graph) (void)hipGraphDestroy(ctx->tile_graph);
  if (ctx->tile_ev) (void)hipEventDestroy(ctx->tile_ev);
  if (ctx->tile_stream) (void)hipStreamDestroy(ctx->tile_stream);
  if (ctx->tile_host) (void)hipHostFree(ctx->tile_host);
  delete ctx;
}

const char* eodabe_strerror(int s) {
  switch (s) {
    case EODABE_OK: return "ok";
    case EODABE_EINVAL: return "invalid argument";
    case EODABE_EWORKSPACE: return "workspace missing or too small";
    case EODABE_ECAPACITY: return "rank exceeds r_cap";
    case EODABE_ENONFINITE: return "A holds NaN or Inf";
    case EODABE_EHIP: return "HIP runtime error";
    case EODABE_ENODEVICE: return "no gfx950 device";
    case EODABE_ESCRATCH: return "the problem needs more workspace than the static scratch holds";
    case EODABE_ESYNC: return "a barrier across workgroups timed out (device shared); outputs void";
    case EODABE_WTOL_FLOOR: return "warning: tol below the data-type floor";
    default: return "unknown status";
  }
}

int eodabe_last_hip_error(const eodabe_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

size_t eodabe_workspace_size(const eodabe_ctx* ctx, int64_t m, int64_t n, int64_t r_cap) {
  if (!ctx) return 0;
  Geo g;
  // assume the worst case (packing needed) so the size is valid for any A
  if (!plan(ctx, m, n, 1, (const void*)1, r_cap, g)) return 0;
  g.packed = true;
  g.lda_eff = rup(std::max<int64_t>(g.nn, 1), 4);
  return carve(nullptr, g).total;
}

static int factor_impl(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, double tol,
                       void* ws, size_t ws_bytes, void* Ut, void* core, void* Vt, int64_t r_cap,
                       eodabe_info* info, void* Qbasis, double* diagT, int64_t diag_cap,
                       bool basis_only) {
  TRY(check_ctx(ctx));
  if (!info) return EODABE_EINVAL;
  std::memset(info, 0, sizeof(*info));
  if (m < 0 || n < 0 || lda < n || lda < 1) return EODABE_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return EODABE_EINVAL;
  if ((m > 0 && n > 0) && !A) return EODABE_EINVAL;
  if (!basis_only && (m > 0 && n > 0) && (!Ut || !core || !Vt)) return EODABE_EINVAL;
  if (basis_only && (m > 0 && n > 0) && !Qbasis) return EODABE_EINVAL;
  Geo g;
  if (!plan(ctx, m, n, lda, A, r_cap, g)) return EODABE_EINVAL;
  const size_t need = eodabe_workspace_size(ctx, m, n, r_cap);
  if (!ws || ws_bytes < need) return EODABE_EWORKSPACE;
  if (m == 0 || n == 0) return EODABE_OK;
  TRY(check_dev(ctx));
  WS w = carve(ws, g);
  hipStream_t st = ctx->stream;
  const bool f64 = ctx->o.a_dtype == EODABE_F64;
  int status = EODABE_OK;
  // dtype floor warning: tol < 8 u sqrt(n)
  const double u = f64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
  if (tol < 8.0 * u * std::sqrt((double)std::min(m, n))) {
    status = EODABE_WTOL_FLOOR;
    info->status_flags |= 1;
  }
  if (g.transposed) info->status_flags |= 2;
  // A low-precision sketch column carries rounding noise of about
  // u_lp ||A||_F / sqrt(3) in its component orthogonal to the basis, the
  // quantity the stop test of Alg. 1 compares with tol ||A||_F: below
  // tol = 2 u_lp (u_lp = 2^-11 FP16, 2^-8 BF16) the test could not fire on
  // such sketches, so the blocks sketch in FP32 (the plain path) instead.
  if (g.lp) {
    const double ulp = g.lp == EODABE_SKETCH_F16 ? 0x1p-11 : 0x1p-8;
    if (tol < 2.0 * ulp) {
      g.lp = 0;
      info->status_flags |= 8;
    }
  }
  int64_t rank = 0;
  int blocks = 0;
  double norm_a = 0.0;
  auto body = [&](auto tag) -> int {
    typedef decltype(tag) T;
    const T* Ae = (const T*)A;
    if (g.packed) {
      TRY(copy2d<T>(ctx, st, (const T*)A, lda, (T*)w.apack, g.lda_eff, g.mm, g.nn, g.transposed ? 1 : 0));
      Ae = (const T*)w.apack;
    }
    // With a small enough basis the closing steps are enqueued right behind
    // each chunk of blocks, gated on the device-side stop flag, so a
    // factorization that stops in its first chunk needs one host sync.
    const bool can_spec = !g.transposed && !basis_only && ctx->o.power_iters == 0 && !g.lp && !g.paired;
    auto after_chunk = [&](int64_t jend) -> int {
      if (!can_spec) return 0;
      const int64_t rb = std::min<int64_t>(g.nn, jend * (int64_t)g.b);
      bool sent = false;
      if (rb <= 0 || rb > 64) return 0;
      TRY(close_small<T>(ctx, st, g, w, Ae, rb, Gate{w.st, g.r_cap}, &w.st->rank, (T*)Ut, m, (T*)Vt,
                         n, (T*)core, g.r_cap, SPEC_BLOCK, &sent));
      return sent ? 2 : 1;
    };
    bool spec_ran = false;
    TRY(run_basis<T>(ctx, st, g, w, Ae, tol, &rank, &blocks, &norm_a, after_chunk, &spec_ran));
    info->rank = rank;
    info->blocks = blocks;
    info->norm_a = norm_a;
    info->eps = tol * norm_a;
    // the control block was read after the last chunk: d_stop is final
    info->relres_est = (norm_a > 0.0 && g.nn > 0) ? ctx->host_state->d_stop / norm_a : 0.0;
    if (diagT && diag_cap > 0) {
      const int64_t cnt = std::min<int64_t>(diag_cap, std::min<int64_t>(rank + 1, g.nn));
      HIPCHK(hipMemcpy(diagT, w.diag_log, cnt * sizeof(double), hipMemcpyDeviceToHost));
    }
    if (basis_only) {
      if (rank > g.r_cap) return EODABE_ECAPACITY;
      if (g.transposed) return EODABE_EINVAL;   // basis of A^T: not offered
      TRY(copy2d<T>(ctx, st, (T*)w.q, g.ldy, (T*)Qbasis, g.mm, rank, g.ldy, 0));
      HIPCHK(hipStreamSynchronize(st));
      return 0;
    }
    if (rank > g.r_cap) return EODABE_ECAPACITY;
    if (rank == 0) {
      HIPCHK(hipStreamSynchronize(st));
      return 0;
    }
    if (spec_ran) {                  // closing steps done; the state was read after them
      if (ctx->host_state->floored) info->status_flags |= 4;
      return 0;
    }
    // Low-precision form: a basis built from sketches of the FP16/BF16 copy
    // of A is tilted from the one FP32 sketches give by up to the copy's
    // rounding over the weakest captured singular value.  One more subspace
    // iteration (Alg. 2, power iteration; its A^T Q from the copy, A Q~ in
    // FP32) maps it back through A before the FP32 projection, so the error
    // is won back.
    const bool refine = g.lp && blocks >= 3;
    if (refine) info->status_flags |= 16;
    if (!g.transposed) {
      TRY(run_close<T>(ctx, st, g, w, Ae, rank, (T*)Ut, m, (T*)Vt, n, (T*)core, g.r_cap, refine));
    } else {
      // factor of A^T = U' D' V'^T (U' nn... here mm = n rows): A = V' D'^T U'^T.
      // U' -> ybig (column-major n x r), V'^T -> cbuf (r x m), D' -> rb_tmp
      T* ut = (T*)w.ybig;            // U' column-major (ld = ldy)
      TRY(run_close<T>(ctx, st, g, w, Ae, rank, ut, g.ldy, (T*)w.cbuf, g.ldk, (T*)w.tbig, rank, refine));
      Ops<T> ops{ctx, st};
      if (rank <= 128) {
        // QR(D'^T) = Q'' R'' on one workgroup: D' column-major (FP64) -> rb2;
        // U_out = V' Q'' (one MFMA pass), core = R'', Vt_out = U'^T.
        dim3 gt((unsigned)cdiv(rank, 32), (unsigned)cdiv(rank, 32));
        hipLaunchKernelGGL((k_copy2d<T, double>), gt, dim3(32, 8), 0, st, (const T*)w.tbig, rank, w.rb2,
                           rank, rank, rank, 1);
        LAUNCHCHK();
        TRY(small_qr<T>(ctx, st, nullptr, w.rb2, (int)rank, w.rb4, (T*)core, g.r_cap, w.st, Gate{}, nullptr,
                        w.sq128, w.deadbig, w.dg, w.cbmask));
        const ApplyJob ju{w.cbuf, g.ldk, Ut, m, w.rb4, m, 0, (int)rank, (int)rank, nullptr, nullptr, nullptr};
        TRY(ops.apply(ju, nullptr, (int)rank));
        TRY(copy2d<T>(ctx, st, ut, g.ldy, (T*)Vt, n, rank, n, 0));
      } else {
        // D'^T (r x r): tbig holds D' row-major (ld r) = D'^T column-major.
        const int64_t cnt = rank * rank;
        hipLaunchKernelGGL((k_copy2d<T, double>), dim3((unsigned)cdiv(cnt, 32), 1), dim3(32, 8), 0, st,
                           (const T*)w.tbig, cnt, w.rb4, cnt, (int64_t)1, cnt, 0);
        LAUNCHCHK();
        TRY(cholqr2<double>(ctx, st, g, w, w.rb4, rank, rank, (int)rank, w.rb3, 0, (double*)w.tbig));
        // U_out = V' Q'' : V' column-major m x r is cbuf (element (i,a) at a*ldk + i)
        TRY(ops.update_d((T*)Ut, m, (const T*)w.cbuf, g.ldk, m, rank, (int)rank, w.rb4, rank));
        // Vt_out = U'^T : U' column-major n x r (ld ldy) -> row a = column a
        TRY(copy2d<T>(ctx, st, ut, g.ldy, (T*)Vt, n, rank, n, 0));
        dim3 grid((unsigned)cdiv(rank, 32), (unsigned)cdiv(rank, 32));
        hipLaunchKernelGGL((k_copy2d<double, T>), grid, dim3(32, 8), 0, st, w.rb3, rank, (T*)core, g.r_cap,
                           rank, rank, 1);
        LAUNCHCHK();
      }
    }
    HIPCHK(hipMemcpyAsync(ctx->host_state, w.st, sizeof(State), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->prof_on) prof_collect(ctx, 0x7fffffff, false, rank);
    if (ctx->host_state->sync_fail) return EODABE_ESYNC;
    if (ctx->host_state->floored) info->status_flags |= 4;
    return 0;
  };
  int s = f64 ? body(double{}) : body(float{});
  if (s < 0) return s;
  return status;
}

int eodabe_factor(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, double tol,
                  void* ws, size_t ws_bytes, void* Ut, void* core, void* Vt, int64_t r_cap,
                  eodabe_info* info) {
  return factor_impl(ctx, A, m, n, lda, tol, ws, ws_bytes, Ut, core, Vt, r_cap, info, nullptr,
                     nullptr, 0, false);
}

int eodabe_factor_noalloc(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda,
                          double tol, void* Ut, void* core, void* Vt, int64_t r_cap, eodabe_info* info) {
  TRY(check_ctx(ctx));
  if (!info) return EODABE_EINVAL;
  std::memset(info, 0, sizeof(*info));
  TRY(check_dev(ctx));
  if (!ctx->scratch) return EODABE_ENODEVICE;
  const size_t need = eodabe_workspace_size(ctx, m, n, r_cap);
  if (need == 0) return EODABE_EINVAL;
  if (need > (size_t)EODABE_NOALLOC_SCRATCH_BYTES) return EODABE_ESCRATCH;
  // per-kernel timing would create events; it is suspended for this call
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  const int s = factor_impl(ctx, A, m, n, lda, tol, ctx->scratch, (size_t)EODABE_NOALLOC_SCRATCH_BYTES,
                            Ut, core, Vt, r_cap, info, nullptr, nullptr, 0, false);
  ctx->prof_on = prof;
  return s;
}

// Complex input: the factorization of the realification [[Re A, -Im A],
// [Im A, Re A]] with the test columns in pairs (omega, i omega) and the stop
// test at pair-leading columns, which is the complex algorithm carried out
// in real arithmetic (real Gram-Schmidt over pair-ordered realified columns
// is complex Gram-Schmidt), then unpacked.
namespace {
struct CplxPlan {
  int64_t rc, ld2;
  size_t off_a, off_u, off_d, off_v, off_in, inner, total;
};
bool cplx_plan(eodabe_ctx* ctx, int64_t m, int64_t n, int64_t r_cap, CplxPlan& p) {
  if (m < 0 || n < 0) return false;
  const int64_t mn = std::min(m, n);
  p.rc = r_cap == 0 ? mn : r_cap;
  if (p.rc < 0 || p.rc > mn) return false;
  const size_t e = ctx->o.a_dtype == EODABE_F64 ? 8 : 4;
  p.ld2 = rup(std::max<int64_t>(2 * n, 1), 4);
  ctx->cplx_pairs = true;
  p.inner = (m == 0 || n == 0) ? 256 : eodabe_workspace_size(ctx, 2 * m, 2 * n, 2 * p.rc);
  ctx->cplx_pairs = false;
  if (p.inner == 0) return false;
  Carver c(nullptr);
  const int64_t rc2 = std::max<int64_t>(2 * p.rc, 1);
  c.take<char>(0);
  p.off_a = (size_t)rup((int64_t)c.off, 256);
  c.take<char>((int64_t)(2 * std::max<int64_t>(m, 1) * p.ld2 * e));
  p.off_u = (size_t)rup((int64_t)c.off, 256);
  c.take<char>((int64_t)(rc2 * 2 * std::max<int64_t>(m, 1) * e));
  p.off_d = (size_t)rup((int64_t)c.off, 256);
  c.take<char>((int64_t)(rc2 * rc2 * e));
  p.off_v = (size_t)rup((int64_t)c.off, 256);
  c.take<char>((int64_t)(rc2 * 2 * std::max<int64_t>(n, 1) * e));
  p.off_in = (size_t)rup((int64_t)c.off, 256);
  c.take<char>((int64_t)p.inner);
  p.total = c.off + 256;
  return true;
}
}  // namespace

size_t eodabe_complex_workspace_size(eodabe_ctx* ctx, int64_t m, int64_t n, int64_t r_cap) {
  if (!ctx) return 0;
  CplxPlan p;
  return cplx_plan(ctx, m, n, r_cap, p) ? p.total : 0;
}

int eodabe_factor_complex(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, double tol,
                          void* ws, size_t ws_bytes, void* Ut, void* core, void* Vt, int64_t r_cap,
                          eodabe_info* info) {
  TRY(check_ctx(ctx));
  if (!info) return EODABE_EINVAL;
  std::memset(info, 0, sizeof(*info));
  if (m < 0 || n < 0 || lda < n || lda < 1) return EODABE_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return EODABE_EINVAL;
  if (ctx->o.sketch_dtype != EODABE_SKETCH_NATIVE) return EODABE_EINVAL;
  CplxPlan p;
  if (!cplx_plan(ctx, m, n, r_cap, p)) return EODABE_EINVAL;
  if (!ws || ws_bytes < p.total) return EODABE_EWORKSPACE;
  if (m == 0 || n == 0) return EODABE_OK;
  if (!A || !Ut || !core || !Vt) return EODABE_EINVAL;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  char* base = (char*)ws;
  void* Ar = base + p.off_a;
  void* Utr = base + p.off_u;
  void* Dr = base + p.off_d;
  void* Vtr = base + p.off_v;
  const bool f64 = ctx->o.a_dtype == EODABE_F64;
  {
    dim3 grid((unsigned)cdiv(n, 256), (unsigned)m);
    if (f64)
      hipLaunchKernelGGL(k_cplx_pack<double>, grid, dim3(256), 0, st, (const double*)A, m, n, lda, (double*)Ar, p.ld2);
    else
      hipLaunchKernelGGL(k_cplx_pack<float>, grid, dim3(256), 0, st, (const float*)A, m, n, lda, (float*)Ar, p.ld2);
    LAUNCHCHK();
  }
  // ||A_r||_F = sqrt(2) ||A||_F: tol / sqrt(2) keeps eps = tol ||A||_F
  eodabe_info ri{};
  ctx->cplx_pairs = true;
  const int s = factor_impl(ctx, Ar, 2 * m, 2 * n, p.ld2, tol * 0.70710678118654752440, base + p.off_in, p.inner,
                            Utr, Dr, Vtr, 2 * p.rc, &ri, nullptr, nullptr, 0, false);
  ctx->cplx_pairs = false;
  info->rank = ri.rank / 2;
  info->blocks = ri.blocks;
  info->status_flags = ri.status_flags;
  info->norm_a = ri.norm_a * 0.70710678118654752440;
  info->eps = ri.eps;
  info->relres_est = ri.relres_est * 1.41421356237309504880;
  if (s < 0) return s;
  const int64_t r = info->rank;
  if (r > 0) {
    dim3 grid((unsigned)cdiv(std::max(std::max(m, n), p.rc), 256), (unsigned)r);
    if (f64)
      hipLaunchKernelGGL(k_cplx_unpack<double>, grid, dim3(256), 0, st, (const double*)Utr, (const double*)Dr,
                         (const double*)Vtr, m, n, r, 2 * p.rc, (double*)Ut, (double*)core, (double*)Vt, p.rc);
    else
      hipLaunchKernelGGL(k_cplx_unpack<float>, grid, dim3(256), 0, st, (const float*)Utr, (const float*)Dr,
                         (const float*)Vtr, m, n, r, 2 * p.rc, (float*)Ut, (float*)core, (float*)Vt, p.rc);
    LAUNCHCHK();
  }
  HIPCHK(hipStreamSynchronize(st));
  return s;
}

int eodabe_basis(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, double tol,
                 void* ws, size_t ws_bytes, void* Q, int64_t r_cap, double* diagT, int64_t diag_cap,
                 eodabe_info* info) {
  if (m < n) return EODABE_EINVAL;
  return factor_impl(ctx, A, m, n, lda, tol, ws, ws_bytes, nullptr, nullptr, nullptr, r_cap, info, Q,
                     diagT, diag_cap, true);
}

int eodabe_philox(eodabe_ctx* ctx, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                  int64_t count, uint32_t* out) {
  TRY(check_ctx(ctx));
  if (count < 0 || (count > 0 && !out)) return EODABE_EINVAL;
  if (count == 0) return EODABE_OK;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), c0, c1, c2, count, out);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  return EODABE_OK;
}

int eodabe_omega(eodabe_ctx* ctx, int dtype, int64_t n, int64_t col0, int64_t ncols, int64_t ldo,
                 void* out) {
  TRY(check_ctx(ctx));
  if (n < 0 || col0 < 0 || ncols < 0 || ldo < n || ncols > 65535) return EODABE_EINVAL;
  if (dtype != EODABE_F32 && dtype != EODABE_F64) return EODABE_EINVAL;
  if (n == 0 || ncols == 0) return EODABE_OK;
  if (!out) return EODABE_EINVAL;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  const uint32_t k0 = (uint32_t)(ctx->o.seed & 0xffffffffu), k1 = (uint32_t)(ctx->o.seed >> 32);
  dim3 grid((unsigned)cdiv(cdiv(ldo, 4), 256), (unsigned)ncols);
  if (dtype == EODABE_F32)
    hipLaunchKernelGGL(k_omega<float>, grid, dim3(256), 0, st, k0, k1, n, col0, (int)ncols, ldo,
                       (float*)out, nullptr, 0);
  else
    hipLaunchKernelGGL(k_omega<double>, grid, dim3(256), 0, st, k0, k1, n, col0, (int)ncols, ldo,
                       (double*)out, nullptr, 0);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  return EODABE_OK;
}

size_t eodabe_sketch_workspace_size(const eodabe_ctx* ctx, int64_t m, int64_t n, int64_t ncols) {
  if (!ctx || m < 0 || n < 0 || ncols < 0 || ncols > BN_MAX) return 0;
  SketchPlan p = sketch_plan(m, n, ncols);
  SketchLp lp;
  if (ctx->o.a_dtype == EODABE_F64) {
    double *a, *b, *c, *d;
    return sketch_carve<double>(nullptr, m, n, p, &a, &b, &c, &d, &lp);
  }
  float *a, *b, *c, *d;
  return sketch_carve<float>(nullptr, m, n, p, &a, &b, &c, &d, &lp);
}

int eodabe_sketch(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, int64_t col0,
                  int64_t ncols, void* Y, int64_t ldy, void* ws, size_t ws_bytes) {
  TRY(check_ctx(ctx));
  if (m < 0 || n < 0 || lda < n || ncols < 0 || ncols > BN_MAX || ldy < m || col0 < 0)
    return EODABE_EINVAL;
  if (m == 0 || n == 0 || ncols == 0) return EODABE_OK;
  if (!A || !Y) return EODABE_EINVAL;
  if (!ws || ws_bytes < eodabe_sketch_workspace_size(ctx, m, n, ncols)) return EODABE_EWORKSPACE;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  const SketchPlan p = sketch_plan(m, n, ncols);
  const int64_t bn = p.bn, ldk = p.ldk, ldyp = p.ldyp;
  const uint32_t k0 = (uint32_t)(ctx->o.seed & 0xffffffffu), k1 = (uint32_t)(ctx->o.seed >> 32);
  auto body = [&](auto tag) -> int {
    typedef decltype(tag) T;
    T *om, *yp, *ap, *yr;
    SketchLp lp;
    sketch_carve<T>(ws, m, n, p, &om, &yp, &ap, &yr, &lp);
    const T* Ae = (const T*)A;
    int64_t la = lda;
    if (!(((uintptr_t)A % 16 == 0) && (lda % 4 == 0))) {
      TRY(copy2d<T>(ctx, st, (const T*)A, lda, ap, ldk, m, n, 0));
      Ae = ap;
      la = ldk;
    }
    const int lpm0 = ctx->o.a_dtype == EODABE_F32 ? ctx->o.sketch_dtype : 0;
    const bool rows = !lpm0 && use_sketch_rows(m, p.s, bn);
    if (rows) {
      dim3 grid((unsigned)cdiv(cdiv(rup(n, 16), 4), 256), (unsigned)bn);
      hipLaunchKernelGGL((k_omega_tiled<T>), grid, dim3(256), 0, st, k0, k1, n, col0, (int)ncols, (int)(bn / 16),
                         om, nullptr, 0, StateInit{});
    } else {
      dim3 grid((unsigned)cdiv(cdiv(ldk, 4), 256), (unsigned)bn);
      hipLaunchKernelGGL((k_omega<T>), grid, dim3(256), 0, st, k0, k1, n, col0, (int)ncols, ldk, om,
                         nullptr, 0);
      if (ncols < bn)
        hipLaunchKernelGGL(k_zero<T>, dim3(64), dim3(256), 0, st, om + ncols * ldk, (bn - ncols) * ldk);
    }
    LAUNCHCHK();
    Ops<T> ops{ctx, st};
    const int64_t ystr = ldyp * bn;
    const int lpm = ctx->o.a_dtype == EODABE_F32 ? ctx->o.sketch_dtype : 0;
    if (lpm) {
      // low-precision form: max |A| -> scale, write the FP16/BF16 copy of A,
      // then sketch the copy (the two FP32 passes' Y partials are discarded)
      hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, st, lp.st, 1.0, (int64_t*)nullptr, 0,
                         (int32_t*)nullptr, (int64_t)0, (int32_t*)nullptr, 0, lpm, 0);
      TRY(ops.sketch(Ae, la, om, ldk, m, (int)bn, n, (int)p.s, yp, ldyp, ystr, lp.normp, nullptr, 0,
                     lp.maxp));
      const int64_t nparts = (int64_t)eff_splits(n, (int)p.s) * std::max<int64_t>(cdiv(m, 128), 1);
      hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(256), 0, st, lp.normp, lp.maxp, nparts, lp.st);
      TRY(ops.sketch(Ae, la, om, ldk, m, (int)bn, n, (int)p.s, yp, ldyp, ystr, nullptr, nullptr, 0,
                     nullptr, lpm, lp.alp, lp.ld_lp, lp.st));
      if constexpr (sizeof(T) == 4)
        TRY(ops.sketch_lp(lpm, lp.alp, lp.ld_lp, om, ldk, m, (int)bn, n, (int)p.s, yp, ldyp, ystr, lp.st,
                          nullptr, 0));
    } else if (rows) {
      TRY(ops.sketch_rows(Ae, la, om, m, (int)bn, n, yr, ldyp, nullptr, nullptr, 0));
    } else {
      TRY(ops.sketch(Ae, la, om, ldk, m, (int)bn, n, (int)p.s, yp, ldyp, ystr, nullptr, nullptr, 0));
    }
    if (!rows)
      TRY(ops.reduce_wide((const T*)yp, eff_splits(n, (int)p.s), ystr, ystr, yr));
    TRY(copy2d<T>(ctx, st, yr, ldyp, (T*)Y, ldy, ncols, m, 0));
    HIPCHK(hipStreamSynchronize(st));
    return 0;
  };
  return ctx->o.a_dtype == EODABE_F64 ? body(double{}) : body(float{});
}


// ---------------------------------------------------------------------------
// Applications: colour-image compression and hyperspectral classification.
// ---------------------------------------------------------------------------
namespace {
struct ImgPlan {
  int64_t rc, per, nparts;
  size_t fws, total;
  size_t off_b, off_parts, off_metrics;
};
bool img_plan(eodabe_ctx* ctx, int channels, int64_t h, int64_t w, ImgPlan& p) {
  if (channels < 1 || channels > IMG_MAX_CH || h < 1 || w < 1) return false;
  p.rc = std::min(h, w);
  p.per = p.rc * (h + p.rc + w);
  p.fws = eodabe_workspace_size(ctx, h, w, p.rc);
  if (p.fws == 0) return false;
  p.nparts = (int64_t)channels * cdiv(h, 64) * cdiv(w, 64);
  Carver c(nullptr);
  c.take<char>((int64_t)p.fws);
  c.take<char>(1);
  p.off_b = (size_t)rup((int64_t)c.off, 256);
  c.take<float>((int64_t)channels * p.rc * w);
  p.off_parts = (size_t)rup((int64_t)c.off, 256);
  c.take<ImgSums>(p.nparts);
  p.off_metrics = (size_t)rup((int64_t)c.off, 256);
  c.take<ImgMetrics>(1);
  p.total = c.off + 256;
  return true;
}
}  // namespace

size_t eodabe_image_workspace_size(eodabe_ctx* ctx, int channels, int64_t h, int64_t w) {
  if (!ctx) return 0;
  ImgPlan p;
  return img_plan(ctx, channels, h, w, p) ? p.total : 0;
}

int eodabe_compress_image(eodabe_ctx* ctx, const float* img, int channels, int64_t h, int64_t w, double tol,
                          void* ws, size_t ws_bytes, float* factors, int64_t factors_len, float* recon,
                          eodabe_image_info* info) {
  TRY(check_ctx(ctx));
  if (!info) return EODABE_EINVAL;
  std::memset(info, 0, sizeof(*info));
  if (!img || !factors || !recon || ctx->o.a_dtype != EODABE_F32) return EODABE_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return EODABE_EINVAL;
  ImgPlan p;
  if (!img_plan(ctx, channels, h, w, p)) return EODABE_EINVAL;
  if (factors_len < (int64_t)channels * p.per) return EODABE_EINVAL;
  if (!ws || ws_bytes < p.total) return EODABE_EWORKSPACE;
  TRY(check_dev(ctx));
  char* base = (char*)ws;
  float* Bbuf = (float*)(base + p.off_b);
  ImgSums* parts = (ImgSums*)(base + p.off_parts);
  ImgMetrics* met = (ImgMetrics*)(base + p.off_metrics);
  // 1. each channel through EOD-ABE, one single-matrix factorization after
  //    the other (the channels as tiles of one persistent launch occupy only
  //    as many CUs as there are channels: 1.20 ms for a 1024^2 RGB image
  //    against about 0.3 ms this way)
  int64_t ranks[IMG_MAX_CH] = {0, 0, 0, 0};
  for (int c = 0; c < channels; ++c) {
    float* Ut = factors + (int64_t)c * p.per;
    eodabe_info fi{};
    const int e = eodabe_factor(ctx, img + (int64_t)c * h * w, h, w, w, tol, ws, p.fws, Ut, Ut + p.rc * h,
                                Ut + p.rc * (h + p.rc), p.rc, &fi);
    if (e < 0) return e;
    ranks[c] = fi.rank;
  }
  // 2. reconstruction U_hat (D_hat V_hat^T) with the criteria fused in
  ImgJob job{};
  int rmax = 0;
  for (int c = 0; c < channels; ++c) {
    const float* Ut = factors + (int64_t)c * p.per;
    job.Ut[c] = Ut;
    job.core[c] = Ut + p.rc * h;
    job.Vt[c] = Ut + p.rc * (h + p.rc);
    job.B[c] = Bbuf + (int64_t)c * p.rc * w;
    job.r[c] = (int)ranks[c];
    rmax = std::max(rmax, (int)ranks[c]);
  }
  job.rc = (int)p.rc;
  hipStream_t st = ctx->stream;
  if (rmax > 0) {
    hipLaunchKernelGGL(k_img_dvt, dim3((unsigned)cdiv(w, 256), (unsigned)rmax, (unsigned)channels), dim3(256), 0,
                       st, job, w);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_img_recon, dim3((unsigned)cdiv(w, 64), (unsigned)cdiv(h, 64), (unsigned)channels),
                     dim3(256), 0, st, job, img, h, w, recon, parts);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_img_metrics, dim3(1), dim3(256), 0, st, parts, p.nparts, (double)channels * h * w, met);
  LAUNCHCHK();
  ImgMetrics hm{};
  HIPCHK(hipMemcpyAsync(&hm, met, sizeof(hm), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // 3. storage accounting of the introduction: (h + w) r + r (r + 1) / 2
  //    entries per channel against h w, and the rank below which the
  //    factors take less
  double stored = 0.0;
  for (int c = 0; c < channels; ++c) {
    info->rank[c] = ranks[c];
    const double r = (double)ranks[c];
    stored += (double)(h + w) * r + r * (r + 1.0) / 2.0;
  }
  info->channels = channels;
  info->relerr = hm.relerr;
  info->psnr = hm.psnr;
  info->ssim = hm.ssim;
  info->stored = stored;
  info->full = (double)channels * h * w;
  info->reduction = 1.0 - stored / info->full;
  const double hd = (double)h, wd = (double)w;
  info->rank_bound = std::sqrt(hd * hd + wd * wd + 4.0 * hd * wd + hd + wd + 0.25) - (hd + wd + 0.5);
  return EODABE_OK;
}

int eodabe_features(eodabe_ctx* ctx, const float* Ut, const float* core, int64_t m, int64_t r, int64_t r_cap,
                    float* F, int64_t ldf) {
  TRY(check_ctx(ctx));
  if (m < 0 || r < 0 || r_cap < r || ldf < r || r > 65535) return EODABE_EINVAL;
  if (m == 0 || r == 0) return EODABE_OK;
  if (!Ut || !core || !F) return EODABE_EINVAL;
  TRY(check_dev(ctx));
  hipLaunchKernelGGL(k_features, dim3((unsigned)cdiv(m, 256), (unsigned)r), dim3(256), 0, ctx->stream, Ut, core, m,
                     (int)r, r_cap, F, ldf);
  LAUNCHCHK();
  return EODABE_OK;
}

size_t eodabe_knn_workspace_size(int nclass) {
  if (nclass < 1 || nclass > KNN_CMAX) return 0;
  return (size_t)nclass * nclass * sizeof(unsigned long long) + 256;
}

int eodabe_knn_cv(eodabe_ctx* ctx, const float* F, int64_t m, int d, int64_t ldf, const int32_t* labels,
                  const int32_t* fold, int k, int nclass, int32_t* pred, void* ws, size_t ws_bytes,
                  int64_t* confusion, double* oa) {
  TRY(check_ctx(ctx));
  if (m < 1 || d < 1 || d > KNN_DMAX || ldf < d || k < 1 || k > KNN_KMAX || nclass < 1 || nclass > KNN_CMAX)
    return EODABE_EINVAL;
  if (!F || !labels || !fold || !pred) return EODABE_EINVAL;
  if (!ws || ws_bytes < eodabe_knn_workspace_size(nclass)) return EODABE_EWORKSPACE;
  TRY(check_dev(ctx));
  hipStream_t st = ctx->stream;
  unsigned long long* conf = (unsigned long long*)ws;
  const int64_t nc2 = (int64_t)nclass * nclass;
  hipLaunchKernelGGL(k_zero<unsigned long long>, dim3(1), dim3(256), 0, st, conf, nc2);
  hipLaunchKernelGGL(k_knn_cv, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, st, F, m, d, ldf, labels, fold, k,
                     nclass, pred, conf);
  LAUNCHCHK();
  std::vector<unsigned long long> hc((size_t)nc2);
  HIPCHK(hipMemcpyAsync(hc.data(), conf, (size_t)nc2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  unsigned long long tr = 0, tot = 0;
  for (int i = 0; i < nclass; ++i)
    for (int j = 0; j < nclass; ++j) {
      const unsigned long long v = hc[(size_t)i * nclass + j];
      if (confusion) confusion[(size_t)i * nclass + j] = (int64_t)v;
      tot += v;
      if (i == j) tr += v;
    }
  if (oa) *oa = tot ? (double)tr / (double)tot : 0.0;
  return EODABE_OK;
}

}  // extern "C"
