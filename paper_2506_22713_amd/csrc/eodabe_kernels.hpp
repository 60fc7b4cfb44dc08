// Device kernels of the EOD-ABE hot path for CDNA4 (gfx950, wave64).
//
// Layout conventions (all sizes in elements):
//   A      row-major m x n, lda            (input, read only)
//   Omega  stored transposed: row j of the buffer is column c0+j of Omega
//   Y, Z   column-major m x f (ld >= m, multiple of 4): the current block
//   Q      column-major m x w (ldq): the basis accumulated so far
//   G, R   small FP64 matrices, element (i, j) at j*ld + i
// Every GEMM here is a "stream one operand, reduce over K" skinny product;
// the MFMA micro-kernels use v_mfma_*_16x16x4 with each lane loading four
// consecutive K values (16 B for FP32) per operand, so both operands are
// read with dwordx4 loads and the four MFMAs of a chunk consume them in
// K-order 4g+v (g = lane/16, v = 0..3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace eodabe {

typedef float  f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr double U64 = 1.1102230246251565e-16;   // 2^-53
constexpr double FLOOR_C = 64.0;                 // pivot floor: FLOOR_C * u64 * G(k,k)
constexpr double PIV_MIN = 1e-290;               // smaller pivots count as non-positive (1/p overflows)

// Largest divisor of n that is at most 8 (loads per batch).
constexpr int batch_of(int n) {
  for (int b = 8; b > 1; --b)
    if (n % b == 0) return b;
  return 1;
}

// Control block shared by the kernels of one factorization (device memory).
struct State {
  double eps;            // tol * ||A||_F
  double normsq;         // ||A||_F^2
  double tol;
  int32_t stop_block;    // first block whose stop test fired (INT32_MAX: none yet)
  int32_t nonfinite;     // ||A||_F not finite
  int32_t floored;       // a pivot was floored in the closing QRs
  int32_t paired;        // complex input (realified): stops only at pair-leading columns
  int64_t rank;          // basis width after the latest decided block
  uint32_t counter[8];   // arrival counters: [0] the Gram kernels' (reset by their last workgroup); [1] block 0's and
                         // [2] the closing's one-launch CholeskyQR2 (one launch each, zeroed here); [3] the later blocks'
                         // (shared, reset by the last workgroup out)
  double lp_scale;       // power of two applied to A before rounding it to FP16 (1 for BF16)
  int32_t lp_mode;       // 0: none, 1: FP16, 2: BF16 (low-precision sketch form)
  int32_t sync_fail;     // a barrier across workgroups timed out (outputs void)
  double d_stop;         // |T(l,l)| of the column whose test stopped the loop (0: none)
};
static_assert(sizeof(State) % 8 == 0, "the control block is copied in 8-byte words");

// The reset of the control block and the per-block logs at the start of a
// factorization; thread t of nt threads in all clears its share.
struct StateInit {
  State* st;                 // null: nothing to reset
  double tol;
  int64_t* wlog;
  int nwlog;
  int32_t* dead;
  int64_t ndead;
  int32_t* acc;
  int nacc;
  int lp_mode;
  int paired;
};

__device__ __forceinline__ void init_state_part(const StateInit& a, int64_t t, int64_t nt) {
  if (t == 0) {
    State* st = a.st;
    st->eps = 0.0; st->normsq = 0.0; st->tol = a.tol;
    st->stop_block = 0x7fffffff; st->nonfinite = 0; st->floored = 0; st->paired = a.paired; st->rank = 0;
    for (int i = 0; i < 8; ++i) st->counter[i] = 0u;
    st->lp_scale = 1.0; st->lp_mode = a.lp_mode; st->sync_fail = 0; st->d_stop = 0.0;
  }
  for (int64_t i = t; i < a.nwlog; i += nt) a.wlog[i] = 0;
  for (int64_t i = t; i < a.ndead; i += nt) a.dead[i] = 0;
  for (int64_t i = t; i < a.nacc; i += nt) a.acc[i] = 0;
}

// Low-precision copies of A for the sketch: IEEE binary16 or bfloat16,
// both rounded to nearest even from FP32 and stored as 16-bit patterns.
__device__ __forceinline__ uint16_t to_f16_bits(float x) {
  const _Float16 h = (_Float16)x;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ uint16_t to_bf16_bits(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <int LPT>
__device__ __forceinline__ uint16_t to_lp_bits(float x) {
  if constexpr (LPT == 1) return to_f16_bits(x);
  else return to_bf16_bits(x);
}
// Scale for the FP16 copy: 2^(14 - e) with max|A| = f 2^e, f in [0.5, 1),
// so the largest entry lands in [2^13, 2^14).  BF16 needs none.
__device__ __forceinline__ double lp_scale_of(float maxabs, int lp_mode) {
  if (lp_mode != 1 || !(maxabs > 0.0f) || !(maxabs < INFINITY)) return 1.0;
  int e = 0;
  (void)frexpf(maxabs, &e);
  return ldexp(1.0, 14 - e);
}

// Gate of closing-step kernels enqueued before the host has seen the stop
// flag of the basis loop: they run only once the loop has stopped, ||A||_F
// is finite and the rank r satisfies 0 < r <= r_cap; otherwise every such
// kernel returns at once (a later, host-checked launch takes over).
struct Gate {
  const State* st;       // null: always open
  int64_t r_cap;
};
// Handing a workgroup's global stores to other workgroups: every wave
// waits until its own stores have reached L2 (s_waitcnt vmcnt(0); the
// immediate keeps expcnt and lgkmcnt at their no-wait maxima), the
// workgroup meets, and thread 0 alone then takes the device-scope release,
// one L2 write-back for the workgroup instead of one per wave.  The
// receiving side mirrors it: thread 0 takes the acquire (one L1/L2
// invalidate) before the barrier that lets its waves read.
__device__ __forceinline__ void wg_stores_done() {
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
}

__device__ __forceinline__ bool gate_shut(const Gate& g) {
  if (!g.st) return false;
  return g.st->stop_block == 0x7fffffff || g.st->nonfinite != 0 || g.st->rank <= 0 ||
         g.st->rank > g.r_cap;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Two standard normals from two uniform words: u1 = (x+1) 2^-32 in (0,1],
// u2 = y 2^-32 in [0,1), r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).
// Evaluated in FP64 and rounded to FP32.
__device__ __forceinline__ void box_muller(uint32_t x, uint32_t y, float& z0, float& z1) {
  const double u1 = ((double)x + 1.0) * 2.3283064365386963e-10;
  const double u2 = (double)y * 2.3283064365386963e-10;
  const double rad = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(2.0 * 3.141592653589793 * u2, &s, &c);
  z0 = (float)(rad * c);
  z1 = (float)(rad * s);
}

// Rows 4q .. 4q+3 of column c of Omega: Philox counter (q, c, 0, 0); words
// (x0,x1) -> rows 4q, 4q+1 and (x2,x3) -> rows 4q+2, 4q+3.
__device__ __forceinline__ void omega4(uint32_t k0, uint32_t k1, int64_t q, int64_t c, float (&z)[4]) {
  U4 r = philox4x32_10(U4{(uint32_t)q, (uint32_t)c, 0u, 0u}, k0, k1);
  box_muller(r.x, r.y, z[0], z[1]);
  box_muller(r.z, r.w, z[2], z[3]);
}

__global__ void k_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                         int64_t count, uint32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  U4 r = philox4x32_10(U4{c0 + (uint32_t)i, c1, c2, 0u}, k0, k1);
  out[4 * i + 0] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
}

// out[j*ldo + i] = Omega(i, col0 + j), i < n; zero for n <= i < ldo.
// Entry (i, c): Philox counter (i/4, c, 0, 0); words (x0,x1) -> rows 4q, 4q+1,
// (x2,x3) -> rows 4q+2, 4q+3.
template <typename T>
__global__ void k_omega(uint32_t k0, uint32_t k1, int64_t n, int64_t col0, int ncols,
                        int64_t ldo, T* __restrict__ out, const int32_t* __restrict__ stop_block,
                        int block_id) {
  if (stop_block && *stop_block < block_id) return;
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (4 * q >= ldo || j >= ncols) return;
  float z[4] = {0.f, 0.f, 0.f, 0.f};
  if (4 * q < n) omega4(k0, k1, q, col0 + j, z);
  T* o = out + (int64_t)j * ldo + 4 * q;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (4 * q + e < ldo) o[e] = (4 * q + e < n) ? (T)z[e] : (T)0;
}

// Test-matrix columns col0 .. col0+ncols-1 (zero columns up to 16 ct) in the
// tiled layout k_sketch_rows reads: the four entries of rows 4q .. 4q+3 of
// column c sit together at ((q/4 ct + c/16) 64 + (q%4) 16 + c%16) 4, so one
// wave reads the operand of a 16-row chunk of a 16-column tile as 1 KiB
// contiguous.  Entries past n (up to the next multiple of 16) are zero.
// Same values as k_omega (each entry a pure function of (seed, row, column)).
// Grid: (ceil(rup(n, 16) / 4 / 256), 16 ct).
// With init.st set (the first launch of a factorization, block 0, which no
// stop can gate) the grid also resets the control block and the logs, as
// k_init_state does, and reads no stop flag.
template <typename T>
__global__ void k_omega_tiled(uint32_t k0, uint32_t k1, int64_t n, int64_t col0, int ncols, int ct,
                              T* __restrict__ out, const int32_t* __restrict__ stop_block, int block_id,
                              StateInit init) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (init.st) {
    const int64_t nx = (int64_t)gridDim.x * blockDim.x;
    init_state_part(init, j * nx + q, nx * gridDim.y);
  } else if (stop_block && *stop_block < block_id) {
    return;
  }
  const int64_t n16 = (n + 15) / 16 * 16;
  if (4 * q >= n16 || j >= 16 * ct) return;
  float z[4] = {0.f, 0.f, 0.f, 0.f};
  if (j < ncols && 4 * q < n) omega4(k0, k1, q, col0 + j, z);
  T* o = out + ((((q >> 2) * ct + (j >> 4)) * 64 + (q & 3) * 16 + (j & 15)) << 2);
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] = (j < ncols && 4 * q + e < n) ? (T)z[e] : (T)0;
}

// Columns of the test matrix of a realified complex problem (nn = 2 nc rows):
// real column 2c + p is the realification of omega_c (p = 0) or of
// i omega_c (p = 1), omega_c = (g_2c + i g_2c+1) / sqrt(2) the complex
// standard Gaussian column c (g_j the FP64 Box-Muller column j of the real
// test matrix, each part rounded to FP32 after the scaling):
//   p = 0: rows [0, nc) Re omega_c, rows [nc, 2 nc) Im omega_c;
//   p = 1: rows [0, nc) -Im omega_c, rows [nc, 2 nc) Re omega_c.
// Layout as k_omega: out[j*ldo + i] for real column col0 + j.
__device__ __forceinline__ double gauss64(uint32_t k0, uint32_t k1, int64_t row, int64_t col) {
  const U4 r = philox4x32_10(U4{(uint32_t)(row >> 2), (uint32_t)col, 0u, 0u}, k0, k1);
  const int e = (int)(row & 3);
  const uint32_t x = e < 2 ? r.x : r.z, y = e < 2 ? r.y : r.w;
  const double u1 = ((double)x + 1.0) * 2.3283064365386963e-10;
  const double u2 = (double)y * 2.3283064365386963e-10;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(2.0 * 3.141592653589793 * u2, &sn, &cs);
  return (e & 1) ? rad * sn : rad * cs;
}

template <typename T>
__global__ void k_omega_paired(uint32_t k0, uint32_t k1, int64_t nn, int64_t col0, int ncols, int64_t ldo,
                               T* __restrict__ out, const int32_t* __restrict__ stop_block, int block_id) {
  if (stop_block && *stop_block < block_id) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= ldo || j >= ncols) return;
  const int64_t nc = nn / 2;
  T v = (T)0;
  if (i < nn) {
    const int64_t jr = col0 + j, c = jr >> 1;
    const int p = (int)(jr & 1);
    const bool top = i < nc;
    const int64_t ii = top ? i : i - nc;
    // Re omega for (p = 0, top) and (p = 1, bottom); Im omega otherwise
    const bool want_re = (p == 0) == top;
    const double g = gauss64(k0, k1, ii, want_re ? 2 * c : 2 * c + 1) * 0.70710678118654752440;
    const float gf = (float)g;
    v = (T)((p == 1 && top) ? -gf : gf);
  }
  out[(int64_t)j * ldo + i] = v;
}

// Pair structure of a realified complex block: column 2p + 1 := J column
// 2p with J [a; b] = [-b; a] (halves of length nn / 2), i.e. the partner
// column is i times the leading one.  Every realified matrix commutes with
// J, so this only discards the independent rounding of the partner, which a
// cancelling step (projection of a weak direction) would otherwise amplify.
// Columns: X + c * ld, length nn; ncols even.
template <typename T>
__global__ void k_pair_fix(T* __restrict__ X, int64_t ld, int64_t nn, int64_t ncols,
                           const int32_t* __restrict__ stop_block, int block_id) {
  if (stop_block && *stop_block < block_id) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, p = blockIdx.y;
  if (i >= nn || 2 * p + 1 >= ncols) return;
  const int64_t h = nn / 2;
  const T* lead = X + (2 * p) * ld;
  X[(2 * p + 1) * ld + i] = i < h ? -lead[i + h] : lead[i - h];
}

// Complex input (interleaved real, imaginary) m x n, row stride lda complex
// elements, to its realification [[Re A, -Im A], [Im A, Re A]] (2m x 2n,
// row-major, row stride ldr).
template <typename T>
__global__ void k_cplx_pack(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda, T* __restrict__ Ar,
                            int64_t ldr) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, i = blockIdx.y;
  if (j >= n || i >= m) return;
  const T re = A[2 * (i * lda + j)], im = A[2 * (i * lda + j) + 1];
  Ar[i * ldr + j] = re;
  Ar[i * ldr + n + j] = -im;
  Ar[(m + i) * ldr + j] = im;
  Ar[(m + i) * ldr + n + j] = re;
}

// Complex factors from those of the realification (pair-ordered rank index):
//   U column a = rows [0, m) + i rows [m, 2m) of realified column 2a,
//   V^H row a = conj of the same for V,
//   D(p, q) = Dr(2p, 2q) + i Dr(2p + 1, 2q).
// Outputs interleaved complex: Ut (r_cap x m), core (r_cap x r_cap), Vt (r_cap x n).
template <typename T>
__global__ void k_cplx_unpack(const T* __restrict__ Utr, const T* __restrict__ Dr, const T* __restrict__ Vtr,
                              int64_t m, int64_t n, int64_t r, int64_t rc2, T* __restrict__ Ut, T* __restrict__ core,
                              T* __restrict__ Vt, int64_t rc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, a = blockIdx.y;
  if (a >= r) return;
  if (t < m) {
    const T* u = Utr + (2 * a) * (2 * m);
    Ut[2 * (a * m + t)] = u[t];
    Ut[2 * (a * m + t) + 1] = u[m + t];
  }
  if (t < n) {
    const T* v = Vtr + (2 * a) * (2 * n);
    Vt[2 * (a * n + t)] = v[t];
    Vt[2 * (a * n + t) + 1] = -v[n + t];
  }
  if (t < rc) {
    T re = (T)0, im = (T)0;
    if (t < r) {
      re = Dr[(2 * a) * rc2 + 2 * t];
      im = Dr[(2 * a + 1) * rc2 + 2 * t];
    }
    core[2 * (a * rc + t)] = re;
    core[2 * (a * rc + t) + 1] = im;
  }
}

// ---------------------------------------------------------------------------
// MFMA wrappers: D(16x16) += A(16x4) B(4x16).  Lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  Accumulator register e of lane l holds D[row][l%16]
// with row = Mfma::row(l/16, e): 4(l/16)+e for the f32 instruction,
// 4e+(l/16) for the f64 one.
// ---------------------------------------------------------------------------
template <typename Tacc> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static constexpr bool rows_contiguous = true;
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static constexpr bool rows_contiguous = false;
  static __device__ __forceinline__ int row(int g, int e) { return 4 * e + g; }
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Four consecutive elements.
template <typename T> struct V4 { T v[4]; };
template <typename T>
__device__ __forceinline__ V4<T> ld4(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    f32x4 x = *reinterpret_cast<const f32x4*>(p);
    r.v[0] = x[0]; r.v[1] = x[1]; r.v[2] = x[2]; r.v[3] = x[3];
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 a = q[0], b = q[1];
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}
template <typename T>
__device__ __forceinline__ V4<T> ld4_masked(const T* p, int64_t k, int64_t kend) {
  V4<T> r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r.v[e] = (k + e < kend) ? p[e] : (T)0;
  return r;
}

// ---------------------------------------------------------------------------
// NT GEMM partials: out_s(M x N) = X(M x K) * Z(N x K)^T over K-split s.
// X row-major (ldx), Z row-major (ldz); both K-contiguous, ldx/ldz multiples
// of 4 and 16-byte aligned bases.  out_s element (m, j) at
// out + s*part_stride + j*ldo + m  (column-major; ldo multiple of 4).
// Workgroup = 4 waves; wave w owns rows [m0 + 16*RT*w, +16*RT) and all 16*CT
// columns of the grid-z tile.  If sumsq != nullptr, each workgroup of grid-z
// tile 0 writes sum(X^2) over the elements it read to sumsq[block id].
// M_dev / block control: if wlog != nullptr the row count M is read from
// wlog[block_id] (basis width known only on the device) and the kernel
// returns at once when *stop_block < block_id.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tacc, int RT, int CT>
__global__ __launch_bounds__(256) void k_gemm_nt(
    const Tin* __restrict__ X, int64_t ldx, const Tin* __restrict__ Z, int64_t ldz,
    int64_t M, int64_t N, int64_t K, int64_t kchunk, Tacc* __restrict__ out, int64_t ldo,
    int64_t part_stride, double* __restrict__ sumsq, const int64_t* __restrict__ wlog,
    const int32_t* __restrict__ stop_block, int block_id) {
  typedef Mfma<Tacc> MF;
  if (stop_block && *stop_block < block_id) return;
  if (wlog) M = wlog[block_id];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * (64 * RT) + wv * (16 * RT);
  const int64_t n0 = (int64_t)blockIdx.z * (16 * CT);
  const int s = blockIdx.y;
  const int64_t kb = (int64_t)s * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  const bool do_ss = (sumsq != nullptr) && blockIdx.z == 0;
  double ss = 0.0;
  __shared__ double ss_red[4];
  if (m0 >= M || kb >= ke) {       // nothing to do for this wave (still reach the reduction)
    if (do_ss) {
      if (lane == 0) ss_red[wv] = 0.0;
      __syncthreads();
      if (threadIdx.x == 0)
        sumsq[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ss_red[0] + ss_red[1] + ss_red[2] + ss_red[3];
    }
    return;
  }
  const Tin* xp[RT];
  bool xvalid[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = m0 + 16 * t + r;
    xvalid[t] = row < M;
    xp[t] = X + (xvalid[t] ? row : (M - 1)) * ldx + 4 * g;
  }
  const Tin* zp[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) {
    const int64_t col = n0 + 16 * u + r;
    zp[u] = Z + (col < N ? col : (N - 1)) * ldz + 4 * g;
  }
  typename MF::acc_t acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[t][u] = MF::zero();

  const int64_t kfull = kb + ((ke - kb) / 16) * 16;
  V4<Tin> a[RT], b[CT];
  int64_t k = kb;
  if (k < kfull) {
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t] = ld4(xp[t] + k);
#pragma unroll
    for (int u = 0; u < CT; ++u) b[u] = ld4(zp[u] + k);
  }
  for (; k < kfull; k += 16) {
    V4<Tin> an[RT], bn[CT];
    const bool more = k + 16 < kfull;
    if (more) {
#pragma unroll
      for (int t = 0; t < RT; ++t) an[t] = ld4(xp[t] + k + 16);
#pragma unroll
      for (int u = 0; u < CT; ++u) bn[u] = ld4(zp[u] + k + 16);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u)
          acc[t][u] = MF::op((Tacc)a[t].v[v], (Tacc)b[u].v[v], acc[t][u]);
    if (do_ss) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
        if (xvalid[t])
#pragma unroll
          for (int v = 0; v < 4; ++v) ss += (double)a[t].v[v] * (double)a[t].v[v];
    }
    if (more) {
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t] = an[t];
#pragma unroll
      for (int u = 0; u < CT; ++u) b[u] = bn[u];
    }
  }
  if (kfull < ke) {                 // ragged K tail
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t] = ld4_masked(xp[t] + kfull, kfull + 4 * g, ke);
#pragma unroll
    for (int u = 0; u < CT; ++u) b[u] = ld4_masked(zp[u] + kfull, kfull + 4 * g, ke);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u)
          acc[t][u] = MF::op((Tacc)a[t].v[v], (Tacc)b[u].v[v], acc[t][u]);
    if (do_ss) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
        if (xvalid[t])
#pragma unroll
          for (int v = 0; v < 4; ++v) ss += (double)a[t].v[v] * (double)a[t].v[v];
    }
  }
  Tacc* o = out + (int64_t)s * part_stride;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const int64_t col = n0 + 16 * u + r;
      if (col >= N) continue;
      if constexpr (MF::rows_contiguous) {
        const int64_t row = m0 + 16 * t + 4 * g;
        Tacc* p = o + col * ldo + row;
        if (row + 3 < M && ((ldo & 3) == 0) && ((part_stride & 3) == 0)) {
          *reinterpret_cast<f32x4*>(p) = acc[t][u];
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e < M) p[e] = acc[t][u][e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = m0 + 16 * t + MF::row(g, e);
          if (row < M) o[col * ldo + row] = acc[t][u][e];
        }
      }
    }
  }
  if (do_ss) {
    // wave reduction then workgroup reduction (fixed order: deterministic)
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0) ss_red[wv] = ss;
    __syncthreads();
    if (threadIdx.x == 0)
      sumsq[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ss_red[0] + ss_red[1] + ss_red[2] + ss_red[3];
  }
}

// ---------------------------------------------------------------------------
// Sketch Y = A Omega_j (Alg. 1), K-split partials, on MFMA.
// A row-major (lda multiple of 4, 16-byte aligned); Omega^T row-major
// (N x ldk, N <= 16*CT columns).  Workgroup = 4 waves on 4 row tiles of 16*RT rows, one K-range
// [kb, ke) per grid-y index.  The workgroup's Omega slab (bn x KS) is staged
// in LDS once per slab (rows padded by 16 bytes), so only A streams from
// HBM; A is prefetched four chunks (16 K each) ahead in registers.  Output
// partial s: element (i, c) at out + s*part_stride + c*ldo + i.  Optional
// per-workgroup sum of squares of A (tile z == 0 only) for ||A||_F.
// ---------------------------------------------------------------------------
template <typename T, int RT, int CT>
struct SketchCfg {
  static constexpr int KS = (16 * CT * (int)sizeof(T) <= 128) ? 256 : 128;
  static constexpr int LDO = KS + 16 / (int)sizeof(T);
};

template <typename T, int RT, int CT, int LPW>
__global__ __launch_bounds__(256) void k_sketch(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ Om, int64_t ldk, int64_t M, int N,
    int64_t K, int64_t kchunk, T* __restrict__ out, int64_t ldo, int64_t part_stride,
    double* __restrict__ sumsq, float* __restrict__ maxabs, uint16_t* __restrict__ lp_out,
    int64_t ld_lp, const State* __restrict__ lp_st, const int32_t* __restrict__ stop_block,
    int block_id) {
  typedef Mfma<T> MF;
  typedef SketchCfg<T, RT, CT> Cfg;
  constexpr int KS = Cfg::KS, LDO = Cfg::LDO, NC = 16 * CT;
  if (stop_block && *stop_block < block_id) return;
  __shared__ T oms[NC * LDO];
  __shared__ double ss_red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * (64 * RT) + wv * (16 * RT);
  const int s = blockIdx.y;
  const int64_t kb = (int64_t)s * kchunk, ke = min(K, kb + kchunk);
  const bool do_ss = sumsq != nullptr;
  double ss = 0.0;
  float mx = 0.0f;
  float lps = 1.0f;                       // scale of the low-precision copy (LPW != 0)
  if constexpr (LPW != 0) lps = (float)lp_st->lp_scale;
  const T* ap[RT];
  bool aval[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = m0 + 16 * t + r;
    aval[t] = row < M;
    ap[t] = A + (aval[t] ? row : (M - 1)) * lda + 4 * g;
  }
  typename MF::acc_t acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[t][u] = MF::zero();
  const bool active = (m0 < M);
  // A chunks in flight: the first slab's four are requested before its
  // Omega staging, so the two memory latencies overlap
  // (chunk indices past the slab's last full chunk are clamped to it: the
  // loads stay unconditional, so the wait counts stay exact, and the
  // duplicates are never used)
  V4<T> a[4][RT];
  {
    const int nfull0 = (int)(min(ke, kb + KS) - kb) / 16;
    if (active && nfull0 > 0)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t) a[q][t] = ld4(ap[t] + kb + 16 * min(q, nfull0 - 1));
  }
  for (int64_t sb = kb; sb < ke; sb += KS) {
    const int64_t se = min(ke, sb + KS);
    const int slen = (int)(se - sb);
    __syncthreads();
    // stage Omega^T[0:NC, sb:se] (zero beyond se and N), a thread's loads
    // all in flight before its LDS stores
    constexpr int NST = NC * (KS / 4) / 256, NB = batch_of(NST);
    static_assert(NC * (KS / 4) % 256 == 0 && NST % NB == 0, "staging split");
#pragma unroll
    for (int q0 = 0; q0 < NST; q0 += NB) {
      V4<T> sv[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int idx = tid + 256 * (q0 + q);
        const int c = idx / (KS / 4), k4 = (idx - c * (KS / 4)) * 4;
        const T* src = Om + (int64_t)(c < N ? c : 0) * ldk + sb + k4;
        if (c < N && k4 + 3 < slen) sv[q] = ld4(src);
        else if (c < N) sv[q] = ld4_masked(src, k4, slen);
        else
#pragma unroll
          for (int e = 0; e < 4; ++e) sv[q].v[e] = (T)0;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int idx = tid + 256 * (q0 + q);
        const int c = idx / (KS / 4), k4 = (idx - c * (KS / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) oms[c * LDO + k4 + e] = sv[q].v[e];
      }
    }
    __syncthreads();
    if (!active) continue;
    const int nfull = slen / 16;
    auto compute = [&](const V4<T>(&a)[RT], int kl) {
      V4<T> b[CT];
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        const T* q = &oms[(16 * u + r) * LDO + kl + 4 * g];
#pragma unroll
        for (int e = 0; e < 4; ++e) b[u].v[e] = q[e];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int u = 0; u < CT; ++u) acc[t][u] = MF::op(a[t].v[v], b[u].v[v], acc[t][u]);
      if (do_ss) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
          if (aval[t])
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              ss += (double)a[t].v[v] * (double)a[t].v[v];
              mx = fmaxf(mx, fabsf((float)a[t].v[v]));
            }
      }
      if constexpr (LPW != 0) {            // low-precision copy of this chunk of A
        const int64_t k = sb + kl + 4 * g;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          if (!aval[t]) continue;
          uint16_t* dst = lp_out + (m0 + 16 * t + r) * ld_lp + k;
          if (k + 3 < se) {
            uint2 pk;
            pk.x = (uint32_t)to_lp_bits<LPW>((float)a[t].v[0] * lps) |
                   ((uint32_t)to_lp_bits<LPW>((float)a[t].v[1] * lps) << 16);
            pk.y = (uint32_t)to_lp_bits<LPW>((float)a[t].v[2] * lps) |
                   ((uint32_t)to_lp_bits<LPW>((float)a[t].v[3] * lps) << 16);
            *reinterpret_cast<uint2*>(dst) = pk;
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (k + v < se) dst[v] = to_lp_bits<LPW>((float)a[t].v[v] * lps);
          }
        }
      }
    };
    // 4-deep register pipeline over the full 16-K chunks of this slab (the
    // first slab's chunks were requested before the staging).  The steady
    // state has no branches, so each chunk waits only for its own loads.
    if (sb != kb && nfull > 0)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t) a[q][t] = ld4(ap[t] + sb + 16 * min(q, nfull - 1));
    int c = 0;
    for (; c + 8 <= nfull; c += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        compute(a[q], 16 * (c + q));
#pragma unroll
        for (int t = 0; t < RT; ++t) a[q][t] = ld4(ap[t] + sb + 16 * (c + q + 4));
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {            // last one or two groups (fewer than 8 chunks left)
      if (c + q < nfull) {
        compute(a[q], 16 * (c + q));
        if (c + q + 4 < nfull)
#pragma unroll
          for (int t = 0; t < RT; ++t) a[q][t] = ld4(ap[t] + sb + 16 * (c + q + 4));
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (c + 4 + q < nfull) compute(a[q], 16 * (c + 4 + q));
    if (nfull * 16 < slen) {                  // ragged tail of the slab
      V4<T> at[RT];
      const int64_t k = sb + 16 * nfull;
#pragma unroll
      for (int t = 0; t < RT; ++t) at[t] = ld4_masked(ap[t] + k, k + 4 * g, se);
      compute(at, 16 * nfull);
    }
  }
  if (active) {
    T* o = out + (int64_t)s * part_stride;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        const int64_t col = 16 * u + r;
        if (col >= N) continue;
        if constexpr (MF::rows_contiguous) {
          const int64_t row = m0 + 16 * t + 4 * g;
          T* p = o + col * ldo + row;
          if (row + 3 < M && ((ldo & 3) == 0) && ((part_stride & 3) == 0)) {
            *reinterpret_cast<f32x4*>(p) = acc[t][u];
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (row + e < M) p[e] = acc[t][u][e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t row = m0 + 16 * t + MF::row(g, e);
            if (row < M) o[col * ldo + row] = acc[t][u][e];
          }
        }
      }
    }
  }
  if (do_ss) {
    __shared__ float mx_red[4];
    for (int off = 32; off > 0; off >>= 1) {
      ss += __shfl_xor(ss, off);
      mx = fmaxf(mx, __shfl_xor(mx, off));
    }
    if (lane == 0) {
      ss_red[wv] = ss;
      mx_red[wv] = mx;
    }
    __syncthreads();
    if (tid == 0) {
      const int64_t p = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
      sumsq[p] = ss_red[0] + ss_red[1] + ss_red[2] + ss_red[3];
      if (maxabs) maxabs[p] = fmaxf(fmaxf(mx_red[0], mx_red[1]), fmaxf(mx_red[2], mx_red[3]));
    }
  }
}

// ---------------------------------------------------------------------------
// Sketch Y = A Omega_j (Alg. 1) without K-split partials, for matrices tall
// enough that 16-row tiles fill the chip.  A workgroup of NW waves owns one
// 16-row tile of A and splits its K range NW ways; each wave streams its part
// of the 16 rows with a register ring of dwordx4 loads and accumulates on
// MFMA.  The test matrix comes in the tiled layout of k_omega_tiled (Omt,
// 16 CT columns), so each operand load of a wave is 1 KiB contiguous from L2
// (a workgroup uses all of Omega_j exactly once: no reuse for LDS to
// capture; in the plain column layout the same loads, 16 rows of 64 bytes,
// made the kernel half again slower).  The NW partial tiles are summed in
// LDS in a fixed tree order and wave 0 writes the tile of Y (column-major,
// ldy): no partial buffer in HBM and no separate fold.  SS 1: one partial
// per workgroup of the sum of squares of A (FP32 squares of four entries,
// accumulated in FP64; FP64 data: FP64 throughout), SS 2: also max |a|; LPW:
// the low-precision copy of A, as in k_sketch.  A row-major with lda % 4 == 0
// and 16-byte alignment; rows past M are read at the last row and never
// reach an output; columns N .. 16 CT - 1 are computed and not stored.
// ---------------------------------------------------------------------------
template <typename T, int CT, int NW, int LPW, int SS, int D = ((CT * (int)sizeof(T) <= 16) ? 4 : 2)>
__global__ __launch_bounds__(64 * NW) void k_sketch_rows(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ Omt, int64_t M, int N, int64_t K,
    T* __restrict__ Y, int64_t ldy, double* __restrict__ sumsq, float* __restrict__ maxabs,
    uint16_t* __restrict__ lp_out, int64_t ld_lp, const State* __restrict__ lp_st,
    const int32_t* __restrict__ stop_block, int block_id) {
  typedef Mfma<T> MF;
  typedef typename MF::acc_t acc_t;
  // D: 16-K chunks in flight per wave
  static_assert(NW >= 2 && (NW & (NW - 1)) == 0, "NW: power of two");
  if (stop_block && *stop_block < block_id) return;
  __shared__ acc_t red[NW / 2][CT][64];
  __shared__ double ss_red[NW];
  __shared__ float mx_red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * 16;
  const int64_t kchunk = ((K + NW - 1) / NW + 15) / 16 * 16;
  const int64_t kb = min(K, (int64_t)wv * kchunk), ke = min(K, kb + kchunk);
  double ss = 0.0;
  float mx = 0.0f;
  float lps = 1.0f;
  if constexpr (LPW != 0) lps = (float)lp_st->lp_scale;
  const int64_t row = m0 + r;
  const bool aval = row < M;
  const T* ap = A + (aval ? row : (M - 1)) * lda + 4 * g;
  const T* op = Omt + lane * 4;             // + (chunk CT + u) 256
  acc_t acc[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) acc[u] = MF::zero();
  auto compute = [&](const V4<T>& a, const V4<T>(&b)[CT], int64_t k) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int u = 0; u < CT; ++u) acc[u] = MF::op(a.v[v], b[u].v[v], acc[u]);
    if constexpr (SS != 0) {
      if (aval) {
        if constexpr (sizeof(T) == 4) {
          float q = a.v[0] * a.v[0];
          q = fmaf(a.v[1], a.v[1], q);
          q = fmaf(a.v[2], a.v[2], q);
          q = fmaf(a.v[3], a.v[3], q);
          ss += (double)q;
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) ss = fma((double)a.v[v], (double)a.v[v], ss);
        }
        if constexpr (SS == 2)
#pragma unroll
          for (int v = 0; v < 4; ++v) mx = fmaxf(mx, fabsf((float)a.v[v]));
      }
    }
    if constexpr (LPW != 0) {
      if (aval) {
        const int64_t kk = k + 4 * g;
        uint16_t* dst = lp_out + row * ld_lp + kk;
        if (kk + 3 < ke) {
          uint2 pk;
          pk.x = (uint32_t)to_lp_bits<LPW>((float)a.v[0] * lps) |
                 ((uint32_t)to_lp_bits<LPW>((float)a.v[1] * lps) << 16);
          pk.y = (uint32_t)to_lp_bits<LPW>((float)a.v[2] * lps) |
                 ((uint32_t)to_lp_bits<LPW>((float)a.v[3] * lps) << 16);
          *reinterpret_cast<uint2*>(dst) = pk;
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (kk + v < ke) dst[v] = to_lp_bits<LPW>((float)a.v[v] * lps);
        }
      }
    }
  };
  auto load = [&](V4<T>& a, V4<T>(&b)[CT], int64_t k) {
    a = ld4(ap + k);
#pragma unroll
    for (int u = 0; u < CT; ++u) b[u] = ld4(op + ((k >> 4) * CT + u) * 256);
  };
  const int64_t nfull = (ke - kb) / 16;
  if (nfull > 0) {
    // D-deep ring; chunk indices past the last full chunk are clamped to it
    // in the prologue (never used), so every load is unconditional and each
    // chunk waits only for its own loads
    V4<T> ab[D], bb[D][CT];
#pragma unroll
    for (int q = 0; q < D; ++q) load(ab[q], bb[q], kb + 16 * min((int64_t)q, nfull - 1));
    int64_t i = 0;
    for (; i + 2 * D <= nfull; i += D) {
#pragma unroll
      for (int q = 0; q < D; ++q) {
        compute(ab[q], bb[q], kb + 16 * (i + q));
        load(ab[q], bb[q], kb + 16 * (i + q + D));
      }
    }
#pragma unroll
    for (int q = 0; q < D; ++q) {
      if (i + q < nfull) {
        compute(ab[q], bb[q], kb + 16 * (i + q));
        if (i + q + D < nfull) load(ab[q], bb[q], kb + 16 * (i + q + D));
      }
    }
#pragma unroll
    for (int q = 0; q < D; ++q)
      if (i + D + q < nfull) compute(ab[q], bb[q], kb + 16 * (i + D + q));
  }
  if (kb + 16 * nfull < ke) {                 // ragged tail: masked loads, zero past ke
    const int64_t k = kb + 16 * nfull;
    V4<T> a = ld4_masked(ap + k, k + 4 * g, ke), b[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) b[u] = ld4_masked(op + ((k >> 4) * CT + u) * 256, k + 4 * g, ke);
    compute(a, b, k);
  }
  // fixed-order tree over the K parts: waves [h, 2h) hand their tiles to
  // waves [0, h) for h = NW/2, ..., 1
#pragma unroll
  for (int h = NW / 2; h >= 1; h >>= 1) {
    if (wv >= h && wv < 2 * h)
#pragma unroll
      for (int u = 0; u < CT; ++u) red[wv - h][u][lane] = acc[u];
    __syncthreads();
    if (wv < h)
#pragma unroll
      for (int u = 0; u < CT; ++u) acc[u] += red[wv][u][lane];
    __syncthreads();
  }
  if (wv == 0) {
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const int64_t col = 16 * u + r;
      if (col >= N) continue;
      if constexpr (MF::rows_contiguous) {
        const int64_t r0 = m0 + 4 * g;
        T* p = Y + col * ldy + r0;
        if (r0 + 3 < M && (ldy & 3) == 0) {
          *reinterpret_cast<f32x4*>(p) = acc[u];
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r0 + e < M) p[e] = acc[u][e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t rr = m0 + MF::row(g, e);
          if (rr < M) Y[col * ldy + rr] = acc[u][e];
        }
      }
    }
  }
  if constexpr (SS != 0) {
    for (int off = 32; off > 0; off >>= 1) {
      ss += __shfl_xor(ss, off);
      mx = fmaxf(mx, __shfl_xor(mx, off));
    }
    if (lane == 0) {
      ss_red[wv] = ss;
      mx_red[wv] = mx;
    }
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      float mt = 0.0f;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        t += ss_red[q];
        mt = fmaxf(mt, mx_red[q]);
      }
      sumsq[blockIdx.x] = t;
      if constexpr (SS == 2) maxabs[blockIdx.x] = mt;
    }
  }
}

// ---------------------------------------------------------------------------
// Low-precision sketch partials: out_s (M x N, N <= 16*CT) = (A_lp Omega_lp)
// / scale over K-split s, with A_lp the FP16 (LPT 1) or BF16 (LPT 2) copy of
// A (row-major, ld_lp, 16-bit patterns) and Omega_lp = Omega^T rounded the
// same way while it is staged in LDS; v_mfma_f32_16x16x16 f16 / bf16 with
// FP32 accumulation.  Workgroup = 4 waves x 32 rows; each lane loads 8
// consecutive K values of a row (16 bytes) per 32-wide K chunk and feeds
// them to two MFMAs (K offsets 8g..8g+3 and 8g+4..8g+7 of lane group g;
// Omega uses the same offsets, so the K sum is complete).  Partials as in
// k_sketch (column-major, out + s*part_stride + col*ldo + row).
// ---------------------------------------------------------------------------
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
template <int LPT>
__device__ __forceinline__ f32x4 mfma_lp(uint2 a, uint2 b, f32x4 c) {
  if constexpr (LPT == 1)
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b),
                                                c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                     __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
}

template <int CT>
struct SketchLpCfg {
  static constexpr int KS = CT <= 4 ? 512 : 256;   // K per LDS slab
  static constexpr int LDO = KS + 8;               // padded row of the staged Omega (16-bit)
};

template <int LPT, int CT>
__global__ __launch_bounds__(256) void k_sketch_lp(
    const uint16_t* __restrict__ A, int64_t ld_lp, const float* __restrict__ Om, int64_t ldk,
    int64_t M, int N, int64_t K, int64_t kchunk, float* __restrict__ out, int64_t ldo,
    int64_t part_stride, const State* __restrict__ lp_st, const int32_t* __restrict__ stop_block,
    int block_id) {
  constexpr int RT = 2, KS = SketchLpCfg<CT>::KS, LDO = SketchLpCfg<CT>::LDO, NC = 16 * CT;
  if (stop_block && *stop_block < block_id) return;
  __shared__ __align__(16) uint16_t oms[NC * LDO];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * (64 * RT) + wv * (16 * RT);
  const int s = blockIdx.y;
  const int64_t kb = (int64_t)s * kchunk, ke = min(K, kb + kchunk);
  const float inv_scale = (float)(1.0 / lp_st->lp_scale);
  const uint16_t* ap[RT];
  bool aval[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = m0 + 16 * t + r;
    aval[t] = row < M;
    ap[t] = A + (aval[t] ? row : (M - 1)) * ld_lp + 8 * g;
  }
  f32x4 acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool active = (m0 < M);
  for (int64_t sb = kb; sb < ke; sb += KS) {
    const int64_t se = min(ke, sb + KS);
    const int slen = (int)(se - sb);
    __syncthreads();
    // stage Omega^T[0:NC, sb:se] rounded to the low precision (zero beyond
    // se and N), a thread's loads all in flight before its LDS stores
    constexpr int NST = NC * (KS / 4) / 256, NB = batch_of(NST);
    static_assert(NC * (KS / 4) % 256 == 0 && NST % NB == 0, "staging split");
#pragma unroll
    for (int q0 = 0; q0 < NST; q0 += NB) {
      V4<float> sv[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int idx = tid + 256 * (q0 + q);
        const int c = idx / (KS / 4), k4 = (idx - c * (KS / 4)) * 4;
        const float* src = Om + (int64_t)(c < N ? c : 0) * ldk + sb + k4;
        if (c < N && k4 + 3 < slen) sv[q] = ld4(src);
        else if (c < N) sv[q] = ld4_masked(src, k4, slen);
        else
#pragma unroll
          for (int e = 0; e < 4; ++e) sv[q].v[e] = 0.f;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int idx = tid + 256 * (q0 + q);
        const int c = idx / (KS / 4), k4 = (idx - c * (KS / 4)) * 4;
        uint2 pk;
        pk.x = (uint32_t)to_lp_bits<LPT>(sv[q].v[0]) | ((uint32_t)to_lp_bits<LPT>(sv[q].v[1]) << 16);
        pk.y = (uint32_t)to_lp_bits<LPT>(sv[q].v[2]) | ((uint32_t)to_lp_bits<LPT>(sv[q].v[3]) << 16);
        *reinterpret_cast<uint2*>(&oms[c * LDO + k4]) = pk;
      }
    }
    __syncthreads();
    if (!active) continue;
    const int nfull = slen / 32;
    auto compute = [&](const uint4 (&a)[RT], int kl) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint2 b[CT];
#pragma unroll
        for (int u = 0; u < CT; ++u)
          b[u] = *reinterpret_cast<const uint2*>(&oms[(16 * u + r) * LDO + kl + 8 * g + 4 * h]);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const uint2 av = h == 0 ? uint2{a[t].x, a[t].y} : uint2{a[t].z, a[t].w};
#pragma unroll
          for (int u = 0; u < CT; ++u) acc[t][u] = mfma_lp<LPT>(av, b[u], acc[t][u]);
        }
      }
    };
    // 4-deep register pipeline over the full 32-K chunks of this slab
    uint4 a[4][RT];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nfull)
#pragma unroll
        for (int t = 0; t < RT; ++t) a[q][t] = *reinterpret_cast<const uint4*>(ap[t] + sb + 32 * q);
    for (int c = 0; c < nfull; c += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (c + q < nfull) {
          compute(a[q], 32 * (c + q));
          if (c + q + 4 < nfull)
#pragma unroll
            for (int t = 0; t < RT; ++t)
              a[q][t] = *reinterpret_cast<const uint4*>(ap[t] + sb + 32 * (c + q + 4));
        }
      }
    }
    if (nfull * 32 < slen) {                  // ragged tail: element loads, zero beyond se
      uint4 at[RT];
      const int64_t k = sb + 32 * nfull + 8 * g;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (k + e < se) ? ap[t][k - 8 * g + e] : (uint16_t)0;
        at[t].x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        at[t].y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
        at[t].z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
        at[t].w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
      }
      compute(at, 32 * nfull);
    }
  }
  if (!active) return;
  float* o = out + (int64_t)s * part_stride;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const int64_t col = 16 * u + r;
      if (col >= N) continue;
      const int64_t row = m0 + 16 * t + 4 * g;
      float* p = o + col * ldo + row;
      if (row + 3 < M && ((ldo & 3) == 0) && ((part_stride & 3) == 0)) {
        *reinterpret_cast<f32x4*>(p) = acc[t][u] * inv_scale;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (row + e < M) p[e] = acc[t][u][e] * inv_scale;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// NN GEMM partials: out_s(M x N) = X(M x K) * Z(K x N) over K-split s, with X
// row-major K-contiguous (ldx) and Z row-major N-contiguous (ldz).  Used for
// C = Q^T A (X = Q^T, i.e. Q column-major; Z = A).  out_s row-major
// (element (m, j) at s*part_stride + m*ldo + j).
// Lane l loads rows k0+4g+v (v = 0..3) of Z at columns j0+4r .. 4r+3, so a
// wave covers a 16-row step x 64 columns with dwordx4 loads; MFMA tile u
// (0..3) holds columns j0 + 4j + u.  Each wave computes 16*RT rows of out
// and keeps PF of its steps in flight in registers.  Workgroup = 4 waves =
// 4 consecutive 64-column panels.  Grid: x = K split, y = 256-column panel,
// z = 16*RT-row tile of out.  Workgroups are dealt to the XCDs round-robin
// by linear index, so with the split in x an XCD streams whole row ranges of
// Z (all panels of rows kb..ke) rather than the same column stripe of every
// row; on the 4096^2 projection this takes the kernel from 18.2 to 14.6 us.
// ---------------------------------------------------------------------------
template <typename T, int RT>
struct NnCfg {
  static constexpr int PF = sizeof(T) == 4 ? (RT <= 2 ? 4 : 3) : (RT <= 2 ? 3 : 2);
};

template <typename T, int RT>
__global__ __launch_bounds__(256) void k_gemm_nn(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ Z, int64_t ldz,
    int64_t M, int64_t N, int64_t K, int64_t kchunk, T* __restrict__ out, int64_t ldo,
    int64_t part_stride, Gate gate, const int64_t* __restrict__ M_dev) {
  typedef Mfma<T> MF;
  constexpr int PF = NnCfg<T, RT>::PF;
  if (gate_shut(gate)) return;
  if (M_dev) M = *M_dev;                // row count known on the device only
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t j0 = ((int64_t)blockIdx.y * 4 + wv) * 64;
  const int64_t m0 = (int64_t)blockIdx.z * (16 * RT);
  const int s = blockIdx.x;
  const int64_t kb = (int64_t)s * kchunk, ke = min(K, kb + kchunk);
  if (j0 >= N || kb >= ke || m0 >= M) return;
  const int64_t jc = j0 + 4 * r;                       // first of this lane's 4 columns
  const bool jvec = (jc + 3 < N);
  const T* xp[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = m0 + 16 * t + r;
    xp[t] = X + (row < M ? row : (M - 1)) * ldx + 4 * g;
  }
  typename MF::acc_t acc[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = MF::zero();
  // one 16-row step at k: X chunk (masked past ke) and Z rows k+4g+v
  auto load = [&](V4<T>(&a)[RT], V4<T>(&zv)[4], int64_t k) {
    const bool full = (k + 16 <= ke);
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t] = full ? ld4(xp[t] + k) : ld4_masked(xp[t] + k, k + 4 * g, ke);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t kr = k + 4 * g + v;
      if (kr < ke && jvec) {
        zv[v] = ld4(Z + kr * ldz + jc);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) zv[v].v[u] = (kr < ke && jc + u < N) ? Z[kr * ldz + jc + u] : (T)0;
      }
    }
  };
  auto mma = [&](const V4<T>(&a)[RT], const V4<T>(&zv)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = MF::op(a[t].v[v], zv[v].v[u], acc[t][u]);
  };
  // one full step at k, no branches: in a panel that ends inside the
  // matrix (N a multiple of 4, so a lane's four columns are all in or all
  // out) the lanes past N read the panel's first columns and zero them by a
  // select
  const int64_t jl = jvec ? jc : j0;
  auto loadf = [&](V4<T>(&a)[RT], V4<T>(&zv)[4], int64_t k) {
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t] = ld4(xp[t] + k);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const V4<T> x = ld4(Z + (k + 4 * g + v) * ldz + jl);
#pragma unroll
      for (int u = 0; u < 4; ++u) zv[v].v[u] = jvec ? x.v[u] : (T)0;
    }
  };
  const int64_t nfull = (ke - kb) / 16;
  if ((j0 + 64 <= N || (N & 3) == 0) && nfull > 0) {
    // PF-deep ring over the full steps; the steady state has no branches,
    // so each step waits only for its own loads (step indices past the last
    // full step are clamped to it in the prologue and never used)
    V4<T> ab[PF][RT], zb[PF][4];
#pragma unroll
    for (int q = 0; q < PF; ++q) loadf(ab[q], zb[q], kb + 16 * min((int64_t)q, nfull - 1));
    int64_t i = 0;
    for (; i + 2 * PF <= nfull; i += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        mma(ab[q], zb[q]);
        loadf(ab[q], zb[q], kb + 16 * (i + q + PF));
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      if (i + q < nfull) {
        mma(ab[q], zb[q]);
        if (i + q + PF < nfull) loadf(ab[q], zb[q], kb + 16 * (i + q + PF));
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (i + PF + q < nfull) mma(ab[q], zb[q]);
    if (kb + 16 * nfull < ke) {               // ragged last step
      V4<T> a1[RT], z1[4];
      load(a1, z1, kb + 16 * nfull);
      mma(a1, z1);
    }
  } else {
    // a partial panel of a matrix whose width is not a multiple of 4 (or no
    // full step): one masked step at a time
    for (int64_t k = kb; k < ke; k += 16) {
      V4<T> a1[RT], z1[4];
      load(a1, z1, k);
      mma(a1, z1);
    }
  }
  T* o = out + (int64_t)s * part_stride;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = m0 + 16 * t + MF::row(g, e);
      if (row >= M) continue;
      T* p = o + row * ldo + jc;
      if (jvec && ((ldo & 3) == 0)) {
        if constexpr (sizeof(T) == 4) {
          *reinterpret_cast<f32x4*>(p) = f32x4{acc[t][0][e], acc[t][1][e], acc[t][2][e], acc[t][3][e]};
        } else {
          reinterpret_cast<double2*>(p)[0] = double2{acc[t][0][e], acc[t][1][e]};
          reinterpret_cast<double2*>(p)[1] = double2{acc[t][2][e], acc[t][3][e]};
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (jc + u < N) p[u] = acc[t][u][e];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Low-precision NN GEMM partials: out_s (M x N, FP32) = (X_lp Z_lp) / scale
// over K-split s, with Z the FP16 (LPT 1) or BF16 (LPT 2) copy of A
// (row-major 16-bit patterns, ldz, scaled by lp_st->lp_scale) and X FP32
// (row-major K-contiguous: Q^T with Q column-major) rounded to the same
// format as it is loaded; v_mfma_f32_16x16x16 f16 / bf16, FP32 accumulation.
// The lane layout is k_gemm_nn's: lane (r, g) loads rows k+4g+v (v = 0..3)
// of Z at columns j0+4r .. j0+4r+3 (8 bytes each) and the four K values
// 4g .. 4g+3 of its X rows, so one MFMA covers a 16-row step; the B operand
// of tile u is element u of the four Z rows.  Used for the first product
// A^T Q of the low-precision form's subspace iterations.
// ---------------------------------------------------------------------------
template <int LPT, int RT>
__global__ __launch_bounds__(256) void k_gemm_nn_lp(
    const float* __restrict__ X, int64_t ldx, const uint16_t* __restrict__ Z, int64_t ldz, int64_t M,
    int64_t N, int64_t K, int64_t kchunk, float* __restrict__ out, int64_t ldo, int64_t part_stride,
    const State* __restrict__ lp_st) {
  constexpr int PF = 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t j0 = ((int64_t)blockIdx.y * 4 + wv) * 64;
  const int64_t m0 = (int64_t)blockIdx.z * (16 * RT);
  const int s = blockIdx.x;
  const int64_t kb = (int64_t)s * kchunk, ke = min(K, kb + kchunk);
  if (j0 >= N || kb >= ke || m0 >= M) return;
  const float inv_scale = (float)(1.0 / lp_st->lp_scale);
  const int64_t jc = j0 + 4 * r;
  const bool jvec = (jc + 3 < N);
  const float* xp[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = m0 + 16 * t + r;
    xp[t] = X + (row < M ? row : (M - 1)) * ldx + 4 * g;
  }
  f32x4 acc[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  // X chunk of a step rounded to the low precision: 4 K values -> uint2
  auto pack_x = [&](const V4<float>& a) {
    uint2 pk;
    pk.x = (uint32_t)to_lp_bits<LPT>(a.v[0]) | ((uint32_t)to_lp_bits<LPT>(a.v[1]) << 16);
    pk.y = (uint32_t)to_lp_bits<LPT>(a.v[2]) | ((uint32_t)to_lp_bits<LPT>(a.v[3]) << 16);
    return pk;
  };
  // B operand of tile u: element u of the four Z rows (16-bit each)
  auto mma = [&](const V4<float>(&a)[RT], const uint2 (&zv)[4]) {
    uint2 xb[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) xb[t] = pack_x(a[t]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int sh = (u & 1) * 16;
      uint32_t e[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) e[v] = (((u < 2) ? zv[v].x : zv[v].y) >> sh) & 0xffffu;
      const uint2 b = uint2{e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
#pragma unroll
      for (int t = 0; t < RT; ++t) acc[t][u] = mfma_lp<LPT>(xb[t], b, acc[t][u]);
    }
  };
  // one 16-row step at k, masked (rows past ke, columns past N read as 0)
  auto load = [&](V4<float>(&a)[RT], uint2 (&zv)[4], int64_t k) {
    const bool full = (k + 16 <= ke);
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t] = full ? ld4(xp[t] + k) : ld4_masked(xp[t] + k, k + 4 * g, ke);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t kr = k + 4 * g + v;
      if (kr < ke && jvec) {
        zv[v] = *reinterpret_cast<const uint2*>(Z + kr * ldz + jc);
      } else {
        uint32_t h[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) h[u] = (kr < ke && jc + u < N) ? (uint32_t)Z[kr * ldz + jc + u] : 0u;
        zv[v] = uint2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
      }
    }
  };
  // one full step in a full panel: no masks
  auto loadf = [&](V4<float>(&a)[RT], uint2 (&zv)[4], int64_t k) {
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t] = ld4(xp[t] + k);
#pragma unroll
    for (int v = 0; v < 4; ++v) zv[v] = *reinterpret_cast<const uint2*>(Z + (k + 4 * g + v) * ldz + jc);
  };
  const int64_t nfull = (ke - kb) / 16;
  if (j0 + 64 <= N && nfull > 0) {
    // PF-deep ring, branch-free steady state (prologue indices clamped)
    V4<float> ab[PF][RT];
    uint2 zb[PF][4];
#pragma unroll
    for (int q = 0; q < PF; ++q) loadf(ab[q], zb[q], kb + 16 * min((int64_t)q, nfull - 1));
    int64_t i = 0;
    for (; i + 2 * PF <= nfull; i += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        mma(ab[q], zb[q]);
        loadf(ab[q], zb[q], kb + 16 * (i + q + PF));
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      if (i + q < nfull) {
        mma(ab[q], zb[q]);
        if (i + q + PF < nfull) loadf(ab[q], zb[q], kb + 16 * (i + q + PF));
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (i + PF + q < nfull) mma(ab[q], zb[q]);
    if (kb + 16 * nfull < ke) {
      V4<float> a1[RT];
      uint2 z1[4];
      load(a1, z1, kb + 16 * nfull);
      mma(a1, z1);
    }
  } else {
    for (int64_t k = kb; k < ke; k += 16) {
      V4<float> a1[RT];
      uint2 z1[4];
      load(a1, z1, k);
      mma(a1, z1);
    }
  }
  float* o = out + (int64_t)s * part_stride;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = m0 + 16 * t + 4 * g + e;
      if (row >= M) continue;
      float* p = o + row * ldo + jc;
      if (jvec && ((ldo & 3) == 0)) {
        *reinterpret_cast<f32x4*>(p) = f32x4{acc[t][0][e], acc[t][1][e], acc[t][2][e], acc[t][3][e]} * inv_scale;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (jc + u < N) p[u] = acc[t][u][e] * inv_scale;
      }
    }
  }
}

// out[i] = sum_s parts[s*stride + i] (fixed order), i < count.  Optional
// block control as in k_gemm_nt.
template <typename T>
__global__ void k_reduce_parts(const T* __restrict__ parts, int nparts, int64_t stride,
                               int64_t count, T* __restrict__ out,
                               const int32_t* __restrict__ stop_block, int block_id, Gate gate) {
  if (stop_block && *stop_block < block_id) return;
  if (gate_shut(gate)) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    T acc = parts[i];
    for (int s = 1; s < nparts; ++s) acc += parts[(int64_t)s * stride + i];
    out[i] = acc;
  }
}

// out[i] = sum_s parts[s*stride + i] for many partials, deterministic.
// P threads share a group of four consecutive elements: thread p sums the
// partials s = p, p + P, p + 2P, ... in that order, up to 16 loads in
// flight, and the P sums are added in the order p = 0, 1, ..., P-1 through
// LDS (P = 1: the plain order s = 0, 1, ...).  P > 1 serves many partials
// over few elements, where a thread per group would need one memory round
// trip per 16 partials.  The vector path needs stride a multiple of 4 and
// 16-byte aligned parts and out, else a thread folds its elements one at a
// time.  128-thread workgroups, count / (512 / P) of them.
template <typename T, int P>
__global__ __launch_bounds__(128) void k_fold_parts(const T* __restrict__ parts, int nparts, int64_t stride,
                                                    int64_t count, T* __restrict__ out,
                                                    const int32_t* __restrict__ stop_block, int block_id,
                                                    Gate gate) {
  static_assert(P >= 1 && P <= 16 && (P & (P - 1)) == 0, "P: power of two up to 16");
  if (stop_block && *stop_block < block_id) return;
  if (gate_shut(gate)) return;
  __shared__ T red[P > 1 ? 128 * 4 : 1];
  const int p = threadIdx.x % P, grp = threadIdx.x / P;
  const int64_t i0 = ((int64_t)blockIdx.x * (128 / P) + grp) * 4;
  const bool live = i0 < count;
  const bool vec = i0 + 3 < count && (stride & 3) == 0 && (((uintptr_t)parts | (uintptr_t)out) & 15) == 0;
  V4<T> acc;
#pragma unroll
  for (int e = 0; e < 4; ++e) acc.v[e] = (T)0;
  if (live && vec) {
    constexpr int NB = 16;
    for (int s0 = p; s0 < nparts; s0 += NB * P) {
      V4<T> v[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int sq = min(s0 + q * P, nparts - 1);  // clamped: the load stays unconditional
        v[q] = ld4(parts + (int64_t)sq * stride + i0);
      }
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (s0 + q * P < nparts)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc.v[e] += v[q].v[e];
    }
  } else if (live) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < count)
        for (int s = p; s < nparts; s += P) acc.v[e] += parts[(int64_t)s * stride + i0 + e];
  }
  if constexpr (P > 1) {
#pragma unroll
    for (int e = 0; e < 4; ++e) red[threadIdx.x * 4 + e] = acc.v[e];
    __syncthreads();
    if (p != 0) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      T a = (T)0;
      for (int q = 0; q < P; ++q) a += red[(threadIdx.x + q) * 4 + e];
      acc.v[e] = a;
    }
  }
  if (!live) return;
  if (vec) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<f32x4*>(out + i0) = f32x4{acc.v[0], acc.v[1], acc.v[2], acc.v[3]};
    } else {
      reinterpret_cast<double2*>(out + i0)[0] = double2{acc.v[0], acc.v[1]};
      reinterpret_cast<double2*>(out + i0)[1] = double2{acc.v[2], acc.v[3]};
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < count) out[i0 + e] = acc.v[e];
  }
}

// Column-block reduction for a column-major matrix with leading dimension ld
// where only rows < rows_dev (read from wlog[block_id] when given) matter:
// out(i, c) = sum_s parts_s(i, c), i < rows, c < cols.
template <typename T>
__global__ void k_reduce_cols(const T* __restrict__ parts, int nparts, int64_t stride,
                              int64_t rows, int64_t cols, int64_t ld, T* __restrict__ out,
                              const int64_t* __restrict__ wlog, const int32_t* __restrict__ stop_block,
                              int block_id) {
  if (stop_block && *stop_block < block_id) return;
  if (wlog) rows = wlog[block_id];
  const int64_t total = rows * cols;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / rows, i = idx - c * rows;
    const int64_t off = c * ld + i;
    T acc = parts[off];
    for (int s = 1; s < nparts; ++s) acc += parts[(int64_t)s * stride + off];
    out[off] = acc;
  }
}

// ---------------------------------------------------------------------------
// Y (m x f) -= Q (m x w) W (w x f), or Y = Q W without subtract (Y, Q
// column-major; W column-major ldw).  On MFMA: FP32 operands and
// accumulation when TW is float, FP64 (f64 MFMA) when TW is double.  A
// workgroup takes 64 rows and 64 columns of Y (wave: 16 rows x 4 column
// tiles); W is staged in LDS 64 rows at a time and each wave issues all 16
// Q loads of a chunk before its MFMAs.  w from wlog when given.
// ---------------------------------------------------------------------------
template <typename T, typename TW>
__global__ __launch_bounds__(256) void k_update_rows(
    T* __restrict__ Y, int64_t ldy, const T* __restrict__ Q, int64_t ldq, int64_t m, int64_t w,
    int f, const TW* __restrict__ W, int64_t ldw, int subtract,
    const int64_t* __restrict__ wlog, const int32_t* __restrict__ stop_block, int block_id) {
  typedef Mfma<TW> MF;
  constexpr int LDS_W = 64 + (sizeof(TW) == 8 ? 1 : 4);
  if (stop_block && *stop_block < block_id) return;
  if (wlog) w = wlog[block_id];
  if (w == 0 && subtract) return;
  __shared__ TW Ws[64 * LDS_W];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * wv;
  const int c0 = blockIdx.y * 64;
  const int fc = (int)min((int64_t)64, (int64_t)f - c0);
  const int64_t arow = row0 + r;
  const bool aok = arow < m;
  typename MF::acc_t acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = MF::zero();
  for (int64_t a0 = 0; a0 < w; a0 += 64) {
    const int na = (int)min((int64_t)64, w - a0);
    // this wave's Q operands for the chunk (row arow, columns a0 + 4kk + g)
    TW qa[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + g;
      qa[kk] = (aok && k < na) ? (TW)Q[(a0 + k) * ldq + arow] : (TW)0;
    }
    __syncthreads();
    for (int idx = tid; idx < 64 * 64; idx += 256) {
      const int k = idx >> 6, c = idx & 63;
      Ws[k * LDS_W + c] = (k < na && c < fc) ? W[(int64_t)(c0 + c) * ldw + a0 + k] : (TW)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = MF::op(qa[kk], Ws[(4 * kk + g) * LDS_W + 16 * u + r], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = 16 * u + r;
    if (c >= fc) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = row0 + MF::row(g, e);
      if (row < m) {
        T* p = Y + (int64_t)(c0 + c) * ldy + row;
        *p = subtract ? (T)((TW)*p - acc[u][e]) : (T)acc[u][e];
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Y (m x f, column-major ldy) -= Q W (or = Q W when subtract is 0) for the
// block re-orthogonalisation: Q m x w column-major (ldq), W w x f with
// element (a, c) at c*ldw + a, same type as Y; w read on the device from
// wlog[block_id] when given.  One workgroup per 16-row tile and 16*CT
// columns; its NW waves split the w products (K) and hand their partial
// tiles down a fixed tree in LDS, wave 0 updates Y.  Lane (r, g) reads Q at
// row r of the tile and W at column 16u + r, K index 4i + g, straight from
// memory (both small and L2-resident here), two 16-K steps in flight.
// ---------------------------------------------------------------------------
template <typename T, int CT, int NW>
__global__ __launch_bounds__(64 * NW) void k_update_tiles(
    T* __restrict__ Y, int64_t ldy, const T* __restrict__ Q, int64_t ldq, int64_t m, int64_t w, int f,
    const T* __restrict__ W, int64_t ldw, int subtract, const int64_t* __restrict__ wlog,
    const int32_t* __restrict__ stop_block, int block_id) {
  typedef Mfma<T> MF;
  typedef typename MF::acc_t acc_t;
  static_assert(NW >= 2 && (NW & (NW - 1)) == 0, "NW: power of two");
  if (stop_block && *stop_block < block_id) return;
  if (wlog) w = wlog[block_id];
  if (w == 0 && subtract) return;
  __shared__ acc_t red[NW / 2][CT][64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 16;
  const int c0 = blockIdx.y * 16 * CT;
  const int64_t row = row0 + r;
  const bool rok = row < m;
  const int64_t kc = ((w + NW - 1) / NW + 15) / 16 * 16;
  const int64_t kb = min(w, (int64_t)wv * kc), ke = min(w, kb + kc);
  const T* qp = Q + (rok ? row : 0) + g * ldq;            // + k * ldq
  const T* wp[CT];
  bool cok[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) {
    const int c = c0 + 16 * u + r;
    cok[u] = c < f;
    wp[u] = W + (int64_t)(cok[u] ? c : 0) * ldw + g;       // + k
  }
  acc_t acc[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) acc[u] = MF::zero();
  // a 16-K step at k: four K values per lane (4i + g), masked past ke
  auto load = [&](T (&a)[4], T (&b)[4][CT], int64_t k) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t kk = k + 4 * i;
      const bool kok = kk + g < ke;
      a[i] = (kok && rok) ? qp[kk * ldq] : (T)0;
#pragma unroll
      for (int u = 0; u < CT; ++u) b[i][u] = (kok && cok[u]) ? wp[u][kk] : (T)0;
    }
  };
  auto mma = [&](const T (&a)[4], const T (&b)[4][CT]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < CT; ++u) acc[u] = MF::op(a[i], b[i][u], acc[u]);
  };
  if (kb < ke) {
    T a0[4], b0[4][CT], a1[4], b1[4][CT];
    load(a0, b0, kb);
    int64_t k = kb;
    for (; k + 16 < ke; k += 32) {
      load(a1, b1, k + 16);
      mma(a0, b0);
      if (k + 32 < ke) load(a0, b0, k + 32);
      mma(a1, b1);
    }
    if (k < ke) mma(a0, b0);
  }
#pragma unroll
  for (int h = NW / 2; h >= 1; h >>= 1) {
    if (wv >= h && wv < 2 * h)
#pragma unroll
      for (int u = 0; u < CT; ++u) red[wv - h][u][lane] = acc[u];
    __syncthreads();
    if (wv < h)
#pragma unroll
      for (int u = 0; u < CT; ++u) acc[u] += red[wv][u][lane];
    __syncthreads();
  }
  if (wv != 0) return;
#pragma unroll
  for (int u = 0; u < CT; ++u) {
    if (!cok[u]) continue;
    T* py = Y + (int64_t)(c0 + 16 * u + r) * ldy;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t rr = row0 + MF::row(g, e);
      if (rr < m) py[rr] = subtract ? py[rr] - acc[u][e] : acc[u][e];
    }
  }
}

// ---------------------------------------------------------------------------
// Small FP64 matrices (f <= F <= 64, F in {16, 32, 64}) are kept in LDS
// row-major with leading dimension F + 1 (the odd stride spreads a column
// over the banks).
// ---------------------------------------------------------------------------
template <int F>
struct SmallCfg {
  static constexpr int LD = F + 1;
  static constexpr int SIZE = F * (F + 1);        // doubles per matrix
  static constexpr int NR = F / 4;                // elimination: rows held per wave
  static constexpr int NCL = (2 * F + 63) / 64;   // elimination: columns of [G | I] per lane
};

// Up to two f x f FP64 matrices src[h] (element (i, j) at j*ld_src + i,
// ld_src = f unless given) into LDS as dst[h][i*ld + j], zero outside f x f
// (f <= F <= 64, 256 threads); a thread's loads are all in flight before its
// first LDS store, so the staging costs one memory round trip.
template <int F, int NM = 1>
__device__ __forceinline__ void stage_small(const double* const (&src)[NM], int f, double* const (&dst)[NM],
                                            int ld, int ld_src = 0) {
  static_assert(F <= 64, "register budget");
  constexpr int NQ = (F * F + 255) / 256;
  const int64_t lsrc = ld_src > 0 ? ld_src : f;   // source leading dimension (f when packed)
  double v[NM][NQ];
#pragma unroll
  for (int h = 0; h < NM; ++h)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = threadIdx.x + 256 * q;
      const int jj = idx / F, i = idx - jj * F;
      v[h][q] = (idx < F * F && i < f && jj < f) ? src[h][(int64_t)jj * lsrc + i] : 0.0;
    }
#pragma unroll
  for (int h = 0; h < NM; ++h)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = threadIdx.x + 256 * q;
      const int jj = idx / F, i = idx - jj * F;
      if (idx < F * F) dst[h][i * ld + jj] = v[h][q];
    }
}

// C = op(A) op(B) for F x F FP64 matrices in LDS on the four waves of the
// workgroup (v_mfma_f64_16x16x4, one 16 x 16 tile per wave at a time);
// element (i, j) of the product is handed to out(i, j, v).
template <int F, bool TA, bool TB, typename Out>
__device__ __forceinline__ void lds_gemm(const double* A, const double* B, Out out) {
  typedef Mfma<double> MF;
  constexpr int TT = F / 16, LD = F + 1;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  for (int tile = wv; tile < TT * TT; tile += 4) {
    const int ti = tile / TT, tj = tile - ti * TT;
    const int ar = 16 * ti + r, bc = 16 * tj + r;
    typename MF::acc_t acc = MF::zero();
#pragma unroll 4
    for (int k0 = 0; k0 < F; k0 += 4) {
      const int kk = k0 + g;
      const double a = TA ? A[kk * LD + ar] : A[ar * LD + kk];
      const double b = TB ? B[bc * LD + kk] : B[kk * LD + bc];
      acc = MF::op(a, b, acc);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) out(16 * ti + MF::row(g, e), bc, acc[e]);
  }
}

// ---------------------------------------------------------------------------
// Cholesky with inverse, on the four waves of a workgroup, of a symmetric
// positive semi-definite f x f matrix G (FP64, f <= F): elimination over
// the augmented rows [G | I].  With G = L U (L unit lower, U = diag(alpha)
// R) the elimination turns I into L^{-1} = diag(alpha) R^{-T}, so row k of
// the right half divided by alpha_k is column k of R^{-1}.  Pivot rules:
//   dead column (flag in dmask_in): R(k,k) = 1, row k and column k of R
//     zero, no elimination;
//   p <= FLOOR_C u64 G(k,k), p <= PIV_MIN or not finite: floored to
//     FLOOR_C u64 G(k,k) on a first pass (R(k,k) = sqrt(floor), rest of row
//     k zero, no elimination) and marked dead otherwise (R(k,k) = 1);
//   else R(k,k) = sqrt(p), R(k,c) = S(k,c)/R(k,k) for live c > k and every
//     later row i subtracts S(k,i)/p times row k (dead columns excluded),
// with p = S(k,k) of the current Schur complement S.
// Blocked by panels of 8 pivots (the same arithmetic, reordered): the 8
// panel rows are published in LDS; every thread factors the 8 x 8 diagonal
// block in registers (pivot rules above) and applies the panel's unit lower
// factor to the columns it owns, which gives the panel rows of R (S part)
// and of R^{-T} (right half); the rows below take the rank-8 update
// S(i,:) -= sum_j R(k_j,i) X(j,:).  Two barriers per panel.
// Layout: lane c owns column c of [G | I] (two columns per lane when
// F = 64); wave w holds rows 8(p + s/2) + 4(s%2) + w in slot s during panel
// p (slots move down by two after each panel).
// Gs: G on entry (row-major, ld F+1), R on exit (zero below the diagonal
// and in rows >= f); Ri: R^{-1} on exit (zero in columns >= f); work:
// 24F doubles; dgs: F doubles.  Returns the dead mask afterwards and the
// number of floored pivots (uniform over the workgroup).  dg_in (optional):
// the diagonal the floor rule refers to (G's own diagonal when null; the
// trailing block of a blocked factorization passes the original one).
// nolive_out (optional): bits of the pivots that did not eliminate (dead or
// floored).
// ---------------------------------------------------------------------------
template <int F>
__device__ void chol_inv(double* Gs, double* Ri, double* work, double* dgs, int f,
                         uint64_t dmask_in, int first_pass, uint64_t* dmask_out, int* nfloor,
                         const double* dg_in = nullptr, uint64_t* nolive_out = nullptr) {
  typedef SmallCfg<F> C;
  constexpr int LD = C::LD, NR = C::NR, NCL = C::NCL, W2 = 2 * F;
  double* P = work;                      // panel rows: P[j*W2 + c], j < 8
  double* XT = work + 8 * W2;            // multipliers: XT[j*F + i] = R(kp+j, i)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index (scalar)
  for (int i = tid; i < f; i += 256) dgs[i] = dg_in ? dg_in[i] : Gs[i * LD + i];
  double M[NR][NCL];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = 8 * (s / 2) + 4 * (s % 2) + w;
#pragma unroll
    for (int q = 0; q < NCL; ++q) {
      const int c = lane + 64 * q;
      double v = 0.0;
      if (i < f && c < W2) {
        if (c < F) v = c < f ? Gs[i * LD + c] : 0.0;
        else v = (c - F == i) ? 1.0 : 0.0;
      }
      M[s][q] = v;
    }
  }
  __syncthreads();                       // G consumed: Gs now receives R; dgs ready
  uint64_t dout = dmask_in, nlive = 0;
  int nfl = 0;
  for (int kp = 0; kp < f; kp += 8) {
    // (a) publish the panel rows kp + w and kp + 4 + w
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < NCL; ++q) {
        const int c = lane + 64 * q;
        if (c < W2) P[(4 * h + w) * W2 + c] = M[h][q];
      }
    __syncthreads();
    // (b) 8 x 8 diagonal block in registers: R_loc (upper triangle of d).
    // Fast path when no panel pivot is dead or padding and every pivot
    // passes the floor test; otherwise the block is reloaded and factored
    // with the full pivot rules.
    double d[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = i; j < 8; ++j) d[i][j] = P[i * W2 + kp + j];
    double yv[NCL][8];
#pragma unroll
    for (int q = 0; q < NCL; ++q) {
      const int c = lane + 64 * q;
#pragma unroll
      for (int j = 0; j < 8; ++j) yv[q][j] = P[j * W2 + (c < W2 ? c : 0)];
    }
    double dgk[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dgk[j] = dgs[kp + j];
    double alpha[8], ia[8];
    bool okj[8];
    bool fast = kp + 8 <= f && ((dmask_in >> kp) & 0xffull) == 0;
    if (fast) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double piv = d[j][j];
        const bool ok = piv > FLOOR_C * U64 * dgk[j] && piv > PIV_MIN && piv < INFINITY;
        fast = fast && ok;
        // 1/sqrt(p): hardware estimate and two Newton steps (about 1 ulp)
        double y = __builtin_amdgcn_rsq(piv);
        y = y * fma(-0.5 * piv, y * y, 1.5);
        y = y * fma(-0.5 * piv, y * y, 1.5);
        alpha[j] = piv * y;
        ia[j] = y;
        okj[j] = true;
#pragma unroll
        for (int i = j + 1; i < 8; ++i) d[j][i] *= y;
#pragma unroll
        for (int i = j + 1; i < 8; ++i)
#pragma unroll
          for (int i2 = i; i2 < 8; ++i2) d[i][i2] = fma(-d[j][i], d[j][i2], d[i][i2]);
      }
    }
    if (!fast) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = i; j < 8; ++j) d[i][j] = P[i * W2 + kp + j];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kp + j;
        const bool valid = k < f;
        const double piv = d[j][j];
        const double flo = FLOOR_C * U64 * dgk[j];
        int fl;
        double a, y;
        if (!valid) {
          fl = 3;
          a = 1.0;
          y = 1.0;
        } else if ((dmask_in >> k) & 1ull) {
          fl = 2;
          a = 1.0;
          y = 1.0;
        } else if (!(piv > flo) || !(piv > PIV_MIN) || !(piv < INFINITY)) {
          fl = first_pass ? 1 : 2;
          a = first_pass ? sqrt(flo > 1e-300 ? flo : 1e-300) : 1.0;
          y = 1.0 / a;
        } else {
          fl = 0;
          y = __builtin_amdgcn_rsq(piv);
          y = y * fma(-0.5 * piv, y * y, 1.5);
          y = y * fma(-0.5 * piv, y * y, 1.5);
          a = piv * y;
        }
        if (fl == 2) dout |= 1ull << k;
        if (fl == 1 || fl == 2) nlive |= 1ull << k;
        nfl += (fl == 1);
        alpha[j] = a;
        ia[j] = y;
        okj[j] = (fl == 0);
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
          const bool live = okj[j] && kp + i < f && !((dmask_in >> (kp + i)) & 1ull);
          d[j][i] = live ? d[j][i] * y : 0.0;        // R_loc(j, i)
        }
#pragma unroll
        for (int i = j + 1; i < 8; ++i)
#pragma unroll
          for (int i2 = i; i2 < 8; ++i2) d[i][i2] = fma(-d[j][i], d[j][i2], d[i][i2]);
      }
    }
    // own columns: z_j = (v_j - sum_{i<j} R_loc(i,j) z_i) / alpha_j, i.e. the
    // panel rows after the panel's elimination, scaled; X = z with the S part
    // masked (R(k_j, c) = 0 for a dead column c or a pivot that did not
    // eliminate)
    double X[NCL][8];
#pragma unroll
    for (int q = 0; q < NCL; ++q) {
      const int c = lane + 64 * q;
      const bool sdead = c < F && ((dmask_in >> (c < F ? c : 0)) & 1ull);
      double z[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        double acc = yv[q][j];
#pragma unroll
        for (int i = 0; i < j; ++i) acc = fma(-d[i][j], z[i], acc);
        z[j] = acc * ia[j];
        X[q][j] = (c < F && (!okj[j] || sdead)) ? 0.0 : z[j];
      }
    }
    // panel rows of R, columns of R^{-1}, multipliers: rows 2w and 2w+1 by wave w
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kp + j;
      if ((j >> 1) != w || k >= f) continue;
#pragma unroll
      for (int q = 0; q < NCL; ++q) {
        const int c = lane + 64 * q;
        if (c >= W2) continue;
        if (c < F) {
          Gs[k * LD + c] = (c == k) ? alpha[j] : (c > k ? X[q][j] : 0.0);
          XT[j * F + c] = X[q][j];
        } else {
          const int cc = c - F;
          Ri[cc * LD + k] = cc <= k ? X[q][j] : 0.0;
        }
      }
    }
    __syncthreads();
    // (c) rank-8 update of the rows below the panel
#pragma unroll
    for (int s = 2; s < NR; ++s) {
      const int i = kp + 8 * (s / 2) + 4 * (s % 2) + w;
      if (i >= f) continue;
      double mj[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) mj[j] = XT[j * F + i];
#pragma unroll
      for (int q = 0; q < NCL; ++q)
#pragma unroll
        for (int j = 0; j < 8; ++j) M[s][q] = fma(-mj[j], X[q][j], M[s][q]);
    }
#pragma unroll
    for (int s = 0; s + 2 < NR; ++s)
#pragma unroll
      for (int q = 0; q < NCL; ++q) M[s][q] = M[s + 2][q];
#pragma unroll
    for (int q = 0; q < NCL; ++q) {
      M[NR - 2][q] = 0.0;
      M[NR - 1][q] = 0.0;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < (F - f) * F; idx += 256) {   // padding rows / columns
    const int a = f + idx / F, b = idx - (idx / F) * F;
    Gs[a * LD + b] = 0.0;
    Ri[b * LD + a] = 0.0;
  }
  __syncthreads();
  *dmask_out = dout;
  *nfloor = nfl;
  if (nolive_out) *nolive_out = nlive;
}


// ---------------------------------------------------------------------------
// chol_inv for the common case, f <= F <= 32: no dead column and every
// pivot above the floor.  The rows and columns past f are padded by the
// identity, so every 8-pivot panel is whole and the elimination runs fully
// without a branch in its panels; the arithmetic on rows and columns < f is that
// of chol_inv's fast panels (the same operations in the same order), so R
// and R^{-1} are bit for bit chol_inv's.  Returns false (uniform) when a
// pivot fails the floor test or is not finite: R, R^{-1} and Gs are then
// void and the caller restores G and runs chol_inv.  Gs: G on entry
// (row-major, ld F+1), R on exit; Ri: R^{-1}; work: 24F doubles; dgs: F
// doubles.  Layout as in chol_inv: lane c owns column c of [G | I]; wave w
// holds rows 8(p + s/2) + 4(s%2) + w in slot s during panel p.
// ---------------------------------------------------------------------------
template <int F>
__device__ __forceinline__ bool chol_inv_fast(double* Gs, double* Ri, double* work, double* dgs, int f) {
  typedef SmallCfg<F> C;
  constexpr int LD = C::LD, NR = C::NR, W2 = 2 * F;
  static_assert(F % 8 == 0 && W2 <= 64, "one column of [G | I] per lane");
  double* P = work;                      // panel rows: P[j*W2 + c], j < 8
  double* XT = work + 8 * W2;            // multipliers: XT[j*F + i] = R(kp+j, i)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane;
  const bool live = c < W2;
  for (int i = tid; i < F; i += 256) dgs[i] = i < f ? Gs[i * LD + i] : 1.0;
  double M[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = 8 * (s / 2) + 4 * (s % 2) + w;
    double v = 0.0;
    if (c < F) v = (i < f && c < f) ? Gs[i * LD + c] : (i == c ? 1.0 : 0.0);
    else if (live) v = (c - F == i) ? 1.0 : 0.0;
    M[s] = v;
  }
  __syncthreads();                       // G consumed: Gs now receives R; dgs ready
  bool ok = true;
  const int cl = live ? c : 0;
#pragma unroll 1
  for (int p = 0; p < F / 8; ++p) {              // a loop: the code stays small enough for the I-cache
    const int kp = 8 * p;
    if (live) {
      P[w * W2 + c] = M[0];
      P[(4 + w) * W2 + c] = M[1];
    }
    __syncthreads();
    double d[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = i; j < 8; ++j) d[i][j] = P[i * W2 + kp + j];
    double yv[8], dgk[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      yv[j] = P[j * W2 + cl];
      dgk[j] = dgs[kp + j];
    }
    double alpha[8], ia[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double piv = d[j][j];
      ok = ok && piv > FLOOR_C * U64 * dgk[j] && piv > PIV_MIN && piv < INFINITY;
      double y = __builtin_amdgcn_rsq(piv);
      y = y * fma(-0.5 * piv, y * y, 1.5);
      y = y * fma(-0.5 * piv, y * y, 1.5);
      alpha[j] = piv * y;
      ia[j] = y;
#pragma unroll
      for (int i = j + 1; i < 8; ++i) d[j][i] *= y;
#pragma unroll
      for (int i = j + 1; i < 8; ++i)
#pragma unroll
        for (int i2 = i; i2 < 8; ++i2) d[i][i2] = fma(-d[j][i], d[j][i2], d[i][i2]);
    }
    double X[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      double acc = yv[j];
#pragma unroll
      for (int i = 0; i < j; ++i) acc = fma(-d[i][j], X[i], acc);
      X[j] = acc * ia[j];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {        // rows kp + 2w + h of R, columns of R^{-1}, multipliers
      double xj = X[0], aj = alpha[0];
#pragma unroll
      for (int j = 1; j < 8; ++j)
        if (j == 2 * w + h) {
          xj = X[j];
          aj = alpha[j];
        }
      const int j = 2 * w + h, k = kp + j;
      if (c < F) {
        Gs[k * LD + c] = (c == k) ? aj : (c > k ? xj : 0.0);
        XT[j * F + c] = xj;
      } else if (live) {
        const int cc = c - F;
        Ri[cc * LD + k] = cc <= k ? xj : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 2; s < NR; ++s) {           // rank-8 update of the rows below the panel
      if (s >= NR - 2 * p) break;            // slots past the matrix
      const int i = kp + 8 * (s / 2) + 4 * (s % 2) + w;
      double mj[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) mj[j] = XT[j * F + i];
#pragma unroll
      for (int j = 0; j < 8; ++j) M[s] = fma(-mj[j], X[j], M[s]);
    }
#pragma unroll
    for (int s = 0; s + 2 < NR; ++s) M[s] = M[s + 2];
    M[NR - 2] = 0.0;
    M[NR - 1] = 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < (F - f) * F; idx += 256) {   // padding rows / columns
    const int a = f + idx / F, b = idx - (idx / F) * F;
    Gs[a * LD + b] = 0.0;
    Ri[b * LD + a] = 0.0;
  }
  __syncthreads();
  return ok;
}

// ---------------------------------------------------------------------------
// C = op(A) op(B) for FP64 matrices in global or LDS memory (M, N, K <=
// 128): element (i,k) of op(A) at TA ? A[k*lda + i] : A[i*lda + k], (k,j)
// of op(B) at TB ? B[j*ldb + k] : B[k*ldb + j]; element (i, j) of the
// product is handed to out(i, j, v) for i < M, j < N.  The four waves take
// the 16 x 16 tiles in turn; a tile loads its K strip 64 at a time before
// the MFMAs, so a chunk costs one memory round trip.
// ---------------------------------------------------------------------------
template <bool TA, bool TB, typename Out>
__device__ __forceinline__ void gmm64(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                                      Out out) {
  typedef Mfma<double> MF;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int TM = (M + 15) / 16, TN = (N + 15) / 16, KC = (K + 63) / 64;
  const int ntile = TM * TN > wv ? (TM * TN - wv + 3) / 4 : 0;   // this wave's tiles: wv, wv + 4, ...
  const int items = ntile * KC;                                 // (tile, 64-deep chunk) in order
  // operands of the next item load while the current one computes (two
  // named buffers keep the register arrays statically indexed)
  double a0[16], b0[16], a1[16], b1[16];
  auto load = [&](double(&a)[16], double(&b)[16], int it) {
    const int tile = wv + 4 * (it / KC), k0 = 64 * (it % KC);
    const int ti = tile / TN, tj = tile - ti * TN;
    const int ar = 16 * ti + r, bc = 16 * tj + r;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int kk = k0 + 4 * q + g;
      const bool ok = kk < K;
      a[q] = (ok && ar < M) ? (TA ? A[(int64_t)kk * lda + ar] : A[(int64_t)ar * lda + kk]) : 0.0;
      b[q] = (ok && bc < N) ? (TB ? B[(int64_t)bc * ldb + kk] : B[(int64_t)kk * ldb + bc]) : 0.0;
    }
  };
  typename MF::acc_t acc = MF::zero();
  auto step = [&](const double(&a)[16], const double(&b)[16], int it) {
#pragma unroll
    for (int q = 0; q < 16; ++q) acc = MF::op(a[q], b[q], acc);
    if (it % KC == KC - 1) {
      const int tile = wv + 4 * (it / KC);
      const int ti = tile / TN, tj = tile - ti * TN;
      const int bc = 16 * tj + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * ti + MF::row(g, e);
        if (i < M && bc < N) out(i, bc, acc[e]);
      }
      acc = MF::zero();
    }
  };
  if (items > 0) load(a0, b0, 0);
  for (int it = 0; it < items; it += 2) {
    if (it + 1 < items) load(a1, b1, it + 1);
    step(a0, b0, it);
    if (it + 2 < items) load(a0, b0, it + 2);
    if (it + 1 < items) step(a1, b1, it + 1);
  }
}

// C = op(A) op(B) for M, N, K <= 64 with both operands staged in LDS first
// (every thread's loads in flight at once: one memory round trip), then
// 16 x 16 FP64 MFMA tiles from LDS, four per wave.  Element (i,k) of op(A)
// at TA ? A[k*lda + i] : A[i*lda + k], (k,j) of op(B) at TB ? B[j*ldb + k] :
// B[k*ldb + j]; element (i, j) of the product goes to out(i, j, v) for
// i < M, j < N.  sm: GMM64S_LDS doubles of LDS; the call begins and ends
// with a barrier, so consecutive calls may share sm.
constexpr int GMM64S_LD = 65;
constexpr int GMM64S_LDS = 2 * 64 * GMM64S_LD;
template <bool TA, bool TB, typename Out>
__device__ __forceinline__ void gmm64s(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                                       double* sm, Out out) {
  typedef Mfma<double> MF;
  constexpr int LD = GMM64S_LD;
  double* As = sm;                 // As[i*LD + k] = op(A)(i, k)
  double* Bs = sm + 64 * LD;       // Bs[k*LD + j] = op(B)(k, j)
  const int tid = threadIdx.x;
  __syncthreads();                 // earlier readers of sm are done
  double va[16], vb[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q;
    const int hi = idx >> 6, lo = idx & 63;   // lo runs along contiguous memory
    // op(A): TA -> memory (k = hi, i = lo) contiguous in i; else (i = hi, k = lo)
    {
      const int i = TA ? lo : hi, k = TA ? hi : lo;
      va[q] = (i < M && k < K) ? (TA ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k]) : 0.0;
    }
    // op(B): TB -> memory (j = hi, k = lo) contiguous in k; else (k = hi, j = lo)
    {
      const int j = TB ? hi : lo, k = TB ? lo : hi;
      vb[q] = (k < K && j < N) ? (TB ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j]) : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q;
    const int hi = idx >> 6, lo = idx & 63;
    {
      const int i = TA ? lo : hi, k = TA ? hi : lo;
      As[i * LD + k] = va[q];
    }
    {
      const int j = TB ? hi : lo, k = TB ? lo : hi;
      Bs[k * LD + j] = vb[q];
    }
  }
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int TM = (M + 15) / 16, TN = (N + 15) / 16, KS = (K + 3) / 4;
  // wave wv: tiles wv, wv + 4, wv + 8, wv + 12 of the TM x TN grid (row-major)
  typename MF::acc_t acc[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = MF::zero();
  for (int kk = 0; kk < KS; ++kk) {
    const int k = 4 * kk + g;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int tile = wv + 4 * h;
      if (tile < TM * TN) {
        const int ti = tile / TN, tj = tile - ti * TN;
        acc[h] = MF::op(As[(16 * ti + r) * LD + k], Bs[k * LD + 16 * tj + r], acc[h]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int tile = wv + 4 * h;
    if (tile < TM * TN) {
      const int ti = tile / TN, tj = tile - ti * TN;
      const int j = 16 * tj + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * ti + MF::row(g, e);
        if (i < M && j < N) out(i, j, acc[h][e]);
      }
    }
  }
  __syncthreads();
}

// LDS (doubles) used by chol_inv128.
constexpr int CHOL128_LDS = 3 * SmallCfg<64>::SIZE + 24 * 64 + 2 * 64;

// ---------------------------------------------------------------------------
// Cholesky with inverse of a symmetric positive semi-definite f x f matrix,
// 64 < f <= 128, blocked 2 x 2 over 64 on the four waves of a workgroup.
// It yields the R of the unblocked elimination with the pivot rules of
// chol_inv (up to rounding order):
//   R11 = chol(G11);
//   R12 = R11^{-T} G12 with the rows of pivots that did not eliminate and
//         the dead columns set to zero (those rows of R12 never enter the
//         elimination);
//   R22 = chol(G22 - R12^T R12), its floor rule referred to G22's diagonal;
//   R^{-1} = [R11^{-1}, -R11^{-1} R12 R22^{-1}; 0, R22^{-1}].
// G (read only, symmetric), R, Rinv: global FP64, leading dimension ldg;
// R and Rinv row-major (element (i,j) at i*ldg + j), or column-major (at
// j*ldg + i) with CM.  lds: CHOL128_LDS doubles.  dm_in / dm_out: dead
// masks of columns 0-63 and 64-127.  Returns the number of floored pivots
// (uniform).
// ---------------------------------------------------------------------------
template <bool CM = false>
__device__ int chol_inv128(const double* G, int ldg, int f, double* R, double* Rinv, double* lds,
                           uint64_t dm_in0, uint64_t dm_in1, int first_pass, uint64_t* dm_out0,
                           uint64_t* dm_out1) {
  auto at = [&](int i, int j) -> int64_t { return CM ? (int64_t)j * ldg + i : (int64_t)i * ldg + j; };
  typedef SmallCfg<64> S;
  constexpr int LD = S::LD;
  double* Gs = lds;                        // block being factored -> its R
  double* Ri = Gs + S::SIZE;               // its inverse
  double* T = Ri + S::SIZE;                // R12 (64 x n2), then P = R11^{-1} R12
  double* work = T + S::SIZE;
  double* dgs = work + 24 * 64;
  double* dg2 = dgs + 64;                  // diagonal of G22
  const int tid = threadIdx.x, n2 = f - 64;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    Gs[i * LD + j] = G[(int64_t)i * ldg + j];
  }
  for (int j = tid; j < n2; j += 256) dg2[j] = G[(int64_t)(64 + j) * ldg + 64 + j];
  __syncthreads();
  uint64_t nl1 = 0, nl2 = 0;
  int nf1 = 0, nf2 = 0;
  chol_inv<64>(Gs, Ri, work, dgs, 64, dm_in0, first_pass, dm_out0, &nf1, nullptr, &nl1);
  // R11, R11^{-1}; zero lower-left blocks
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    R[at(i, j)] = Gs[i * LD + j];
    Rinv[at(i, j)] = Ri[i * LD + j];
  }
  for (int idx = tid; idx < n2 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    R[at(64 + i, j)] = 0.0;
    Rinv[at(64 + i, j)] = 0.0;
  }
  // R12 = R11^{-T} G12, masked
  gmm64<true, false>(Ri, LD, G + 64, ldg, 64, n2, 64, [&](int i, int j, double v) {
    const bool z = ((nl1 >> i) & 1ull) || ((dm_in1 >> j) & 1ull);
    T[i * LD + j] = z ? 0.0 : v;
  });
  __syncthreads();
  // S = G22 - R12^T R12 (into Gs; R11 is stored), R12 out
  gmm64<true, false>(T, LD, T, LD, n2, n2, 64, [&](int i, int j, double v) {
    Gs[i * LD + j] = G[(int64_t)(64 + i) * ldg + 64 + j] - v;
  });
  for (int idx = tid; idx < 64 * n2; idx += 256) {
    const int i = idx / n2, j = idx - i * n2;
    R[at(i, 64 + j)] = T[i * LD + j];
  }
  __syncthreads();
  chol_inv<64>(Gs, Ri, work, dgs, n2, dm_in1, first_pass, dm_out1, &nf2, dg2, &nl2);
  for (int idx = tid; idx < n2 * n2; idx += 256) {
    const int i = idx / n2, j = idx - i * n2;
    R[at(64 + i, 64 + j)] = Gs[i * LD + j];
    Rinv[at(64 + i, 64 + j)] = Ri[i * LD + j];
  }
  __syncthreads();
  // R^{-1}_12 = -(R11^{-1} R12) R22^{-1}
  gmm64<CM, false>(Rinv, ldg, T, LD, 64, n2, 64, [&](int i, int j, double v) { Gs[i * LD + j] = v; });
  __syncthreads();
  gmm64<false, false>(Gs, LD, Ri, LD, 64, n2, n2, [&](int i, int j, double v) { Rinv[at(i, 64 + j)] = -v; });
  __syncthreads();
  return nf1 + nf2;
}

// ---------------------------------------------------------------------------
// QR of M^T (M = R2 R1, or M = R2 when R1 is null; f x f, 64 < f <= 128) by
// CholeskyQR2 in FP64 on one workgroup, with the matrices in global memory:
// G = M M^T = Rh1^T Rh1, Z1 = M^T Rh1^{-1}, Z1^T Z1 = Rh2^T Rh2, Qh =
// Z1 Rh2^{-1}, Rh = Rh2 Rh1 (first Cholesky floored, the second kills what
// stays non-positive).  R1, R2: element (i,j) at j*ldi + i (CMI) or
// i*ldi + j.  Qh and Rh go out through put_q(i, j, v) and put_r(i, j, v).
// scr: 7 buffers of 128 x 128 doubles.  lds: CHOL128_LDS doubles.  Returns
// the number of floored pivots.
// ---------------------------------------------------------------------------
template <bool CMI, typename PutQ, typename PutR>
__device__ int small_qr_mid(double* lds, const double* R1g, const double* R2g, int f, int ldi, double* scr,
                            PutQ put_q, PutR put_r) {
  constexpr int LB = 128;
  constexpr int64_t B2 = (int64_t)LB * LB;
  double* M = scr;
  double* G = scr + B2;
  double* H1 = scr + 2 * B2;
  double* H1i = scr + 3 * B2;
  double* Z1 = scr + 4 * B2;
  double* H2 = scr + 5 * B2;
  double* H2i = scr + 6 * B2;
  if (R1g) {
    gmm64<CMI, CMI>(R2g, ldi, R1g, ldi, f, f, f, [&](int i, int j, double v) { M[i * LB + j] = v; });
  } else {
    for (int idx = threadIdx.x; idx < f * f; idx += 256) {
      const int i = idx / f, j = idx - i * f;
      M[i * LB + j] = CMI ? R2g[(int64_t)j * ldi + i] : R2g[(int64_t)i * ldi + j];
    }
  }
  __syncthreads();
  gmm64<false, true>(M, LB, M, LB, f, f, f, [&](int i, int j, double v) { G[i * LB + j] = v; });
  __syncthreads();
  uint64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
  int nf = chol_inv128(G, LB, f, H1, H1i, lds, 0ull, 0ull, 1, &a0, &a1);
  gmm64<true, false>(M, LB, H1i, LB, f, f, f, [&](int i, int j, double v) { Z1[i * LB + j] = v; });
  __syncthreads();
  gmm64<true, false>(Z1, LB, Z1, LB, f, f, f, [&](int i, int j, double v) { G[i * LB + j] = v; });
  __syncthreads();
  nf += chol_inv128(G, LB, f, H2, H2i, lds, a0, a1, 0, &b0, &b1);
  gmm64<false, false>(Z1, LB, H2i, LB, f, f, f, put_q);
  gmm64<false, false>(H2, LB, H1, LB, f, f, f, put_r);
  __syncthreads();
  return nf;
}

// One f x f FP64 product of the split closing QR (64 < f <= 128): out =
// op(A) op(B), both operands column-major with leading dimension f, element
// (i,k) of op(A) at TA ? A[k*f + i] : A[i*f + k], (k,j) of op(B) at TB ?
// B[j*f + k] : B[k*f + j].  One workgroup per 32 x 32 output block (each
// wave one 16 x 16 tile, gmm64, the same K order as the one-workgroup form);
// out column-major (ld f) or, with ROWOUT, row-major with leading dimension
// ldo, rounded to T.
template <typename T, bool TA, bool TB, bool ROWOUT>
__global__ __launch_bounds__(256) void k_sq_prod(const double* __restrict__ A, const double* __restrict__ B, int f,
                                                 T* __restrict__ out, int64_t ldo) {
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  if (i0 >= f || j0 >= f) return;
  const int mt = min(32, f - i0), nt = min(32, f - j0);
  const double* As = TA ? A + i0 : A + (int64_t)i0 * f;
  const double* Bs = TB ? B + (int64_t)j0 * f : B + j0;
  gmm64<TA, TB>(As, f, Bs, f, mt, nt, f, [&](int i, int j, double v) {
    if constexpr (ROWOUT) out[(int64_t)(i0 + i) * ldo + (j0 + j)] = (T)v;
    else out[(int64_t)(j0 + j) * f + (i0 + i)] = (T)v;
  });
}

// Closing QR (as k_small_qr) for 64 < f <= 128: R1, R2 column-major f x f
// (R1 may be null), Qh -> Qout (column-major), Rh -> Dout (type T,
// row-major ldd); scr: 7 x 128 x 128 doubles.
template <typename T>
__global__ __launch_bounds__(256) void k_small_qr128(const double* __restrict__ R1g,
                                                     const double* __restrict__ R2g, int f,
                                                     double* __restrict__ Qout, T* __restrict__ Dout,
                                                     int64_t ldd, State* st, int count_floors, double* scr) {
  __shared__ double lds[CHOL128_LDS];
  const int nf = small_qr_mid<true>(lds, R1g, R2g, f, f, scr,
                                    [&](int i, int j, double v) { Qout[(int64_t)j * f + i] = v; },
                                    [&](int i, int j, double v) { Dout[(int64_t)i * ldd + j] = (T)v; });
  if (count_floors && threadIdx.x == 0 && nf && st) atomicAdd(&st->floored, nf);
}

// ---------------------------------------------------------------------------
// Cholesky with inverse of a symmetric positive semi-definite f x f matrix of
// any width, right-looking over panels of 64 columns with the pivot rules of
// chol_inv (the same R as the unblocked elimination up to rounding order;
// see chol_inv128 for the blocked form of the rules), R^{-1} by block back
// substitution.  Each step is a kernel, so the independent block products of
// a step run on different workgroups (G overwritten by the Schur complements;
// G, R, Rinv column-major, leading dimension ld; P = ceil(f / 64) panels):
//   k_cb_init       zero the blocks below the diagonal, dg = diag(G), dead
//                   flags reset when fresh;
//   k_cb_diag(p)    one workgroup: R_pp and R_pp^{-1} of the current Schur
//                   block (floor rule against dg), dead flags of the panel,
//                   mask of the pivots that did not eliminate -> nolive[p];
//   k_cb_look(p)    one workgroup per pair p < q <= r: it forms R_pq =
//                   R_pp^{-T} S_pq and R_pr (rows of pivots that did not
//                   eliminate and columns already dead zeroed) in LDS, and
//                   S_qr -= R_pq^T R_pr; the pair (q, q) also writes R_pq
//                   (every workgroup forms a block from the same operands
//                   in the same order, so the copies agree bit for bit);
//                   workgroup 0 takes (p+1, p+1) in LDS, writes R_{p,p+1}
//                   and goes on with the diagonal step p+1 while the others
//                   update the rest (the next diagonal factorization
//                   overlaps this step's trailing update).  The dead flags
//                   that step p+1 finds go to deadmask[p+1]: the other
//                   workgroups of the launch still read the flags panel
//                   p+1 had before, and no later step reads the new ones;
//                   the first k_cb_inv launch writes them to dead;
//   k_cb_inv(L, s)  R^{-1} by recursive doubling over groups of L = 1, 2,
//                   4, ... blocks: for adjacent groups A = [a, a+L) and
//                   C = [a+L, a+2L) (a = 0, 2L, ...) the block of rows A,
//                   columns C of R^{-1} is -A^{-1} R_AC C^{-1}, A^{-1} and
//                   C^{-1} finished at smaller L; stage 0 forms T = R_AC
//                   C^{-1} into G (free after the factorization), stage 1
//                   the blocks -A^{-1} T, stage 2 both for L = 1; one
//                   workgroup per output block, log2(P) levels instead of
//                   P - 1 dependent diagonals; stage 2 also writes the dead
//                   flags of panels 1 .. P-1 from deadmask.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cb_width(int f, int p) { return (f - 64 * p) < 64 ? f - 64 * p : 64; }

__global__ void k_cb_init(const double* __restrict__ G, int ld, int f, double* __restrict__ R,
                          double* __restrict__ Rinv, double* __restrict__ dg, int32_t* __restrict__ dead, int fresh,
                          const int32_t* __restrict__ stopb, int blk) {
  if (stopb && *stopb < blk) return;       // a speculative block after the stop
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)f * f; idx += nt) {
    const int j = (int)(idx / f), i = (int)(idx - (int64_t)j * f);
    if (i / 64 > j / 64) {
      R[(int64_t)j * ld + i] = 0.0;
      Rinv[(int64_t)j * ld + i] = 0.0;
    }
    if (i == j) {
      dg[i] = G[(int64_t)j * ld + i];
      if (fresh) dead[i] = 0;
    }
  }
}

__global__ __launch_bounds__(256) void k_cb_diag(const double* __restrict__ G, int ld, int f, int p,
                                                 double* __restrict__ R, double* __restrict__ Rinv,
                                                 const double* __restrict__ dg, int32_t* __restrict__ dead,
                                                 uint64_t* __restrict__ nolive, int first_pass, State* st,
                                                 int count_floors, const int32_t* __restrict__ stopb, int blk) {
  if (stopb && *stopb < blk) return;       // a speculative block after the stop
  typedef SmallCfg<64> S;
  constexpr int LD = S::LD;
  __shared__ double Gs[S::SIZE], Ri[S::SIZE], work[24 * 64], dgs[64];
  const int tid = threadIdx.x, k0 = 64 * p, pw = cb_width(f, p);
  uint64_t dm = 0, dmo = 0, nl = 0;
  for (int c = 0; c < pw; ++c) dm |= (uint64_t)(dead[k0 + c] != 0) << c;
  stage_small<64>({G + (int64_t)k0 * ld + k0}, pw, {Gs}, LD, ld);
  __syncthreads();
  int nf = 0;
  chol_inv<64>(Gs, Ri, work, dgs, pw, dm, first_pass, &dmo, &nf, dg + k0, &nl);
  for (int idx = tid; idx < pw * pw; idx += 256) {
    const int i = idx / pw, j = idx - i * pw;
    R[(int64_t)(k0 + j) * ld + k0 + i] = Gs[i * LD + j];
    Rinv[(int64_t)(k0 + j) * ld + k0 + i] = Ri[i * LD + j];
  }
  for (int c = tid; c < pw; c += 256) dead[k0 + c] = (int32_t)((dmo >> c) & 1ull);
  if (tid == 0) {
    nolive[p] = nl;
    if (count_floors && nf && st) atomicAdd(&st->floored, nf);
  }
}

__global__ __launch_bounds__(256) void k_cb_look(double* __restrict__ G, int ld, int f, int p,
                                                 double* __restrict__ R, double* __restrict__ Rinv,
                                                 const double* __restrict__ dg, const int32_t* __restrict__ dead,
                                                 uint64_t* __restrict__ nolive, uint64_t* __restrict__ deadmask,
                                                 int first_pass, State* st, int count_floors,
                                                 const int32_t* __restrict__ stopb, int blk) {
  if (stopb && *stopb < blk) return;       // a speculative block after the stop
  typedef SmallCfg<64> S;
  constexpr int LD = S::LD;
  static_assert(S::SIZE >= 64 * LD, "a 64 x 64 block per buffer");
  __shared__ double sm[GMM64S_LDS];
  __shared__ double Gs[S::SIZE], Ri[S::SIZE], work[24 * 64], dgs[64];
  const int k0 = 64 * p, pw = cb_width(f, p);
  const uint64_t nl = nolive[p];
  // R_pq = R_pp^{-T} S_pq with the masked entries zeroed, into dst (column j
  // at dst + j*LD) and, if store, into R
  auto rblock = [&](int q, double* dst, bool store) {
    const int c0 = 64 * q, qw = cb_width(f, q);
    gmm64s<false, true>(Rinv + (int64_t)k0 * ld + k0, ld, G + (int64_t)c0 * ld + k0, ld, pw, qw, pw, sm,
                        [&](int i, int j, double v) {
                          const bool z = ((nl >> i) & 1ull) || dead[c0 + j] != 0;
                          const double x = z ? 0.0 : v;
                          dst[j * LD + i] = x;
                          if (store) R[(int64_t)(c0 + j) * ld + k0 + i] = x;
                        });
  };
  if (blockIdx.x != 0) {
    // trailing block pair (q, r), p < q <= r < P, enumerated row by row;
    // pair 0 = (p+1, p+1) belongs to workgroup 0
    const int P = (f + 63) / 64;
    int idx = blockIdx.x, q = p + 1;
    while (idx >= P - q) {
      idx -= P - q;
      ++q;
    }
    const int r = q + idx;
    const int cq = 64 * q, cr = 64 * r, qw = cb_width(f, q), rw = cb_width(f, r);
    rblock(q, Gs, q == r);
    if (r != q) rblock(r, Ri, false);
    gmm64s<false, true>(Gs, LD, r != q ? Ri : Gs, LD, qw, rw, pw, sm,
                        [&](int i, int j, double v) { G[(int64_t)(cr + j) * ld + cq + i] -= v; });
    return;
  }
  // workgroup 0: R_{p,p+1}, S_{p+1,p+1} -= R_{p,p+1}^T R_{p,p+1} in LDS,
  // then the diagonal step p+1 on it (as k_cb_diag)
  const int tid = threadIdx.x, p1 = p + 1, c1 = 64 * p1, w1 = cb_width(f, p1);
  uint64_t dm = 0, dmo = 0, nl1 = 0;
  for (int c = 0; c < w1; ++c) dm |= (uint64_t)(dead[c1 + c] != 0) << c;
  rblock(p1, Ri, true);
  stage_small<64>({G + (int64_t)c1 * ld + c1}, w1, {Gs}, LD, ld);
  gmm64s<false, true>(Ri, LD, Ri, LD, w1, w1, pw, sm, [&](int i, int j, double v) { Gs[i * LD + j] -= v; });
  int nf = 0;
  chol_inv<64>(Gs, Ri, work, dgs, w1, dm, first_pass, &dmo, &nf, dg + c1, &nl1);
  for (int idx = tid; idx < w1 * w1; idx += 256) {
    const int i = idx / w1, j = idx - i * w1;
    R[(int64_t)(c1 + j) * ld + c1 + i] = Gs[i * LD + j];
    Rinv[(int64_t)(c1 + j) * ld + c1 + i] = Ri[i * LD + j];
  }
  if (tid == 0) {
    nolive[p1] = nl1;
    deadmask[p1] = dmo;
    if (count_floors && nf && st) atomicAdd(&st->floored, nf);
  }
}

__global__ __launch_bounds__(256) void k_cb_inv(const double* __restrict__ R, double* __restrict__ Rinv,
                                                double* __restrict__ G, int ld, int f, int L, int stage,
                                                const uint64_t* __restrict__ deadmask, int32_t* __restrict__ dead,
                                                const int32_t* __restrict__ stopb, int blk) {
  if (stopb && *stopb < blk) return;       // a speculative block after the stop
  if (stage == 2 && blockIdx.x == 0)
    for (int c = 64 + threadIdx.x; c < f; c += 256) dead[c] = (int32_t)((deadmask[c >> 6] >> (c & 63)) & 1ull);
  constexpr int LD = SmallCfg<64>::LD;
  __shared__ double Acc[64 * LD];
  __shared__ double sm[GMM64S_LDS];
  const int P = (f + 63) / 64;
  // this workgroup's pair (groups A = [a, a+L), C = [a+L, a+2L)) and block (i, j)
  int idx = blockIdx.x, a = 0, cw = 0;
  for (;; a += 2 * L) {
    cw = min(a + 2 * L, P) - (a + L);
    if (idx < L * cw) break;
    idx -= L * cw;
  }
  const int i = a + idx / cw, j = a + L + idx % cw;
  const int wi = cb_width(f, i), wj = cb_width(f, j), ci = 64 * i, cj = 64 * j;
  if (stage != 1) {
    // T_ij = sum_{a+L <= m <= j} R_im (R^{-1})_mj
    for (int m = a + L; m <= j; ++m) {
      const bool first = m == a + L;
      gmm64s<true, true>(R + (int64_t)(64 * m) * ld + ci, ld, Rinv + (int64_t)cj * ld + 64 * m, ld, wi, wj,
                         cb_width(f, m), sm,
                         [&](int r, int c, double v) { Acc[r * LD + c] = first ? v : Acc[r * LD + c] + v; });
    }
    if (stage == 0) {
      for (int e = threadIdx.x; e < wi * wj; e += 256) {
        const int r = e / wj, c = e - r * wj;
        G[(int64_t)(cj + c) * ld + ci + r] = Acc[r * LD + c];
      }
      return;
    }
    // stage 2 (L = 1, A = {i}): (R^{-1})_ij = -(R^{-1})_ii T_ij, T still in LDS
    gmm64s<true, false>(Rinv + (int64_t)ci * ld + ci, ld, Acc, LD, wi, wj, wi, sm,
                        [&](int r, int c, double v) { Rinv[(int64_t)(cj + c) * ld + ci + r] = -v; });
    return;
  }
  // (R^{-1})_ij = -sum_{i <= k < a+L} (R^{-1})_ik T_kj, T from G
  for (int k = i; k < a + L; ++k) {
    const bool first = k == i;
    gmm64s<true, true>(Rinv + (int64_t)(64 * k) * ld + ci, ld, G + (int64_t)cj * ld + 64 * k, ld, wi, wj,
                       cb_width(f, k), sm,
                       [&](int r, int c, double v) { Acc[r * LD + c] = first ? v : Acc[r * LD + c] + v; });
  }
  for (int e = threadIdx.x; e < wi * wj; e += 256) {
    const int r = e / wj, c = e - r * wj;
    Rinv[(int64_t)(cj + c) * ld + ci + r] = -Acc[r * LD + c];
  }
}

// The panel-blocked Cholesky with inverse (the k_cb_* steps) for two
// panels, 64 < f <= 128, on one workgroup with every block in LDS: R11 and
// its inverse by chol_inv<64> (floor rule against G's own diagonal); R12 =
// R11^{-T} G12 with the rows of pivots that did not eliminate and the
// columns already dead zeroed; S22 = G22 - R12^T R12; R22 and its inverse by
// chol_inv<64> (floor rule against G22's original diagonal); (R^{-1})12 =
// -R11^{-1} (R12 R22^{-1}).  The same R and R^{-1} as the separate launches
// up to rounding order; G (column-major, ld) is not modified.  Outputs as
// k_cb_*: R, R^{-1} column-major (ld), per-column dead flags.
__global__ __launch_bounds__(256) void k_chol2p(const double* __restrict__ G, int ld, int f,
                                                double* __restrict__ R, double* __restrict__ Rinv,
                                                int32_t* __restrict__ dead, int first_pass, int fresh, State* st,
                                                int count_floors, const int32_t* __restrict__ stopb, int blk) {
  if (stopb && *stopb < blk) return;       // a speculative block after the stop
  typedef SmallCfg<64> S;
  constexpr int LD = S::LD;
  __shared__ double A[S::SIZE], B[S::SIZE], C[S::SIZE], D[S::SIZE], work[24 * 64], dgs[64], dg1[64];
  const int tid = threadIdx.x, w1 = f - 64;
  // lower-left blocks of R and R^{-1}
  for (int idx = tid; idx < w1 * 64; idx += 256) {
    const int i = 64 + idx / 64, j = idx % 64;
    R[(int64_t)j * ld + i] = 0.0;
    Rinv[(int64_t)j * ld + i] = 0.0;
  }
  uint64_t dm0 = 0, dm1 = 0;
  if (!fresh) {
    for (int c = 0; c < 64; ++c) dm0 |= (uint64_t)(dead[c] != 0) << c;
    for (int c = 0; c < w1; ++c) dm1 |= (uint64_t)(dead[64 + c] != 0) << c;
  }
  // G11 -> A, G12 -> C, G22 -> D (row-major, zero padded); each thread's
  // loads in flight before its stores
  {
    constexpr int NQ = 64 * 64 / 256;
    double va[NQ], vc[NQ], vd[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = tid + 256 * q, j = idx / 64, i = idx % 64;      // element (i, j)
      va[q] = G[(int64_t)j * ld + i];
      vc[q] = j < w1 ? G[(int64_t)(64 + j) * ld + i] : 0.0;
      vd[q] = (i < w1 && j < w1) ? G[(int64_t)(64 + j) * ld + 64 + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = tid + 256 * q, j = idx / 64, i = idx % 64;
      A[i * LD + j] = va[q];
      C[i * LD + j] = vc[q];
      D[i * LD + j] = vd[q];
      if (i == j) dg1[i] = vd[q];
    }
  }
  __syncthreads();
  uint64_t dmo0 = 0, nl0 = 0, dmo1 = 0, nl1 = 0;
  int nf0 = 0, nf1 = 0;
  chol_inv<64>(A, B, work, dgs, 64, dm0, first_pass, &dmo0, &nf0, nullptr, &nl0);
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx / 64, j = idx % 64;
    R[(int64_t)j * ld + i] = A[i * LD + j];
    Rinv[(int64_t)j * ld + i] = B[i * LD + j];
  }
  __syncthreads();
  // R12 = R11^{-T} G12, masked, into A (and R)
  lds_gemm<64, true, false>(B, C, [&](int i, int j, double v) {
    const bool z = j >= w1 || ((nl0 >> i) & 1ull) || ((dm1 >> j) & 1ull);
    A[i * LD + j] = z ? 0.0 : v;
    if (j < w1) R[(int64_t)(64 + j) * ld + i] = z ? 0.0 : v;
  });
  __syncthreads();
  // S22 = G22 - R12^T R12
  lds_gemm<64, true, false>(A, A, [&](int i, int j, double v) {
    if (i < w1 && j < w1) D[i * LD + j] -= v;
  });
  __syncthreads();
  chol_inv<64>(D, C, work, dgs, w1, dm1, first_pass, &dmo1, &nf1, dg1, &nl1);
  for (int idx = tid; idx < w1 * w1; idx += 256) {
    const int i = idx / w1, j = idx % w1;
    R[(int64_t)(64 + j) * ld + 64 + i] = D[i * LD + j];
    Rinv[(int64_t)(64 + j) * ld + 64 + i] = C[i * LD + j];
  }
  __syncthreads();
  // T = R12 R22^{-1} into D, then (R^{-1})12 = -R11^{-1} T
  lds_gemm<64, false, false>(A, C, [&](int i, int j, double v) { D[i * LD + j] = v; });
  __syncthreads();
  lds_gemm<64, false, false>(B, D, [&](int i, int j, double v) {
    if (j < w1) Rinv[(int64_t)(64 + j) * ld + i] = -v;
  });
  for (int c = tid; c < f; c += 256)
    dead[c] = (int32_t)(c < 64 ? ((dmo0 >> c) & 1ull) : ((dmo1 >> (c - 64)) & 1ull));
  if (tid == 0 && count_floors && (nf0 + nf1) && st) atomicAdd(&st->floored, nf0 + nf1);
}

// Arguments of the Cholesky that closes a Gram pass (k_gram_rows, and the
// global-memory path for wide blocks).
struct CholArgs {
  double* R;               // R out: f x f, element (i,j) at j*f + i (lower part zero); may be null
  double* Rinv;            // R^{-1} out, same layout; may be null
  int32_t* dead;           // per-column dead flags (in/out)
  int first_pass;          // floor (1) or kill (0) non-positive pivots
  int fresh;               // ignore incoming dead flags (a new factorization)
  State* st;
  int count_floors;        // add floored pivots to st->floored
  const double* R1;        // non-null: stop test of a basis block (diag of R1)
  int64_t col0, n;
  int64_t* wlog;
  int32_t* acc;
  double* diag_log;
  const double* norm_parts;  // non-null: finish ||A||_F and eps = tol ||A||_F first
  const float* max_parts;    // with norm_parts: per-workgroup max |A| -> st->lp_scale
  int64_t n_norm;
  Gate gate;               // closing steps enqueued ahead of the stop flag
  const int64_t* f_dev;    // non-null: block width read on the device (<= the template width)
};

// ---------------------------------------------------------------------------
// Gram matrix G = Z^T Z (FP64) of a rows x f block, then chol_inv of G:
//   MODE 0: Z = X as stored (column-major, type T);
//   MODE 1: Z = X W with W f x f FP64 (element (i,j) at j*f + i), formed
//           panel by panel in FP64 on MFMA, rounded to T and written back
//           over X; G is the Gram of the rounded Z, so the next Cholesky
//           factor corrects the block actually stored (the second pass of
//           CholeskyQR2 must see the Z it orthogonalises).
// Each workgroup stages panels of RPW rows of X in LDS (grid-stride),
// accumulates on f64 MFMA with its 4 waves splitting the panel rows, folds
// the waves in fixed order and writes its partial to parts[blockIdx.x]
// (element (i,j) at j*f + i).  The last workgroup to arrive (device-scope
// counter) sums the partials in fixed order and runs chol_inv plus the
// epilogues in ca: R, R^{-1}, dead flags, floors, the ||A||_F finish and
// the stop test of Alg. 1:
//   d_c = |T(c,c)| = R(c,c) R1(c,c) (0 for dead columns); the first c with
//   d_c <= eps keeps columns 0..c-1 and stops the loop, otherwise all f are
//   kept and the loop ends after the last column of Omega.
// ---------------------------------------------------------------------------
template <typename T, int F, int MODE>
struct GramCfg {
  typedef SmallCfg<F> S;
  static constexpr int RPW = MODE == 0 ? (F * (int)sizeof(T) <= 128 ? 256 : 128)
                                       : (F <= 32 ? 256 : (sizeof(T) == 4 ? 128 : 64));
  static constexpr int LDX = RPW + 16 / (int)sizeof(T);   // X panel column stride (T elements)
  static constexpr int LDZ = RPW + 2;                     // Z panel column stride (doubles)
  static constexpr int PBASE = MODE == 1 ? S::SIZE : 0;   // W first (MODE 1), then the phases
  static constexpr int XD = (F * LDX * (int)sizeof(T) + 7) / 8;
  static constexpr int ZD = MODE == 1 ? F * LDZ : 0;
  static constexpr int FOLD = (F / 16) * (F / 16) * 256;
  static constexpr int LOOPD = XD + ZD > FOLD ? XD + ZD : FOLD;
  static constexpr int CHAIND = 2 * S::SIZE + 24 * F + F;
  static constexpr int TOTAL = PBASE + (LOOPD > CHAIND ? LOOPD : CHAIND);
};

template <typename T, int F, int MODE>
__global__ __launch_bounds__(256) void k_gram_rows(
    T* __restrict__ X, int64_t ld, int64_t rows, int f, const double* __restrict__ Wg,
    double* __restrict__ parts, uint32_t* __restrict__ counter, const int32_t* __restrict__ stop_block,
    int block_id, CholArgs ca) {
  typedef Mfma<double> MF;
  typedef GramCfg<T, F, MODE> Cfg;
  typedef SmallCfg<F> S;
  constexpr int TT = F / 16, RPW = Cfg::RPW, LDX = Cfg::LDX, LDZ = Cfg::LDZ, LD = S::LD;
  static_assert(Cfg::TOTAL * 8 <= 160 * 1024, "LDS budget");
  if (stop_block && *stop_block < block_id) return;
  if (gate_shut(ca.gate)) return;
  if (ca.f_dev) f = (int)*ca.f_dev;
  if (f > F) return;                    // cannot happen: the launch width bounds the rank
  __shared__ __align__(16) double lds[Cfg::TOTAL];
  double* Wl = lds;                                   // MODE 1: W, row-major ld F+1
  double* ph = lds + Cfg::PBASE;
  T* pan = reinterpret_cast<T*>(ph);                  // X panel: pan[c*LDX + row]
  double* pz = ph + Cfg::XD;                          // MODE 1: Z panel: pz[c*LDZ + row]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  if constexpr (MODE == 1) stage_small<F>({Wg}, f, {Wl}, LD);
  typename MF::acc_t acc[TT][TT];
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int u = 0; u < TT; ++u) acc[t][u] = MF::zero();
  const int64_t npan = (rows + RPW - 1) / RPW;
  constexpr int NIT = F * RPW / 256;
  static_assert(NIT <= 32, "staging registers");
  for (int64_t pnl = blockIdx.x; pnl < npan; pnl += gridDim.x) {
    const int64_t rb = pnl * RPW;
    __syncthreads();                          // previous panel consumed (and W ready)
    {                                         // stage X (zero outside rows x f), all loads in flight
      T xv[NIT];
#pragma unroll
      for (int q = 0; q < NIT; ++q) {
        const int idx = tid + 256 * q;
        const int c = idx / RPW, rl = idx - c * RPW;
        const int64_t row = rb + rl;
        xv[q] = (c < f && row < rows) ? X[(int64_t)c * ld + row] : (T)0;
      }
#pragma unroll
      for (int q = 0; q < NIT; ++q) {
        const int idx = tid + 256 * q;
        const int c = idx / RPW, rl = idx - c * RPW;
        pan[c * LDX + rl] = xv[q];
      }
    }
    __syncthreads();
    if constexpr (MODE == 1) {                // Z panel = X panel W (FP64 MFMA), rounded to T
      for (int rt = wv; rt < RPW / 16; rt += 4) {
        double a[F / 4];
#pragma unroll
        for (int kk = 0; kk < F / 4; ++kk) a[kk] = (double)pan[(4 * kk + g) * LDX + 16 * rt + r];
        typename MF::acc_t z[TT];
#pragma unroll
        for (int u = 0; u < TT; ++u) z[u] = MF::zero();
#pragma unroll
        for (int kk = 0; kk < F / 4; ++kk)
#pragma unroll
          for (int u = 0; u < TT; ++u) z[u] = MF::op(a[kk], Wl[(4 * kk + g) * LD + 16 * u + r], z[u]);
#pragma unroll
        for (int u = 0; u < TT; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            pz[(16 * u + r) * LDZ + 16 * rt + MF::row(g, e)] = (double)(T)z[u][e];
      }
      __syncthreads();
      {                                       // write Z back over X (LDS reads batched)
        double zv[NIT];
#pragma unroll
        for (int q = 0; q < NIT; ++q) {
          const int idx = tid + 256 * q;
          const int c = idx / RPW, rl = idx - c * RPW;
          zv[q] = pz[c * LDZ + rl];
        }
#pragma unroll
        for (int q = 0; q < NIT; ++q) {
          const int idx = tid + 256 * q;
          const int c = idx / RPW, rl = idx - c * RPW;
          const int64_t row = rb + rl;
          if (c < f && row < rows) X[(int64_t)c * ld + row] = (T)zv[q];
        }
      }
    }
    // Gram over this panel: wave wv takes rows [wv*RPW/4, (wv+1)*RPW/4)
    constexpr int PW = RPW / 4;
#pragma unroll
    for (int k0 = 0; k0 < PW; k0 += 16) {
      const int kr = wv * PW + k0 + 4 * g;
      V4<double> a[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          a[t].v[e] = MODE == 1 ? pz[(16 * t + r) * LDZ + kr + e] : (double)pan[(16 * t + r) * LDX + kr + e];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
          for (int u = t; u < TT; ++u) acc[t][u] = MF::op(a[t].v[v], a[u].v[v], acc[t][u]);
    }
  }
  // fold the 4 waves (fixed order) through LDS
  __syncthreads();
  double* red = ph;
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int t = 0; t < TT; ++t)
#pragma unroll
        for (int u = t; u < TT; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            double* qq = &red[((t * TT + u) * 4 + e) * 64 + lane];
            *qq = (w == 0) ? acc[t][u][e] : *qq + acc[t][u][e];
          }
    }
    __syncthreads();
  }
  // workgroup partial, symmetric fill: tile (t,u) register e of lane l is
  // G[16t + 4e + l/16][16u + l%16]
  double* Pw = parts + (int64_t)blockIdx.x * f * f;
  for (int idx = tid; idx < TT * TT * 256; idx += 256) {
    const int l = idx & 63, e = (idx >> 6) & 3, tu = idx >> 8;
    const int t = tu / TT, u = tu - t * TT;
    if (u < t) continue;
    const int i = 16 * t + MF::row(l >> 4, e), jj = 16 * u + (l & 15);
    if (i < f && jj < f) {
      const double v = red[idx];
      Pw[(int64_t)jj * f + i] = v;
      Pw[(int64_t)i * f + jj] = v;
    }
  }
  // the last workgroup to arrive folds all partials in fixed order
  wg_stores_done();
  __shared__ int s_last;
  if (tid == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    s_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
    if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (!s_last) return;
  const int ff = f * f;
  double* Gs = ph;                   // G, then R
  double* Ri = Gs + S::SIZE;         // R^{-1}
  double* rowbuf = Ri + S::SIZE;     // elimination work area, 24F
  double* dgs = rowbuf + 24 * F;
  {
    // upper triangle, all partials of an element loaded before summing them
    // in order b = 0, 1, ...
    constexpr int EPT = (F * F + 255) / 256;
    const unsigned nb = gridDim.x;
    double sum[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) sum[e] = 0.0;
    constexpr int PB = EPT == 1 ? 96 : (EPT <= 4 ? 16 : 4);   // partials per batch (loads in flight)
    for (unsigned b = 0; b < nb; b += PB) {
      double v[EPT][PB];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 256 * e;
        const int c = idx / (f > 0 ? f : 1), rr = idx - c * f;
        const bool ok = idx < ff && rr <= c;
#pragma unroll
        for (int q = 0; q < PB; ++q)
          v[e][q] = (ok && b + q < nb) ? parts[(int64_t)(b + q) * ff + idx] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < EPT; ++e)
#pragma unroll
        for (int q = 0; q < PB; ++q) sum[e] += v[e][q];
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + 256 * e;
      const int c = idx / (f > 0 ? f : 1), rr = idx - c * f;
      if (idx < ff && rr <= c) {
        Gs[rr * LD + c] = sum[e];
        Gs[c * LD + rr] = sum[e];
      }
    }
  }
  if (tid == 0) *counter = 0u;
  State* st = ca.st;
  if (ca.norm_parts) {               // ||A||_F from the sketch partials (fixed order)
    // all four waves, 8 loads per thread in flight; the thread sums, the
    // wave sums and the four wave sums (in wave order) are each formed in a
    // fixed order
    double a = 0.0;
    float mx = 0.0f;
    for (int64_t i0 = 0; i0 < ca.n_norm; i0 += 256 * 8) {
      double pv[8];
      float mv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t i = i0 + tid + 256 * q;
        pv[q] = i < ca.n_norm ? ca.norm_parts[i] : 0.0;
        mv[q] = (ca.max_parts && i < ca.n_norm) ? ca.max_parts[i] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (i0 + tid + 256 * q < ca.n_norm) a += pv[q];
        mx = fmaxf(mx, mv[q]);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off);
      mx = fmaxf(mx, __shfl_xor(mx, off));
    }
    __shared__ double s_norm[4];
    __shared__ float s_max[4];
    if (lane == 0) {
      s_norm[wv] = a;
      s_max[wv] = mx;
    }
    __syncthreads();
    a = ((s_norm[0] + s_norm[1]) + s_norm[2]) + s_norm[3];
    mx = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
    if (tid == 0) {
      st->normsq = a;
      const bool bad = !(a < INFINITY);
      st->nonfinite = bad ? 1 : 0;
      st->eps = bad ? 0.0 : st->tol * sqrt(a);
      st->lp_scale = lp_scale_of(mx, st->lp_mode);
    }
  }
  int dl = 0;
  if (lane < f && !ca.fresh) dl = ca.dead[lane];
  const uint64_t dmask_in = __ballot(dl != 0);
  __syncthreads();
  uint64_t dmask;
  int nfl;
  chol_inv<F>(Gs, Ri, rowbuf, dgs, f, dmask_in, ca.first_pass, &dmask, &nfl);
  for (int idx = tid; idx < ff; idx += 256) {
    const int c = idx / f, rr = idx - c * f;          // element (rr, c) at c*f + rr
    if (ca.R) ca.R[idx] = Gs[rr * LD + c];
    if (ca.Rinv) ca.Rinv[idx] = Ri[rr * LD + c];
  }
  if (tid < f) ca.dead[tid] = (int32_t)((dmask >> tid) & 1ull);
  if (ca.count_floors && tid == 0 && nfl) atomicAdd(&st->floored, nfl);
  if (!ca.R1 || wv != 0) return;
  // stop test (Alg. 1) on wave 0: first column whose |T(c,c)| <= eps
  const int j = lane;
  const bool mine = j < f;
  const double eps = st->eps;
  double d = 0.0;
  bool hit = false;
  if (mine) {
    d = ((dmask >> j) & 1ull) ? 0.0 : Gs[j * LD + j] * ca.R1[(int64_t)j * f + j];
    hit = ((d <= eps) && (!st->paired || ((ca.col0 + j) & 1) == 0)) || st->nonfinite;
  }
  const unsigned long long mask = __ballot(hit);
  const int keep = mask ? (int)__ffsll((long long)mask) - 1 : f;
  if (mine && j <= keep) ca.diag_log[ca.col0 + j] = d;
  const double dk = __shfl(d, keep & 63);     // the stopping column's value (when one hit)
  if (j == 0) {
    if (mask != 0ull) st->d_stop = dk;
    const bool stop = (mask != 0ull) || (ca.col0 + f >= ca.n);
    ca.acc[block_id] = keep;
    const int64_t wn = ca.wlog[block_id] + keep;
    ca.wlog[block_id + 1] = wn;
    st->rank = wn;
    if (stop) st->stop_block = block_id;
  }
}

// ---------------------------------------------------------------------------
// Barrier across the workgroups of one launch, for launches small enough
// that all their workgroups are resident at once (at most CQR2_GMAX
// workgroups of 256 threads on a device of 256 CUs).  The workgroup's
// global stores are handed over as wg_stores_done describes (thread 0 takes
// the release), thread 0 arrives on the counter, waits for `target`
// arrivals and takes the acquire before the barrier that lets its waves
// read what the others wrote.  The wait is bounded by the 100 MHz wall
// clock: past CQR2_WAIT_TICKS (about 1.3 s; a resident grid arrives within
// microseconds) the workgroup sets st->sync_fail and goes on, so every wave
// still ends; the call then reports EODABE_ESYNC and its outputs are void.
// Each counter serves one launch per factorization and is zeroed by the
// state initialisation.
// ---------------------------------------------------------------------------
constexpr int CQR2_GMAX = 32;
constexpr int CQR2_RPW = 256;
// basis width up to which the projection runs in the launch: beyond it the
// 16-32 workgroups' MFMA work on W = Q^T Y and Y -= Q W outweighs the
// launches saved (at widths 160-256 on 4096 rows: 3-5 % slower than the
// separate K-split kernels on the whole GPU)
constexpr int CQR2_PROJ_WMAX = 128;
constexpr uint64_t CQR2_WAIT_TICKS = 1ull << 27;

__device__ __forceinline__ void grid_barrier(uint32_t* ctr, uint32_t target, State* st,
                                             uint64_t wait_ticks = CQR2_WAIT_TICKS) {
  wg_stores_done();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomicAdd(ctr, 1u);
    const uint64_t t0 = wall_clock64();
    while (atomicAdd(ctr, 0u) < target) {        // a read-modify-write: the device-coherent value
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > wait_ticks) {
        atomicMax(&st->sync_fail, 1);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Arguments of k_cqr2.  Matrices R1, R2 and their inverses: f x f FP64,
// element (i,j) at j*f + i, written by workgroup 0 when non-null.
struct Cqr2Args {
  const void* X;             // block: rows x f, element (i,c) at c*ldx + i (read only)
  int64_t ldx, rows;
  int f;
  const int64_t* f_dev;      // non-null: f read on the device (<= the template width)
  double* parts;             // 2 * gridDim.x * f * f doubles: the partial Grams of both passes
  uint32_t* counter;         // barrier counter, zero at launch
  const int32_t* stop_block; // non-null: return at once for a block after the stop
  int block_id;
  Gate gate;                 // closing steps enqueued ahead of the stop flag
  State* st;
  double *R1, *R1inv, *R2, *R2inv;
  int32_t* dead;             // per-column dead flags: read on the first pass unless fresh, written at the end
  int fresh;
  int count_floors;          // add floored pivots to st->floored
  const double* norm_parts;  // non-null: finish ||A||_F and eps = tol ||A||_F first (block 0)
  const float* max_parts;    // with norm_parts: per-workgroup max |A| -> st->lp_scale
  int64_t n_norm;
  int stop_test;             // run the stop test of Alg. 1 and write the kept columns at wlog[block_id]
  int64_t col0, n;
  int64_t* wlog;
  int32_t* acc;
  double* diag_log;
  void* Q;                   // output Z1 R2^{-1}: column c at Q + (zoff + c)*ldq
  int64_t ldq;
  // closing of Alg. 2 (with close_qr): M = R2 R1, M^T = Qh Rh by CholeskyQR2
  // in FP64 on every workgroup (the steps of k_small_qr); Rh -> Dout (type T,
  // row-major ldd) and Qh -> Qh_out (f x f, element (i,j) at j*f + i) by
  // workgroup 0; with Uout, U = Uq Qh (Uq: m_u x f, element (i,c) at
  // c*ldq_u + i; U likewise with ldu), rows split evenly over the workgroups
  int close_qr;
  void* Dout;
  int64_t ldd;
  double* Qh_out;
  const void* Uq;
  int64_t ldq_u;
  void* Uout;
  int64_t ldu, m_u;
  State* state_out;          // non-null (host-mapped): workgroup 0 copies the control block there
                             // once it is final, whether the gate let the closing run or not
  // block Gram-Schmidt against the basis before each pass (the PROJ form):
  // W = Qb^T Y, Y -= Qb W with Qb the basis (rows x wb, element (i,c) at
  // c*ldqb + i) and wb = *w_dev <= CQR2_PROJ_WMAX
  const void* Qb;
  int64_t ldqb;
  const int64_t* w_dev;
  void* wparts;              // CQR2_GMAX * CQR2_PROJ_WMAX * F elements of T: the partial W per workgroup
  int reuse_counter;         // the last workgroup out resets the counter (launches that share one)
  // failure injection for the tests of the time-out path: every barrier
  // waits for one arrival more than the launch makes, for at most
  // wait_ticks, so each one times out and every wave still ends
  uint32_t wait_extra;
  uint64_t wait_ticks;       // 0: CQR2_WAIT_TICKS
};

// The control block into host-mapped memory (thread 0 of workgroup 0): an
// acquire fence first, so the words read are the device's latest (the
// floor count was just updated by an atomic).
__device__ __forceinline__ void state_send(const Cqr2Args& a) {
  if (!a.state_out || blockIdx.x != 0 || threadIdx.x != 0) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const uint64_t* src = reinterpret_cast<const uint64_t*>(a.st);
  uint64_t* dst = reinterpret_cast<uint64_t*>(a.state_out);
  for (int i = 0; i < (int)(sizeof(State) / 8); ++i) dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int F, bool PROJ = false>
struct Cqr2Cfg {
  typedef SmallCfg<F> S;
  static constexpr int LDW = F + 1;                                 // folded W, row stride (T elements)
  static constexpr int WMAX = CQR2_PROJ_WMAX;
  static constexpr int WD = PROJ ? (WMAX * LDW * (int)sizeof(T) + 7) / 8 : 0;
  static constexpr int LDX = CQR2_RPW + 16 / (int)sizeof(T);      // panel column stride (T elements)
  static constexpr int XD = (F * LDX * (int)sizeof(T) + 7) / 8;    // panel, in doubles
  static constexpr int RED = (F / 16) * (F / 16) * 256;             // wave fold of a partial Gram
  static constexpr int CH = 2 * S::SIZE + 24 * F + F;               // G/R, R^{-1}, elimination rows, diagonal
  static constexpr int WORK = RED > CH ? RED : CH;
  static constexpr int TOTAL = XD + WORK + F + 8 + S::SIZE + WD;    // + R1's diagonal + scalars + R1 + W
  static_assert(XD >= 3 * S::SIZE, "the closing QR's three work matrices fit the panel area");
};

// ---------------------------------------------------------------------------
// CholeskyQR2 of a block (f <= F <= 32 columns, at most CQR2_GMAX panels of
// CQR2_RPW rows) in one launch, one workgroup per row panel, the panel held
// in LDS throughout (Alg. 1, "compute QR" of the sketch; Alg. 2, QR(C^T)):
//   pass 0: partial Gram of the panel; barrier; every workgroup sums all
//           partials in the same fixed order and runs chol_inv with the
//           floor rule (R1, R1^{-1}: the same bits in every workgroup);
//           Z1 = X R1^{-1} (FP64 MFMA, rounded to T) replaces the panel;
//   pass 1: partial Gram of Z1; barrier; sum, chol_inv with the kill rule
//           (R2, R2^{-1}); with stop_test the first column c with
//           |T(c,c)| = R2(c,c) R1(c,c) <= eps ends the kept width (every
//           workgroup takes the same decision); Q = Z1 R2^{-1} for the
//           kept columns.
// PROJ (a later block of the basis loop, basis width <= CQR2_PROJ_WMAX):
// before each pass the panel is projected against the basis (block
// Gram-Schmidt, BCGS2 over the two passes): W = Qb^T Y from per-workgroup
// partials summed in a fixed order after a barrier, then Y -= Qb W in place.
// close_qr (the closing of Alg. 2): after pass 1 every workgroup also runs
// the QR of R^T = (R2 R1)^T on its own LDS (the steps of k_small_qr) and
// forms its rows of U = Uq Qh.
// The arithmetic is that of the kernels it replaces (k_gram_rows modes 0
// and 1, k_apply, k_small_qr; for PROJ the K-split projection and update up
// to the grouping of the partial sums): the same fold order and MFMA
// sequences.  Workgroup 0 alone writes R1, R2, their inverses, the dead
// flags, the floors and the state.
// ---------------------------------------------------------------------------
template <typename T, int F, bool PROJ>
__global__ __launch_bounds__(256) void k_cqr2(Cqr2Args a) {
  typedef Mfma<double> MF;
  typedef Cqr2Cfg<T, F, PROJ> Cfg;
  typedef SmallCfg<F> S;
  constexpr int TT = F / 16, RPW = CQR2_RPW, LDX = Cfg::LDX, LD = S::LD, PW = RPW / 4, KS = F / 4;
  static_assert(F <= 32, "register budget of the Gram tiles");
  static_assert(Cfg::TOTAL * 8 <= 160 * 1024, "LDS budget");
  // early exits read state written by earlier launches only: the same for every workgroup
  if (a.stop_block && *a.stop_block < a.block_id) return;
  const int f = a.f_dev ? (int)*a.f_dev : a.f;
  if (gate_shut(a.gate) || f <= 0 || f > F) {
    state_send(a);
    return;
  }
  __shared__ __align__(16) double lds[Cfg::TOTAL];
  T* pan = reinterpret_cast<T*>(lds);            // pan[c*LDX + row]
  double* Gs = lds + Cfg::XD;                    // G, then R
  double* Ri = Gs + S::SIZE;                     // R^{-1}
  double* rowbuf = Ri + S::SIZE;
  double* dgs = rowbuf + 24 * F;
  double* red = Gs;                              // wave fold, before the Cholesky takes the area
  double* r1d = lds + Cfg::XD + Cfg::WORK;       // R1's diagonal
  int* sx = reinterpret_cast<int*>(r1d + F);
  double* R1s = r1d + F + 8;                     // R1 (the closing QR needs all of it)
  T* Ws = reinterpret_cast<T*>(R1s + S::SIZE);   // PROJ: the folded W, Ws[a*LDW + c]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, g = lane >> 4;
  const T* X = reinterpret_cast<const T*>(a.X);
  const int64_t rb = (int64_t)blockIdx.x * RPW;
  const unsigned G = gridDim.x;
  const int ff = f * f;
  const bool lead = blockIdx.x == 0;
  State* st = a.st;
  const int64_t zoff = (a.stop_test && a.wlog) ? a.wlog[a.block_id] : 0;
  // everything read from earlier launches is requested now, ahead of the
  // barriers (after them the caches are invalidated and each read would be
  // a round trip on the critical path)
  const int paired = st->paired;
  const double tol = st->tol;
  const int lp_mode = st->lp_mode;
  const double eps_g = st->eps;
  const int nonf_g = st->nonfinite;
  const int dead0 = (lane < f && !a.fresh) ? a.dead[lane] : 0;
  double pv0[8];
  float mv0[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t i = lane + 64 * q;
    const bool in = a.norm_parts && wv == 0 && i < a.n_norm;
    pv0[q] = in ? a.norm_parts[i] : 0.0;
    mv0[q] = (in && a.max_parts) ? a.max_parts[i] : 0.0f;
  }
  {                                              // stage the panel (zero outside rows x f), all loads in flight
    constexpr int NIT = F * RPW / 256;
    T xv[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
      const int idx = tid + 256 * q;
      const int c = idx / RPW, rl = idx - c * RPW;
      const int64_t row = rb + rl;
      xv[q] = (c < f && row < a.rows) ? X[(int64_t)c * a.ldx + row] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
      const int idx = tid + 256 * q;
      const int c = idx / RPW, rl = idx - c * RPW;
      pan[c * LDX + rl] = xv[q];
    }
  }
  // this thread's elements of the packed upper triangle of G: p = tid + 256 e
  // is (prr, pcc) with p = pcc (pcc + 1) / 2 + prr, prr <= pcc
  constexpr int EPT = (F * (F + 1) / 2 + 255) / 256;
  const int np = f * (f + 1) / 2;
  int prr[EPT], pcc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int p = tid + 256 * e;
    int c = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    while (c > 0 && c * (c + 1) / 2 > p) --c;
    while ((c + 1) * (c + 2) / 2 <= p) ++c;
    pcc[e] = c;
    prr[e] = p - c * (c + 1) / 2;
  }
  uint64_t dmask = 0;
  double eps_l = 0.0;
  bool nonf_l = false;
  unsigned bars = 0;                             // barriers passed (their arrival targets are multiples of G)
  const uint64_t wticks = a.wait_ticks ? a.wait_ticks : CQR2_WAIT_TICKS;
  const int wb = PROJ ? (int)*a.w_dev : 0;       // basis width (uniform; <= Cfg::WMAX by the host's bound)
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();                             // panel (pass 1: Z1) complete
    if constexpr (PROJ) {
      if (wb > 0 && wb <= Cfg::WMAX) {
        // block Gram-Schmidt: W = Qb^T Y over all rows, Y -= Qb W
        typedef Mfma<T> MT;
        constexpr int LDW = Cfg::LDW, NCH = RPW / 16;
        const T* Qb = reinterpret_cast<const T*>(a.Qb);
        T* WP = reinterpret_cast<T*>(a.wparts);
        T* myWP = WP + (int64_t)blockIdx.x * CQR2_PROJ_WMAX * F;
        const int TA = (wb + 15) / 16;
        // (1) this panel's W_g = Q_g^T Y_g (T-precision MFMA), tile (ta, tc)
        //     per wave in turn; the 16-row chunks' Q loads all in flight
        for (int tile = wv; tile < TA * TT; tile += 4) {
          const int ta = tile / TT, tc = tile - ta * TT;
          const int acol = 16 * ta + r;
          const bool aok = acol < wb;
          const T* qc = Qb + (int64_t)(aok ? acol : 0) * a.ldqb + rb;
          typename MT::acc_t acc = MT::zero();
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            V4<T> q4[NCH / 2];
#pragma unroll
            for (int c8 = 0; c8 < NCH / 2; ++c8) {
              const int ch = h * (NCH / 2) + c8;
              const int64_t r0 = rb + 16 * ch + 4 * g;       // this lane's four rows
              if (aok && r0 + 3 < a.rows) {
                q4[c8] = ld4(qc + 16 * ch + 4 * g);
              } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) q4[c8].v[t] = (aok && r0 + t < a.rows) ? qc[16 * ch + 4 * g + t] : (T)0;
              }
            }
#pragma unroll
            for (int c8 = 0; c8 < NCH / 2; ++c8) {
              const int ch = h * (NCH / 2) + c8;
#pragma unroll
              for (int t = 0; t < 4; ++t)
                acc = MT::op(q4[c8].v[t], pan[(16 * tc + r) * LDX + 16 * ch + 4 * g + t], acc);
            }
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int am = 16 * ta + MT::row(g, e), cn = 16 * tc + r;
            if (am < wb && cn < f) myWP[am * F + cn] = (T)acc[e];
          }
        }
        grid_barrier(a.counter, (++bars) * G + a.wait_extra, st, wticks);
        // (2) W = sum of the G partials in order g = 0, 1, ... (every
        //     workgroup the same), four consecutive columns per load; a
        //     thread takes its groups of four one after another, sixteen
        //     partials' loads in flight
        {
          const int nq = wb * (F / 4);                 // groups of four elements of W
          for (int qi = tid; qi < nq; qi += 256) {
            V4<T> sw;
#pragma unroll
            for (int e = 0; e < 4; ++e) sw.v[e] = (T)0;
            for (unsigned g0 = 0; g0 < G; g0 += 16) {
              V4<T> v[16];
#pragma unroll
              for (int i = 0; i < 16; ++i) {
                if (g0 + i < G) {
                  v[i] = ld4(WP + (int64_t)(g0 + i) * CQR2_PROJ_WMAX * F + 4 * qi);
                } else {
#pragma unroll
                  for (int e = 0; e < 4; ++e) v[i].v[e] = (T)0;
                }
              }
#pragma unroll
              for (int i = 0; i < 16; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) sw.v[e] += v[i].v[e];
            }
            const int am = qi / (F / 4), c4 = 4 * (qi - am * (F / 4));
#pragma unroll
            for (int e = 0; e < 4; ++e) Ws[am * LDW + c4 + e] = (c4 + e < f) ? sw.v[e] : (T)0;
          }
        }
        __syncthreads();
        // (3) Y_g -= Q_g W in place: wave wv takes output tiles (row tile,
        //     column tile) in turn, K = wb in steps of 4, eight steps' loads
        //     in flight
        for (int tile = wv; tile < NCH * TT; tile += 4) {
          const int rt = tile / TT, tc = tile - rt * TT;
          const int64_t row = rb + 16 * rt + r;
          const bool rok = row < a.rows;
          typename MT::acc_t acc = MT::zero();
          for (int s0 = 0; s0 < wb; s0 += 32) {
            T qv[8], wv8[8];
#pragma unroll
            for (int st8 = 0; st8 < 8; ++st8) {
              const int ak = s0 + 4 * st8 + g;
              const bool kok = ak < wb;
              qv[st8] = (kok && rok) ? Qb[(int64_t)ak * a.ldqb + row] : (T)0;
              wv8[st8] = kok ? Ws[ak * LDW + 16 * tc + r] : (T)0;
            }
#pragma unroll
            for (int st8 = 0; st8 < 8; ++st8) acc = MT::op(qv[st8], wv8[st8], acc);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int lr = 16 * rt + MT::row(g, e), cc = 16 * tc + r;
            pan[cc * LDX + lr] = (T)(pan[cc * LDX + lr] - acc[e]);
          }
        }
        __syncthreads();
      }
    }
    typename MF::acc_t acc[TT][TT];
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int u = 0; u < TT; ++u) acc[t][u] = MF::zero();
#pragma unroll
    for (int k0 = 0; k0 < PW; k0 += 16) {        // wave wv: panel rows [wv*PW, (wv+1)*PW)
      const int kr = wv * PW + k0 + 4 * g;
      V4<double> av[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) av[t].v[e] = (double)pan[(16 * t + r) * LDX + kr + e];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
          for (int u = t; u < TT; ++u) acc[t][u] = MF::op(av[t].v[v], av[u].v[v], acc[t][u]);
    }
    for (int w = 0; w < 4; ++w) {                // fold the 4 waves (fixed order)
      if (wv == w) {
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
          for (int u = t; u < TT; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              double* qq = &red[((t * TT + u) * 4 + e) * 64 + lane];
              *qq = (w == 0) ? acc[t][u][e] : *qq + acc[t][u][e];
            }
      }
      __syncthreads();
    }
    double sum[EPT];                             // G's upper triangle, kept for a second Cholesky
    // one workgroup: its wave fold is the Gram (the same sums as the fold of
    // a single partial), no partial and no barrier.  Compiled into the
    // 16-column form only: the 32-column form's code sits near the size of
    // the instruction cache, and the branch alone slowed it measurably.
    bool one = false;
    if constexpr (!PROJ && F <= 16) one = G == 1;
    if (one) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        sum[e] = 0.0;
        if (tid + 256 * e < np) {
          const int i = prr[e], jj = pcc[e], il = i & 15;
          sum[e] += red[(((i >> 4) * TT + (jj >> 4)) * 4 + (il >> 2)) * 64 + (il & 3) * 16 + (jj & 15)];
        }
      }
      __syncthreads();                           // the fold area (Gs) read before Gs is written
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if (tid + 256 * e < np) {
          Gs[prr[e] * LD + pcc[e]] = sum[e];
          Gs[pcc[e] * LD + prr[e]] = sum[e];
        }
      }
    } else {
      // partials hold G's upper triangle packed column by column: (i, j), i <= j, at j(j+1)/2 + i
      double* pp = a.parts + (int64_t)pass * G * ff;
      double* Pw = pp + (int64_t)blockIdx.x * np;  // this workgroup's partial
      for (int idx = tid; idx < TT * TT * 256; idx += 256) {
        const int l = idx & 63, e = (idx >> 6) & 3, tu = idx >> 8;
        const int t = tu / TT, u = tu - t * TT;
        if (u < t) continue;
        const int i = 16 * t + MF::row(l >> 4, e), jj = 16 * u + (l & 15);
        if (i <= jj && jj < f) Pw[jj * (jj + 1) / 2 + i] = red[idx];
      }
      grid_barrier(a.counter, (++bars) * G + a.wait_extra, st, wticks);
      {                                            // all partials, order b = 0, 1, ...
        constexpr int PB = 16;
#pragma unroll
        for (int e = 0; e < EPT; ++e) sum[e] = 0.0;
        for (unsigned b = 0; b < G; b += PB) {
          double v[EPT][PB];
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int idx = tid + 256 * e;
            const bool ok = idx < np;
#pragma unroll
            for (int q = 0; q < PB; ++q) v[e][q] = (ok && b + q < G) ? pp[(int64_t)(b + q) * np + idx] : 0.0;
          }
#pragma unroll
          for (int e = 0; e < EPT; ++e)
#pragma unroll
            for (int q = 0; q < PB; ++q) sum[e] += v[e][q];
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          if (tid + 256 * e < np) {
            Gs[prr[e] * LD + pcc[e]] = sum[e];
            Gs[pcc[e] * LD + prr[e]] = sum[e];
          }
        }
      }
    }
    if (pass == 0 && a.norm_parts && wv == 0) {  // ||A||_F from the sketch partials (fixed order)
      double s = 0.0;
      float mx = 0.0f;
#pragma unroll
      for (int q = 0; q < 8; ++q) {             // the first 512, prefetched
        if (lane + 64 * q < a.n_norm) s += pv0[q];
        mx = fmaxf(mx, mv0[q]);
      }
      for (int64_t i0 = 64 * 8; i0 < a.n_norm; i0 += 64 * 8) {
        double pv[8];
        float mv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int64_t i = i0 + lane + 64 * q;
          pv[q] = i < a.n_norm ? a.norm_parts[i] : 0.0;
          mv[q] = (a.max_parts && i < a.n_norm) ? a.max_parts[i] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (i0 + lane + 64 * q < a.n_norm) s += pv[q];
          mx = fmaxf(mx, mv[q]);
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        mx = fmaxf(mx, __shfl_xor(mx, off));
      }
      nonf_l = !(s < INFINITY);
      eps_l = nonf_l ? 0.0 : tol * sqrt(s);
      if (lead && lane == 0) {
        st->normsq = s;
        st->nonfinite = nonf_l ? 1 : 0;
        st->eps = eps_l;
        st->lp_scale = lp_scale_of(mx, lp_mode);
      }
    }
    uint64_t dmask_in = dmask;
    if (pass == 0) dmask_in = __ballot(dead0 != 0);
    __syncthreads();
    int nfl = 0;
    // the branch-free elimination first; the full pivot rules only when it
    // meets a dead column or a pivot at or below the floor
    const bool fast = dmask_in == 0ull && chol_inv_fast<F>(Gs, Ri, rowbuf, dgs, f);
    if (!fast) {
      if (dmask_in == 0ull) {                    // Gs was overwritten: G again from the registers
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          if (tid + 256 * e < np) {
            Gs[prr[e] * LD + pcc[e]] = sum[e];
            Gs[pcc[e] * LD + prr[e]] = sum[e];
          }
        }
        __syncthreads();
      }
      [[clang::noinline]] chol_inv<F>(Gs, Ri, rowbuf, dgs, f, dmask_in, pass == 0, &dmask, &nfl);
    } else {
      dmask = 0ull;
    }
    if (lead) {
      double* Ro = pass == 0 ? a.R1 : a.R2;
      double* Rio = pass == 0 ? a.R1inv : a.R2inv;
      for (int idx = tid; idx < ff; idx += 256) {
        const int c = idx / f, rr = idx - c * f;  // element (rr, c) at c*f + rr
        if (Ro) Ro[idx] = Gs[rr * LD + c];
        if (Rio) Rio[idx] = Ri[rr * LD + c];
      }
      if (a.count_floors && tid == 0 && nfl) atomicAdd(&st->floored, nfl);
      if (pass == 1 && tid < f) a.dead[tid] = (int32_t)((dmask >> tid) & 1ull);
    }
    if (pass == 0) {
      if (tid < F) r1d[tid] = Gs[tid * LD + tid];
      if (a.close_qr)
        for (int idx = tid; idx < S::SIZE; idx += 256) R1s[idx] = Gs[idx];
      // Z1 = X R1^{-1} in place: wave wv takes 16-row tiles wv, wv + 4, ...
      // (each tile's rows are read whole before they are written)
      for (int rt = wv; rt < RPW / 16; rt += 4) {
        double av[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) av[kk] = (double)pan[(4 * kk + g) * LDX + 16 * rt + r];
        typename MF::acc_t z[TT];
#pragma unroll
        for (int u = 0; u < TT; ++u) z[u] = MF::zero();
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
#pragma unroll
          for (int u = 0; u < TT; ++u) z[u] = MF::op(av[kk], Ri[(4 * kk + g) * LD + 16 * u + r], z[u]);
#pragma unroll
        for (int u = 0; u < TT; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) pan[(16 * u + r) * LDX + 16 * rt + MF::row(g, e)] = (T)z[u][e];
      }
    }
  }
  // stop test (Alg. 1) on wave 0 of every workgroup: first column whose
  // |T(c,c)| <= eps
  int keep = f;
  if (a.stop_test) {
    if (wv == 0) {
      const int j = lane;
      const bool mine = j < f;
      const double eps = a.norm_parts ? eps_l : eps_g;
      const bool nonf = a.norm_parts ? nonf_l : (nonf_g != 0);
      double d = 0.0;
      bool hit = false;
      if (mine) {
        d = ((dmask >> j) & 1ull) ? 0.0 : Gs[j * LD + j] * r1d[j];
        hit = ((d <= eps) && (!paired || ((a.col0 + j) & 1) == 0)) || nonf;
      }
      const unsigned long long mask = __ballot(hit);
      const int kp = mask ? (int)__ffsll((long long)mask) - 1 : f;
      if (lane == 0) sx[0] = kp;
      if (lead) {
        if (mine && j <= kp) a.diag_log[a.col0 + j] = d;
        const double dk = __shfl(d, kp & 63);
        if (j == 0) {
          if (mask != 0ull) st->d_stop = dk;
          const bool stop = (mask != 0ull) || (a.col0 + f >= a.n);
          a.acc[a.block_id] = kp;
          const int64_t wn = zoff + kp;
          a.wlog[a.block_id + 1] = wn;
          st->rank = wn;
          if (stop) st->stop_block = a.block_id;
        }
      }
    }
    __syncthreads();
    keep = sx[0];
  }
  // Q = Z1 R2^{-1} for the kept columns (the apply's tile order and sums)
  T* Q = reinterpret_cast<T*>(a.Q);
  for (int rt = wv; rt < RPW / 16; rt += 4) {
    double av[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) av[kk] = (double)pan[(4 * kk + g) * LDX + 16 * rt + r];
    typename MF::acc_t z[TT];
#pragma unroll
    for (int u = 0; u < TT; ++u) z[u] = MF::zero();
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
      for (int u = 0; u < TT; ++u) z[u] = MF::op(av[kk], Ri[(4 * kk + g) * LD + 16 * u + r], z[u]);
#pragma unroll
    for (int u = 0; u < TT; ++u) {
      const int col = 16 * u + r;
      if (col >= keep) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = rb + 16 * rt + MF::row(g, e);
        if (row < a.rows) Q[(zoff + col) * a.ldq + row] = (T)z[u][e];
      }
    }
  }
  if (a.reuse_counter && tid == 0) {            // every workgroup is past its last barrier: reset for the next launch
    if (atomicAdd(a.counter, 1u) == (bars + 1) * G - 1) atomicExch(a.counter, 0u);
  }
  if (!a.close_qr) return;
  // U = Uq Qh at the end runs over this workgroup's rows in 16-row tiles,
  // four per wave at a time; Uq (the basis, final before this launch) is
  // read now for the first four, so their loads overlap the QR of R^T
  const T* Uq = reinterpret_cast<const T*>(a.Uq);
  const int64_t chunk = (((a.m_u + G - 1) / G + 15) / 16) * 16;
  const int64_t u0 = (int64_t)blockIdx.x * chunk, u1 = min(a.m_u, u0 + chunk);
  constexpr int NB = 4;
  T xa[NB][KS];
  auto load_u = [&](int64_t t0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t arow = t0 + 64 * b + r;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = 4 * kk + g;
        xa[b][kk] = (arow < u1 && k < f) ? Uq[(int64_t)k * a.ldq_u + arow] : (T)0;
      }
    }
  };
  if (a.Uout) load_u(u0 + 16 * wv);
  // closing QR (Alg. 2, QR(R^T)), redundantly on every workgroup
  __syncthreads();                               // the panel and R2^{-1} are free
  double* B0 = lds;
  double* B1 = lds + S::SIZE;
  double* B2 = lds + 2 * S::SIZE;
  double* B3 = Ri;
  double* Qs = Gs;                               // Qh (R2 is dead once M is formed)
  lds_gemm<F, false, false>(Gs, R1s, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });   // M = R2 R1
  __syncthreads();
  lds_gemm<F, false, true>(B0, B0, [&](int i, int jj, double v) { B1[i * LD + jj] = v; });     // M M^T
  __syncthreads();
  uint64_t dm1 = 0ull, dm2 = 0ull;
  int nf1 = 0, nf2 = 0;
  if (!chol_inv_fast<F>(B1, B2, rowbuf, dgs, f)) {
    lds_gemm<F, false, true>(B0, B0, [&](int i, int jj, double v) { B1[i * LD + jj] = v; });
    __syncthreads();
    [[clang::noinline]] chol_inv<F>(B1, B2, rowbuf, dgs, f, 0ull, 1, &dm1, &nf1);                                 // Rh1, Rh1^{-1}
  }
  lds_gemm<F, true, false>(B0, B2, [&](int i, int jj, double v) { B3[i * LD + jj] = v; });     // Z = M^T Rh1^{-1}
  __syncthreads();
  lds_gemm<F, true, false>(B3, B3, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });     // Z^T Z
  __syncthreads();
  if (!(dm1 == 0ull && chol_inv_fast<F>(B0, B2, rowbuf, dgs, f))) {
    if (dm1 == 0ull) {
      lds_gemm<F, true, false>(B3, B3, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });
      __syncthreads();
    }
    [[clang::noinline]] chol_inv<F>(B0, B2, rowbuf, dgs, f, dm1, 0, &dm2, &nf2);                                  // Rh2, Rh2^{-1}
  }
  lds_gemm<F, false, false>(B3, B2, [&](int i, int jj, double v) {                            // Qh = Z Rh2^{-1}
    Qs[i * LD + jj] = v;
    if (lead && i < f && jj < f) a.Qh_out[(int64_t)jj * f + i] = v;
  });
  T* Dout = reinterpret_cast<T*>(a.Dout);
  if (lead)
    lds_gemm<F, false, false>(B0, B1, [&](int i, int jj, double v) {                          // Rh = Rh2 Rh1
      if (i < f && jj < f) Dout[(int64_t)i * a.ldd + jj] = (T)v;
    });
  if (lead && a.count_floors && tid == 0 && nf1 + nf2) atomicAdd(&st->floored, nf1 + nf2);
  state_send(a);                                 // the control block is final here
  if (!a.Uout) return;
  __syncthreads();                               // Qh complete
  // U = Uq Qh (the apply's operand order and sums)
  T* U = reinterpret_cast<T*>(a.Uout);
  for (int64_t t0 = u0 + 16 * wv; t0 < u1; t0 += 64 * NB) {
    if (t0 != u0 + 16 * wv) load_u(t0);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      typename MF::acc_t z[TT];
#pragma unroll
      for (int u = 0; u < TT; ++u) z[u] = MF::zero();
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
#pragma unroll
        for (int u = 0; u < TT; ++u) z[u] = MF::op((double)xa[b][kk], Qs[(4 * kk + g) * LD + 16 * u + r], z[u]);
#pragma unroll
      for (int u = 0; u < TT; ++u) {
        const int col = 16 * u + r;
        if (col >= f) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = t0 + 64 * b + MF::row(g, e);
          if (row < u1) U[col * a.ldu + row] = (T)z[u][e];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Z = X W (FP64 MFMA, rounded to T) for one or two jobs (blockIdx.y):
// X column-major rows x f (ldx), W f x f FP64 (element (i,j) at j*f + i,
// any shape), Z column-major (ldz), columns zoff .. zoff+ncols-1 written.
// With zoff_dev / ncols_dev the offset and count are read on the device
// (the basis append: zoff = wlog[block], ncols = acc[block]).  Up to 32
// columns a workgroup stages W once and takes 64-row blocks grid-stride, the
// next block's rows of X loading while the current block is multiplied;
// wider, it takes one block (the launch covers every block).  Each wave computes 16
// complete rows and reads a block's rows before it writes them (no other
// workgroup touches the block), so Z may alias X when zoff = 0 and ldz = ldx.
// ---------------------------------------------------------------------------
struct ApplyJob {
  const void* X;
  int64_t ldx;
  void* Z;
  int64_t ldz;
  const double* W;
  int64_t rows, zoff;
  int f, ncols;
  const int64_t* zoff_dev;
  const int32_t* ncols_dev;
  const int64_t* f_dev;          // if set: f = ncols = *f_dev (closing steps)
};

template <typename T, int F>
__global__ __launch_bounds__(256) void k_apply(ApplyJob j0, ApplyJob j1,
                                               const int32_t* __restrict__ stop_block, int block_id,
                                               Gate gate) {
  typedef Mfma<double> MF;
  constexpr int TT = F / 16, LD = F + 1, KS = F / 4;
  if (stop_block && *stop_block < block_id) return;
  if (gate_shut(gate)) return;
  const ApplyJob jb = blockIdx.y == 0 ? j0 : j1;
  const int64_t nrb = (jb.rows + 63) / 64;      // 64-row blocks, taken grid-stride
  int64_t rb = blockIdx.x;
  if (rb >= nrb) return;
  __shared__ double Wl[F * LD];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, g = lane >> 4;
  const int f = jb.f_dev ? (int)*jb.f_dev : jb.f;
  if (f > F) return;                    // cannot happen: the launch width bounds the rank
  const int ncols = jb.f_dev ? f : (jb.ncols_dev ? jb.ncols_dev[block_id] : jb.ncols);
  const int64_t zoff = jb.zoff_dev ? jb.zoff_dev[block_id] : jb.zoff;
  const T* X = reinterpret_cast<const T*>(jb.X);
  T* Z = reinterpret_cast<T*>(jb.Z);
  // this wave's 16 rows of block rbk (lane r holds row 16*wv + r)
  T xa[KS];
  auto load_x = [&](int64_t rbk) {
    const int64_t arow = rbk * 64 + 16 * wv + r;
    const bool aok = arow < jb.rows;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int k = 4 * kk + g;
      xa[kk] = (aok && k < f) ? X[(int64_t)k * jb.ldx + arow] : (T)0;
    }
  };
  // the first block's X rows requested first, then W: both round trips overlap
  load_x(rb);
  if constexpr (F <= 64) {
    stage_small<F>({jb.W}, f, {Wl}, LD);
  } else {
    // 16 loads per thread in flight at a time, coalesced down each column of W
    for (int q0 = 0; q0 < F * F / 256; q0 += 16) {
      double wq[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * (q0 + q);
        const int jj = idx / F, i = idx - jj * F;
        wq[q] = (i < f && jj < f) ? jb.W[(int64_t)jj * f + i] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * (q0 + q);
        const int jj = idx / F, i = idx - jj * F;
        Wl[i * LD + jj] = wq[q];
      }
    }
  }
  __syncthreads();
  auto block = [&](int64_t rbk) {                // Z rows of block rbk from xa
    double a[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) a[kk] = (double)xa[kk];
    if constexpr (F <= 32)                       // the next block's rows in flight
      if (rbk + gridDim.x < nrb) load_x(rbk + gridDim.x);
    const int64_t rbase = rbk * 64 + 16 * wv;
    typename MF::acc_t z[TT];
#pragma unroll
    for (int u = 0; u < TT; ++u) z[u] = MF::zero();
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
      for (int u = 0; u < TT; ++u) z[u] = MF::op(a[kk], Wl[(4 * kk + g) * LD + 16 * u + r], z[u]);
#pragma unroll
    for (int u = 0; u < TT; ++u) {
      const int col = 16 * u + r;
      if (col >= ncols) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = rbase + MF::row(g, e);
        if (row < jb.rows) Z[(zoff + col) * jb.ldz + row] = (T)z[u][e];
      }
    }
  };
  if constexpr (F <= 32) {
    for (; rb < nrb; rb += gridDim.x) block(rb);
  } else {
    // wider: one block per workgroup (in a loop the compiler would keep the
    // loop-invariant W operands in registers, more than there are)
    block(rb);
  }
}

// k_apply for 64 < f <= 128 with the output columns split over workgroups
// (blockIdx.z: a slice of 32), each staging only its 32 columns of W (33 KB
// of LDS instead of 132 KB, so four workgroups fit a CU and the FP64 MFMA
// work spreads over four times as many CUs).  Each output element is
// formed by the same MFMA sequence as in k_apply, so the results are bit
// for bit the same.  Z must not alias X (a slice would overwrite columns
// another slice still reads).
template <typename T, int F>
__global__ __launch_bounds__(256) void k_apply_cols(ApplyJob j0, ApplyJob j1,
                                                    const int32_t* __restrict__ stop_block, int block_id,
                                                    Gate gate) {
  typedef Mfma<double> MF;
  constexpr int CW = 32, TC = CW / 16, LDC = CW + 1, KS = F / 4;
  if (stop_block && *stop_block < block_id) return;
  if (gate_shut(gate)) return;
  const ApplyJob jb = blockIdx.y == 0 ? j0 : j1;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  if (row0 >= jb.rows) return;
  const int f = jb.f_dev ? (int)*jb.f_dev : jb.f;
  if (f > F) return;                    // cannot happen: the launch width bounds the rank
  const int ncols = jb.f_dev ? f : (jb.ncols_dev ? jb.ncols_dev[block_id] : jb.ncols);
  const int c0 = (int)blockIdx.z * CW;
  if (c0 >= ncols) return;
  const int64_t zoff = jb.zoff_dev ? jb.zoff_dev[block_id] : jb.zoff;
  __shared__ double Wl[F * LDC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, g = lane >> 4;
  const T* X = reinterpret_cast<const T*>(jb.X);
  T* Z = reinterpret_cast<T*>(jb.Z);
  const int64_t rbase = row0 + 16 * wv;
  const int64_t arow = rbase + r;
  const bool aok = arow < jb.rows;
  T xa[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int k = 4 * kk + g;
    xa[kk] = (aok && k < f) ? X[(int64_t)k * jb.ldx + arow] : (T)0;
  }
  {                                     // W's slice: all loads in flight, coalesced down each column
    constexpr int NQ = F * CW / 256;
    double wq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = tid + 256 * q;
      const int jj = idx / F, i = idx - jj * F;
      wq[q] = (i < f && c0 + jj < f) ? jb.W[(int64_t)(c0 + jj) * f + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = tid + 256 * q;
      const int jj = idx / F, i = idx - jj * F;
      Wl[i * LDC + jj] = wq[q];
    }
  }
  double a[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) a[kk] = (double)xa[kk];
  __syncthreads();
  typename MF::acc_t z[TC];
#pragma unroll
  for (int u = 0; u < TC; ++u) z[u] = MF::zero();
#pragma unroll
  for (int kk = 0; kk < KS; ++kk)
#pragma unroll
    for (int u = 0; u < TC; ++u) z[u] = MF::op(a[kk], Wl[(4 * kk + g) * LDC + 16 * u + r], z[u]);
#pragma unroll
  for (int u = 0; u < TC; ++u) {
    const int col = c0 + 16 * u + r;
    if (col >= ncols) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = rbase + MF::row(g, e);
      if (row < jb.rows) Z[(zoff + col) * jb.ldz + row] = (T)z[u][e];
    }
  }
}

// ---------------------------------------------------------------------------
// Closing QR of Alg. 2 on one workgroup: M = R2 R1 (the two Cholesky factors
// of the CholeskyQR2 of C^T, f x f, element (i,j) at j*f + i; M = R2 when R1
// is null), then M^T = Qh Rh by CholeskyQR2 in FP64 (first pass floored,
// the second kills what stays non-positive).  Qh -> Qout (element (i,j) at
// j*f + i), Rh = Rh2 Rh1 -> Dout (type T, row-major, ldd).
// ---------------------------------------------------------------------------
template <typename T, int F>
__global__ __launch_bounds__(256) void k_small_qr(const double* __restrict__ R1g,
                                                  const double* __restrict__ R2g, int f,
                                                  double* __restrict__ Qout, T* __restrict__ Dout,
                                                  int64_t ldd, State* st, int count_floors, Gate gate,
                                                  const int64_t* __restrict__ f_dev) {
  typedef SmallCfg<F> S;
  constexpr int LD = S::LD;
  if (gate_shut(gate)) return;
  if (f_dev) f = (int)*f_dev;
  if (f > F) return;                    // cannot happen: the launch width bounds the rank
  __shared__ double B0[S::SIZE], B1[S::SIZE], B2[S::SIZE], B3[S::SIZE];
  __shared__ double rowbuf[24 * F], dgs[F];
  const int tid = threadIdx.x;
  if (R1g) stage_small<F, 2>({R2g, R1g}, f, {B1, B2}, LD);
  else stage_small<F>({R2g}, f, {B0}, LD);
  __syncthreads();
  if (R1g) {
    lds_gemm<F, false, false>(B1, B2, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });  // M
    __syncthreads();
  }
  lds_gemm<F, false, true>(B0, B0, [&](int i, int jj, double v) { B1[i * LD + jj] = v; });   // M M^T
  __syncthreads();
  uint64_t dm1, dm2;
  int nf1, nf2;
  chol_inv<F>(B1, B2, rowbuf, dgs, f, 0ull, 1, &dm1, &nf1);                 // Rh1 (B1), Rh1^{-1} (B2)
  lds_gemm<F, true, false>(B0, B2, [&](int i, int jj, double v) { B3[i * LD + jj] = v; });   // Z1 = M^T Rh1^{-1}
  __syncthreads();
  lds_gemm<F, true, false>(B3, B3, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });   // Z1^T Z1
  __syncthreads();
  chol_inv<F>(B0, B2, rowbuf, dgs, f, dm1, 0, &dm2, &nf2);                  // Rh2 (B0), Rh2^{-1} (B2)
  lds_gemm<F, false, false>(B3, B2, [&](int i, int jj, double v) {          // Qh = Z1 Rh2^{-1}
    if (i < f && jj < f) Qout[(int64_t)jj * f + i] = v;
  });
  lds_gemm<F, false, false>(B0, B1, [&](int i, int jj, double v) {          // Rh = Rh2 Rh1
    if (i < f && jj < f) Dout[(int64_t)i * ldd + jj] = (T)v;
  });
  if (count_floors && tid == 0 && nf1 + nf2) atomicAdd(&st->floored, nf1 + nf2);
}

// Stop test of Alg. 1 for blocks wider than 64 columns (one thread); the
// same rule as the tail of k_cholesky.
__global__ void k_decide(const double* __restrict__ R1, const double* __restrict__ R2,
                         const int32_t* __restrict__ dead, int f, int64_t col0, int64_t n,
                         State* st, int64_t* __restrict__ wlog, int32_t* __restrict__ acc,
                         double* __restrict__ diag_log, int block_id) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (st->stop_block < block_id) return;
  const double eps = st->eps;
  int keep = f;
  bool stop = false;
  for (int c = 0; c < f; ++c) {
    const double d = dead[c] ? 0.0 : R2[(int64_t)c * f + c] * R1[(int64_t)c * f + c];
    diag_log[col0 + c] = d;
    const bool lead = !st->paired || ((col0 + c) & 1) == 0;
    if ((d <= eps && lead) || st->nonfinite) { keep = c; stop = true; st->d_stop = d; break; }
  }
  if (col0 + f >= n) stop = true;
  acc[block_id] = keep;
  wlog[block_id + 1] = wlog[block_id] + keep;
  st->rank = wlog[block_id + 1];
  if (stop) st->stop_block = block_id;
}

// ||A||_F from per-workgroup partial sums (fixed order), eps = tol ||A||_F,
// and the scale of the low-precision copy from the per-workgroup max |A|.
__global__ void k_finish_norm(const double* __restrict__ parts, const float* __restrict__ maxp,
                              int64_t nparts, State* st) {
  __shared__ double red[256];
  __shared__ float redm[256];
  double a = 0.0;
  float mx = 0.0f;
  for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) {
    a += parts[i];
    if (maxp) mx = fmaxf(mx, maxp[i]);
  }
  red[threadIdx.x] = a;
  redm[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[threadIdx.x] += red[threadIdx.x + off];
      redm[threadIdx.x] = fmaxf(redm[threadIdx.x], redm[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double s = red[0];
    st->normsq = s;
    const bool bad = !(s < INFINITY);   // NaN or Inf
    st->nonfinite = bad ? 1 : 0;
    st->eps = bad ? 0.0 : st->tol * sqrt(s);
    st->lp_scale = lp_scale_of(redm[0], st->lp_mode);
  }
}

__global__ void k_init_state(State* st, double tol, int64_t* wlog, int nwlog, int32_t* dead,
                             int64_t ndead, int32_t* acc, int nacc, int lp_mode, int paired) {
  const StateInit a{st, tol, wlog, nwlog, dead, ndead, acc, nacc, lp_mode, paired};
  init_state_part(a, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// Fill with zeros (graph-safe replacement for memset).
template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

// R = R2 * R1 (upper triangular f x f, element (i,j) at j*f+i).  Writes the
// product transposed if transpose_out (element (i,j) of R at i*f + j).  One
// workgroup per 64 x 64 tile of the product (grid P x P, P = ceil(f / 64)),
// the sum over k restricted to [i0, j0 + 64) where both factors can be
// non-zero; tiles below the diagonal are zero.
__global__ __launch_bounds__(256) void k_trimul(const double* __restrict__ R2, const double* __restrict__ R1,
                                                int f, double* __restrict__ out, int transpose_out) {
  const int P = (f + 63) / 64, bi = blockIdx.x % P, bj = blockIdx.x / P;
  const int i0 = 64 * bi, j0 = 64 * bj;
  const int mi = (f - i0) < 64 ? f - i0 : 64, nj = (f - j0) < 64 ? f - j0 : 64;
  auto put = [&](int i, int j, double v) {
    if (transpose_out) out[(int64_t)(i0 + i) * f + j0 + j] = v;
    else out[(int64_t)(j0 + j) * f + i0 + i] = v;
  };
  if (bi > bj) {
    for (int idx = threadIdx.x; idx < mi * nj; idx += 256) put(idx / nj, idx % nj, 0.0);
    return;
  }
  const int k0 = i0, K = j0 + nj - i0;
  gmm64<true, true>(R2 + (int64_t)k0 * f + i0, f, R1 + (int64_t)j0 * f + k0, f, mi, nj, K, put);
}

// Generic 2-D copy with optional transpose and type conversion:
// dst(i, j) at dst[i*ldd + j] = src(i, j) (no transpose, src[i*lds + j]) or
// src(j, i) (transpose, src[j*lds + i]), for i < rows, j < cols.
template <typename Ts, typename Td>
__global__ void k_copy2d(const Ts* __restrict__ src, int64_t lds, Td* __restrict__ dst, int64_t ldd,
                         int64_t rows, int64_t cols, int transpose) {
  __shared__ Ts tile[32][33];
  const int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
  if (!transpose) {
    for (int ty = threadIdx.y; ty < 32; ty += blockDim.y) {
      const int64_t i = bi + ty, j = bj + threadIdx.x;
      if (i < rows && j < cols) dst[i * ldd + j] = (Td)src[i * lds + j];
    }
    return;
  }
  // dst(i,j) = src(j,i): read a 32x32 tile of src rows bj.., cols bi..
  for (int ty = threadIdx.y; ty < 32; ty += blockDim.y) {
    const int64_t sr = bj + ty, sc = bi + threadIdx.x;
    tile[ty][threadIdx.x] = (sr < cols && sc < rows) ? src[sr * lds + sc] : (Ts)0;
  }
  __syncthreads();
  for (int ty = threadIdx.y; ty < 32; ty += blockDim.y) {
    const int64_t i = bi + ty, j = bj + threadIdx.x;
    if (i < rows && j < cols) dst[i * ldd + j] = (Td)tile[threadIdx.x][ty];
  }
}

}  // namespace eodabe
