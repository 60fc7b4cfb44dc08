// Batched EOD-ABE for many small matrices (tiles): one workgroup factors a
// whole tile (Alg. 1 + Alg. 2, q = 0) with the same arithmetic as the
// single-matrix path (FP32 data, FP64 Grams, Cholesky with inverse), taking
// tiles from a device work queue until it is empty.  Tiles up to
// TILE_MAX x TILE_MAX; ranks up to TILE_RMAX are finished in the kernel
// (a tile whose rank goes above reports status TS_RANK and is left to the
// caller).  Ranks up to 64 close on LDS-resident FP64 matrices; wider ranks
// use the 2 x 2-blocked Cholesky with inverse on L2-resident ones.
#pragma once
#include "eodabe_kernels.hpp"

namespace eodabe {

constexpr int TILE_MAX = 1024;                 // largest tile side
constexpr int TILE_RMAX = 128;                 // rank finished inside the kernel
constexpr int TILE_BMAX = 64;                  // largest block width
constexpr int TILE_QW = TILE_RMAX + TILE_BMAX; // basis columns held (rank + one block)

enum TileStatus : int32_t { TS_OK = 0, TS_RANK = 1, TS_NONFINITE = 2, TS_CAPACITY = 3 };

struct TileDesc {
  const float* A;        // row-major h x w, leading dimension lda
  int64_t h, w, lda;
  int64_t out_off;       // element offset of this tile's outputs in the pool
  int64_t r_cap;         // output capacity: Ut r_cap x h, core r_cap x r_cap, Vt r_cap x w
  int32_t b;             // block width (<= TILE_BMAX)
  int32_t index;         // position in the caller's arrays
};

struct TileResult {
  int64_t rank;
  int32_t blocks;
  int32_t status;
  double norm;
};

// Scratch of one workgroup (floats unless marked).
struct TileSlot {
  static constexpr int64_t LD = TILE_MAX;                // leading dimension of tall buffers
  static constexpr int64_t OM = 0;                       // Omega^T rows, TILE_BMAX x LD
  static constexpr int64_t Y = OM + TILE_BMAX * LD;      // block, LD x TILE_BMAX
  static constexpr int64_t Q = Y + LD * TILE_BMAX;       // basis, LD x TILE_QW
  static constexpr int64_t CT = Q + LD * TILE_QW;        // C^T, LD x TILE_RMAX
  static constexpr int64_t VP = CT + LD * TILE_RMAX;     // V' of a wide tile, LD x TILE_RMAX
  static constexpr int64_t FLOATS = VP + LD * TILE_RMAX;
  // FP64 matrices after the floats: ranks <= 64 (64 x 64, column-major)
  static constexpr int64_t SM = 64 * 64;
  static constexpr int64_t R1 = 0, R2 = SM, QH = 2 * SM, DH = 3 * SM, QH2 = 4 * SM, DH2 = 5 * SM;
  // ranks 65..128 (128 x 128, row-major, leading dimension LB)
  static constexpr int LB = 128;
  static constexpr int64_t B2 = (int64_t)LB * LB;
  static constexpr int64_t BIG = 6 * SM;                 // 16 buffers of B2
  static constexpr int64_t DOUBLES = BIG + 16 * B2;
  static constexpr int64_t BYTES = FLOATS * 4 + DOUBLES * 8;
};

// LDS arena (doubles): the closing QR's 4 small matrices, its work area and
// diagonal, then 72 scalars that live across phases (||A||^2, R1 diagonal).
constexpr int TILE_SQR = 4 * SmallCfg<64>::SIZE + 24 * 64 + 64;
constexpr int TILE_LDS = TILE_SQR + 72;
// basis-phase carve: Gram/R, R^{-1}, Cholesky work, diagonal; W = Q^T Y
// (TILE_QW x TILE_BMAX) from 0; the reductions' fold buffer after both.
constexpr int TL_GS = 0, TL_RI = SmallCfg<64>::SIZE, TL_WORK = 2 * SmallCfg<64>::SIZE,
              TL_DGS = TL_WORK + 24 * 64, TL_W = 0, TL_FOLD = TILE_QW * TILE_BMAX, TL_FOLD_N = 16 * 256;
static_assert(TL_DGS + 64 <= TL_FOLD, "Cholesky carve below the fold buffer");
static_assert(CHOL128_LDS <= TILE_SQR && 128 * 129 <= TILE_SQR, "wide-rank closing inside the arena");
static_assert(TL_FOLD + TL_FOLD_N <= TILE_SQR, "basis carve inside the arena");

// ---------------------------------------------------------------------------
// Omega_j^T for the tile: rows j < f of column col0 + j, zero rows f..fpad-1.
// ---------------------------------------------------------------------------
__device__ void tile_omega(float* Om, int64_t ldk, int64_t n, int64_t col0, int f, int fpad,
                           uint32_t k0, uint32_t k1) {
  const int64_t nq = ldk / 4;
  for (int64_t idx = threadIdx.x; idx < (int64_t)fpad * nq; idx += 256) {
    const int j = (int)(idx / nq);
    const int64_t q = idx - (int64_t)j * nq;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (j < f && 4 * q < n) omega4(k0, k1, q, col0 + j, z);
#pragma unroll
    for (int e = 0; e < 4; ++e) Om[(int64_t)j * ldk + 4 * q + e] = (j < f && 4 * q + e < n) ? z[e] : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Y (m x nb, column-major ldy) = A B^T: A m x n row-major (lda), B given by
// its rows (row c at B + c*ldb, n entries, 16-byte aligned; rows >= nb read
// as zero), nb <= 64.  Wave w takes 64-row panels w, w+4, ...; each element
// of A is read once.  AL: rows of A 16-byte aligned (vector loads), else
// scalar loads.  ss (LDS, may be null): sum of squares of A.
// ---------------------------------------------------------------------------
template <bool AL>
__device__ __forceinline__ V4<float> tile_lda4(const float* p) {
  if constexpr (AL) {
    return ld4(p);
  } else {
    V4<float> v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v.v[e] = p[e];
    return v;
  }
}
// CTR = ceil(nb / 16) column tiles.  The loads of a full 16-column step are
// unconditional (rows of B past nb are read at row nb - 1 and zeroed by a
// select), and the steady state of the PF-deep ring has no branches, so
// each step waits only for its own loads.  Kept out of line, like the X^T Y
// routine below: the tile kernel is validated with these two as calls (an
// inlined build failed the batched parity test with an illegal address).
template <bool AL, int CTR>
__device__ __noinline__ void tile_rowprod_t(const float* A, int64_t lda, int64_t m, int64_t n, const float* B,
                                            int64_t ldb, int nb, float* Yb, int64_t ldy, double* ss,
                                            double* red) {
  typedef Mfma<float> MF;
  constexpr int RT = 4, PF = 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  const int64_t nfull = n / 16;
  double sq = 0.0;
  const float* bp[CTR];
  bool bval[CTR];
#pragma unroll
  for (int u = 0; u < CTR; ++u) {
    const int bc = 16 * u + r;
    bval[u] = bc < nb;
    bp[u] = B + (int64_t)(bval[u] ? bc : (nb > 0 ? nb - 1 : 0)) * ldb + 4 * g;
  }
  for (int64_t p0 = (int64_t)wv * 64; p0 < m; p0 += 256) {
    const float* ap[RT];
    bool aval[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int64_t row = p0 + 16 * t + r;
      aval[t] = row < m;
      ap[t] = A + (aval[t] ? row : (m - 1)) * lda + 4 * g;
    }
    MF::acc_t acc[RT][CTR];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < CTR; ++u) acc[t][u] = MF::zero();
    auto step = [&](const V4<float>(&av)[RT], const V4<float>(&bv)[CTR]) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int u = 0; u < CTR; ++u) acc[t][u] = MF::op(av[t].v[v], bv[u].v[v], acc[t][u]);
      if (ss) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
          if (aval[t])
#pragma unroll
            for (int v = 0; v < 4; ++v) sq += (double)av[t].v[v] * (double)av[t].v[v];
      }
    };
    V4<float> a[PF][RT], bq[PF][CTR];
    auto loadf = [&](int q, int64_t st) {        // a full step: no masks
      const int64_t k = 16 * st;
#pragma unroll
      for (int t = 0; t < RT; ++t) a[q][t] = tile_lda4<AL>(ap[t] + k);
#pragma unroll
      for (int u = 0; u < CTR; ++u) {
        const V4<float> v = ld4(bp[u] + k);
#pragma unroll
        for (int e = 0; e < 4; ++e) bq[q][u].v[e] = bval[u] ? v.v[e] : 0.f;
      }
    };
    if (nfull > 0) {
#pragma unroll
      for (int q = 0; q < PF; ++q) loadf(q, min((int64_t)q, nfull - 1));   // clamped, never used twice
      int64_t c = 0;
      for (; c + 2 * PF <= nfull; c += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          step(a[q], bq[q]);
          loadf(q, c + q + PF);
        }
      }
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        if (c + q < nfull) {
          step(a[q], bq[q]);
          if (c + q + PF < nfull) loadf(q, c + q + PF);
        }
      }
#pragma unroll
      for (int q = 0; q < PF; ++q)
        if (c + PF + q < nfull) step(a[q], bq[q]);
    }
    if (16 * nfull < n) {                        // ragged last step, masked
      const int64_t k = 16 * nfull;
      V4<float> at[RT], bt[CTR];
#pragma unroll
      for (int t = 0; t < RT; ++t) at[t] = ld4_masked(ap[t] + k, k + 4 * g, n);
#pragma unroll
      for (int u = 0; u < CTR; ++u) {
        const V4<float> v = ld4_masked(bp[u] + k, k + 4 * g, n);
#pragma unroll
        for (int e = 0; e < 4; ++e) bt[u].v[e] = bval[u] ? v.v[e] : 0.f;
      }
      step(at, bt);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < CTR; ++u) {
        const int64_t row = p0 + 16 * t + 4 * g;
        const int col = 16 * u + r;
        if (col < nb) {
          float* py = Yb + (int64_t)col * ldy + row;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e < m) py[e] = acc[t][u][e];
        }
      }
  }
  if (ss) {
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (lane == 0) red[wv] = sq;
    __syncthreads();
    if (threadIdx.x == 0) *ss = red[0] + red[1] + red[2] + red[3];
  }
  __syncthreads();
}
template <bool AL>
__device__ __forceinline__ void tile_rowprod(const float* A, int64_t lda, int64_t m, int64_t n, const float* B,
                                             int64_t ldb, int nb, float* Yb, int64_t ldy, double* ss,
                                             double* red) {
  const int ct = (nb + 15) / 16;
  if (ct <= 1) tile_rowprod_t<AL, 1>(A, lda, m, n, B, ldb, nb, Yb, ldy, ss, red);
  else if (ct == 2) tile_rowprod_t<AL, 2>(A, lda, m, n, B, ldb, nb, Yb, ldy, ss, red);
  else if (ct == 3) tile_rowprod_t<AL, 3>(A, lda, m, n, B, ldb, nb, Yb, ldy, ss, red);
  else tile_rowprod_t<AL, 4>(A, lda, m, n, B, ldb, nb, Yb, ldy, ss, red);
}

// ---------------------------------------------------------------------------
// Ct (n x r, column-major ldc) = A^T Q: A m x n row-major (lda), Q m x r
// column-major (ldq multiple of 4, 16-byte aligned columns), r <= 64.
// Wave w takes 64-column chunks of A (w, w+4, ...), so A is read once;
// element (j, i) of the product at i*ldc + j.  ss (LDS, may be null): sum
// of squares of A.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_colprod(const float* A, int64_t lda, int64_t m, int64_t n, const float* Q,
                                             int64_t ldq, int r, float* Ct, int64_t ldc, double* ss,
                                             double* red) {
  typedef Mfma<float> MF;
  constexpr int PF = 3;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, rr = lane & 15, g = lane >> 4;
  const int TR = (r + 15) / 16;
  const int64_t nsteps = (m + 15) / 16;
  double sq = 0.0;
  for (int64_t c0 = 64 * (int64_t)wv; c0 < n; c0 += 256) {
    MF::acc_t acc[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t][u] = MF::zero();
    // operands of a 16-row step loaded PF steps ahead (see tile_rowprod)
    V4<float> qv[PF][4];
    float av[PF][4][4];
    auto load = [&](int q, int64_t st) {
      const int64_t kr = 16 * st + 4 * g;
      const bool full = kr + 4 <= m;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int qc = 16 * t + rr;
        const float* qp = Q + (int64_t)qc * ldq + kr;
        if (t < TR && qc < r) qv[q][t] = full ? ld4(qp) : ld4_masked(qp, kr, m);
        else qv[q][t] = V4<float>{{0.f, 0.f, 0.f, 0.f}};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t ac = c0 + 16 * u + rr;
#pragma unroll
        for (int e = 0; e < 4; ++e) av[q][u][e] = (ac < n && kr + e < m) ? A[(kr + e) * lda + ac] : 0.f;
      }
    };
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (q < nsteps) load(q, q);
    for (int64_t c = 0; c < nsteps; c += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        if (c + q < nsteps) {
          if (ss) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int e = 0; e < 4; ++e) sq += (double)av[q][u][e] * (double)av[q][u][e];
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (t < TR)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[t][u] = MF::op(qv[q][t].v[v], av[q][u][v], acc[t][u]);
          if (c + q + PF < nsteps) load(q, c + q + PF);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < TR) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t j = c0 + 16 * u + rr;
          if (j < n) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int i = 16 * t + 4 * g + e;
              if (i < r) Ct[(int64_t)i * ldc + j] = acc[t][u][e];
            }
          }
        }
      }
    }
  }
  if (ss) {
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (lane == 0) red[wv] = sq;
    __syncthreads();
    if (threadIdx.x == 0) *ss = red[0] + red[1] + red[2] + red[3];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// out (LDS or global, row-major, leading dimension ldo) = X^T Y in FP64: X
// m x wx and Y m x wy column-major (ldx, ldy multiples of 4, 16-byte aligned
// columns; columns beyond wx / wy read as zero), wx, wy <= 64.  Waves split
// the rows (16-row steps, interleaved) and accumulate every 16 x 16 tile of
// the product at once; the partial tiles are folded in wave order through
// red (16 * 256 doubles, disjoint from out).  TX, TY: tile counts of X and
// Y; full steps load without branches (clamped columns zeroed by a select).
// ---------------------------------------------------------------------------
template <int TX, int TY>
__device__ __noinline__ void tile_xty_t(const float* X, int64_t ldx, int wx, const float* Yb, int64_t ldy,
                                        int wy, int64_t m, double* out, int ldo, double* red) {
  typedef Mfma<double> MF;
  constexpr int PF = 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  MF::acc_t acc[TX][TY];
#pragma unroll
  for (int t = 0; t < TX; ++t)
#pragma unroll
    for (int u = 0; u < TY; ++u) acc[t][u] = MF::zero();
  const float* xb[TX];
  const float* yb0[TY];
  bool xval[TX], yval[TY];
#pragma unroll
  for (int t = 0; t < TX; ++t) {
    const int c = 16 * t + r;
    xval[t] = c < wx;
    xb[t] = X + (int64_t)(xval[t] ? c : (wx > 0 ? wx - 1 : 0)) * ldx + 4 * g;
  }
#pragma unroll
  for (int u = 0; u < TY; ++u) {
    const int c = 16 * u + r;
    yval[u] = c < wy;
    yb0[u] = Yb + (int64_t)(yval[u] ? c : (wy > 0 ? wy - 1 : 0)) * ldy + 4 * g;
  }
  auto step = [&](const V4<float>(&xa)[TX], const V4<float>(&ya)[TY]) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < TX; ++t)
#pragma unroll
        for (int u = 0; u < TY; ++u) acc[t][u] = MF::op((double)xa[t].v[v], (double)ya[u].v[v], acc[t][u]);
  };
  // this wave's 16-row steps start at 16 wv + 64 s; a step is full when all
  // its 16 rows are < m
  const int64_t nfull = m >= 16 * (int64_t)wv + 16 ? (m - 16 * (int64_t)wv - 16) / 64 + 1 : 0;
  V4<float> xa[PF][TX], ya[PF][TY];
  auto loadf = [&](int q, int64_t st) {
    const int64_t k = 16 * (int64_t)wv + 64 * st;
#pragma unroll
    for (int t = 0; t < TX; ++t) {
      const V4<float> v = ld4(xb[t] + k);
#pragma unroll
      for (int e = 0; e < 4; ++e) xa[q][t].v[e] = xval[t] ? v.v[e] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < TY; ++u) {
      const V4<float> v = ld4(yb0[u] + k);
#pragma unroll
      for (int e = 0; e < 4; ++e) ya[q][u].v[e] = yval[u] ? v.v[e] : 0.f;
    }
  };
  if (nfull > 0) {
#pragma unroll
    for (int q = 0; q < PF; ++q) loadf(q, min((int64_t)q, nfull - 1));
    int64_t c = 0;
    for (; c + 2 * PF <= nfull; c += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        step(xa[q], ya[q]);
        loadf(q, c + q + PF);
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      if (c + q < nfull) {
        step(xa[q], ya[q]);
        if (c + q + PF < nfull) loadf(q, c + q + PF);
      }
    }
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (c + PF + q < nfull) step(xa[q], ya[q]);
  }
  {
    const int64_t k = 16 * (int64_t)wv + 64 * nfull;   // this wave's ragged step, if any
    if (k < m) {
      const int64_t kr = k + 4 * g;
      V4<float> xt[TX], yt[TY];
#pragma unroll
      for (int t = 0; t < TX; ++t) {
        const V4<float> v = ld4_masked(xb[t] + k, kr, m);
#pragma unroll
        for (int e = 0; e < 4; ++e) xt[t].v[e] = xval[t] ? v.v[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < TY; ++u) {
        const V4<float> v = ld4_masked(yb0[u] + k, kr, m);
#pragma unroll
        for (int e = 0; e < 4; ++e) yt[u].v[e] = yval[u] ? v.v[e] : 0.f;
      }
      step(xt, yt);
    }
  }
  // fold the waves in order
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int t = 0; t < TX; ++t)
#pragma unroll
        for (int u = 0; u < TY; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            double* q = &red[((t * TY + u) * 4 + e) * 64 + lane];
            *q = (w == 0) ? acc[t][u][e] : *q + acc[t][u][e];
          }
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < TX * TY * 256; idx += 256) {
    const int l = idx & 63, e = (idx >> 6) & 3, tu = idx >> 8;
    const int t = tu / TY, u = tu - t * TY;
    const int i = 16 * t + MF::row(l >> 4, e), j = 16 * u + (l & 15);
    if (i < wx && j < wy) out[i * ldo + j] = red[idx];
  }
  __syncthreads();
}
template <int TX>
__device__ __forceinline__ void tile_xty_y(const float* X, int64_t ldx, int wx, const float* Yb, int64_t ldy,
                                           int wy, int64_t m, double* out, int ldo, double* red) {
  const int ty = (wy + 15) / 16;
  if (ty <= 1) tile_xty_t<TX, 1>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
  else if (ty == 2) tile_xty_t<TX, 2>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
  else if (ty == 3) tile_xty_t<TX, 3>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
  else tile_xty_t<TX, 4>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
}
__device__ __forceinline__ void tile_xty(const float* X, int64_t ldx, int wx, const float* Yb, int64_t ldy,
                                         int wy, int64_t m, double* out, int ldo, double* red) {
  const int tx = (wx + 15) / 16;
  if (tx <= 1) tile_xty_y<1>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
  else if (tx == 2) tile_xty_y<2>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
  else if (tx == 3) tile_xty_y<3>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
  else tile_xty_y<4>(X, ldx, wx, Yb, ldy, wy, m, out, ldo, red);
}

// ---------------------------------------------------------------------------
// Z (column-major, ldz, columns zoff .. zoff+ncols-1) = X (m x f, ldx) W
// (f x ncols FP64, LDS or global, element (i,j) at i*ldw + j), f <= 4 KSM,
// on f64 MFMA; each wave computes 16 whole rows at a time, so Z may alias X.
// ---------------------------------------------------------------------------
template <int KSM = 16>
__device__ __forceinline__ void tile_apply(const float* X, int64_t ldx, int64_t m, int f, const double* W,
                                           int ldw, float* Z, int64_t ldz, int64_t zoff, int ncols) {
  typedef Mfma<double> MF;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  const int TT = (ncols + 15) / 16, KS = (f + 3) / 4;
  for (int64_t row0 = 16 * (int64_t)wv; row0 < m; row0 += 64) {
    const int64_t arow = row0 + r;
    double a[KSM];
#pragma unroll
    for (int kk = 0; kk < KSM; ++kk) {
      const int k = 4 * kk + g;
      a[kk] = (kk < KS && k < f && arow < m) ? (double)X[(int64_t)k * ldx + arow] : 0.0;
    }
    for (int u = 0; u < TT; ++u) {
      MF::acc_t z = MF::zero();
      const int col = 16 * u + r;
#pragma unroll
      for (int kk = 0; kk < KSM; ++kk) {
        if (kk < KS) {
          const int k = 4 * kk + g;
          const double b = (k < f && col < ncols) ? W[k * ldw + col] : 0.0;
          z = MF::op(a[kk], b, z);
        }
      }
      if (col < ncols) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = row0 + MF::row(g, e);
          if (row < m) Z[(zoff + col) * ldz + row] = (float)z[e];
        }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Y (m x f) -= Q (m x w) W (w x f, FP64 in LDS, element (i,j) at i*ldw + j),
// in FP32 on MFMA (the projection step of block Gram-Schmidt), f <= 64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_update(float* Yb, int64_t ldy, const float* Q, int64_t ldq, int64_t m,
                                            int w, int f, const double* W, int ldw) {
  typedef Mfma<float> MF;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  const int TT = (f + 15) / 16;
  for (int64_t row0 = 16 * (int64_t)wv; row0 < m; row0 += 64) {
    const int64_t arow = row0 + r;
    MF::acc_t z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) z[u] = MF::zero();
    for (int k0 = 0; k0 < w; k0 += 4) {
      const int k = k0 + g;
      const float a = (k < w && arow < m) ? Q[(int64_t)k * ldq + arow] : 0.f;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < TT) {
          const int col = 16 * u + r;
          const float b = (k < w && col < f) ? (float)W[k * ldw + col] : 0.f;
          z[u] = MF::op(a, b, z[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int col = 16 * u + r;
      if (u < TT && col < f) {
        const int64_t row = row0 + 4 * g;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (row + e < m) Yb[(int64_t)col * ldy + row + e] -= z[u][e];
      }
    }
  }
  __syncthreads();
}

// Cholesky with inverse of G (LDS, row-major ld F+1) for the smallest
// template width F >= f; R overwrites G, R^{-1} goes to Ri (ld F+1).
// The leading dimension used is F+1 for the chosen F; callers pass ldF.
__device__ int chol_width(int f) { return f <= 16 ? 16 : (f <= 32 ? 32 : 64); }
__device__ void tile_chol(double* Gs, double* Ri, double* work, double* dgs, int f, uint64_t dmask_in,
                          int first_pass, uint64_t* dmask_out, int* nfl) {
  const int F = chol_width(f);
  if (F == 16) chol_inv<16>(Gs, Ri, work, dgs, f, dmask_in, first_pass, dmask_out, nfl);
  else if (F == 32) chol_inv<32>(Gs, Ri, work, dgs, f, dmask_in, first_pass, dmask_out, nfl);
  else chol_inv<64>(Gs, Ri, work, dgs, f, dmask_in, first_pass, dmask_out, nfl);
}

// ---------------------------------------------------------------------------
// QR of M^T (M = R2 R1, or R2 when R1 is null; f x f FP64 in global memory,
// element (i,j) at j*f + i) by CholeskyQR2 in FP64 on the LDS arena (as the
// closing QR of the single-matrix path).  Qh -> Qout, Rh -> Dout (FP64,
// both element (i,j) at j*f + i).
// ---------------------------------------------------------------------------
template <int F>
__device__ void tile_small_qr(double* lds, const double* R1g, const double* R2g, int f, double* Qout,
                              double* Dout, int* nfloor) {
  typedef SmallCfg<F> S;
  constexpr int LD = S::LD;
  double* B0 = lds;
  double* B1 = B0 + S::SIZE;
  double* B2 = B1 + S::SIZE;
  double* B3 = B2 + S::SIZE;
  double* work = B3 + S::SIZE;
  double* dgs = work + 24 * F;
  const int tid = threadIdx.x;
  double* Mt = R1g ? B1 : B0;
  for (int idx = tid; idx < F * F; idx += 256) {
    const int i = idx / F, jj = idx - i * F;
    const bool ok = i < f && jj < f;
    Mt[i * LD + jj] = ok ? R2g[(int64_t)jj * f + i] : 0.0;
    if (R1g) B2[i * LD + jj] = ok ? R1g[(int64_t)jj * f + i] : 0.0;
  }
  __syncthreads();
  if (R1g) {
    lds_gemm<F, false, false>(B1, B2, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });
    __syncthreads();
  }
  lds_gemm<F, false, true>(B0, B0, [&](int i, int jj, double v) { B1[i * LD + jj] = v; });
  __syncthreads();
  uint64_t dm1, dm2;
  int nf1, nf2;
  chol_inv<F>(B1, B2, work, dgs, f, 0ull, 1, &dm1, &nf1);
  lds_gemm<F, true, false>(B0, B2, [&](int i, int jj, double v) { B3[i * LD + jj] = v; });
  __syncthreads();
  lds_gemm<F, true, false>(B3, B3, [&](int i, int jj, double v) { B0[i * LD + jj] = v; });
  __syncthreads();
  chol_inv<F>(B0, B2, work, dgs, f, dm1, 0, &dm2, &nf2);
  lds_gemm<F, false, false>(B3, B2, [&](int i, int jj, double v) {
    if (i < f && jj < f) Qout[(int64_t)jj * f + i] = v;
  });
  lds_gemm<F, false, false>(B0, B1, [&](int i, int jj, double v) {
    if (i < f && jj < f) Dout[(int64_t)jj * f + i] = v;
  });
  __syncthreads();
  *nfloor = nf1 + nf2;
}
__device__ void tile_small_qr_any(double* lds, const double* R1g, const double* R2g, int f, double* Qout,
                                  double* Dout, int* nfloor) {
  if (f <= 16) tile_small_qr<16>(lds, R1g, R2g, f, Qout, Dout, nfloor);
  else if (f <= 32) tile_small_qr<32>(lds, R1g, R2g, f, Qout, Dout, nfloor);
  else tile_small_qr<64>(lds, R1g, R2g, f, Qout, Dout, nfloor);
}

// Load an f x f FP64 matrix (element (i,j) at j*f + i) into LDS row-major (ld).
__device__ void tile_load_small(const double* Mg, int f, double* out, int ld) {
  for (int idx = threadIdx.x; idx < f * f; idx += 256) {
    const int j = idx / f, i = idx - j * f;
    out[i * ld + j] = Mg[idx];
  }
  __syncthreads();
}
// Store the leading f x f block of an LDS row-major matrix (ld) to global
// (element (i,j) at j*f + i).
__device__ void tile_store_small(const double* in, int ld, int f, double* Mg) {
  for (int idx = threadIdx.x; idx < f * f; idx += 256) {
    const int j = idx / f, i = idx - j * f;
    Mg[idx] = in[i * ld + j];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Ranks 65..128: FP64 matrices row-major with leading dimension LB in the
// slot (L2-resident); the LDS arena stages the right-hand factors.
// ---------------------------------------------------------------------------
// G = X^T X (f x f, 64 < f <= 128) of X (rows x f, column-major ldx): the
// blocks G11, G12 and G22 (chol_inv128 does not read G21).
__device__ __attribute__((noinline)) void tile_gram_big(const float* X, int64_t ldx, int f, int64_t rows,
                                                        double* G, double* red) {
  constexpr int LB = TileSlot::LB;
  const int f2 = f - 64;
  tile_xty(X, ldx, 64, X, ldx, 64, rows, G, LB, red);
  tile_xty(X, ldx, 64, X + 64 * ldx, ldx, f2, rows, G + 64, LB, red);
  tile_xty(X + 64 * ldx, ldx, f2, X + 64 * ldx, ldx, f2, rows, G + 64 * LB + 64, LB, red);
}

// Z (columns 0..ncols-1, ldz) = X (m x f, ldx) W with W (f x ncols, f <= 128)
// row-major in global memory (ld LB), staged through the arena (ld 129).
__device__ __attribute__((noinline)) void tile_apply_big(const float* X, int64_t ldx, int64_t m, int f,
                                                         const double* Wg, double* lds, float* Z, int64_t ldz,
                                                         int ncols) {
  for (int idx = threadIdx.x; idx < f * ncols; idx += 256) {
    const int i = idx / ncols, j = idx - i * ncols;
    lds[i * 129 + j] = Wg[(int64_t)i * TileSlot::LB + j];
  }
  __syncthreads();
  tile_apply<32>(X, ldx, m, f, lds, 129, Z, ldz, 0, ncols);
}

// QR of M^T (M = R2 R1, or R2 when R1 is null; f x f, 64 < f <= 128):
// small_qr_mid on row-major matrices (leading dimension LB); Qh and Rh out
// row-major; scr: 7 buffers of B2.
__device__ __attribute__((noinline)) void tile_small_qr_big(double* lds, const double* R1g, const double* R2g,
                                                            int f, double* Qh, double* Rh, double* scr) {
  constexpr int LB = TileSlot::LB;
  small_qr_mid<false>(lds, R1g, R2g, f, LB, scr, [&](int i, int j, double v) { Qh[i * LB + j] = v; },
                      [&](int i, int j, double v) { Rh[i * LB + j] = v; });
}

// ---------------------------------------------------------------------------
// One tile: Alg. 1 with BCGS2 + CholeskyQR2 blocks and the device rank
// test, then Alg. 2 (q = 0): C^T = A^T Q, CholeskyQR2 of C^T, QR of
// (R2 R1)^T, U = Q Qh.  A wide tile (h < w) is factored as A^T without
// moving it: its sketch A^T Omega and its C^T = A Q are the two products
// of a tall tile with the roles of the routines exchanged; the core is
// then re-triangularised.
// ---------------------------------------------------------------------------
__device__ void tile_factor(const TileDesc& td, float* slot, double* sdbl, double* lds, float* out_pool,
                            TileResult* res, double tol, uint32_t k0, uint32_t k1) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int64_t LD = TileSlot::LD;
  const bool tr = td.h < td.w;
  const int64_t m = tr ? td.w : td.h, n = tr ? td.h : td.w;     // oriented: m >= n
  const bool al = ((uintptr_t)td.A % 16 == 0) && (td.lda % 4 == 0);
  // LDS carve for the basis phase
  double* Gs = lds + TL_GS;                          // Gram -> R (ld chol_width(f) + 1)
  double* Ri = lds + TL_RI;                          // R^{-1}
  double* work = lds + TL_WORK;                      // Cholesky work area (24 x 64)
  double* dgs = lds + TL_DGS;                        // Cholesky diagonal
  double* Wp = lds + TL_W;                           // W = Q^T Y (TILE_QW x TILE_BMAX)
  double* fold = lds + TL_FOLD;                      // wave fold buffer of the reductions
  double* scal = lds + TILE_SQR;                     // [0] ||A||^2, [1..64] R1 diagonal
  __shared__ int s_keep, s_stop;
  float* Om = slot + TileSlot::OM;
  float* Yb = slot + TileSlot::Y;
  float* Q = slot + TileSlot::Q;
  const int64_t ldk = ((n + 3) / 4) * 4;
  const int b = td.b;
  int64_t wcols = 0;
  int blocks = 0;
  int status = TS_OK;
  double eps = 0.0;
  for (int64_t col0 = 0; col0 < n; col0 += b) {
    const int f = (int)((n - col0) < b ? (n - col0) : b);
    const int fpad = ((f + 15) / 16) * 16;
    ++blocks;
    tile_omega(Om, ldk, n, col0, f, fpad, k0, k1);
    __syncthreads();
    double* ss = (col0 == 0) ? &scal[0] : nullptr;
    // Y = A_o Omega_j (A_o the oriented tile, m x n)
    if (tr) tile_colprod(td.A, td.lda, n, m, Om, ldk, f, Yb, LD, ss, fold);
    else if (al) tile_rowprod<true>(td.A, td.lda, m, n, Om, ldk, f, Yb, LD, ss, fold);
    else tile_rowprod<false>(td.A, td.lda, m, n, Om, ldk, f, Yb, LD, ss, fold);
    if (col0 == 0) {
      const double a = scal[0];
      if (!(a < INFINITY)) {
        status = TS_NONFINITE;
        break;
      }
      eps = tol * sqrt(a);
    }
    // two rounds of [project against Q, Gram, Cholesky]; normalise between
    const int LDG = chol_width(f) + 1;
    uint64_t dm1 = 0, dm2 = 0;
    int nf = 0;
    for (int pass = 0; pass < 2; ++pass) {
      if (wcols > 0) {
        // W = Q^T Y (wcols x f), then Y -= Q W
        for (int64_t q0 = 0; q0 < wcols; q0 += 64) {
          const int wq = (int)((wcols - q0) < 64 ? (wcols - q0) : 64);
          tile_xty(Q + q0 * LD, LD, wq, Yb, LD, f, m, Wp + q0 * TILE_BMAX, TILE_BMAX, fold);
        }
        tile_update(Yb, LD, Q, LD, m, (int)wcols, f, Wp, TILE_BMAX);
      }
      tile_xty(Yb, LD, f, Yb, LD, f, m, Gs, LDG, fold);
      tile_chol(Gs, Ri, work, dgs, f, pass == 0 ? 0ull : dm1, pass == 0, pass == 0 ? &dm1 : &dm2, &nf);
      if (pass == 0) {
        for (int c = tid; c < f; c += 256) scal[1 + c] = Gs[c * LDG + c];   // R1 diag
        __syncthreads();
        tile_apply(Yb, LD, m, f, Ri, LDG, Yb, LD, 0, f);                      // Y := Y R1^{-1}
      }
    }
    // rank test (Alg. 1): first column with d_c = R2(c,c) R1(c,c) <= eps
    if (wv == 0) {
      bool hit = false;
      if (lane < f) {
        const double d = ((dm2 >> lane) & 1ull) ? 0.0 : Gs[lane * LDG + lane] * scal[1 + lane];
        hit = d <= eps;
      }
      const unsigned long long mask = __ballot(hit);
      if (lane == 0) {
        s_keep = mask ? (int)__ffsll((long long)mask) - 1 : f;
        s_stop = (mask != 0ull) || (col0 + f >= n);
      }
    }
    __syncthreads();
    const int keep = s_keep;
    const int stop = s_stop;
    if (keep > 0) tile_apply(Yb, LD, m, f, Ri, LDG, Q, LD, wcols, keep);      // append Z R2^{-1}
    wcols += keep;
    if (stop) break;
    if (wcols > TILE_RMAX) {                        // the rank will exceed the in-kernel cap
      status = TS_RANK;
      break;
    }
  }
  const int64_t r = wcols;
  if (status == TS_OK && r > TILE_RMAX) status = TS_RANK;
  if (status == TS_OK && r > td.r_cap) status = TS_CAPACITY;
  if (status == TS_OK && r > 0) {
    const int ri = (int)r;
    // a9: C^T = A_o^T Q (n x r), 64 columns of Q at a time
    float* Ct = slot + TileSlot::CT;
    for (int c0 = 0; c0 < ri; c0 += 64) {
      const int rc = (ri - c0) < 64 ? ri - c0 : 64;
      if (!tr) tile_colprod(td.A, td.lda, m, n, Q + c0 * LD, LD, rc, Ct + c0 * LD, LD, nullptr, fold);
      else if (al) tile_rowprod<true>(td.A, td.lda, n, m, Q + c0 * LD, LD, rc, Ct + c0 * LD, LD, nullptr, fold);
      else tile_rowprod<false>(td.A, td.lda, n, m, Q + c0 * LD, LD, rc, Ct + c0 * LD, LD, nullptr, fold);
    }
    float* Ut = out_pool + td.out_off;
    float* core = Ut + td.r_cap * td.h;
    float* Vt = core + td.r_cap * td.r_cap;
    // V = C^T R2^{-1}: the output V (tall tile) or V' (wide tile)
    float* Vdst = tr ? slot + TileSlot::VP : Vt;
    const int64_t ldv = tr ? LD : td.w;
    if (ri <= 64) {
      // a10: C^T = V R by CholeskyQR2 (V over C^T in place), R1, R2 kept
      const int LDG = chol_width(ri) + 1;
      uint64_t dm1 = 0, dm2 = 0;
      int nf = 0;
      tile_xty(Ct, LD, ri, Ct, LD, ri, n, Gs, LDG, fold);
      tile_chol(Gs, Ri, work, dgs, ri, 0ull, 1, &dm1, &nf);
      tile_store_small(Gs, LDG, ri, sdbl + TileSlot::R1);
      tile_apply(Ct, LD, n, ri, Ri, LDG, Ct, LD, 0, ri);
      tile_xty(Ct, LD, ri, Ct, LD, ri, n, Gs, LDG, fold);
      tile_chol(Gs, Ri, work, dgs, ri, dm1, 0, &dm2, &nf);
      tile_store_small(Gs, LDG, ri, sdbl + TileSlot::R2);
      tile_apply(Ct, LD, n, ri, Ri, LDG, Vdst, ldv, 0, ri);
      // a11: (R2 R1)^T = Qh Rh on the arena
      int nfq = 0;
      tile_small_qr_any(lds, sdbl + TileSlot::R1, sdbl + TileSlot::R2, ri, sdbl + TileSlot::QH,
                        sdbl + TileSlot::DH, &nfq);
      // U_hat = Q Qh (m x r)
      const int LDW = chol_width(ri) + 1;
      tile_load_small(sdbl + TileSlot::QH, ri, Gs, LDW);
      if (!tr) {
        tile_apply(Q, LD, m, ri, Gs, LDW, Ut, td.h, 0, ri);                   // U (h x r)
        for (int idx = tid; idx < ri * ri; idx += 256) {                       // core = Rh
          const int i = idx / ri, j = idx - i * ri;
          core[(int64_t)i * td.r_cap + j] = (float)sdbl[TileSlot::DH + (int64_t)j * ri + i];
        }
      } else {
        // A^T = U' D' V'^T with U' = Q Qh (w x r) and V' (h x r): A = V' D'^T U'^T,
        // QR(D'^T) = Q'' R'': U = V' Q'', core = R'', V = U'.
        tile_apply(Q, LD, m, ri, Gs, LDW, Vt, td.w, 0, ri);                   // V = U' (w x r)
        int nfq2 = 0;
        // M = D' (element (i,j) at j*r + i) -> QR(M^T) = QR(D'^T)
        tile_small_qr_any(lds, nullptr, sdbl + TileSlot::DH, ri, sdbl + TileSlot::QH2, sdbl + TileSlot::DH2,
                          &nfq2);
        tile_load_small(sdbl + TileSlot::QH2, ri, Gs, LDW);
        tile_apply(slot + TileSlot::VP, LD, n, ri, Gs, LDW, Ut, td.h, 0, ri);  // U = V' Q'' (h x r)
        for (int idx = tid; idx < ri * ri; idx += 256) {
          const int i = idx / ri, j = idx - i * ri;
          core[(int64_t)i * td.r_cap + j] = (float)sdbl[TileSlot::DH2 + (int64_t)j * ri + i];
        }
      }
    } else {
      // the same steps with the blocked 128-wide Cholesky and L2-resident matrices
      constexpr int LB = TileSlot::LB;
      constexpr int64_t B2 = TileSlot::B2;
      double* dd = sdbl + TileSlot::BIG;
      double* Gg = dd;
      double* R1g = dd + B2;
      double* R1i = dd + 2 * B2;
      double* R2g = dd + 3 * B2;
      double* R2i = dd + 4 * B2;
      double* Qh = dd + 5 * B2;
      double* Rh = dd + 6 * B2;
      double* Qh2 = dd + 7 * B2;
      double* Rh2 = dd + 8 * B2;
      double* scr = dd + 9 * B2;                    // 7 buffers
      uint64_t d10 = 0, d11 = 0, d20 = 0, d21 = 0;
      tile_gram_big(Ct, LD, ri, n, Gg, fold);
      chol_inv128(Gg, LB, ri, R1g, R1i, lds, 0ull, 0ull, 1, &d10, &d11);
      tile_apply_big(Ct, LD, n, ri, R1i, lds, Ct, LD, ri);
      tile_gram_big(Ct, LD, ri, n, Gg, fold);
      chol_inv128(Gg, LB, ri, R2g, R2i, lds, d10, d11, 0, &d20, &d21);
      tile_apply_big(Ct, LD, n, ri, R2i, lds, Vdst, ldv, ri);
      tile_small_qr_big(lds, R1g, R2g, ri, Qh, Rh, scr);
      const double* Rc = Rh;
      if (!tr) {
        tile_apply_big(Q, LD, m, ri, Qh, lds, Ut, td.h, ri);                   // U (h x r)
      } else {
        tile_apply_big(Q, LD, m, ri, Qh, lds, Vt, td.w, ri);                   // V = U' (w x r)
        tile_small_qr_big(lds, nullptr, Rh, ri, Qh2, Rh2, scr);                // QR(D'^T)
        tile_apply_big(slot + TileSlot::VP, LD, n, ri, Qh2, lds, Ut, td.h, ri); // U = V' Q''
        Rc = Rh2;
      }
      for (int idx = tid; idx < ri * ri; idx += 256) {
        const int i = idx / ri, j = idx - i * ri;
        core[(int64_t)i * td.r_cap + j] = (float)Rc[(int64_t)i * LB + j];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    TileResult o;
    o.rank = r;
    o.blocks = blocks;
    o.status = status;
    o.norm = sqrt(scal[0]);
    res[td.index] = o;
  }
  __syncthreads();
}

// Persistent launch: workgroup g uses scratch slot g and takes tiles in the
// order of descs (largest first) from the queue until it is empty.
__global__ __launch_bounds__(256) void k_tiles(const TileDesc* __restrict__ descs, int ntiles,
                                               uint32_t* __restrict__ queue, char* __restrict__ scratch,
                                               float* __restrict__ out_pool, TileResult* __restrict__ res,
                                               double tol, uint32_t k0, uint32_t k1) {
  __shared__ __align__(16) double lds[TILE_LDS];
  __shared__ int s_t;
  float* slot = reinterpret_cast<float*>(scratch + (int64_t)blockIdx.x * TileSlot::BYTES);
  double* sdbl = reinterpret_cast<double*>(slot + TileSlot::FLOATS);
  for (;;) {
    if (threadIdx.x == 0) s_t = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int t = s_t;
    __syncthreads();
    if (t >= ntiles) break;
    tile_factor(descs[t], slot, sdbl, lds, out_pool, res, tol, k0, k1);
  }
}

}  // namespace eodabe
