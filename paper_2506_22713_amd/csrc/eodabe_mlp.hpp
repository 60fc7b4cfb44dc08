// Learned rank predictor that warm-starts the basis size of Alg. 1: a GELU
// MLP 67 -> 256 -> 256 -> 256 -> 2 in FP32, trained and run by the kernels
// below.  Inputs: the first 64 values d_c = |T(c,c)| of the stopping test
// (the diagonal of the R factor of A Omega[:, :64], normalised by d_0 on a
// clamped log10 scale), log2 m, log2 n and log10(eps / d_0), the stopping
// threshold eps = tol ||A||_F on the scale of those values.  Head 0 regresses
// log(1 + rank); head 1 is the 0.9-quantile of the same quantity (pinball
// loss) and sizes the warm start.
#pragma once
#include "eodabe_kernels.hpp"

namespace eodabe {

constexpr int MLP_IN = 67, MLP_H = 256, MLP_OUT = 2;
constexpr double MLP_TAU = 0.9;
// flat parameter layout: W1 (H x IN, row-major), b1, W2 (H x H), b2, W3, b3, W4 (OUT x H), b4
constexpr int64_t MLP_W1 = 0, MLP_B1 = MLP_W1 + (int64_t)MLP_H * MLP_IN, MLP_W2 = MLP_B1 + MLP_H,
                  MLP_B2 = MLP_W2 + (int64_t)MLP_H * MLP_H, MLP_W3 = MLP_B2 + MLP_H,
                  MLP_B3 = MLP_W3 + (int64_t)MLP_H * MLP_H, MLP_W4 = MLP_B3 + MLP_H,
                  MLP_B4 = MLP_W4 + (int64_t)MLP_OUT * MLP_H, MLP_NPARAM = MLP_B4 + MLP_OUT;

// Input c of the network from the stopping-test values (c < 64), the
// geometry (c = 64, 65) or the threshold eps = tol ||A||_F of the test on
// the same scale as the d_c (c = 66).  Shared by the host (training sets)
// and the inference kernel.
__host__ __device__ inline float mlp_feature(const double* d, int c, int64_t m, int64_t n, double eps) {
  if (c < 64) {
    if (!(d[0] > 0.0) || !(d[c] > 0.0)) return -1.0f;
    const double l = log10(d[c] / d[0]);
    return (float)((l < -16.0 ? -16.0 : l) / 16.0);
  }
  if (c == 64) return (float)(log2((double)m) / 16.0);
  if (c == 65) return (float)(log2((double)n) / 16.0);
  if (!(d[0] > 0.0) || !(eps > 0.0)) return -1.0f;
  double l = log10(eps / d[0]);
  l = l < -16.0 ? -16.0 : (l > 16.0 ? 16.0 : l);
  return (float)(l / 16.0);
}

// Warm-start width from the quantile head: d0 = b ceil((rhat (1 + margin) + 1) / b),
// rhat = exp(y1) - 1, at least one block.
__host__ __device__ inline int64_t mlp_width(double y1, int b, double margin) {
  double rhat = exp(y1) - 1.0;
  if (!(rhat > 0.0)) rhat = 0.0;
  if (rhat > 1e9) rhat = 1e9;
  const double q = ceil((rhat * (1.0 + margin) + 1.0) / b);
  return (int64_t)b * (int64_t)(q < 1.0 ? 1.0 : q);
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// ---------------------------------------------------------------------------
// C (M x N, row-major ldc) = op(A) op(B) (+ bias[j]) in FP32 on MFMA:
// op(A)(i,k) = TA ? A[k*lda + i] : A[i*lda + k], op(B)(k,j) = TB ?
// B[j*ldb + k] : B[k*ldb + j].  A 64 x 64 tile per workgroup; K in chunks of
// 16 staged through LDS; wave w computes rows 32 (w / 2) .. + 32 and columns
// 32 (w % 2) .. + 32 as 2 x 2 MFMA tiles.
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_mlp_gemm(const float* __restrict__ A, int lda, const float* __restrict__ B,
                                                  int ldb, float* __restrict__ C, int ldc, int M, int N, int K,
                                                  const float* __restrict__ bias) {
  typedef Mfma<float> MF;
  __shared__ float As[64][17], Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, g = lane >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = 32 * (wv >> 1), wj = 32 * (wv & 1);
  MF::acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = MF::zero();
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int idx = tid; idx < 64 * 16; idx += 256) {
      // A tile: rows i0..i0+63, k0..k0+15 ; B tile: k0..k0+15, cols j0..j0+63
      const int ii = TA ? (idx & 63) : (idx >> 4), kk = TA ? (idx >> 6) : (idx & 15);
      const int gi = i0 + ii, gk = k0 + kk;
      As[ii][kk] = (gi < M && gk < K) ? (TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]) : 0.f;
      const int jj = TB ? (idx >> 4) : (idx & 63), kb = TB ? (idx & 15) : (idx >> 6);
      const int gj = j0 + jj, gkb = k0 + kb;
      Bs[kb][jj] = (gj < N && gkb < K) ? (TB ? B[(int64_t)gj * ldb + gkb] : B[(int64_t)gkb * ldb + gj]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[a][c] = MF::op(As[wi + 16 * a + r][ks + g], Bs[ks + g][wj + 16 * c + r], acc[a][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int j = j0 + wj + 16 * c + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + wi + 16 * a + MF::row(g, e);
        if (i < M && j < N) C[(int64_t)i * ldc + j] = acc[a][c][e] + (bias ? bias[j] : 0.f);
      }
    }
}

__global__ void k_gelu_fwd(const float* __restrict__ Z, float* __restrict__ H, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    H[i] = gelu_f(Z[i]);
}

// dZ = dH * GELU'(Z) (in place over dH allowed)
__global__ void k_gelu_bwd(const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ,
                           int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dZ[i] = dH[i] * gelu_grad_f(Z[i]);
}

// Loss (1/B) sum_b [(y_b0 - t_b)^2 + rho_tau(t_b - y_b1)] on one workgroup
// (FP64 accumulation, fixed order) and its gradient dY (B x 2).
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T, int B,
                                                  float* __restrict__ dY, double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  const double invB = 1.0 / B;
  for (int b = threadIdx.x; b < B; b += 256) {
    const double y0 = Y[2 * b], y1 = Y[2 * b + 1], t = T[b];
    const double u = t - y1;
    s += (y0 - t) * (y0 - t) + (u > 0 ? MLP_TAU * u : (MLP_TAU - 1.0) * u);
    dY[2 * b] = (float)(2.0 * (y0 - t) * invB);
    dY[2 * b + 1] = (float)((u > 0 ? -MLP_TAU : 1.0 - MLP_TAU) * invB);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * invB;
}

// out[j] = sum_b G[b*N + j] (bias gradients)
__global__ void k_colsum(const float* __restrict__ G, int B, int N, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += G[(int64_t)b * N + j];
  out[j] = s;
}

// One Adam step with bias-corrected moments.  The coefficients come from
// the host, formed in FP64 and rounded once: beta, 1 - beta and the bias
// corrections c = 1 - beta^step.
struct AdamCoef {
  float lr, b1, omb1, b2, omb2, c1, c2, eps;
};
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, AdamCoef a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = a.b1 * m[i] + a.omb1 * gi;
    const float vi = a.b2 * v[i] + a.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
  }
}

// Result of one warm-start inference (device).
struct MlpPred {
  int64_t d0;       // warm-start width
  double y0, y1;    // both heads (log(1 + rank))
};

// Single-sample inference on one workgroup, straight from the stopping-test
// values on the device: features, three GELU layers (thread j computes
// unit j), the two heads, and the warm-start width.
__global__ __launch_bounds__(256) void k_mlp_infer1(const float* __restrict__ P, const double* __restrict__ diag,
                                                    int64_t m, int64_t n, const State* __restrict__ st, int b,
                                                    double margin, MlpPred* __restrict__ out) {
  __shared__ float x[MLP_IN], h[2][MLP_H];
  const int j = threadIdx.x;
  if (j < MLP_IN) x[j] = mlp_feature(diag, j, m, n, st->eps);
  __syncthreads();
  float z = P[MLP_B1 + j];
  for (int k = 0; k < MLP_IN; ++k) z += P[MLP_W1 + (int64_t)j * MLP_IN + k] * x[k];
  h[0][j] = gelu_f(z);
  __syncthreads();
  z = P[MLP_B2 + j];
  for (int k = 0; k < MLP_H; ++k) z += P[MLP_W2 + (int64_t)j * MLP_H + k] * h[0][k];
  h[1][j] = gelu_f(z);
  __syncthreads();
  z = P[MLP_B3 + j];
  for (int k = 0; k < MLP_H; ++k) z += P[MLP_W3 + (int64_t)j * MLP_H + k] * h[1][k];
  __syncthreads();
  h[0][j] = gelu_f(z);
  __syncthreads();
  if (j < MLP_OUT) {
    float y = P[MLP_B4 + j];
    for (int k = 0; k < MLP_H; ++k) y += P[MLP_W4 + (int64_t)j * MLP_H + k] * h[0][k];
    x[j] = y;
  }
  __syncthreads();
  if (j == 0) {
    MlpPred o;
    o.y0 = x[0];
    o.y1 = x[1];
    o.d0 = mlp_width(x[1], b, margin);
    *out = o;
  }
}

}  // namespace eodabe
