// Device kernels of the two applications the paper evaluates EOD-ABE on:
//   * colour-image compression (introduction and section 4.1): each channel
//     is factored, reconstructed as U_hat D_hat V_hat^T, and the quality
//     criteria PSNR, global SSIM and RelErr are reduced in FP64 in a fixed
//     order, fused into the reconstruction pass;
//   * hyperspectral dimensionality reduction (section 4.2): pixel features
//     U_hat D_hat and KNN classification of every pixel by the pixels of the
//     other cross-validation folds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eodabe_kernels.hpp"

namespace eodabe {

constexpr int IMG_MAX_CH = 4;

// Per-channel factor locations of one image (passed by value).
struct ImgJob {
  const float* Ut[IMG_MAX_CH];   // r_cap x h row-major: row a is column a of U_hat
  const float* core[IMG_MAX_CH]; // r_cap x r_cap row-major: D_hat
  const float* Vt[IMG_MAX_CH];   // r_cap x w row-major: V_hat^T
  float* B[IMG_MAX_CH];          // scratch r x w: D_hat V_hat^T
  int r[IMG_MAX_CH];             // rank of the channel
  int rc;                        // r_cap of every channel
};

// B = D_hat V_hat^T for each channel (grid: w / 256 x r_max x channels);
// D_hat upper triangular, so B(a, j) = sum_{b >= a} D(a, b) Vt(b, j).
__global__ __launch_bounds__(256) void k_img_dvt(ImgJob job, int64_t w) {
  const int c = blockIdx.z, a = blockIdx.y;
  const int64_t j = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int r = job.r[c];
  if (a >= r || j >= w) return;
  const float* D = job.core[c] + (int64_t)a * job.rc;
  const float* V = job.Vt[c];
  float acc = 0.f;
  for (int b = a; b < r; ++b) acc = fmaf(D[b], V[(int64_t)b * w + j], acc);
  job.B[c][(int64_t)a * w + j] = acc;
}

// Sums of one image pass: x = reconstruction, y = original.
struct ImgSums {
  double sx, sy, sxx, syy, sxy, sdd;
};

// A_hat = U_hat B for every channel (64 x 64 output tile per workgroup,
// 16 rows per wave on v_mfma_f32_16x16x4f32, the K loop over the rank),
// written to recon; the same pass accumulates the six FP64 sums of the
// criteria against the original image and writes one partial per
// workgroup (fixed tile order, so the fold is deterministic).
__global__ __launch_bounds__(256) void k_img_recon(ImgJob job, const float* __restrict__ img, int64_t h,
                                                   int64_t w, float* __restrict__ recon,
                                                   ImgSums* __restrict__ parts) {
  typedef Mfma<float> MF;
  __shared__ double red[6][4];
  const int c = blockIdx.z;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, g = lane >> 4;
  const int64_t i0 = blockIdx.y * (int64_t)64 + 16 * wv, j0 = blockIdx.x * (int64_t)64;
  const int r = job.r[c];
  const float* U = job.Ut[c];
  const float* B = job.B[c];
  MF::acc_t acc[4] = {MF::zero(), MF::zero(), MF::zero(), MF::zero()};
  const int64_t ia = i0 + lr;
  for (int a0 = 0; a0 < r; a0 += 4) {
    const int a = a0 + g;
    const bool ka = a < r;
    const float av = (ka && ia < h) ? U[(int64_t)a * h + ia] : 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t jb = j0 + 16 * t + lr;
      const float bv = (ka && jb < w) ? B[(int64_t)a * w + jb] : 0.f;
      acc[t] = MF::op(av, bv, acc[t]);
    }
  }
  const float* Y = img + (int64_t)c * h * w;
  float* X = recon + (int64_t)c * h * w;
  double s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t jj = j0 + 16 * t + lr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t ii = i0 + MF::row(g, e);
      if (ii < h && jj < w) {
        const float xv = acc[t][e];
        const double x = xv, y = Y[ii * w + jj], d = x - y;
        X[ii * w + jj] = xv;
        s[0] += x; s[1] += y; s[2] += x * x; s[3] += y * y; s[4] += x * y; s[5] += d * d;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double v = s[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[q][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t pid = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    double* o = &parts[pid].sx;
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
  }
}

// Criteria of section 4.1 over the whole image.
struct ImgMetrics {
  double relerr, psnr, ssim, sdd, syy, n;
};

// One workgroup: fold the partials in a fixed order, then the criteria:
// PSNR = 10 log10(255^2 N / sdd), SSIM of the vectorised images with
// c1 = (0.01 255)^2, c2 = (0.03 255)^2 and 1/(N-1) (co)variances,
// RelErr = sqrt(sdd / syy).
__global__ __launch_bounds__(256) void k_img_metrics(const ImgSums* __restrict__ parts, int64_t nparts,
                                                     double N, ImgMetrics* __restrict__ out) {
  __shared__ double red[6][256];
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t p = threadIdx.x; p < nparts; p += 256) {
    const double* q = &parts[p].sx;
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] += q[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sx = red[0][0], sy = red[1][0], sxx = red[2][0], syy = red[3][0], sxy = red[4][0],
                 sdd = red[5][0];
    const double mx = sx / N, my = sy / N;
    const double vx = (sxx - sx * mx) / (N - 1.0), vy = (syy - sy * my) / (N - 1.0);
    const double cxy = (sxy - sx * my) / (N - 1.0);
    const double c1 = (0.01 * 255.0) * (0.01 * 255.0), c2 = (0.03 * 255.0) * (0.03 * 255.0);
    ImgMetrics m;
    m.sdd = sdd;
    m.syy = syy;
    m.n = N;
    m.relerr = syy > 0.0 ? sqrt(sdd / syy) : 0.0;
    m.psnr = sdd > 0.0 ? 10.0 * log10(255.0 * 255.0 * N / sdd) : INFINITY;
    m.ssim = (2.0 * mx * my + c1) * (2.0 * cxy + c2) / ((mx * mx + my * my + c1) * (vx + vy + c2));
    *out = m;
  }
}

// Pixel features F = U_hat D_hat (m x r, row-major, ldf): F(i, a) =
// sum_{b <= a} U(i, b) D(b, a) with D upper triangular (grid: m / 256 x r).
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ Ut, const float* __restrict__ core,
                                                  int64_t m, int r, int64_t rc, float* __restrict__ F,
                                                  int64_t ldf) {
  const int a = blockIdx.y;
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= m || a >= r) return;
  float acc = 0.f;
  for (int b = 0; b <= a; ++b) acc = fmaf(Ut[(int64_t)b * m + i], core[(int64_t)b * rc + a], acc);
  F[i * ldf + a] = acc;
}

constexpr int KNN_KMAX = 16;
constexpr int KNN_DMAX = 32;
constexpr int KNN_CMAX = 64;

// KNN classification of every point by the points of the other folds
// (ten-fold cross-validation in one pass).  One thread per query point; the
// candidates stream through LDS 256 at a time.  Squared distances are
// summed feature by feature in FP64 from the FP32 features with separate
// multiply and add (no contraction), so they are the same bits as any
// implementation of that definition; the k nearest are the smallest
// (distance, index) pairs (candidates arrive in index order, and a new one
// enters only when strictly closer); the vote goes to the most frequent
// label, ties to the smaller label.  pred[i] receives the class and
// conf[pred * nclass + label] counts it.
__global__ __launch_bounds__(256) void k_knn_cv(const float* __restrict__ F, int64_t m, int d, int64_t ldf,
                                                const int32_t* __restrict__ label,
                                                const int32_t* __restrict__ fold, int k, int nclass,
                                                int32_t* __restrict__ pred,
                                                unsigned long long* __restrict__ conf) {
  __shared__ float cf[256 * KNN_DMAX];
  __shared__ int32_t cfold[256], clab[256];
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  const bool active = i < m;
  double xi[KNN_DMAX];
#pragma unroll
  for (int a = 0; a < KNN_DMAX; ++a) xi[a] = (active && a < d) ? (double)F[i * ldf + a] : 0.0;
  const int fi = active ? fold[i] : -1;
  double bd[KNN_KMAX];
  int32_t bl[KNN_KMAX];
#pragma unroll
  for (int s = 0; s < KNN_KMAX; ++s) {
    bd[s] = INFINITY;
    bl[s] = -1;
  }
  double worst = INFINITY;                          // bd[k - 1], kept with static indices
  for (int64_t j0 = 0; j0 < m; j0 += 256) {
    __syncthreads();
    {
      const int64_t j = j0 + threadIdx.x;
      const bool ok = j < m;
      for (int a = 0; a < d; ++a) cf[threadIdx.x * d + a] = ok ? F[j * ldf + a] : 0.f;
      cfold[threadIdx.x] = ok ? fold[j] : fi;       // past the end: same fold, skipped
      clab[threadIdx.x] = ok ? label[j] : 0;
    }
    __syncthreads();
    const int nc = (int)((m - j0) < 256 ? (m - j0) : 256);
    for (int t = 0; t < nc; ++t) {
      if (cfold[t] == fi) continue;
      double dd = 0.0;
      {
#pragma clang fp contract(off)
#pragma unroll
        for (int a = 0; a < KNN_DMAX; ++a) {
          if (a < d) {
            const double u = (double)cf[t * d + a] - xi[a];
            dd = dd + u * u;
          }
        }
      }
      if (!(dd < worst)) continue;
      // insert into the sorted list of the first k entries
      const int lt = clab[t];
#pragma unroll
      for (int s = KNN_KMAX - 1; s > 0; --s) {
        if (s < k) {
          if (dd < bd[s - 1]) {
            bd[s] = bd[s - 1];
            bl[s] = bl[s - 1];
          } else if (dd < bd[s]) {
            bd[s] = dd;
            bl[s] = lt;
          }
        }
      }
      if (dd < bd[0]) {
        bd[0] = dd;
        bl[0] = lt;
      }
#pragma unroll
      for (int s = 0; s < KNN_KMAX; ++s)
        if (s == k - 1) worst = bd[s];
    }
  }
  if (!active) return;
  int best = KNN_CMAX, bestc = -1;
#pragma unroll
  for (int s = 0; s < KNN_KMAX; ++s) {
    if (s >= k || bl[s] < 0) continue;
    int cnt = 0;
#pragma unroll
    for (int t = 0; t < KNN_KMAX; ++t) cnt += (t < k && bl[t] == bl[s]) ? 1 : 0;
    if (cnt > bestc || (cnt == bestc && bl[s] < best)) {
      bestc = cnt;
      best = bl[s];
    }
  }
  if (bestc < 0) best = 0;   // no candidate in other folds
  pred[i] = best;
  atomicAdd(&conf[(int64_t)best * nclass + label[i]], 1ull);
}

}  // namespace eodabe
