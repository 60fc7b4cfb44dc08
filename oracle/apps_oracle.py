"""Plain FP64 CPU oracle for the two applications of EOD-ABE that the paper
evaluates: colour-image compression (introduction, storage example; section
4.1, quality criteria) and hyperspectral dimensionality reduction with KNN
classification under ten-fold cross-validation (section 4.2).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library.  Every function is written for checking by eye against the passage
it cites.  Readings where the paper is silent or garbled (listed in the
design notes):

* PSNR: the paper writes 255^2 n^2 / ||A_hat - A||_F^2 for an n x n image;
  n^2 is the number of values, so a colour image of c channels of h x w
  uses N = c h w (the usual mean-squared-error form).  An exact
  reconstruction has PSNR = +inf.
* SSIM: one global window over the vectorised images, as the paper
  defines it (x, y the vector forms).  The printed numerator factor
  "4 mu_x mu_y" would make SSIM(A, A) about 2, while the paper's tables
  report values below 1; the factor is read as the standard 2 mu_x mu_y.
  The constants, which the paper leaves unnamed, are the customary
  c1 = (0.01 * 255)^2 and c2 = (0.03 * 255)^2, and variances and the
  covariance use the 1/(N - 1) normalisation.
* Hyperspectral features: the rows of U_hat D_hat (pixels x r), the
  compressed representation of each pixel's spectrum (A ~= (U_hat D_hat)
  V_hat^T, equal to Q Q^T A V_hat).
* KNN: the paper does not state k; Euclidean distance; the k training
  points with the smallest (squared distance, index) pairs vote, ties in
  the vote go to the smallest class label.  Squared distances are summed
  feature by feature in FP64 from the FP32 feature values, with no fused
  multiply-add, so both sides take the same integer decisions.
* Ten-fold cross-validation: every pixel is classified once, by the
  pixels of the other nine folds.
"""
from __future__ import annotations

import math

import numpy as np

from . import eodabe_oracle as O

C1 = (0.01 * 255.0) ** 2
C2 = (0.03 * 255.0) ** 2


# ---------------------------------------------------------------------------
# Section 4.1: the three quality criteria.
# ---------------------------------------------------------------------------
def psnr(A: np.ndarray, Ahat: np.ndarray) -> float:
    """PSNR = 10 log10(255^2 N / ||A_hat - A||_F^2), N values (section 4.1)."""
    A = np.asarray(A, dtype=np.float64)
    d2 = float(np.sum((np.asarray(Ahat, dtype=np.float64) - A) ** 2))
    return math.inf if d2 == 0.0 else 10.0 * math.log10(255.0 ** 2 * A.size / d2)


def ssim_global(A: np.ndarray, Ahat: np.ndarray) -> float:
    """SSIM of the vectorised images x = A_hat, y = A (section 4.1):
    (2 mu_x mu_y + c1)(2 s_xy + c2) / ((mu_x^2 + mu_y^2 + c1)(s_x^2 + s_y^2 + c2))."""
    x = np.asarray(Ahat, dtype=np.float64).ravel()
    y = np.asarray(A, dtype=np.float64).ravel()
    N = x.size
    mx, my = x.mean(), y.mean()
    vx = np.sum((x - mx) ** 2) / (N - 1)
    vy = np.sum((y - my) ** 2) / (N - 1)
    cxy = np.sum((x - mx) * (y - my)) / (N - 1)
    return float((2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2)))


def relerr(A: np.ndarray, Ahat: np.ndarray) -> float:
    """RelErr = ||A - A_hat||_F / ||A||_F (section 4.1)."""
    A = np.asarray(A, dtype=np.float64)
    n = np.linalg.norm(A)
    return 0.0 if n == 0 else float(np.linalg.norm(A - np.asarray(Ahat, dtype=np.float64)) / n)


def compress_image(img: np.ndarray, tol: float, k, seed: int = 0) -> dict:
    """Compress each channel of a c x h x w image by EOD-ABE (Alg. 2, q = 0)
    and reconstruct it as U_hat D_hat V_hat^T; report the criteria of
    section 4.1 over the whole image and the storage count of the
    introduction: each channel keeps (h + w) r + r (r + 1) / 2 entries of
    its factors against h w of its own, and storing the factors pays while
    r is below the bound of O.storage_rank_bound.  k: block size, or one
    per channel."""
    img = np.asarray(img, dtype=np.float64)
    c, h, w = img.shape
    ks = list(k) if isinstance(k, (list, tuple)) else [k] * c
    rec = np.empty_like(img)
    ranks, facs = [], []
    for ch in range(c):
        res = O.eod_abe(img[ch], tol, k=ks[ch], q=0, seed=seed)
        rec[ch] = res.U @ res.D @ res.V.T
        ranks.append(res.rank)
        facs.append(res)
    stored = sum(O.storage_bytes(h, w, r) for r in ranks)
    return dict(ranks=ranks, factors=facs, recon=rec, psnr=psnr(img, rec), ssim=ssim_global(img, rec),
                relerr=relerr(img, rec), stored=stored, full=c * h * w,
                reduction=1.0 - stored / (c * h * w), rank_bound=O.storage_rank_bound(h, w))


# ---------------------------------------------------------------------------
# Section 4.2: features, KNN, ten-fold cross-validation, overall accuracy.
# ---------------------------------------------------------------------------
def hsi_features(U: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Reduced pixels: rows of U_hat D_hat (pixels x r)."""
    return np.asarray(U, dtype=np.float64) @ np.asarray(D, dtype=np.float64)


def _sq_dist(F: np.ndarray, i: int, J: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances from pixel i to pixels J, accumulated
    feature by feature in FP64 (a separate multiply and add per term)."""
    d = np.zeros(J.size, dtype=np.float64)
    for a in range(F.shape[1]):
        t = F[J, a] - F[i, a]
        d = d + t * t
    return d


def knn_cv(F: np.ndarray, labels: np.ndarray, fold: np.ndarray, k: int, nclass: int):
    """KNN classification of every pixel by the pixels of the other folds.
    F: features (FP32 values); returns (predictions, confusion n[i][j] =
    pixels of class j classified as i, OA = sum_i n_ii / sum_ij n_ij)."""
    F = np.asarray(F, dtype=np.float32).astype(np.float64)
    m = F.shape[0]
    pred = np.empty(m, dtype=np.int32)
    idx = np.arange(m)
    for i in range(m):
        J = idx[fold != fold[i]]
        d = _sq_dist(F, i, J)
        nn = J[np.lexsort((J, d))[:k]]            # smallest (distance, index)
        votes = np.bincount(labels[nn], minlength=nclass)
        pred[i] = int(np.argmax(votes))           # first maximum: smallest label
    conf = np.zeros((nclass, nclass), dtype=np.int64)
    for p, t in zip(pred, labels):
        conf[p, t] += 1
    oa = float(np.trace(conf)) / float(conf.sum())
    return pred, conf, oa
