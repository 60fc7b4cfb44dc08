"""Pins for the application-layer oracle (CPU only): the quality criteria of
section 4.1 against closed forms and a hand-worked case, the storage example
of the introduction reproduced end to end, and the KNN / cross-validation
of section 4.2 against hand-worked cases and invariants."""
import math
import os

import numpy as np
import pytest

import oracle.apps_oracle as P
import oracle.eodabe_oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- criteria
def test_psnr_constant_offset_closed_form():
    A = W.image(1, 64, 0.0, width=48).astype(np.float64)
    for delta in (0.5, 3.0, 40.0):
        assert abs(P.psnr(A, A + delta) - 10 * math.log10(255.0 ** 2 / delta ** 2)) <= 1e-12
    assert P.psnr(A, A) == math.inf


def test_ssim_identity_and_offset_closed_form():
    A = W.image(2, 40, 0.0, width=30).astype(np.float64)
    assert abs(P.ssim_global(A, A) - 1.0) <= 1e-14
    # a constant offset leaves variances and covariance unchanged: only the
    # luminance term remains, (2 mu (mu + d) + c1) / (mu^2 + (mu + d)^2 + c1)
    mu, d = A.mean(), 9.0
    want = (2 * mu * (mu + d) + P.C1) / (mu * mu + (mu + d) ** 2 + P.C1)
    assert abs(P.ssim_global(A, A + d) - want) <= 1e-13


def test_ssim_two_pixel_hand_example():
    # x = (255, 0) reconstructs y = (0, 255): equal means 127.5, variances
    # 2 * 127.5^2 / (2 - 1) = 32512.5 each, covariance -32512.5, so
    # SSIM = (c2 - 65025) / (c2 + 65025) with c2 = (0.03 * 255)^2 = 58.5225
    y = np.array([[0.0, 255.0]])
    x = np.array([[255.0, 0.0]])
    c2 = 58.5225
    assert abs(P.ssim_global(y, x) - (c2 - 65025.0) / (c2 + 65025.0)) <= 1e-15
    assert abs(P.ssim_global(y, x) - (-0.9982016185)) <= 1e-10


def test_relerr_of_scaled_image():
    A = W.image(3, 32, 0.1).astype(np.float64)
    for a in (0.9, 1.25):
        assert abs(P.relerr(A, a * A) - abs(1 - a)) <= 1e-14


# ---------------------------------------------------------------- storage example, end to end
def test_storage_example_through_compression():
    g = {}
    for l in open(os.path.join(GOLD, "storage_example.txt")):
        if l.strip() and not l.startswith("#"):
            k, *v = l.split()
            g[k] = v
    m, n = int(g["m"][0]), int(g["n"][0])
    ranks = [int(x) for x in g["ranks"]]
    img = W.exact_rank_rgb(0, m, n, tuple(ranks)).astype(np.float64)
    res = P.compress_image(img, 1e-4, 32, seed=0)
    assert res["ranks"] == ranks
    assert res["stored"] == int(g["total_factored"][0]) and res["full"] == int(g["total_full"][0])
    assert round(100 * res["reduction"], 2) == float(g["reduction_percent"][0])
    assert all(r < res["rank_bound"] for r in ranks)
    # exact ranks: the reconstruction is the image up to its FP32 rounding
    assert res["relerr"] < 1e-6 and res["ssim"] > 1 - 1e-10 and res["psnr"] > 100


def test_compress_image_matches_per_channel_factorization():
    img = W.rgb_image(1, 96, 80, noise_std=0.5).astype(np.float64)
    res = P.compress_image(img, 1e-3, 16, seed=4)
    for c in range(3):
        f = O.eod_abe(img[c], 1e-3, k=16, seed=4)
        assert res["ranks"][c] == f.rank
    d2 = sum(np.linalg.norm(img[c] - res["recon"][c]) ** 2 for c in range(3))
    assert abs(res["relerr"] - math.sqrt(d2) / np.linalg.norm(img)) <= 1e-14
    assert abs(res["psnr"] - 10 * math.log10(255.0 ** 2 * img.size / d2)) <= 1e-10


# ---------------------------------------------------------------- section 4.2
def test_features_reproduce_exact_rank_data():
    A = W.lowrank_haar(5, m=300, n=60, r=9, noise_std=0.0)
    res = O.eod_abe(A, 1e-10, k=8, seed=5)
    F = P.hsi_features(res.U, res.D)
    assert F.shape == (300, 9)
    assert np.linalg.norm(F @ res.V.T - A) <= 1e-12 * np.linalg.norm(A)
    assert abs(np.linalg.norm(F) - np.linalg.norm(A)) <= 1e-12 * np.linalg.norm(A)


def test_knn_hand_example():
    # six points on a line, two folds (even / odd positions), k = 1:
    #   x:      0    1    2    10   11   12
    #   label:  0    0    1    1    1    0
    #   fold:   0    1    0    1    0    1
    # each point looks only at the other fold: 0 -> 1 (label 0), 1 -> 0 or 2
    # (tie at distance 1: smaller index 0, label 0), 2 -> 1 (0), 10 -> 11 (1),
    # 11 -> 10 or 12 (tie: index 3, label 1), 12 -> 11 (1)
    F = np.array([[0.0], [1.0], [2.0], [10.0], [11.0], [12.0]], dtype=np.float32)
    lab = np.array([0, 0, 1, 1, 1, 0], dtype=np.int32)
    fold = np.array([0, 1, 0, 1, 0, 1], dtype=np.int32)
    pred, conf, oa = P.knn_cv(F, lab, fold, 1, 2)
    assert pred.tolist() == [0, 0, 0, 1, 1, 1]
    assert conf.tolist() == [[2, 1], [1, 2]]          # n[i][j]: class j predicted as i
    assert abs(oa - 4 / 6) <= 1e-15
    # k = 3 on the same points: 2's neighbours in fold 1 are 1, 10, 12
    # (labels 0, 1, 0): majority 0; a 1-1 vote with k = 2 goes to label 0
    pred3, _, _ = P.knn_cv(F, lab, fold, 3, 2)
    assert pred3[2] == 0
    F2 = np.array([[0.0], [1.0], [1.0], [5.0]], dtype=np.float32)
    pred2, _, _ = P.knn_cv(F2, np.array([1, 1, 0, 0], np.int32), np.array([0, 1, 1, 1], np.int32), 2, 2)
    assert pred2[0] == 0


def test_knn_separated_clusters_and_accuracy_formula():
    rng = np.random.default_rng(3)
    centres = rng.uniform(-100, 100, (5, 4))
    lab = rng.integers(0, 5, 400).astype(np.int32)
    F = (centres[lab] + rng.standard_normal((400, 4))).astype(np.float32)
    fold = (np.arange(400) % 10).astype(np.int32)
    pred, conf, oa = P.knn_cv(F, lab, fold, 5, 5)
    assert oa == 1.0 and np.array_equal(pred, lab)
    # OA = sum_i n_ii / sum_ij n_ij equals the fraction of correct labels
    lab2 = lab.copy()
    lab2[::7] = (lab2[::7] + 1) % 5
    pred, conf, oa = P.knn_cv(F, lab2, fold, 1, 5)
    assert conf.sum() == 400 and abs(oa - np.mean(pred == lab2)) <= 1e-15
