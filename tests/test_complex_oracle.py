"""Pins for the complex oracle (CPU only): the complex Gaussian test matrix,
Theorem th3.4 in complex arithmetic, exact-rank recovery with unitary
factors and a real non-negative diagonal of D, the Eckart-Young optimum
from a complex SVD, the wide orientation, and planted mistakes."""
import numpy as np
import pytest

import oracle.complex_oracle as C
import workloads as W


def _orth(X):
    return np.linalg.norm(X.conj().T @ X - np.eye(X.shape[1]))


def test_complex_gaussian_moments():
    z = C.omega_complex(5, 4096, 0, 32).ravel()
    N = z.size
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 5 * np.sqrt(1.0 / N)
    assert abs(np.mean(z.real ** 2) - 0.5) < 5 * np.sqrt(0.5 / N)
    assert abs(np.mean(z * z)) < 5 * np.sqrt(1.0 / N)            # circular: E z^2 = 0
    # both parts are FP32 values; a column depends only on (seed, column)
    assert np.array_equal(z.real, z.real.astype(np.float32).astype(np.float64))
    assert np.array_equal(C.omega_complex(5, 100, 7, 3)[:, 1], C.omega_complex(5, 100, 8, 1)[:, 0])


@pytest.mark.parametrize("seed", range(3))
def test_diagT_equals_qr_of_complex_sketch(seed):
    A = W.lowrank_complex(seed, m=200, n=150, r=22, noise_std=1e-10)
    nrm = np.linalg.norm(A)
    be = C.basis_ext_c(A, 1e-7 * nrm, 8, seed)
    d = be["diagT"]
    R = np.linalg.qr(A @ C.omega_complex(seed, 150, 0, d.size))[1]
    ref = np.abs(np.diag(R))
    assert np.max(np.abs(ref - d)) <= 1e-12 * nrm
    ranks = {k: C.eod_abe_c(A, 1e-7, k=k, seed=seed).rank for k in (1, 5, 8, 32)}
    assert len(set(ranks.values())) == 1 and be["rank"] == 22, ranks


@pytest.mark.parametrize("r", [1, 7, 20])
def test_complex_exact_rank(r):
    A = W.lowrank_complex(40 + r, m=180, n=120, r=r)
    res = C.eod_abe_c(A, 1e-10, k=8, seed=r)
    assert res.rank == r
    assert C.rel_err_c(A, res.U, res.D, res.V) <= 1e-12
    assert _orth(res.U) < 1e-12 and _orth(res.V) < 1e-12
    assert np.allclose(np.tril(res.D, -1), 0)
    dg = np.diag(res.D)
    assert np.all(np.abs(dg.imag) <= 1e-14 * np.abs(dg).max()) and np.all(dg.real >= 0)
    Qb = res.Qbasis
    assert np.linalg.norm(res.U @ res.D @ res.V.conj().T - Qb @ (Qb.conj().T @ A)) <= 1e-13 * np.linalg.norm(A)
    sA = np.linalg.svd(A, compute_uv=False)[:r]
    assert np.max(np.abs(np.linalg.svd(res.D, compute_uv=False) - sA) / sA) <= 1e-12


@pytest.mark.parametrize("seed", range(2))
def test_complex_eckart_young_with_power_iteration(seed):
    A = W.lowrank_complex(seed, m=300, n=200, r=15, noise_std=1e-12)
    res = C.eod_abe_c(A, 1e-8, k=16, q=1, seed=seed)
    assert abs(C.rel_err_c(A, res.U, res.D, res.V) - C.eckart_young_c(A, res.rank)) <= 1e-10


def test_complex_wide_matrix():
    A = W.lowrank_complex(7, m=90, n=260, r=11)
    res = C.eod_abe_c(A, 1e-10, k=8, seed=7)
    assert res.rank == 11 and res.U.shape == (90, 11) and res.V.shape == (260, 11)
    assert C.rel_err_c(A, res.U, res.D, res.V) <= 1e-12
    assert _orth(res.U) < 1e-12 and _orth(res.V) < 1e-12 and np.allclose(np.tril(res.D, -1), 0)


def test_real_input_keeps_its_rank():
    # a real matrix of exact rank r has complex rank r
    A = W.lowrank_haar(3, m=150, n=100, r=9, noise_std=0.0).astype(np.complex128)
    assert C.eod_abe_c(A, 1e-10, k=4, seed=3).rank == 9


def test_planted_missing_conjugate_is_caught(monkeypatch):
    A = W.lowrank_complex(9, m=120, n=80, r=6)
    good = C.eod_abe_c(A, 1e-10, k=4, seed=9)
    assert C.rel_err_c(A, good.U, good.D, good.V) <= 1e-12
    orig = C.basis_ext_c

    def no_conj(A_, eps, k, seed, lowp=False):           # projection with Q^T instead of Q^H
        out = orig(A_, eps, k, seed, lowp)
        Q = out["Q"]
        out["Q"] = np.linalg.qr(Q.conj())[0]
        return out
    monkeypatch.setattr(C, "basis_ext_c", no_conj)
    bad = C.eod_abe_c(A, 1e-10, k=4, seed=9)
    assert C.rel_err_c(A, bad.U, bad.D, bad.V) > 1e-3
