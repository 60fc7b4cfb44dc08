"""Plain complex128 CPU oracle for EOD-ABE on complex input, the paper's own
setting (A in C^{m x n}, A ~= U D V^H with U, V column-orthonormal and D
upper triangular; introduction and section 3).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library.  Alg. 1 and Alg. 2 are followed step by step in complex
arithmetic, with library primitives (matmul, LAPACK Householder QR, SVD) as
steps.  Readings (listed in the design notes):

* The Gaussian test matrix is complex standard normal: column c is
  (g_2c + i g_2c+1) / sqrt(2), g_j the FP64 Box-Muller column j of the real
  test matrix (same counter-based generator), each part rounded to FP32
  after the scaling; so E |omega_i|^2 = 1 and |T(l,l)|^2 estimates the
  squared residual norm exactly as in the real case.
* eps = tol ||A||_F; the stopping test compares |T(l,l)| (the moduli of the
  diagonal of the block's QR) with eps.
* Every QR is Householder with the phases fixed so the triangular factor has
  a real non-negative diagonal, which makes every factor unique.
* The projection is applied twice, as in the real oracle.
* m < n: factor A^H = U' D' V'^H, then A = V' D'^H U'^H and D'^H = Q' R'
  (one more QR), so U = V' Q', D = R', V = U'.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import eodabe_oracle as O

SQRT_HALF = math.sqrt(0.5)


def omega_complex(seed: int, n: int, col0: int, ncols: int) -> np.ndarray:
    """Columns col0 .. col0+ncols-1 of the n x n complex Gaussian test matrix."""
    g = O.gaussian_columns64(seed, n, 2 * col0, 2 * ncols)
    re = (g[:, 0::2] * SQRT_HALF).astype(np.float32).astype(np.float64)
    im = (g[:, 1::2] * SQRT_HALF).astype(np.float32).astype(np.float64)
    return re + 1j * im


def qr_posdiag_c(Y: np.ndarray):
    """Economy Householder QR with the diagonal of R real and >= 0."""
    P, T = np.linalg.qr(Y, mode="reduced")
    d = np.diag(T)
    ph = np.ones_like(d)
    nz = np.abs(d) > 0
    ph[nz] = d[nz] / np.abs(d[nz])
    return P * ph[None, :], np.conj(ph)[:, None] * T


def basis_ext_c(A: np.ndarray, eps: float, k: int, seed: int, lowp: bool = False) -> dict:
    """Alg. 1 on complex A: Y_j = (I - Q Q^H) A Omega_j (twice), QR of Y_j,
    stop at the first l with |T_j(l,l)| <= eps (keep columns before it).
    lowp: the emulation with complex64 data (A, Omega, Y, Q held in
    complex64, the QR in complex128), used only to classify instances."""
    m, n = A.shape
    Aw = A.astype(np.complex64) if lowp else A
    Q = np.zeros((m, 0), dtype=Aw.dtype)
    diag_log: list[float] = []
    blocks = 0
    c = 0
    while c < n:
        f = min(k, n - c)
        Om = omega_complex(seed, n, c, f)
        if lowp:
            Om = Om.astype(np.complex64)
        Y = Aw @ Om
        for _ in range(2):
            Y = Y - Q @ (Q.conj().T @ Y)
        P, T = qr_posdiag_c(Y.astype(np.complex128))
        d = np.abs(np.diag(T))
        blocks += 1
        hit = np.nonzero(d <= eps)[0]
        if hit.size:
            ell = int(hit[0])
            diag_log.extend(d[: ell + 1].tolist())
            Q = np.concatenate([Q, P[:, :ell].astype(Q.dtype)], axis=1)
            return dict(Q=Q.astype(np.complex128), diagT=np.array(diag_log), rank=Q.shape[1], blocks=blocks)
        diag_log.extend(d.tolist())
        Q = np.concatenate([Q, P.astype(Q.dtype)], axis=1)
        c += f
    return dict(Q=Q.astype(np.complex128), diagT=np.array(diag_log), rank=Q.shape[1], blocks=blocks)


@dataclass
class ComplexResult:
    U: np.ndarray
    D: np.ndarray
    V: np.ndarray
    rank: int
    eps: float
    diagT: np.ndarray
    blocks: int
    Qbasis: np.ndarray = field(repr=False)


def _tall(A, tol, k, q, seed, lowp):
    m, n = A.shape
    nrm = float(np.linalg.norm(A))
    eps = tol * nrm
    if nrm == 0.0:
        z = np.zeros
        return ComplexResult(z((m, 0), complex), z((0, 0), complex), z((n, 0), complex), 0, 0.0,
                             np.zeros(0), 0, z((m, 0), complex))
    be = basis_ext_c(A, eps, k, seed, lowp)
    Q = be["Q"]
    r = Q.shape[1]
    if r == 0:
        z = np.zeros
        return ComplexResult(z((m, 0), complex), z((0, 0), complex), z((n, 0), complex), 0, eps,
                             be["diagT"], be["blocks"], Q)
    for _ in range(q):                                  # Alg. 2, power iteration
        Qt, _ = qr_posdiag_c(A.conj().T @ Q)
        Q, _ = qr_posdiag_c(A @ Qt)
    C = Q.conj().T @ A                                  # C = Q^H A
    V, R = qr_posdiag_c(C.conj().T)                     # C^H = V R
    Qh, Rh = qr_posdiag_c(R.conj().T)                   # R^H = Q_hat R_hat
    return ComplexResult(Q @ Qh, Rh, V, r, eps, be["diagT"], be["blocks"], Q)


def eod_abe_c(A: np.ndarray, tol: float, k: int = 16, q: int = 0, seed: int = 0,
              lowp: bool = False) -> ComplexResult:
    """EOD-ABE (Alg. 2 around Alg. 1) on complex A; k complex columns per block."""
    A = np.asarray(A, dtype=np.complex128)
    m, n = A.shape
    if m >= n:
        return _tall(A, tol, k, q, seed, lowp)
    t = _tall(A.conj().T, tol, k, q, seed, lowp)
    if t.rank == 0:
        return ComplexResult(t.V, t.D, t.U, 0, t.eps, t.diagT, t.blocks, t.Qbasis)
    Qp, Rp = qr_posdiag_c(t.D.conj().T)
    return ComplexResult(t.V @ Qp, Rp, t.U, t.rank, t.eps, t.diagT, t.blocks, t.Qbasis)


def rel_err_c(A, U, D, V) -> float:
    A = np.asarray(A, dtype=np.complex128)
    n = np.linalg.norm(A)
    return 0.0 if n == 0 else float(np.linalg.norm(A - U @ D @ V.conj().T) / n)


def eckart_young_c(A, r: int) -> float:
    s = np.linalg.svd(np.asarray(A, dtype=np.complex128), compute_uv=False)
    tot = float(np.sqrt(np.sum(s * s)))
    return float(np.sqrt(np.sum(s[r:] ** 2)) / tot) if tot > 0 else 0.0


def precision_stable_c(A, tol: float, k: int = 16, seed: int = 0):
    """The rank band rule of O.precision_stable with complex64 data."""
    A = np.asarray(A, dtype=np.complex128)
    if A.shape[0] < A.shape[1]:
        A = A.conj().T
    nrm = float(np.linalg.norm(A))
    if nrm == 0.0:
        return True, 0, 0
    eps = tol * nrm
    b64 = basis_ext_c(A, eps, k, seed)
    blp = basis_ext_c(A, eps, k, seed, lowp=True)
    nc = min(len(b64["diagT"]), len(blp["diagT"]))
    d64, dlp = b64["diagT"][:nc], blp["diagT"][:nc]
    rho2 = np.maximum(dlp * dlp - d64 * d64, 0.0)
    S = O.ORDER_SPREAD
    lo = np.sqrt(d64 * d64 + rho2 / (S * S))
    hi = np.sqrt(d64 * d64 + (S * S) * rho2)
    near = bool(np.any((lo <= eps) & (eps <= hi)))
    return (b64["rank"] == blp["rank"]) and not near, b64["rank"], blp["rank"]
