"""Plain FP64 CPU oracle for EOD-ABE (Xu, Shen, Liu, Jia: "A Novel Adaptive
Low-Rank Matrix Approximation Method for Image Compression and
Reconstruction", arXiv 2506.22713).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library: the only thing both sides share is the seeded input generators in
``workloads/``, which hold none of the method's arithmetic.  The Gaussian
test matrix, a random draw the method makes, is fixed by a counter-based
generator (Philox4x32-10, Salmon et al., SC'11) that this file implements on
its own from the published definition; the HIP library implements the same
definition independently.

Every function follows a passage of the paper (cited in its docstring) and is
written for checking by eye: library primitives (matmul, LAPACK Householder
QR, SVD) serve as steps, with no blocking, fusion or reordering beyond what
the paper states.  Readings adopted where the paper is silent or ambiguous
(all listed in the design notes):

* eps = tol * ||A||_F  (the stopping test of Alg. 1 compares |T_j(l,l)| with
  an absolute eps; the tolerance is taken relative to ||A||_F).
* Every QR is Householder (LAPACK) with the sign fixed so that the triangular
  factor has a non-negative diagonal; this makes all factors unique.
* The projection (I - Q Q^T) of Alg. 1 is applied twice ("twice is enough");
  identical in exact arithmetic, needed for an orthonormal Q in floating point.
* Column c of the Gaussian test matrix is a pure function of (seed, c), so
  Omega = [Omega_1, ..., Omega_{s+1}] is the same n x n matrix for every
  block size k (the setting of Theorem th3.4).
* Empty last block (f_{s+1} = 0) is skipped; if the test never fires the
  rank is n.  If m < n the factorization of A^T is computed and transposed
  back, with one more QR to keep the core upper triangular.
* Real arithmetic only.

Functions without a pin of their own: none (see tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "PHILOX_M0", "PHILOX_M1", "PHILOX_W0", "PHILOX_W1",
    "philox4x32_10", "omega_columns", "qr_posdiag", "basis_ext", "eod_abe",
    "EodAbeResult", "rel_err", "eckart_young_relerr", "storage_bytes",
    "storage_rank_bound", "siam_bound_sq", "precision_stable",
]

# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC'11, section 4 and the Random123 reference definition).
# ---------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9  # golden ratio
PHILOX_W1 = 0xBB67AE85  # sqrt(3) - 1
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: tuple[int, int]) -> np.ndarray:
    """Philox4x32 with 10 rounds.

    ``ctr``: (N, 4) uint32 counters; ``key``: two 32-bit words.
    One round maps (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is bumped by (W0, W1) before every round after the first.
    """
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4).copy()
    k0 = np.uint64(key[0] & 0xFFFFFFFF)
    k1 = np.uint64(key[1] & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = np.uint64(PHILOX_M0) * c[:, 0]          # < 2^64, exact in uint64
        p1 = np.uint64(PHILOX_M1) * c[:, 2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c = np.stack([hi1 ^ c[:, 1] ^ k0, lo1, hi0 ^ c[:, 3] ^ k1, lo0], axis=1)
    return c.astype(np.uint32)


def _seed_key(seed: int) -> tuple[int, int]:
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def omega_columns(seed: int, n: int, col0: int, ncols: int) -> np.ndarray:
    """Columns col0 .. col0+ncols-1 of the n x n standard Gaussian test matrix
    Omega (Alg. 1, "Draw an n x f_j standard Gaussian matrix").

    Entry (i, c): Philox4x32-10 with counter (i // 4, c, 0, 0) and key
    (seed lo, seed hi) gives four words x0..x3; Box-Muller (FP64) turns
    (x0, x1) into rows 4q, 4q+1 and (x2, x3) into rows 4q+2, 4q+3 with
    u1 = (x + 1) 2^-32 in (0, 1], u2 = x 2^-32 in [0, 1),
    z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
    Values are rounded to FP32 (the precision the GPU stores them in) and
    returned in FP64, so FP32 and FP64 runs use the same Omega.
    """
    return gaussian_columns64(seed, n, col0, ncols).astype(np.float32).astype(np.float64)


def gaussian_columns64(seed: int, n: int, col0: int, ncols: int) -> np.ndarray:
    """The FP64 Box-Muller values of omega_columns before their rounding to
    FP32 (same counters, same transform)."""
    out = np.empty((n, ncols), dtype=np.float64)
    if n == 0 or ncols == 0:
        return out
    nq = (n + 3) // 4
    q = np.arange(nq, dtype=np.uint64)
    key = _seed_key(seed)
    for j in range(ncols):
        c = col0 + j
        ctr = np.zeros((nq, 4), dtype=np.uint64)
        ctr[:, 0] = q
        ctr[:, 1] = c
        x = philox4x32_10(ctr, key).astype(np.float64)
        z = np.empty((nq, 4), dtype=np.float64)
        for a, bb in ((0, 1), (2, 3)):
            u1 = (x[:, a] + 1.0) * 2.0 ** -32
            u2 = x[:, bb] * 2.0 ** -32
            rad = np.sqrt(-2.0 * np.log(u1))
            z[:, a] = rad * np.cos(2.0 * np.pi * u2)
            z[:, bb] = rad * np.sin(2.0 * np.pi * u2)
        out[:, j] = z.reshape(-1)[:n]
    return out


# ---------------------------------------------------------------------------
# QR with a non-negative diagonal (any QR is allowed by the paper; the sign
# convention makes the factors unique).
# ---------------------------------------------------------------------------
def qr_posdiag(Y: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Economy Householder QR (LAPACK via numpy) with diag(R) >= 0."""
    P, T = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(T))
    s[s == 0] = 1.0
    return P * s[None, :], T * s[:, None]


# ---------------------------------------------------------------------------
# Low-precision sketch operands (the FP16 / BF16 sketch form).  Not part of
# the paper: this emulates a run whose sketches from the third block on
# multiply FP16 or BF16 copies of A and Omega (exact products, wide
# accumulation), so that its rank and error can be compared with the GPU.
# ---------------------------------------------------------------------------
def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest, ties to even); returned as
    FP64 holding the bfloat16 values.  bfloat16 keeps the FP32 exponent and
    the top 7 fraction bits."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to IEEE binary16 (nearest, ties to even)."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def lp_scale(A: np.ndarray, mode: str) -> float:
    """Power of two applied to A before the FP16 rounding: with
    max|A| = f 2^e, f in [0.5, 1), the scale 2^(14-e) puts the largest entry
    in [2^13, 2^14) (FP16 holds up to 65504).  BF16 has FP32's range: 1."""
    mx = float(np.max(np.abs(A))) if A.size else 0.0
    if mode != "f16" or not (mx > 0.0) or not math.isfinite(mx):
        return 1.0
    _, e = math.frexp(np.float32(mx))
    return math.ldexp(1.0, 14 - e)


def lp_round(x: np.ndarray, mode: str) -> np.ndarray:
    return round_f16(x) if mode == "f16" else round_bf16(x)


# ---------------------------------------------------------------------------
# Alg. 1, BasisExt (section 3.1).
# ---------------------------------------------------------------------------
def basis_ext(A: np.ndarray, eps: float, k: int, seed: int,
              sketch_dtype=np.float64) -> dict:
    """Randomized blocked basis extraction (Alg. 1).

    For j = 1, 2, ...: draw Omega_j (n x f_j, global columns (j-1)k ...),
    set Y_j = (I - Q Q^T) A Omega_j, QR Y_j = P_j T_j; if some l has
    |T_j(l,l)| <= eps take the smallest, append P_j(:, 1:l-1) and stop;
    otherwise append P_j.  f_j = k except the last block n - s k (skipped
    when empty).  Theorem th3.4: diag(T) equals the diagonal of the R factor
    of the QR of A Omega; Remark rem3.6: rank = number of accepted columns.

    ``sketch_dtype=np.float32`` is an emulation of a run whose matrix data
    (A, Omega, Y, Q) is held in FP32 while the small QR stays in FP64; it
    is used only to classify instances as precision-stable.
    ``sketch_dtype="f16"`` / ``"bf16"``: the low-precision sketch form, in
    which blocks 3, 4, ... use Y_j = (round(s A) round(Omega_j)) / s with s
    from lp_scale (the products of the rounded operands are exact in FP64).
    The form is defined this way (blocks 1 and 2 sketch A itself: the first
    finds max|A| for the FP16 scale, the second writes the rounded copy);
    when a block read the copy, eod_abe adds one subspace iteration before
    the projection and takes the first product of every subspace iteration,
    A^T Q, from the copy (Q rounded the same way): (round(s A)^T round(Q)) / s.
    """
    m, n = A.shape
    lp = sketch_dtype if isinstance(sketch_dtype, str) else None
    lo = sketch_dtype == np.float32
    Aw = A.astype(np.float32) if lo else A
    if lp:
        sc = lp_scale(A, lp)
        A_lp = lp_round((A * sc).astype(np.float32), lp)
    Q = np.zeros((m, 0), dtype=Aw.dtype)
    diag_log: list[float] = []
    blocks = 0
    c = 0
    while c < n:
        f = min(k, n - c)
        Om = omega_columns(seed, n, c, f)
        if lo:
            Om = Om.astype(np.float32)
        if lp and blocks >= 2:
            Y = (A_lp @ lp_round(Om, lp)) / sc
        else:
            Y = Aw @ Om
        for _ in range(2):
            Y = Y - Q @ (Q.T @ Y)
        P, T = qr_posdiag(Y.astype(np.float64))
        d = np.abs(np.diag(T))
        blocks += 1
        hit = np.nonzero(d <= eps)[0]
        if hit.size:
            ell = int(hit[0])                   # 0-based: keep columns 0..ell-1
            diag_log.extend(d[: ell + 1].tolist())
            Q = np.concatenate([Q, P[:, :ell].astype(Q.dtype)], axis=1)
            return dict(Q=Q.astype(np.float64), diagT=np.array(diag_log),
                        rank=Q.shape[1], blocks=blocks, stopped=True)
        diag_log.extend(d.tolist())
        Q = np.concatenate([Q, P.astype(Q.dtype)], axis=1)
        c += f
    return dict(Q=Q.astype(np.float64), diagT=np.array(diag_log),
                rank=Q.shape[1], blocks=blocks, stopped=False)


# ---------------------------------------------------------------------------
# Alg. 2, EOD-ABE via subspace iteration (section 3.2).
# ---------------------------------------------------------------------------
@dataclass
class EodAbeResult:
    U: np.ndarray          # m x r, orthonormal columns (U_hat = Q_q Q_hat)
    D: np.ndarray          # r x r upper triangular (D_hat = R_hat), diag >= 0
    V: np.ndarray          # n x r, orthonormal columns (V_hat = Q)
    rank: int
    eps: float
    diagT: np.ndarray      # |T(l,l)| examined by Alg. 1, in order
    blocks: int
    Qbasis: np.ndarray = field(repr=False)   # Q_q, m x r
    R_values: np.ndarray = field(repr=False)  # diag of R from QR(C^T)


def _eod_abe_tall(A, tol, k, q, seed, sketch_dtype):
    m, n = A.shape
    nrm = float(np.sqrt(np.sum(A * A)))
    eps = tol * nrm
    if nrm == 0.0:
        z = np.zeros
        return EodAbeResult(z((m, 0)), z((0, 0)), z((n, 0)), 0, 0.0,
                            np.zeros(0), 0, z((m, 0)), np.zeros(0))
    be = basis_ext(A, eps, k, seed, sketch_dtype)
    Q = be["Q"]
    r = Q.shape[1]
    if r == 0:
        z = np.zeros
        return EodAbeResult(z((m, 0)), z((0, 0)), z((n, 0)), 0, eps,
                            be["diagT"], be["blocks"], Q, np.zeros(0))
    lp_iter = isinstance(sketch_dtype, str) and be["blocks"] >= 3
    if lp_iter:
        # low-precision form: a block sketched the rounded copy, so one more
        # subspace iteration refines the basis, and each iteration takes
        # A^T Q from the copy with Q rounded the same way (the form's
        # definition; the paper's method has no such step)
        q += 1
        sc = lp_scale(A, sketch_dtype)
        A_lp = lp_round((A * sc).astype(np.float32), sketch_dtype)
    for _ in range(q):                    # steps 2-7: power (subspace) iteration
        if lp_iter:
            Yt = (A_lp.T @ lp_round(Q.astype(np.float32), sketch_dtype)) / sc
        else:
            Yt = A.T @ Q
        Qt, _ = qr_posdiag(Yt)            # Y~_j = A^H Q_{j-1} = Q~_j R~_j
        Q, _ = qr_posdiag(A @ Qt)         # Y_j = A Q~_j = Q_j R_j
    C = Q.T @ A                           # step 8: C = Q_q^H A
    V, R = qr_posdiag(C.T)                # step 9: C^H = Q R
    Qh, Rh = qr_posdiag(R.T)              # step 10: R^H = Q_hat R_hat
    U = Q @ Qh                            # step 11: U_hat = Q_q Q_hat
    return EodAbeResult(U, Rh, V, r, eps, be["diagT"], be["blocks"], Q,
                        np.diag(R).copy())


def eod_abe(A: np.ndarray, tol: float, k: int = 32, q: int = 0, seed: int = 0,
            sketch_dtype=np.float64) -> EodAbeResult:
    """EOD-ABE (Alg. 2): A ~= U_hat D_hat V_hat^T with rank found by Alg. 1.

    A is promoted to FP64 (exact for FP32 input).  For m < n the
    factorization of A^T (= U' D' V'^T) is transposed back:
    A = V' D'^T U'^T and D'^T = Q' R' (QR), so U = V' Q', D = R', V = U'.
    """
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    if not (tol > 0 and math.isfinite(tol)):
        raise ValueError("tol must be positive and finite")
    if not 1 <= k:
        raise ValueError("block size must be >= 1")
    m, n = A.shape
    if m >= n:
        return _eod_abe_tall(A, tol, k, q, seed, sketch_dtype)
    t = _eod_abe_tall(A.T, tol, k, q, seed, sketch_dtype)
    if t.rank == 0:
        return EodAbeResult(t.V, t.D, t.U, 0, t.eps, t.diagT, t.blocks,
                            t.Qbasis, t.R_values)
    Qp, Rp = qr_posdiag(t.D.T)
    return EodAbeResult(t.V @ Qp, Rp, t.U, t.rank, t.eps, t.diagT, t.blocks,
                        t.Qbasis, t.R_values)


# ---------------------------------------------------------------------------
# Quality measures and the storage criterion (sections 1 and 4.1).
# ---------------------------------------------------------------------------
def rel_err(A: np.ndarray, U: np.ndarray, D: np.ndarray, V: np.ndarray) -> float:
    """RelErr = ||A - U D V^T||_F / ||A||_F (section 4.1, third criterion)."""
    A = np.asarray(A, dtype=np.float64)
    nrm = np.linalg.norm(A)
    if nrm == 0:
        return 0.0
    return float(np.linalg.norm(A - U @ D @ V.T) / nrm)


def eckart_young_relerr(A: np.ndarray, r: int) -> float:
    """Optimal rank-r relative error sqrt(sum_{i>r} sigma_i^2)/||A||_F from a
    full SVD (eq. udvd2: the best rank-r approximation in Frobenius norm)."""
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    tot = float(np.sqrt(np.sum(s * s)))
    return float(np.sqrt(np.sum(s[r:] ** 2)) / tot) if tot > 0 else 0.0


def storage_bytes(m: int, n: int, r: int) -> float:
    """Entries kept by the factors U (m x r), D (r x r upper) and V (n x r):
    (m + n) r + r (r + 1) / 2 (introduction, storage example)."""
    return (m + n) * r + r * (r + 1) / 2


def storage_rank_bound(m: int, n: int) -> float:
    """Largest rank for which the factors take less storage than A (m n):
    the positive root of r^2 + (2(m+n)+1) r - 2mn = 0, i.e.
    sqrt(m^2 + n^2 + 4mn + m + n + 1/4) - (m + n + 1/2) (introduction)."""
    return math.sqrt(m * m + n * n + 4 * m * n + m + n + 0.25) - (m + n + 0.5)


def siam_bound_sq(A: np.ndarray, r: int, Omega_r: np.ndarray, q: int = 0) -> float:
    """Deterministic part of Theorem siam for one draw:
    ||A - A_hat||_F^2 <= alpha^{4q} ||Sigma_0 Lambda_2 Lambda_1^+||_F^2
                         + ||Sigma_0||_F^2,
    alpha = sigma_{r+1}/sigma_r, Lambda_1 = V_r^T Omega, Lambda_2 = V_0^T Omega
    (V from the SVD of A, Omega the n x d test matrix actually used)."""
    A = np.asarray(A, dtype=np.float64)
    _, s, Vt = np.linalg.svd(A, full_matrices=True)
    n = A.shape[1]
    sfull = np.zeros(n)
    sfull[: s.size] = s
    L1 = Vt[:r] @ Omega_r
    L2 = Vt[r:] @ Omega_r
    S0 = sfull[r:]
    lead = np.linalg.norm((S0[:, None] * L2) @ np.linalg.pinv(L1)) ** 2
    alpha = sfull[r] / sfull[r - 1] if r < n and sfull[r - 1] > 0 else 0.0
    return float(alpha ** (4 * q) * lead + np.sum(S0 ** 2))


# Factor by which the summation-order-dependent part of an FP32 |T(l,l)|
# may differ between valid FP32 implementations (three orders measured in
# the pins differ by up to 1.95x; the pin asserts every one lies within this
# factor of the emulation's).
ORDER_SPREAD = 3.0


def precision_stable(A: np.ndarray, tol: float, k: int = 32, seed: int = 0,
                     lowp=np.float32) -> tuple[bool, int, int]:
    """Classify an instance as precision-stable: the FP64 run of Alg. 1 and
    the emulation with lower-precision data (FP32 data by default, or the
    "f16" / "bf16" sketch form) return the same rank, and eps lies outside
    every examined column's rounding band.

    The band: the emulated value splits as d_lp^2 = d_64^2 + rho^2, where
    d_64 (the FP64 run on the same input) is fixed by the input and rho is
    the part that rounding inside the run adds.  rho depends on the order in
    which a correct implementation sums, by up to ORDER_SPREAD either way,
    so its value may be anywhere in
    [sqrt(d_64^2 + rho^2 / S^2), sqrt(d_64^2 + S^2 rho^2)], S = ORDER_SPREAD.
    If eps falls there, the column's side of eps, and so the rank, is not a
    property of the input (rank parity is then a margin property)."""
    m, n = A.shape
    At = np.asarray(A, dtype=np.float64)
    if m < n:
        At = At.T
    nrm = float(np.sqrt(np.sum(At * At)))
    if nrm == 0.0:
        return True, 0, 0
    eps = tol * nrm
    b64 = basis_ext(At, eps, k, seed)
    blp = basis_ext(At, eps, k, seed, lowp)
    r64, rlp = b64["rank"], blp["rank"]
    nc = min(len(b64["diagT"]), len(blp["diagT"]))
    d64, dlp = b64["diagT"][:nc], blp["diagT"][:nc]
    rho2 = np.maximum(dlp * dlp - d64 * d64, 0.0)
    S = ORDER_SPREAD
    lo = np.sqrt(d64 * d64 + rho2 / (S * S))
    hi = np.sqrt(d64 * d64 + (S * S) * rho2)
    near = bool(np.any((lo <= eps) & (eps <= hi)))
    return (r64 == rlp) and not near, r64, rlp
