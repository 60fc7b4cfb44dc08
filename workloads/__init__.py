"""Seeded synthetic inputs for EOD-ABE tests and benchmarks.

This module holds input generators only: none of the method's arithmetic
lives here, so both the CPU oracle and the GPU path may use it.  Every
generator is a pure function of its arguments (NumPy ``default_rng(seed)``).

Workloads (shapes and value models stand in for the paper's data sets,
which are not available):

* ``lowrank_haar``   exact-rank matrix U diag(s) V^T + E with Haar U, V and
                     s_i = 10^{-3(i-1)/(r-1)} (512 x 512, rank 20 by default).
* ``lowrank_complex`` the complex analogue U diag(s) V^H + E (complex Haar
                     U, V; E circular complex Gaussian).
* ``image``          image-like matrix in [0, 255]: Gaussian blobs (rank 1
                     each) plus low-frequency cosine modes (rank <= 2 each)
                     plus i.i.d. pixel noise (stand-in for the paper's
                     photographs, section 4.1).
* ``hyperspectral``  pixels x bands = Dirichlet abundances x smooth spline
                     endmember spectra + noise (stand-in for Indian Pines,
                     section 4.2).
* ``rgb_image``      three channels of ``image`` (independent seeds): a
                     colour-image stand-in (section 4.1 uses 512 x 512 and
                     768 x 512 photographs).
* ``exact_rank_rgb`` three non-negative channels of chosen exact ranks in
                     [0, 255] (the 220 x 220 example of the introduction,
                     ranks 50, 52, 53).
* ``hyperspectral_labelled``  the hyperspectral matrix with a class label
                     per pixel (its dominant endmember) and a seeded fold
                     index for ten-fold cross-validation (section 4.2).
* ``tiles``          many image tiles of uneven size, each of exact rank
                     rho in [5, 80] plus small noise.
* ``mat2``           strictly rank-deficient U [Sigma 0; 0 0] V^T with sorted
                     uniform singular values (section 4.5, eq. mat2).
* ``robustness``     Matrix I-IV of section 4.3.
* ``spectrum_sigma`` / ``spectrum_torch``  U diag(sigma) V^T + noise with a
                     chosen singular-value profile (geometric, polynomial or
                     stepped decay), Haar U and V, built on a torch device
                     from a seeded generator (training and evaluation sets
                     of the learned warm start, 4096 x 4096 evaluation
                     matrices).
"""
from __future__ import annotations

import numpy as np

__all__ = ["haar", "lowrank_haar", "lowrank_complex", "image", "rgb_image", "exact_rank_rgb", "hyperspectral",
           "hyperspectral_labelled", "tiles", "tile_shapes", "mat2", "robustness", "devils_stairs_sigma",
           "spectrum_sigma", "spectrum_torch"]


def haar(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    """n x r matrix with orthonormal columns, Haar-distributed: Q factor of a
    Gaussian matrix with the signs fixed by diag(R) > 0 (Mezzadri 2007)."""
    G = rng.standard_normal((n, r))
    Qm, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Qm * s[None, :]


def lowrank_haar(seed: int, m: int = 512, n: int = 512, r: int = 20,
                 noise_std: float = 1e-12, decades: float = 3.0,
                 dtype=np.float64) -> np.ndarray:
    """A = U diag(s) V^T + E: U (m x r), V (n x r) Haar, s_i =
    10^{-decades (i-1)/(r-1)}, E i.i.d. N(0, noise_std^2)."""
    rng = np.random.default_rng(seed)
    U = haar(rng, m, r)
    V = haar(rng, n, r)
    s = 10.0 ** (-decades * np.arange(r) / max(r - 1, 1)) if r > 0 else np.zeros(0)
    A = (U * s[None, :]) @ V.T
    if noise_std:
        A = A + noise_std * rng.standard_normal((m, n))
    return A.astype(dtype)


def lowrank_complex(seed: int, m: int = 400, n: int = 300, r: int = 20, noise_std: float = 0.0,
                    decades: float = 3.0) -> np.ndarray:
    """Complex m x n matrix U diag(s) V^H + E: U, V the unitary factors of
    QR of complex Gaussian matrices with the phases of R's diagonal
    removed (Haar), s_i = 10^{-decades (i-1)/(r-1)}, E with independent
    N(0, noise_std^2 / 2) real and imaginary parts (complex128)."""
    rng = np.random.default_rng(seed)

    def chaar(k):
        G = rng.standard_normal((k, r)) + 1j * rng.standard_normal((k, r))
        Qm, R = np.linalg.qr(G)
        d = np.diag(R)
        return Qm * (d / np.abs(d))[None, :]

    U, V = chaar(m), chaar(n)
    s = 10.0 ** (-decades * np.arange(r) / max(r - 1, 1)) if r > 0 else np.zeros(0)
    A = (U * s[None, :]) @ V.conj().T
    if noise_std:
        A = A + noise_std * np.sqrt(0.5) * (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    return A


def image(seed: int, size: int = 4096, noise_std: float = 0.5, blobs: int = 64,
          modes: int = 32, sigma_px=(20.0, 400.0), dtype=np.float32,
          width: int | None = None) -> np.ndarray:
    """Image-like size x width matrix with values in [0, 255] before noise.

    64 isotropic Gaussian blobs (centre uniform over the image, sigma uniform
    in [20, 400] px, amplitude U[-1, 1]; each is a separable outer product,
    rank 1) plus 32 cosine modes cos(2 pi (fx x + fy y)/N + phi) with
    fx, fy in {0..7} and amplitude U[-0.3, 0.3] (rank <= 2 each), affinely
    scaled to [0, 255] without clipping, plus i.i.d. N(0, noise_std^2).
    Signal rank <= blobs + 2 modes + 1.
    """
    rng = np.random.default_rng(seed)
    h = size
    w = size if width is None else width
    y = np.arange(h, dtype=np.float64)
    x = np.arange(w, dtype=np.float64)
    # the image is a sum of outer products: collect the factors, one matmul
    fy, fx = [], []
    for _ in range(blobs):
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        sg = rng.uniform(*sigma_px)
        amp = rng.uniform(-1.0, 1.0)
        fy.append(amp * np.exp(-0.5 * ((y - cy) / sg) ** 2))
        fx.append(np.exp(-0.5 * ((x - cx) / sg) ** 2))
    n_ref = float(max(h, w))
    for _ in range(modes):
        ky, kx = rng.integers(0, 8, size=2)
        phi = rng.uniform(0, 2 * np.pi)
        amp = rng.uniform(-0.3, 0.3)
        ay = 2 * np.pi * ky * y / n_ref
        ax = 2 * np.pi * kx * x / n_ref + phi
        # cos(ay + ax) = cos ay cos ax - sin ay sin ax  (rank <= 2)
        fy += [amp * np.cos(ay), -amp * np.sin(ay)]
        fx += [np.cos(ax), np.sin(ax)]
    img = np.stack(fy, axis=1) @ np.stack(fx, axis=1).T
    lo, hi = img.min(), img.max()
    img = (img - lo) * (255.0 / (hi - lo)) if hi > lo else np.zeros_like(img)
    if noise_std:
        img += noise_std * rng.standard_normal((h, w))
    return img.astype(dtype)


def rgb_image(seed: int, h: int = 512, w: int = 512, noise_std: float = 0.05,
              dtype=np.float32) -> np.ndarray:
    """channels x h x w colour image: channel c is ``image(3 seed + c)``."""
    return np.stack([image(3 * seed + c, h, noise_std, width=w, dtype=np.float64)
                     for c in range(3)]).astype(dtype)


def exact_rank_rgb(seed: int, h: int = 220, w: int = 220, ranks=(50, 52, 53),
                   dtype=np.float32) -> np.ndarray:
    """Non-negative channels of exact ranks: channel c = W_c H_c with W_c
    (h x r_c) and H_c (r_c x w) uniform in [0, 1], scaled so the largest
    entry is 255."""
    rng = np.random.default_rng(seed)
    out = []
    for r in ranks:
        C = rng.uniform(0, 1, (h, r)) @ rng.uniform(0, 1, (r, w))
        out.append(C * (255.0 / C.max()))
    return np.stack(out).astype(dtype)


def _clamped_spline(xk: np.ndarray, yk: np.ndarray, xs: np.ndarray) -> np.ndarray:
    from scipy.interpolate import CubicSpline
    return CubicSpline(xk, yk, bc_type="clamped")(xs)


def hyperspectral(seed: int, pixels: int = 262144, bands: int = 200,
                  endmembers: int = 15, knots: int = 40, alpha: float = 0.5,
                  noise_std: float = 1e-3, dtype=np.float32) -> np.ndarray:
    """pixels x bands matrix = abundances (Dirichlet(alpha 1)) @ endmember
    spectra + N(0, noise_std^2).  Each spectrum is a clamped cubic spline
    through ``knots`` U[0,1] control points on [0, 1], clipped to [0, 1]."""
    return _hyperspectral(seed, pixels, bands, endmembers, knots, alpha, noise_std)[0].astype(dtype)


def _hyperspectral(seed, pixels, bands, endmembers, knots, alpha, noise_std):
    rng = np.random.default_rng(seed)
    xk = np.linspace(0.0, 1.0, knots)
    xs = np.linspace(0.0, 1.0, bands)
    E = np.stack([np.clip(_clamped_spline(xk, rng.uniform(0, 1, knots), xs), 0, 1)
                  for _ in range(endmembers)])
    Ab = rng.dirichlet(alpha * np.ones(endmembers), size=pixels)
    A = Ab @ E
    if noise_std:
        A += noise_std * rng.standard_normal((pixels, bands))
    return A, Ab


def hyperspectral_labelled(seed: int, pixels: int = 21025, bands: int = 200, endmembers: int = 15,
                           knots: int = 40, alpha: float = 0.5, noise_std: float = 1e-3,
                           folds: int = 10, dtype=np.float32):
    """(A, labels, fold): the hyperspectral matrix of ``hyperspectral`` (same
    seed, same values; 21025 = 145 x 145 pixels by default, the Indian Pines
    scene's size), the label of each pixel = its dominant endmember (argmax
    abundance, 0-based), and its cross-validation fold = position in a
    seeded random permutation modulo ``folds``."""
    A, Ab = _hyperspectral(seed, pixels, bands, endmembers, knots, alpha, noise_std)
    labels = np.argmax(Ab, axis=1).astype(np.int32)
    perm = np.random.default_rng(seed + 7919).permutation(pixels)
    fold = np.empty(pixels, dtype=np.int32)
    fold[perm] = np.arange(pixels) % folds
    return A.astype(dtype), labels, fold


def tile_shapes(seed: int, count: int = 1024, lo: int = 64, hi: int = 1024,
                rank_lo: int = 5, rank_hi: int = 80):
    """(h, w, rho) per tile: h, w uniform integers in [lo, hi], rho uniform
    in [rank_lo, rank_hi] (capped at min(h, w))."""
    rng = np.random.default_rng(seed)
    h = rng.integers(lo, hi + 1, size=count)
    w = rng.integers(lo, hi + 1, size=count)
    rho = np.minimum(rng.integers(rank_lo, rank_hi + 1, size=count), np.minimum(h, w))
    return [(int(a), int(b), int(c)) for a, b, c in zip(h, w, rho)]


def tiles(seed: int, count: int = 1024, lo: int = 64, hi: int = 1024,
          rank_lo: int = 5, rank_hi: int = 80, noise_std: float = 1e-4,
          dtype=np.float32):
    """List of tiles c U diag(s) V^T + N(0, noise_std^2) with exact-rank
    content rho (Haar U, V; s_i = 10^{-3(i-1)/(rho-1)}; c = 255/max|U S V^T|
    so the content spans [-255, 255])."""
    shapes = tile_shapes(seed, count, lo, hi, rank_lo, rank_hi)
    out = []
    for t, (h, w, rho) in enumerate(shapes):
        rng = np.random.default_rng([seed, t])
        U = haar(rng, h, rho)
        V = haar(rng, w, rho)
        s = 10.0 ** (-3.0 * np.arange(rho) / max(rho - 1, 1))
        T = (U * s[None, :]) @ V.T
        T *= 255.0 / np.abs(T).max()
        if noise_std:
            T += noise_std * rng.standard_normal((h, w))
        out.append(T.astype(dtype))
    return out


def mat2(seed: int, n: int, r: int, dtype=np.float64) -> np.ndarray:
    """Strictly rank-deficient n x n matrix U [Sigma 0; 0 0] V^T, U and V
    orthogonal (Q of a Gaussian), Sigma = uniform(0,1) values sorted
    descending (section 4.5, eq. mat2)."""
    rng = np.random.default_rng(seed)
    U = haar(rng, n, r)
    V = haar(rng, n, r)
    s = np.sort(rng.uniform(0.0, 1.0, r))[::-1]
    return ((U * s[None, :]) @ V.T).astype(dtype)


def devils_stairs_sigma(n: int, step: int = 15, drop: float = 0.8) -> np.ndarray:
    """sigma_i = 10^{-drop floor((i-1)/step)} (section 4.3, Matrix II)."""
    i = np.arange(1, n + 1)
    return 10.0 ** (-drop * np.floor((i - 1) / step))


def robustness(kind: str, seed: int, n: int = 1000, alpha: float = 0.005,
               dtype=np.float64) -> np.ndarray:
    """Matrix I-IV of section 4.3 (U, V Haar n x n).

    I:   rank 20, sigma_1..sigma_20 linear from 1 to 1e-25, plus
         alpha * sigma_r * E with E Gaussian scaled to unit spectral norm
         (the reading that gives the stated gap ~ 1/alpha; sigma_r is taken
         as the smallest singular value above the noise, 1/20 here on the
         linear grid's last step above 1e-25 -- see the design notes).
    II:  devil's stairs, sigma_i = 10^{-0.8 floor((i-1)/15)}.
    III: sigma_i = exp(-i/6).      IV: sigma_i = i^{-2}.
    """
    rng = np.random.default_rng(seed)
    U = haar(rng, n, n)
    V = haar(rng, n, n)
    i = np.arange(1, n + 1, dtype=np.float64)
    if kind == "I":
        r = 20
        s = np.zeros(n)
        s[:r] = np.linspace(1.0, 1e-25, r)
        A = (U * s[None, :]) @ V.T
        E = rng.standard_normal((n, n))
        E /= np.linalg.norm(E, 2)
        A = A + alpha * s[r - 2] * E
    elif kind == "II":
        A = (U * devils_stairs_sigma(n)[None, :]) @ V.T
    elif kind == "III":
        A = (U * np.exp(-i / 6.0)[None, :]) @ V.T
    elif kind == "IV":
        A = (U * (i ** -2.0)[None, :]) @ V.T
    else:
        raise ValueError(kind)
    return A.astype(dtype)


def spectrum_sigma(kind: str, r: int, param: float) -> np.ndarray:
    """Singular values s_0 >= ... >= s_{r-1} > 0 with s_0 = 1:
    geom    s_i = 10^{-param i / r}          (param decades over the rank)
    poly    s_i = (1 + i)^{-param}
    stairs  s_i = 10^{-0.8 floor(i / param)}  (steps of param values)"""
    i = np.arange(r, dtype=np.float64)
    if kind == "geom":
        return 10.0 ** (-param * i / r)
    if kind == "poly":
        return (1.0 + i) ** (-param)
    if kind == "stairs":
        return 10.0 ** (-0.8 * np.floor(i / max(param, 1.0)))
    raise ValueError(kind)


def spectrum_torch(seed: int, m: int, n: int, sigma: np.ndarray, noise_std: float = 0.0,
                   device: str = "cuda", dtype=None):
    """A = U diag(sigma) V^T + N(0, noise_std^2) on a torch device: U (m x r)
    and V (n x r) Haar (Q factors of seeded Gaussians with the signs of
    diag(R) folded in), FP64 arithmetic, returned in dtype (FP64 default)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = len(sigma)
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)

    def haar_t(rows):
        G = torch.randn(rows, r, generator=g, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(G)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d
    U, V = haar_t(m), haar_t(n)
    A = (U * s) @ V.T
    if noise_std:
        A += noise_std * torch.randn(m, n, generator=g, device=device, dtype=torch.float64)
    return A if dtype is None else A.to(dtype)
