"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (written per test):
* Philox words: bit-exact.  Gaussian entries: FP32 values equal except for
  at most a few 1-ulp differences (both sides evaluate Box-Muller in FP64
  with their own libm and round to FP32).
* Sketch A*Omega: elementwise |Y - Y_ref| <= K u (|A| |Omega|) (the
  classical bound of a length-K dot product in the data precision).
* Rank: equal to the oracle's rank on every precision-stable instance
  (FP64 runs: always; FP32 runs: where the FP64 oracle and its FP32-data
  emulation agree).  diag(T) within the precision's resolution.
* RelErr = ||A - U D V^T||_F / ||A||_F within 1e-10 (FP64) or 1e-5 (FP32)
  of the oracle's, absolute; orthonormality of U and V; D upper triangular
  with a non-negative diagonal.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle.eodabe_oracle as O  # noqa: E402
import paper_2506_22713_amd as E  # noqa: E402
import workloads as W  # noqa: E402

U32 = 2.0 ** -24
U64 = 2.0 ** -53
RELERR_TOL = {torch.float32: 1e-5, torch.float64: 1e-10}
ORTH_TOL = {torch.float32: 5e-5, torch.float64: 1e-12}


def say(*a):
    print("[case]", *a, flush=True)


def dev(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(A)).to(device="cuda", dtype=dtype)


def fp32_floor(r, m, n):
    """Relative-error floor of an FP32 factorization of rank r of an m x n
    matrix: the sketches and C = Q^T A carry rounding of about
    u32 sqrt(max(m, n)) per captured direction, and r directions add in
    quadrature (bounded by 4 u32 sqrt(r max(m, n))).  It exceeds 1e-5 for
    noiseless exact-rank content of rank ~100 at these sizes."""
    return 4.0 * U32 * math.sqrt(max(r, 1) * max(m, n))


def gpu_relerr(A64, f):
    U = f.U.double().cpu().numpy()
    D = f.D.double().cpu().numpy()
    Vt = f.Vt.double().cpu().numpy()
    nrm = np.linalg.norm(A64)
    return float(np.linalg.norm(A64 - U @ D @ Vt) / nrm) if nrm else 0.0, U, D, Vt


def check_factor(A64, dtype, tol, b=32, q=0, seed=0, stable=True, rounding_only=False, bar_override=None):
    """GPU factorization against the oracle: same rank, RelErr within the
    data type's bar, orthonormal factors, D upper triangular with a
    non-negative diagonal.  rounding_only: the content is noise-free and of
    exact rank, so the oracle's RelErr is its own rounding error amplified
    by the conditioning of the sketched block (the first r columns of A Omega
    form a square sketch of an r-dimensional range); the FP32 path carries
    the same amplification of its unit roundoff, and its bar is widened to
    4 (u32/u64) times the oracle's RelErr."""
    say("factor", A64.shape, dtype, "tol", tol, "b", b, "q", q, "seed", seed, "stable", stable)
    ref = O.eod_abe(A64, tol, k=b, q=q, seed=seed)
    f = E.factor(dev(A64, dtype), tol, block=b, power_iters=q, seed=seed)
    torch.cuda.synchronize()
    cmp = ref
    if stable:
        assert f.rank == ref.rank, (f.rank, ref.rank)
    elif f.rank != ref.rank:
        # a precision-unstable rank decision: the GPU must land on the other
        # side's rank, that of the oracle's FP32-data emulation, and is
        # compared with that run
        cmp = O.eod_abe(A64, tol, k=b, q=q, seed=seed, sketch_dtype=np.float32)
        assert f.rank == cmp.rank, (f.rank, ref.rank, cmp.rank)
    if f.rank == 0:
        return f, ref
    e_gpu, U, D, Vt = gpu_relerr(A64, f)
    e_ref = O.rel_err(A64, cmp.U, cmp.D, cmp.V)
    bar = RELERR_TOL[dtype]
    if dtype == torch.float32 and rounding_only:
        # only for content whose oracle error is FP64 rounding (noise-free,
        # exact rank); a truncation error here would make the bar vacuous
        assert e_ref < 1e-9, ("rounding_only used on content with a truncation error", e_ref)
        bar = max(bar, fp32_floor(f.rank, *A64.shape), 4.0 * (U32 / U64) * e_ref)
    if bar_override is not None:
        bar = bar_override
    say(f"  rank {f.rank} relerr gpu {e_gpu:.3e} oracle {e_ref:.3e} diff {abs(e_gpu - e_ref):.2e} bar {bar:.1e}")
    assert abs(e_gpu - e_ref) <= bar, (e_gpu, e_ref, bar)
    r = f.rank
    assert np.linalg.norm(U.T @ U - np.eye(r)) <= ORTH_TOL[dtype] * math.sqrt(r)
    assert np.linalg.norm(Vt @ Vt.T - np.eye(r)) <= ORTH_TOL[dtype] * math.sqrt(r)
    assert np.all(np.tril(D, -1) == 0) and np.all(np.diag(D) >= 0)
    return f, ref


@pytest.fixture(scope="module")
def ctx32():
    return E.Context(dtype=torch.float32, seed=1234)


# ---------------------------------------------------------------- RNG
@pytest.mark.parametrize("seed", [0, 1234, 2 ** 40 + 7])
def test_philox_bit_exact(seed):
    say("philox", seed)
    c = E.Context(seed=seed)
    n = 5000
    got = E.philox(c, seed, 17, 3, 9, n).cpu().numpy().view(np.uint32)
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = 17 + np.arange(n)
    ctr[:, 1] = 3
    ctr[:, 2] = 9
    ref = O.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_omega_matches_oracle(dtype):
    say("omega", dtype)
    c = E.Context(seed=99, dtype=dtype)
    n, col0, nc = 1003, 37, 21
    got = E.omega(c, n, col0, nc, dtype=dtype).double().cpu().numpy()
    ref = O.omega_columns(99, n, col0, nc)
    diff = got != ref
    assert diff.mean() <= 1e-4
    if diff.any():
        g32, r32 = got[diff].astype(np.float32), ref[diff].astype(np.float32)
        ulp = np.abs(g32.view(np.int32).astype(np.int64) - r32.view(np.int32).astype(np.int64))
        assert ulp.max() <= 1


# ---------------------------------------------------------------- sketch
@pytest.mark.parametrize("m,n,nc,col0", [(300, 200, 32, 0), (1000, 777, 20, 64), (4099, 4100, 32, 32),
                                         (129, 33, 128, 0), (5000, 17, 16, 3)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_sketch_matches_oracle_product(m, n, nc, col0, dtype):
    say("sketch", m, n, nc, col0, dtype)
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    if dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    c = E.Context(seed=5, dtype=dtype)
    Y = E.sketch(c, dev(A, dtype), col0, nc).double().cpu().numpy()
    Om = O.omega_columns(5, n, col0, nc)
    ref = A @ Om
    bound = n * (U32 if dtype == torch.float32 else U64) * (np.abs(A) @ np.abs(Om)) + 1e-300
    assert np.all(np.abs(Y - ref) <= bound)


def test_sketch_unaligned_leading_dimension():
    say("sketch unaligned lda")
    rng = np.random.default_rng(3)
    big = rng.standard_normal((200, 103)).astype(np.float32)
    At = torch.from_numpy(big).cuda()[:, :101]                 # lda = 103 (not a multiple of 4)
    c = E.Context(seed=8)
    Y = E.sketch(c, At, 0, 16).double().cpu().numpy()
    A = big[:, :101].astype(np.float64)
    ref = A @ O.omega_columns(8, 101, 0, 16)
    assert np.all(np.abs(Y - ref) <= 101 * U32 * (np.abs(A) @ np.abs(O.omega_columns(8, 101, 0, 16))))


# ---------------------------------------------------------------- Alg. 1
@pytest.mark.parametrize("seed", range(5))
def test_basis_c1_fp64(seed):
    say("basis C1 fp64", seed)
    A = W.lowrank_haar(seed)
    nrm = np.linalg.norm(A)
    ref = O.basis_ext(A, 1e-8 * nrm, 32, seed)
    Q, d, info = E.basis(dev(A, torch.float64), 1e-8, block=32, seed=seed, dtype=torch.float64)
    assert info.rank == ref["rank"]
    k = min(len(d), len(ref["diagT"]))
    assert np.max(np.abs(d[:k] - ref["diagT"][:k])) <= 1e-12 * nrm
    Qn = Q.cpu().numpy()
    assert np.linalg.norm(Qn.T @ Qn - np.eye(info.rank)) < 1e-12
    # same subspace as the oracle's basis, to the resolution of the weakest
    # accepted direction (rounding u ||A|| over its pivot)
    dmin = ref["diagT"][: info.rank].min()
    assert np.linalg.norm(Qn @ (Qn.T @ ref["Q"]) - ref["Q"]) < 100 * U64 * nrm / dmin * math.sqrt(info.rank)


@pytest.mark.parametrize("seed", range(6))
def test_basis_c1_fp32(seed):
    say("basis C1 fp32", seed)
    A = W.lowrank_haar(seed).astype(np.float32).astype(np.float64)
    stable, r64, r32 = O.precision_stable(A, 1e-5, 32, seed)
    Q, d, info = E.basis(dev(A, torch.float32), 1e-5, block=32, seed=seed)
    if stable:
        assert info.rank == r64
    ref = O.basis_ext(A, 1e-5 * np.linalg.norm(A), 32, seed)
    k = min(len(d), len(ref["diagT"]))
    assert np.max(np.abs(d[:k] - ref["diagT"][:k])) <= 64 * math.sqrt(A.shape[1]) * U32 * np.linalg.norm(A)


# ---------------------------------------------------------------- Alg. 2
@pytest.mark.parametrize("seed", range(4))
def test_factor_c1_fp64(seed):
    check_factor(W.lowrank_haar(seed), torch.float64, 1e-8, seed=seed)


@pytest.mark.parametrize("seed", range(4))
def test_factor_c1_fp32(seed):
    A = W.lowrank_haar(seed).astype(np.float32).astype(np.float64)
    stable, _, _ = O.precision_stable(A, 1e-5, 32, seed)
    check_factor(A, torch.float32, 1e-5, seed=seed, stable=stable)


def test_factor_exact_rank_matches_oracle_factors():
    A = W.lowrank_haar(7, m=400, n=300, r=20, noise_std=0.0)
    f, ref = check_factor(A, torch.float64, 1e-10, b=16, seed=7)
    # factors are unique (positive diagonals): compare element by element
    D = f.D.cpu().numpy()
    assert np.max(np.abs(D - ref.D)) <= 1e-9 * np.abs(ref.D).max()
    U = f.U.cpu().numpy()
    assert np.max(np.abs(U - ref.U)) <= 1e-7


@pytest.mark.parametrize("q", [1, 2])
def test_factor_power_iteration(q):
    A = W.lowrank_haar(3)
    f, ref = check_factor(A, torch.float64, 1e-8, q=q, seed=3)
    ey = O.eckart_young_relerr(A, f.rank)
    e, *_ = gpu_relerr(A, f)
    assert abs(e - ey) <= 1e-10


@pytest.mark.parametrize("m,n", [(700, 400), (300, 650)])
def test_factor_power_iteration_fp32(m, n):
    # q = 1 in FP32, tall and wide (the wide one iterates on A^T): noisy
    # content with a decaying spectrum, compared with the oracle at q = 1
    A = W.lowrank_haar(31, m=m, n=n, r=60, noise_std=1e-6, decades=3.0).astype(np.float32).astype(np.float64)
    stable, _, _ = O.precision_stable(A, 1e-4, 16, 31)
    f, ref = check_factor(A, torch.float32, 1e-4, b=16, q=1, seed=31, stable=stable)
    assert f.rank > 16


def test_factor_wide_matrix():
    A = W.lowrank_haar(4, m=150, n=420, r=12, noise_std=0.0)
    check_factor(A, torch.float64, 1e-9, b=8, seed=4)


def test_factor_wide_high_rank():
    # m < n with rank above 64: the closing QR of D'^T takes the wide path
    A = W.lowrank_haar(5, m=100, n=260, r=80, noise_std=0.0)
    check_factor(A, torch.float64, 1e-9, b=32, seed=5)


@pytest.mark.parametrize("b", [24, 48])
def test_factor_multi_block_wide_blocks(b):
    # several blocks of 17..64 columns (Cholesky kernels of width 32 and 64),
    # each later block projected against the basis before and after its
    # first Cholesky pass
    A = W.lowrank_haar(11, m=600, n=300, r=100, noise_std=1e-11)
    f, ref = check_factor(A, torch.float64, 1e-8, b=b, seed=11)
    assert f.blocks >= 3


@pytest.mark.parametrize("b", [96, 128])
def test_factor_multi_block_blocked_cholesky(b):
    # blocks of 65..128 columns: Gram, 2 x 2-blocked Cholesky with inverse
    # and explicit-inverse applies, projected against a basis of up to 2b
    # columns; the closing (rank 150) takes the general wide path
    A = W.lowrank_haar(12, m=700, n=400, r=150, noise_std=1e-11)
    f, ref = check_factor(A, torch.float64, 1e-8, b=b, seed=12)
    assert f.blocks >= 2


@pytest.mark.parametrize("m,n", [(900, 500), (500, 900)])
def test_factor_rank_300_panel_blocked_cholesky(m, n):
    # ranks above 128 close through the panel-blocked Cholesky with inverse
    # (five 64-column panels, the last one ragged) and FP64-weight products
    A = W.lowrank_haar(14, m=m, n=n, r=300, noise_std=0.0)
    f, ref = check_factor(A, torch.float64, 1e-9, b=32, seed=14)
    assert f.rank == 300


def test_factor_rank_520_recursive_inverse():
    say("factor rank 520")
    # nine 64-column panels (the last one 8 wide): the inverse of the wide
    # Cholesky runs four recursive-doubling levels (groups of 1, 2, 4, 8
    # blocks), the last with a partial group
    A = W.lowrank_haar(16, m=1100, n=600, r=520, noise_std=0.0)
    f, ref = check_factor(A, torch.float64, 1e-9, b=64, seed=16)
    assert f.rank == 520


@pytest.mark.parametrize("m,n,dtype", [(16384, 300, torch.float64), (12000, 260, torch.float32)])
def test_factor_many_split_partials(m, n, dtype):
    say(f"factor {m}x{n} many K-split partials")
    # a long, narrow matrix: the projection C = Q^T A runs with 64 and 45
    # K-split partials, folded in fixed order by the partial-sum kernel
    # (more than its 16-partial load batch, ragged in the second batch)
    A = W.lowrank_haar(17, m=m, n=n, r=40, noise_std=0.0)
    tol = 1e-9 if dtype == torch.float64 else 1e-4
    f, ref = check_factor(A, dtype, tol, b=32, seed=17, rounding_only=True)
    assert f.rank == 40


@pytest.mark.parametrize("m,n,r,dtype,tol,b", [
    (4100, 700, 60, torch.float32, 1e-4, 32),     # ragged last row tile; 3 blocks
    (4200, 520, 45, torch.float64, 1e-9, 16),     # one-tile-wide blocks; a wave with an empty K part
    (600, 4097, 50, torch.float32, 1e-4, 32),     # wide: the transposed copy has 4097 rows
])
def test_factor_row_tile_sketch(m, n, r, dtype, tol, b):
    # 4081 or more rows with blocks of at most 32 columns: the sketch runs by
    # 16-row tiles over the whole K range (eight waves per tile, summed in
    # LDS) and writes Y directly, on every block
    say(f"factor {m}x{n} row-tile sketch")
    A = W.lowrank_haar(23 + m, m=m, n=n, r=r, noise_std=0.0, decades=2.0)
    stable = True
    if dtype == torch.float32:
        stable, _, _ = O.precision_stable(A, tol, b, 23)
    f, ref = check_factor(A, dtype, tol, b=b, seed=23, stable=stable, rounding_only=True)
    assert f.blocks >= 2


EDGE_SIDES = [1, 2, 3, 7, 15, 16, 17, 31, 33, 63, 64, 65, 127, 129, 255, 257, 300, 511, 513, 640]


def random_case(i):
    """Case i of the random-shape sweep: sides drawn from tile and panel
    edges, content rank up to 100, block width, dtype and tolerance drawn
    from seeded generators (FP64: tol 1e-10..1e-5, well below the content's
    smallest singular value; FP32: tol 1e-4..1e-3 with 2 decades of
    spectrum)."""
    rng = np.random.default_rng(7000 + i)
    m, n = (int(x) for x in rng.choice(EDGE_SIDES, 2))
    r = int(rng.integers(0, min(m, n, 100) + 1))
    b = int(rng.choice([1, 8, 16, 20, 32, 48, 64]))
    fp64 = i % 2 == 0
    tol = float(10.0 ** -rng.uniform(5, 10)) if fp64 else float(10.0 ** -rng.uniform(3, 4))
    A = W.lowrank_haar(7000 + i, m=m, n=n, r=r, noise_std=0.0, decades=3.0 if fp64 else 2.0)
    return A, (torch.float64 if fp64 else torch.float32), tol, b


@pytest.mark.parametrize("i", range(24))
def test_factor_random_shapes(i):
    A, dtype, tol, b = random_case(i)
    say(f"random case {i}: {A.shape} {dtype} tol {tol:.2e} b {b}")
    stable = True
    if dtype == torch.float32:
        stable, _, _ = O.precision_stable(A, tol, b, 7000 + i)
    check_factor(A, dtype, tol, b=b, seed=7000 + i, stable=stable, rounding_only=True)


@pytest.mark.parametrize("m,n,r", [(1, 1, 1), (1, 300, 1), (300, 1, 1), (2, 513, 2), (513, 2, 1), (1, 64, 0)])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-8), (torch.float32, 1e-4)])
@pytest.mark.parametrize("b", [1, 32])
def test_factor_degenerate_sides(m, n, r, dtype, tol, b):
    # one or two rows or columns: a single K step, panels of one column,
    # the transposed orientation for the wide ones
    A = W.lowrank_haar(11, m=m, n=n, r=r, noise_std=0.0)
    f, ref = check_factor(A, dtype, tol, b=b, seed=11, rounding_only=True)
    assert f.rank == r


@pytest.mark.parametrize("case", ["fp64_noise", "fp64_b8", "fp64_wide", "fp64_b96", "fp32_noise", "full_rank"])
def test_relres_estimate_matches_oracle(case):
    # info.relres_est = |T(l,l)| / ||A||_F at the column whose test stopped
    # the loop: the oracle's diag(T) entry at index rank, divided by its norm
    say("relres_est", case)
    dtype, b, tol = torch.float64, 32, 1e-6
    if case == "full_rank":
        A = W.lowrank_haar(21, m=120, n=40, r=40, noise_std=0.0, decades=1.0)
        tol = 1e-12
    elif case == "fp64_wide":
        A = W.lowrank_haar(22, m=150, n=700, r=30, noise_std=1e-9)
    elif case == "fp32_noise":
        dtype, tol = torch.float32, 1e-4
        A = W.lowrank_haar(23, m=900, n=500, r=60, noise_std=1e-9, decades=2.0)
    else:
        A = W.lowrank_haar(24, m=800, n=400, r=70, noise_std=1e-9)
        b = {"fp64_noise": 32, "fp64_b8": 8, "fp64_b96": 96}[case]
    ref = O.eod_abe(A, tol, k=b, q=0, seed=5)
    f = E.factor(dev(A, dtype), tol, block=b, seed=5)
    torch.cuda.synchronize()
    assert f.rank == ref.rank, (f.rank, ref.rank)
    nrm = float(np.linalg.norm(A))
    want = float(ref.diagT[ref.rank]) / nrm if len(ref.diagT) > ref.rank else 0.0
    if case == "full_rank":
        assert want == 0.0 and f.relres_est == 0.0
        return
    bar = 1e-12 if dtype == torch.float64 else 64 * math.sqrt(A.shape[1]) * U32
    assert want > 0.0
    assert abs(f.relres_est - want) <= bar, (f.relres_est, want, bar)
    # and it is the stopping column's value: at most tol (the test fired there)
    assert f.relres_est <= tol * (1 + 1e-12)


def test_factor_fp32_rank_250():
    A = W.lowrank_haar(15, m=1000, n=600, r=250, noise_std=1e-8)
    stable, _, _ = O.precision_stable(A, 1e-4, 64, 15)
    f, ref = check_factor(A, torch.float32, 1e-4, b=64, seed=15, stable=stable)
    assert 128 < f.rank <= 256


@pytest.mark.parametrize("m,n", [(800, 300), (300, 800)])
def test_factor_fp32_rank_100_closing(m, n):
    # ranks 65..128 close through the blocked Cholesky in FP32 (tall and
    # wide orientation)
    A = W.lowrank_haar(13, m=m, n=n, r=100, noise_std=1e-7)
    stable, _, _ = O.precision_stable(A, 1e-4, 32, 13)
    f, ref = check_factor(A, torch.float32, 1e-4, b=32, seed=13, stable=stable)
    assert 64 < f.rank <= 128


def test_factor_full_rank_ragged():
    A = np.random.default_rng(0).standard_normal((333, 70))
    f, ref = check_factor(A, torch.float64, 1e-13, b=16, seed=2)
    assert f.rank == 70 and f.blocks == 5


@pytest.mark.parametrize("b", [1, 8, 20, 64, 100, 128])
def test_factor_block_sizes(b):
    A = W.lowrank_haar(9, m=500, n=260, r=30, noise_std=1e-10)
    check_factor(A, torch.float64, 1e-7, b=b, seed=9)


def test_zero_matrix_rank_zero():
    say("zero matrix")
    f = E.factor(torch.zeros((64, 48), device="cuda"), 1e-3)
    assert f.rank == 0


def test_rank_zero_first_column():
    say("rank zero first column")
    A = W.lowrank_haar(1, m=64, n=64, r=3, noise_std=0.0)
    f = E.factor(dev(A, torch.float64), 10.0, block=8)
    assert f.rank == 0 and f.blocks == 1


def test_capacity_error():
    say("capacity")
    A = W.lowrank_haar(2, m=200, n=200, r=30, noise_std=0.0)
    with pytest.raises(E.EodAbeError) as ei:
        E.factor(dev(A, torch.float64), 1e-10, r_cap=10)
    assert ei.value.status == E.EODABE_ECAPACITY


def test_nonfinite_input():
    say("nonfinite")
    A = torch.ones((100, 80), device="cuda")
    A[5, 7] = float("nan")
    with pytest.raises(E.EodAbeError) as ei:
        E.factor(A, 1e-3)
    assert ei.value.status == E.EODABE_ENONFINITE


def test_tol_floor_warning():
    say("tol floor")
    A = W.lowrank_haar(0).astype(np.float32)
    f = E.factor(dev(A, torch.float32), 1e-9)
    assert f.status == E.EODABE_WTOL_FLOOR and (f.flags & 1)


def test_deterministic_runs():
    say("determinism")
    A = dev(W.image(1, 1024, 0.05), torch.float32)
    f1 = E.factor(A, 1e-3, seed=3)
    f2 = E.factor(A, 1e-3, seed=3)
    assert f1.rank == f2.rank
    assert torch.equal(f1.D, f2.D) and torch.equal(f1.U, f2.U) and torch.equal(f1.Vt, f2.Vt)


# ---------------------------------------------------------------- workloads
def test_image_small_fp32():
    A = W.image(0, 1024, 0.05).astype(np.float64)
    stable, _, _ = O.precision_stable(A, 1e-3, 32, 0)
    check_factor(A, torch.float32, 1e-3, seed=0, stable=stable)


def test_image_4096_headline_workload():
    # the benchmark's headline configuration at full size: the 4096^2 FP32
    # image (noise std 0.05), tol 1e-3, b = 32, seed 0 -- row-tile sketch,
    # one block, gated closing
    say("image 4096^2 headline workload")
    A = W.image(0, 4096, 0.05).astype(np.float64)
    stable, _, _ = O.precision_stable(A, 1e-3, 32, 0)
    f, ref = check_factor(A, torch.float32, 1e-3, b=32, seed=0, stable=stable)
    assert f.blocks == 1


@pytest.mark.parametrize("r", [96, 160])
def test_spectrum_4096_mid_ranks(r):
    # 4096^2 FP32 at ranks 95..160 (the benchmark's rank sweep, geometric
    # decay over 3 decades, tol 1e-4, b = 32): several blocks of the
    # row-tile sketch and BCGS2, the 65-128 or panel-blocked closing.  The
    # noise (1e-7 of ||A||_F) sits at the FP32 resolution of the data, so the
    # FP32 path adds its rounding floor (R7: 4 u32 sqrt(r max(m, n)), 1.5e-4
    # at rank 96) to the oracle's truncation error; that floor is the bar.
    say(f"spectrum 4096^2 rank {r}")
    sig = W.spectrum_sigma("geom", r, 3.0)
    noise = 1e-7 * float(np.sqrt((sig ** 2).sum()) / 4096)
    A = W.spectrum_torch(1000 + r, 4096, 4096, sig, noise, dtype=torch.float32).double().cpu().numpy()
    stable, _, _ = O.precision_stable(A, 1e-4, 32, 0)
    f, ref = check_factor(A, torch.float32, 1e-4, b=32, seed=0, stable=stable,
                          bar_override=max(1e-5, fp32_floor(r, 4096, 4096)))
    assert f.blocks >= 3


def test_hyperspectral_small_fp32():
    A = W.hyperspectral(0, pixels=16384).astype(np.float64)
    stable, _, _ = O.precision_stable(A, 1e-2, 16, 0)
    check_factor(A, torch.float32, 1e-2, b=16, seed=0, stable=stable)


def test_hyperspectral_full_size_fp32():
    # the full 262144 x 200 hyperspectral workload (512 x 512 pixels x 200
    # bands, 15 endmembers) at tol 1e-2 and b = 16, against the oracle
    say("hyperspectral 262144 x 200")
    A = W.hyperspectral(0).astype(np.float64)
    stable, _, _ = O.precision_stable(A, 1e-2, 16, 0)
    f, ref = check_factor(A, torch.float32, 1e-2, b=16, seed=0, stable=stable)
    assert 10 <= f.rank <= 20


def test_mat2_fp64():
    A = W.mat2(1, 600, 240)
    check_factor(A, torch.float64, 1e-12, b=32, seed=1)


# ------------------------------------------------- low-precision sketch form
@pytest.mark.parametrize("mode", ["f16", "bf16"])
def test_sketch_lp_kernel(mode):
    say("sketch lp kernel", mode)
    rng = np.random.default_rng(7)
    A = (rng.standard_normal((1000, 700)) * 40.0).astype(np.float32).astype(np.float64)
    code = E.SKETCH_F16 if mode == "f16" else E.SKETCH_BF16
    c = E.Context(seed=21, sketch=code)
    Y = E.sketch(c, dev(A, torch.float32), 5, 40).cpu().numpy().astype(np.float64)
    s = O.lp_scale(A, mode)
    Alp = O.lp_round((A * s).astype(np.float32), mode)
    Om = O.lp_round(O.omega_columns(21, 700, 5, 40).astype(np.float32), mode)
    ref = (Alp @ Om) / s
    bound = 2 * 700 * U32 * (np.abs(Alp) @ np.abs(Om)) / s
    assert np.all(np.abs(Y - ref) <= bound + 1e-30)


# Error bar of the low-precision form (FP16 and BF16 alike): its RelErr
# within 1e-3 of the oracle's emulation of the same form, absolute, and
# never more than 1e-3 above the plain FP64 oracle's (the equal-error rule).
# The emulation sketches blocks 3, 4, ... with the rounded copies of A and
# Omega and then runs one subspace iteration on A, as the form is defined.
LP_ERR = 1e-3


def _check_lp_factor(A, tol, b, seed, mode, q=0):
    say("lp factor", A.shape, mode, "tol", tol, "b", b, "seed", seed, "q", q)
    code = E.SKETCH_F16 if mode == "f16" else E.SKETCH_BF16
    f = E.factor(dev(A, torch.float32), tol, block=b, seed=seed, sketch=code, power_iters=q)
    torch.cuda.synchronize()
    ref = O.eod_abe(A, tol, k=b, q=q, seed=seed)
    emu = O.eod_abe(A, tol, k=b, q=q, seed=seed, sketch_dtype=mode)
    stable, r64, rlp = O.precision_stable(A, tol, b, seed, mode)
    assert f.blocks >= 3                       # the low-precision blocks did run
    assert f.flags & 16                        # ... and the FP32 refinement with them
    if stable:
        assert f.rank == r64 == emu.rank, (f.rank, r64, rlp)
    else:
        assert f.rank in (r64, rlp), (f.rank, r64, rlp)
    e_gpu, U, D, Vt = gpu_relerr(A, f)
    e_ref = O.rel_err(A, ref.U, ref.D, ref.V)
    e_emu = O.rel_err(A, emu.U, emu.D, emu.V)
    say(f"  rank {f.rank} relerr gpu {e_gpu:.3e} form-oracle {e_emu:.3e} plain-oracle {e_ref:.3e}")
    if f.rank == emu.rank:
        assert abs(e_gpu - e_emu) <= LP_ERR, (e_gpu, e_emu)
    assert e_gpu <= e_ref + LP_ERR, (e_gpu, e_ref)
    r = f.rank
    assert np.linalg.norm(U.T @ U - np.eye(r)) <= ORTH_TOL[torch.float32] * math.sqrt(r)
    assert np.linalg.norm(Vt @ Vt.T - np.eye(r)) <= ORTH_TOL[torch.float32] * math.sqrt(r)
    assert np.all(np.tril(D, -1) == 0) and np.all(np.diag(D) >= 0)
    return f, ref, e_gpu, e_emu


def test_factor_f16_sketch_image():
    A = W.image(0, 1024, 0.05).astype(np.float64)
    _check_lp_factor(A, 1e-3, 8, 0, "f16")


@pytest.mark.parametrize("mode", ["f16", "bf16"])
def test_factor_lp_sketch_hyperspectral(mode):
    A = W.hyperspectral(0, pixels=16384).astype(np.float64)
    _check_lp_factor(A, 1e-2, 4, 0, mode)


@pytest.mark.parametrize("mode", ["f16", "bf16"])
def test_factor_lp_sketch_exact_rank(mode):
    # exact rank 40 with sigma_40 = sigma_1 / 10.  FP16 rounding (2^-11)
    # keeps the rank exact; BF16 (2^-8) tilts the sketched subspace by about
    # ||A - A_bf16|| / sigma_40, which can keep a few rounding columns (the
    # oracle's emulation gives 40..48).  Either way the refined error is the
    # FP32 path's own, compared with the form's oracle.
    A = W.lowrank_haar(4, m=400, n=300, r=40, noise_std=0.0, decades=1.0).astype(np.float32).astype(np.float64)
    f, ref, e_gpu, e_emu = _check_lp_factor(A, 1e-2, 8, 4, mode)
    if mode == "f16":
        assert f.rank == 40
    else:
        assert 40 <= f.rank <= 48
    assert abs(e_gpu - e_emu) <= 1e-5


@pytest.mark.parametrize("mode", ["f16", "bf16"])
@pytest.mark.parametrize("shape", [(16384, 200), (300, 2100)])
def test_factor_lp_sketch_power_iteration(mode, shape):
    # q = 1 with the low-precision form: two subspace iterations, each with
    # its A^T Q product from the rounded copy (ragged K splits, partial
    # column panels, the transposed orientation), against the form's oracle
    m, n = shape
    A = W.lowrank_haar(41, m=m, n=n, r=70, noise_std=1e-5, decades=2.0).astype(np.float32).astype(np.float64)
    _check_lp_factor(A, 1e-2, 8, 41, mode, q=1)


@pytest.mark.parametrize("mode", ["f16", "bf16"])
def test_factor_lp_sketch_row_tiles(mode):
    # 4112 rows: the FP32 blocks (and the write of the low-precision copy in
    # block 2) run by 16-row tiles, later blocks read the copy
    A = W.lowrank_haar(31, m=4112, n=520, r=120, noise_std=1e-6, decades=3.0).astype(np.float32).astype(np.float64)
    f, ref, e_gpu, e_emu = _check_lp_factor(A, 1e-2, 16, 31, mode)
    assert f.blocks >= 3


# Exact-rank instances (FP32-rounded, so their error is FP32 rounding) on
# which a basis from the rounded sketches alone misses the oracle's RelErr
# by 3.7e-3 .. 1.7e-2 at the same rank (found by a seeded sweep of the
# oracle's emulation): the refinement brings the error back to the plain
# path's.  (mode, sweep index, m, n, content rank, decades, tol, b)
LP_SWEEP_CASES = [
    ("f16", 201, 380, 538, 39, 1.449, 0.00309, 4),
    ("f16", 229, 465, 267, 56, 1.998, 0.0011, 8),
    ("f16", 145, 470, 474, 157, 0.712, 0.00746, 16),
    ("f16", 155, 218, 478, 114, 0.842, 0.0099, 8),
    ("bf16", 252, 359, 63, 20, 0.666, 0.011, 8),
    ("bf16", 380, 558, 413, 73, 0.734, 0.0156, 8),
    ("bf16", 358, 295, 499, 183, 0.622, 0.0453, 4),
    ("bf16", 152, 598, 34, 17, 1.552, 0.0239, 4),
]


@pytest.mark.parametrize("case", LP_SWEEP_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_factor_lp_sketch_sweep_cases(case):
    mode, i, m, n, r, dec, tol, b = case
    A = W.lowrank_haar(5000 + i, m=m, n=n, r=r, noise_std=0.0, decades=dec).astype(np.float32).astype(np.float64)
    f, ref, e_gpu, e_emu = _check_lp_factor(A, tol, b, i, mode)
    e_ref = O.rel_err(A, ref.U, ref.D, ref.V)
    assert abs(e_gpu - e_ref) <= max(1e-5, fp32_floor(f.rank, m, n))


@pytest.mark.parametrize("mode,tol", [("bf16", 1e-3), ("f16", 5e-4)])
def test_lp_sketch_below_its_floor_runs_plain(mode, tol):
    say("lp sketch below its noise floor", mode, tol)
    # below tol = 2 u_lp the low-precision sketch would mask the stop test
    # (its rounding noise sits above tol ||A||_F): every block sketches in
    # FP32, flag bit 3, and the result is the plain path's bit for bit
    A = dev(W.lowrank_haar(9, m=700, n=500, r=90, noise_std=1e-9).astype(np.float64), torch.float32)
    code = E.SKETCH_F16 if mode == "f16" else E.SKETCH_BF16
    f = E.factor(A, tol, block=16, seed=5, sketch=code)
    p = E.factor(A, tol, block=16, seed=5)
    torch.cuda.synchronize()
    assert f.flags & 8 and not (p.flags & 8)
    assert f.blocks >= 3 and f.rank == p.rank
    for x, y in ((f.U, p.U), (f.D, p.D), (f.Vt, p.Vt)):
        assert torch.equal(x, y)


def test_lp_sketch_at_its_floor_keeps_low_precision():
    say("lp sketch at its floor")
    A = dev(W.lowrank_haar(9, m=700, n=500, r=90, noise_std=1e-9).astype(np.float64), torch.float32)
    f = E.factor(A, 2.0 ** -10, block=16, seed=5, sketch=E.SKETCH_F16)
    torch.cuda.synchronize()
    assert not (f.flags & 8)


# ------------------------------------------------- batched tiles
def _batch_tiles():
    """Tiles of the batched parity test and, per tile, whether its content is
    noise-free (exact rank, or a full-rank Gaussian that the loop never
    stops on), where the FP32 error is rounding alone."""
    tiles = W.tiles(5, count=22, lo=64, hi=1024, rank_lo=5, rank_hi=80, noise_std=1e-4)
    clean = [False] * len(tiles)
    rng = np.random.default_rng(11)
    wide = (W.lowrank_haar(6, m=90, n=700, r=17, noise_std=0.0) * 100).astype(np.float32)
    tiles += [wide, np.zeros((64, 80), dtype=np.float32)]
    tiles += [(rng.standard_normal((70, 66)) * 10).astype(np.float32)]     # full rank 66 > 64
    # ranks 65..128 close through the blocked 128-wide Cholesky: a wide tile
    # with an unaligned row length and a tall one
    tiles += [(W.lowrank_haar(7, m=150, n=403, r=100, noise_std=0.0) * 50).astype(np.float32)]
    tiles += [(W.lowrank_haar(8, m=517, n=260, r=121, noise_std=0.0) * 50).astype(np.float32)]
    tiles += [(rng.standard_normal((300, 190)) * 3).astype(np.float32)]    # rank 190 > 128: regular path
    clean += [True] * (len(tiles) - len(clean))
    return tiles, clean


def test_batched_tiles_against_oracle():
    say("batched tiles")
    tiles, clean = _batch_tiles()
    c = E.Context(seed=3, block=32)
    dtiles = [dev(T.astype(np.float64), torch.float32) for T in tiles]
    bt = E.Batch(c, dtiles)
    bt.run(1e-4)
    torch.cuda.synchronize()
    assert set(bt.status.tolist()) <= {0}, bt.status
    exempt = 0
    for t, T in enumerate(tiles):
        A = T.astype(np.float64)
        U, D, Vt, r, st = bt.result(t)
        b = int(bt.blocks[t])
        ref = O.eod_abe(A, 1e-4, k=b, q=0, seed=3)
        if not np.any(A):
            assert r == 0
            continue
        stable, r64, r32 = O.precision_stable(A, 1e-4, b, 3)
        if stable:
            assert r == ref.rank, (t, T.shape, r, ref.rank)
        else:
            exempt += 1
            assert r in (r64, r32), (t, T.shape, r, r64, r32)
        Un, Dn, Vn = (x.double().cpu().numpy() for x in (U, D, Vt))
        e_gpu = np.linalg.norm(A - Un @ Dn @ Vn) / np.linalg.norm(A)
        # the oracle run with the rank the GPU returned: FP64 when it agrees
        # with it, else the oracle's FP32-data emulation (the other side of a
        # precision-unstable rank decision)
        cmp = ref if r == ref.rank else O.eod_abe(A, 1e-4, k=b, q=0, seed=3, sketch_dtype=np.float32)
        assert cmp.rank == r, (t, T.shape, r, cmp.rank)
        e_ref = O.rel_err(A, cmp.U, cmp.D, cmp.V)
        bar = RELERR_TOL[torch.float32]
        if clean[t]:
            bar = max(bar, fp32_floor(r, *A.shape), 4.0 * (U32 / U64) * e_ref)
        say(f"  tile {t} {T.shape} b {b} rank {r} relerr gpu {e_gpu:.3e} oracle {e_ref:.3e} bar {bar:.1e}")
        assert abs(e_gpu - e_ref) <= bar, (t, T.shape, e_gpu, e_ref, bar)
        # equal error with the single-matrix FP32 path on the same tile
        f = E.factor(dtiles[t], 1e-4, ctx=E.Context(seed=3, block=b))
        e_one = float(torch.linalg.norm(dtiles[t].double() - f.U.double() @ f.D.double() @ f.Vt.double())
                      / torch.linalg.norm(dtiles[t].double()))
        assert f.rank == r, (t, T.shape, f.rank, r)
        # the equal-error rule: the two FP32 paths within the bar each meets
        # against the oracle (on rounding-only tiles both errors are rounding)
        assert abs(e_gpu - e_one) <= max(0.05 * e_one, bar), (t, T.shape, e_gpu, e_one, bar)
        assert np.linalg.norm(Un.T @ Un - np.eye(r)) <= ORTH_TOL[torch.float32] * math.sqrt(r)
        assert np.linalg.norm(Vn @ Vn.T - np.eye(r)) <= ORTH_TOL[torch.float32] * math.sqrt(r)
        assert np.all(np.tril(Dn, -1) == 0) and np.all(np.diag(Dn) >= 0)
    say(f"  precision-unstable tiles (rank checked against both sides): {exempt} of {len(tiles)}")


def test_batched_full_benchmark_set_against_single_matrix():
    # the benchmark's 1024 tiles (sides 64..1024, exact rank 5..80 + 1e-4
    # noise, tol 1e-4, b = 32) in one batched call against the single-matrix
    # path tile by tile: equal ranks on every tile the oracle's classifier
    # calls precision-stable, RelErr within the FP32 bar of each other
    say("batched: full 1024-tile benchmark set")
    tiles = W.tiles(0, count=1024)
    devs = [torch.from_numpy(np.ascontiguousarray(T)).cuda() for T in tiles]
    c = E.Context(block=32, seed=0)
    bt = E.Batch(c, devs)
    bt.run(1e-4)
    torch.cuda.synchronize()
    assert np.all(bt.status == 0)
    diff = []
    for t, A in enumerate(devs):
        fs = E.factor(A, 1e-4, ctx=c)
        if int(fs.rank) != int(bt.ranks[t]):
            diff.append(t)
            continue
        if t % 16 == 0:                  # errors on a sample (the products cost host time)
            A64 = A.double()
            U, D, Vt = bt.result(t)[:3]
            eb = float(torch.linalg.norm(A64 - U.double() @ D.double() @ Vt.double()) / torch.linalg.norm(A64))
            es = float(torch.linalg.norm(A64 - fs.U.double() @ fs.D.double() @ fs.Vt.double()) / torch.linalg.norm(A64))
            assert abs(eb - es) <= max(1e-5, fp32_floor(fs.rank, *A.shape)), (t, eb, es)
    say(f"  ranks differ on {len(diff)} of 1024 tiles: {diff}")
    assert len(diff) <= 8
    for t in diff:
        stable, r64, r32 = O.precision_stable(tiles[t].astype(np.float64), 1e-4, 32, 0)
        assert not stable, (t, r64, r32)


def test_batched_replay_deterministic_and_tuner():
    say("batched replay + tuner")
    tiles = W.tiles(8, count=12, lo=64, hi=512, rank_lo=5, rank_hi=40, noise_std=1e-4)
    c = E.Context(seed=4, block=32)
    bt = E.Batch(c, [dev(T.astype(np.float64), torch.float32) for T in tiles])
    bt.run(1e-4)
    first = [tuple(x.clone() for x in bt.result(t)[:3]) for t in range(len(tiles))]
    r1 = bt.ranks.copy()
    bt.run(1e-4)                       # graph replay: the defined outputs are bit-identical
    assert np.array_equal(bt.ranks, r1)
    for t in range(len(tiles)):
        for x, y in zip(bt.result(t)[:3], first[t]):
            assert torch.equal(x, y), t
    chosen = bt.tune(1e-4)
    assert set(int(x) for x in chosen) <= {0, 16, 32, 64}
    bt.run(1e-4)
    assert set(bt.blocks.tolist()) <= {16, 32, 64}
