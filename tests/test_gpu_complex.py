"""GPU parity of complex input (the paper's setting A in C^{m x n}) through
the C ABI, against the complex128 oracle.

Bars: rank equal to the oracle's on precision-stable instances (complex128
runs: always); RelErr within 1e-10 (complex128) or 1e-5 (complex64, noisy
content; noise-free exact-rank content takes the FP32 rounding-floor bar of
the real tests); ||U^H U - I||, ||V^H V - I|| within 1e-12 sqrt(r) /
5e-5 sqrt(r); D upper triangular with a real non-negative diagonal; on
exact-rank content the unique factors equal the oracle's elementwise."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle.complex_oracle as C  # noqa: E402
import paper_2506_22713_amd as E  # noqa: E402
import workloads as W  # noqa: E402

U32, U64 = 2.0 ** -24, 2.0 ** -53


def say(*a):
    print("[case]", *a, flush=True)


def check(A, dtype, tol, k, seed, q=0, stable=True, rounding_only=False):
    say(f"complex {A.shape} {dtype} tol {tol} k {k} q {q} seed {seed}")
    ref = C.eod_abe_c(A, tol, k=k, q=q, seed=seed)
    real = torch.float32 if dtype == torch.complex64 else torch.float64
    f = E.factor_complex(torch.from_numpy(A).to(device="cuda", dtype=dtype), tol,
                         ctx=E.Context(dtype=real, block=k, power_iters=q, seed=seed))
    torch.cuda.synchronize()
    if stable:
        assert f.rank == ref.rank, (f.rank, ref.rank)
    if f.rank == 0:
        return f, ref
    U, D, Vh = (x.to(torch.complex128).cpu().numpy() for x in (f.U, f.D, f.Vt))
    e_gpu = float(np.linalg.norm(A - U @ D @ Vh) / np.linalg.norm(A))
    e_ref = C.rel_err_c(A, ref.U, ref.D, ref.V)
    r = f.rank
    if dtype == torch.complex128:
        bar, obar = 1e-10, 1e-12
    else:
        bar, obar = 1e-5, 5e-5
        if rounding_only:
            bar = max(bar, 4 * U32 * math.sqrt(r * max(A.shape)), 4 * (U32 / U64) * e_ref)
    say(f"  rank {r} (oracle {ref.rank}) relerr gpu {e_gpu:.3e} oracle {e_ref:.3e} bar {bar:.1e}")
    if r == ref.rank:
        assert abs(e_gpu - e_ref) <= bar, (e_gpu, e_ref, bar)
    assert np.linalg.norm(U.conj().T @ U - np.eye(r)) <= obar * math.sqrt(r)
    assert np.linalg.norm(Vh @ Vh.conj().T - np.eye(r)) <= obar * math.sqrt(r)
    assert np.all(np.tril(D, -1) == 0)
    dg = np.diag(D)
    assert np.all(dg.real >= 0) and np.all(np.abs(dg.imag) <= (1e-12 if dtype == torch.complex128 else 1e-5)
                                            * np.abs(dg).max())
    return f, ref


@pytest.mark.parametrize("m,n", [(300, 200), (120, 330)])
def test_complex128_exact_rank_factors(m, n):
    A = W.lowrank_complex(1, m=m, n=n, r=17, decades=2.0)
    f, ref = check(A, torch.complex128, 1e-10, 8, 3)
    assert f.rank == 17
    for got, want in ((f.U, ref.U), (f.D, ref.D), (f.Vt, ref.V.conj().T)):
        g = got.cpu().numpy()
        assert np.max(np.abs(g - want)) <= 1e-8 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("m,n,k", [(400, 260, 16), (230, 500, 8), (333, 70, 32)])
def test_complex128_noisy(m, n, k):
    A = W.lowrank_complex(2 + m, m=m, n=n, r=40, noise_std=1e-11, decades=3.0)
    check(A, torch.complex128, 1e-7, k, 5)


def test_complex128_power_iteration():
    A = W.lowrank_complex(6, m=300, n=200, r=15, noise_std=1e-12)
    f, ref = check(A, torch.complex128, 1e-8, 16, 6, q=1)
    U, D, Vh = (x.cpu().numpy() for x in (f.U, f.D, f.Vt))
    e = np.linalg.norm(A - U @ D @ Vh) / np.linalg.norm(A)
    assert abs(e - C.eckart_young_c(A, f.rank)) <= 1e-10


def test_complex128_rank_above_64():
    # realified rank 2 r > 128: the wide closing path on the realification
    A = W.lowrank_complex(7, m=300, n=220, r=80, decades=2.0)
    f, ref = check(A, torch.complex128, 1e-10, 16, 7)
    assert f.rank == 80


@pytest.mark.parametrize("m,n,noise", [(500, 300, 1e-7), (260, 640, 1e-7)])
def test_complex64_noisy(m, n, noise):
    A = W.lowrank_complex(8 + n, m=m, n=n, r=30, noise_std=noise, decades=2.0)
    A = A.astype(np.complex64).astype(np.complex128)
    stable, _, _ = C.precision_stable_c(A, 1e-4, 16, 9)
    check(A, torch.complex64, 1e-4, 16, 9, stable=stable)


def test_complex64_exact_rank():
    A = W.lowrank_complex(10, m=256, n=192, r=24, decades=1.5).astype(np.complex64).astype(np.complex128)
    stable, _, _ = C.precision_stable_c(A, 1e-4, 8, 2)
    f, ref = check(A, torch.complex64, 1e-4, 8, 2, stable=stable, rounding_only=True)
    assert f.rank == 24


def test_complex_full_rank_and_zero():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((90, 40)) + 1j * rng.standard_normal((90, 40))
    f, ref = check(A, torch.complex128, 1e-13, 16, 1)
    assert f.rank == 40 and f.blocks == 3
    z = E.factor_complex(torch.zeros((50, 30), dtype=torch.complex128, device="cuda"), 1e-3)
    assert z.rank == 0
