"""eodabe_factor_noalloc (workspace in the library's static device scratch)
against eodabe_factor (caller workspace) through the C ABI: two calls in a
row, the second smaller, so the second reads a scratch the first left
behind; the outputs must be the same bits.  Also the size limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2506_22713_amd as E  # noqa: E402
import workloads as W  # noqa: E402


def _dev(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(A)).to(device="cuda", dtype=dtype)


# (m, n, content rank, noise, tol, block, r_cap): the first call largest,
# then smaller ones; a wide matrix (transposed inside) and a rank > 64 case
CASES = [
    (torch.float32, [(1500, 1100, 90, 1e-9, 1e-4, 32, 256), (600, 400, 20, 1e-9, 1e-4, 32, 0)]),
    (torch.float64, [(800, 700, 40, 1e-11, 1e-8, 16, 128), (300, 520, 12, 1e-11, 1e-8, 16, 0)]),
]


@pytest.mark.parametrize("dtype,calls", CASES, ids=["f32", "f64"])
def test_noalloc_matches_factor(dtype, calls):
    for i, (m, n, r, noise, tol, b, rc) in enumerate(calls):
        print(f"[case] noalloc call {i}: {m}x{n} {dtype} tol {tol} b {b} r_cap {rc}", flush=True)
        c = E.Context(dtype=dtype, seed=17, block=b)
        A = _dev(W.lowrank_haar(300 + i, m=m, n=n, r=r, noise_std=noise), dtype)
        ref = E.factor(A, tol, ctx=c, r_cap=rc)
        out = E.alloc_outputs(A, rc)
        got = E.factor_noalloc(A, tol, c, out, r_cap=rc)
        torch.cuda.synchronize()
        assert got.status == ref.status and got.rank == ref.rank and got.blocks == ref.blocks
        assert got.flags == ref.flags and got.eps == ref.eps
        for x, y in ((got.U, ref.U), (got.D, ref.D), (got.Vt, ref.Vt)):
            assert torch.equal(x, y)


def test_noalloc_rejects_problem_beyond_scratch():
    print("[case] noalloc size limit", flush=True)
    c = E.Context(dtype=torch.float32, seed=1)
    A = torch.zeros((4096, 4096), device="cuda")
    need = E._lib.eodabe_workspace_size(c.h, 4096, 4096, 0)
    assert need > E.NOALLOC_SCRATCH_BYTES
    info = E.Info()
    out = [torch.empty(1, device="cuda") for _ in range(3)]
    st = E._lib.eodabe_factor_noalloc(c.h, A.data_ptr(), 4096, 4096, 4096, 1e-3, out[0].data_ptr(),
                                      out[1].data_ptr(), out[2].data_ptr(), 0, ctypes.byref(info))
    assert st == E.EODABE_ESCRATCH
    assert b"static scratch" in E._lib.eodabe_strerror(st)
