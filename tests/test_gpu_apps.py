"""GPU parity of the application layers through the C ABI: colour-image
compression (introduction storage example; section 4.1 criteria) and the
hyperspectral features + KNN cross-validation of section 4.2, against the
CPU oracle.

Bars: ranks equal to the oracle's on precision-stable channels; RelErr
within the FP32 bar (1e-5, absolute); PSNR within the PSNR change that bar
allows, 20 log10(1 + 1e-5 / RelErr_oracle) dB; SSIM within 1e-6; storage
counts exact (integer formula of the ranks).  Features within FP32
rounding of the oracle's; KNN predictions, confusion matrix and OA bit-exact
against the oracle run on the same features (integer decisions taken on the
same FP64 distances)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle.apps_oracle as P  # noqa: E402
import oracle.eodabe_oracle as O  # noqa: E402
import paper_2506_22713_amd as E  # noqa: E402
import workloads as W  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def _check_image(img, tol, seed=0, block=32):
    c, h, w = img.shape
    say(f"image {c}x{h}x{w} tol {tol} seed {seed}")
    ctx = E.Context(dtype=torch.float32, seed=seed, block=block)
    out = E.compress_image(torch.from_numpy(img).cuda(), tol, ctx)
    torch.cuda.synchronize()
    inf = out.info
    img64 = img.astype(np.float64)
    k = block
    ref = P.compress_image(img64, tol, k, seed=seed)
    ranks = [int(inf.rank[ch]) for ch in range(c)]
    say(f"  ranks gpu {ranks} oracle {ref['ranks']}  relerr {inf.relerr:.4e} / {ref['relerr']:.4e}"
        f"  psnr {inf.psnr:.4f} / {ref['psnr']:.4f}  ssim {inf.ssim:.8f} / {ref['ssim']:.8f}")
    for ch in range(c):
        stable, r64, r32 = O.precision_stable(img64[ch], tol, k, seed)
        if stable:
            assert ranks[ch] == ref["ranks"][ch], (ch, ranks, ref["ranks"])
    if ranks == ref["ranks"]:
        assert abs(inf.relerr - ref["relerr"]) <= 1e-5
        bar = 20 * math.log10(1 + 1e-5 / max(ref["relerr"], 1e-300)) + 1e-9
        assert abs(inf.psnr - ref["psnr"]) <= bar, (inf.psnr, ref["psnr"], bar)
        assert abs(inf.ssim - ref["ssim"]) <= 1e-6
    # the reported criteria are those of the returned reconstruction, and the
    # reconstruction is the product of the returned factors
    rec = out.recon.double().cpu().numpy()
    d2 = float(np.sum((rec - img64) ** 2))
    assert abs(inf.relerr - math.sqrt(d2) / np.linalg.norm(img64)) <= 1e-12 + 1e-9 * inf.relerr
    assert abs(inf.ssim - P.ssim_global(img64, rec)) <= 1e-12
    for ch, (U, D, Vt) in enumerate(out.factors):
        prod = (U.double() @ D.double() @ Vt.double()).cpu().numpy()
        assert np.max(np.abs(prod - rec[ch])) <= 1e-4 * max(1.0, np.abs(img64[ch]).max())
    stored = sum(O.storage_bytes(h, w, r) for r in ranks)
    assert inf.stored == stored and inf.full == c * h * w
    assert abs(inf.rank_bound - O.storage_rank_bound(h, w)) <= 1e-9
    return inf, ref


def test_image_storage_example():
    # the introduction's 220 x 220 example: channels of exact ranks 50, 52,
    # 53 are compressed from 145200 to 72284 entries, 50.22 %
    img = W.exact_rank_rgb(0, 220, 220, (50, 52, 53))
    inf, ref = _check_image(img, 1e-4)
    assert [int(inf.rank[c]) for c in range(3)] == [50, 52, 53]
    assert inf.stored == 72284 and inf.full == 145200
    assert round(100 * inf.reduction, 2) == 50.22


@pytest.mark.parametrize("h,w,noise,tol", [(512, 512, 0.05, 1e-3), (768, 512, 0.2, 1e-3), (333, 517, 0.5, 5e-3)])
def test_image_rgb_against_oracle(h, w, noise, tol):
    _check_image(W.rgb_image(1, h, w, noise_std=noise), tol, seed=2)


def test_image_above_tile_size():
    _check_image(W.rgb_image(3, 1100, 1300, noise_std=0.05), 1e-3, seed=5)


def test_image_grayscale_one_channel():
    _check_image(W.rgb_image(4, 300, 200, noise_std=0.1)[:1].copy(), 1e-3, seed=1)


@pytest.mark.parametrize("tol,k", [(1e-1, 5), (3e-2, 5), (1e-2, 1), (1e-2, 7)])
def test_hsi_features_and_knn(tol, k):
    # synthetic scene of Indian Pines' shape class (pixels x 200 bands, 15
    # classes = dominant endmember), ten folds; the paper sweeps eps over
    # 0.1 .. 0.01 to get 3 .. 13 features
    A, lab, fold = W.hyperspectral_labelled(0, pixels=6000)
    say(f"hsi 6000 x 200 tol {tol} k {k}")
    A64 = A.astype(np.float64)
    f = E.factor(torch.from_numpy(A).cuda(), tol, block=16, seed=0)
    F = E.features(f)
    torch.cuda.synchronize()
    ref = O.eod_abe(A64, tol, k=16, seed=0)
    assert f.rank == ref.rank
    Fr = P.hsi_features(ref.U, ref.D)
    Fg = F.double().cpu().numpy()
    assert np.max(np.abs(Fg - Fr)) <= 1e-4 * np.abs(Fr).max(), np.max(np.abs(Fg - Fr))
    pred, conf, oa = E.knn_cv(F.contiguous(), torch.from_numpy(lab).cuda(), torch.from_numpy(fold).cuda(), k, 15)
    torch.cuda.synchronize()
    p_ref, c_ref, oa_ref = P.knn_cv(F.cpu().numpy(), lab, fold, k, 15)
    say(f"  features {f.rank}  OA gpu {oa:.4f} oracle {oa_ref:.4f}")
    assert np.array_equal(pred.cpu().numpy(), p_ref)
    assert np.array_equal(conf, c_ref) and oa == oa_ref


def test_knn_hand_example_on_gpu():
    F = torch.tensor([[0.0], [1.0], [2.0], [10.0], [11.0], [12.0]], device="cuda")
    lab = torch.tensor([0, 0, 1, 1, 1, 0], dtype=torch.int32, device="cuda")
    fold = torch.tensor([0, 1, 0, 1, 0, 1], dtype=torch.int32, device="cuda")
    pred, conf, oa = E.knn_cv(F, lab, fold, 1, 2)
    assert pred.cpu().tolist() == [0, 0, 0, 1, 1, 1]
    assert conf.tolist() == [[2, 1], [1, 2]] and abs(oa - 4 / 6) <= 1e-15
