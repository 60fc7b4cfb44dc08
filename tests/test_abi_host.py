"""Host-side checks of the C ABI (no GPU needed): the shared library loads,
exports every function include/eodabe.h declares, validates options and
sizes, and plans workspace, using a host-only context."""
import ctypes
import os
import re
import subprocess

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "eodabe.h")
LIB = os.path.join(ROOT, "paper_2506_22713_amd", "libeodabe.so")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eodabe_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def E():
    if not os.path.exists(LIB):
        pytest.fail("libeodabe.so not built (run python -m paper_2506_22713_amd.build)")
    import paper_2506_22713_amd as E
    return E


def test_every_declared_symbol_is_exported(E):
    names = _declared()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert getattr(lib, n) is not None
    assert set(E.EXPORTED) <= set(names)


def test_strerror_and_defaults(E):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 1):
        assert E.strerror(code) and E.strerror(code) != "unknown status"
    assert "barrier" in E.strerror(E.EODABE_ESYNC)
    o = E.Opts()
    E._lib.eodabe_default_opts(ctypes.byref(o))
    assert o.block == 32 and o.power_iters == 0 and o.a_dtype == E.F32


@pytest.mark.parametrize("bad", [dict(block=0), dict(block=129), dict(power_iters=-1),
                                 dict(power_iters=17), dict(blocks_per_sync=-1)])
def test_option_validation(E, bad):
    with pytest.raises(E.EodAbeError) as ei:
        E.Context(host_only=True, **bad)
    assert ei.value.status == E.EODABE_EINVAL


def test_workspace_planning(E):
    import torch
    c = E.Context(host_only=True)
    s1 = c.workspace_size(512, 512)
    s2 = c.workspace_size(4096, 4096)
    s3 = c.workspace_size(4096, 4096, 400)
    assert 0 < s1 < s2 and 0 < s3 < s2
    assert c.workspace_size(200, 500) > 0          # wide: transposed plan
    assert c.workspace_size(10, 10, 11) == 0       # r_cap > min(m, n)
    assert c.workspace_size(-1, 10) == 0
    c64 = E.Context(host_only=True, dtype=torch.float64)
    assert c64.workspace_size(512, 512) > s1


def test_info_layout(E):
    # eodabe_info: int64 rank, int blocks, int status_flags, then norm_a,
    # eps and relres_est (doubles) at 16, 24 and 32
    assert ctypes.sizeof(E.Info) == 40
    assert E.Info.relres_est.offset == 32 and E.Info.eps.offset == 24 and E.Info.norm_a.offset == 16


def test_factor_argument_errors_without_device(E):
    c = E.Context(host_only=True)
    info = E.Info()
    f = E._lib.eodabe_factor
    ws = ctypes.create_string_buffer(16)
    # NULL context, bad sizes, bad lda, bad tol: rejected before any device use
    assert f(None, None, 4, 4, 4, 1e-3, None, 0, None, None, None, 0, ctypes.byref(info)) == E.EODABE_EINVAL
    assert f(c.h, None, -1, 4, 4, 1e-3, None, 0, None, None, None, 0, ctypes.byref(info)) == E.EODABE_EINVAL
    assert f(c.h, ws, 4, 4, 3, 1e-3, None, 0, ws, ws, ws, 0, ctypes.byref(info)) == E.EODABE_EINVAL
    for tol in (0.0, -1.0, float("nan"), float("inf")):
        assert f(c.h, ws, 4, 4, 4, tol, None, 0, ws, ws, ws, 0, ctypes.byref(info)) == E.EODABE_EINVAL
    # workspace too small
    assert f(c.h, ws, 4, 4, 4, 1e-3, ws, 16, ws, ws, ws, 0, ctypes.byref(info)) == E.EODABE_EWORKSPACE
    # empty problem: nothing to do
    need = c.workspace_size(0, 5)
    big = ctypes.create_string_buffer(need)
    assert f(c.h, None, 0, 5, 5, 1e-3, big, need, None, None, None, 0, ctypes.byref(info)) == E.EODABE_OK
    # a well-formed call on a host-only context reports the missing device
    need = c.workspace_size(4, 4)
    big = ctypes.create_string_buffer(need)
    assert f(c.h, ws, 4, 4, 4, 1e-3, big, need, ws, ws, ws, 0, ctypes.byref(info)) == E.EODABE_ENODEVICE


def test_fast_entry_matches_ctypes_call(E):
    """The CPython entry of eodabe_factor (argument conversion in C) is built,
    bound to the library ctypes loaded, and returns what the ctypes call
    returns on the same arguments (status, then the info fields)."""
    assert E._fastcall is not None
    fc = E._fastcall.factor
    c = E.Context(host_only=True)
    ws = ctypes.create_string_buffer(16)
    a = ctypes.addressof(ws)
    need = c.workspace_size(4, 4)
    big = ctypes.create_string_buffer(need)
    b = ctypes.addressof(big)
    cases = [
        (0, 0, 4, 4, 4, 1e-3, 0, 0, 0, 0, 0, 0),                  # NULL context
        (c.h.value, 0, -1, 4, 4, 1e-3, 0, 0, 0, 0, 0, 0),        # bad size
        (c.h.value, a, 4, 4, 3, 1e-3, 0, 0, a, a, a, 0),          # lda < n
        (c.h.value, a, 4, 4, 4, float("nan"), 0, 0, a, a, a, 0),  # bad tol
        (c.h.value, a, 4, 4, 4, 1e-3, a, 16, a, a, a, 0),         # workspace too small
        (c.h.value, a, 4, 4, 4, 1e-3, b, need, a, a, a, 0),       # no device
    ]
    for args in cases:
        info = E.Info()
        ref = E._lib.eodabe_factor(*(x if not isinstance(x, int) or i in (2, 3, 4, 7, 11) else (x or None)
                                     for i, x in enumerate(args)), ctypes.byref(info))
        got = fc(*args)
        assert got == (ref, info.rank, info.blocks, info.status_flags, info.norm_a, info.eps, info.relres_est), args
    assert got[0] == E.EODABE_ENODEVICE
    with pytest.raises(TypeError):
        fc(0, 0, 4)


def test_factorization_views_alias_the_outputs(E):
    """factor()'s result makes U = Ut[:r]^T, D = core[:r, :r] and Vt[:r] on
    first access: views of the caller's buffers, nothing copied."""
    m, n, rc, r = 7, 5, 5, 3
    Ut = torch.arange(rc * m, dtype=torch.float32).reshape(rc, m)
    core = torch.arange(rc * rc, dtype=torch.float32).reshape(rc, rc)
    Vt = torch.arange(rc * n, dtype=torch.float32).reshape(rc, n)
    f = E.Factorization((Ut, core, Vt), r, 1, 0.5, 2.0, 0, 0, 0.1)
    assert f.rank == r and f.blocks == 1 and f.eps == 0.5 and f.norm_a == 2.0 and f.relres_est == 0.1
    assert f.U.shape == (m, r) and f.D.shape == (r, r) and f.Vt.shape == (r, n)
    assert torch.equal(f.U, Ut[:r].T) and torch.equal(f.D, core[:r, :r]) and torch.equal(f.Vt, Vt[:r])
    assert f.U.data_ptr() == Ut.data_ptr() and f.D.data_ptr() == core.data_ptr() and f.Vt.data_ptr() == Vt.data_ptr()
    assert f.U is f.U                              # made once
    core[0, 0] = -1.0                              # a view: later writes show through
    assert f.D[0, 0].item() == -1.0
    assert "rank=3" in repr(f)


def test_batched_argument_errors_without_device(E):
    """Host checks of eodabe_factor_batched: sizes, tol, dtype, output pool
    extent and workspace, all before any device use."""
    import numpy as np
    import torch
    c = E.Context(host_only=True)
    f = E._lib.eodabe_factor_batched
    buf = ctypes.create_string_buffer(64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)

    def call(m, n, lda, rc, off, pool_len, tol=1e-3, ctx=None, ws_bytes=64):
        nt = len(m)
        ptrs = (ctypes.c_void_p * nt)(*([ctypes.addressof(buf)] * nt))
        a = [np.asarray(x, dtype=np.int64) for x in (m, n, lda, off, rc)]
        ranks, status = np.zeros(nt, np.int64), np.zeros(nt, np.int32)
        return f((ctx or c).h, nt, ctypes.cast(ptrs, ctypes.c_void_p), p(a[0]), p(a[1]), p(a[2]), tol, buf,
                 ws_bytes, buf, pool_len, p(a[3]), p(a[4]), p(ranks), p(status), None)

    ok = dict(m=[8], n=[6], lda=[6], rc=[0], off=[0], pool_len=6 * (8 + 6 + 6))
    assert call(**ok) == E.EODABE_EWORKSPACE                     # everything valid but the workspace
    assert call(**{**ok, "m": [0]}) == E.EODABE_EINVAL
    assert call(**{**ok, "n": [1025]}) == E.EODABE_EINVAL        # tiles are at most 1024 x 1024
    assert call(**{**ok, "lda": [5]}) == E.EODABE_EINVAL
    assert call(**{**ok, "rc": [7]}) == E.EODABE_EINVAL          # r_cap > min(m, n)
    assert call(**{**ok, "off": [-1]}) == E.EODABE_EINVAL
    assert call(**{**ok, "pool_len": 6 * 20 - 1}) == E.EODABE_EINVAL   # outputs overrun the pool
    assert call(**{**ok, "off": [1]}) == E.EODABE_EINVAL
    assert call(**{**ok, "rc": [2], "off": [6 * 20 - 2 * 16]}) == E.EODABE_EWORKSPACE   # fits exactly
    for tol in (0.0, float("nan")):
        assert call(**ok, tol=tol) == E.EODABE_EINVAL
    c64 = E.Context(host_only=True, dtype=torch.float64)
    assert call(**ok, ctx=c64) == E.EODABE_EINVAL                # FP32 tiles only
    wsz = E._lib.eodabe_batched_workspace_size
    assert wsz(c.h, 1000) > wsz(c.h, 1) > 0 and wsz(None, 1) == 0 and wsz(c.h, -1) == 0


def test_predictor_features_match_oracle(E):
    """eodabe_mlp_features (host) against the oracle's feature map."""
    import numpy as np
    from oracle import predictor_oracle as PO
    from paper_2506_22713_amd import predictor as PR
    rng = np.random.default_rng(3)
    cases = [10.0 ** (-0.1 * np.arange(64)), np.exp(-rng.random(64).cumsum()), 10.0 ** (-1.0 * np.arange(64)),
             np.concatenate([np.ones(10), np.zeros(54)])]
    for d, (m, n, eps) in zip(cases, [(4096, 4096, 1e-3), (777, 300, 1e-8), (65, 65, 0.5), (1000, 999, 1e40)]):
        got = PR.features(d, m, n, eps)
        ref = PO.features(d, m, n, eps).astype(np.float32)
        assert np.array_equal(got, ref), (got - ref)


def test_predictor_checkpoint_roundtrip(tmp_path):
    """Checkpoint format: JSON header + params, m, v; resume keeps the step."""
    import numpy as np
    import torch
    from paper_2506_22713_amd import predictor as PR
    pr = PR.Predictor(seed=5, device="cpu")
    pr.m.uniform_(-1, 1)
    pr.v.uniform_(0, 1)
    pr.step = 17
    path = str(tmp_path / "p.ckpt")
    pr.save(path, meta={"note": "roundtrip"})
    q = PR.Predictor.load(path, device="cpu")
    assert q.step == 17 and q.meta["note"] == "roundtrip"
    for a, b in ((pr.params, q.params), (pr.m, q.m), (pr.v, q.v)):
        assert torch.equal(a, b)
    with open(path, "rb") as fh:
        head = fh.readline()
    assert b'"format": "eodabe-mlp-1"' in head
    assert PR.init_params(5).size == PR.NPARAM == 149506


def test_status_codes_match_header(E):
    """Every status code the header defines has the same value in the
    binding and a message of its own."""
    import re
    hdr = open(os.path.join(ROOT, "include", "eodabe.h")).read()
    codes = dict((n, int(v)) for n, v in re.findall(r"#define (EODABE_(?:OK|E[A-Z]+|W[A-Z_]+))\s+(-?\d+)", hdr))
    assert {"EODABE_OK", "EODABE_ESYNC", "EODABE_ESCRATCH", "EODABE_WTOL_FLOOR"} <= set(codes)
    msgs = set()
    for name, v in codes.items():
        assert getattr(E, name) == v, name
        m = E.strerror(v)
        assert m != "unknown status", name
        msgs.add(m)
    assert len(msgs) == len(codes)
