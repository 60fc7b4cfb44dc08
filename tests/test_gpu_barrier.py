"""The barrier across the workgroups of the one-launch CholeskyQR2 is bounded:
if its arrivals do not all come within the wait, every workgroup sets the
control block's sync flag and runs on, every kernel ends, and the call
returns EODABE_ESYNC with its outputs void; the context stays usable.  The
time-out is forced from the host (a test-only knob read when a context is
created makes each barrier wait for one arrival more than the launch makes,
for 10 microseconds), so no kernel is left waiting."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2506_22713_amd as E  # noqa: E402


def _matrix(m=2048, n=1024, r=12, seed=5):
    g = np.random.default_rng(seed)
    A = (g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 1e-4 * g.standard_normal((m, n)))
    return torch.from_numpy(A.astype(np.float32)).cuda()


def test_barrier_timeout_reports_esync_and_context_recovers(monkeypatch):
    A = _matrix()
    monkeypatch.setenv("EODABE_TEST_BARRIER_FAIL", "1")
    bad = E.Context(block=32, seed=0)
    monkeypatch.delenv("EODABE_TEST_BARRIER_FAIL")
    with pytest.raises(E.EodAbeError) as ei:
        E.factor(A, 1e-3, ctx=bad)
    assert ei.value.status == E.EODABE_ESYNC
    torch.cuda.synchronize()
    # a later call on a normal context gives the right answer; so does the
    # same forced context's next call fail the same way (nothing stuck)
    good = E.Context(block=32, seed=0)
    f = E.factor(A, 1e-3, ctx=good)
    assert f.rank == 12
    A64 = A.double()
    err = float(torch.linalg.norm(A64 - f.U.double() @ f.D.double() @ f.Vt.double()) / torch.linalg.norm(A64))
    assert err < 1e-3
    with pytest.raises(E.EodAbeError) as ei2:
        E.factor(A, 1e-3, ctx=bad)
    assert ei2.value.status == E.EODABE_ESYNC
