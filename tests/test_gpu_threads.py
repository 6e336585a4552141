"""Several host threads calling the library at once: sorts on the same
stream share that stream's workspace one after another, sorts on different
streams run side by side; every result equals the oracle's."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _run_threads(jobs):
    errors = []

    def work(fn):
        try:
            fn()
        except Exception as e:  # reported by the main thread
            errors.append(e)

    ts = [threading.Thread(target=work, args=(j,)) for j in jobs]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=300)
    assert not any(t.is_alive() for t in ts), "a sorting thread did not finish"
    if errors:
        raise errors[0]


@needs_gpu
@pytest.mark.parametrize("same_stream", [True, False])
def test_threads_sort_concurrently(same_stream):
    xs = [inputs.uniform_u32(n, seed=40 + i) for i, n in enumerate((1 << 20, 300007, 1 << 19, 77777))]
    devs = [to_device(x) for x in xs]
    torch.cuda.synchronize()
    shared = torch.cuda.Stream()
    streams = [shared if same_stream else torch.cuda.Stream() for _ in xs]

    def job(i):
        def fn():
            for _ in range(3):  # the same keys again: sorted input stays sorted
                qms.qms_sort(devs[i], stream=streams[i])
            streams[i].synchronize()
        return fn

    _run_threads([job(i) for i in range(len(xs))])
    torch.cuda.synchronize()
    for x, d in zip(xs, devs):
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(to_host(d), want)


@needs_gpu
def test_release_keeps_a_workspace_in_use():
    """qms_release_workspaces while a server holds its workspace: the busy
    workspace is kept (QMS_ERR_INVALID says so) and the server still sorts."""
    x = inputs.uniform_u32(200003, seed=9)
    d = to_device(x)
    torch.cuda.synchronize()
    with qms.Server(hbm_budget_bytes=1 << 30, device=0) as srv:
        t0 = srv.submit(d)
        while srv.poll(t0)[0] != qms.QMS_OK:
            pass
        lib = qms.load_library()
        rc = lib.qms_release_workspaces()
        assert rc in (qms.QMS_OK, qms.QMS_ERR_INVALID)
        y = inputs.uniform_u32(100000, seed=10)
        e = to_device(y)
        torch.cuda.synchronize()
        t1 = srv.submit(e)
        while srv.poll(t1)[0] != qms.QMS_OK:
            pass
    want, _, _ = oracle.sort(y, counted=False)
    np.testing.assert_array_equal(to_host(e), want)
