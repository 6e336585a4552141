"""The request loop (qms_server_*): requests of mixed sizes and dtypes are
admitted against the HBM budget, batched, sorted and completed; each must
equal the oracle's sort of that request."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _requests(count, seed, lo_exp=0, hi_exp=16):
    lens = inputs.log_uniform_lengths(count, seed=seed, lo_exp=lo_exp, hi_exp=hi_exp)
    kinds = inputs.uniform_u32(count, seed=seed, stream=9) & 1
    out = []
    for j, (n, k) in enumerate(zip(lens, kinds)):
        n = int(n)
        x = inputs.uniform_u32(n, seed=seed * 1000 + j) if k == 0 else \
            inputs.uniform_f32(n, seed=seed * 1000 + j)
        out.append(x)
    return out


def _wait_all(srv, tickets, timeout=120.0):
    lat = {}
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            st, l = srv.poll(t)
            if st == qms.QMS_OK:
                lat[t] = l
                pending.discard(t)
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(pending)} requests still pending")
        time.sleep(0.0005)
    return lat


@needs_gpu
def test_server_sorts_mixed_requests():
    reqs = _requests(120, seed=3) + [np.zeros(0, np.uint32), np.array([5], np.uint32)]
    devs = [to_device(x) for x in reqs]
    torch.cuda.synchronize()
    with qms.Server(hbm_budget_bytes=1 << 30, device=0) as srv:
        tickets = [srv.submit(d) for d in devs]
        lat = _wait_all(srv, tickets)
        assert all(v >= 0 for v in lat.values())
        st = srv.stats()
        assert st["completed"] == len(reqs)
        assert st["completed_keys"] == sum(x.size for x in reqs)
        assert st["batches"] >= 1
    for x, d in zip(reqs, devs):
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(to_host(d).view(np.uint32), want.view(np.uint32))


@needs_gpu
def test_server_budget_admission_fifo():
    """A budget of 1 MB with requests of 100,000 keys (400 kB): at most two are
    admitted at a time, the others wait; none is dropped."""
    reqs = [inputs.uniform_u32(100000, seed=s) for s in range(12)]
    devs = [to_device(x) for x in reqs]
    torch.cuda.synchronize()
    budget = 1 << 20
    with qms.Server(hbm_budget_bytes=budget, device=0, max_batch=8) as srv:
        tickets = [srv.submit(d) for d in devs]
        _wait_all(srv, tickets)
        st = srv.stats()
        assert st["completed"] == len(reqs)
        assert st["peak_admitted_bytes"] <= budget
        assert st["waited_for_budget"] > 0
    for x, d in zip(reqs, devs):
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(to_host(d), want)


@needs_gpu
def test_server_errors():
    d = to_device(inputs.uniform_u32(1000, seed=1))
    with qms.Server(hbm_budget_bytes=1000, device=0) as srv:
        with pytest.raises(qms.QmsError) as e:
            srv.submit(d)  # 4000 bytes > budget
        assert e.value.code == qms.QMS_ERR_BUDGET
        with pytest.raises(qms.QmsError) as e:
            srv.poll(12345)
        assert e.value.code == qms.QMS_ERR_INVALID
        small = d[:200].clone()
        t = srv.submit(small)
        _wait_all(srv, [t])
        with pytest.raises(qms.QmsError) as e:
            srv.poll(t)  # retired
        assert e.value.code == qms.QMS_ERR_INVALID
    lib = qms.load_library()
    host = np.zeros(16, dtype=np.uint32)
    with qms.Server(hbm_budget_bytes=1 << 20, device=0) as srv:
        import ctypes
        tk = ctypes.c_uint64()
        rc = lib.qms_server_submit(srv._h, host.ctypes.data, 16, qms.QMS_U32, None,
                                   ctypes.byref(tk))
        assert rc == qms.QMS_ERR_INVALID
        rc = lib.qms_server_submit(srv._h, host.ctypes.data, 16, 7, None, ctypes.byref(tk))
        assert rc == qms.QMS_ERR_UNSUPPORTED


@needs_gpu
def test_server_destroy_drains():
    reqs = _requests(40, seed=8, lo_exp=10, hi_exp=18)
    devs = [to_device(x) for x in reqs]
    torch.cuda.synchronize()
    srv = qms.Server(hbm_budget_bytes=1 << 30, device=0)
    for dv in devs:
        srv.submit(dv)
    srv.close()  # must wait for every request
    for x, dv in zip(reqs, devs):
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(to_host(dv).view(np.uint32), want.view(np.uint32))


@needs_gpu
def test_server_waits_for_the_producing_stream():
    """Keys written by work still queued on the caller's stream at submit:
    the server's batch waits for the event recorded there, so it sorts the
    written keys, not the zeros the tensor held before."""
    x = inputs.uniform_u32(1 << 20, seed=21)
    src = to_device(x)
    dst = torch.zeros_like(src)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with qms.Server(hbm_budget_bytes=1 << 30, device=0) as srv:
        with torch.cuda.stream(side):
            # a few milliseconds of queued work ahead of the copy
            a = torch.rand(4096, 4096, device="cuda")
            for _ in range(8):
                a = a @ a
                a = a / a.abs().amax().clamp_min(1.0)
            dst.copy_(src)
        t = srv.submit(dst, stream=side)
        _wait_all(srv, [t])
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(dst), want)


@needs_gpu
def test_server_64_bit_keys():
    """uint64 and float64 requests beside 32-bit ones, bit-exact with the
    oracle's 64-bit build; the budget counts 8 bytes per key."""
    rng = np.random.default_rng(5)
    reqs = [rng.integers(0, 2 ** 64, int(n), dtype=np.uint64) for n in (3, 1000, 70001, 1 << 18)]
    reqs += [rng.standard_normal(int(n)) for n in (2, 5000, 100003)]
    reqs += [inputs.uniform_u32(50000, seed=3)]
    devs = []
    for x in reqs:
        if x.dtype == np.uint64:
            devs.append(torch.from_numpy(x.view(np.int64)).cuda())
        elif x.dtype == np.float64:
            devs.append(torch.from_numpy(x).cuda())
        else:
            devs.append(to_device(x))
    torch.cuda.synchronize()
    with qms.Server(hbm_budget_bytes=1 << 30, device=0) as srv:
        tickets = [srv.submit(d) for d in devs]
        _wait_all(srv, tickets)
        assert srv.stats()["completed_keys"] == sum(x.size for x in reqs)
    with qms.Server(hbm_budget_bytes=8 * 999, device=0) as srv:
        with pytest.raises(qms.QmsError) as e:
            srv.submit(devs[1])  # 1000 keys of 8 bytes > 7992 bytes
        assert e.value.code == qms.QMS_ERR_BUDGET
    for x, d in zip(reqs, devs):
        want, _, _ = oracle.sort(x, counted=False)
        got = d.cpu().numpy()
        if x.dtype == np.uint64:
            got = got.view(np.uint64)
        elif x.dtype == np.uint32:
            got = got.view(np.uint32)
        np.testing.assert_array_equal(got, want)
