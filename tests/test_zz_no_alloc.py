"""qms_sort_noalloc (the entry point that allocates nothing) against
qms_sort, through the C ABI: bit-exact on two calls in a row (the second on
fewer keys), 32- and 64-bit keys, no change in the device's free memory
across calls, sizes above the limit rejected."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _noalloc(t: torch.Tensor, dt: int) -> int:
    lib = qms.load_library()
    return lib.qms_sort_noalloc(ctypes.c_void_p(t.data_ptr()), t.numel(), dt,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@needs_gpu
def test_noalloc_matches_qms_sort_twice():
    big = inputs.uniform_u32((1 << 22) + 12345, seed=70)
    small = inputs.make_keys("sorted_swaps", 300007, seed=71)
    wide = np.random.default_rng(72).integers(0, 2 ** 64, 500001, dtype=np.uint64)
    # references through the existing entry point (this allocates its workspace)
    refs = []
    for x in (big, small):
        r = to_device(x)
        qms.qms_sort(r)
        refs.append(r)
    rw = torch.from_numpy(wide.view(np.int64)).cuda()
    qms.qms_sort(rw)
    torch.cuda.synchronize()
    # a first call sets the library's scratch up on this device
    warm = to_device(inputs.uniform_u32(50000, seed=73))
    assert _noalloc(warm, qms.QMS_U32) == qms.QMS_OK, qms.last_error()
    a, b = to_device(big), to_device(small)
    c = torch.from_numpy(wide.view(np.int64)).cuda()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    assert _noalloc(a, qms.QMS_U32) == qms.QMS_OK, qms.last_error()
    torch.cuda.synchronize()
    assert _noalloc(b, qms.QMS_U32) == qms.QMS_OK, qms.last_error()
    torch.cuda.synchronize()
    assert _noalloc(c, qms.QMS_U64) == qms.QMS_OK, qms.last_error()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    np.testing.assert_array_equal(to_host(a), to_host(refs[0]))
    np.testing.assert_array_equal(to_host(b), to_host(refs[1]))
    np.testing.assert_array_equal(c.cpu().numpy(), rw.cpu().numpy())


@needs_gpu
def test_noalloc_f32_and_limits():
    x = inputs.normal_f32(1 << 20, seed=74)
    ref = to_device(x)
    qms.qms_sort(ref)
    t = to_device(x)
    qms.qms_sort_noalloc(t)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(t).view(np.uint32), to_host(ref).view(np.uint32))
    lib = qms.load_library()
    small = torch.zeros(16, dtype=torch.int32, device="cuda")
    rc = lib.qms_sort_noalloc(ctypes.c_void_p(small.data_ptr()), (1 << 28) + 1, qms.QMS_U32, None)
    assert rc == qms.QMS_ERR_UNSUPPORTED
    assert "2^28" in qms.last_error()
    rc = lib.qms_sort_noalloc(None, 5, qms.QMS_U32, None)
    assert rc == qms.QMS_ERR_INVALID
    host = np.zeros(16, dtype=np.uint32)
    rc = lib.qms_sort_noalloc(ctypes.c_void_p(host.ctypes.data), 16, qms.QMS_U32, None)
    assert rc == qms.QMS_ERR_INVALID
