"""One in-place sort of more than 2^32 uint32 keys.

The input is a Weyl sequence over the 32-bit words, key[j] = (A j + B) mod
2^32 for j < 2^32 (A odd: every word exactly once), followed by d copies of
the word 7.  Its sorted order has a closed form: 0, 1, ..., 6, then d + 1
sevens, then 8, ..., 2^32 - 1, i.e. out[i] = i for i <= 7, 7 for
7 <= i <= 7 + d, and i - d after that.  tests/test_oracle_pins.py checks
that closed form against the oracle on the same construction over 12-bit
words; here every output word is compared with it, slice by slice on the
device.  The first round's range holds 2^32 + d keys, so it is partitioned
as blocks and gathered by rotations (QMS_U32 keys, no scratch beyond the
library's workspace)."""
import time

import pytest

torch = pytest.importorskip("torch")

from paper_1804_10062_amd import qms  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

A, B = 0x9E3779B1, 0x7F4A7C15
D = 1 << 20
N = (1 << 32) + D
CHUNK = 1 << 28


def _expected(i: torch.Tensor) -> torch.Tensor:
    return torch.where(i <= 7, i, torch.where(i <= 7 + D, torch.full_like(i, 7), i - D))


@needs_gpu
def test_sort_beyond_2_32_keys():
    free, _ = torch.cuda.mem_get_info()
    if free < 4 * N + (8 << 30):
        pytest.skip("needs about 26 GB of free device memory")
    keys = torch.empty(N, dtype=torch.int32, device="cuda")
    for j0 in range(0, 1 << 32, CHUNK):
        j = torch.arange(j0, j0 + CHUNK, dtype=torch.int64, device="cuda")
        w = (j * A + B) & 0xFFFFFFFF
        keys[j0:j0 + CHUNK] = (w - ((w >> 31) << 32)).to(torch.int32)  # two's complement view
    keys[1 << 32:] = 7
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qms.qms_sort(keys)
    torch.cuda.synchronize()
    print(f"2^32 + 2^20 uint32 keys sorted in {time.perf_counter() - t0:.3f} s", flush=True)
    sched = qms.qms_last_schedule()
    assert sched and sched[0][0] == N  # the first round took the whole array
    bad = 0
    for i0 in range(0, N, CHUNK):
        i1 = min(N, i0 + CHUNK)
        got = keys[i0:i1].to(torch.int64) & 0xFFFFFFFF
        want = _expected(torch.arange(i0, i1, dtype=torch.int64, device="cuda"))
        bad += int((got != want).sum())
    assert bad == 0, f"{bad} words differ from the sorted order"
