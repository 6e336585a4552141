"""Run-time tunables (qms_set_tuning) and the autotuner: they change speed,
never results.  Every tuning must give the oracle's sorted keys bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import autotune, inputs, qms  # noqa: E402
from tests.gpu_helpers import to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

# (merge_ways, partition_tile, chunk_span, base_tile)
TUNINGS = [(4, 4096, 16384, 0), (4, 4096, 16384, 16384), (2, 4096, 16384, 16384),
           (4, 8192, 32768, 8192),
           (2, 16384, 4096, 4096), (4, 65536, 1 << 20, 2048), (4, 4096, 16384, 4096),
           (2, 8192, 16384, 2048)]
FIELDS = ("merge_ways", "partition_tile", "chunk_span", "base_tile", "final_tile")


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    if torch.cuda.is_available():
        autotune.reset_tuning()


@needs_gpu
@pytest.mark.parametrize("tuning", TUNINGS)
@pytest.mark.parametrize("kind,n", [("uniform", 1 << 20), ("sorted_swaps", 300007),
                                    ("zipf", 200003), ("reverse", 1 << 18)])
def test_tuned_sort_matches_oracle(tuning, kind, n):
    qms.qms_set_tuning(*tuning)
    got = qms.qms_get_tuning()
    assert {f: got[f] for f in FIELDS[:len(tuning)]} == dict(zip(FIELDS, tuning))
    x = inputs.make_keys(kind, n, seed=11)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
@pytest.mark.parametrize("tuning", TUNINGS[:5])
def test_tuned_pairs_and_f32(tuning):
    qms.qms_set_tuning(*tuning)
    x = inputs.normal_f32(123457, seed=3)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t).view(np.uint32), want.view(np.uint32))
    k = inputs.make_keys("zipf", 99991, seed=2)
    kt = to_device(k)
    vt = torch.arange(k.size, dtype=torch.int32, device="cuda")
    qms.qms_sort_pairs(kt, vt)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(k, counted=False)
    np.testing.assert_array_equal(to_host(kt), want)
    assert np.array_equal(k[to_host(vt).view(np.int32).astype(np.int64)], want)


@needs_gpu
def test_invalid_tuning_rejected_and_unchanged():
    before = qms.qms_get_tuning()
    for bad in [(3, 4096, 16384), (4, 4095, 16384), (4, 6144, 16384), (4, 4096, 100),
                (4, 1 << 17, 16384), (4, 4096, (1 << 20) + 1),
                (4, 4096, 16384, 1024), (4, 4096, 16384, 3072), (4, 4096, 16384, 32768),
                (4, 4096, 16384, 0, 4096), (4, 4096, 16384, 0, 3 << 20),
                (4, 4096, 16384, 0, 1 << 31)]:  # final_tile: a power of two in [8192, 2^30]
        with pytest.raises(qms.QmsError):
            qms.qms_set_tuning(*bad)
    assert qms.qms_get_tuning() == before


@needs_gpu
def test_autotune_batch_picks_a_candidate_and_keeps_results():
    lens = inputs.log_uniform_lengths(300, seed=9, lo_exp=6, hi_exp=17)
    off = inputs.offsets_from_lengths(lens)
    x = inputs.uniform_u32(int(off[-1]), seed=9)
    keys = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    rep = autotune.autotune_batch(keys, ot, host_offsets=off, reps=1)
    assert len(rep["trials"]) == len(autotune.CANDIDATES)
    assert qms.qms_get_tuning() == rep["best"]
    # the sample itself was not modified
    np.testing.assert_array_equal(to_host(keys), x)
    qms.qms_sort_batch(keys, ot, host_offsets=off)
    torch.cuda.synchronize()
    got = to_host(keys)
    for j in range(0, lens.size, 37):
        a, b = int(off[j]), int(off[j + 1])
        want, _, _ = oracle.sort(x[a:b], counted=False)
        np.testing.assert_array_equal(got[a:b], want)
