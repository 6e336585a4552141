"""Batched sorting (qms_sort_batch): many independent arrays advance together
through the phases of the QuickMergesort loop.  Every segment must come out
exactly as the oracle sorts it on its own."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import (as_u64, segment_ids, segment_multiset_hash,  # noqa: E402
                               segments_sorted, to_device, to_host)

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _lengths(count, seed, lo_exp, hi_exp, extra=()):
    L = inputs.log_uniform_lengths(count, seed=seed, lo_exp=lo_exp, hi_exp=hi_exp)
    return np.concatenate([L, np.array(extra, dtype=np.int64)])


def _run_batch(x: np.ndarray, lens, vals=False):
    off = inputs.offsets_from_lengths(lens)
    kt = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    vt = None
    if vals:
        vt = torch.arange(x.size, dtype=torch.int32, device="cuda")
    qms.qms_sort_batch(kt, ot, vals=vt, host_offsets=off)
    torch.cuda.synchronize()
    return off, kt, vt


@needs_gpu
@pytest.mark.parametrize("dtype", ["u32", "f32"])
def test_batch_matches_oracle_per_segment(dtype):
    lens = _lengths(300, seed=11, lo_exp=0, hi_exp=15, extra=(0, 1, 0, 2, 4096, 4097, 70000))
    rng = np.random.default_rng(3)
    lens = lens[rng.permutation(lens.size)]
    n = int(lens.sum())
    x = inputs.uniform_u32(n, seed=12) if dtype == "u32" else inputs.normal_f32(n, seed=12)
    off, kt, _ = _run_batch(x, lens)
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(kt).view(np.uint32), want.view(np.uint32))


@needs_gpu
def test_batch_duplicates_and_structured():
    parts = [inputs.zipf_u32(50000, seed=1), inputs.sorted_u32(30000), inputs.reverse_u32(9000),
             np.full(20000, 7, dtype=np.uint32), inputs.sorted_with_swaps_u32(100000, seed=2),
             inputs.uniform_u32(5, seed=3), np.zeros(0, dtype=np.uint32)]
    lens = np.array([p.size for p in parts], dtype=np.int64)
    x = np.concatenate(parts)
    off, kt, _ = _run_batch(x, lens)
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(kt), want)


@needs_gpu
def test_batch_pairs():
    lens = _lengths(150, seed=21, lo_exp=0, hi_exp=14, extra=(0, 1, 30000))
    n = int(lens.sum())
    x = inputs.zipf_u32(n, seed=22)
    off, kt, vt = _run_batch(x, lens, vals=True)
    ko = to_host(kt)
    vo = to_host(vt)
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(ko, want)
    # payload = original index: stays inside its segment, and carries its key
    for j in range(lens.size):
        a, b = int(off[j]), int(off[j + 1])
        v = vo[a:b].astype(np.int64)
        assert np.array_equal(np.sort(v), np.arange(a, b))
        assert np.array_equal(x[v], ko[a:b])


@needs_gpu
@pytest.mark.parametrize("tuning", ["autotuned", "loop"])
def test_batch_config3_20000_arrays_f32(tuning):
    """20,000 arrays, lengths log-uniform in [2^6, 2^20] (seed 5), float32
    N(0,1) keys generated on the device (about 2.2e9 keys, 8.6 GB): every
    segment sorted with its own multiset, and 256 segments (the longest and
    the shortest among them) element by element against the oracle.  Once at
    the tuning the autotuner picks on every 20th array of the batch, once
    with the loop running down to the base tile."""
    from paper_1804_10062_amd import autotune
    lens = inputs.log_uniform_lengths(20000, seed=5, lo_exp=6, hi_exp=20)
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    kt = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    kt[kt == 0] = 0.0  # no negative zero
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    try:
        if tuning == "autotuned":
            sample = np.arange(0, lens.size, 20)
            s_lens = lens[sample]
            s_off = inputs.offsets_from_lengths(s_lens)
            s_keys = torch.cat([kt[int(off[j]):int(off[j + 1])] for j in sample])
            s_ot = torch.from_numpy(s_off.view(np.int64)).cuda()
            autotune.autotune_batch(s_keys, s_ot, host_offsets=s_off, reps=1)
            del s_keys
        seg = segment_ids(ot, n)
        h_in = segment_multiset_hash(kt, seg)
        rng = np.random.default_rng(0)
        picks = set(rng.choice(lens.size, 254, replace=False).tolist())
        picks |= {int(np.argmax(lens)), int(np.argmin(lens))}
        picks = sorted(picks)
        before = {j: kt[int(off[j]):int(off[j + 1])].cpu().numpy() for j in picks}
        qms.qms_sort_batch(kt, ot, host_offsets=off)
        torch.cuda.synchronize()
    finally:
        if tuning == "autotuned":
            autotune.reset_tuning()
    assert segments_sorted(kt, ot)
    assert segment_multiset_hash(kt, seg) == h_in
    assert len(picks) >= 200
    for j in picks:
        got = kt[int(off[j]):int(off[j + 1])].cpu().numpy()
        want, _, _ = oracle.sort(before[j], counted=False)
        np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


def _big_segments_exact():
    lens = np.array([(1 << 25) + 4097, 4097, 70_000_001, 1, 300_000, 0, 9], dtype=np.int64)
    n = int(lens.sum())
    x = inputs.uniform_u32(n, seed=21)
    off = inputs.offsets_from_lengths(lens)
    kt = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(kt, ot, host_offsets=off)
    torch.cuda.synchronize()
    got = to_host(kt)
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(got, want)


@needs_gpu
def test_batch_segments_with_several_scan_chunks():
    """Segments above 8,192 partition tiles (2^25 keys at the default tile)
    are scanned by several workgroups, one row of the scan grid per segment;
    small segments beside them by one.  Every segment against the oracle."""
    _big_segments_exact()


@needs_gpu
@pytest.mark.final_path
def test_batch_segments_with_several_scan_chunks_defaults():
    """The same at the library's default tuning."""
    from paper_1804_10062_amd import autotune
    autotune.reset_tuning()
    _big_segments_exact()
