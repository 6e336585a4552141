"""Autotuner for the run-time tunables of libqms (qms_set_tuning).

The batched solves pick their partition and merge parameters by measurement:
each candidate tuning sorts fresh copies of a sample of the workload (a
device-resident batch the caller provides), timed with events on the sorting
stream, and the fastest is kept and set.  Tunings change speed, never
results.  torch provides the copies and the events; all sorting runs in
libqms.

    from paper_1804_10062_amd import autotune
    report = autotune.autotune_batch(sample_keys, sample_offsets)
"""
from __future__ import annotations

import itertools
from typing import Iterable, Optional, Sequence, Tuple

from . import qms

FIELDS = ("merge_ways", "partition_tile", "chunk_span", "base_tile", "final_tile")
# (merge_ways, partition_tile, chunk_span, base_tile, final_tile); base_tile
# is QuickMergeXsort's X_THRESH, the run width at which the Mergesort calls
# the base case (0: automatic).  final_tile (the range size at or below
# which a single array's range leaves the loop for the in-place network;
# 0: automatic) does not apply to batches, whose rounds are planned on the
# device and run down to the base tile, so it stays at its default here.
CANDIDATES: Tuple[Tuple[int, int, int, int, int], ...] = tuple(
    c + (0,) for c in itertools.product((4, 2), (4096, 8192), (16384, 32768), (0, 8192)))


def _time_batch(keys, offsets, vals, ref_keys, ref_vals, stream, host_offsets) -> float:
    """One sort of a fresh copy of the batch; GPU time in ms."""
    import torch
    keys.copy_(ref_keys)
    if vals is not None:
        vals.copy_(ref_vals)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    qms.qms_sort_batch(keys, offsets, vals=vals, host_offsets=host_offsets, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def autotune_batch(keys, offsets, vals=None, host_offsets=None,
                   candidates: Iterable[Sequence[int]] = CANDIDATES,
                   reps: int = 3, stream=None) -> dict:
    """Time every candidate tuning on the batch (keys, offsets[, vals];
    host_offsets: an optional numpy copy of offsets) and set the fastest.
    Each candidate's figure is its best of `reps` sorts; the candidates are
    timed in turn within each repetition, so that a drift of the clocks
    during the search weighs on all of them alike.  The inputs are left as
    they were (each trial sorts a copy).
    Returns {"best": {...}, "trials": [{..., "ms": t}, ...]}."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    cands = [tuple(c) for c in candidates]
    work_k = torch.empty_like(keys)
    work_v = None if vals is None else torch.empty_like(vals)
    before = qms.qms_get_tuning()
    best_ms = [float("inf")] * len(cands)
    settings = [None] * len(cands)
    try:
        with torch.cuda.stream(stream):
            for _ in range(reps):
                for i, cand in enumerate(cands):
                    qms.qms_set_tuning(*cand)
                    settings[i] = qms.qms_get_tuning()
                    ms = _time_batch(work_k, offsets, work_v, keys, vals, stream, host_offsets)
                    best_ms[i] = min(best_ms[i], ms)
    except Exception:
        qms.qms_set_tuning(*(before[f] for f in FIELDS))
        raise
    trials = [dict(zip(FIELDS, settings[i].values()), ms=round(best_ms[i], 4))
              for i in range(len(cands))]
    best = min(trials, key=lambda t: t["ms"])
    qms.qms_set_tuning(*(best[f] for f in FIELDS))
    return {"best": {f: best[f] for f in FIELDS}, "trials": trials}


DEFAULTS = (4, 4096, 16384, 0, 0)


def reset_tuning() -> None:
    """Back to the library defaults."""
    qms.qms_set_tuning(*DEFAULTS)
