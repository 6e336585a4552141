"""Benchmark: QuickMergesort of one array of 2^28 uint32 keys on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one complete in-place sort (partition rounds, base case, swap-merge
levels) of a fresh, device-resident copy of the 2^28-key workload: K + W
copies are uploaded before the timed region, so the timed region holds
exactly K sorts and nothing else.  The headline is uniform keys (seed 2);
nearly-sorted (1% random transpositions, seed 3) and reverse-sorted inputs
are timed the same way and reported beside it.

One JSON line goes to stdout with, besides the contract fields:
  roofline      for the dominant kernel (the swap-merge pass: k_merge4 for
                the 4-way passes, k_merge for a first 2-way pass):
                algorithmic bytes per launch (16 B per element of the merged
                side) over its mean launch duration, timed with HIP events on
                the sorting stream in a second pass of K sorts right after the
                timed region (events around ~500 launches per sort add a few
                percent, so the headline region runs without them); `traffic` is the
                HBM traffic per launch measured by rocprofv3 counters
                (profiles/pmc_qms_sort_u32_2e28.json) while the kernel source
                is unchanged since that measurement, else null;
  kernel_rooflines  the other hot kernels against their own bounds: the base
                case against the VALU issue peak (VALU instructions per sort
                from the same counter file over its event-timed time), the
                partition exchange against HBM with its measured traffic;
  whole_sort    every algorithmic byte of the executed schedule (base case,
                merge passes, counting, exchange) over the time per sort,
                against the same peak;
  cpu_baseline  the CPU oracle (single thread, pinned to one core) on the
                whole 2^28-key workload, in Gkeys/s;
  kernels       per-kernel-class launches, time and achieved GB/s;
  distributions Gkeys/s of the three inputs, and of 2^26 key/payload pairs
                (Zipf(1.1) keys over [0, 2^10), payload = index);
  batched       20,000 float32 arrays in one qms_sort_batch call against one
                qms_sort call per array (a 1-in-10 sample of the arrays);
  serving       open-loop Poisson request streams at 2k/10k/50k requests/s
                through the library's server: throughput, p50/p99 latency.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_KEYS = 1 << 28
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_qms_sort_u32_2e28.json")
VALU_PEAK = 256 * 2.4e9  # wave64 VALU instructions per second (one per CU per cycle)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dist-steps", type=int, default=3,
                    help="timed sorts for the nearly-sorted and reverse inputs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=28)
    ap.add_argument("--only-uniform", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-threshold-sweep", action="store_true")
    ap.add_argument("--per-array-stride", type=int, default=10)
    ap.add_argument("--serving-requests", type=int, default=20000)
    ap.add_argument("--serving-warmup", type=int, default=1000)
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for rocprofv3 counter passes: one 1 GiB device copy "
                         "(calibration kernel of known size) and one sort of the workload")
    return ap.parse_args()


def _oracle_child(keys, core, conn):
    """Child process: pin to `core`, time the oracle's sort of `keys`."""
    import numpy as np
    try:
        os.sched_setaffinity(0, {core})
    except OSError:
        pass
    import oracle
    t0 = time.perf_counter()
    oracle.sort_inplace_fast(keys, False)
    dt = time.perf_counter() - t0
    conn.send((dt, bool(np.all(keys[1:] >= keys[:-1]))))
    conn.close()


def _oracle_on_one_core(keys):
    """The C oracle on a copy of `keys` in a forked child pinned to one core
    (the child touches no GPU state); returns (seconds, core)."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    cores = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else [0]
    core = cores[-1]
    a, b = ctx.Pipe(duplex=False)
    p = ctx.Process(target=_oracle_child, args=(keys.copy(), core, b))
    p.start()
    dt, ok = a.recv()
    p.join()
    assert ok, "oracle output not sorted"
    return dt, core


def measured_kernel(name: str):
    """The rocprofv3 counter record of one kernel from the committed summary
    (per sort of the headline workload), if the kernel's source files (its
    own and the headers it includes) are unchanged since it was taken; else
    None."""
    try:
        d = json.load(open(PMC_FILE))
        k = d["kernels"][name]
        h = hashlib.sha256()
        for f in k.get("sources", [k["source"]]):
            h.update(open(os.path.join(ROOT, f), "rb").read())
        h = h.hexdigest()[:16]
    except (OSError, ValueError, KeyError):
        return None
    return k if h == k.get("source_sha256_16") else None


def time_sorts(copies, qms, torch, profile: bool, dtype=None):
    """Sort every tensor in `copies` (one step each); returns (seconds, profile)."""
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    if profile:
        qms.qms_profile_begin()
    t0 = time.perf_counter()
    for t in copies:
        qms.qms_sort(t, stream=stream, dtype=dtype)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = qms.qms_profile_end() if profile else None
    return t1 - t0, prof


def bench_batched(qms, torch, np, inputs, per_array_stride: int, reps: int = 3):
    """20,000 arrays, lengths log-uniform in [2^6, 2^20] (seed 5), float32
    N(0,1) keys drawn on the device: one qms_sort_batch call for all of them
    (rounds planned on the device; the call returns before the GPU has run
    them), the same call captured once in a HIP graph and replayed, and one
    qms_sort call per array (every `per_array_stride`-th array, same
    kernels, same stream)."""
    lens = inputs.log_uniform_lengths(20000, seed=5, lo_exp=6, hi_exp=20)
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    src = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    src[src == 0] = 0.0
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    # tiles and merge arity picked by the autotuner on a sample of the batch
    # (every 20th array, about 5% of the keys), outside the timed region
    from paper_1804_10062_amd import autotune
    sidx = list(range(0, lens.size, 20))
    slens = lens[sidx]
    soff = inputs.offsets_from_lengths(slens)
    sample = torch.cat([src[int(off[j]):int(off[j + 1])] for j in sidx])
    sot = torch.from_numpy(soff.view(np.int64)).cuda()
    tune = autotune.autotune_batch(sample, sot, host_offsets=soff)
    del sample
    from tests.gpu_helpers import segments_sorted
    work = src.clone()
    times, calls = [], []
    for _ in range(reps + 1):
        work.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qms.qms_sort_batch(work, ot, host_offsets=off)
        t1 = time.perf_counter()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        calls.append(t1 - t0)
    qms.qms_batch_check()
    assert segments_sorted(work, ot), "batched output not sorted"
    t_batch = min(times[1:])
    # the whole batch as one HIP graph (captured on its own stream after a
    # warm-up call there, which creates that stream's workspace)
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        qms.qms_sort_batch(work, ot, host_offsets=off)
    gs.synchronize()
    graph = torch.cuda.CUDAGraph()
    work.copy_(src)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=gs):
        qms.qms_sort_batch(work, ot, host_offsets=off)
    gtimes = []
    for _ in range(reps):
        work.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        gtimes.append(time.perf_counter() - t0)
        assert segments_sorted(work, ot), "graph replay output not sorted"
    with torch.cuda.stream(gs):
        qms.qms_batch_check(stream=gs)
    t_graph = min(gtimes)
    del graph
    work.copy_(src)
    idx = list(range(0, lens.size, per_array_stride))
    keys_sub = int(sum(int(lens[j]) for j in idx))
    views = [work[int(off[j]):int(off[j + 1])] for j in idx]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in views:
        qms.qms_sort(v)
    torch.cuda.synchronize()
    t_per = time.perf_counter() - t0
    batched = n / t_batch / 1e9
    graphed = n / t_graph / 1e9
    per_array = keys_sub / t_per / 1e9
    # the per-array sample's input keys, kept on the host for the CPU leg
    host_sample = [src[int(off[j]):int(off[j + 1])].cpu().numpy().view(np.uint32).copy()
                   for j in idx]
    del work, src
    return host_sample, {
        "workload": "20,000 float32 arrays, lengths log-uniform in [2^6, 2^20] (seed 5), "
                    f"N(0,1) keys; {n} keys in all",
        "batched_Gkeys_per_s": round(batched, 3),
        "batched_ms": round(t_batch * 1e3, 2),
        "call_returns_after_ms": round(min(calls[1:]) * 1e3, 2),
        "graph_Gkeys_per_s": round(graphed, 3),
        "graph_ms": round(t_graph * 1e3, 2),
        "per_array_Gkeys_per_s": round(per_array, 4),
        "per_array_sample": f"every {per_array_stride}th array ({len(idx)} arrays, "
                            f"{keys_sub} keys), one qms_sort call each",
        "speedup": round(batched / per_array, 2),
        "graph_speedup": round(graphed / per_array, 2),
        "tuning": tune["best"],
        # every candidate the autotuner timed, keyed by all five tunables
        "autotune_trials_ms": {"/".join(str(t[f]) for f in autotune.FIELDS): t["ms"]
                               for t in tune["trials"]},
        "autotune_key": "/".join(autotune.FIELDS),
    }


def _request_hashes(torch, pool, off, ids):
    """Order-independent hash of each request's 32-bit words (requests
    `ids`, ranges off[j]..off[j+1] of the pool), summed in int64 chunks."""
    from tests.gpu_helpers import _C1, _C2
    out = torch.zeros(len(ids), dtype=torch.int64, device=pool.device)
    for q, j in enumerate(ids):
        a, b = int(off[j]), int(off[j + 1])
        acc = 0
        for c in range(a, b, 1 << 26):
            x = pool[c:min(b, c + (1 << 26))].to(torch.int64) & 0xFFFFFFFF
            h = x * _C1
            h = h ^ ((h >> 29) & ((1 << 35) - 1))
            h = h * _C2
            h = h ^ ((h >> 32) & 0xFFFFFFFF)
            acc = acc + h.sum()
        out[q] = acc
    return out


def _requests_sorted(torch, pool, off, is_f, ids):
    """Per request: keys non-decreasing (unsigned, or IEEE total order for
    float32 requests)."""
    ok = torch.ones(len(ids), dtype=torch.bool, device=pool.device)
    for q, j in enumerate(ids):
        a, b = int(off[j]), int(off[j + 1])
        if b - a < 2:
            continue
        u = pool[a:b].to(torch.int64) & 0xFFFFFFFF
        if is_f[j]:
            u = torch.where(u >= (1 << 31), -(u - (1 << 31)) - 1, u)
        ok[q] = bool((u[1:] >= u[:-1]).all())
    return ok


def bench_serving(qms, torch, np, inputs, loads, count: int, warmup: int,
                  budget: int = 64 << 30, oracle_every: int = 100):
    """Open-loop Poisson arrivals of sort requests (sizes floor(2^(10+14u)),
    uint32 or float32 with probability 1/2, uniform values) submitted to the
    library's server; latency = completion - scheduled arrival.  Per load:
    `warmup` requests first (not measured), then `count` measured ones.  All
    requests' keys are drawn on the device before the load starts; every
    measured request is checked on the device afterwards (sorted, and the
    same multiset hash as its input), every `oracle_every`-th one against
    the oracle."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    total_req = warmup + count
    u = inputs.unit_f64(total_req, seed=7, stream=11)
    sizes = np.floor(2.0 ** (10 + 14 * u)).astype(np.int64)
    is_f = (inputs.uniform_u32(total_req, seed=7, stream=12) & 1).astype(bool)
    off = np.zeros(total_req + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    total = int(off[-1])
    pool = torch.empty(total, dtype=torch.int32, device="cuda")
    pool_f = pool.view(torch.float32)
    measured = list(range(warmup, total_req))
    picks = measured[::oracle_every]
    out = {}
    for rate in loads:
        # keys of every request, drawn on the device
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1000 + int(rate))
        for c in range(0, total, 1 << 28):
            m = min(total, c + (1 << 28)) - c
            pool[c:c + m].random_(-(1 << 31), (1 << 31) - 1, generator=gen)
        for j in np.nonzero(is_f)[0]:
            a, b = int(off[j]), int(off[j + 1])
            pool_f[a:b].uniform_(0.0, 1.0, generator=gen)
        h_in = _request_hashes(torch, pool, off, measured)
        before = {j: pool[int(off[j]):int(off[j + 1])].cpu().numpy().copy() for j in picks}
        views = [(pool_f if is_f[j] else pool)[int(off[j]):int(off[j + 1])]
                 for j in range(total_req)]
        torch.cuda.synchronize()
        srv = qms.Server(hbm_budget_bytes=budget, device=0)
        # warm-up requests, then the measured load
        wt = [srv.submit(views[j]) for j in range(warmup)]
        for t in wt:
            while srv.poll(t)[0] != qms.QMS_OK:
                time.sleep(0.0002)
        arr = inputs.poisson_arrivals(count, float(rate), seed=100 + int(rate))
        tickets = []
        late = np.zeros(count)
        t0 = time.perf_counter()
        for q, j in enumerate(measured):
            due = t0 + arr[q]
            while time.perf_counter() < due:
                pass
            tickets.append(srv.submit(views[j]))
            late[q] = time.perf_counter() - due
        lat = np.zeros(count)
        pending = dict(enumerate(tickets))
        while pending:
            for q, t in list(pending.items()):
                st, l = srv.poll(t)
                if st == qms.QMS_OK:
                    lat[q] = l + late[q]
                    del pending[q]
            if pending:
                time.sleep(0.0002)
        st = srv.stats()
        srv.close()
        torch.cuda.synchronize()
        ok_sorted = _requests_sorted(torch, pool, off, is_f, measured)
        h_out = _request_hashes(torch, pool, off, measured)
        bad = int((~ok_sorted).sum().item()) + int((h_out != h_in).sum().item())
        assert bad == 0, f"{bad} served requests not sorted or not a permutation"

        def check(j):
            want, _, _ = oracle.sort(before[j].view(np.float32) if is_f[j] else
                                     before[j].view(np.uint32), counted=False)
            got = pool[int(off[j]):int(off[j + 1])].cpu().numpy()
            return np.array_equal(got.view(np.uint32), want.view(np.uint32))
        with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
            oracle_ok = all(ex.map(check, picks))
        assert oracle_ok, "a served request differs from the oracle"
        done_at = max(arr[q] + lat[q] for q in range(count))
        keys = int(sum(int(sizes[j]) for j in measured))
        p99_by_len = {str(m): round(float(np.percentile(lat[:m], 99)) * 1e3, 3)
                      for m in (count // 4, count // 2, count)}
        out[f"{rate}_req_per_s"] = {
            "offered_Gkeys_per_s": round(keys / arr[-1] / 1e9, 2),
            "completed_req_per_s": round(count / done_at, 1),
            "throughput_Gkeys_per_s": round(keys / done_at / 1e9, 3),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p99_ms_over_first_requests": p99_by_len,
            "batches": st["batches"],
            "peak_admitted_GB": round(st["peak_admitted_bytes"] / 1e9, 3),
            "waited_for_budget": st["waited_for_budget"],
            "submit_late_p99_ms": round(float(np.percentile(late, 99)) * 1e3, 3),
            "verified_on_device": count,
            "oracle_checked": len(picks),
        }
        del views, before
    del pool, pool_f
    return {"requests_per_load": count, "warmup_requests": warmup,
            "hbm_budget_GB": budget / 2**30,
            "sizes": "floor(2^(10 + 14u)) keys, u uniform (seed 7)", "loads": out}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: qms sorts on one GPU; --gpus {args.gpus} is not supported "
              "(the sort of one array is not sharded across GPUs here)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1804_10062_amd import inputs, qms

    qms.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup

    print(f"[bench] generating uniform u32 n=2^28 seed 2", file=sys.stderr, flush=True)
    host = inputs.uniform_u32(N_KEYS, seed=2)
    src = torch.from_numpy(host.view(np.int32)).to(dev)
    if args.pmc_run:
        # calibration: a plain copy of exactly 2^30 bytes (read 1 GiB, write 1 GiB)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        qms.qms_sort(dst)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_run": True, "copy_bytes": N_KEYS * 4,
                          "rounds": len(qms.qms_last_schedule())}))
        return
    copies = [src.clone() for _ in range(K + W)]
    torch.cuda.synchronize()

    print(f"[bench] warmup {W}", file=sys.stderr, flush=True)
    time_sorts(copies[:W], qms, torch, profile=False)
    print(f"[bench] timed {K} steps", file=sys.stderr, flush=True)
    secs, _ = time_sorts(copies[W:], qms, torch, profile=False)
    sched = qms.qms_last_schedule()
    # the last sorted copy must be sorted and a permutation of the input
    from tests.gpu_helpers import is_sorted, multiset_hash
    ok = is_sorted(copies[-1]) and multiset_hash(copies[-1]) == multiset_hash(src)
    if not ok:
        print("bench.py: output check FAILED", file=sys.stderr)
        sys.exit(1)
    # the same K steps again on fresh copies, every launch bracketed by HIP
    # events on the sorting stream (per-kernel durations for the roofline);
    # kept out of the headline timing because the events add a little time
    print(f"[bench] event-timed {K} steps", file=sys.stderr, flush=True)
    for i in range(K):
        copies[W + i].copy_(src)
    secs_prof, prof = time_sorts(copies[W:], qms, torch, profile=True)
    # the box's copy bandwidth in this run: a device copy of 1 GiB (read
    # 1 GiB, write 1 GiB), best of 5, timed with events
    cdst = copies[0]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    copy_ms = []
    for _ in range(6):
        ev0.record()
        cdst.copy_(src)
        ev1.record()
        ev1.synchronize()
        copy_ms.append(ev0.elapsed_time(ev1))
    copy_gbs = 2.0 * N_KEYS * 4 / (min(copy_ms[1:]) / 1e3) / 1e9
    del copies, cdst

    ms = secs / K * 1e3
    value = N_KEYS / (secs / K) / 1e9

    def kstat(d):
        return {
            "launches_per_step": d["launches"] / K,
            "ms_per_step": d["total_ms"] / K,
            "mean_launch_us": d["total_ms"] / d["launches"] * 1e3,
            "algorithmic_GB_per_step": d["bytes"] / K / 1e9,
            "achieved_GBs": (d["bytes"] / 1e9) / (d["total_ms"] / 1e3) if d["bytes"] else None,
        }

    # kernel classes, and the swap-merge passes by the binary level they
    # start at (a 4-way pass covers that level and the next)
    kernels, merge_levels = {}, {}
    for name, d in prof.items():
        if d["launches"] == 0:
            continue
        if name.startswith("merge_level_"):
            st = kstat(d)
            st["bytes_per_launch"] = d["bytes"] / d["launches"]
            st["pct_of_copy"] = (round(100.0 * st["achieved_GBs"] / copy_gbs, 1)
                                 if st["achieved_GBs"] else None)
            merge_levels[name[len("merge_level_"):]] = st
        else:
            kernels[name] = kstat(d)
    prof = {k: v for k, v in prof.items() if not k.startswith("merge_level_")}
    mk = prof["merge"]
    achieved = (mk["bytes"] / 1e9) / (mk["total_ms"] / 1e3)
    pm = measured_kernel("k_merge4")
    traffic = (None if pm is None else
               round((pm["fetch_bytes_per_sort"] + pm["write_bytes_per_sort"]) / pm["dispatches_per_sort"]))
    roofline = {
        "kernel": "swap-merge pass (k_merge4, k_merge)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": mk["bytes"] / mk["launches"],
        "mean_launch_us": mk["total_ms"] / mk["launches"] * 1e3,
        "launches": mk["launches"],
        # the same against a plain device copy of 1 GiB measured in this run
        "copy_GBs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
    }
    # the base case against the VALU issue peak, the exchange against HBM
    # with its measured traffic, the split searches' fetches
    kernel_rooflines = {}
    tk, pv = prof.get("tile_sort"), measured_kernel("k_tile_sort")
    if tk and pv and "SQ_INSTS_VALU_per_sort" in pv:
        rate = pv["SQ_INSTS_VALU_per_sort"] / (tk["total_ms"] / K / 1e3)
        kernel_rooflines["tile_sort"] = {
            "kernel": "k_tile_sort (bitonic base case)", "bound": "alu",
            "achieved": round(rate / 1e9, 1), "peak": round(VALU_PEAK / 1e9, 1),
            "unit": "G wave64 VALU instructions/s", "frac": round(rate / VALU_PEAK, 4),
            "valu_instructions_per_key": round(
                pv["SQ_INSTS_VALU_per_sort"] * 64 / (tk["bytes"] / K / 8.0), 1),
            "hbm_GBs": round(tk["bytes"] / 1e9 / (tk["total_ms"] / 1e3), 1)}
    sk, ps = prof.get("part_swap"), measured_kernel("k_part_swap")
    if sk and ps:
        t = sk["total_ms"] / K / 1e3
        tb = ps["fetch_bytes_per_sort"] + ps["write_bytes_per_sort"]
        alg = sk["bytes"] / K
        kernel_rooflines["part_swap"] = {
            "kernel": "k_part_swap (rank-matched exchange, pass A)", "bound": "hbm",
            "achieved": round(tb / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(tb / t / 1e9 / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(tb / t / 1e9 / copy_gbs, 4),
            "traffic_per_sort": tb, "algorithmic_per_sort": round(alg),
            "traffic_over_algorithmic": round(tb / alg, 3) if alg else None}
    ms_, pm_ = prof.get("merge_split"), measured_kernel("k_merge_split")
    if ms_ and pm_:
        kernel_rooflines["merge_split"] = {
            "kernel": "k_merge_split (merge-path searches)", "bound": "latency",
            "ms_per_sort": round(ms_["total_ms"] / K, 3),
            "fetch_GB_per_sort": round(pm_["fetch_bytes_per_sort"] / 1e9, 3)}
    # the whole sort against the same peak: all algorithmic bytes of the
    # executed schedule (base case, merge passes, counting, pass-A exchange)
    # over the headline time per sort
    sort_gb = sum(d["bytes"] for d in prof.values()) / K / 1e9
    whole_sort = {"algorithmic_GB_per_sort": round(sort_gb, 3),
                  "GB_s": round(sort_gb / (ms / 1e3), 1),
                  "frac": round(sort_gb / (ms / 1e3) / HBM_PEAK_GBS, 4),
                  "frac_of_copy": round(sort_gb / (ms / 1e3) / copy_gbs, 4),
                  "B_per_key": round(sort_gb * 1e9 / N_KEYS, 1)}

    dists = {"uniform": round(value, 3)}
    if not args.only_uniform:
        for name, kind, seed in (("nearly_sorted_1pct", "sorted_swaps", 3),
                                 ("reverse", "reverse", 0)):
            print(f"[bench] {name}", file=sys.stderr, flush=True)
            h = inputs.make_keys(kind, N_KEYS, seed)
            s2 = torch.from_numpy(h.view(np.int32)).to(dev)
            cps = [s2.clone() for _ in range(args.dist_steps + 1)]
            time_sorts(cps[:1], qms, torch, profile=False)
            sec2, _ = time_sorts(cps[1:], qms, torch, profile=False)
            if not is_sorted(cps[-1]):
                print(f"bench.py: {name} output not sorted", file=sys.stderr)
                sys.exit(1)
            dists[name] = round(N_KEYS / (sec2 / args.dist_steps) / 1e9, 3)
            dists[name + "_rounds"] = len(qms.qms_last_schedule())
            del cps, s2
        # key/payload pairs: 2^26 Zipf(1.1) keys over [0, 2^10), payload = index
        print("[bench] pairs", file=sys.stderr, flush=True)
        npairs = 1 << 26
        hk = inputs.zipf_u32(npairs, seed=4)
        k0 = torch.from_numpy(hk.view(np.int32)).to(dev)
        v0 = torch.arange(npairs, dtype=torch.int32, device=dev)
        ks = [k0.clone() for _ in range(args.dist_steps + 1)]
        vs = [v0.clone() for _ in range(args.dist_steps + 1)]
        torch.cuda.synchronize()
        qms.qms_sort_pairs(ks[0], vs[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for kt, vt in zip(ks[1:], vs[1:]):
            qms.qms_sort_pairs(kt, vt)
        torch.cuda.synchronize()
        sec2 = time.perf_counter() - t0
        if not is_sorted(ks[-1]):
            print("bench.py: pairs output not sorted", file=sys.stderr)
            sys.exit(1)
        dists["pairs_zipf_2e26"] = round(npairs / (sec2 / args.dist_steps) / 1e9, 3)
        del ks, vs, k0, v0
        # 64-bit keys (wide records): 2^27 uniform uint64 keys, the same 1 GiB
        print("[bench] u64", file=sys.stderr, flush=True)
        n64 = 1 << 27
        g64 = torch.Generator(device=dev)
        g64.manual_seed(6)
        w0 = torch.randint(-2 ** 63, 2 ** 63 - 1, (n64,), dtype=torch.int64, device=dev,
                           generator=g64)
        ws64 = [w0.clone() for _ in range(args.dist_steps + 1)]
        del w0
        time_sorts(ws64[:1], qms, torch, profile=False)
        sec2, _ = time_sorts(ws64[1:], qms, torch, profile=False)
        last = ws64[-1]
        hi, lo = (last >> 32) & 0xFFFFFFFF, last & 0xFFFFFFFF
        if not bool(((hi[:-1] < hi[1:]) | ((hi[:-1] == hi[1:]) & (lo[:-1] <= lo[1:]))).all()):
            print("bench.py: u64 output not sorted", file=sys.stderr)
            sys.exit(1)
        dists["u64_2e27"] = round(n64 / (sec2 / args.dist_steps) / 1e9, 3)
        dists["u64_2e27_GB_per_s_keys"] = round(8 * n64 / (sec2 / args.dist_steps) / 1e9, 1)
        del ws64, last, hi, lo
        # expensive comparisons (Experiments section: a comparator that
        # applies the logarithm to the integer keys): a random order of
        # 1..2^26 sorted with the plain uint32 order and with QMS_U32_LOG,
        # whose every comparison evaluates two double logarithms, at the
        # automatic X_THRESH (2048 for the logarithm order, 16384 for plain
        # keys) and at 16384 (more network comparisons per key, fewer merge
        # levels)
        print("[bench] log comparator", file=sys.stderr, flush=True)
        from paper_1804_10062_amd import autotune
        nl = 1 << 26
        s3 = torch.from_numpy(inputs.permutation_u32(nl, seed=11).view(np.int32)).to(dev)
        want = torch.arange(1, nl + 1, dtype=torch.int64, device=dev)
        logcmp = {"workload": "a random order of 1..2^26 (uint32), SplitMix64-keyed Feistel permutation, seed 11"}
        try:
            for label, bt in (("auto", 0), ("16384", 16384)):
                qms.qms_set_tuning(4, 4096, 16384, bt, 0)
                for name, code in (("plain", qms.QMS_U32), ("log", qms.QMS_U32_LOG)):
                    cps = [s3.clone() for _ in range(3)]
                    time_sorts(cps[:1], qms, torch, profile=False, dtype=code)
                    sec3, _ = time_sorts(cps[1:], qms, torch, profile=False, dtype=code)
                    if not bool((cps[-1].to(torch.int64) == want).all()):
                        print(f"bench.py: log comparator {name} output wrong", file=sys.stderr)
                        sys.exit(1)
                    logcmp[f"{name}_Gkeys_per_s_x_{label}"] = round(nl / (sec3 / 2) / 1e9, 3)
                    del cps
            # the logarithm order leaves the loop at 2^22 keys by default;
            # the same sort with the plain keys' exit size, 2^24, for the
            # trade-off between network comparisons and partition rounds
            qms.qms_set_tuning(4, 4096, 16384, 0, 1 << 24)
            cps = [s3.clone() for _ in range(3)]
            time_sorts(cps[:1], qms, torch, profile=False, dtype=qms.QMS_U32_LOG)
            sec3, _ = time_sorts(cps[1:], qms, torch, profile=False, dtype=qms.QMS_U32_LOG)
            if not bool((cps[-1].to(torch.int64) == want).all()):
                print("bench.py: log comparator at final_tile 2^24 output wrong", file=sys.stderr)
                sys.exit(1)
            logcmp["log_Gkeys_per_s_x_auto_final_2e24"] = round(nl / (sec3 / 2) / 1e9, 3)
            del cps
        finally:
            autotune.reset_tuning()
        logcmp["log_over_plain_time_x_auto"] = round(
            logcmp["plain_Gkeys_per_s_x_auto"] / logcmp["log_Gkeys_per_s_x_auto"], 2)
        dists["log_comparator_2e26"] = logcmp
        del s3, want

    # QuickMergeXsort's threshold (Sec. "QuickMergeXsort"): the same uniform
    # workload with the Mergesort stopping at runs of base_tile keys; the
    # bitonic base case spends lg(t)(lg(t)+1)/4 compare-exchanges per key,
    # every merge level one pass over the data
    xthresh = None
    if not args.only_uniform and not args.no_threshold_sweep:
        from paper_1804_10062_amd import autotune
        xthresh = {}
        try:
            for t0 in (0, 16384, 8192, 4096, 2048):
                print(f"[bench] X_THRESH {t0}", file=sys.stderr, flush=True)
                qms.qms_set_tuning(4, 4096, 16384, t0)
                cps = [src.clone() for _ in range(args.dist_steps + 1)]
                time_sorts(cps[:1], qms, torch, profile=False)
                sec2, _ = time_sorts(cps[1:], qms, torch, profile=False)
                if not is_sorted(cps[-1]):
                    print(f"bench.py: X_THRESH {t0} output not sorted", file=sys.stderr)
                    sys.exit(1)
                lg = int(t0 or 16384).bit_length() - 1
                first = qms.qms_last_schedule()[0]
                xthresh["auto" if t0 == 0 else str(t0)] = {
                    "Gkeys_per_s": round(N_KEYS / (sec2 / args.dist_steps) / 1e9, 3),
                    "ms_per_sort": round(sec2 / args.dist_steps * 1e3, 3),
                    "network_compare_exchanges_per_key": lg * (lg + 1) / 4,
                    "first_round_merge_levels": int(first[4])}
                del cps
        finally:
            autotune.reset_tuning()

    # X at the loop level: a range a partition round leaves with at most
    # final_tile keys leaves the loop and is sorted in place by the bitonic
    # network (8192: the loop runs down to the base tile, as in the paper;
    # the automatic default is 2^24 for these keys)
    final_sweep = None
    if not args.only_uniform and not args.no_threshold_sweep:
        from paper_1804_10062_amd import autotune
        final_sweep = {}
        try:
            for ft in (8192, 1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 25):
                print(f"[bench] final_tile {ft}", file=sys.stderr, flush=True)
                d = autotune.DEFAULTS
                qms.qms_set_tuning(d[0], d[1], d[2], d[3], ft)
                cps = [src.clone() for _ in range(args.dist_steps + 1)]
                time_sorts(cps[:1], qms, torch, profile=False)
                sec2, _ = time_sorts(cps[1:], qms, torch, profile=False)
                if not is_sorted(cps[-1]):
                    print(f"bench.py: final_tile {ft} output not sorted", file=sys.stderr)
                    sys.exit(1)
                final_sweep[str(ft)] = {
                    "Gkeys_per_s": round(N_KEYS / (sec2 / args.dist_steps) / 1e9, 3),
                    "ms_per_sort": round(sec2 / args.dist_steps * 1e3, 3),
                    "partition_rounds": len(qms.qms_last_schedule())}
                del cps
        finally:
            autotune.reset_tuning()

    batched, batched_host = None, None
    if not args.no_batched:
        print("[bench] batched vs per-array", file=sys.stderr, flush=True)
        batched_host, batched = bench_batched(qms, torch, np, inputs, args.per_array_stride)
    serving = None
    if not args.no_serving:
        print("[bench] serving", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()  # the serving pool takes about 145 GB
        serving = bench_serving(qms, torch, np, inputs, (2000, 10000, 50000),
                                args.serving_requests, args.serving_warmup)

    cpu = None
    if not args.no_cpu_baseline:
        m = 1 << args.cpu_sample_log2
        print(f"[bench] cpu oracle on 2^{args.cpu_sample_log2} keys, one pinned core",
              file=sys.stderr, flush=True)
        dt, core = _oracle_on_one_core(host[:m])
        cpu = {"value": round(m / dt / 1e9, 5), "unit": "Gkeys/s", "cores": 1,
               "kind": "oracle", "seconds": round(dt, 2), "pinned_core": core,
               "sample": ("the whole" if m == N_KEYS else f"the first 2^{args.cpu_sample_log2} "
                          "keys of the") + " uniform 2^28 workload (seed 2), single-threaded C "
                          "oracle (QuickMergesort of Fig. 2, counters compiled out), in a child "
                          "process pinned to one core"}
        if batched_host is not None:
            # the batched workload's sample on the host's cores: one oracle
            # call per array on a pool of threads (ctypes releases the GIL);
            # at most 16 threads, the host share of one GPU on the box
            import oracle
            from concurrent.futures import ThreadPoolExecutor
            nproc = os.cpu_count() or 1
            workers = max(1, min(16, nproc))
            keys = int(sum(a.size for a in batched_host))
            print(f"[bench] cpu oracle on the batched sample, {workers} threads",
                  file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            with ThreadPoolExecutor(max_workers=workers) as ex:
                list(ex.map(lambda a: oracle.sort_inplace_fast(a, True), batched_host))
            dt = time.perf_counter() - t0
            batched["cpu_baseline"] = {
                "value": round(keys / dt / 1e9, 5), "unit": "Gkeys/s", "cores": workers,
                "nproc": nproc, "kind": "oracle", "seconds": round(dt, 2),
                "sample": f"the per-array sample of the batched workload ({len(batched_host)} "
                          f"float32 arrays, {keys} keys), one C oracle call per array on a "
                          f"pool of {workers} threads"}
            del batched_host

    out = {
        "metric": "Gkeys/s (uint32, n=2^28) + HBM roofline %; batched vs per-array; p99 latency",
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms, 3),
        "ms_per_step_with_event_timing": round(secs_prof / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: uniform uint32 keys from a seeded SplitMix64 stream",
        "config": {"workload": "one array of 2^28 uint32 keys (1 GiB), uniform on [0, 2^32), "
                               "seed 2; in-place QuickMergesort",
                   "n": N_KEYS, "rounds": len(sched)},
        "roofline": roofline,
        "whole_sort": whole_sort,
        "cpu_baseline": cpu,
        "distributions_Gkeys_per_s": dists,
        "x_thresh_tradeoff": xthresh,
        "final_tile_tradeoff": final_sweep,
        "batched": batched,
        "serving": serving,
        "kernels": kernels,
        "kernel_rooflines": kernel_rooflines,
        "merge_levels": merge_levels,
        "copy_GBs": round(copy_gbs, 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
