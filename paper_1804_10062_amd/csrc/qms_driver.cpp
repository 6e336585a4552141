// qms_driver.cpp -- the QuickMergesort loop (Fig. 2's sort()) run for many
// independent segments at once.
//
// Every segment follows the paper's loop: partition its range around the
// median of three keys, Mergesort the smaller side with the larger side as
// swap space, continue on the larger side; a range of at most one base tile
// is finished by the base case in place.  All segments advance in lockstep
// rounds, and every phase of a round is one launch for all segments (task
// tables, qms_device.hpp): count + scan, [split +] swap of pass A, scan,
// [split +] swap of pass B, base case, then one launch pair per merge level.
// The host reads three counters per segment back once per round to size the
// later launches of the round.  A single array is a batch of one (its task
// tables travel by value in the kernel arguments).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <vector>

#include "qms.h"
#include "qms_host.hpp"
#include "qms_internal.hpp"

namespace qms {

namespace {

uint32_t ceil_log2(uint64_t x) {
    uint32_t l = 0;
    while ((1ull << l) < x) ++l;
    return l;
}

// bump allocator over a pinned host arena mirrored at the same offsets in
// device memory
struct Arena {
    char *h;
    char *d;
    size_t cap, used = 0;
    template <class T>
    T *take(size_t count, size_t *off) {
        const size_t o = used;
        used += (count * sizeof(T) + 255) & ~(size_t)255;
        if (used > cap) return nullptr;
        *off = o;
        return (T *)(h + o);
    }
    template <class T>
    const T *dev(size_t off) const {
        return (const T *)(d + off);
    }
};

struct Seg {
    uint32_t *keys, *vals;
    uint64_t lo, hi;
    bool bad_split;  // the last round's smaller side held less than 1/16 of its range
};

// The host arenas alternate between rounds.  An arena's contents go to the
// device by asynchronous copies, so before the host writes it again those
// copies must have run: a round that reads counters back synchronises the
// stream, but a round without a partition does not, so every round records
// an event when it is done with its arena (ArenaUse's destructor, on every
// exit path) and the round that takes the arena next waits for it.
struct ArenaUse {
    Workspace &ws;
    hipStream_t st;
    int slot;
    Arena ar;
    ArenaUse(Workspace &w, hipStream_t s) : ws(w), st(s), slot((int)(w.rounds & 1)) {
        if (ws.arena_busy[slot]) {
            (void)hipEventSynchronize(ws.arena_done[slot]);
            ws.arena_busy[slot] = false;
        }
        ++ws.rounds;
        ar = Arena{(char *)ws.htab[slot], (char *)ws.dtab, ws.tab_bytes};
    }
    ~ArenaUse() {
        // a workspace without events has pageable arenas, whose copies have
        // read the host memory by the time they return
        if (!ws.arena_done[slot]) return;
        if (hipEventRecord(ws.arena_done[slot], st) == hipSuccess) {
            ws.arena_busy[slot] = true;
        } else {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(st);
        }
    }
    ArenaUse(const ArenaUse &) = delete;
    ArenaUse &operator=(const ArenaUse &) = delete;
};

// One round's tables.
int upload(Arena &ar, size_t from, hipStream_t st) {
    if (ar.used <= from) return QMS_OK;
    hipError_t e =
        hipMemcpyAsync(ar.d + from, ar.h + from, ar.used - from, hipMemcpyHostToDevice, st);
    return e == hipSuccess ? QMS_OK : hip_error(e, "task table upload");
}

thread_local std::vector<std::array<uint64_t, kScheduleWords>> g_schedule;

// The median-of-medians pivots of the table entries listed in idx, in groups
// of at most caps.mom (one histogram each).
int mom_pivots(int dt, const PartSeg *pt, const std::vector<uint32_t> &idx, Arena &ar,
               Workspace &ws, hipStream_t st) {
    for (size_t g0 = 0; g0 < idx.size(); g0 += ws.caps.mom) {
        const uint32_t n = (uint32_t)std::min<size_t>(ws.caps.mom, idx.size() - g0);
        const size_t mark = ar.used;
        size_t o_tab, o_pre;
        PartSeg *tab = ar.take<PartSeg>(n, &o_tab);
        uint32_t *pre = ar.take<uint32_t>(n + 1, &o_pre);
        if (!tab || !pre) return set_error(QMS_ERR_NOMEM, "task table arena too small");
        pre[0] = 0;
        for (uint32_t i = 0; i < n; ++i) {
            tab[i] = pt[idx[g0 + i]];
            tab[i].pad = i;
            pre[i + 1] = pre[i] + mom_tiles(tab[i].s);
        }
        if (n > 1) {
            int rc = upload(ar, mark, st);
            if (rc != QMS_OK) return rc;
        }
        TaskRef<PartSeg> R{};
        R.A = n;
        R.one = tab[0];
        R.tab = ar.dev<PartSeg>(o_tab);
        R.pre = ar.dev<uint32_t>(o_pre);
        hipError_t e = launch_mom_pivot(dt, R, pre[n], 0, true, ws, st);
        if (e != hipSuccess) return hip_error(e, "median-of-medians pivot");
    }
    return QMS_OK;
}


}  // namespace

size_t tab_arena_bytes(uint32_t segs) {
    // per segment: partition entry, 5 prefixes, up to 2 sort tasks, 2 prefixes
    // (each table rounded up to 256 bytes by the arena)
    const size_t per = sizeof(PartSeg) + 5 * 4 + 2 * sizeof(SortSeg) + 2 * 2 * 4;
    return per * segs + 64 * 1024;
}

const std::vector<std::array<uint64_t, kScheduleWords>> &last_schedule() { return g_schedule; }

// Arena bytes of the network tables for `count` ranges of at most 2^K keys.
static size_t network_table_bytes(size_t count, uint32_t K, uint32_t lt) {
    const size_t launches = bitonic_passes(K, lt).size();
    return ((count * sizeof(SortSeg) + 255) & ~(size_t)255) +
           launches * (((count + 1) * 4 + 255) & ~(size_t)255);
}

// X at the loop level: the ranges in xf (tiles already sorted in place by
// the base case) are finished by the bitonic network, in place.  Stage k
// takes the ranges of more than 2^(k-1) keys (xf is sorted by size, largest
// first, so they are a prefix of the table).
static int final_network(int dt, bool pairs, std::vector<SortSeg> &xf, Arena &ar, uint32_t T0,
                         double elem_bytes, hipStream_t st) {
    if (xf.empty()) return QMS_OK;
    std::stable_sort(xf.begin(), xf.end(),
                     [](const SortSeg &x, const SortSeg &y) { return x.m > y.m; });
    const uint32_t lt = ceil_log2(T0), K = ceil_log2(xf[0].m);
    const uint32_t n = (uint32_t)xf.size();
    const size_t mark = ar.used;
    size_t o_tab;
    SortSeg *tab = ar.take<SortSeg>(n, &o_tab);
    if (!tab) return set_error(QMS_ERR_NOMEM, "task table arena too small");
    for (uint32_t a = 0; a < n; ++a) tab[a] = xf[a];
    std::vector<BitonicLaunch> passes = bitonic_passes(K, lt);
    std::vector<size_t> o_pre(passes.size(), 0);
    for (size_t i = 0; i < passes.size(); ++i) {
        BitonicLaunch &L = passes[i];
        uint32_t c = 0;  // ranges in stage k: more than 2^(k-1) keys
        while (c < n && tab[c].m > (1ull << (L.k - 1))) ++c;
        L.tasks.A = c;
        if (c == 0) continue;
        L.tasks.one = tab[0];
        uint32_t *pre = ar.take<uint32_t>(c + 1, &o_pre[i]);
        if (!pre) return set_error(QMS_ERR_NOMEM, "task table arena too small");
        pre[0] = 0;
        for (uint32_t a = 0; a < c; ++a) pre[a + 1] = pre[a] + bitonic_items_of(L.kind, L.k, L.lo, L.hi, tab[a].m, T0);
        L.items = pre[c];
        for (uint32_t a = 0; a < c; ++a) L.bytes += 2.0 * elem_bytes * (double)tab[a].m;
    }
    int rc = upload(ar, mark, st);
    if (rc != QMS_OK) return rc;
    for (size_t i = 0; i < passes.size(); ++i) {
        BitonicLaunch &L = passes[i];
        if (L.tasks.A == 0) continue;
        L.tasks.tab = ar.dev<SortSeg>(o_tab);
        L.tasks.pre = ar.dev<uint32_t>(o_pre[i]);
        const hipError_t e = launch_bitonic_pass(dt, pairs, L, st);
        if (e != hipSuccess) return hip_error(e, "final bitonic network");
    }
    return QMS_OK;
}

// Sort a group of segments (count <= caps.segs, total keys < 2^32).
static int sort_group(int dt, bool pairs, std::vector<Seg> &segs, Workspace &ws,
                      hipStream_t st, bool log, const Tuning &tune) {
    // 64-bit keys: twice the bytes per element and the 8,192-element base
    // tile of key/payload pairs
    const bool wide = dtype_wide(dt);
    const double w = (pairs || wide) ? 2.0 : 1.0;
    // T0: the base case's workgroup tile; ranges of at most T0 keys are
    // finished in place by one workgroup.  R0: the run width at which each
    // round's Mergesort stops and calls the base case X (QuickMergeXsort's
    // X_THRESH, a tunable), so that a workgroup tile holds T0 / R0 runs.
    const uint32_t T0 = base_tile_of(pairs, wide);
    // base_tile 0 (automatic): the whole workgroup tile, except that 4-way
    // sorts take half of it when that makes the level count even, so that
    // every pass merges four runs (no 2-way first pass); 64-bit keys take
    // runs of kMergeTile keys, since their 64-bit network costs more per
    // level than a merge level (2^27 uint64: 11.0 against 10.6 Gkeys/s), and
    // so does the logarithm order, whose network comparisons cost more than
    // the merges' (QuickMergeXsort's trade-off; 2^26 keys: 1.95 against
    // 1.56 Gkeys/s)
    const bool auto_r0 = tune.base_tile == 0;
    const bool short_runs = wide || dt == QMS_U32_LOG;
    // 64-bit keys with payloads merge two runs per pass (a 4-way tile of
    // their 96-bit elements would not fit the LDS budget)
    const bool four_way_sort = tune.merge_ways == 4 && !(pairs && wide);
    const uint32_t R0 = auto_r0 ? (short_runs ? (uint32_t)kMergeTile : T0) : std::min(T0, tune.base_tile);
    auto levels = [](uint64_t m, uint32_t r) -> uint32_t {
        return m > r ? ceil_log2((m + r - 1) / r) : 0;
    };
    // run width and level count of a Mergesort of m keys
    auto set_levels = [&](SortSeg &t) {
        t.w0 = R0;
        t.L = levels(t.m, R0);
        if (auto_r0 && four_way_sort && !short_runs && (t.L & 1u)) {
            t.w0 = R0 / 2;
            t.L = levels(t.m, t.w0);
        }
    };
    // region pointers: keys are ew 32-bit words wide
    const uint64_t ew = wide ? 2 : 1;
    auto kptr = [&](const Seg &g, uint64_t off) { return g.keys + ew * off; };
    auto vptr = [&](const Seg &g, uint64_t off) { return g.vals ? g.vals + off : nullptr; };
    // TF: a range that a partition round leaves with at most TF keys leaves
    // the loop and is sorted in place by X, a bitonic network (QuickXsort
    // with X at the loop level; the paper's loop continues down to T0, which
    // final_tile = T0 reproduces).  An input array of at most T0 keys goes to
    // the base case in place; every larger one is partitioned at least once,
    // so its top level is always QuickMergesort's (partition, Mergesort of
    // one side with the other side as its buffer).
    // several arrays in one loop leave it earlier (group_loop_exit)
    uint64_t TF = std::max<uint64_t>(T0, loop_exit_keys(tune, dt));
    if (tune.final_tile == 0 && segs.size() > 1) {
        std::vector<uint64_t> lens(segs.size());
        for (size_t i = 0; i < segs.size(); ++i) lens[i] = segs[i].hi - segs[i].lo;
        TF = group_loop_exit(TF, T0, lens.data(), lens.size());
    }
    // a final range: the base case sorts its tiles in place (L = 0), the
    // network finishes it if it is longer than one tile
    auto final_task = [&](const Seg &g, uint64_t lo, uint32_t s) {
        return SortSeg{kptr(g, lo), vptr(g, lo), nullptr, nullptr, s, 0, 0, T0, 0, 0};
    };
    // per-key bytes of an element (key and payload), for the profile
    const double elem_bytes = (wide ? 8.0 : 4.0) + (pairs ? 4.0 : 0.0);
    // the network tables of one round take at most a quarter of the arena;
    // finals beyond that wait for the next round
    const size_t net_budget = ws.tab_bytes / 4;
    std::vector<uint32_t> active, next;
    // A range that becomes small in a round still holds that round's swap
    // buffer, so it runs one round later (next_finals -> ready_finals).
    std::vector<SortSeg> ready_finals, next_finals, tasks, deferred, xf;
    for (uint32_t i = 0; i < segs.size(); ++i) {
        const Seg &g = segs[i];
        const uint64_t s = g.hi - g.lo;
        if (s > T0) active.push_back(i);
        else if (s > 1) ready_finals.push_back(final_task(g, g.lo, (uint32_t)s));
    }
    while (!active.empty() || !ready_finals.empty()) {
        ArenaUse use(ws, st);
        Arena &ar = use.ar;
        tasks.clear();
        // ---- the finals that run this round: all of at most T0 keys (one
        // tile each), the longer ones while their network tables fit the
        // round's share of the arena; the rest wait for the next round ----
        deferred.clear();
        xf.clear();
        {
            std::vector<SortSeg> big;
            for (const SortSeg &f : ready_finals) {
                if (f.m > T0) big.push_back(f);
                else tasks.push_back(f);
            }
            std::stable_sort(big.begin(), big.end(),
                             [](const SortSeg &x, const SortSeg &y) { return x.m > y.m; });
            for (const SortSeg &f : big) {
                const uint32_t K = ceil_log2(xf.empty() ? f.m : xf[0].m);
                if (!xf.empty() && network_table_bytes(xf.size() + 1, K, ceil_log2(T0)) > net_budget) {
                    deferred.push_back(f);
                    continue;
                }
                xf.push_back(f);
                tasks.push_back(f);
            }
        }
        if (!active.empty()) {
            // ---- partition: count + scan A, then read three counters back.
            // One table entry per range; a range of 2^32 keys or more takes
            // blocks of at most kHugeBlock keys around the pivot of the whole
            // range, gathered by rotations after the exchanges ----
            struct Entry {
                uint32_t seg;
                uint64_t off;  // from the range's start
                uint32_t s;
            };
            std::vector<Entry> ent;
            std::vector<uint32_t> first_entry(active.size() + 1, 0);
            for (size_t i = 0; i < active.size(); ++i) {
                const Seg &g = segs[active[i]];
                const uint64_t s = g.hi - g.lo;
                first_entry[i] = (uint32_t)ent.size();
                if (s < kHugeRange) {
                    ent.push_back(Entry{(uint32_t)i, 0, (uint32_t)s});
                } else {
                    for (uint64_t o = 0; o < s; o += kHugeBlock)
                        ent.push_back(Entry{(uint32_t)i, o, (uint32_t)std::min<uint64_t>(kHugeBlock, s - o)});
                }
            }
            first_entry[active.size()] = (uint32_t)ent.size();
            const uint32_t A = (uint32_t)ent.size();
            if (A > ws.caps.segs) return set_error(QMS_ERR_UNSUPPORTED, "too many ranges for one round");
            auto is_huge = [&](size_t i) { return first_entry[i + 1] - first_entry[i] > 1 ||
                                                  segs[active[i]].hi - segs[active[i]].lo >= kHugeRange; };
            uint64_t sum_s = 0;
            for (const Entry &en : ent) sum_s += en.s;
            uint32_t TP = tune.partition_tile;
            for (;;) {
                uint64_t tot = 0;
                for (const Entry &en : ent) tot += (en.s + TP - 1) / TP;
                if (tot <= ws.caps.tiles) break;
                TP *= 2;
            }
            size_t o_tab, o_pre, o_scan;
            PartSeg *pt = ar.take<PartSeg>(A, &o_tab);
            uint32_t *pc = ar.take<uint32_t>(A + 1, &o_pre);
            uint32_t *ps = ar.take<uint32_t>(A + 1, &o_scan);
            if (!pt || !pc || !ps) return set_error(QMS_ERR_NOMEM, "task table arena too small");
            uint32_t toff = 0, coff = 0, max_nt = 0;
            std::vector<uint32_t> mom_idx;
            pc[0] = 0;
            for (uint32_t a = 0; a < A; ++a) {
                const Entry &en = ent[a];
                const size_t i = en.seg;
                const Seg &g = segs[active[i]];
                const uint32_t s = en.s;
                const uint32_t nt = (s + TP - 1) / TP;
                // the pivot comes from the round state: the median of the
                // medians of three (selected below), or for the blocks of a
                // huge range the median of three of the whole range
                const bool huge = is_huge(i);
                const bool mom = g.bad_split && !huge;
                if (mom) mom_idx.push_back(a);
                const uint32_t fl = (mom || huge) ? kPivotMoM : 0u;
                // the entry's keys start at its own first cell (position 0)
                pt[a] = PartSeg{kptr(g, g.lo + en.off), vptr(g, g.lo + en.off), 0, s, toff, nt, coff,
                                a, fl, 0};
                toff += nt;
                coff += (s + 4095) / 4096 + 2;
                pc[a + 1] = toff;
                max_nt = std::max(max_nt, nt);
            }
            if (coff > ws.caps.chunks)
                return set_error(QMS_ERR_UNSUPPORTED, "batch too large for one round");
            // scans of large ranges take 1024 threads; workgroups per segment
            const uint32_t scan_threads = max_nt > 4 * kBlock ? kScanThreads : kBlock;
            ps[0] = 0;
            for (uint32_t a = 0; a < A; ++a) ps[a + 1] = ps[a] + scan_a_groups(pt[a].nt, scan_threads);
            if (A > 1) {
                int rc = upload(ar, 0, st);
                if (rc != QMS_OK) return rc;
            }
            if (!mom_idx.empty()) {
                int rc = mom_pivots(dt, pt, mom_idx, ar, ws, st);
                if (rc != QMS_OK) return rc;
            }
            for (size_t i = 0; i < active.size(); ++i) {
                if (!is_huge(i)) continue;
                const Seg &g = segs[active[i]];
                const hipError_t e0 = launch_huge_pivot(dt, kptr(g, g.lo), g.hi - g.lo, ws.meta,
                                                        first_entry[i],
                                                        first_entry[i + 1] - first_entry[i], st);
                if (e0 != hipSuccess) return hip_error(e0, "pivot of a huge range");
            }
            PartitionLaunch L{};
            L.tasks.A = A;
            L.tasks.one = pt[0];
            L.tasks.tab = ar.dev<PartSeg>(o_tab);
            L.tasks.pre = ar.dev<uint32_t>(o_pre);
            L.TP = TP;
            L.chunk_span = tune.chunk_span;
            L.scan_threads = scan_threads;
            L.groups = (uint64_t)toff * (TP / kWave) <= ws.caps.groups;
            L.keys_total = (double)sum_s;
            L.ws = &ws;
            L.phase = 0;
            L.grid = toff;
            hipError_t e = launch_partition_phase(dt, pairs, L, st);
            if (e == hipSuccess) {
                L.phase = 6;
                L.tasks.pre = ar.dev<uint32_t>(o_scan);
                L.grid = ps[A];
                e = launch_partition_phase(dt, pairs, L, st);
            }
            if (e != hipSuccess) return hip_error(e, "partition count/scan");
            e = hipMemcpyAsync(ws.h_res, ws.res, sizeof(uint32_t) * 4 * A, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_error(e, "partition readback");

            // ---- work of pass A and pass B per segment ----
            const size_t mark = ar.used;
            size_t o_ca, o_wa, o_cb, o_wb;
            uint32_t *ca = ar.take<uint32_t>(A + 1, &o_ca), *wa = ar.take<uint32_t>(A + 1, &o_wa);
            uint32_t *cb = ar.take<uint32_t>(A + 1, &o_cb), *wb = ar.take<uint32_t>(A + 1, &o_wb);
            if (!ca || !wa || !cb || !wb) return set_error(QMS_ERR_NOMEM, "task table arena too small");
            ca[0] = wa[0] = cb[0] = wb[0] = 0;
            double swap_bytes = 0;
            bool any_b = false;
            for (uint32_t a = 0; a < A; ++a) {
                const uint64_t s = pt[a].s;
                const uint64_t c_lt = ws.h_res[4 * a], c_eq = ws.h_res[4 * a + 1];
                const uint64_t X = ws.h_res[4 * a + 2];
                // c_eq is 0 when the pivot-equal keys stay in the ">= p" side;
                // then the "< p" side is not empty (a block of a huge range
                // need not hold the pivot: all its keys may exceed it)
                if ((c_eq == 0 && c_lt == 0 && !is_huge(ent[a].seg)) || c_lt + c_eq > s)
                    return set_error(QMS_ERR_HIP, "partition returned inconsistent counts");
                const uint64_t nch = chunk_count(X, s, tune.chunk_span);
                ca[a + 1] = ca[a] + (uint32_t)nch;
                wa[a + 1] = wa[a] + (uint32_t)(nch > 1 ? 2 * (nch - 1) : 0);
                if (X > 0) swap_bytes += (wide ? 8.0 : 4.0) * (double)s + 2.0 * 4.0 * w * (double)X;
                // pass B pairs are at most min(#==, #>); size its grids for that
                const uint64_t gt = s - c_lt - c_eq;
                const uint64_t xb = std::min(c_eq, gt);
                uint64_t nb = 0;
                if (xb > 0) {
                    const uint64_t full = (xb + kRankChunk - 1) / kRankChunk;
                    const uint64_t target = (s + tune.chunk_span - 1) / tune.chunk_span;
                    nb = std::min(xb, std::max(full, target));
                    any_b = true;
                }
                cb[a + 1] = cb[a] + (uint32_t)nb;
                wb[a + 1] = wb[a] + (uint32_t)(nb > 1 ? 2 * (nb - 1) : 0);
            }
            if (A > 1) {
                int rc = upload(ar, mark, st);
                if (rc != QMS_OK) return rc;
            }
            if (ca[A] > 0) {
                L.phase = 1;
                L.tasks.pre = ar.dev<uint32_t>(o_wa);
                L.work = wa[A];
                L.grid = (wa[A] + kWaves - 1) / kWaves;
                if ((e = launch_partition_phase(dt, pairs, L, st)) != hipSuccess)
                    return hip_error(e, "split A");
                L.phase = 2;
                L.tasks.pre = ar.dev<uint32_t>(o_ca);
                L.grid = ca[A];
                L.bytes = swap_bytes;
                if ((e = launch_partition_phase(dt, pairs, L, st)) != hipSuccess)
                    return hip_error(e, "swap A");
            }
            if (any_b) {
                L.phase = 4;
                L.grid = A;
                if ((e = launch_partition_phase(dt, pairs, L, st)) != hipSuccess)
                    return hip_error(e, "scan B");
                L.phase = 3;
                L.tasks.pre = ar.dev<uint32_t>(o_wb);
                L.work = wb[A];
                L.grid = (wb[A] + kWaves - 1) / kWaves;
                if ((e = launch_partition_phase(dt, pairs, L, st)) != hipSuccess)
                    return hip_error(e, "split B");
                L.phase = 5;
                L.tasks.pre = ar.dev<uint32_t>(o_cb);
                L.grid = cb[A];
                if ((e = launch_partition_phase(dt, pairs, L, st)) != hipSuccess)
                    return hip_error(e, "swap B");
            }

            // ---- a huge range: gather the blocks' classes, [< p | == p | > p]
            // of each block, into those of the whole range (two rotations per
            // block after the first) ----
            std::vector<uint64_t> agg_lt(active.size(), 0), agg_eq(active.size(), 0);
            for (size_t i = 0; i < active.size(); ++i) {
                const Seg &g = segs[active[i]];
                uint64_t nl = 0, ne = 0, ng = 0;  // classes gathered so far
                for (uint32_t a = first_entry[i]; a < first_entry[i + 1]; ++a) {
                    const uint64_t l = ws.h_res[4 * a], q = ws.h_res[4 * a + 1];
                    const uint64_t r = ent[a].s - l - q;
                    if (a > first_entry[i]) {
                        const uint64_t pos0 = g.lo + nl + ne + ng;  // the block's first cell
                        // its "<" part before the gathered "==" and ">" parts
                        hipError_t e1 = launch_rotate(wide, pairs, g.keys, g.vals, g.lo + nl,
                                                      pos0, pos0 + l, st);
                        // its "==" part before the gathered ">" part
                        if (e1 == hipSuccess)
                            e1 = launch_rotate(wide, pairs, g.keys, g.vals, g.lo + nl + l + ne,
                                               pos0 + l, pos0 + l + q, st);
                        if (e1 != hipSuccess) return hip_error(e1, "gathering a huge range");
                    }
                    nl += l;
                    ne += q;
                    ng += r;
                }
                agg_lt[i] = nl;
                agg_eq[i] = ne;
            }

            // ---- side choice (Fig. 2 sort(): the smaller side is mergesorted
            // with the larger side as swap space; the loop keeps the larger) ----
            next.clear();
            for (size_t i = 0; i < active.size(); ++i) {
                Seg &g = segs[active[i]];
                const uint64_t s = g.hi - g.lo;
                const uint64_t c_lt = agg_lt[i], c_eq = agg_eq[i];
                const uint64_t b1 = g.lo + c_lt, b2 = b1 + c_eq;
                const uint64_t mL = c_lt, mR = g.hi - b2;
                if (std::min(mL, mR) >= (1ull << 32))
                    return set_error(QMS_ERR_UNSUPPORTED, "a Mergesort side of 2^32 keys or more");
                SortSeg t{};
                if (mL <= mR) {
                    t.keys = kptr(g, g.lo);
                    t.vals = vptr(g, g.lo);
                    t.bkeys = kptr(g, b2);
                    t.bvals = vptr(g, b2);
                    t.m = (uint32_t)mL;
                    g.lo = b2;
                } else {
                    t.keys = kptr(g, b2);
                    t.vals = vptr(g, b2);
                    t.bkeys = kptr(g, b1 - mR);
                    t.bvals = vptr(g, b1 - mR);
                    t.m = (uint32_t)mR;
                    g.hi = b1;
                }
                set_levels(t);
                // HybridQuickMergesort's rule with delta = 1/16: a split outside
                // [s/16, 15 s/16] makes the next pivot of this array the
                // median of the medians of three; the one after returns to
                // median-of-3
                const bool mom = g.bad_split && !is_huge(i);
                g.bad_split = std::min(mL, mR) * 16 < s;
                if (t.m > 1) tasks.push_back(t);
                if (log)
                    g_schedule.push_back(
                        {s, c_lt, c_eq, (uint64_t)(s - c_lt - c_eq), t.L, mom ? 1ull : 0ull});
                // the larger side goes on in the loop unless it is small
                // enough for X
                const uint64_t s2 = g.hi - g.lo;
                if (s2 <= TF) {
                    if (s2 > 1) next_finals.push_back(final_task(g, g.lo, (uint32_t)s2));
                } else {
                    next.push_back(active[i]);
                }
            }
            active.swap(next);
        }

        // ---- Mergesort tasks of this round (smaller sides and finals) ----
        ready_finals.swap(deferred);
        for (const SortSeg &f : next_finals) ready_finals.push_back(f);
        next_finals.clear();
        if (tasks.empty()) continue;
        // order: tasks with an even level count first, then odd, each by
        // level count descending.  The passes that start at binary level l
        // then cover a contiguous range: with 4-way passes the passes at l
        // belong to the tasks with L > l and L = l (mod 2), the 2-way first
        // passes (l = 0) to the odd ones; with 2-way passes only
        // (merge_ways 2) every task with L > l runs a 2-way pass at l
        const bool two = !four_way_sort;
        const bool by_parity = !two;
        std::stable_sort(tasks.begin(), tasks.end(), [&](const SortSeg &x, const SortSeg &y) {
            if (by_parity && (x.L & 1u) != (y.L & 1u)) return (x.L & 1u) < (y.L & 1u);
            return x.L > y.L;
        });
        const uint32_t T = (uint32_t)tasks.size();
        const size_t mark = ar.used;
        size_t o_st, o_pt, o_pm;
        SortSeg *stab = ar.take<SortSeg>(T, &o_st);
        uint32_t *ptile = ar.take<uint32_t>(T + 1, &o_pt);
        uint32_t *pmerge = ar.take<uint32_t>(T + 1, &o_pm);
        if (!stab || !ptile || !pmerge) return set_error(QMS_ERR_NOMEM, "task table arena too small");
        ptile[0] = pmerge[0] = 0;
        double base_bytes = 0;
        uint32_t maxL = 0, E = 0;
        for (uint32_t a = 0; a < T; ++a) {
            SortSeg t = tasks[a];
            t.split_off = pmerge[a];
            t.two_way = two ? 1u : 0u;
            stab[a] = t;
            ptile[a + 1] = ptile[a] + (t.m + T0 - 1) / T0;
            // merge splits and run samples: Mergesort tasks only (a range
            // sorted in place, L = 0, writes no samples, so the finals of a
            // round take no room there whatever their number)
            pmerge[a + 1] = pmerge[a] + (t.L ? (t.m + kMergeTile - 1) / kMergeTile : 0u);
            base_bytes += ((merge_passes(t.L, two) & 1) ? 16.0 : 8.0) * w * (double)t.m;
            maxL = std::max(maxL, t.L);
            if (!by_parity || (t.L & 1u) == 0) E = a + 1;
        }
        if (pmerge[T] > ws.caps.splits) return set_error(QMS_ERR_UNSUPPORTED, "too many merge tiles");
        if (T > 1) {
            int rc = upload(ar, mark, st);
            if (rc != QMS_OK) return rc;
        }
        TaskRef<SortSeg> R{};
        R.A = T;
        R.one = stab[0];
        R.tab = ar.dev<SortSeg>(o_st);
        R.pre = ar.dev<uint32_t>(o_pt);
        hipError_t e = launch_tile_sort(dt, pairs, R, ptile[T], 0, base_bytes, ws, st);
        if (e != hipSuccess) return hip_error(e, "base case");
        // the finals' networks (their ranges are disjoint from this round's
        // Mergesort regions)
        int rcx = final_network(dt, pairs, xf, ar, T0, elem_bytes, st);
        if (rcx != QMS_OK) return rcx;
        // one launch group per (binary level, pass kind) over a contiguous
        // range [a0, a1) of the table
        auto run = [&](uint32_t a0, uint32_t a1, uint32_t l, bool four) -> hipError_t {
            if (a1 <= a0) return hipSuccess;
            TaskRef<SortSeg> Rl{};
            Rl.A = a1 - a0;
            Rl.one = stab[a0];
            Rl.tab = ar.dev<SortSeg>(o_st) + a0;
            Rl.pre = ar.dev<uint32_t>(o_pm) + a0;
            Rl.base = pmerge[a0];
            MergeLaunch M;
            M.tasks = Rl;
            M.level = l;
            M.four_way = four;
            M.tiles = pmerge[a1] - pmerge[a0];
            for (uint32_t a = a0; a < a1; ++a) M.bytes += 16.0 * w * (double)stab[a].m;
            return launch_merge_pass(dt, pairs, M, ws, st);
        };
        for (uint32_t l = 0; l < maxL; ++l) {
            if (!by_parity) {
                uint32_t a1 = 0;
                while (a1 < T && stab[a1].L > l) ++a1;
                e = run(0, a1, l, false);
            } else {
                // the class whose passes start at l: even L at even l, odd L at odd l
                const uint32_t c0 = (l & 1u) ? E : 0, c_end = (l & 1u) ? T : E;
                uint32_t a1 = c0;
                while (a1 < c_end && stab[a1].L > l) ++a1;
                e = run(c0, a1, l, true);
                if (e == hipSuccess && l == 0) {
                    // 2-way first passes of the odd tasks
                    uint32_t b1 = E;
                    while (b1 < T && stab[b1].L > 0) ++b1;
                    e = run(E, b1, 0, false);
                }
            }
            if (e != hipSuccess) return hip_error(e, "merge pass");
        }
    }
    return QMS_OK;
}

int mom_pivot_of(int dt, const uint32_t *keys, uint64_t n, Workspace &ws, hipStream_t st,
                 uint64_t *pivot) {
    ArenaUse use(ws, st);
    Arena &ar = use.ar;
    PartSeg seg{(uint32_t *)keys, nullptr, 0, (uint32_t)n, 0, 0, 0, 0, kPivotMoM, 0};
    int rc = mom_pivots(dt, &seg, std::vector<uint32_t>{0}, ar, ws, st);
    if (rc != QMS_OK) return rc;
    uint64_t p = 0;
    hipError_t e = hipMemcpyAsync(&p, ws.meta + M_PIVOT, sizeof(p), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_error(e, "median-of-medians pivot readback");
    *pivot = p;
    return QMS_OK;
}

int sort_segments(int dt, bool pairs, const HostSeg *segs, size_t count, Workspace &ws,
                  hipStream_t st, bool log) {
    if (log) g_schedule.clear();
    const Tuning tune = current_tuning();
    std::vector<Seg> group;
    uint64_t group_keys = 0;
    auto flush = [&]() -> int {
        if (group.empty()) return QMS_OK;
        int rc = sort_group(dt, pairs, group, ws, st, log, tune);
        group.clear();
        group_keys = 0;
        return rc;
    };
    for (size_t i = 0; i < count; ++i) {
        const HostSeg &h = segs[i];
        if (h.n <= 1) continue;
        if (h.n > kMaxSortKeys) return set_error(QMS_ERR_UNSUPPORTED, "array too large");
        // an array of 2^32 keys or more is a group of its own
        if (group.size() == ws.caps.segs || group_keys + h.n >= kHugeRange) {
            int rc = flush();
            if (rc != QMS_OK) return rc;
        }
        group.push_back(Seg{h.keys, h.vals, 0, h.n, false});
        group_keys += h.n;
    }
    return flush();
}

}  // namespace qms
