// qms_basecase.hip -- the base case X of QuickMergeXsort on gfx950.
//
// Sec. "QuickMergeXsort": below a size threshold Mergesort hands a block to a
// sorting algorithm X and then moves the sorted block to the place Mergesort
// expects it.  Here X is a bitonic sorting network run by one 512-thread
// workgroup on a tile of kBaseTileKeys 32-bit keys (kBaseTilePairs key/payload
// pairs or 64-bit keys); the network stops at runs of the Mergesort's run
// width (X_THRESH) when that is smaller than the tile.  Each thread owns
// ITEMS consecutive elements in registers:
//   stride <  ITEMS            compare-exchange inside the thread's registers;
//   stride <  64 * ITEMS       partner in another lane of the same wave,
//                              exchanged with a wave shuffle (no barrier);
//   larger strides             partner in another wave, exchanged through LDS.
// Two modes:
//   in place  -- the sorted tile is written back where it was read;
//   swap      -- the sorted tile is written into the buffer region, and the
//                buffer elements found there move into the vacated source
//                cells (the swap-instead-of-move principle of Sec.
//                "QuickXsort and QuickMergesort"; Fig. 2's msort base case).
// Short tiles are padded with the largest key; for key/payload pairs each
// element carries the key above the element's index in the tile, so padding
// sorts after real keys and the payload is gathered through the index at the
// end.
#include <type_traits>

#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

// Cross-lane exchanges for lane masks 4 and 16 by ds_swizzle (1) or by
// VALU row moves / permlane swaps (0); build-time switches for measurements.
#ifndef QMS_SWIZZLE_4
#define QMS_SWIZZLE_4 1
#endif
#ifndef QMS_SWIZZLE_16
#define QMS_SWIZZLE_16 1
#endif

namespace qms {

// Element types of the network.  FLIP complements an element's order (the
// representation of a descending block, see stage 4); F64 marks elements
// that are positive normal doubles, whose order as doubles is their order as
// unsigned integers.
template <bool PAIRS, class K>
struct TileElem;
template <>
struct TileElem<false, uint32_t> {
    using E = uint32_t;
    static constexpr int ITEMS = kBaseTileKeys / kSortThreads;  // 32
    static constexpr E FLIP = ~0u;
    static constexpr bool F64 = false;
    __device__ static E make(uint32_t k, uint32_t) { return k; }
    __device__ static E pad(uint32_t) { return 0xFFFFFFFFu; }
    __device__ static uint32_t key(E x) { return x; }
    __device__ static uint32_t index(E) { return 0; }
};
// Keys in log order: the same layout, compared through the order's own
// comparison (no single-instruction min/max applies).
template <>
struct TileElem<false, LogKey> {
    using E = LogKey;
    static constexpr int ITEMS = kBaseTileKeys / kSortThreads;  // 32
    static constexpr E FLIP = LogKey{~0u};
    static constexpr bool F64 = false;
    __device__ static E make(uint32_t k, uint32_t) { return LogKey{k}; }
    __device__ static E pad(uint32_t) { return LogKey{0xFFFFFFFFu}; }
    __device__ static uint32_t key(E x) { return x.k; }
    __device__ static uint32_t index(E) { return 0; }
};
// Key/payload pairs: bit 52 (the lowest exponent bit of a double), the key in
// bits 13..44 and the element's index in the tile in bits 0..12.  Every
// element is then a positive normal double, so one v_min_f64 and one
// v_max_f64 settle an in-register compare-exchange (a 64-bit integer compare
// takes a compare and four selects); complementing bits 0..44 reverses the
// order and keeps the exponent bit.
template <>
struct TileElem<true, uint32_t> {
    using E = uint64_t;
    static constexpr int ITEMS = kBaseTilePairs / kSortThreads;  // 16
    static constexpr uint32_t IBITS = 13;
    static constexpr E FLIP = (1ull << (32 + IBITS)) - 1;
    static constexpr bool F64 = true;
    __device__ static E make(uint32_t k, uint32_t i) {
        return (1ull << 52) | ((uint64_t)k << IBITS) | i;
    }
    __device__ static E pad(uint32_t i) { return make(0xFFFFFFFFu, i); }
    __device__ static uint32_t key(E x) { return (uint32_t)(x >> IBITS); }
    __device__ static uint32_t index(E x) { return (uint32_t)x & ((1u << IBITS) - 1); }
};
static_assert(kBaseTilePairs <= (1u << TileElem<true, uint32_t>::IBITS), "tile index bits");
// 64-bit keys without payload: the element is the order-mapped key itself.
template <>
struct TileElem<false, uint64_t> {
    using E = uint64_t;
    static constexpr int ITEMS = kBaseTilePairs / kSortThreads;  // 16
    static constexpr E FLIP = ~0ull;
    static constexpr bool F64 = false;
    __device__ static E make(uint64_t k, uint32_t) { return k; }
    __device__ static E pad(uint32_t) { return ~0ull; }
    __device__ static uint64_t key(E x) { return x; }
    __device__ static uint32_t index(E) { return 0; }
};

// 64-bit keys with payloads: the element is the order-mapped key and the
// element's index in the tile, compared as one (key, index) value, so that no
// two elements tie (the exchanges below keep each element exactly once) and
// the payload is gathered through the index at the end.  Complementing both
// parts reverses the order.
struct WideIdx {
    uint64_t k;
    uint32_t i, pad;
};
__device__ __forceinline__ bool operator<(const WideIdx &a, const WideIdx &b) {
    return a.k < b.k || (a.k == b.k && a.i < b.i);
}
__device__ __forceinline__ WideIdx operator^(const WideIdx &a, const WideIdx &b) {
    return WideIdx{a.k ^ b.k, a.i ^ b.i, 0};
}
__device__ __forceinline__ WideIdx &operator^=(WideIdx &a, const WideIdx &b) {
    a = a ^ b;
    return a;
}
template <>
struct TileElem<true, uint64_t> {
    using E = WideIdx;
    static constexpr int ITEMS = kBaseTileWidePairs / kSortThreads;  // 4
    static constexpr uint32_t IBITS = 31 - __builtin_clz(kBaseTileWidePairs);  // log2 of the tile
    static constexpr E FLIP = WideIdx{~0ull, (1u << IBITS) - 1, 0};
    static constexpr bool F64 = false;
    __device__ static E make(uint64_t k, uint32_t i) { return WideIdx{k, i, 0}; }
    __device__ static E pad(uint32_t i) { return WideIdx{~0ull, i, 0}; }
    __device__ static uint64_t key(E x) { return x.k; }
    __device__ static uint32_t index(E x) { return x.i; }
};
static_assert(kBaseTileWidePairs <= (1u << TileElem<true, uint64_t>::IBITS), "tile index bits");

template <class E>
__device__ __forceinline__ void cmpx(E &a, E &b, bool asc) {
    const E lo = a < b ? a : b;
    const E hi = a < b ? b : a;
    a = asc ? lo : hi;
    b = asc ? hi : lo;
}

// The same for elements that are positive normal doubles (F64 above): the
// double min and max of the bit patterns, written as instructions so that
// no canonicalisation of the operands is added (both return one of the two
// inputs unchanged for such values).
__device__ __forceinline__ void cmpx_f64(uint64_t &a, uint64_t &b, bool asc) {
    uint64_t lo, hi;
    asm("v_min_f64 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
    asm("v_max_f64 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
    a = asc ? lo : hi;
    b = asc ? hi : lo;
}
template <class TE, class E>
__device__ __forceinline__ void cmpx_elem(E &a, E &b, bool asc) {
    if constexpr (TE::F64) {
        cmpx_f64(a, b, asc);
    } else {
        cmpx(a, b, asc);
    }
}

// One side of a compare-exchange whose partner value is y: the smaller of the
// two if keep_min, else the larger.  `bound` is 0 when keep_min and all ones
// otherwise; for 32-bit elements the median of (x, y, bound) is then exactly
// the kept value, a single v_med3_u32.
__device__ __forceinline__ uint32_t keep_side(uint32_t x, uint32_t y, bool, uint32_t bound) {
    return median3(x, y, bound);
}
__device__ __forceinline__ uint64_t keep_side(uint64_t x, uint64_t y, bool keep_min, uint64_t) {
    // x stays when it is on the kept side of y (ties keep either: equal values)
    return (x < y) == keep_min ? x : y;
}
__device__ __forceinline__ WideIdx keep_side(WideIdx x, WideIdx y, bool keep_min, WideIdx) {
    return (x < y) == keep_min ? x : y;  // elements never tie
}
__device__ __forceinline__ LogKey keep_side(LogKey x, LogKey y, bool keep_min, LogKey) {
    return (x < y) == keep_min ? x : y;
}

// The partner lane's element (xor of the lane index).
__device__ __forceinline__ uint32_t shfl_xor_elem(uint32_t v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ uint64_t shfl_xor_elem(uint64_t v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ LogKey shfl_xor_elem(LogKey v, int m) {
    return LogKey{(uint32_t)__shfl_xor((int)v.k, m, kWave)};
}
__device__ __forceinline__ WideIdx shfl_xor_elem(WideIdx v, int m) {
    return WideIdx{__shfl_xor(v.k, m, kWave), (uint32_t)__shfl_xor((int)v.i, m, kWave), 0};
}

// Cross-lane compare-exchange steps of 32-bit elements without the LDS pipe
// (the ds_bpermute of a generic shuffle occupies it, and it is what limits
// the base case): lane masks 1, 2 and 8 are single DPP row moves (quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], row_ror:8 -- a rotation by half a row of 16
// is the xor-8 partner), mask 4 takes row_ror:4 (lane i - 4) or row_ror:12
// (lane i + 4) by the lane's bit 2.  Masks 16 and 32 use the CDNA4 permlane
// swaps on register pairs: v_permlane16_swap / v_permlane32_swap exchange
// rows (halves) between two registers so that both elements of each pair of
// either register sit in one lane, one min/max settles them, and a second
// swap restores the layout.  Every block is ascending here (complemented
// representation), so the lower lane keeps the smaller element.
template <int LM>
__device__ __forceinline__ uint32_t dpp_partner(uint32_t v, uint32_t lane) {
    if constexpr (LM == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (LM == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (LM == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
    } else if constexpr (LM == 4 && QMS_SWIZZLE_4) {
        // ds_swizzle in bit mode, xor mask 4 (one LDS-pipe op, no memory)
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
    } else if constexpr (LM == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);  // xor mask 16
    } else {
        static_assert(LM == 4, "lane mask");
        const uint32_t from_below = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, false);
        const uint32_t from_above = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12C, 0xF, 0xF, false);
        return (lane & 4) ? from_below : from_above;
    }
}

template <int LM, int ITEMS>
__device__ __forceinline__ void lane_step_u32(uint32_t (&r)[ITEMS], uint32_t lane) {
    if constexpr (LM <= 8 || (LM == 16 && QMS_SWIZZLE_16)) {
        const uint32_t bound = (lane & LM) ? ~0u : 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) r[i] = median3(r[i], dpp_partner<LM>(r[i], lane), bound);
    } else {
        static_assert(ITEMS % 2 == 0, "register pairs");
#pragma unroll
        for (int i = 0; i < ITEMS; i += 2) {
            const auto t = LM == 32 ? __builtin_amdgcn_permlane32_swap(r[i], r[i + 1], false, false)
                                    : __builtin_amdgcn_permlane16_swap(r[i], r[i + 1], false, false);
            const uint32_t a = t[0], b = t[1];
            const auto u = LM == 32
                               ? __builtin_amdgcn_permlane32_swap(min(a, b), max(a, b), false, false)
                               : __builtin_amdgcn_permlane16_swap(min(a, b), max(a, b), false, false);
            r[i] = u[0];
            r[i + 1] = u[1];
        }
    }
}

// The partner value of a 32-bit register at lane mask LM, for any mask: DPP
// and swizzles as above, and for mask 32 one permlane32 swap of the register
// with itself (it returns both halves broadcast: the lower half takes the
// copy of the upper half and vice versa).
template <int LM>
__device__ __forceinline__ uint32_t lane_partner(uint32_t v, uint32_t lane) {
    if constexpr (LM == 32) {
        const auto t = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? (uint32_t)t[0] : (uint32_t)t[1];
    } else {
        return dpp_partner<LM>(v, lane);
    }
}

// Key/payload elements (64 bits: key, then index): both halves travel to the
// partner lane, and one 64-bit comparison picks the kept element.
template <int LM, int ITEMS>
__device__ __forceinline__ void lane_step_u64(uint64_t (&r)[ITEMS], uint32_t lane) {
    const bool keep_min = (lane & LM) == 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t lo = lane_partner<LM>((uint32_t)r[i], lane);
        const uint32_t hi = lane_partner<LM>((uint32_t)(r[i] >> 32), lane);
        r[i] = keep_side(r[i], ((uint64_t)hi << 32) | lo, keep_min, 0);
    }
}

// Lane masks 16 and 32 for key/payload elements: as in lane_step_u32, permlane
// swaps of register pairs (one per 32-bit half) bring both elements of each
// compare pair into one lane, one ascending compare-exchange settles them
// (double min/max for the F64 encoding), and the same swaps restore the
// layout.  Every block is ascending here, so the lower lane keeps the
// smaller element.
template <class TE, int LM, int ITEMS>
__device__ __forceinline__ void lane_step_swap64(uint64_t (&r)[ITEMS]) {
    static_assert(ITEMS % 2 == 0 && (LM == 16 || LM == 32), "register pairs");
    auto swap = [](uint32_t x, uint32_t y) {
        const auto t = LM == 32 ? __builtin_amdgcn_permlane32_swap(x, y, false, false)
                                : __builtin_amdgcn_permlane16_swap(x, y, false, false);
        return t;
    };
#pragma unroll
    for (int i = 0; i < ITEMS; i += 2) {
        const auto tl = swap((uint32_t)r[i], (uint32_t)r[i + 1]);
        const auto th = swap((uint32_t)(r[i] >> 32), (uint32_t)(r[i + 1] >> 32));
        uint64_t a = ((uint64_t)(uint32_t)th[0] << 32) | (uint32_t)tl[0];
        uint64_t b = ((uint64_t)(uint32_t)th[1] << 32) | (uint32_t)tl[1];
        cmpx_elem<TE>(a, b, true);
        const auto ul = swap((uint32_t)a, (uint32_t)b);
        const auto uh = swap((uint32_t)(a >> 32), (uint32_t)(b >> 32));
        r[i] = ((uint64_t)(uint32_t)uh[0] << 32) | (uint32_t)ul[0];
        r[i + 1] = ((uint64_t)(uint32_t)uh[1] << 32) | (uint32_t)ul[1];
    }
}

// Lane masks 1, 2, 4 and 8 for the F64 encoding: during the step at mask LM
// the lanes with bit LM set hold their elements negated (sign bit set; sign
// tracks what a lane's elements carry), so one double min of the own element
// and the negated partner keeps the smaller element in the lower lane and the
// negated larger one in the upper lane.  The caller clears the signs after
// the last step.
template <int LM, int ITEMS>
__device__ __forceinline__ void lane_step_neg64(uint64_t (&r)[ITEMS], uint32_t lane,
                                                uint32_t &sign) {
    const uint32_t want = (lane & LM) ? 0x80000000u : 0u;
    const uint64_t flip = (uint64_t)(want ^ sign) << 32;
    sign = want;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        r[i] ^= flip;
        const uint32_t lo = dpp_partner<LM>((uint32_t)r[i], lane);
        const uint32_t hi = dpp_partner<LM>((uint32_t)(r[i] >> 32), lane);
        const uint64_t y = ((uint64_t)hi << 32) | lo;
        uint64_t m;
        asm("v_min_f64 %0, %1, -%2" : "=v"(m) : "v"(r[i]), "v"(y));
        r[i] = m;
    }
}

// Padded LDS index of element e of the tile in natural order: one spare slot
// every ITEMS slots, so that thread t reading its ITEMS consecutive elements
// and lanes reading consecutive elements both avoid bank conflicts.
template <int ITEMS>
__device__ __forceinline__ uint32_t nat_idx(uint32_t e) {
    return e + e / ITEMS;
}

// Sort one tile.  sk/sv: the tile's cells in the source region, dk/dv: in
// the destination region (equal in place); len <= the tile size.
// MERGE_ONLY: the tile holds a bitonic sequence (padded past len with the
// largest key); only the last stage's half-cleaners run (in place, no
// samples).
template <class O, bool PAIRS, bool MERGE_ONLY = false>
__device__ __forceinline__ void tile_sort_block(typename O::K *sk, uint32_t *sv,
                                                typename O::K *dk, uint32_t *dv, uint32_t len,
                                                uint32_t run, bool swap,
                                                typename O::K *samples) {
    using K = typename O::K;
    using TE = TileElem<PAIRS, typename O::NetKey>;
    using E = typename TE::E;
    constexpr int ITEMS = TE::ITEMS;
    constexpr int NT = kSortThreads;
    constexpr uint32_t T = (uint32_t)NT * ITEMS;
    __shared__ E s[T + T / ITEMS];
    __shared__ uint32_t sp[PAIRS ? T : 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);

    // A tile of len < T keys: its keys and padding sorted as the first P
    // positions (P the power of two at or above len, at least ITEMS) are the
    // sorted keys, so the network stops at runs of P (then all ascending) and
    // waves wholly past P skip the compare-exchanges (they still take part in
    // the barriers).  The last stage's half-cleaners of MERGE_ONLY start at
    // P / 2: a partner at P or beyond is padding and never moves.
    const uint32_t P = len >= T ? T : len <= (uint32_t)ITEMS ? (uint32_t)ITEMS
                                                             : 2u << (31 - __builtin_clz(len - 1));

    // 1. coalesced loads (clamped indices, all issued together); in swap mode
    //    each thread then moves the buffer elements of exactly the source
    //    cells it has read into those cells
    {
        K kv[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) kv[r] = ldg(sk + min((uint32_t)r * NT + tid, len - 1));
        if constexpr (MERGE_ONLY) {
            // As loaded, register r of a thread holds position r NT + tid, so
            // the last stage's half-cleaners with strides of NT or more pair
            // registers of one thread: they run here, before the elements go
            // through LDS, ascending as every step of that stage (a partner
            // past len is padding, which compares above every key and so
            // never moves)
            E x[ITEMS];
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t e = (uint32_t)r * NT + tid;
                x[r] = e < len ? TE::make(O::ord(kv[r]), e) : TE::pad(e);
            }
#pragma unroll
            for (int q = ITEMS / 2; q >= 1; q >>= 1) {
                if ((uint32_t)q * NT * 2 > P) continue;  // stride q NT, from P / 2 down
#pragma unroll
                for (int r = 0; r < ITEMS; ++r)
                    if ((r & q) == 0) cmpx_elem<TE>(x[r], x[r | q], true);
            }
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) s[nat_idx<ITEMS>((uint32_t)r * NT + tid)] = x[r];
        } else {
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t e = (uint32_t)r * NT + tid;
                s[nat_idx<ITEMS>(e)] = e < len ? TE::make(O::ord(kv[r]), e) : TE::pad(e);
            }
        }
        if constexpr (PAIRS) {
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) kv[r] = ldg(sv + min((uint32_t)r * NT + tid, len - 1));
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t e = (uint32_t)r * NT + tid;
                if (e < len) sp[e] = (uint32_t)kv[r];
            }
        }
        if (swap) {
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) kv[r] = ldg(dk + min((uint32_t)r * NT + tid, len - 1));
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t e = (uint32_t)r * NT + tid;
                if (e < len) stg(sk + e, kv[r]);
            }
            if constexpr (PAIRS) {
#pragma unroll
                for (int r = 0; r < ITEMS; ++r)
                    kv[r] = ldg(dv + min((uint32_t)r * NT + tid, len - 1));
#pragma unroll
                for (int r = 0; r < ITEMS; ++r) {
                    const uint32_t e = (uint32_t)r * NT + tid;
                    if (e < len) stg(sv + e, (uint32_t)kv[r]);
                }
            }
        }
    }
    __syncthreads();

    // 2. ITEMS consecutive elements per thread
    E r[ITEMS];
    const uint32_t base = tid * ITEMS;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) r[i] = s[nat_idx<ITEMS>(base + i)];

    const uint32_t top = MERGE_ONLY ? run : (run < P ? run : P);
    const bool wact = (tid & ~(uint32_t)(kWave - 1)) * (uint32_t)ITEMS < P;

    // 3. runs of ITEMS / 2 in registers, alternating direction (fixed per
    //    register, since base is a multiple of ITEMS)
#pragma unroll
    for (int k = 2; k < (MERGE_ONLY ? 2 : ITEMS); k <<= 1) {
        if (!wact) break;
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int l = i ^ j;
                if (l > i) cmpx_elem<TE>(r[i], r[l], ((base + i) & k) == 0);
            }
        }
    }

    // 4. merge stages from k = ITEMS up to the run width (the whole tile, or
    //    QuickMergeXsort's X_THRESH when the Mergesort stops earlier), where
    //    the direction of a block depends on the thread.  During merge stage
    //    k a thread's keys are held complemented when its k-block sorts
    //    descending (complementing reverses the unsigned order), so every
    //    compare-exchange below is an ascending one; the representation
    //    changes only between stages.  At the last stage every block ascends
    //    and the keys are plain again: the tile holds T / run sorted runs.
    E cur_mask = E{};
    for (uint32_t k = MERGE_ONLY ? run : ITEMS; k <= top; k <<= 1) {
        const E mask = (k == top || (base & k) == 0) ? E{} : TE::FLIP;
        const E flip = mask ^ cur_mask;
        cur_mask = mask;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) r[i] ^= flip;
        const bool asc = true;
        uint32_t j = (k < P ? k : P) >> 1;
        // MERGE_ONLY: the strides of NT and more ran before the transposition
        if constexpr (MERGE_ONLY) j = j < (uint32_t)NT / 2 ? j : (uint32_t)NT / 2;
        // partners in other waves: exchange through LDS (partners of a
        // thread before P lie before P)
        for (; j >= (uint32_t)kWave * ITEMS; j >>= 1) {
            __syncthreads();  // previous users of s are done
            if (wact) {
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) s[(uint32_t)i * NT + tid] = r[i];
            }
            __syncthreads();
            if (!wact) continue;
            const uint32_t pt = tid ^ (j / ITEMS);
            const bool lower = (tid & (j / ITEMS)) == 0;
            const bool keep_min = asc == lower;
            const E bound = keep_min ? E{} : TE::FLIP;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                r[i] = keep_side(r[i], s[(uint32_t)i * NT + pt], keep_min, bound);
        }
        if (!wact) continue;
        // partners in other lanes of the wave
        if constexpr (std::is_same_v<E, uint32_t>) {
            switch (j / ITEMS) {  // lane masks j / ITEMS down to 1
            case 32:
                lane_step_u32<32>(r, lane);
                [[fallthrough]];
            case 16:
                lane_step_u32<16>(r, lane);
                [[fallthrough]];
            case 8:
                lane_step_u32<8>(r, lane);
                [[fallthrough]];
            case 4:
                lane_step_u32<4>(r, lane);
                [[fallthrough]];
            case 2:
                lane_step_u32<2>(r, lane);
                [[fallthrough]];
            case 1:
                lane_step_u32<1>(r, lane);
                [[fallthrough]];
            default:
                break;
            }
            j = ITEMS / 2;
        } else {
            // pairs take the register-pair swaps at masks 16 and 32 and the
            // signed minimum below; for 64-bit keys (an integer compare and
            // four selects per pair) the partner exchange at every mask
            // measured slightly faster than the swaps
            if constexpr (!std::is_same_v<E, uint64_t>) {
                // (key, index) elements: the shuffle steps below, every mask
            } else if constexpr (TE::F64) {
                const uint32_t lm0 = j / ITEMS;
                if (lm0 >= 32) lane_step_swap64<TE, 32>(r);
                if (lm0 >= 16) lane_step_swap64<TE, 16>(r);
                uint32_t sign = 0;
                if (lm0 >= 8) lane_step_neg64<8>(r, lane, sign);
                if (lm0 >= 4) lane_step_neg64<4>(r, lane, sign);
                if (lm0 >= 2) lane_step_neg64<2>(r, lane, sign);
                if (lm0 >= 1) lane_step_neg64<1>(r, lane, sign);
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) r[i] ^= (uint64_t)sign << 32;
                j = ITEMS / 2;
            } else {
                switch (j / ITEMS) {
                case 32:
                    lane_step_u64<32>(r, lane);
                    [[fallthrough]];
                case 16:
                    lane_step_u64<16>(r, lane);
                    [[fallthrough]];
                case 8:
                    lane_step_u64<8>(r, lane);
                    [[fallthrough]];
                case 4:
                    lane_step_u64<4>(r, lane);
                    [[fallthrough]];
                case 2:
                    lane_step_u64<2>(r, lane);
                    [[fallthrough]];
                case 1:
                    lane_step_u64<1>(r, lane);
                    [[fallthrough]];
                default:
                    break;
                }
                j = ITEMS / 2;
            }
        }
        for (; j >= (uint32_t)ITEMS; j >>= 1) {
            const uint32_t lm = j / ITEMS;
            const bool lower = (lane & lm) == 0;
            const bool keep_min = asc == lower;
            const E bound = keep_min ? E{} : TE::FLIP;
            // all exchanges of the stage first, so that they overlap
            E y[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) y[i] = shfl_xor_elem(r[i], (int)lm);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) r[i] = keep_side(r[i], y[i], keep_min, bound);
        }
        // partners in the thread's own registers
#pragma unroll
        for (int jj = ITEMS / 2; jj >= 1; jj >>= 1) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int l = i ^ jj;
                if (l > i) cmpx_elem<TE>(r[i], r[l], asc);
            }
        }
    }

    // 5. back to natural order in LDS, coalesced stores; every
    //    kSampleStride-th key (order-mapped) is a sample the first merge
    //    level searches
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s[nat_idx<ITEMS>(base + i)] = r[i];
    __syncthreads();
    static_assert((uint32_t)(NT * ITEMS) / kSampleStride <= (uint32_t)NT, "one sample per thread");
    if (!MERGE_ONLY && samples != nullptr && tid * kSampleStride < len)
        stg(samples + tid, TE::key(s[nat_idx<ITEMS>(tid * kSampleStride)]));
#pragma unroll 8
    for (int q = 0; q < ITEMS; ++q) {
        const uint32_t e = (uint32_t)q * NT + tid;
        if (e < len) {
            const E x = s[nat_idx<ITEMS>(e)];
            stg(dk + e, O::unord(TE::key(x)));
            if constexpr (PAIRS) stg(dv + e, sp[TE::index(x)]);
        }
    }
}

// One workgroup per base tile of every Mergesort task in the table.
// Samples: one key per kSampleStride keys of each task, kSamplesPerTile
// entries per merge split tile of the task (the base tile is a multiple of
// kMergeTile).  64-bit keys use
// the 8,192-element tile of key/payload pairs.
template <class O, bool PAIRS>
__device__ __forceinline__ void tile_sort_item(TaskRef<SortSeg> tasks, uint32_t item,
                                               typename O::K *samples) {
    using K = typename O::K;
    constexpr uint32_t T = base_tile_of(PAIRS, sizeof(K) == 8);
    uint32_t t, a;
    const SortSeg g = task_of(tasks, item, &t, &a);
    const uint32_t t0 = t * T;
    if (t0 >= g.m) return;
    const uint32_t len = min(T, g.m - t0);
    const bool swap = (merge_passes(g.L, g.two_way != 0) & 1u) != 0;
    // runs of g.w0 keys (a power of two in [kMergeTile, T]; clamped so that
    // a malformed task still runs a valid network)
    const uint32_t run = g.w0 >= T ? T : (g.w0 <= (uint32_t)kMergeTile ? (uint32_t)kMergeTile : g.w0);
    K *sk = (K *)g.keys + t0;
    K *dk = (K *)(swap ? g.bkeys : g.keys) + t0;
    uint32_t *sv = PAIRS ? g.vals + t0 : nullptr;
    uint32_t *dv = PAIRS ? (swap ? g.bvals : g.vals) + t0 : nullptr;
    // run samples for the first merge pass (none for a range sorted in place)
    tile_sort_block<O, PAIRS>(sk, sv, dk, dv, len, run, swap,
                              g.L ? samples + (uint64_t)g.split_off * kSamplesPerTile +
                                        t0 / kSampleStride
                                  : nullptr);
}
template <class O, bool PAIRS, bool LOOP>
__global__ __launch_bounds__(kSortThreads) void k_tile_sort(TaskRef<SortSeg> tasks, uint32_t first,
                                                            typename O::K *samples) {
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) tile_sort_item<O, PAIRS>(tasks, item, samples);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            tile_sort_item<O, PAIRS>(tasks, item, samples);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}

// tiles: one workgroup each (host-sized), or with tasks.dyn the estimate of
// a device-sized launch, followed by `overflow` looping workgroups for the
// tiles beyond it.
template <class O, bool PAIRS>
static hipError_t tile_sort_t(const TaskRef<SortSeg> &tasks, uint32_t tiles, uint32_t overflow,
                              double bytes, const Workspace &ws, hipStream_t st) {
    if (tiles == 0 && overflow == 0) return hipSuccess;
    ProfScope prof(st, K_TILE_SORT, bytes);
    using K = typename O::K;
    if (tiles)
        hipLaunchKernelGGL((k_tile_sort<O, PAIRS, false>), dim3(tiles), dim3(kSortThreads), 0, st,
                           tasks, 0u, (K *)ws.samples[0]);
    if (overflow)
        hipLaunchKernelGGL((k_tile_sort<O, PAIRS, true>), dim3(overflow), dim3(kSortThreads), 0,
                           st, tasks, tiles, (K *)ws.samples[0]);
    return hipGetLastError();
}

// The in-tile steps of the loop's final network (qms_bitonic.hip): every
// tile of T keys of the tasks holds a bitonic sequence, and the last stage
// of the base case's network (its half-cleaners) sorts it in place.
template <class O, bool PAIRS>
__global__ __launch_bounds__(kSortThreads) void k_tile_merge(TaskRef<SortSeg> tasks,
                                                             uint32_t items) {
    using K = typename O::K;
    constexpr uint32_t T = base_tile_of(PAIRS, sizeof(K) == 8);
    // one workgroup per tile (host-sized), or the plan's count of tiles
    // taken in grid-stride order
    const uint32_t W = work_total(tasks, items);
    for (uint32_t it = blockIdx.x; it < W; it += gridDim.x) {
        uint32_t t, a;
        const SortSeg g = task_of(tasks, it, &t, &a);
        const uint64_t t0 = (uint64_t)t * T;
        const uint32_t len = (uint32_t)(g.m - t0 < T ? g.m - t0 : T);
        K *k = (K *)g.keys + t0;
        uint32_t *v = PAIRS ? g.vals + t0 : nullptr;
        tile_sort_block<O, PAIRS, true>(k, v, k, v, len, T, false, nullptr);
        __syncthreads();  // the LDS is reused by the next tile
    }
}

hipError_t launch_tile_merge(int dt, bool pairs, const TaskRef<SortSeg> &tasks, uint32_t items,
                             hipStream_t st) {
    if (items == 0) return hipSuccess;
    const dim3 g(items), b(kSortThreads);
    switch (dt) {
    case 0:
        if (pairs) hipLaunchKernelGGL((k_tile_merge<OrdU32, true>), g, b, 0, st, tasks, items);
        else hipLaunchKernelGGL((k_tile_merge<OrdU32, false>), g, b, 0, st, tasks, items);
        break;
    case 1:
        if (pairs) hipLaunchKernelGGL((k_tile_merge<OrdF32, true>), g, b, 0, st, tasks, items);
        else hipLaunchKernelGGL((k_tile_merge<OrdF32, false>), g, b, 0, st, tasks, items);
        break;
    case 2:
        if (pairs) hipLaunchKernelGGL((k_tile_merge<OrdU64, true>), g, b, 0, st, tasks, items);
        else hipLaunchKernelGGL((k_tile_merge<OrdU64, false>), g, b, 0, st, tasks, items);
        break;
    case 3:
        if (pairs) hipLaunchKernelGGL((k_tile_merge<OrdF64, true>), g, b, 0, st, tasks, items);
        else hipLaunchKernelGGL((k_tile_merge<OrdF64, false>), g, b, 0, st, tasks, items);
        break;
    case 4:
        if (pairs) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_tile_merge<OrdLogU32, false>), g, b, 0, st, tasks, items);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tile_sort(int dt, bool pairs, const TaskRef<SortSeg> &tasks, uint32_t tiles,
                            uint32_t overflow, double bytes, const Workspace &ws,
                            hipStream_t st) {
    switch (dt) {
    case 0:
        return pairs ? tile_sort_t<OrdU32, true>(tasks, tiles, overflow, bytes, ws, st)
                     : tile_sort_t<OrdU32, false>(tasks, tiles, overflow, bytes, ws, st);
    case 1:
        return pairs ? tile_sort_t<OrdF32, true>(tasks, tiles, overflow, bytes, ws, st)
                     : tile_sort_t<OrdF32, false>(tasks, tiles, overflow, bytes, ws, st);
    case 2:
        return pairs ? tile_sort_t<OrdU64, true>(tasks, tiles, overflow, bytes, ws, st)
                     : tile_sort_t<OrdU64, false>(tasks, tiles, overflow, bytes, ws, st);
    case 3:
        return pairs ? tile_sort_t<OrdF64, true>(tasks, tiles, overflow, bytes, ws, st)
                     : tile_sort_t<OrdF64, false>(tasks, tiles, overflow, bytes, ws, st);
    case 4:
        return pairs ? hipErrorInvalidValue
                     : tile_sort_t<OrdLogU32, false>(tasks, tiles, overflow, bytes, ws, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace qms
