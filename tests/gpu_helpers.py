"""Helpers for GPU tests: host/device transfer and property checks that hold
at any size (sortedness, an order-independent multiset hash, the pairs
invariants).  Plain torch on the device; nothing here sorts."""
import numpy as np
import torch

_M64 = (1 << 64) - 1


def _s64(c: int) -> int:
    c &= _M64
    return c - (1 << 64) if c >= 1 << 63 else c


_C1, _C2, _C3, _C4 = (_s64(0x9E3779B97F4A7C15), _s64(0xBF58476D1CE4E5B9),
                      _s64(0x94D049BB133111EB), _s64(0xD6E8FEB86659FD93))


def to_device(a: np.ndarray) -> torch.Tensor:
    if a.dtype == np.float32:
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    assert a.dtype == np.uint32
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    a = t.cpu().numpy()
    return a if a.dtype == np.float32 else a.view(np.uint32)


def as_u64(t: torch.Tensor) -> torch.Tensor:
    """32-bit words as non-negative int64 (bit pattern, any dtype)."""
    return t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF


def order_key(t: torch.Tensor) -> torch.Tensor:
    """int64 keys whose numeric order is the sort order: unsigned for
    integer tensors, IEEE total order (sign-magnitude) for float32."""
    u = as_u64(t)
    if t.dtype != torch.float32:
        return u
    neg = u >= (1 << 31)
    return torch.where(neg, -(u - (1 << 31)) - 1, u)


def is_sorted(t: torch.Tensor) -> bool:
    if t.numel() < 2:
        return True
    k = order_key(t)
    return bool((k[1:] >= k[:-1]).all().item())


def multiset_hash(t: torch.Tensor, payload: torch.Tensor = None) -> tuple:
    """Two order-independent 64-bit sums of mixed 32-bit words (or of
    (key, payload) pairs).  Equal multisets give equal hashes."""
    x = as_u64(t)
    if payload is not None:
        x = x * (1 << 32) + as_u64(payload)
    out = []
    for a, b in ((_C1, _C2), (_C3, _C4)):
        h = x * a
        h = h ^ ((h >> 29) & ((1 << 35) - 1))
        h = h * b
        h = h ^ ((h >> 32) & 0xFFFFFFFF)
        out.append(int(h.sum().item()))
    return tuple(out)


def check_pairs_exact(keys_in: torch.Tensor, keys_out: torch.Tensor, vals_out: torch.Tensor):
    """Payload = original index: keys sorted, payloads a permutation of
    [0, n), and keys_out[i] == keys_in[vals_out[i]] for every i."""
    n = keys_in.numel()
    assert is_sorted(keys_out)
    v = as_u64(vals_out)
    assert int(v.min().item()) >= 0 and int(v.max().item()) < n
    seen = torch.zeros(n, dtype=torch.int32, device=keys_in.device)
    seen.index_fill_(0, v, 1)
    assert int(seen.sum().item()) == n
    assert bool((as_u64(keys_in)[v] == as_u64(keys_out)).all().item())


def segment_ids(offsets: torch.Tensor, n: int) -> torch.Tensor:
    """Segment index of every position, from offsets (device int64)."""
    lens = offsets[1:] - offsets[:-1]
    return torch.repeat_interleave(torch.arange(lens.numel(), device=offsets.device), lens,
                                   output_size=n)


def segments_sorted(t: torch.Tensor, offsets: torch.Tensor) -> bool:
    """Every segment non-decreasing (boundaries between segments ignored)."""
    n = t.numel()
    if n < 2:
        return True
    k = order_key(t)
    ok = k[1:] >= k[:-1]
    starts = offsets[1:-1]
    starts = starts[(starts > 0) & (starts < n)]
    ok[starts - 1] = True
    return bool(ok.all().item())


def segment_multiset_hash(t: torch.Tensor, seg: torch.Tensor) -> tuple:
    """Order-independent hash of the (segment, word) multiset: equal only if
    every segment kept its own multiset (up to hash collisions)."""
    x = as_u64(t) ^ (seg.to(torch.int64) * _C3)
    out = []
    for a, b in ((_C1, _C2), (_C2, _C4)):
        h = x * a
        h = h ^ ((h >> 29) & ((1 << 35) - 1))
        h = h * b
        h = h ^ ((h >> 32) & 0xFFFFFFFF)
        out.append(int(h.sum().item()))
    return tuple(out)
