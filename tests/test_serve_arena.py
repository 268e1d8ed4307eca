"""CPU checks of the byte-budget admission pieces: the arena allocator of the
serving backend (first fit, 256-byte alignment, merging of freed ranges, no
overlap) and the batch plan-capacity calls of the C ABI (host-only)."""
import numpy as np
import pytest

import paper_2308_00763_amd as pf
from paper_2308_00763_amd.serve import ByteArena


def _check_invariants(a: ByteArena, live):
    # free ranges sorted, disjoint, not adjacent (merged), 256-aligned, in bounds
    for i in range(len(a.starts)):
        assert a.starts[i] % 256 == 0 and a.lens[i] % 256 == 0 and a.lens[i] > 0
        assert a.starts[i] + a.lens[i] <= a.size
        if i:
            assert a.starts[i - 1] + a.lens[i - 1] < a.starts[i]
    spans = sorted((off, ByteArena.rounded(n)) for off, n in live.values())
    for (o1, l1), (o2, _) in zip(spans, spans[1:]):
        assert o1 + l1 <= o2
    for off, ln in spans:  # no live range overlaps a free one
        for s, l in zip(a.starts, a.lens):
            assert off + ln <= s or s + l <= off
    assert a.used == sum(l for _, l in spans)
    assert a.used + sum(a.lens) == a.size


def test_alloc_release_merge():
    a = ByteArena(10 * 256 + 17)
    assert a.size == 2560
    x = a.alloc(1)
    y = a.alloc(256)
    z = a.alloc(257)
    assert (x, y, z) == (0, 256, 512)
    assert a.used == 1024 and a.largest_free() == 1536
    assert a.alloc(1537) is None
    a.release(y, 256)
    assert a.starts == [256, 1024] and a.lens == [256, 1536]
    a.release(x, 1)        # merges with [256, 512)
    assert a.starts == [0, 1024] and a.lens == [512, 1536]
    a.release(z, 257)      # merges both sides: one free range
    assert a.starts == [0] and a.lens == [2560] and a.used == 0
    assert a.high == 1024


def test_double_release_is_refused():
    a = ByteArena(4096)
    x = a.alloc(300)
    a.release(x, 300)
    with pytest.raises(ValueError):
        a.release(x, 300)


def test_random_workload_keeps_invariants_and_fits_what_first_fit_should():
    rng = np.random.default_rng(3)
    a = ByteArena(1 << 22)
    live = {}
    nxt = 0
    for step in range(4000):
        if live and rng.random() < 0.45:
            k = list(live)[int(rng.integers(len(live)))]
            off, n = live.pop(k)
            a.release(off, n)
        else:
            n = int(np.exp(rng.uniform(np.log(100), np.log(300_000))))
            off = a.alloc(n)
            if off is None:
                # first fit fails only when no free range holds the request
                assert a.largest_free() < ByteArena.rounded(n)
            else:
                live[nxt] = (off, n)
                nxt += 1
        if step % 97 == 0:
            _check_invariants(a, live)
    _check_invariants(a, live)
    for off, n in live.values():
        a.release(off, n)
    assert a.starts == [0] and a.lens == [a.size] and a.used == 0


def test_batch_plan_capacity_sizes():
    ps = [pf.make_params(1, 64, 64, "f16") for _ in range(8)]
    base = pf.pf_batch_workspace_bytes(ps)
    assert pf.pf_batch_workspace_bytes_cap(ps, 0) == base
    assert pf.pf_batch_workspace_bytes_cap(ps, 8) == base       # the members' own 8 tiles
    big = pf.pf_batch_workspace_bytes_cap(ps, 100_000)
    # 16 bytes of plan per tile of capacity (tile map and pass-A list, eager and captured)
    # (four 256-byte aligned sections: their padding moves by less than 256 each)
    assert abs((big - base) - 16 * (100_000 - 8)) <= 4 * 256
    for bad in (-1, 1 << 31):
        with pytest.raises(pf.PfError) as ei:
            pf.pf_batch_workspace_bytes_cap(ps, bad)
        assert ei.value.code == pf.PF_ERR_INVALID_ARG


def test_rebind_argument_errors_without_a_device():
    L = pf.lib()
    p = pf.make_params(1000, 64, 64, "f16")
    import ctypes
    assert L.pf_batch_rebind(None, 0, ctypes.byref(p), None, 0) == pf.PF_ERR_INVALID_ARG
