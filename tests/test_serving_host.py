"""Host logic of the serving loop (CPU only): the per-client output ring.

Every admitted request takes a slice of its client's output ring; slices are freed in any
order when their launch completes, and space is reclaimed in allocation order. Checked
against a brute-force byte map on random alloc/free sequences: live slices never overlap,
never leave the ring, are 256-byte aligned, and an allocation is refused only when the live
span (oldest live byte to the next allocation) could not take it.
"""
import random

import pytest

from paper_2606_06697_amd.serving import _Ring


@pytest.mark.parametrize("seed", range(8))
def test_ring_slices_never_overlap(seed):
    rng = random.Random(seed)
    size = rng.choice([4096, 16384, 65536])
    base = 0x7F00_0000_0000
    ring = _Ring(base, size)
    live = {}                                  # start -> (addr, length)
    owner = [None] * size                      # brute-force byte map of live slices
    for step in range(2000):
        if live and rng.random() < 0.45:
            start = rng.choice(list(live))
            addr, n = live.pop(start)
            for k in range(addr - base, addr - base + n):
                assert owner[k] == start
                owner[k] = None
            ring.free(start)
            continue
        want = rng.choice([1, 100, 256, 1000, size // 8, size // 3])
        got = ring.alloc(want)
        n = (want + 255) & ~255
        if got is None:
            # refused: the next allocation cannot fit without passing the oldest live byte
            assert live, "an empty ring refused an allocation that fits"
            continue
        start, addr = got
        assert (addr - base) % 256 == 0 and base <= addr and addr + n <= base + size
        for k in range(addr - base, addr - base + n):
            assert owner[k] is None, (step, "overlap")
            owner[k] = start
        live[start] = (addr, n)
    for start in list(live):
        ring.free(start)
    assert ring.tail == ring.head                # everything reclaimed
    assert ring.alloc(size) is not None          # the whole ring is free again
