"""Pins for the oracle's client handle tokens (CPU only).

The mechanism (slot, generation, keyed tag) is checked against the definition (a history of
every minted token: never minted -> FORGED, released -> STALE, other owner -> CROSS_CLIENT,
other kind -> WRONG_KIND), against published SplitMix64 outputs, and against hand-derived
slot and generation sequences.
"""
import random

import pytest

from oracle import tokens as T


def test_splitmix64_published_outputs():
    """The reference generator seeded with 0 yields 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
    0x06c45d188009454f (states gamma, 2 gamma, 3 gamma before mixing)."""
    g = 0x9E3779B97F4A7C15
    got = [T.splitmix64((k * g) & T.M64) for k in range(3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_token_layout_and_slot_reuse_by_hand():
    t = T.TokenTable(8, key=12345)
    a = t.mint(1, 7)
    b = t.mint(1, 7)
    c = t.mint(2, 9)
    assert [x >> 40 for x in (a, b, c)] == [0, 1, 2]          # lowest free slots, in order
    assert [(x >> 16) & T.GEN_MASK for x in (a, b, c)] == [0, 0, 0]
    assert (b & 0xFFFF) == T.splitmix64(12345 ^ ((1 << 24) | 0)) >> 48
    e = t.mint(1, 7)                                          # slot 3
    t.release(e, 1)
    t.release(b, 1)
    d = t.mint(3, 1)                                          # lowest free: slot 1, generation 1
    assert d >> 40 == 1 and (d >> 16) & T.GEN_MASK == 1 and d != b
    assert t.mint(3, 1) >> 40 == 3                            # then slot 3
    assert t.check(b, 1) == (T.STALE, -1)
    assert t.check(d, 3) == (T.VALID, 1)
    assert t.check(d, 1) == (T.CROSS_CLIENT, -1)
    assert t.check(d, 3, 2) == (T.WRONG_KIND, -1)
    assert t.check(d, 3, 1) == (T.VALID, 1)
    assert t.check(c, 2, T.ANY_KIND) == (T.VALID, 2)
    assert t.check(c ^ 1, 2) == (T.FORGED, -1)                # tag does not match
    assert t.check((9 << 40) | (c & ((1 << 40) - 1)), 2) == (T.FORGED, -1)  # slot >= capacity
    fwd = T.make_token(t.key, 2, 1)                           # a generation not reached yet
    assert t.check(fwd, 2) == (T.FORGED, -1)
    free_slot = T.make_token(t.key, 4, 0)                     # never minted, tag is right
    assert t.check(free_slot, 0) == (T.FORGED, -1)
    with pytest.raises(KeyError):
        t.release(b, 1)                                       # already released
    with pytest.raises(KeyError):
        t.release(d, 1)                                       # not the owner


def test_keys_separate_tables():
    t1, t2 = T.TokenTable(16, key=1), T.TokenTable(16, key=2)
    a = [t1.mint(0, 0) for _ in range(16)]
    b = [t2.mint(0, 0) for _ in range(16)]
    assert all(x != y for x, y in zip(a, b))
    assert all(t2.check(x, 0)[0] == T.FORGED for x in a)


def test_capacity_and_generation_retirement():
    t = T.TokenTable(2, key=5)
    x, y = t.mint(0, 0), t.mint(0, 0)
    with pytest.raises(MemoryError):
        t.mint(0, 0)
    t.gen[0] = T.GEN_MASK - 1                                 # slot 0 near the end of its generations
    t.owner[0] = 0
    x = T.make_token(t.key, 0, T.GEN_MASK - 1)
    t.release(x, 0)
    z = t.mint(0, 0)
    assert z >> 40 == 0 and (z >> 16) & T.GEN_MASK == T.GEN_MASK
    t.release(z, 0)                                           # last generation: slot retired
    t.release(y, 0)
    w = t.mint(0, 0)
    assert w >> 40 == 1
    with pytest.raises(MemoryError):
        t.mint(0, 0)
    assert t.check(z, 0) == (T.STALE, -1)


def _presented(rng, hist, t, clients, kinds):
    """Every minted token by its owner and by others, with right and wrong kinds, plus
    fabricated ones (random words, flipped tags, moved slots, future generations)."""
    out = []
    for tok, (own, kind, _) in hist.minted.items():
        out.append((tok, own, T.ANY_KIND))
        out.append((tok, own, kind))
        out.append((tok, rng.choice(clients), rng.choice(kinds + [T.ANY_KIND])))
        out.append((tok ^ (1 << rng.randrange(16)), own, T.ANY_KIND))
        out.append((tok ^ (1 << (40 + rng.randrange(24))), own, T.ANY_KIND))
        s, g = tok >> 40, (tok >> 16) & T.GEN_MASK
        out.append((T.make_token(t.key, s, (g + 1) & T.GEN_MASK), own, T.ANY_KIND))
    for _ in range(50):
        out.append((rng.getrandbits(64), rng.choice(clients), T.ANY_KIND))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_mechanism_matches_definition(seed):
    rng = random.Random(seed)
    t = T.TokenTable(rng.choice([4, 16, 64]), key=rng.getrandbits(64))
    hist = T.TokenHistory()
    clients, kinds = [0, 1, 2, 7], [0, 1, 5]
    live = []
    for step in range(300):
        if live and rng.random() < 0.4:
            tok, own = live.pop(rng.randrange(len(live)))
            t.release(tok, own)
            hist.release(tok)
        else:
            c, k = rng.choice(clients), rng.choice(kinds)
            try:
                tok = t.mint(c, k)
            except MemoryError:
                assert len(live) == t.cap
                continue
            hist.add(tok, c, k)
            live.append((tok, c))
        if step % 25 == 0:
            pres = _presented(rng, hist, t, clients, kinds)
            for tok, c, k in pres:
                v, s = t.check(tok, c, k)
                assert v == hist.check(tok, c, k), (hex(tok), c, k)
                assert (s >= 0) == (v == T.VALID)
                if v == T.VALID:
                    assert s == tok >> 40
            # the array form agrees with the one-token form
            vv, ss = T.check_many(t, [p[0] for p in pres], [p[1] for p in pres],
                                  [p[2] for p in pres])
            assert [(int(a), int(b)) for a, b in zip(vv, ss)] == [t.check(*p) for p in pres]
