"""Client handle tokens (oracle; test infrastructure only).

The paper's worker hands clients tokens instead of real object handles; the tokens are backed
by tables the worker owns, so it can refuse a fabricated token, a stale one (its object was
released) and one presented by a client that does not own it (Section IV-C). Two forms here:

* ``TokenHistory`` - the definition: every token ever minted, with its owner, kind and whether
  it has been released. A presented token is FORGED if it was never minted, STALE if it was
  released, CROSS_CLIENT if another client owns it, WRONG_KIND if it names another kind of
  object than the one expected, VALID otherwise.
* ``TokenTable`` - the mechanism the library uses, restated: a token is 64 bits,
  ``slot << 40 | gen << 16 | tag``. ``slot`` (24 bits) indexes a slot table of
  ``(owner, generation, kind)``; ``gen`` (24 bits) is the slot's generation when the token was
  minted; ``tag`` (16 bits) is the top of SplitMix64 (Steele, Lea and Flood, 2014) of
  ``key XOR (slot << 24 | gen)`` for the table's secret key, so a client cannot make up a
  token for a slot and generation it was never given. Minting takes the lowest free slot;
  releasing frees the slot and advances its generation (a slot released in its last
  generation is retired instead, so generations never repeat; every token of a retired slot
  is STALE, since each of its generations was minted once).

Readings (the paper gives no encoding): the verdict order above (forged, then stale, then
owner, then kind); a token whose tag checks but whose generation is ahead of its slot's, or
equal to a free slot's, was never minted and is FORGED.
"""
from __future__ import annotations

import heapq

VALID, FORGED, STALE, CROSS_CLIENT, WRONG_KIND = 0, 1, 2, 3, 4
ANY_KIND = 255
SLOT_BITS, GEN_BITS, TAG_BITS = 24, 24, 16
GEN_MASK = (1 << GEN_BITS) - 1
M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One output of SplitMix64 for state ``x`` (the state is advanced by the golden gamma
    0x9e3779b97f4a7c15, then mixed by the published finalizer)."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def tag_of(key: int, slot: int, gen: int) -> int:
    return splitmix64((key ^ ((slot << GEN_BITS) | gen)) & M64) >> (64 - TAG_BITS)


def make_token(key: int, slot: int, gen: int) -> int:
    return (slot << (GEN_BITS + TAG_BITS)) | (gen << TAG_BITS) | tag_of(key, slot, gen)


class TokenTable:
    def __init__(self, capacity: int, key: int):
        assert 1 <= capacity <= (1 << SLOT_BITS)
        self.cap = capacity
        self.key = key & M64
        self.owner = [None] * capacity      # owner client of a live slot, None when free
        self.retired = [False] * capacity
        self.gen = [0] * capacity
        self.kind = [0] * capacity
        self.free = []                       # min-heap of released, reusable slots
        self.next_new = 0

    def mint(self, client: int, kind: int) -> int:
        if self.free:
            s = heapq.heappop(self.free)
        elif self.next_new < self.cap:
            s = self.next_new
            self.next_new += 1
        else:
            raise MemoryError("token table full")
        self.owner[s], self.kind[s] = client, kind
        return make_token(self.key, s, self.gen[s])

    def check(self, token: int, client: int, want_kind: int = ANY_KIND):
        """-> (verdict, slot or -1)"""
        slot = token >> (GEN_BITS + TAG_BITS)
        gen = (token >> TAG_BITS) & GEN_MASK
        if slot >= self.cap or (token & ((1 << TAG_BITS) - 1)) != tag_of(self.key, slot, gen):
            return FORGED, -1
        if gen < self.gen[slot] or self.retired[slot]:
            return STALE, -1
        if gen > self.gen[slot] or self.owner[slot] is None:
            return FORGED, -1
        if self.owner[slot] != client:
            return CROSS_CLIENT, -1
        if want_kind != ANY_KIND and self.kind[slot] != want_kind:
            return WRONG_KIND, -1
        return VALID, slot

    def release(self, token: int, client: int) -> None:
        v, s = self.check(token, client)
        if v != VALID:
            raise KeyError("not a live token of this client")
        self.owner[s] = None
        if self.gen[s] == GEN_MASK:
            self.retired[s] = True          # generations exhausted
            return
        self.gen[s] += 1
        heapq.heappush(self.free, s)


def check_many(table: TokenTable, tokens, clients, kinds=None):
    """``TokenTable.check`` over arrays (uint64 tokens, uint32 clients, uint8 kinds or None)
    with numpy; the 64-bit products of SplitMix64 wrap modulo 2**64 as in the definition."""
    import numpy as np
    tok = np.asarray(tokens).astype(np.uint64)
    cli = np.asarray(clients).astype(np.int64)
    want = (np.full(tok.shape, ANY_KIND, np.int64) if kinds is None
            else np.asarray(kinds).astype(np.int64))
    slot = tok >> np.uint64(GEN_BITS + TAG_BITS)
    gen = (tok >> np.uint64(TAG_BITS)) & np.uint64(GEN_MASK)
    inr = slot < np.uint64(table.cap)
    sc = np.where(inr, slot, 0).astype(np.int64)
    with np.errstate(over="ignore"):
        z = (np.uint64(table.key) ^ ((sc.astype(np.uint64) << np.uint64(GEN_BITS)) | gen))
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    tag_ok = (z >> np.uint64(64 - TAG_BITS)) == (tok & np.uint64((1 << TAG_BITS) - 1))
    rgen = np.array(table.gen, np.int64)[sc]
    owner = np.array([-1 if o is None else o for o in table.owner], np.int64)[sc]
    retired = np.array(table.retired, bool)[sc]
    kind = np.array(table.kind, np.int64)[sc]
    g = gen.astype(np.int64)
    v = np.full(tok.shape, VALID, np.uint8)
    forged = ~inr | ~tag_ok
    stale = ~forged & ((g < rgen) | retired)
    forged |= ~stale & ((g > rgen) | (owner < 0))
    rest = ~forged & ~stale
    cross = rest & (owner != cli)
    wrong = rest & ~cross & (want != ANY_KIND) & (kind != want)
    v[wrong] = WRONG_KIND
    v[cross] = CROSS_CLIENT
    v[stale] = STALE
    v[forged] = FORGED
    out_slot = np.where(v == VALID, sc, -1).astype(np.int32)
    return v, out_slot


class TokenHistory:
    """The definition, by bookkeeping every minted token."""

    def __init__(self):
        self.minted = {}                     # token -> [owner, kind, released]

    def add(self, token: int, client: int, kind: int):
        assert token not in self.minted, "a token was minted twice"
        self.minted[token] = [client, kind, False]

    def release(self, token: int):
        self.minted[token][2] = True

    def check(self, token: int, client: int, want_kind: int = ANY_KIND) -> int:
        rec = self.minted.get(token)
        if rec is None:
            return FORGED
        if rec[2]:
            return STALE
        if rec[0] != client:
            return CROSS_CLIENT
        if want_kind != ANY_KIND and rec[1] != want_kind:
            return WRONG_KIND
        return VALID
