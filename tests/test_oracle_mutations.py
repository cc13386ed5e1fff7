"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in the oracle (monkeypatched for the duration of the test) and
runs the pin tests that should notice it: the brute-force scan, the Table I fixture, the
boundary invariants, the exact rational rounding of the triad, the loop-versus-vectorized
agreement, the unit-gradient counts, the reason codes, the hand-derived straddling
accesses, the trap policy's retirement and the handle tokens' history model. The unmodified oracle passes all of them; every planted mistake must make at least
one of them fail (an assertion, or an error such as reading memory outside an allocation).
"""
import bisect
import copy

import numpy as np
import pytest

import oracle.aperture as AP
import oracle.guarded as G
import oracle.tokens as TK
from oracle.table import (RangeTable, ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED, V_INEXACT,
                          USER, PROTECTED)
import test_oracle_aperture as PA
import test_oracle_guarded as PG
import test_oracle_table as PT
import test_oracle_tokens as PK


def _fails(checks):
    for fn in checks:
        try:
            fn()
        except Exception:
            return True
    return False


TABLE_CHECKS = ([PT.test_table1_fixture, PT.test_boundary_invariants,
                 PT.test_dma_verdict_invariants] +
                [lambda s=s: PT.test_brute_force_exhaustive_boundaries(s) for s in range(12)] +
                [lambda s=s: PT.test_dma_verdict_brute_force(s) for s in range(8)])

GUARD_CHECKS = ([PG.test_access_straddling_the_allocation_end_is_denied,
                 PG.test_triad_matches_exact_rational_rounding,
                 PG.test_scatter_add_unit_gradient_counts, PG.test_fault_reason_codes,
                 PG.test_gather_no_fault_is_take, PG.test_copy_partial_closed_form_values,
                 PG.test_trap_policy_retires_on_a_violation_only, PG.test_sink_by_hand,
                 PG.test_sink_aligns_the_slot_to_the_access_width,
                 PG.test_report_performs_only_inside_registered_ranges,
                 PG.test_report_leaves_a_range_not_declared_backed_alone,
                 PG.test_sink_with_a_zero_quarantine_and_no_denied_store_equals_suppress,
                 PG.test_sink_scatter_add_accumulates_in_the_quarantine,
                 PG.test_remap_copy_from_a_short_allocation_repeats_it,
                 lambda: PG.test_remap_gather_wraps_rows_like_take(1),
                 lambda: PG.test_remap_gather_wraps_rows_like_take(3),
                 PG.test_remap_without_a_binding_suppresses] +
                [lambda s=s: PG.test_redirecting_policies_log_like_suppress_for_copy_and_triad(s)
                 for s in range(4)] +
                [lambda s=s: PG.test_copy_vec_matches_loop(s) for s in range(6)] +
                [lambda s=s: PG.test_triad_vec_matches_loop(s) for s in range(4)] +
                [lambda s=s, w=w, D=D: PG.test_gather_vec_matches_loop(s, w, D)
                 for s in range(3) for (w, D) in [(4, 1), (4, 3), (8, 2)]] +
                [lambda s=s, a=a: PG.test_scatter_vec_matches_loop(s, a)
                 for s in range(3) for a in (False, True)])


# ---- planted mistakes in the classification --------------------------------------------
def _verdict_with(fit=lambda L, room: L <= room, protected_kinds=None, owner_pos=False):
    def verdict(self, addr, length):
        addr, length = int(addr), int(length)
        ent = self.owner_entry(addr)
        if ent is None:
            return V_UNMAPPED, -1
        b, end, kind, rid = ent
        if owner_pos:
            rid = self._bases.index(b)
        if (kind != USER) if protected_kinds is None else (kind in protected_kinds):
            return V_PROTECTED, rid
        if fit(max(length, 1), end - addr):
            return ALLOW, rid
        return V_STRADDLE, rid
    return verdict


def _owner_with(left=False, end_inclusive=False):
    def owner_entry(self, addr):
        a = int(addr)
        k = (bisect.bisect_left if left else bisect.bisect_right)(self._bases, a) - 1
        if k < 0:
            return None
        b = self._bases[k]
        end, kind, rid = self._by_base[b]
        if a < end or (end_inclusive and a == end):
            return (b, end, kind, rid)
        return None
    return owner_entry


def _dma_with(exact):
    def dma_verdict(self, addr, length):
        v, rid = self.verdict(addr, length)
        if v == ALLOW:
            b, end, _, _ = self.owner_entry(addr)
            if not exact(int(addr), int(length), b, end):
                v = V_INEXACT
        return v, rid
    return dma_verdict


TABLE_MUTANTS = {
    "fit is strict (len < end - addr)": ("verdict", _verdict_with(fit=lambda L, room: L < room)),
    "fit off by one (len <= end - addr + 1)": ("verdict",
                                               _verdict_with(fit=lambda L, room: L <= room + 1)),
    "MMIO treated as user memory": ("verdict", _verdict_with(protected_kinds=(PROTECTED,))),
    "owner is the sorted position, not the id": ("verdict", _verdict_with(owner_pos=True)),
    "owner search finds the range ending at addr": ("owner_entry", _owner_with(left=True)),
    "range end counted as inside": ("owner_entry", _owner_with(end_inclusive=True)),
    "DMA exactness ignores the length": ("dma_verdict", _dma_with(lambda a, L, b, e: a == b)),
    "DMA exactness ignores the start": ("dma_verdict", _dma_with(lambda a, L, b, e: a + L == e)),
    "DMA zero length taken as one byte": ("dma_verdict",
                                          _dma_with(lambda a, L, b, e: a == b and max(L, 1) == e - b)),
}


def test_unmodified_oracle_passes_every_pin():
    assert not _fails(TABLE_CHECKS)
    assert not _fails(GUARD_CHECKS)


@pytest.mark.parametrize("name", sorted(TABLE_MUTANTS))
def test_classification_mistake_is_caught(name, monkeypatch):
    attr, fn = TABLE_MUTANTS[name]
    monkeypatch.setattr(RangeTable, attr, fn)
    assert _fails(TABLE_CHECKS), name


# ---- planted mistakes in the aperture classification -------------------------------------
APERTURE_CHECKS = ([PA.test_table1_apertures_fixture] +
                   [lambda s=s: PA.test_brute_force_on_the_apertures_as_ranges(s)
                    for s in range(10)])


def _aperture_with(end_inclusive=False, no_straddle=False, module_is_user=False,
                   swap_protected=False):
    def aperture_verdict(bounds, addr, length):
        b0, b1, b2, b3 = AP.check_bounds(bounds)
        addr, length = int(addr), int(length)
        if addr < b0 or addr > b3 or (addr == b3 and not end_inclusive):
            return V_UNMAPPED, -1
        if addr < b1:
            return V_PROTECTED, AP.MODULE if swap_protected else AP.IO
        if addr < b2 and not module_is_user:
            return V_PROTECTED, AP.IO if swap_protected else AP.MODULE
        if no_straddle or max(length, 1) <= b3 - addr:
            return ALLOW, AP.USER_AP
        return V_STRADDLE, AP.USER_AP
    return aperture_verdict


APERTURE_MUTANTS = {
    "user aperture end counted as inside": _aperture_with(end_inclusive=True),
    "a span past the user aperture allowed": _aperture_with(no_straddle=True),
    "module aperture treated as user memory": _aperture_with(module_is_user=True),
    "I/O and module indices swapped": _aperture_with(swap_protected=True),
}


def test_unmodified_aperture_oracle_passes_its_pins():
    assert not _fails(APERTURE_CHECKS)


@pytest.mark.parametrize("name", sorted(APERTURE_MUTANTS))
def test_aperture_mistake_is_caught(name, monkeypatch):
    monkeypatch.setattr(AP, "aperture_verdict", APERTURE_MUTANTS[name])
    assert _fails(APERTURE_CHECKS), name


# ---- planted mistakes in the guarded kernels --------------------------------------------
def _triad_one_rounding(orig):
    """The per-access triad with the product and the sum rounded once, together."""
    def triad_vec(table, mem, log, seq, a, b, c, s, n, policy=G.SUPPRESS_LOG):
        deny = G._Denier(table, log, seq, G.OP_TRIAD, policy)
        ba, bb, bc = table.binding(a), table.binding(b), table.binding(c)
        for i in range(n):
            vals = []
            for op_i, (p, bind) in enumerate(((b, bb), (c, bc))):
                A = p + 4 * i
                if G._allowed(bind, A, 4):
                    vals.append(np.float64(G._f32(mem.read(A, 4))))
                else:
                    vals.append(np.float64(0.0))
                    deny(i, op_i, A, 4)
            r = np.float32(vals[0] + np.float64(np.float32(s)) * vals[1])
            A = a + 4 * i
            if G._allowed(ba, A, 4):
                mem.write(A, r.tobytes())
            else:
                deny(i, 2, A, 4)
    return triad_vec


def _scatter_overwrites(orig):
    def scatter_vec(table, mem, log, seq, dst, row_bytes, idx_ptr, src, n, w=4,
                    accumulate=False, policy=G.SUPPRESS_LOG):
        return orig(table, mem, log, seq, dst, row_bytes, idx_ptr, src, n, w, False, policy)
    return scatter_vec


def _reason_without_remap(table, A, w):
    if A < 0 or A > G.U64_MAX:
        return V_UNMAPPED, -1
    return table.verdict(A, w)


def _allowed_strict(bind, A, w):
    return bind[0] <= A and A + w < bind[1]


def _allowed_first_byte(bind, A, w):
    return bind[0] <= A < bind[1]


def _trap_retires_every_call(orig):
    def guarded_call(kernel, table, mem, log, seq, *args, policy=G.SUPPRESS_LOG, **kw):
        if log.retired:
            return G.ETRAPPED
        kernel(table, mem, log, seq, *args, policy=policy, **kw)
        if policy == G.TRAP:
            log.retired = True
            return G.ETRAPPED
        return G.OK
    return guarded_call


def _retired_handle_keeps_running(orig):
    def guarded_call(kernel, table, mem, log, seq, *args, policy=G.SUPPRESS_LOG, **kw):
        was = log.retired
        log.retired = False
        rc = orig(kernel, table, mem, log, seq, *args, policy=policy, **kw)
        log.retired = log.retired or was
        return G.ETRAPPED if log.retired else rc
    return guarded_call


def _trapping_call_rolled_back(orig):
    def guarded_call(kernel, table, mem, log, seq, *args, policy=G.SUPPRESS_LOG, **kw):
        snap = copy.deepcopy(mem)
        rc = orig(kernel, table, mem, log, seq, *args, policy=policy, **kw)
        if rc == G.ETRAPPED:
            mem.__dict__.update(snap.__dict__)
        return rc
    return guarded_call


def _target_unaligned(self, A, w, bind=(0, 0)):
    if self.policy == G.SINK:
        qb, qs = self.q
        return qb + (A % (1 << 64)) % qs
    return _ORIG_TARGET(self, A, w, bind)


def _target_report_everywhere(self, A, w, bind=(0, 0)):
    if self.policy == G.REPORT:
        return A
    return _ORIG_TARGET(self, A, w, bind)


def _target_report_ignores_backing(self, A, w, bind=(0, 0)):
    if self.policy == G.REPORT:
        ent = self.t.owner_entry(A)
        if ent is not None and 0 <= A and A + w <= ent[1]:
            return A
        return None
    return _ORIG_TARGET(self, A, w, bind)


def _target_remap_by_size(self, A, w, bind=(0, 0)):
    if self.policy == G.REMAP and bind[1] > bind[0]:
        lo, hi = bind
        return lo + ((A - lo) % (hi - lo)) // w * w
    return _ORIG_TARGET(self, A, w, bind)


def _store_dropped(self, mem, A, data, bind=(0, 0)):
    return None


def _add_overwrites(self, mem, A, val, dt, bind=(0, 0)):
    t = self.target(A, dt().itemsize, bind)
    if t is not None:
        mem.write(t, dt(val).tobytes())


_ORIG_TARGET = G._Denier.target

DENIER_MUTANTS = {
    "sink slot not aligned to the access width": ("target", _target_unaligned),
    "report performs outside registered ranges": ("target", _target_report_everywhere),
    "report performs in ranges not declared backed": ("target", _target_report_ignores_backing),
    "remap wraps by the allocation size, not whole elements": ("target", _target_remap_by_size),
    "redirected stores dropped": ("store", _store_dropped),
    "redirected scatter-add overwrites": ("add", _add_overwrites),
}


@pytest.mark.parametrize("name", sorted(DENIER_MUTANTS))
def test_redirect_mistake_is_caught(name, monkeypatch):
    attr, fn = DENIER_MUTANTS[name]
    monkeypatch.setattr(G._Denier, attr, fn)
    assert _fails(GUARD_CHECKS), name


GUARD_MUTANTS = {
    "triad rounded once (fused)": ("triad_vec", _triad_one_rounding),
    "scatter-add overwrites": ("scatter_vec", _scatter_overwrites),
    "reason keeps ALLOW for cross-allocation": ("reason", lambda orig: _reason_without_remap),
    "access check excludes the last element": ("_allowed", lambda orig: _allowed_strict),
    "access check tests the first byte only": ("_allowed", lambda orig: _allowed_first_byte),
    "trap retires the handle on a clean call": ("guarded_call", _trap_retires_every_call),
    "retired handle keeps running its calls": ("guarded_call", _retired_handle_keeps_running),
    "trapping call rolled back instead of suppressed": ("guarded_call", _trapping_call_rolled_back),
}


@pytest.mark.parametrize("name", sorted(GUARD_MUTANTS))
def test_guard_mistake_is_caught(name, monkeypatch):
    attr, make = GUARD_MUTANTS[name]
    monkeypatch.setattr(G, attr, make(getattr(G, attr)))
    assert _fails(GUARD_CHECKS), name


# ---- planted mistakes in the handle tokens -----------------------------------------------
TOKEN_CHECKS = ([PK.test_splitmix64_published_outputs, PK.test_token_layout_and_slot_reuse_by_hand,
                 PK.test_keys_separate_tables, PK.test_capacity_and_generation_retirement] +
                [lambda s=s: PK.test_mechanism_matches_definition(s) for s in range(6)])


def _check_with(stale_as_forged=False, skip_owner=False, skip_kind=False):
    def check(self, token, client, want_kind=TK.ANY_KIND):
        slot = token >> 40
        gen = (token >> 16) & TK.GEN_MASK
        if slot >= self.cap or (token & 0xFFFF) != TK.tag_of(self.key, slot, gen):
            return TK.FORGED, -1
        if gen < self.gen[slot] or self.retired[slot]:
            return (TK.FORGED if stale_as_forged else TK.STALE), -1
        if gen > self.gen[slot] or self.owner[slot] is None:
            return TK.FORGED, -1
        if not skip_owner and self.owner[slot] != client:
            return TK.CROSS_CLIENT, -1
        if not skip_kind and want_kind != TK.ANY_KIND and self.kind[slot] != want_kind:
            return TK.WRONG_KIND, -1
        return TK.VALID, slot
    return check


def _release_keeps_generation(self, token, client):
    v, s = self.check(token, client)
    if v != TK.VALID:
        raise KeyError("not live")
    self.owner[s] = None
    import heapq
    heapq.heappush(self.free, s)


def _mint_highest_free(self, client, kind):
    if self.free:
        s = max(self.free)
        self.free.remove(s)
        import heapq
        heapq.heapify(self.free)
    elif self.next_new < self.cap:
        s = self.next_new
        self.next_new += 1
    else:
        raise MemoryError("full")
    self.owner[s], self.kind[s] = client, kind
    return TK.make_token(self.key, s, self.gen[s])


TOKEN_MUTANTS = {
    "stale token reported as forged": (TK.TokenTable, "check", _check_with(stale_as_forged=True)),
    "owner not checked": (TK.TokenTable, "check", _check_with(skip_owner=True)),
    "kind not checked": (TK.TokenTable, "check", _check_with(skip_kind=True)),
    "release keeps the generation": (TK.TokenTable, "release", _release_keeps_generation),
    "mint takes the highest free slot": (TK.TokenTable, "mint", _mint_highest_free),
    "tag ignores the key": (TK, "tag_of", lambda key, slot, gen: TK.splitmix64((slot << 24) | gen) >> 48),
}


def test_unmodified_token_oracle_passes_every_pin():
    assert not _fails(TOKEN_CHECKS)


@pytest.mark.parametrize("name", sorted(TOKEN_MUTANTS))
def test_token_mistake_is_caught(name, monkeypatch):
    owner, attr, fn = TOKEN_MUTANTS[name]
    monkeypatch.setattr(owner, attr, fn)
    assert _fails(TOKEN_CHECKS), name
