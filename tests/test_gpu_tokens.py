"""Client handle tokens on the GPU against the oracle (Section IV-C: fabricated, stale and
cross-client handles are refused).

The library and the oracle's slot table get the same key and the same mints and releases, so
the minted tokens must be equal bit for bit, and the device check must give the oracle's
verdicts and slots for every presented token: live tokens by their owner and by others, with
right and wrong kinds, released ones, and fabricated ones (random words, flipped tag bits,
moved slots, generations not issued). The verdicts are also compared with the history model
(every token ever minted). Cases: a small table through many mint/release rounds, a
2^20-slot table with a ragged batch of 2^22 + 5 tokens, checks on two streams around changes,
and the host-side errors.
"""
import random

import numpy as np
import pytest
import torch

from gpu_util import guard_mod, need_gpu
from oracle import tokens as T

pytestmark = pytest.mark.gpu


def presented(rng, minted, key, clients, kinds, k_random=100):
    out = []
    for tok, (own, kind) in minted.items():
        out.append((tok, own, T.ANY_KIND))
        out.append((tok, own, kind))
        out.append((tok, rng.choice(clients), rng.choice(kinds + [T.ANY_KIND])))
        out.append((tok ^ (1 << rng.randrange(16)), own, T.ANY_KIND))
        out.append((tok ^ (1 << (40 + rng.randrange(24))), own, T.ANY_KIND))
        s, g = tok >> 40, (tok >> 16) & T.GEN_MASK
        out.append((T.make_token(key, s, (g + 1) & T.GEN_MASK), own, T.ANY_KIND))
    for _ in range(k_random):
        out.append((rng.getrandbits(64), rng.choice(clients), T.ANY_KIND))
    return out


def device_check(g, ts, pres, with_kinds=True, stream=None):
    tok = torch.tensor(np.array([p[0] for p in pres], np.uint64).view(np.int64), device="cuda")
    cli = torch.tensor(np.array([p[1] for p in pres], np.uint32).view(np.int32), device="cuda")
    knd = (torch.tensor(np.array([p[2] for p in pres], np.uint8), device="cuda")
           if with_kinds else None)
    v, s = ts.check(tok, cli, knd, stream)
    torch.cuda.synchronize()
    return v.cpu().numpy(), s.cpu().numpy()


def test_tokens_small_table_many_rounds():
    need_gpu()
    g = guard_mod()
    rng = random.Random(7)
    key = rng.getrandbits(64)
    ts = g.TokenTable(64, key)
    ot = T.TokenTable(64, key)
    hist = T.TokenHistory()
    clients, kinds = [0, 1, 2, 9, 0xFFFFFFFD], [0, 3, 254]
    live, minted = [], {}
    seen = set()
    for step in range(600):
        if live and rng.random() < 0.45:
            tok, own = live.pop(rng.randrange(len(live)))
            ts.release(tok, own)
            ot.release(tok, own)
            hist.release(tok)
        else:
            c, k = rng.choice(clients), rng.choice(kinds)
            if len(live) == 64:
                with pytest.raises(g.AgileError) as e:
                    ts.mint(c, k)
                assert e.value.code == g.AGILE_ENOSPC
                continue
            tok = ts.mint(c, k)
            assert tok == ot.mint(c, k)
            hist.add(tok, c, k)
            live.append((tok, c))
            minted[tok] = (c, k)
        if step % 60 == 0:
            pres = presented(rng, minted, key, clients, kinds)
            for with_kinds in (True, False):
                v, s = device_check(g, ts, pres, with_kinds)
                kk = [p[2] for p in pres] if with_kinds else None
                ev, es = T.check_many(ot, [p[0] for p in pres], [p[1] for p in pres], kk)
                assert np.array_equal(v, ev) and np.array_equal(s, es), step
                hv = [hist.check(p[0], p[1], p[2] if with_kinds else T.ANY_KIND) for p in pres]
                assert v.tolist() == hv, step
                seen |= set(v.tolist())
    assert seen == {0, 1, 2, 3, 4}
    ts.close()


def test_tokens_large_table_ragged_batch():
    need_gpu()
    g = guard_mod()
    rng = np.random.default_rng(3)
    key = 0x1234_5678_9ABC_DEF0
    cap = 1 << 20
    ts = g.TokenTable(cap, key)
    ot = T.TokenTable(cap, key)
    nmint = 600_000
    owners = rng.integers(0, 64, nmint)
    kinds = rng.integers(0, 8, nmint)
    toks = np.empty(nmint, np.uint64)
    for i in range(nmint):
        o, k = int(owners[i]), int(kinds[i])
        toks[i] = ts.mint(o, k)
        assert int(toks[i]) == ot.mint(o, k)
    rel = rng.choice(nmint, nmint // 3, replace=False)
    for i in rel.tolist():
        ts.release(int(toks[i]), int(owners[i]))
        ot.release(int(toks[i]), int(owners[i]))
    n = (1 << 22) + 5
    pick = rng.integers(0, nmint, n)
    tok = toks[pick].copy()
    cli = owners[pick].astype(np.uint32)
    want = kinds[pick].astype(np.uint8)
    r = rng.random(n)
    cli[r < 0.1] = rng.integers(0, 64, int((r < 0.1).sum()))              # often another client
    want[(r >= 0.1) & (r < 0.2)] = T.ANY_KIND
    want[(r >= 0.2) & (r < 0.25)] = 7 - want[(r >= 0.2) & (r < 0.25)] % 8  # wrong kind
    fl = (r >= 0.25) & (r < 0.3)
    tok[fl] ^= np.uint64(1) << rng.integers(0, 64, int(fl.sum())).astype(np.uint64)
    rnd = r >= 0.97
    tok[rnd] = rng.integers(0, 2**63, int(rnd.sum()), dtype=np.int64).astype(np.uint64) * 2 + 1
    td = torch.from_numpy(tok.view(np.int64)).cuda()
    cd = torch.from_numpy(cli.view(np.int32)).cuda()
    kd = torch.from_numpy(want).cuda()
    v, s = ts.check(td, cd, kd)
    torch.cuda.synchronize()
    ev, es = T.check_many(ot, tok, cli, want)
    v, s = v.cpu().numpy(), s.cpu().numpy()
    bad = np.flatnonzero((v != ev) | (s != es))
    assert bad.size == 0, (bad.size, [(hex(int(tok[k])), int(v[k]), int(ev[k])) for k in bad[:5]])
    assert np.bincount(v, minlength=5).min() > 1000
    ts.close()


def test_tokens_two_streams_see_changes_in_order():
    need_gpu()
    g = guard_mod()
    key = 99
    ts = g.TokenTable(16, key)
    a = ts.mint(1, 0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    pres = [(a, 1, T.ANY_KIND)]
    with torch.cuda.stream(s1):
        v1, _ = device_check(g, ts, pres, stream=s1)
    ts.release(a, 1)
    b = ts.mint(1, 0)                       # same slot, next generation
    with torch.cuda.stream(s2):
        v2, _ = device_check(g, ts, pres + [(b, 1, T.ANY_KIND)], stream=s2)
    assert v1.tolist() == [T.VALID] and v2.tolist() == [T.STALE, T.VALID]
    with pytest.raises(g.AgileError) as e:
        ts.release(a, 1)                    # stale: nothing happens
    assert e.value.code == g.AGILE_ENOENT
    with pytest.raises(g.AgileError) as e:
        ts.release(b, 2)                    # not the owner
    assert e.value.code == g.AGILE_ENOENT
    for bad in ((0xFFFFFFFE, 0), (0, 255)):
        with pytest.raises(g.AgileError) as e:
            ts.mint(*bad)
        assert e.value.code == g.AGILE_EINVAL
    ts.close()
