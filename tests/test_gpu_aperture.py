"""Fixed address apertures on the device (Section IV-E, Table I; Section V-A).

* layout: the I/O, module and user apertures back to back, each rounded up to the
  granularity; Table I's sizes at Table I's base address when the runtime grants the hint (the
  hand-derived Table I fixture is then checked as it stands);
* the coarse check ``agile_validate_aperture`` against the oracle, bit-exact, on every
  boundary address with lengths that reach every boundary, random and extreme queries, ragged
  sizes (bytes past n untouched) and without the index output;
* allocations: each with physical memory of its own, mapped at the lowest free address of its
  aperture in a reservation of its own, registered in a range table with the kind of their
  aperture, readable and writable by the guarded kernels
  (parity with the oracle, fault log included); table validation agrees with the apertures (a table
  ALLOW is an aperture ALLOW, a table PROTECTED an aperture PROTECTED); a freed allocation is
  UNMAPPED in the table but still ALLOW for the apertures, and its addresses are reused.
"""
import os

import numpy as np
import pytest
import torch

from gpu_util import Twin, guard_mod, log_matches, need_gpu
from oracle import aperture as AP
from oracle import guarded as G
from oracle.memory import Memory
from oracle.table import MMIO, PROTECTED, USER

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
MiB, GiB = 1 << 20, 1 << 30


def up(x, g):
    return (x + g - 1) // g * g


def qtensor(addr, length):
    """(addr, len) uint64 pairs as a device int64 tensor of shape (n, 2)."""
    addr = np.asarray(addr, dtype=np.uint64)
    length = np.asarray(length, dtype=np.uint64)
    return torch.from_numpy(np.stack([addr, length], 1).view(np.int64).copy()).cuda()


def run_validate(g, ap, addr, length, with_region=True):
    addr = np.asarray(addr, dtype=np.uint64)
    length = np.asarray(length, dtype=np.uint64)
    n = addr.size
    q = qtensor(addr, length)
    v = torch.full((n + 64,), 0xEE, dtype=torch.uint8, device="cuda")
    r = torch.full((n + 64,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    g.agile_validate_aperture(ap, q, n, v, r if with_region else None)
    torch.cuda.synchronize()
    v, r = v.cpu().numpy(), r.cpu().numpy()
    assert (v[n:] == 0xEE).all() and (r[n:] == 0x5A5A5A5A).all(), "wrote past n"
    if not with_region:
        assert (r == 0x5A5A5A5A).all()
    return v[:n], r[:n]


def boundary_queries(bounds):
    qa, ql = [], []
    for b in bounds:
        for d in range(-2, 3):
            a = b + d
            lens = {0, 1, 2, 7, 4096, (1 << 64) - 1}
            for c in bounds:
                if c > a:
                    lens.update({c - a - 1, c - a, c - a + 1})
            for L in sorted(lens):
                qa.append(a)
                ql.append(L)
    return np.array(qa, dtype=np.uint64), np.array(ql, dtype=np.uint64)


def random_queries(bounds, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = bounds[0] - GiB, bounds[3] + GiB
    addr = rng.integers(lo, hi, n, dtype=np.uint64)
    length = (2.0 ** rng.uniform(0, 40, n)).astype(np.uint64)
    length[rng.random(n) < 0.05] = 0
    extreme = np.array([0, 1, (1 << 64) - 1, (1 << 64) - 2, bounds[3] - 1], dtype=np.uint64)
    addr[:extreme.size] = extreme
    return addr, length


def check_parity(g, ap, bounds, addr, length, what):
    v, r = run_validate(g, ap, addr, length)
    ev, er = AP.aperture_verdict_many(bounds, addr, length)
    bad = np.flatnonzero((v != ev) | (r != er))
    assert bad.size == 0, (what, int(bad.size), hex(int(addr[bad[0]])), int(length[bad[0]]),
                           int(v[bad[0]]), int(ev[bad[0]]), int(r[bad[0]]), int(er[bad[0]]))
    return v, r


def test_layout_and_validation_parity():
    need_gpu()
    g = guard_mod()
    ap = g.agile_aperture_create(0, (64 * MiB + 5, 256 * MiB, 4 * GiB))
    try:
        bounds, mapped, gran = g.agile_aperture_info(ap)
        assert mapped == (0, 0, 0)
        assert gran > 0 and gran & (gran - 1) == 0
        assert bounds[0] % gran == 0
        assert bounds[1] - bounds[0] == up(64 * MiB + 5, gran)
        assert bounds[2] - bounds[1] == 256 * MiB and bounds[3] - bounds[2] == 4 * GiB
        addr, length = boundary_queries(bounds)
        check_parity(g, ap, bounds, addr, length, "boundaries")
        addr, length = random_queries(bounds, 1 << 20, 3)
        v, r = check_parity(g, ap, bounds, addr, length, "random")
        assert len(set(v.tolist())) == 4          # every verdict occurs
        for n in (1, 5, 1023, 1025, 4097, 77777):  # ragged sizes and tails
            check_parity(g, ap, bounds, addr[:n], length[:n], f"n={n}")
        v2, _ = run_validate(g, ap, addr, length, with_region=False)
        assert np.array_equal(v2, v)
        g.agile_validate_aperture(ap, 0, 0, 0, 0)   # n == 0 is a no-op
        q = torch.zeros(4, 2, dtype=torch.int64, device="cuda")
        with pytest.raises(g.AgileError) as e:
            g.agile_validate_aperture(ap, q.data_ptr() + 8, 2, q, None)
        assert e.value.code == g.AGILE_EINVAL
    finally:
        g.agile_aperture_destroy(ap)


def test_table1_layout():
    """Table I's apertures (64 GiB I/O, 448 GiB module, 1 TiB user), asked for at Table I's
    base; no physical memory is attached."""
    need_gpu()
    g = guard_mod()
    b0 = AP.TABLE1[0]
    sizes = [AP.TABLE1[k + 1] - AP.TABLE1[k] for k in range(3)]
    ap = g.agile_aperture_create(0, sizes, base_hint=b0)
    try:
        bounds, _, gran = g.agile_aperture_info(ap)
        assert [bounds[k + 1] - bounds[k] for k in range(3)] == sizes
        print("Table I reservation at", hex(bounds[0]), "granularity", gran)
        rows = []
        for line in open(os.path.join(HERE, "golden", "table1_apertures.txt")):
            f = line.split("#", 1)[0].split()
            if f:
                rows.append((int(f[0], 0), int(f[1], 0), int(f[2]), int(f[3])))
        addr = np.array([a for a, *_ in rows], dtype=np.uint64)
        length = np.array([L for _, L, *_ in rows], dtype=np.uint64)
        if bounds[0] != b0:   # placed elsewhere: the same offsets from the actual base
            shift = np.uint64((bounds[0] - b0) % (1 << 64))
            inside = (addr >= np.uint64(b0 - (1 << 40))) & (addr < np.uint64(AP.TABLE1[3] + (1 << 40)))
            addr = np.where(inside, addr + shift, addr)
        v, r = check_parity(g, ap, bounds, addr, length, "Table I")
        if bounds[0] == b0:
            assert v.tolist() == [x[2] for x in rows] and r.tolist() == [x[3] for x in rows]
    finally:
        g.agile_aperture_destroy(ap)


def test_allocations_are_registered_and_guarded():
    need_gpu()
    g = guard_mod()
    tw = Twin(64)
    ap = g.agile_aperture_create(0, (16 * MiB, 64 * MiB, 1 * GiB), (4 * MiB, MiB, 256 * MiB))
    try:
        bounds, mapped, gran = g.agile_aperture_info(ap)
        assert mapped == (0, 0, 0)
        rng = np.random.default_rng(9)
        # (name, aperture, requested bytes, oracle kind)
        plan = [("A", g.AP_USER, MiB + 3, USER), ("B", g.AP_USER, 5 * MiB, USER),
                ("M", g.AP_MODULE, 64 << 10, PROTECTED), ("I", g.AP_IO, 4096, MMIO),
                ("X", g.AP_USER, 8 * 4096, USER)]
        addr, ids, size = {}, {}, {}
        for name, region, nb, kind in plan:
            p, rid = g.agile_aperture_alloc(ap, region, nb, tw.h)
            assert rid == tw.ot.insert(p, nb, kind)
            addr[name], ids[name], size[name] = p, rid, nb
        # lowest fit in each aperture, granule-aligned
        assert addr["A"] == bounds[2] and addr["B"] == bounds[2] + up(MiB + 3, gran)
        assert addr["X"] == addr["B"] + up(5 * MiB, gran)
        assert addr["M"] == bounds[1] and addr["I"] == bounds[0]
        assert len(tw.rt) == 5
        # each allocation maps its request rounded up to the granularity
        _, mapped, _ = g.agile_aperture_info(ap)
        assert mapped == (up(4096, gran), up(64 << 10, gran),
                          up(MiB + 3, gran) + up(5 * MiB, gran) + up(8 * 4096, gran))

        # fill A, B, X and M with known bytes (unguarded copies from torch memory)
        mem = Memory()
        for name in ("A", "B", "X", "M"):
            data = rng.integers(0, 256, size[name], dtype=np.uint8)
            src = torch.from_numpy(data).cuda()
            g.agile_unguarded_copy(addr[name], src, size[name])
            if name != "M":
                mem.add(addr[name], data)
        torch.cuda.synchronize()

        def read(name):
            out = torch.empty(size[name], dtype=torch.uint8, device="cuda")
            g.agile_unguarded_copy(out, addr[name], size[name])
            torch.cuda.synchronize()
            return out.cpu().numpy()

        ol = G.FaultLog()
        # guarded copy A -> B running 1000 bytes past A's requested end (still mapped memory:
        # the guard binds A to its requested size)
        nb = size["A"] + 1000
        g.agile_guarded_copy(tw.h, addr["B"], addr["A"], nb)
        G.copy_loop(tw.ot, mem, ol, tw.next_seq(), addr["B"], addr["A"], nb)
        assert np.array_equal(read("B"), mem.buffer(addr["B"]))
        log_matches(tw, ol, "copy past A")

        # guarded gather from table A with rows reaching back into the module aperture (M is
        # PROTECTED: suppressed and logged with M's id) and past B's end
        rb, n = 16, 512
        rows_a = size["A"] // rb
        idx = rng.integers(0, rows_a, n).astype(np.int64)
        idx[7] = (addr["M"] - addr["A"]) // rb            # first row of M
        idx[100] = (addr["M"] + 4096 - addr["A"]) // rb
        idx[300] = rows_a + 3                               # past A's end
        ib = torch.from_numpy(idx.view(np.uint8).copy()).cuda()
        g.agile_unguarded_copy(addr["X"], ib, idx.nbytes)
        mem.write(addr["X"], idx.tobytes())
        g.agile_guarded_gather(tw.h, addr["B"], addr["A"], rb, addr["X"], n, g.DTYPE_F32)
        G.gather_loop(tw.ot, mem, ol, tw.next_seq(), addr["B"], addr["A"], rb, addr["X"], n, 4)
        assert np.array_equal(read("B"), mem.buffer(addr["B"]))
        assert ol.first["verdict"] == g.V_PROTECTED and ol.first["owner"] == ids["M"]
        log_matches(tw, ol, "gather into the module aperture")

        # table validation agrees with the oracle table and with the apertures
        qa = [addr["A"], addr["A"] + size["A"] - 1, addr["A"] + size["A"], addr["B"] - 1,
              addr["M"], addr["M"] + 100, addr["I"], addr["I"] + 4095, addr["X"],
              bounds[2] + 512 * MiB, bounds[0] - 1, bounds[3]]
        ql = [size["A"], 1, 1, 1, 8, 8, 1, 1, size["X"] + 1, 16, 1, 1]
        qa = np.array(qa, dtype=np.uint64)
        ql = np.array(ql, dtype=np.uint64)
        q = qtensor(qa, ql)
        tv = torch.empty(qa.size, dtype=torch.uint8, device="cuda")
        to = torch.empty(qa.size, dtype=torch.int32, device="cuda")
        g.agile_validate_ptrs(tw.h, q, qa.size, tv, to)
        torch.cuda.synchronize()
        ev, eo = tw.ot.verdict_many(qa, ql)
        assert np.array_equal(tv.cpu().numpy(), ev) and np.array_equal(to.cpu().numpy(), eo)
        av, _ = run_validate(g, ap, qa, ql)
        assert np.array_equal(av, AP.aperture_verdict_many(bounds, qa, ql)[0])
        assert (av[ev == g.ALLOW] == g.ALLOW).all()
        assert (av[ev == g.V_PROTECTED] == g.V_PROTECTED).all()

        # free B: gone from the table, still inside the user aperture; its addresses come back
        g.agile_aperture_free(ap, addr["B"])
        tw.ot.remove(ids["B"])
        assert len(tw.rt) == 4
        g.agile_validate_ptrs(tw.h, qtensor([addr["B"]], [16]), 1, tv, to)
        torch.cuda.synchronize()
        assert int(tv[0]) == g.V_UNMAPPED
        assert tw.ot.verdict(addr["B"], 16)[0] == g.V_UNMAPPED
        av, _ = run_validate(g, ap, [addr["B"]], [16])
        assert int(av[0]) == g.ALLOW
        p, rid = g.agile_aperture_alloc(ap, g.AP_USER, 2 * MiB, tw.h)
        assert p == addr["B"] and rid == tw.ot.insert(p, 2 * MiB, USER)
        with pytest.raises(g.AgileError) as e:
            g.agile_aperture_free(ap, addr["B"] + gran)
        assert e.value.code == g.AGILE_ENOENT
        with pytest.raises(g.AgileError) as e:
            g.agile_aperture_alloc(ap, g.AP_IO, 32 * MiB, tw.h)
        assert e.value.code == g.AGILE_EINVAL          # larger than the aperture
        with pytest.raises(g.AgileError) as e:
            g.agile_aperture_alloc(ap, g.AP_IO, 8 * MiB, tw.h)
        assert e.value.code == g.AGILE_ENOSPC          # fits the aperture, not its budget
    finally:
        g.agile_aperture_destroy(ap)
    assert len(tw.rt) == 0       # destroy removed what was still registered
    tw.close()


def test_full_size_sampled():
    """2^28 queries with the bench's mix against Table I's sizes (placed by the runtime), in
    the launch the bench times; 2^20 sampled outputs against the oracle, and the verdict
    histogram of the whole output against the oracle's on the same inputs drawn again on the
    host in chunks."""
    need_gpu()
    g = guard_mod()
    from synth import aperture_table, make_queries
    n = 1 << 28
    ap = g.agile_aperture_create(0, (64 << 30, 448 << 30, 1 << 40))
    try:
        bounds, _, _ = g.agile_aperture_info(ap)
        q = make_queries(aperture_table(bounds), n, 11, device="cuda")
        v = torch.empty(n, dtype=torch.uint8, device="cuda")
        r = torch.empty(n, dtype=torch.int32, device="cuda")
        g.agile_validate_aperture(ap, q, n, v, r)
        torch.cuda.synchronize()
        rng = np.random.default_rng(11)
        pos = np.sort(rng.choice(n, 1 << 20, replace=False))
        pos_t = torch.from_numpy(pos).cuda()
        qs = q[pos_t].cpu().numpy().view(np.uint64)
        ev, er = AP.aperture_verdict_many(bounds, qs[:, 0], qs[:, 1])
        assert np.array_equal(v[pos_t].cpu().numpy(), ev)
        assert np.array_equal(r[pos_t].cpu().numpy(), er)
        # the whole output: per-verdict counts equal the oracle's on every query
        counts = torch.bincount(v.long(), minlength=4).cpu().numpy()
        want = np.zeros(4, dtype=np.int64)
        for c0 in range(0, n, 1 << 24):
            qc = q[c0:c0 + (1 << 24)].cpu().numpy().view(np.uint64)
            want += np.bincount(AP.aperture_verdict_many(bounds, qc[:, 0], qc[:, 1])[0],
                                minlength=4)
        assert np.array_equal(counts[:4], want)
        del q, v, r
    finally:
        g.agile_aperture_destroy(ap)


def test_each_allocation_maps_its_own_memory():
    """Section V-A: memory is created, mapped and made accessible per allocation. Thirty
    allocations of mixed sizes (3 B to 96 MiB, ragged; the patterns that lose device access when
    mapped side by side in one large reservation among them) in the user and module apertures
    of Table I's sizes, packed at the granularity, then freed and made again in the holes; every
    live allocation holds its own bytes (a distinct pattern written through it reads back from
    it alone), mapped bytes are accounted per aperture, and the table follows every step."""
    need_gpu()
    g = guard_mod()
    tw = Twin(256)
    ap = g.agile_aperture_create(0, (64 << 30, 448 << 30, 1 << 40))
    try:
        bounds, _, gran = g.agile_aperture_info(ap)
        rng = np.random.default_rng(17)
        live = {}   # address -> (region, bytes, pattern seed)

        def alloc(region, nb):
            p, rid = g.agile_aperture_alloc(ap, region, nb, tw.h)
            assert rid == tw.ot.insert(p, nb, USER if region == g.AP_USER else PROTECTED)
            assert p % gran == 0 and bounds[region] <= p and p + nb <= bounds[region + 1]
            seed = int(rng.integers(1 << 30))
            data = np.random.default_rng(seed).integers(0, 256, nb, dtype=np.uint8)
            g.agile_unguarded_copy(p, torch.from_numpy(data).cuda(), nb)
            live[p] = (region, nb, seed, rid)
            return p

        def check_all():
            torch.cuda.synchronize()
            for p, (region, nb, seed, _) in live.items():
                out = torch.empty(nb, dtype=torch.uint8, device="cuda")
                g.agile_unguarded_copy(out, p, nb)
                want = np.random.default_rng(seed).integers(0, 256, nb, dtype=np.uint8)
                assert np.array_equal(out.cpu().numpy(), want), hex(p)
            _, mapped, _ = g.agile_aperture_info(ap)
            for k in range(3):
                assert mapped[k] == sum(up(nb, gran) for r, nb, _, _ in live.values() if r == k)
            assert len(tw.rt) == len(live)

        sizes = [4096, MiB + 13, 3, 256 << 10, 96 * MiB + 5, 2 * MiB, 2 * MiB + 1, 64 << 10,
                 5000, 17 * MiB, 12 << 10, 4 * MiB - 1]
        order = []
        for k in range(24):
            region = g.AP_USER if k % 4 else g.AP_MODULE
            order.append(alloc(region, sizes[k % len(sizes)]))
        check_all()
        # free every third allocation, then allocate again: the holes are reused lowest-fit
        for p in order[::3]:
            g.agile_aperture_free(ap, p)
            tw.ot.remove(live.pop(p)[3])
        check_all()
        again = []
        for k in range(6):
            region = g.AP_USER if k % 2 else g.AP_MODULE
            again.append(alloc(region, sizes[(k * 5) % len(sizes)]))
        freed = sorted(order[::3])
        assert min(again) <= max(freed)          # some hole was reused
        check_all()
        # table validation of the live allocations: ALLOW inside, PROTECTED in the module
        # aperture's ones, UNMAPPED in the freed units no allocation took back
        qa = np.array([p for p in live] + [p + nb - 1 for p, (_, nb, _, _) in live.items()],
                      dtype=np.uint64)
        ql = np.ones(qa.size, dtype=np.uint64)
        q = qtensor(qa, ql)
        tv = torch.empty(qa.size, dtype=torch.uint8, device="cuda")
        to = torch.empty(qa.size, dtype=torch.int32, device="cuda")
        g.agile_validate_ptrs(tw.h, q, qa.size, tv, to)
        torch.cuda.synchronize()
        ev, eo = tw.ot.verdict_many(qa, ql)
        assert np.array_equal(tv.cpu().numpy(), ev) and np.array_equal(to.cpu().numpy(), eo)
    finally:
        g.agile_aperture_destroy(ap)
    assert len(tw.rt) == 0
    tw.close()
