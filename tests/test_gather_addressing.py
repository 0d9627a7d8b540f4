"""CPU emulation of the matcher's candidate addressing (no device).

A query's candidates are the six bucket runs (one per table) concatenated in
table order; candidate e must load the bucket-table entry at position
t*n + b_t + (e - start_t) of the table t whose run holds it, and carry 8t
for the union test.  The matcher finds that position two ways, emulated here
exactly as the kernel computes it, word by word:

  by table (8-slot and band kernels): the run starts P1..P5 of tables 1..5 are
    compared with e; their count o is the table, and the run table holds
    C_t = t*n + b_t - start_t at word o;
  by ordinal (4- and 6-slot plain kernels): the tile setup writes, per query,
    the run word (C << 10 | 8t) of each non-empty run at its ordinal among
    the non-empty runs, a 64-bit mask per 64-candidate chunk with bit j set
    for a run starting at candidate 64u + j + 1 (runs after the first
    non-empty one, starting within the register slots), and 3-bit counts of
    such starts at or below 64, 128, ...; a lane of chunk u finds its run's
    ordinal as that count plus the mask bits below it (mbcnt), and its byte
    offset as (word >> 6) + 16 e.

Every candidate of random and edge-case run layouts must get its true
position and table, and every lane past the runs an in-bounds position.

The band kernel reads keypoints run by run instead, in 64-wide chunks whose
lanes past a run's end read the entries after it: every entry must be tested
once with its own table, and no read may pass the 64 keypoints kept after the
last table.
"""
import numpy as np
import pytest

N_TABLES = 6


def runs_of(lens, n, rng):
    """Bucket starts b_t (within table t's n entries) for run lengths lens."""
    return [int(rng.integers(0, n - L + 1)) for L in lens]


def truth(lens, b, n):
    """Entry position and table of every candidate, by definition."""
    pos, tab = [], []
    for t, (L, bt) in enumerate(zip(lens, b)):
        for i in range(L):
            pos.append(t * n + bt + i)
            tab.append(t)
    return np.array(pos, np.int64), np.array(tab, np.int64)


def setup_ordinal(lens, b, n, ns):
    """The tile setup of the masked kernels: run table words by ordinal,
    chunk masks (2 words per chunk), packed start counts."""
    qt = [0] * (8 + 2 * ns)
    acc = cnt = pre = 0
    P = [0] * 6
    for t in range(N_TABLES):
        L, bt = lens[t], b[t]
        start = acc
        cu = (t * n + bt - start) & 0xFFFFFFFF
        if t > 0:
            P[t - 1] = start if (L != 0 and cnt != 0) else 0xFFFFFFFF
        if L != 0:
            qt[cnt] = ((cu << 10) | (8 * t)) & 0xFFFFFFFF
            if cnt != 0 and start <= 64 * ns:
                w = 8 + ((start - 1) >> 5)
                qt[w] |= 1 << ((start - 1) & 31)
            if cnt != 0:
                for bnd in range(1, ns):
                    pre += int(start <= 64 * bnd) << (3 * (bnd - 1))
            cnt += 1
        acc += L
    P[5] = acc
    qt[6] = pre  # (the key bytes 4-5 sit in bits 16-31 and are not read here)
    return qt, P


def mbcnt(mask64, lane, base):
    return base + bin(mask64 & ((1 << lane) - 1)).count("1")


def gather_ordinal(qt, P, ns):
    """Byte offset (16 B per entry) and 8t of every lane of the C chunks."""
    total = P[5]
    C = (total + 63) >> 6
    assert 1 <= C <= ns
    pre = qt[6]
    out = []
    for u in range(C):
        sm = qt[8 + 2 * u] | (qt[9 + 2 * u] << 32)
        o0 = 0 if u == 0 else (pre >> (3 * (u - 1))) & 7
        for lane in range(64):
            e = 64 * u + lane
            live = u + 1 < C or e < total
            o = mbcnt(sm, lane, o0)
            cw = qt[o if live else 0]
            boff = (cw >> 6) + ((e << 4) if live else 0)
            out.append((e, live, boff & 0xFFFFFFFF, cw & 63))
    return out


def setup_by_table(lens, b, n):
    qt = [0] * 8
    acc = 0
    P = [0] * 6
    for t in range(N_TABLES):
        start = acc
        qt[t] = (t * n + b[t] - start) & 0xFFFFFFFF
        if t > 0:
            P[t - 1] = start
        acc += lens[t]
    P[5] = acc
    return qt, P


def entry_pos_by_table(e, qt, P):
    ec = e if e < P[5] else 0
    o = sum(int(ec >= p) for p in P[:5])
    return ec + qt[o], 8 * o


def layouts(rng, n, cap):
    """Edge cases then random run lengths, total at most cap."""
    fixed = [[0, 0, 0, 0, 0, 1], [1, 0, 0, 0, 0, 0], [0, 0, 64, 0, 0, 0], [64, 64, 64, 64, 0, 0],
             [0, 63, 1, 0, 64, 0], [65, 0, 0, 0, 0, 0], [1, 1, 1, 1, 1, 1], [0, 0, 0, 0, 0, 0]]
    for f in fixed:
        if sum(f) <= cap:
            yield f
    for _ in range(400):
        k = rng.integers(0, 3, N_TABLES)  # many empty and short runs
        lens = np.where(k == 0, 0, np.where(k == 1, rng.integers(1, 8, N_TABLES), rng.integers(1, cap // 3 + 2, N_TABLES)))
        while lens.sum() > cap:
            lens[rng.integers(0, N_TABLES)] //= 2
        yield [int(x) for x in lens]
    # run starts exactly on chunk boundaries
    for s in range(1, cap // 64):
        yield [64 * s, 0, cap - 64 * s, 0, 0, 0]
        yield [0, 64 * s - 1, 1, 0, cap - 64 * s, 0]


@pytest.mark.parametrize("ns", [4, 6])
def test_ordinal_addressing(ns):
    rng = np.random.default_rng(ns)
    for n in (300, 9001, 14000):
        cap = 64 * ns
        for lens in layouts(rng, n, cap):
            if max(lens) > n:
                continue
            total = sum(lens)
            b = runs_of(lens, n, rng)
            if total == 0:
                continue  # no chunk is read
            pos, tab = truth(lens, b, n)
            qt, P = setup_ordinal(lens, b, n, ns)
            for e, live, boff, w8 in gather_ordinal(qt, P, ns):
                assert boff % 16 == 0 and 0 <= boff // 16 < N_TABLES * n, (lens, e)
                if live and e < total:
                    assert boff // 16 == pos[e] and w8 == 8 * tab[e], (ns, n, lens, b, e)


def test_by_table_addressing():
    rng = np.random.default_rng(8)
    for n in (300, 20000, 65535):
        for lens in layouts(rng, n, 3000):
            if max(lens) > n or sum(lens) == 0:
                continue
            b = runs_of(lens, n, rng)
            pos, tab = truth(lens, b, n)
            qt, P = setup_by_table(lens, b, n)
            total = sum(lens)
            for e in range(total + 70):
                p, w8 = entry_pos_by_table(e, qt, P)
                assert 0 <= p < N_TABLES * n
                if e < total:
                    assert p == pos[e] and w8 == 8 * tab[e], (n, lens, e)


def test_run_words_fit_32_bits():
    """C << 10 stays below 2^32 for the largest image (C <= 6 n)."""
    n = 65535
    assert ((6 * n) << 10) < 2**32


def band_pass_reads(lens, b, n):
    """The band kernel's band pass, as it addresses keypoints: the run of
    table t starts at entry rb = t*n + b_t; the first 64 entries of every run
    are read as one chunk (lane l at rb + l), then 64 more at a time while
    the run lasts (lane l at rb + i0 + l); a lane tests its entry only if
    i0 + l < the run's length.  Returns every read position and the
    (position, table) pairs tested."""
    reads, tested = [], []
    for t in range(N_TABLES):
        rb, rl = t * n + b[t], lens[t]
        i0 = 0
        while True:
            for lane in range(64):
                p = rb + i0 + lane
                reads.append(p)
                if i0 + lane < rl:
                    tested.append((p, t))
            i0 += 64
            if i0 >= rl:
                break
    return reads, tested


def test_band_pass_addressing():
    """Every bucket entry of the query's six runs is tested once with its own
    table, and no read goes more than 64 keypoints past the last table: the
    band call keeps 512 bytes (64 keypoints of 8 bytes) after its tables."""
    rng = np.random.default_rng(11)
    for n in (1, 64, 300, 12000, 65535):
        for lens in layouts(rng, n, 3000):
            if max(lens) > n:
                continue
            b = runs_of(lens, n, rng)
            pos, tab = truth(lens, b, n)
            reads, tested = band_pass_reads(lens, b, n)
            assert min(reads) >= 0 and max(reads) < N_TABLES * n + 64, (n, lens, b)
            assert sorted(tested) == sorted(zip(pos.tolist(), tab.tolist())), (n, lens, b)
            # survivors go to the LDS list as (8t << 24) | pos
            assert N_TABLES * n + 64 < 2**24
    # the keypoint byte offset (pos << 3) of the largest image fits 32 bits
    assert ((N_TABLES * 65535 + 64) << 3) < 2**32
