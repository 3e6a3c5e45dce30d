"""Host-side checks of the split-precision kernel's LDS layout: rows of 32
bfloat16 (four 16-byte chunks) whose chunk index is XOR-ed with
g(row) = ((row >> 2) ^ (row >> 1)) mod 4.  The matrix-core fragment reads
(lane l: row l mod 16 of a 16-row tile, chunk l // 16) and the staging writes
(thread e: row e // 4, chunk e mod 4) must fall on distinct 16-byte bank
slots within 8, 16 and 32 consecutive lanes (the LDS bank-conflict counter
reads zero for both patterns on gfx950 with this g; the earlier
((row >> 1) mod 4) ^ ((row >> 3) mod 2), distinct within 16 lanes only,
measured two-way conflicts on the fragment reads)."""


def g(row):
    return ((row >> 2) ^ (row >> 1)) & 3


def slot(row, chunk, nslots):
    # 16-byte slot of the swizzled chunk; a row is 64 bytes (4 slots)
    return (4 * row + (chunk ^ g(row))) % nslots


def _distinct(addrs, group, nslots):
    return all(len({slot(r, c, nslots) for r, c in addrs[i:i + group]}) == group
               for i in range(0, len(addrs), group))


def test_fragment_reads_conflict_free():
    for base in range(0, 256, 16):            # fragment tiles start on 16-row boundaries
        lanes = [(base + (l & 15), l >> 4) for l in range(64)]
        assert _distinct(lanes, 16, 16)
        assert _distinct(lanes, 8, 8)
        assert _distinct(lanes, 32, 32)


def test_staging_writes_conflict_free():
    for first in range(0, 1024, 64):          # one wavefront's items e = first .. first + 63
        lanes = [(e // 4, e % 4) for e in range(first, first + 64)]
        assert _distinct(lanes, 16, 16)
        assert _distinct(lanes, 8, 8)
        assert _distinct(lanes, 32, 32)


def test_unswizzled_layout_would_conflict():
    # the check has teeth: without the XOR, rows 0 and 4 of a fragment read
    # share banks (row pitch 64 bytes = 16 banks)
    lanes = [(l & 15, l >> 4) for l in range(16)]
    assert len({(4 * r + c) % 16 for r, c in lanes}) < 16
