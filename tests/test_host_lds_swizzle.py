"""Host check of the LDS swizzles of the 16-column tile products.

The tile-product kernels stage an RP x RP tile (RP = 8T) row-major in LDS with
the column index XORed by f(i) = M i over GF(2) (masks m_t in
csrc/kernels_block.hip).  With LDS as 64 banks of 4 bytes, one wave
instruction (64 lanes of E bytes) touches at least 64 E / 256 bank rows, so
the best possible is 1 lane per bank group for 4-byte and 2 for 8-byte
elements.  This test rebuilds f from the masks in the source and counts, for
every instruction of the three access patterns (the staging writes of the
T x T lane sub-blocks, the row-pass operand reads A[16s + p][4kb + q] and the
transposed reads A[4kb + q][16s + p]), the largest number of lanes that fall
into one bank group.
"""
import os
import re

import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2501_17656_amd", "csrc", "kernels_block.hip")


def masks():
    text = open(SRC).read()
    body = text[text.index("__device__ __forceinline__ int swz(int i)"):]
    body = body[:body.index("return")]
    out = {}
    # branches in order: RP == 16; RP == 32 && EB == 4; RP == 32; EB == 4 (RP 64); else (RP 64, EB 8)
    blocks = re.findall(r"\{([^{}]*m0 = [^{}]*)\}", body)
    keys = [(16, 4), (32, 4), (32, 8), (64, 4), (64, 8)]
    assert len(blocks) == 5, blocks
    for key, blk in zip(keys, blocks):
        m = dict((int(k), int(v)) for k, v in re.findall(r"m(\d) = (\d+)", blk))
        out[key] = [m.get(t, 0) for t in range(6)]
    out[(16, 8)] = out[(16, 4)]             # the RP = 16 branch serves both widths
    return out


def f_of(mask, i):
    return sum((bin(i & mt).count("1") & 1) << t for t, mt in enumerate(mask))


def worst_conflict(rp, eb, mask):
    T = rp // 8
    nb = 256 // eb                           # bank groups of eb bytes
    writes = [[(T * a + u, T * b + v) for a in range(8) for b in range(8)] for u in range(T) for v in range(T)]
    rows = [[(16 * s + p, 4 * kb + q) for q in range(4) for p in range(16)]
            for s in range(rp // 16) for kb in range(rp // 4)]
    cols = [[(4 * kb + q, 16 * s + p) for q in range(4) for p in range(16)]
            for s in range(rp // 16) for kb in range(rp // 4)]
    worst = 0
    for pattern in (writes, rows, cols):
        for ins in pattern:
            count = {}
            for i, j in ins:
                col = j ^ f_of(mask, i)
                assert 0 <= col < rp
                g = (i * rp + col) % nb
                count[g] = count.get(g, 0) + 1
            worst = max(worst, max(count.values()))
    return worst


# worst lanes per bank group with the swizzle (the minimum is 1 for 4-byte
# and 2 for 8-byte elements), and without it
EXPECTED = {(16, 4): (2, 4), (16, 8): (4, 8), (32, 4): (2, 8), (32, 8): (2, 16), (64, 4): (1, 16),
            (64, 8): (2, 16)}


@pytest.mark.parametrize("rp,eb", sorted(EXPECTED))
def test_swizzle_bank_conflicts(rp, eb):
    mask = masks()[(rp, eb)]
    ideal = max(1, 64 * eb // 256)
    worst = worst_conflict(rp, eb, mask)
    no_swizzle = worst_conflict(rp, eb, [0] * 6)
    assert (worst, no_swizzle) == EXPECTED[(rp, eb)]
    assert ideal <= worst <= 2 * ideal
