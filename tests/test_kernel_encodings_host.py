"""Host checks of the integer encodings the HIP kernels rely on (no GPU).

* detect, packed level 0: a lane builds 16-bit keys value << 8 | (row count
  << lc | column in window) from 4-pixel words with two byte permutes, keeps
  the extremes with packed 16-bit max/min and adds the pixels with a
  sum-of-absolute-differences; expanded at the end, its extremes and sum must
  equal the scalar keys value << 16 | row << 8 | column of the tile (Eq. 1 in
  integers) over the same pixels. Emulated here with the byte-select rule of
  v_perm_b32 (selector bytes 0-3 pick bytes of the second operand, 4-7 of
  the first).
* matchers: inserting two keys x, y into a sorted pair k1 <= k2 at once gives
  the two smallest of the four as min3(k1, x, y) and min(k2, med3(k1, x, y)).
"""
import itertools

import numpy as np


def perm(s0: int, s1: int, sel: int) -> int:
    data = (s0 << 32) | s1
    out = 0
    for i in range(4):
        b = (sel >> (8 * i)) & 255
        out |= ((data >> (8 * b)) & 255) << (8 * i)
    return out


def pk(a: int, b: int, f) -> int:
    return f(a & 0xFFFF, b & 0xFFFF) | (f(a >> 16, b >> 16) << 16)


def level0_geometry(L0: int, T: int):
    nw = (T // L0) ** 2
    G = 1
    while G < 64 and 2 * G <= L0 and 2 * G * nw <= 256:
        G *= 2
    rows_pl = (L0 + G - 1) // G
    lc = 0
    while (1 << lc) < L0:
        lc += 1
    rb = 0
    while (1 << rb) < rows_pl:
        rb += 1
    return G, lc, rb


def scalar_lane(pix, r0, r1, c0, c1, g, G):
    kmax, kmin, s = 0, 0xFFFFFFFF, 0
    for r in range(r0 + g, r1, G):
        for c in range(c0, c1):
            v = int(pix[r, c])
            key = (v << 16) | (r << 8) | c
            kmax, kmin, s = max(kmax, key), min(kmin, key), s + v
    return kmax, kmin, s


def packed_lane(pix, r0, r1, c0, c1, g, G, lc):
    pmax, pmin, s, ri = 0, 0xFFFFFFFF, 0, 0
    for r in range(r0 + g, r1, G):
        cb = ((ri << lc) * 0x01010101 + 0x03020100) & 0xFFFFFFFF
        c = c0
        while c + 4 <= c1:
            w4 = sum(int(pix[r, c + i]) << (8 * i) for i in range(4))
            lo, hi = perm(w4, cb, 0x05010400), perm(w4, cb, 0x07030602)
            pmax = pk(pmax, pk(lo, hi, max), max)
            pmin = pk(pmin, pk(lo, hi, min), min)
            s += sum((w4 >> (8 * i)) & 255 for i in range(4))
            c += 4
            cb = (cb + 0x04040404) & 0xFFFFFFFF
        while c < c1:
            v = int(pix[r, c])
            k = (v << 8) | ((ri << lc) | (c - c0))
            pmax, pmin, s = pk(pmax, k | (k << 16), max), pk(pmin, k | (k << 16), min), s + v
            c += 1
        ri += 1
    if ri == 0:
        return 0, 0xFFFFFFFF, 0
    km, kn = max(pmax & 0xFFFF, pmax >> 16), min(pmin & 0xFFFF, pmin >> 16)
    msk = (1 << lc) - 1

    def expand(k):
        return ((k >> 8) << 16) | ((r0 + g + ((k & 255) >> lc) * G) << 8) | (c0 + (k & msk))
    return expand(km), expand(kn), s


def test_detect_packed_level0_keys():
    rng = np.random.default_rng(0)
    checked = 0
    for L0 in (4, 8, 12, 16, 20, 24, 32, 64, 128):
        T = 128 if 128 % L0 == 0 else L0 * (128 // L0)
        G, lc, rb = level0_geometry(L0, T)
        assert L0 % 4 == 0 and lc + rb <= 8          # the packed form applies
        for trial in range(40):
            th, tw = int(rng.integers(1, T + 1)), int(rng.integers(1, T + 1))
            pix = rng.integers(0, int(rng.choice([2, 3, 256])), (T, T))
            n0 = T // L0
            wy, wx = int(rng.integers(0, n0)), int(rng.integers(0, n0))
            r0, c0 = wy * L0, wx * L0
            if not (r0 < th and c0 < tw):
                continue
            r1, c1 = min(r0 + L0, th), min(c0 + L0, tw)
            for g in range(G):
                assert packed_lane(pix, r0, r1, c0, c1, g, G, lc) == \
                    scalar_lane(pix, r0, r1, c0, c1, g, G)
                checked += 1
    assert checked > 1000


def test_pair_insertion_identity():
    for k1, k2, x, y in itertools.product(range(6), repeat=4):
        if k1 > k2:
            continue
        s = sorted([k1, k2, x, y])
        assert min(k1, x, y) == s[0]
        assert min(k2, sorted([k1, x, y])[1]) == s[1]
