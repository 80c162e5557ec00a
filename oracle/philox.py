"""Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) in plain Python -- oracle, test
infrastructure only.  Written from the published round function: each of ten rounds
multiplies counter words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 (32x32 -> 64 bits) and
mixes the halves with the other counter words and the key; the key is bumped by
0x9E3779B9 / 0xBB67AE85 between rounds.  Pinned by the known-answer vectors that the
authors publish with their library (tests/golden/philox4x32_10_kat.json)."""

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return (c0, c1, c2, c3)
