"""Second, independent Philox4x32-10 in pure Python (test infrastructure only).

Written from the round function and key schedule published by Salmon, Moraes,
Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11): each of
the ten rounds multiplies counter words 0 and 2 by two fixed odd constants,
swaps and xors the high halves with the other words and the round key, and
the key is advanced by the two Weyl increments between rounds.  The test suite
checks this copy and the C copy against each other and against the published
known-answer vectors.
"""

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def _mulhilo(a: int, b: int):
    p = a * b
    return (p >> 32) & MASK, p & MASK


def philox4x32(key, ctr, rounds: int = 10):
    k0, k1 = key[0] & MASK, key[1] & MASK
    x0, x1, x2, x3 = (c & MASK for c in ctr)
    for _ in range(rounds):
        h0, l0 = _mulhilo(M0, x0)
        h1, l1 = _mulhilo(M1, x2)
        x0, x1, x2, x3 = h1 ^ x1 ^ k0, l1, h0 ^ x3 ^ k1, l0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return [x0, x1, x2, x3]
