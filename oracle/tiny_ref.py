"""Pure-Python big-integer restatement of the engines -- TEST INFRASTRUCTURE.

Used only by tests to cross-check the C oracle on tiny inputs with an
arithmetic that cannot overflow or truncate.  The MRG jump here uses plain
3x3 matrix powers, a different algorithm from the C oracle's polynomial
method ([L99] companion matrices; [L02] substream spacing 2^76).
"""
from __future__ import annotations

M1 = 2**32 - 209
M2 = 2**32 - 22853

# Companion matrices acting on (x[n-3], x[n-2], x[n-1]) ([L99]).
A1 = ((0, 1, 0), (0, 0, 1), (M1 - 810728, 1403580, 0))
A2 = ((0, 1, 0), (0, 0, 1), (M2 - 1370589, 0, 527612))

PHILOX32 = dict(w=32, m=(0xD2511F53, 0xCD9E8D57), weyl=(0x9E3779B9, 0xBB67AE85))


def philox(ctr, key, rounds=10, w=32, m=PHILOX32["m"], weyl=PHILOX32["weyl"]):
    mask = (1 << w) - 1
    x = [int(c) & mask for c in ctr]
    k = [int(key[0]) & mask, int(key[1]) & mask]
    for r in range(rounds):
        if r:
            k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
        p0 = m[0] * x[0]
        p1 = m[1] * x[2]
        x = [(p1 >> w) ^ x[1] ^ k[0], p1 & mask, (p0 >> w) ^ x[3] ^ k[1], p0 & mask]
    return x


def philox_words(seed: int, pos: int, n: int):
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = []
    for i in range(n):
        p = (pos + i) % (1 << 130)
        b = p >> 2
        ctr = [(b >> (32 * j)) & 0xFFFFFFFF for j in range(4)]
        out.append(philox(ctr, key)[p & 3])
    return out


def mrg_seed(seed: int):
    return [(seed & 0xFFFFFFFF) % M1, 1, 1, ((seed >> 32) & 0xFFFFFFFF) % M2, 1, 1]


def mrg_step(st):
    x1 = (1403580 * st[1] - 810728 * st[0]) % M1
    x2 = (527612 * st[5] - 1370589 * st[3]) % M2
    new = [st[1], st[2], x1, st[4], st[5], x2]
    y = x1 - x2 if x1 > x2 else x1 - x2 + M1
    return y, new


def mrg_words(st, n):
    out = []
    st = [int(v) for v in st]
    for _ in range(n):
        y, st = mrg_step(st)
        out.append(y)
    return out, st


def matmul(a, b, m):
    return tuple(tuple(sum(a[i][k] * b[k][j] for k in range(3)) % m for j in range(3))
                 for i in range(3))


def matpow(a, n, m):
    r = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    while n:
        if n & 1:
            r = matmul(r, a, m)
        a = matmul(a, a, m)
        n >>= 1
    return r


def matvec(a, v, m):
    return [sum(a[i][j] * v[j] for j in range(3)) % m for i in range(3)]


def mrg_skip(st, n):
    st = [int(v) for v in st]
    return matvec(matpow(A1, n, M1), st[:3], M1) + matvec(matpow(A2, n, M2), st[3:], M2)
