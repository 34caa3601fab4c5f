"""Independent brute-force references on Python integers, for pinning the CPU
oracle on tiny rings.  Nothing here is shared with the oracle or the HIP path:
schoolbook negacyclic products, CRT with exact integer rounding, direct
polynomial substitution, and a decimal-arithmetic evaluation of the encoding
sum.
"""
from __future__ import annotations

from decimal import Decimal, getcontext


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def negacyclic(a, b, N, mod=None):
    """Schoolbook product in Z[X]/(X^N + 1) (optionally reduced mod `mod`)."""
    out = [0] * N
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            k = i + j
            if k < N:
                out[k] += ai * bj
            else:
                out[k - N] -= ai * bj
    if mod is not None:
        out = [x % mod for x in out]
    return out


def substitute(a, g, N, mod):
    """a(X^g) mod (X^N + 1, mod), by direct substitution."""
    out = [0] * N
    for j, aj in enumerate(a):
        e = j * g
        sign = -1 if (e // N) % 2 else 1
        out[e % N] = (out[e % N] + sign * aj) % mod
    return out


def crt(residues, moduli):
    """Integer in [0, prod) with the given residues."""
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += r * Mi * pow(Mi, -1, m)
    return x % M, M


def centered(x, q):
    x %= q
    return x - q if x > q // 2 else x


def round_div(a: int, b: int) -> int:
    """round(a / b) to nearest for odd b > 0 (no ties)."""
    return (2 * a + b) // (2 * b)


def round_half_away(num: Decimal) -> int:
    if num >= 0:
        return int((num + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR"))
    return -int((-num + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR"))


def _pi(prec: int) -> Decimal:
    """pi by Machin's formula in decimal arithmetic."""
    getcontext().prec = prec + 10

    def arctan_inv(x: int) -> Decimal:
        x = Decimal(x)
        total, term, n, sign = Decimal(0), 1 / x, 1, 1
        x2 = x * x
        while True:
            t = term / n
            if t == 0 or abs(t) < Decimal(10) ** (-(prec + 8)):
                break
            total += sign * t
            term /= x2
            n += 2
            sign = -sign
        return total

    return 4 * (4 * arctan_inv(5) - arctan_inv(239))


def _cos(x: Decimal, prec: int) -> Decimal:
    getcontext().prec = prec + 10
    total, term, n = Decimal(1), Decimal(1), 0
    x2 = x * x
    while True:
        n += 2
        term = -term * x2 / (n * (n - 1))
        if abs(term) < Decimal(10) ** (-(prec + 8)):
            break
        total += term
    return total


def encode_exact(z, N: int, scale, prec: int = 60):
    """m_j = (2/N) sum_k z_k cos(pi * (5^k mod 2N) * j / N); returns the
    decimal values scale * m_j (z given as floats, converted exactly)."""
    pi = _pi(prec)
    getcontext().prec = prec + 10
    cos_tab = [_cos(pi * t / N, prec) for t in range(2 * N)]
    e = [pow(5, k, 2 * N) for k in range(N // 2)]
    zs = [Decimal(float(v)) for v in z]
    sc = Decimal(float(scale))
    out = []
    for j in range(N):
        acc = Decimal(0)
        for k in range(len(zs)):
            if zs[k] != 0:
                acc += zs[k] * cos_tab[(e[k] * j) % (2 * N)]
        out.append(sc * acc * 2 / N)
    return out
