"""Radical inversion in prime bases and the Halton sequence (Sec. 2.2) — test infrastructure.

phi_{b,sigma}(i) = sum_k sigma_b(a_k(i)) b^(-k-1) for the base-b digits a_k of i (Sec. 2.2).
The index is first reduced modulo the largest power of b that fits in 32 bits (the listing's
`max_powers`), and the 32-bit result is floor(2^32 phi) — the integer the listing forms by
exact division before map_u32_to_unifloat.

Digit permutations sigma_b:
  * identity;
  * Faure's recursive permutations (Sec. 2.2): sigma_2 = (0, 1); for even b, 2 sigma_{b/2}
    followed by 2 sigma_{b/2} + 1; for odd b, sigma_{b-1} with every value >= (b-1)/2 raised
    by one and (b-1)/2 inserted in the middle;
  * linear scrambling sigma(a) = (f a) mod b with a multiplier f per dimension (the paper's
    multiplier table is not printed, so f is an input).
The Halton sequence takes the j-th prime as the base of dimension j.
"""

from fractions import Fraction

import numpy as np


def primes(count):
    """The first `count` primes, by trial division."""
    out = []
    n = 2
    while len(out) < count:
        if all(n % p for p in out if p * p <= n):
            out.append(n)
        n += 1
    return out


def max_power(b):
    """Largest power of b that fits in 32 bits (b^m <= 2^32 - 1)."""
    q = b
    while q * b <= 0xFFFFFFFF:
        q *= b
    return q


def faure_permutation(b):
    """Faure's permutation sigma_b as a list (definition in the module docstring)."""
    if b == 1:
        return [0]
    if b == 2:
        return [0, 1]
    if b % 2 == 0:
        half = faure_permutation(b // 2)
        return [2 * v for v in half] + [2 * v + 1 for v in half]
    c = (b - 1) // 2
    prev = [v + 1 if v >= c else v for v in faure_permutation(b - 1)]
    return prev[:c] + [c] + prev[c:]


def digit_permutation(b, mode, factor=1):
    if mode == "identity":
        return list(range(b))
    if mode == "faure":
        return faure_permutation(b)
    if mode == "linear":
        return [(factor * a) % b for a in range(b)]
    raise ValueError(mode)


def radical_inverse_u32(i, b, sigma=None):
    """floor(2^32 phi_{b,sigma}(i mod max_power(b))), exact (rationals)."""
    i = int(i) % max_power(b)
    sigma = sigma if sigma is not None else list(range(b))
    phi = Fraction(0)
    scale = Fraction(1, b)
    while i:
        i, a = divmod(i, b)
        phi += sigma[a] * scale
        scale /= b
    return (phi.numerator << 32) // phi.denominator


def halton_points(s, first, n, mode="identity", factors=None):
    """u32 [s][n]: component j of points i in [first, first + n), base = the j-th prime."""
    bases = primes(s)
    out = np.zeros((s, n), dtype=np.uint32)
    for j, b in enumerate(bases):
        sigma = digit_permutation(b, mode, 1 if factors is None else int(factors[j]))
        for k in range(n):
            out[j, k] = radical_inverse_u32(first + k, b, sigma)
    return out
