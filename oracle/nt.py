"""Number theory for the oracle's BGV: primality, the RNS prime chain, roots
of unity.  TEST INFRASTRUCTURE ONLY; written independently of the library.

Prime chain (reading; the paper uses HElib's chain of a given bit budget):
every prime q satisfies q = 1 mod 2N t, so the negacyclic transform exists
mod q and dropping q in a modulus switch leaves the plaintext unchanged
(q^-1 = 1 mod t).  Candidates are k (2N t) + 1 scanned downward in k, each
list below an exclusive integer bound:
  1. special primes: the first ``alpha`` below special_max;
  2. data primes q_1 > q_2 > ... > q_L: the first L below data_max not
     already taken;
  3. q_0: the first below q0_max not already taken.
A modulus switch drops the highest-index data prime first.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

MR_WITNESSES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve primes as witnesses (exact below 3.18e23, far above 2^64)."""
    if n < 2:
        return False
    for p in MR_WITNESSES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in MR_WITNESSES:
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


def primes_below(bound: int, modulus: int, count: int, taken: set) -> List[int]:
    out = []
    k = (bound - 2) // modulus
    while len(out) < count:
        if k <= 0:
            raise ValueError(f"not enough primes = 1 mod {modulus} below {bound}")
        cand = k * modulus + 1
        if cand < bound and cand not in taken and is_prime(cand):
            out.append(cand)
        k -= 1
    return out


@dataclass
class Chain:
    log_n: int
    t: int
    data: List[int]        # q_0, q_1, ..., q_L
    special: List[int]     # p_0, ..., p_{alpha-1}

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def L(self) -> int:
        return len(self.data) - 1

    @property
    def alpha(self) -> int:
        return len(self.special)

    def all_primes(self) -> List[int]:
        return self.data + self.special

    def total_bits(self) -> float:
        import math
        return sum(math.log2(p) for p in self.all_primes())


def make_chain(log_n: int, t: int, n_data: int, q0_max: int, data_max: int,
               alpha: int, special_max: int) -> Chain:
    n = 1 << log_n
    modulus = 2 * n * t
    taken: set = set()
    special = primes_below(special_max, modulus, alpha, taken)
    taken.update(special)
    mids = primes_below(data_max, modulus, n_data - 1, taken)
    taken.update(mids)
    q0 = primes_below(q0_max, modulus, 1, taken)
    return Chain(log_n, t, q0 + mids, special)


def prime_factors(n: int) -> List[int]:
    out, p = [], 2
    while p * p <= n:
        if n % p == 0:
            out.append(p)
            while n % p == 0:
                n //= p
        p += 1
    if n > 1:
        out.append(n)
    return out


def root_of_unity(order: int, q: int) -> int:
    """Smallest element of multiplicative order exactly ``order`` mod prime q
    found from generators g = 2, 3, ... (order must divide q - 1)."""
    assert (q - 1) % order == 0
    fac = prime_factors(order)
    for g in range(2, q):
        r = pow(g, (q - 1) // order, q)
        if all(pow(r, order // f, q) != 1 for f in fac):
            return r
    raise ValueError("no root found")


def slot_root(t: int, n: int) -> int:
    """zeta = 3^((t-1)/2N) mod t: the 2N-th root of unity mod t that fixes
    the slot order (3 generates the multiplicative group mod 65537)."""
    assert (t - 1) % (2 * n) == 0
    z = pow(3, (t - 1) // (2 * n), t)
    assert pow(z, n, t) == t - 1
    return z
