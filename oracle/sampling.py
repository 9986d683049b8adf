"""Randomness of keys and encryptions.  TEST INFRASTRUCTURE ONLY.

Every random draw comes from one SHAKE-256 stream (FIPS 202, here Python's
hashlib) per (seed, domain, object, limb):
    stream = SHAKE-256(seed[32] || domain (ASCII) || le64(object) || le32(limb))
read from its start.  Samplers:
  * uniform mod q: next 8 bytes little-endian, masked to bitlen(q) bits,
    accepted if < q;
  * ternary: next byte b; b = 255 is rejected; b mod 3 = 0, 1, 2 -> 0, 1, -1;
  * error: centered binomial with eta = 21: next 6 bytes little-endian as a
    48-bit word w, e = popcount(w & (2^21-1)) - popcount((w >> 21) & (2^21-1)).
Ternary and error polynomials are drawn once per polynomial (limb field 0);
uniform polynomials are drawn per limb with the prime's global index as limb.
"""
from __future__ import annotations

import hashlib

import numpy as np


def stream(seed: bytes, domain: str, obj: int, limb: int, nbytes: int) -> bytes:
    assert len(seed) == 32
    msg = seed + domain.encode("ascii") + int(obj).to_bytes(8, "little") + int(limb).to_bytes(4, "little")
    return hashlib.shake_256(msg).digest(nbytes)


def uniform(seed: bytes, domain: str, obj: int, limb: int, q: int, n: int) -> np.ndarray:
    bits = q.bit_length()
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    need = n
    nbytes = 8 * (n + n // 8 + 64)
    while True:
        words = np.frombuffer(stream(seed, domain, obj, limb, nbytes), dtype="<u8") & mask
        acc = words[words < np.uint64(q)]
        if len(acc) >= need:
            return acc[:need].astype(np.uint64)
        nbytes *= 2


def ternary(seed: bytes, domain: str, obj: int, n: int) -> np.ndarray:
    nbytes = n + n // 16 + 64
    while True:
        b = np.frombuffer(stream(seed, domain, obj, 0, nbytes), dtype=np.uint8)
        b = b[b != 255]
        if len(b) >= n:
            v = (b[:n] % 3).astype(np.int64)
            v[v == 2] = -1
            return v
        nbytes *= 2


def cbd21(seed: bytes, domain: str, obj: int, n: int) -> np.ndarray:
    raw = np.frombuffer(stream(seed, domain, obj, 0, 6 * n), dtype=np.uint8).reshape(n, 6).astype(np.uint64)
    w = np.zeros(n, dtype=np.uint64)
    for i in range(6):
        w |= raw[:, i] << np.uint64(8 * i)
    lo = w & np.uint64((1 << 21) - 1)
    hi = (w >> np.uint64(21)) & np.uint64((1 << 21) - 1)

    def popcount(x):
        c = np.zeros(n, dtype=np.int64)
        for b in range(21):
            c += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
        return c
    return popcount(lo) - popcount(hi)
