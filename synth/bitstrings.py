"""Seeded bitstring batches.

Packing: uint64, bit q holds the value of qubit q (qubit 0 in the LSB).  A
printed string lists qubit 0 first, as the paper prints "100" for q0=1.

Samples from a real device at low fidelity are nearly uniform, so uniform
draws stand in for experimental samples.  The "prefix" batch fixes the first
`n_fixed` qubits (ids 0..n_fixed-1) to one seeded random value and draws the
rest uniformly, so the batch shares the sub-contractions that only see the
fixed qubits.
"""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_bitstrings(n: int, k: int, seed: int) -> np.ndarray:
    if not 1 <= n <= 64:
        raise ValueError("n must be in [1, 64]")
    rng = _rng(seed)
    out = np.zeros(k, dtype=np.uint64)
    # Draw 32 bits at a time so that any n <= 64 is covered.
    lo = rng.integers(0, 1 << 32, size=k, dtype=np.uint64)
    hi = rng.integers(0, 1 << 32, size=k, dtype=np.uint64)
    out = lo | (hi << np.uint64(32))
    if n < 64:
        out &= np.uint64((1 << n) - 1)
    return out


def prefix_bitstrings(n: int, k: int, n_fixed: int, seed: int) -> np.ndarray:
    if not 0 <= n_fixed <= n:
        raise ValueError("n_fixed must be in [0, n]")
    rng = _rng(seed)
    fixed = int(rng.integers(0, 1 << n_fixed)) if n_fixed else 0
    free_bits = n - n_fixed
    vals = uniform_bitstrings(max(free_bits, 1), k, seed + 7919)
    if free_bits == 0:
        vals[:] = 0
    return (vals << np.uint64(n_fixed)) | np.uint64(fixed)


def config_bitstrings(name: str, n: int) -> np.ndarray:
    if name == "small_4x5_m8":
        return uniform_bitstrings(n, 1000, 2001)
    if name == "medium_6x6_m12":
        return prefix_bitstrings(n, 10_000, 20, 2002)
    if name == "share_53q_m14":
        return uniform_bitstrings(n, 300_000, 2005)
    raise KeyError(name)


def bits_to_str(x: int, n: int) -> str:
    return "".join("1" if (int(x) >> q) & 1 else "0" for q in range(n))
