"""Counter-based sketch matrix (oracle).

The paper's compression cites a randomised algorithm but fixes no random
source. Both the oracle and the HIP library implement the same counter-based
rule from the published SplitMix64 generator (Steele, Lea & Flood, OOPSLA
2014): one output step maps a 64-bit state z to
    z += 0x9E3779B97F4A7C15
    z  = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z  = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out = z ^ (z >> 31)            (all arithmetic mod 2^64).
Entry (i, j) of the N x l sketch uses the state seed XOR (i*l + j) and its two
low output bits b0, b1:  Omega_ij = ((1 - 2 b0) + i (1 - 2 b1)) / sqrt(2).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state: np.ndarray) -> np.ndarray:
    z = np.asarray(state, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def sketch(seed: int, n: int, ell: int) -> np.ndarray:
    """The N x l complex sketch matrix."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(ell, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        idx = i * np.uint64(ell) + j
    z = splitmix64(np.uint64(seed) ^ idx)
    b0 = (z & np.uint64(1)).astype(np.float64)
    b1 = ((z >> np.uint64(1)) & np.uint64(1)).astype(np.float64)
    return ((1.0 - 2.0 * b0) + 1j * (1.0 - 2.0 * b1)) / np.sqrt(2.0)
