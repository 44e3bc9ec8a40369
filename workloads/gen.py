"""Seeded synthetic arrays: random RNS limbs, slot vectors, images.

Inputs only.  Nothing here performs homomorphic arithmetic; values are drawn
with numpy's PCG64 from an explicit seed so the oracle and the GPU library can
be handed identical inputs.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(int(seed)))


def random_limbs(seed: int, mods, N: int) -> np.ndarray:
    """[len(mods)][N] uint64, limb l uniform in [0, mods[l])."""
    g = rng(seed)
    return np.stack([g.integers(0, int(m), N, dtype=np.uint64) for m in mods])


def random_ct(seed: int, q, level: int, N: int, npoly: int = 2) -> np.ndarray:
    """A ciphertext-shaped array [npoly][level+1][N] of uniform residues.

    Uniform residues are what a fresh RLWE ciphertext looks like to anyone
    without the key, so they exercise every code path of the evaluator."""
    g = rng(seed)
    return np.stack([np.stack([g.integers(0, int(q[l]), N, dtype=np.uint64) for l in range(level + 1)])
                     for _ in range(npoly)])


def uniform_slots(seed: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, n)


def images(seed: int, batch: int, C: int, H: int, W: int) -> np.ndarray:
    """Image-shaped inputs with pixels uniform in [0, 1] (stand-ins for CIFAR /
    Tiny-ImageNet shaped data; no dataset item is used)."""
    return rng(seed).uniform(0.0, 1.0, (batch, C, H, W))
