"""Seed derivation: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) turns (master seed, cell index)
into an independent 64-bit seed per r-cell, which seeds a numpy PCG64 generator."""
import numpy as np

_MASK = (1 << 64) - 1


def splitmix64(state: int) -> tuple[int, int]:
    """One SplitMix64 step: returns (output, new_state)."""
    state = (state + 0x9E3779B97F4A7C15) & _MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31), state


def cell_seed(master: int, cell: int) -> int:
    """Per-cell seed: SplitMix64 output after (cell + 1) steps from the master seed."""
    state = master & _MASK
    out = 0
    for _ in range(cell + 1):
        out, state = splitmix64(state)
    return out


def generator(master: int, cell: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(cell_seed(master, cell)))
