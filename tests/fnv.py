"""FNV-1a 64 (Fowler, Noll, Vo) over many byte strings at once (numpy, test side)."""
import numpy as np

BASIS = np.uint64(0xCBF29CE484222325)
PRIME = np.uint64(0x100000001B3)


def fnv1a64(msgs: np.ndarray) -> np.ndarray:
    """msgs uint8 [N, L] -> uint64 [N]."""
    msgs = np.ascontiguousarray(msgs, np.uint8)
    h = np.full(msgs.shape[0], BASIS, np.uint64)
    with np.errstate(over="ignore"):
        for j in range(msgs.shape[1]):
            h ^= msgs[:, j].astype(np.uint64)
            h *= PRIME
    return h
