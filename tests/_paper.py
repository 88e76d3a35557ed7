"""Readers for the paper fixtures under tests/golden (printed values, cited in each file)."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# D2Q9 velocities and weights as the paper states them (column order of C in Eq. (85);
# weights after Eq. (38)). Independent of the oracle's own tables.
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def matrix(name: str) -> np.ndarray:
    """A printed matrix (rationals allowed), times its printed scalar factor if any is noted."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(Fraction(tok)) for tok in line.split()])
    return np.array(rows)


def table(name: str):
    """Rows of a whitespace table: list of token lists (comments dropped)."""
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def R_general(K1: np.ndarray, k0: float) -> np.ndarray:
    """Eq. (77): R_ij = w_i c_i . [(K1 - k0 I) c_j] / c_s^2."""
    c = np.stack([CX, CY], axis=1)
    M = K1 - k0 * np.eye(2)
    return 3.0 * W[:, None] * (c @ M @ c.T)


def P_general(K2: np.ndarray, k0: float) -> np.ndarray:
    """Eq. (77): P_ij = w_i (c_i c_i - c_s^2 I) : [(K2 - k0 Ihat) o (c_j c_j)] / (2 c_s^4)."""
    c = np.stack([CX, CY], axis=1)
    out = np.zeros((9, 9))
    Q = K2 - k0 * np.ones((2, 2))
    for i in range(9):
        Hi = np.outer(c[i], c[i]) - np.eye(2) / 3.0
        for j in range(9):
            out[i, j] = W[i] * np.sum(Hi * (Q * np.outer(c[j], c[j]))) * 4.5
    return out
