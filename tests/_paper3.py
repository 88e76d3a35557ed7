"""D3Q19 lattice as the paper fixes it, for the 3-D pins (fixtures under tests/golden)."""
import numpy as np

from tests._paper import matrix

# Velocities: rows 2-4 of C in Eq. (86) are c_x, c_y, c_z of the columns.
_C = matrix("eq86_C_d3q19.txt")
CX, CY, CZ = _C[1], _C[2], _C[3]
# Weights are not printed; the printed R of Eq. (80) fixes them (R_ii = 3 w_i |c_i|^2 (k1 - k0),
# checked in test_oracle_d3q19): 1/3 at rest, 1/18 on the axes, 1/36 on the face diagonals.
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
C3 = np.stack([CX, CY, CZ], axis=1)


def R_general(K1: np.ndarray, k0: float) -> np.ndarray:
    """Eq. (77): R_ij = w_i c_i . [(K1 - k0 I) c_j] / c_s^2 on D3Q19."""
    return 3.0 * W[:, None] * (C3 @ (K1 - k0 * np.eye(3)) @ C3.T)


def P_general(K2: np.ndarray, k0: float) -> np.ndarray:
    """Eq. (77): P_ij = w_i (c_i c_i - c_s^2 I) : [(K2 - k0 Ihat) o (c_j c_j)] / (2 c_s^4) on D3Q19."""
    out = np.zeros((19, 19))
    Q = K2 - k0 * np.ones((3, 3))
    for i in range(19):
        Hi = np.outer(C3[i], C3[i]) - np.eye(3) / 3.0
        for j in range(19):
            out[i, j] = W[i] * np.sum(Hi * (Q * np.outer(C3[j], C3[j]))) * 4.5
    return out
