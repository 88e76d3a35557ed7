"""Pins of the three-dimensional (D3Q19) oracle against the paper's printed Appendix matrices,
its identities and closed forms (`-m "not gpu"`).

* Eq. (86) C holds the natural moments of Eq. (84); T = H C (Eqs. (87), (89), (91)); Eq. (77)
  reproduces the printed P of Eq. (81) and the printed R of Eq. (80) except one entry (row 3,
  column 8, printed +2: the row of c_2 = -c_1 must be minus the row of c_1, so it is -2); T
  diagonalises R and P (Eq. (93)) and gives the block S_f of Eq. (100) for full K1, K2.
* The oracle's collision is f - (k0 I + R + P) f_neq with those matrices; its equilibrium has the
  moments of Eq. (9) for a general D; G (Eq. (11)) and the source (Eq. (8), Scheme 2) enter as stated.
* Dynamics: the exact one-step map of a Fourier mode (from Eq. (77), Eq. (11), Eq. (38)); its
  hydrodynamic eigenvalue gives the diffusion tensor of Eq. (30); second-order convergence to the
  3-D anisotropic Gaussian hill; the steady slip of half-way bounce-back is that of Eq. (61) and
  vanishes with the k2 of Eq. (62); a uniform state under six equal walls is a fixed point.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import oracle3 as O3
from tests import _paper3 as P3
from tests._paper import matrix


def printed_R():
    R = matrix("eq80_R_d3q19.txt").copy()
    assert R[2, 7] == 2.0  # the printed entry
    R[2, 7] = -2.0         # read as -2 (see the module docstring)
    return R


def test_C_rows_are_natural_moments():
    C = matrix("eq86_C_d3q19.txt")
    order = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 0, 1), (1, 1, 0), (0, 1, 1), (0, 2, 0),
             (0, 0, 2), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 0, 2), (0, 1, 2), (0, 2, 1), (2, 2, 0), (2, 0, 2),
             (0, 2, 2)]
    for r, (o, p, q) in enumerate(order):
        np.testing.assert_array_equal(C[r], P3.CX ** o * P3.CY ** p * P3.CZ ** q)
    # The oracle's own velocity table is the same.
    np.testing.assert_array_equal(O3.CX, P3.CX)
    np.testing.assert_array_equal(O3.CY, P3.CY)
    np.testing.assert_array_equal(O3.CZ, P3.CZ)


def test_printed_T_is_H_times_C():
    C, H, T = matrix("eq86_C_d3q19.txt"), matrix("eq91_H_d3q19.txt"), matrix("eq89_T_d3q19.txt")
    np.testing.assert_allclose(H @ C, T, atol=1e-15)


@pytest.mark.parametrize("k0,k1,k2", [(1.0, 1.25, 0.7), (0.6, 1.9, 1.3), (1.4, 0.5, 1.0)])
def test_eq77_reproduces_printed_R_and_P(k0, k1, k2):
    raw = matrix("eq80_R_d3q19.txt") * (k1 - k0) / 12.0
    R = printed_R() * (k1 - k0) / 12.0
    Pm = matrix("eq81_P_d3q19.txt") * (k2 - k0) / 24.0
    Rg = P3.R_general(k1 * np.eye(3), k0)
    np.testing.assert_allclose(Rg, R, atol=1e-15)
    # Exactly one printed entry differs.
    assert np.count_nonzero(np.abs(Rg - raw) > 1e-12) == 1
    np.testing.assert_allclose(P3.P_general(k2 * np.ones((3, 3)), k0), Pm, atol=1e-15)
    # The printed R fixes the weights: R_ii = 3 w_i |c_i|^2 (k1 - k0).
    norm2 = P3.CX ** 2 + P3.CY ** 2 + P3.CZ ** 2
    np.testing.assert_allclose(np.diag(R)[1:], 3 * P3.W[1:] * norm2[1:] * (k1 - k0), atol=1e-15)


def test_T_diagonalises_R_and_P_eq93():
    k0, k1, k2 = 0.9, 1.3, 0.6
    T = matrix("eq89_T_d3q19.txt")
    Ti = np.linalg.inv(T)
    R = printed_R() * (k1 - k0) / 12.0
    Pm = matrix("eq81_P_d3q19.txt") * (k2 - k0) / 24.0
    np.testing.assert_allclose(T @ R @ Ti, np.diag([0] + [k1 - k0] * 3 + [0] * 15), atol=1e-14)
    np.testing.assert_allclose(T @ Pm @ Ti, np.diag([0] * 4 + [k2 - k0] * 6 + [0] * 9), atol=1e-14)


def test_block_relaxation_matrix_eq100():
    k0 = 1.1
    K1 = np.array([[1.3, -0.2, 0.1], [0.15, 1.6, 0.05], [-0.1, 0.2, 1.2]])
    K2 = np.array([[0.7, 1.2, 0.9], [0.4, 1.5, 0.6], [1.1, 0.8, 1.3]])
    T = matrix("eq89_T_d3q19.txt")
    S = T @ (k0 * np.eye(19) + P3.R_general(K1, k0) + P3.P_general(K2, k0)) @ np.linalg.inv(T)
    # Order of the second moments in T: M200, M101, M110, M011, M020, M002 (Eq. (84)).
    expect = np.diag([k0, 0, 0, 0, K2[0, 0], (K2[0, 2] + K2[2, 0]) / 2, (K2[0, 1] + K2[1, 0]) / 2,
                      (K2[1, 2] + K2[2, 1]) / 2, K2[1, 1], K2[2, 2]] + [k0] * 9)
    expect[1:4, 1:4] = K1
    np.testing.assert_allclose(S, expect, atol=1e-14)


def _k1_problem(k0, K1, K2, flux_a=(0.0, 0.0, 0.0)):
    """A problem whose K1 is the given matrix: A = c_s^2 (K1^-1 - I/2) (Eq. (30))."""
    A = (np.linalg.inv(K1) - 0.5 * np.eye(3)) / 3.0
    A = 0.5 * (A + A.T)
    return O3.Problem3(1, 1, 1, flux_a=flux_a, A0=(A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]), k0=k0,
                       K2=np.asarray(K2).ravel())


@pytest.mark.parametrize("k0,k1,k2", [(1.0, 1.25, 0.7), (0.6, 1.9, 1.3)])
def test_collision_equals_printed_matrices(k0, k1, k2):
    rng = np.random.default_rng(19)
    p = _k1_problem(k0, k1 * np.eye(3), np.full((3, 3), k2))
    R = printed_R() * (k1 - k0) / 12.0
    Pm = matrix("eq81_P_d3q19.txt") * (k2 - k0) / 24.0
    for _ in range(5):
        f = rng.random(19)
        phi = f.sum()
        feq = P3.W * phi  # Eq. (7) with B = 0, D = phi I
        expect = f - (k0 * np.eye(19) + R + Pm) @ (f - feq)
        np.testing.assert_allclose(O3.collide_node(p, f, phi), expect, atol=2e-15)


def test_collision_full_blocks_eq77():
    rng = np.random.default_rng(20)
    K1 = np.array([[1.3, -0.2, 0.1], [-0.2, 1.6, 0.05], [0.1, 0.05, 1.2]])  # symmetric: A = A^T
    K2 = np.array([[0.7, 1.2, 0.9], [0.4, 1.5, 0.6], [1.1, 0.8, 1.3]])
    k0 = 0.8
    u = np.array([0.03, -0.02, 0.01])
    p = _k1_problem(k0, K1, K2, flux_a=u)
    for _ in range(4):
        f = rng.random(19)
        phi = f.sum()
        feq = P3.W * (phi + 3.0 * (P3.C3 @ (u * phi)))
        expect = f - (k0 * np.eye(19) + P3.R_general(K1, k0) + P3.P_general(K2, k0)) @ (f - feq)
        np.testing.assert_allclose(O3.collide_node(p, f, phi), expect, atol=5e-15)


def test_equilibrium_moments_eq9():
    rng = np.random.default_rng(21)
    for _ in range(4):
        phi = rng.random()
        B = rng.normal(size=3) * 0.1
        D = rng.normal(size=(3, 3)) * 0.2
        D = D + D.T + phi * np.eye(3)
        feq = O3.equilibrium(phi, B, D.ravel())
        assert feq.sum() == pytest.approx(phi, abs=1e-15)
        np.testing.assert_allclose(P3.C3.T @ feq, B, atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", feq, P3.C3, P3.C3), D / 3.0, atol=1e-15)


def test_G_and_source_from_equilibrium():
    # From f = f_eq(phi): f+ - f = G (Eq. (11)) + w_i (S + (S - S_prev)/2) (Eq. (8), Scheme 2).
    K1 = np.array([[1.2, 0.1, 0.0], [0.1, 1.4, -0.1], [0.0, -0.1, 1.1]])
    a, b = np.array([0.02, 0.01, -0.03]), np.array([0.04, 0.0, 0.02])
    p = _k1_problem(1.0, K1, np.ones((3, 3)))
    p.flux_a, p.flux_b = tuple(a), tuple(b)
    phi, phi_prev, S, S_prev = 0.8, 0.7, 2e-3, 1e-3
    Bf = lambda v: a * v + b * v * v / 2
    f = O3.equilibrium(phi, Bf(phi), (phi * np.eye(3)).ravel())
    dB = Bf(phi) - Bf(phi_prev)
    G = 3.0 * P3.W * (P3.C3 @ ((np.eye(3) - K1 / 2) @ dB))
    expect = f + G + P3.W * (S + 0.5 * (S - S_prev))
    np.testing.assert_allclose(O3.collide_node(p, f, phi_prev, S, S_prev), expect, atol=2e-15)


def mode_map(k, A, u, k0, K2):
    """20x20 one-step map on (F in C^19, phi(t-1)) for f = F exp(i k.x), B = phi u, constant A."""
    K1 = np.linalg.inv(3.0 * A + 0.5 * np.eye(3))  # Eq. (30)
    Om = k0 * np.eye(19) + P3.R_general(K1, k0) + P3.P_general(K2, k0)
    E = P3.W * (1.0 + 3.0 * (P3.C3 @ u))
    g = 3.0 * P3.W * (P3.C3 @ ((np.eye(3) - K1 / 2.0) @ u))
    one = np.ones(19)
    Lam = np.diag(np.exp(-1j * (P3.C3 @ k)))
    Cm = np.eye(19) - Om @ (np.eye(19) - np.outer(E, one)) + np.outer(g, one)
    M = np.zeros((20, 20), dtype=complex)
    M[:19, :19] = Lam @ Cm
    M[:19, 19] = -Lam @ g
    M[19, :19] = one
    return M, E


A3 = np.array([[0.05, 0.01, 0.005], [0.01, 0.04, -0.008], [0.005, -0.008, 0.03]])


def test_fourier_mode_exact():
    n = (10, 8, 6)
    k = np.array([2 * np.pi / n[0], 2 * np.pi * 2 / n[1], 2 * np.pi / n[2]])
    u = np.array([0.03, -0.02, 0.01])
    k0 = 0.9
    K2 = np.array([[0.8, 1.3, 1.0], [0.5, 1.2, 0.7], [1.1, 0.9, 1.4]])
    p = O3.Problem3(*n, flux_a=tuple(u), A0=(A3[0, 0], A3[0, 1], A3[0, 2], A3[1, 1], A3[1, 2], A3[2, 2]), k0=k0,
                    K2=K2.ravel())
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    phase = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    o = O3.Oracle3(p, np.real(phase), nthreads=1)
    M, E = mode_map(k, A3, u, k0, K2)
    s = np.concatenate([E, [1.0]]).astype(complex)
    for _ in range(3):
        o.step(5)
        for _ in range(5):
            s = M @ s
        np.testing.assert_allclose(o.phi(), np.real(phase * s[:19].sum()), rtol=0, atol=2e-14)


def test_eq30_diffusion_tensor_from_leading_eigenvalue():
    u = np.array([0.02, -0.01, 0.015])
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        out = []
        for eps in (0.02, 0.01):
            k = eps * d
            M, _ = mode_map(k, A3, u, 1.0, np.ones((3, 3)))
            lam = np.linalg.eigvals(M)
            lead = lam[np.argmax(np.abs(lam))]
            out.append((-np.log(lead) - 1j * (k @ u)) / eps ** 2)
        # Real part -> k^T A k / eps^2 with O(eps) corrections (Richardson over the two eps).
        est = 2 * out[1] - out[0]
        assert est.real == pytest.approx(d @ A3 @ d, rel=2e-4)


def test_second_order_convergence_gaussian_hill():
    errs = []
    for n, steps in ((12, 36), (24, 144), (48, 576)):
        u = np.array([0.02, -0.01, 0.015]) * 12 / n
        s0 = n / 6
        x0 = (n / 2, n / 2, n / 2)
        p = O3.Problem3(n, n, n, flux_a=tuple(u), A0=(A3[0, 0], A3[0, 1], A3[0, 2], A3[1, 1], A3[1, 2], A3[2, 2]))
        o = O3.Oracle3(p, O3.gaussian_hill3((n, n, n), 0.0, x0, s0, u, A3)).step(steps)
        ref = O3.gaussian_hill3((n, n, n), steps, x0, s0, u, A3)
        errs.append(np.sum(np.abs(o.phi() - ref)) / np.sum(np.abs(ref)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 <= q <= 2.2 for q in orders), (errs, orders)


def hbb_steady3(N, k0, k1, k2, dphi=1.0):
    alpha = (1.0 / k1 - 0.5) / 3.0
    S = 2.0 * alpha * dphi / N ** 2
    p = O3.Problem3(2, 3, N, flux_a=(0.1, 0.05, 0.0), A0=(alpha, 0, 0, alpha, 0, alpha), k0=k0, K2=(k2,),
                    bc_type=(0, 0, 0, 0, 1, 1), bc_value=(0, 0, 0, 0, 0.0, dphi))
    o = O3.Oracle3(p, np.zeros((N, 3, 2)), source=np.full((N, 3, 2), S), nthreads=1)
    prev = o.phi()
    for _ in range(400):
        o.step(1000)
        cur = o.phi()
        if O.residual(cur, prev) < 1e-15:
            break
        prev = cur
    return cur


@pytest.mark.parametrize("N,k1,k2,k0", [(5, 1.25, None, 1.0), (5, 1.25, 0.5, 1.0), (10, 0.8, 1.5, 1.4),
                                        (10, 1.7, None, 0.6)])
def test_hbb_slip_eq61_holds_on_d3q19(N, k1, k2, k0):
    if k2 is None:
        k2 = O.k2_hbb(k1)
    phi = hbb_steady3(N, k0, k1, k2)
    Z = (np.arange(N) + 0.5) / N
    expect = Z * (2.0 - Z) + O.hbb_slip(k1, k2, 1.0, N)
    np.testing.assert_allclose(phi, np.broadcast_to(expect[:, None, None], phi.shape), rtol=0, atol=1e-13)


def test_uniform_state_is_fixed_point_with_edges():
    c = 0.37
    p = O3.Problem3(5, 4, 6, flux_a=(0.03, -0.02, 0.01), A0=(0.02, 0.005, 0.0, 0.01, 0.002, 0.03), k0=1.0,
                    K2=(0.8,), bc_type=(1,) * 6, bc_value=(c,) * 6)
    o = O3.Oracle3(p, np.full((6, 4, 5), c), nthreads=1).step(40)
    np.testing.assert_allclose(o.phi(), c, rtol=0, atol=1e-15)


def test_mass_conservation_periodic():
    p = O3.Problem3(9, 7, 5, flux_a=(0.02, -0.01, 0.03), flux_b=(0.05, 0.0, -0.02),
                    A0=(0.05, 0.01, 0.0, 0.04, 0.005, 0.03), beta=1.0, k0=0.9, K2=(1.1,))
    phi0 = np.random.default_rng(3).random((5, 7, 9))
    o = O3.Oracle3(p, phi0, nthreads=1)
    m0 = o.phi().sum()
    o.step(60)
    assert abs(o.phi().sum() - m0) <= 1e-13 * abs(m0)
