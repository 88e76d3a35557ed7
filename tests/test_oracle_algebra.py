"""Pins of the oracle's single-node algebra against the paper's printed matrices and identities.

Each test states the passage it checks. The expected values come from the paper's
printed matrices (tests/golden) or from identities the paper states, never from the
oracle itself.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import _paper as P

RNG = np.random.default_rng(1902)


def iso_problem(k0, k1, k2, a=(0.0, 0.0)):
    """A problem whose K1 is k1 I: A = alpha I with alpha from Eq. (30)."""
    alpha = (1.0 / k1 - 0.5) / 3.0
    return O.Problem(1, 1, flux_a=a, A0=(alpha, 0.0, alpha), k0=k0, K2=(k2,) * 4)


def feq_linear(phi, B):
    """Eq. (7) with D = phi I: w_i (phi + c_i.B / c_s^2)."""
    return P.W * (phi + 3.0 * (P.CX * B[0] + P.CY * B[1]))


# --------------------------------------------------------------------------------------
# The paper's matrices among themselves (Appendix).
# --------------------------------------------------------------------------------------

def test_printed_T_is_H_times_C():
    # Eq. (87): T = H C with C of Eq. (85), H of Eq. (90), T of Eq. (88).
    C, H, T = P.matrix("eq85_C_d2q9.txt"), P.matrix("eq90_H_d2q9.txt"), P.matrix("eq88_T_d2q9.txt")
    np.testing.assert_allclose(H @ C, T, atol=1e-15)


def test_C_rows_are_natural_moments():
    # Eq. (82)-(83): rows of C are sum_i c_ix^o c_iy^p for (o,p) in the printed order.
    C = P.matrix("eq85_C_d2q9.txt")
    order = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (2, 1), (1, 2), (2, 2)]
    for r, (o, p) in enumerate(order):
        np.testing.assert_array_equal(C[r], P.CX ** o * P.CY ** p)


@pytest.mark.parametrize("k0,k1,k2", [(1.0, 1.25, 0.7), (0.6, 1.9, 1.3), (1.4, 0.5, 1.0)])
def test_eq77_reproduces_printed_R_and_P(k0, k1, k2):
    # Eq. (77) with K1 = k1 I, K2 = k2 Ihat gives the printed Eqs. (78), (79).
    R = P.matrix("eq78_R_d2q9.txt") * (k1 - k0) / 12.0
    Pm = P.matrix("eq79_P_d2q9.txt") * (k2 - k0) / 12.0
    np.testing.assert_allclose(P.R_general(k1 * np.eye(2), k0), R, atol=1e-15)
    np.testing.assert_allclose(P.P_general(k2 * np.ones((2, 2)), k0), Pm, atol=1e-15)


def test_T_diagonalises_R_and_P():
    # Eq. (92): T R T^-1 = diag(0, k1-k0, k1-k0, 0, ...); T P T^-1 = diag(0,0,0, k2-k0 x3, 0,0,0).
    k0, k1, k2 = 0.9, 1.3, 0.6
    T = P.matrix("eq88_T_d2q9.txt")
    Ti = np.linalg.inv(T)
    R = P.matrix("eq78_R_d2q9.txt") * (k1 - k0) / 12.0
    Pm = P.matrix("eq79_P_d2q9.txt") * (k2 - k0) / 12.0
    np.testing.assert_allclose(T @ R @ Ti, np.diag([0, k1 - k0, k1 - k0, 0, 0, 0, 0, 0, 0]), atol=1e-14)
    np.testing.assert_allclose(T @ Pm @ Ti, np.diag([0, 0, 0, k2 - k0, k2 - k0, k2 - k0, 0, 0, 0]), atol=1e-14)


def test_block_relaxation_matrix_eq99():
    # Eq. (99): T (k0 I + R + P) T^-1 is block diagonal with K1 on (jx, jy), k2_11,
    # (k2_12 + k2_21)/2, k2_22 on the second moments and k0 elsewhere.
    k0 = 1.1
    K1 = np.array([[1.3, -0.2], [0.15, 1.6]])
    K2 = np.array([[0.7, 1.2], [0.4, 1.5]])
    T = P.matrix("eq88_T_d2q9.txt")
    S = T @ (k0 * np.eye(9) + P.R_general(K1, k0) + P.P_general(K2, k0)) @ np.linalg.inv(T)
    expect = np.diag([k0, 0, 0, K2[0, 0], (K2[0, 1] + K2[1, 0]) / 2, K2[1, 1], k0, k0, k0])
    expect[1:3, 1:3] = K1
    np.testing.assert_allclose(S, expect, atol=1e-14)


# --------------------------------------------------------------------------------------
# The oracle against them.
# --------------------------------------------------------------------------------------

def test_oracle_velocities_and_weights():
    # Weights after Eq. (38) and the velocity order of Eq. (85), read from the oracle's
    # equilibrium: f_eq(phi=1, B=0) = w_i and f_eq(phi=0, B=e_a) = 3 w_i c_ia.
    np.testing.assert_allclose(O.equilibrium(1.0, (0, 0), (1, 0, 0, 1)), P.W, rtol=1e-15)
    np.testing.assert_allclose(O.equilibrium(0.0, (1, 0), (0, 0, 0, 0)), 3 * P.W * P.CX, atol=1e-16)
    np.testing.assert_allclose(O.equilibrium(0.0, (0, 1), (0, 0, 0, 0)), 3 * P.W * P.CY, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments_eq9(seed):
    # Eq. (9): sum f_eq = phi, sum c f_eq = B, sum c c f_eq = c_s^2 D, for a general D.
    r = np.random.default_rng(seed)
    phi = r.uniform(-2, 2)
    B = r.uniform(-1, 1, 2)
    D = r.uniform(-1, 1, 4)
    D[2] = D[1]
    feq = O.equilibrium(phi, B, D)
    assert feq.sum() == pytest.approx(phi, abs=1e-14)
    np.testing.assert_allclose([np.dot(P.CX, feq), np.dot(P.CY, feq)], B, atol=1e-14)
    M2 = np.array([[np.dot(P.CX * P.CX, feq), np.dot(P.CX * P.CY, feq)],
                   [np.dot(P.CY * P.CX, feq), np.dot(P.CY * P.CY, feq)]])
    np.testing.assert_allclose(M2, D.reshape(2, 2) / 3.0, atol=1e-14)


@pytest.mark.parametrize("k0,k1,k2", [(1.0, 1.25, 8 * (1.25 - 2) / (3 * (1.25 - 4))),
                                      (1.0, 1.0 / 0.53, 1.0 / 7.0), (0.7, 1.6, 1.1), (1.5, 0.8, 0.3)])
def test_oracle_collision_is_printed_matrix_form(k0, k1, k2):
    # Eq. (6) for K1 = k1 I, K2 = k2 Ihat must equal f - (k0 I + R + P) f_neq (Eq. (eqq11))
    # with R, P the printed Eqs. (78), (79).
    R = P.matrix("eq78_R_d2q9.txt") * (k1 - k0) / 12.0
    Pm = P.matrix("eq79_P_d2q9.txt") * (k2 - k0) / 12.0
    u = (0.03, -0.05)
    prob = iso_problem(k0, k1, k2, a=u)
    for _ in range(4):
        f = RNG.uniform(0.0, 0.3, 9)
        phi = f.sum()
        fneq = f - feq_linear(phi, (u[0] * phi, u[1] * phi))
        expect = f - (k0 * np.eye(9) + R + Pm) @ fneq
        got = O.collide_node(prob, f, phi_prev=phi)
        np.testing.assert_allclose(got, expect, atol=2e-15)


def test_oracle_collision_anisotropic_eq77():
    # Eq. (6) with full K1 (from an anisotropic A via Eq. (30)) and a non-symmetric K2.
    A = np.array([[0.02, 0.008], [0.008, 0.01]])
    K1 = np.linalg.inv(3.0 * A + 0.5 * np.eye(2))
    K2 = np.array([[0.8, 1.3], [0.5, 1.2]])
    k0 = 0.9
    u = (0.02, 0.01)
    prob = O.Problem(1, 1, flux_a=u, A0=(A[0, 0], A[0, 1], A[1, 1]), k0=k0, K2=K2.ravel())
    Om = k0 * np.eye(9) + P.R_general(K1, k0) + P.P_general(K2, k0)
    for _ in range(4):
        f = RNG.uniform(0.0, 0.3, 9)
        phi = f.sum()
        fneq = f - feq_linear(phi, (u[0] * phi, u[1] * phi))
        np.testing.assert_allclose(O.collide_node(prob, f, phi_prev=phi), f - Om @ fneq, atol=2e-15)


def test_oracle_k1_follows_phi_through_eq30():
    # A(phi) = A0 (1 + beta phi^2): K1 of Eq. (30) is evaluated at the node's own phi.
    A0 = np.array([[0.01, 0.0], [0.0, 0.005]])
    beta = 1.0
    k0 = 1.0
    b = (0.05, 0.05)
    prob = O.Problem(1, 1, flux_b=b, A0=(A0[0, 0], 0.0, A0[1, 1]), beta=beta, k0=k0, K2=(1.0,) * 4)
    for _ in range(3):
        f = RNG.uniform(0.0, 0.4, 9)
        phi = f.sum()
        K1 = np.linalg.inv(3.0 * A0 * (1 + beta * phi ** 2) + 0.5 * np.eye(2))
        Om = k0 * np.eye(9) + P.R_general(K1, k0) + P.P_general(np.ones((2, 2)), k0)
        B = (b[0] * phi ** 2 / 2, b[1] * phi ** 2 / 2)
        fneq = f - feq_linear(phi, B)
        np.testing.assert_allclose(O.collide_node(prob, f, phi_prev=phi), f - Om @ fneq, atol=2e-15)


def test_correction_term_eq11():
    # From equilibrium (f_neq = 0) with phi(t-1) != phi(t), f+ - f is G of Eq. (11):
    # G_i = w_i c_i . (I - K1/2) dB / c_s^2 with dB = B(phi(t)) - B(phi(t-1)).
    A = np.array([[0.02, 0.008], [0.008, 0.01]])
    K1 = np.linalg.inv(3.0 * A + 0.5 * np.eye(2))
    a, b = (0.02, -0.01), (0.04, 0.03)
    prob = O.Problem(1, 1, flux_a=a, flux_b=b, A0=(A[0, 0], A[0, 1], A[1, 1]), k0=1.0, K2=(0.8,) * 4)
    phi, phi_prev = 0.7, 0.55
    Bf = lambda p: np.array([a[0] * p + b[0] * p * p / 2, a[1] * p + b[1] * p * p / 2])
    f = feq_linear(phi, Bf(phi))
    G = O.collide_node(prob, f, phi_prev=phi_prev) - f
    gv = (np.eye(2) - K1 / 2) @ (Bf(phi) - Bf(phi_prev))
    np.testing.assert_allclose(G, 3 * P.W * (P.CX * gv[0] + P.CY * gv[1]), atol=1e-16)
    assert abs(G.sum()) < 1e-15


def test_source_moments_eq10_and_scheme2():
    # Eq. (8), (10): S_i = w_i S, sum S_i = S, sum c_i S_i = 0; Scheme 2 adds (S - S_prev)/2.
    prob = iso_problem(1.0, 1.2, 0.9, a=(0.01, 0.02))
    phi = 0.4
    f = feq_linear(phi, (0.01 * phi, 0.02 * phi))
    S, Sp = 0.013, 0.007
    d = O.collide_node(prob, f, phi_prev=phi, S=S, S_prev=Sp) - f
    np.testing.assert_allclose(d, P.W * (S + 0.5 * (S - Sp)), atol=1e-16)
    assert d.sum() == pytest.approx(S + 0.5 * (S - Sp), abs=1e-15)
    assert abs(np.dot(P.CX, d)) < 1e-16 and abs(np.dot(P.CY, d)) < 1e-16


def test_collision_conserves_phi():
    # Sum_i f_i^+ = sum_i f_i + S' (Eq. (9), (10)): no other term changes the zeroth moment.
    A = np.array([[0.03, -0.01], [-0.01, 0.02]])
    prob = O.Problem(1, 1, flux_a=(0.01, 0.03), flux_b=(0.02, 0.0), A0=(A[0, 0], A[0, 1], A[1, 1]),
                     beta=0.5, k0=0.7, K2=(0.6, 1.1, 0.9, 1.4))
    for _ in range(5):
        f = RNG.uniform(0.0, 0.5, 9)
        out = O.collide_node(prob, f, phi_prev=f.sum() * 0.9, S=0.01)
        assert out.sum() == pytest.approx(f.sum() + 0.01, abs=1e-15)


def test_k0_relaxes_only_the_S0_moments():
    # Eq. (95)/(99): in moment space k0 acts on (m6, m7, m8) and not on j or the p block.
    T = P.matrix("eq88_T_d2q9.txt")
    base = dict(k1=1.3, k2=0.8)
    f = RNG.uniform(0.0, 0.3, 9)
    m_a = T @ O.collide_node(iso_problem(0.6, **base), f, phi_prev=f.sum())
    m_b = T @ O.collide_node(iso_problem(1.4, **base), f, phi_prev=f.sum())
    np.testing.assert_allclose(m_a[:6], m_b[:6], atol=1e-15)
    assert np.max(np.abs(m_a[6:] - m_b[6:])) > 1e-4


# --------------------------------------------------------------------------------------
# Table 1: LBGK, RLBM and MLBM as special cases (textbook updates written independently).
# --------------------------------------------------------------------------------------

def _first_moment(v):
    return np.array([np.dot(P.CX, v), np.dot(P.CY, v)])


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_lbgk_special_case(tau):
    # Table 1: k0 = k1 = k2 = 1/tau gives f+ = f - (f - f_eq)/tau (+ G + S).
    u = (0.04, -0.02)
    prob = iso_problem(1 / tau, 1 / tau, 1 / tau, a=u)
    f = RNG.uniform(0.0, 0.3, 9)
    phi = f.sum()
    feq = feq_linear(phi, (u[0] * phi, u[1] * phi))
    np.testing.assert_allclose(O.collide_node(prob, f, phi_prev=phi), f - (f - feq) / tau, atol=2e-15)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_rlbm_special_case_eq2(tau):
    # Eq. (2): f+ = f - f_neq - (1/tau - 1) w_i c_i . M1_neq / c_s^2; Table 1: k0 = 1, k1 = 1/tau, k2 = 1.
    u = (0.04, -0.02)
    prob = iso_problem(1.0, 1 / tau, 1.0, a=u)
    f = RNG.uniform(0.0, 0.3, 9)
    phi = f.sum()
    fneq = f - feq_linear(phi, (u[0] * phi, u[1] * phi))
    M1 = _first_moment(fneq)
    expect = f - fneq - (1 / tau - 1) * 3 * P.W * (P.CX * M1[0] + P.CY * M1[1])
    np.testing.assert_allclose(O.collide_node(prob, f, phi_prev=phi), expect, atol=2e-15)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_mlbm_special_case_eq3(tau):
    # Eq. (3): f+ = f - f_neq/tau - (1/tau_Z - 1/tau) w_i c_i . M1_neq / c_s^2, tau_Z = tau - Z;
    # Table 1: k0 = 1/tau, k1 = 1/tau_Z, k2 = 1/tau.
    Z = 1e-4
    u = (0.04, -0.02)
    prob = iso_problem(1 / tau, 1 / (tau - Z), 1 / tau, a=u)
    f = RNG.uniform(0.0, 0.3, 9)
    phi = f.sum()
    fneq = f - feq_linear(phi, (u[0] * phi, u[1] * phi))
    M1 = _first_moment(fneq)
    expect = f - fneq / tau - (1 / (tau - Z) - 1 / tau) * 3 * P.W * (P.CX * M1[0] + P.CY * M1[1])
    np.testing.assert_allclose(O.collide_node(prob, f, phi_prev=phi), expect, atol=2e-15)


def test_k2_rule_example():
    # Section 4.1.1: with k1 = 1.25 the optimal k2 from Eq. (62) is 0.7273.
    assert O.k2_hbb(1.25) == pytest.approx(0.7273, abs=5e-5)
    # Eq. (61) vanishes on Eq. (62).
    for k1 in (0.5, 1.25, 1.9):
        assert O.hbb_slip(k1, O.k2_hbb(k1), 1.0, 10) == pytest.approx(0.0, abs=1e-16)
