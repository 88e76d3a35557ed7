"""Pins of the oracle's time stepping (streaming, bounce-back, G, sources) against closed forms,
exact linear analysis and numbers the paper prints.

Expected values come from the paper (Eq. (61)-(62), Eq. (71), Table 3, Section 4.1.1), from the
exact Fourier-mode map of the linear scheme assembled from Eq. (77), or from invariants; none
is produced by the oracle itself.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import _paper as P


# --------------------------------------------------------------------------------------
# Conservation (Eq. (9), periodic domain, S = 0).
# --------------------------------------------------------------------------------------

def test_mass_conserved_nonlinear_periodic():
    rng = np.random.default_rng(7)
    n = 40
    prob = O.Problem(n, n - 7, flux_a=(0.01, -0.02), flux_b=(0.05, 0.05),
                     A0=(0.01, 0.002, 0.005), beta=1.0, k0=0.8, K2=(0.9, 1.1, 0.7, 1.2))
    phi0 = rng.uniform(0.0, 1.0, (n - 7, n))
    o = O.Oracle(prob, phi0)
    m0 = o.phi().sum()
    o.step(300)
    assert abs(o.phi().sum() - m0) / m0 < 1e-13


# --------------------------------------------------------------------------------------
# Half-way bounce-back steady diffusion: Eq. (49), (61), (62); Section 4.1.1.
# --------------------------------------------------------------------------------------

def hbb_steady(N, k0, k1, k2, ux=0.1, phi_bottom=0.0, dphi=1.0, nx=2, max_steps=400000):
    """Steady state of Eqs. (31)-(32) with HBB walls (x periodic, y in [0, N])."""
    alpha = (1.0 / k1 - 0.5) / 3.0  # Eq. (30)
    S = 2.0 * alpha * dphi / N ** 2
    prob = O.Problem(nx, N, flux_a=(ux, 0.0), A0=(alpha, 0.0, alpha), k0=k0, K2=(k2,) * 4,
                     bc_type=(O.PERIODIC, O.PERIODIC, O.DIRICHLET, O.DIRICHLET),
                     bc_value=(0.0, 0.0, phi_bottom, phi_bottom + dphi))
    o = O.Oracle(prob, np.zeros((N, nx)), source=np.full((N, nx), S), nthreads=1)
    prev = o.phi()
    res_hist = []
    steps = 0
    while steps < max_steps:
        o.step(1000)
        steps += 1000
        cur = o.phi()
        res_hist.append(O.residual(cur, prev))  # Eq. (64)
        prev = cur
        if res_hist[-1] < 1e-15:
            break
    return cur, res_hist


@pytest.mark.parametrize("N", [5, 10])
@pytest.mark.parametrize("k1,k2,k0", [(1.25, None, 1.0), (1.25, 0.5, 1.0), (1.25, 1.0, 0.6), (0.8, 1.5, 1.4),
                                      (1.7, 0.9, 1.0), (1.7, None, 0.6), (0.8, None, 1.4)])
def test_hbb_slip_eq61(N, k1, k2, k0):
    # Eq. (49) with the slip of Eq. (61); with k2 of Eq. (62) the slip vanishes. k0 has no
    # effect on the steady state (Section 4.1.1, Fig. 2a).
    if k2 is None:
        k2 = O.k2_hbb(k1)
    dphi = 1.0
    phi, res = hbb_steady(N, k0, k1, k2, dphi=dphi)
    assert res[-1] < 1e-15
    Y = (np.arange(N) + 0.5) / N  # y_n = (n - 1/2)/N below Eq. (49)
    slip = O.hbb_slip(k1, k2, dphi, N)
    expect = dphi * Y * (2.0 - Y) + slip
    np.testing.assert_allclose(phi, np.broadcast_to(expect[:, None], phi.shape), rtol=0, atol=1e-13)


def test_hbb_paper_instance_exact():
    # Section 4.1.1: N = 5 (dx = L/5), k1 = 1.25, k2 = 8(k1-2)/(3(k1-4)) = 0.7273: the
    # steady solution is the exact parabola (GRE at machine level, Fig. 3 text).
    k1 = 1.25
    phi, res = hbb_steady(5, 1.0, k1, O.k2_hbb(k1))
    Y = (np.arange(5) + 0.5) / 5
    ref = np.broadcast_to((Y * (2 - Y))[:, None], phi.shape)
    assert O.gre(phi, ref) < 1e-13
    # The residual of Eq. (64) falls monotonically to the stopping level.
    assert all(b <= a for a, b in zip(res, res[1:]))


def test_uniform_state_is_fixed_point_with_corners():
    # All four walls Dirichlet at the same value c, S = 0: phi = c is a steady solution of the
    # scheme (f = f_eq(c) maps to itself, bounce-back included, corners included).
    c = 0.37
    n = 9
    prob = O.Problem(n, n + 2, flux_a=(0.03, -0.02), A0=(0.02, 0.005, 0.01), k0=1.0, K2=(0.8,) * 4,
                     bc_type=(O.DIRICHLET,) * 4, bc_value=(c,) * 4)
    o = O.Oracle(prob, np.full((n + 2, n), c), nthreads=1)
    o.step(50)
    np.testing.assert_allclose(o.phi(), c, rtol=0, atol=1e-15)


def test_linear_profile_between_walls_is_exact():
    # S = 0 between two HBB walls: the steady solution is the exact linear profile for any
    # rates (Eq. (61) with S = 0 has no slip; the wall relation of Eq. (60) holds exactly).
    N = 8
    prob = O.Problem(3, N, flux_a=(0.05, 0.0), A0=(0.05, 0.0, 0.05), k0=0.7, K2=(1.3,) * 4,
                     bc_type=(O.PERIODIC, O.PERIODIC, O.DIRICHLET, O.DIRICHLET), bc_value=(0, 0, 1.0, 3.0))
    o = O.Oracle(prob, np.zeros((N, 3)), nthreads=1)
    o.step(60000)
    Y = (np.arange(N) + 0.5) / N
    np.testing.assert_allclose(o.phi(), np.broadcast_to((1.0 + 2.0 * Y)[:, None], (N, 3)), atol=1e-13)


# --------------------------------------------------------------------------------------
# Exact Fourier-mode map of the linear scheme (Eq. (77), Eq. (11), Eq. (38)).
# --------------------------------------------------------------------------------------

def mode_map(k, A, u, k0, K2):
    """10x10 one-step map on (F in C^9, phi(t-1)) for f = F exp(i k.x), B = phi u, constant A."""
    K1 = np.linalg.inv(3.0 * A + 0.5 * np.eye(2))  # Eq. (30)
    Om = k0 * np.eye(9) + P.R_general(K1, k0) + P.P_general(K2, k0)
    E = P.W * (1.0 + 3.0 * (P.CX * u[0] + P.CY * u[1]))
    gv = (np.eye(2) - K1 / 2.0) @ np.asarray(u)
    g = 3.0 * P.W * (P.CX * gv[0] + P.CY * gv[1])
    one = np.ones(9)
    Lam = np.diag(np.exp(-1j * (k[0] * P.CX + k[1] * P.CY)))
    C = np.eye(9) - Om @ (np.eye(9) - np.outer(E, one)) + np.outer(g, one)
    M = np.zeros((10, 10), dtype=complex)
    M[:9, :9] = Lam @ C
    M[:9, 9] = -Lam @ g
    M[9, :9] = one
    return M, E


def test_fourier_mode_exact():
    nx, ny = 16, 12
    k = (2 * np.pi * 1 / nx, 2 * np.pi * 2 / ny)
    A = np.array([[0.02, 0.008], [0.008, 0.01]])
    u = (0.03, -0.02)
    k0 = 0.9
    K2 = np.array([[0.8, 1.3], [0.5, 1.2]])
    prob = O.Problem(nx, ny, flux_a=u, A0=(A[0, 0], A[0, 1], A[1, 1]), k0=k0, K2=K2.ravel())
    X, Y = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    phase = np.exp(1j * (k[0] * X + k[1] * Y))
    o = O.Oracle(prob, np.real(phase))
    M, E = mode_map(k, A, u, k0, K2)
    s = np.concatenate([E, [1.0]]).astype(complex)
    for _ in range(4):
        o.step(10)
        for _ in range(10):
            s = M @ s
        np.testing.assert_allclose(o.phi(), np.real(phase * s[:9].sum()), rtol=0, atol=2e-14)


def test_eq30_diffusion_tensor_from_leading_eigenvalue():
    # Chapman-Enskog, Eq. (29)-(30): the hydrodynamic eigenvalue of the mode map satisfies
    # ln(lambda) = -i k.u - k^T A k + higher order.
    A = np.array([[0.02, 0.008], [0.008, 0.01]])
    K2 = np.array([[0.8, 1.1], [1.1, 1.2]])
    for u in [(0.0, 0.0), (0.02, -0.01)]:
        for kv in [(1.0, 2.0), (2.0, -1.0)]:
            k = 2 * np.pi / 800 * np.asarray(kv)
            M, _ = mode_map(k, A, u, 1.0, K2)
            ev = np.linalg.eigvals(M)
            lam = ev[np.argmin(np.abs(ev - 1.0))]
            ln = np.log(lam)
            kak = k @ A @ k
            assert -ln.real == pytest.approx(kak, rel=2e-3)
            assert -ln.imag == pytest.approx(k @ np.asarray(u), rel=1e-2, abs=1e-9)


# --------------------------------------------------------------------------------------
# Gaussian hill (Eq. (71)): closed form and second-order convergence (Fig. 12 text).
# --------------------------------------------------------------------------------------

def hill_gre(N, steps, u, A, k2=1.0):
    sigma = 6.0 * N / 64
    x0 = (N / 2, N / 2)
    K = np.asarray(A)
    prob = O.Problem(N, N, flux_a=u, A0=(K[0, 0], K[0, 1], K[1, 1]), k0=1.0, K2=(k2,) * 4)
    o = O.Oracle(prob, O.gaussian_hill(N, N, 0.0, x0, sigma, u, K))
    o.step(steps)
    return O.gre(o.phi(), O.gaussian_hill(N, N, float(steps), x0, sigma, u, K))


@pytest.mark.parametrize("A", [[[0.01, 0.0], [0.0, 0.01]], [[0.01, 0.005], [0.005, 0.02]]])
def test_gaussian_hill_second_order(A):
    # Diffusive refinement: N = 64 -> 128, sigma and steps scale as N and N^2, u as 1/N.
    e64 = hill_gre(64, 2000, (0.05, 0.05), A)
    e128 = hill_gre(128, 8000, (0.025, 0.025), A)
    assert e64 < 1e-2
    order = np.log2(e64 / e128)
    assert 1.8 < order < 2.3, (e64, e128, order)


# --------------------------------------------------------------------------------------
# Table 3 (Section 4.1.2): printed GREs, Dirichlet HBB walls carrying the exact solution.
# --------------------------------------------------------------------------------------

def table3_gre(model, u0, n=100):
    """Paper setup: [0,2]^2, dx = 1/50, c = 5, tau = 0.8, alpha = 0.01, t = 1 (250 steps)."""
    dx = 2.0 / n
    dt = dx / 5.0
    alpha, tau = 0.01, 0.8
    alu = alpha * dt / dx ** 2
    k1 = O.k1_isotropic(alu)
    assert abs(k1 - 1 / tau) < 1e-12
    k0, k2 = {"OB-TriRT": (1.0, O.k2_hbb(k1)), "LBGK": (k1, k1), "RLBM": (1.0, 1.0)}[model]
    ulu = u0 * dt / dx
    prob = O.Problem(n, n, flux_a=(ulu, ulu), A0=(alu, 0.0, alu), k0=k0, K2=(k2,) * 4,
                     bc_type=(O.DIRICHLET,) * 4)
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)
    lam = 1.0 - 2.0 * np.pi ** 2 * alpha

    def exact(X, Y, t):
        return np.exp(lam * t) * np.sin(np.pi * (X + Y))

    def source(t):  # S of Section 4.1.2 in lattice units (times dt)
        return dt * np.exp(lam * t) * (np.sin(np.pi * (X + Y)) + np.pi * 2 * u0 * np.cos(np.pi * (X + Y)))

    o = O.Oracle(prob, exact(X, Y, 0.0))
    wall = np.empty((9,) + X.shape)
    nsteps = int(round(1.0 / dt))
    S_prev = source(0.0)
    for s in range(nsteps):
        # Bounce-back value at the wall crossing point x + c_i dx/2, at the new time level.
        for i in range(9):
            wall[i] = exact(X + P.CX[i] * dx / 2, Y + P.CY[i] * dx / 2, (s + 1) * dt)
        S = source(s * dt)
        o.step(1, S=S, S_prev=S_prev, wall=wall)
        S_prev = S
    phi = o.phi()
    if not np.all(np.isfinite(phi)) or np.max(np.abs(phi)) > 10:
        return None
    return O.gre(phi, exact(X, Y, 1.0))


def _table3():
    rows = {r[0]: r[1:] for r in P.table("table3_gre.txt")}
    return rows


@pytest.mark.parametrize("model,col", [("OB-TriRT", 0), ("OB-TriRT", 1), ("OB-TriRT", 3),
                                       ("LBGK", 0), ("LBGK", 1), ("LBGK", 2), ("RLBM", 0), ("RLBM", 1)])
def test_table3_printed_gre(model, col):
    u0 = (0.01, 0.1, 1.0, 2.5)[col]
    printed = float(_table3()[model][col])
    got = table3_gre(model, u0)
    assert got == pytest.approx(printed, rel=3e-3)


def test_table3_lbgk_unstable_at_u0_2p5():
    # Table 3 marks LBGK unstable at u0 = 2.5; OB-TriRT stays stable (previous test).
    assert _table3()["LBGK"][3] == "-"
    assert table3_gre("LBGK", 2.5) is None
