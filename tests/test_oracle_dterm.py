"""Oracle pins of a general D(phi) != phi I (Eq. (1), Eq. (7)): D = (g phi + e |phi|^s) I.

* D = (phi + (beta/3) phi^3) I with a constant A0 and D = phi I with A = A0 (1 + beta phi^2) are
  two discretisations of the same equation, d_t phi + div B = div[A0 (1 + beta phi^2) grad phi]:
  under diffusive refinement their difference vanishes at second order. A wrong D (e scaled by
  1.25) gives a different equation and the difference stalls.
* e = 0, g = 1 is D = phi I bit for bit.
* The equilibrium carries the second moment c_s^2 D (Eq. (9)) for the D of the problem, and
  f_0^eq = w_0 (2 phi - d): positive only while d < 2 phi.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1902_09813_amd import workloads as W
from tests._cases import oracle_problem


def _pair(n, steps, beta, e_scale=1.0):
    # A positive bump on a background, anisotropic A0, velocity scaled with the grid
    # (diffusive refinement: fixed lattice diffusivity, steps x 4 per halving of dx).
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    phi0 = 0.4 + 0.5 * np.exp(-((X - n / 2) ** 2 + (Y - n / 2) ** 2) / (2 * (n / 8) ** 2))
    common = dict(A0=(0.06, 0.01, 0.03), flux_a=(0.02 * 32 / n, -0.01 * 32 / n))
    wa = W.Workload("A_phi", n, n, steps, beta=beta, **common)
    wb = W.Workload("D_phi", n, n, steps, dterm=(1.0, e_scale * beta / 3.0, 3.0), **common)
    out = []
    for w in (wa, wb):
        o = O.Oracle(oracle_problem(w), phi0, nthreads=0)
        o.step(steps)
        out.append(o.phi())
    return out


def test_nonlinear_d_matches_phi_dependent_tensor_at_second_order():
    diffs = []
    for n, steps in ((32, 100), (64, 400), (128, 1600)):
        a, b = _pair(n, steps, beta=2.0)
        diffs.append(np.max(np.abs(a - b)) / 0.5)
    orders = [np.log2(diffs[i] / diffs[i + 1]) for i in range(2)]
    assert all(1.85 <= q <= 2.15 for q in orders), (diffs, orders)
    wrong = []
    for n, steps in ((32, 100), (64, 400)):
        a, b = _pair(n, steps, beta=2.0, e_scale=1.25)
        wrong.append(np.max(np.abs(a - b)) / 0.5)
    assert wrong[1] > 0.9 * wrong[0] and wrong[1] > 20 * diffs[1], (wrong, diffs)


def test_linear_d_is_phi_i():
    n, steps = 24, 40
    w = W.Workload("plain", n, n, steps, A0=(0.05, 0.01, 0.03), flux_a=(0.03, 0.02), flux_b=(0.01, 0.0), seed=3)
    a = O.Oracle(oracle_problem(w), w.phi0(), nthreads=1).step(steps)
    w.dterm = (1.0, 0.0, 2.0)
    b = O.Oracle(oracle_problem(w), w.phi0(), nthreads=1).step(steps)
    assert np.array_equal(a.f, b.f)


@pytest.mark.parametrize("phi,g,e,s", [(0.7, 1.0, 0.3, 3.0), (0.4, 0.5, 0.2, 2.5), (1.3, 0.0, 1.0, 2.0)])
def test_equilibrium_moments_of_d(phi, g, e, s):
    # One node at equilibrium: its populations (oracle init) carry c_s^2 D in the second moment.
    w = W.Workload("node", 1, 1, 0, A0=(0.05, 0.0, 0.05), flux_a=(0.03, -0.02), dterm=(g, e, s))
    o = O.Oracle(oracle_problem(w), np.full((1, 1), phi), nthreads=1)
    f = o.f[:, 0, 0]
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    d = g * phi + e * abs(phi) ** s
    assert np.sum(f) == pytest.approx(phi, abs=1e-15)
    assert np.sum(cx * cx * f) == pytest.approx(d / 3, abs=1e-15)
    assert np.sum(cy * cy * f) == pytest.approx(d / 3, abs=1e-15)
    assert np.sum(cx * cy * f) == pytest.approx(0.0, abs=1e-15)
    assert f[0] == pytest.approx(4.0 / 9.0 * (2 * phi - d), abs=1e-15)
