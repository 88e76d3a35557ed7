"""Oracle pins of the method variants: a space-dependent diffusion tensor A(x) and a source that
changes in time (Eqs. (73)-(76), Table 6; Scheme 2 of Remark III).

* Table 6: the printed global relative errors (Eq. (63)) at t = 3 for alpha = 1e-4 and 1e-6 on
  the 200 x 200 grid (lattice speed 1), within 10 %.
* Convergence to the closed form of Eq. (76) under diffusive refinement (fixed lattice
  diffusivity): second order; with the tensor replaced by a constant one (a wrong A(x)) the
  error stops converging, so the pin sees the space dependence.
* A uniform state with a uniform source exp(g t) s: the scheme stays at equilibrium and phi
  gains S(t) + (S(t) - S(t-1))/2 per step exactly (Eq. (8), Scheme 2, S(-1) := S(0)).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1902_09813_amd import workloads as W
from tests._cases import oracle_problem, oracle_source, run_oracle


def exact_c6(w, steps):
    """Eq. (76) at t = steps * dt on the workload's nodes."""
    e = w.extra
    t = steps * e["dt"]
    c = (np.arange(w.nx) + 0.5) * e["dx"]
    X, Y = np.meshgrid(c, c)
    return np.exp(e["lambda"] * t) * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)


@pytest.mark.parametrize("alpha,printed", [(1e-4, 1.7601e-4), (1e-6, 1.7660e-4)])
def test_table6_global_relative_error(alpha, printed):
    w = W.c6(alpha, 200)
    o = run_oracle(w)
    gre = O.gre(o.phi(), exact_c6(w, w.steps))
    assert gre == pytest.approx(printed, rel=0.10), gre


def c6_diffusive(n, a_lat=0.05, alpha=1e-2, t_end=0.5):
    dx = 1.0 / n
    return W.c6(alpha, n, t_end=t_end, dt=a_lat * dx * dx / alpha)


def test_variable_tensor_converges_at_second_order():
    errs = []
    for n in (24, 48, 96):
        w = c6_diffusive(n)
        errs.append(O.gre(run_oracle(w).phi(), exact_c6(w, w.steps)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 <= q <= 2.3 for q in orders), (errs, orders)
    # The same runs with A0(x) replaced by its mean: the source no longer matches the tensor,
    # and the error stalls.
    wrong = []
    for n in (48, 96):
        w = c6_diffusive(n)
        mean = w.A0_field.mean(axis=(0, 1))
        w.A0_field = np.broadcast_to(mean, w.A0_field.shape).copy()
        wrong.append(O.gre(run_oracle(w).phi(), exact_c6(w, w.steps)))
    assert wrong[1] > 0.7 * wrong[0] and wrong[1] > 20 * errs[2], (wrong, errs)


def test_growing_uniform_source_follows_scheme2_exactly():
    n, steps, g, s0, phi0 = 8, 25, 0.03, 2e-3, 0.7
    w = W.Workload("uniform_growth", n, n, steps, A0=(0.02, 0.005, 0.03), flux_a=(0.04, -0.02),
                   source=("field", np.full((n, n), s0), g), phi0_kind="uniform")
    o = O.Oracle(oracle_problem(w), np.full((n, n), phi0), source=oracle_source(w), nthreads=1)
    from tests._cases import advance
    advance(o, w, steps)
    S = [s0 * np.exp(g * t) for t in range(steps)]
    want = phi0 + sum(1.5 * S[t] - 0.5 * (S[t - 1] if t > 0 else S[0]) for t in range(steps))
    assert np.max(np.abs(o.phi() - want)) <= 1e-14 * steps
