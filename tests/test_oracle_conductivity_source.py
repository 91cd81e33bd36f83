"""Independent pins of the oracle's conductivity and source readings (CPU).

The paper's problem statement (section "Alternating directions splitting
for Maxwell equations") has neither a conductivity nor a current; the
oracle adds both (reading R5): eps dE/dt + sigma E = curl H - J, with the
sigma E term averaged trapezoidally over each half step and J taken at the
half step's midpoint.  These tests check that reading against what the
mathematics fixes, not against a restatement of the oracle's coefficients:

* an exact damped solution of the continuous equations (one cavity mode,
  uniform sigma > 0): the oracle must converge to it at second order in
  tau (the scheme's order, section "Conclusions");
* an exact forced solution (the same mode driven by a smooth distributed
  current): again second order;
* the time-discrete recurrence that the two-substep scheme (scheme1a-
  scheme1d with reading R5) gives for that mode in the continuous space,
  derived by hand below: at a fixed, large tau the oracle must reach it up
  to the spatial error.

For each pin the tests also show that a plausible misreading fails it:
the conductivity number c = sigma tau / (2 eps) instead of / (4 eps), no
(1 + c) in the stiffness coefficient alpha, and the source evaluated at the
end of each half step instead of its midpoint.

The mode (kappa = lambda = 1 of the u^1 family of section "Numerical code
verification"), with s = sqrt(2) and w = pi s:
    E1 = a(t) sin(pi y) sin(pi z),
    H2 = -b2(t) sin(pi y) cos(pi z) / s,   H3 = b3(t) cos(pi y) sin(pi z) / s,
all other components zero; it satisfies the PEC conditions of the paper.
For constant eps, mu, sigma the continuous equations reduce to
    mu b' = w a  (b2 = b3 = b),   eps a' + sigma a = -w b - j(t)
for a current J = j(t) sin(pi y) sin(pi z) e_1.
"""
import numpy as np
import pytest

from oracle import bspline, maxwell, mms

S2 = np.sqrt(2.0)
W = np.pi * S2


def _mode_fields(quad, a, b2, b3):
    """The mode's six components at the quadrature points."""
    Y, Z = quad.Y, quad.Z
    z0 = np.zeros_like(Y)
    return [a * np.sin(np.pi * Y) * np.sin(np.pi * Z), z0, z0,
            z0, -b2 * np.sin(np.pi * Y) * np.cos(np.pi * Z) / S2,
            b3 * np.cos(np.pi * Y) * np.sin(np.pi * Z) / S2]


def _errors(quad, E, H, exact):
    """Relative L2 error of E and of H against the exact fields."""
    out = []
    for F, off in ((E, 0), (H, 3)):
        num = sum(float(np.sum(quad.W * (quad.evaluate(F[c]) - exact[off + c]) ** 2))
                  for c in range(3))
        den = sum(float(np.sum(quad.W * exact[off + c] ** 2)) for c in range(3))
        out.append(np.sqrt(num / den))
    return out


def _damped(eps, mu, sig):
    """Exact a(t), b(t) of the free mode with a(0) = 1, b(0) = 0."""
    g = sig / (2.0 * eps)
    Om = np.sqrt(W * W / (eps * mu) - g * g)
    C = -g / Om

    def a(t):
        return np.exp(-g * t) * (np.cos(Om * t) + C * np.sin(Om * t))

    def da(t):
        e = np.exp(-g * t)
        return e * (-g * (np.cos(Om * t) + C * np.sin(Om * t))
                    + Om * (-np.sin(Om * t) + C * np.cos(Om * t)))

    def b(t):
        return -(eps * da(t) + sig * a(t)) / W

    return a, b


def _forced(eps, mu, sig):
    """A driven mode: a(t) prescribed, b from mu b' = w a, j from the E equation."""
    a = lambda t: np.cos(2 * t) + 0.5 * np.sin(3 * t)
    da = lambda t: -2 * np.sin(2 * t) + 1.5 * np.cos(3 * t)
    b = lambda t: W / mu * (0.5 * np.sin(2 * t) + 0.5 * (1 - np.cos(3 * t)) / 3.0)
    j = lambda t: -(eps * da(t) + sig * a(t) + W * b(t))
    return a, b, j


def _source(j):
    one = lambda x: np.ones_like(x)
    sin = lambda x: np.sin(np.pi * x)
    return maxwell.SeparableSource(comp=0, j=j, fx=one, fy=sin, fz=sin)


class WideC(maxwell.Problem):
    """Misreading: conductivity number c = sigma tau / (2 eps)."""

    def __post_init__(self):
        super().__post_init__()
        tau = self.dt if self.local_dt is None else self.local_dt
        self.coef.update(maxwell.coefficients(self.eps, self.mu, 2.0 * self.sig, tau))


class AlphaNoC(maxwell.Problem):
    """Misreading: alpha = tau^2 / (4 eps mu) without the factor 1 / (1 + c)."""

    def __post_init__(self):
        super().__post_init__()
        self.coef["alpha"] = self.dt ** 2 / (4.0 * self.eps * self.mu)


class LateSource(maxwell.Problem):
    """Misreading: the source at the end of each half step."""

    def source_time(self, sub, t):
        return t + (0.5 if sub == 1 else 1.0) * self.dt


def _run(cls, N, p, eps, mu, sig, steps, T, exact_ab, j=None):
    """Run to time T from the projected exact state; errors of E and H."""
    dt = T / steps
    prob = cls(N, p, eps, mu, sig, dt, _source(j) if j is not None else None)
    quad = mms.Quadrature(N, p)
    a, b = exact_ab
    E, H = mms.project(prob, quad, _mode_fields(quad, a(0.0), b(0.0), b(0.0)))
    E, H, t = prob.run(E, H, 0.0, steps)
    assert t == pytest.approx(T)
    return _errors(quad, E, H, _mode_fields(quad, a(T), b(T), b(T)))


def _orders(errs):
    e = np.array([sum(x) for x in errs])
    return np.log2(e[:-1] / e[1:]), e


def test_exact_mode_fields_solve_the_equations():
    """The damped and forced solutions satisfy the continuous equations
    (finite differences in t, the spatial derivatives of the mode by hand)."""
    eps, mu, sig = 2.0, 1.5, 3.0
    h = 1e-5
    for a, b, j in (_damped(eps, mu, sig) + (lambda t: 0.0,), _forced(eps, mu, sig)):
        for t in (0.0, 0.37, 1.3):
            da = (a(t + h) - a(t - h)) / (2 * h)
            db = (b(t + h) - b(t - h)) / (2 * h)
            assert mu * db == pytest.approx(W * a(t), rel=1e-8, abs=1e-8)
            assert eps * da + sig * a(t) == pytest.approx(-W * b(t) - j(t), rel=1e-7, abs=1e-7)
    a, b = _damped(eps, mu, sig)
    assert a(0.0) == pytest.approx(1.0) and b(0.0) == pytest.approx(0.0, abs=1e-15)


def test_damped_mode_second_order_and_wide_c_fails():
    """Uniform sigma > 0, no source: the oracle converges to the exact damped
    mode at second order; c = sigma tau / (2 eps) does not converge."""
    eps, mu, sig = 1.0, 1.0, 2.0
    N, p, T = 16, 3, 1.0
    ex = _damped(eps, mu, sig)
    good = [_run(maxwell.Problem, N, p, eps, mu, sig, s, T, ex) for s in (8, 16, 32)]
    rates, e = _orders(good)
    assert np.all(rates > 1.8), (rates, e)
    bad = [_run(WideC, N, p, eps, mu, sig, s, T, ex) for s in (8, 16, 32)]
    rates_b, eb = _orders(bad)
    assert np.all(rates_b < 1.2), (rates_b, eb)
    assert eb[-1] > 20 * e[-1]


def test_forced_mode_second_order_and_late_source_fails():
    """A smooth distributed current with sigma > 0: second order with the
    source at the half-step midpoints, first order at the half-step ends."""
    eps, mu, sig = 2.0, 1.5, 3.0
    N, p, T = 16, 3, 1.0
    a, b, j = _forced(eps, mu, sig)
    good = [_run(maxwell.Problem, N, p, eps, mu, sig, s, T, (a, b), j) for s in (8, 16, 32)]
    rates, e = _orders(good)
    assert np.all(rates > 1.8), (rates, e)
    late = [_run(LateSource, N, p, eps, mu, sig, s, T, (a, b), j) for s in (8, 16, 32)]
    rates_l, el = _orders(late)
    assert np.all(np.abs(rates_l - 1.0) < 0.25), (rates_l, el)
    assert el[-1] > 10 * e[-1]


def _mode_recurrence(eps, mu, sig, tau, steps, j):
    """The two-substep scheme (scheme1a-scheme1d, reading R5) on the mode in
    the continuous space: a, b2, b3 after each step.

    Substep 1: eps (a' - a) + sig tau/4 (a' + a) = tau/2 [(C1 H')_1 - (C2 H)_1] - tau/2 j,
               mu (H' - H) = -tau/2 C1 E + tau/2 C2 E'.
    For the mode (C1 H)_1 = -w/2 b3 and (C2 H)_1 = w/2 b2 (times the E1
    shape); C1 E acts on H2 only and C2 E on H3 only (the derivatives of
    E1 along z and along y), which gives
        b2' = b2 + tau w / (2 mu) a,   b3' = b3 + tau w / (2 mu) a',
        (eps + sig tau/4 + tau^2 w^2 / (8 mu)) a' = (eps - sig tau/4) a
                                                   - tau w/4 (b2 + b3) - tau/2 j(t + tau/4).
    Substep 2 is the same with C1 and C2 exchanged:
        b3'' = b3' + tau w / (2 mu) a',  b2'' = b2' + tau w / (2 mu) a'',
        (eps + sig tau/4 + tau^2 w^2 / (8 mu)) a'' = (eps - sig tau/4) a'
                                                    - tau w/4 (b2' + b3') - tau/2 j(t + 3 tau/4).
    """
    a, b2, b3, t = 1.0, 0.0, 0.0, 0.0
    lhs = eps + sig * tau / 4 + tau * tau * W * W / (8 * mu)
    k = tau * W / (2 * mu)
    for _ in range(steps):
        a1 = ((eps - sig * tau / 4) * a - tau * W / 4 * (b2 + b3) - tau / 2 * j(t + tau / 4)) / lhs
        b2, b3 = b2 + k * a, b3 + k * a1
        a2 = ((eps - sig * tau / 4) * a1 - tau * W / 4 * (b2 + b3)
              - tau / 2 * j(t + 3 * tau / 4)) / lhs
        b2, b3 = b2 + k * a2, b3 + k * a1
        a, t = a2, t + tau
    return a, b2, b3


@pytest.mark.parametrize("forced", [False, True])
def test_step_matches_the_continuous_space_mode_recurrence(forced):
    """At a large fixed tau the oracle's fields approach the mode recurrence
    as h -> 0 (spatial error only); the three misreadings stay O(tau^3 sig)
    or O(tau j') away from it."""
    eps, mu, sig = 2.0, 1.5, 4.0
    tau, steps = 0.25, 6
    j = _forced(eps, mu, sig)[2] if forced else (lambda t: 0.0)
    ra, rb2, rb3 = _mode_recurrence(eps, mu, sig, tau, steps, j)

    def err(cls, N, p=3):
        prob = cls(N, p, eps, mu, sig, tau, _source(j) if forced else None)
        quad = mms.Quadrature(N, p)
        E, H = mms.project(prob, quad, _mode_fields(quad, 1.0, 0.0, 0.0))
        E, H, _ = prob.run(E, H, 0.0, steps)
        return _errors(quad, E, H, _mode_fields(quad, ra, rb2, rb3))

    e8, e16 = err(maxwell.Problem, 8), err(maxwell.Problem, 16)
    assert max(e16) < 2e-5, e16
    assert max(e16) < max(e8) / 5, (e8, e16)  # spatial convergence (about h^(p+1))
    misreadings = [WideC, AlphaNoC] + ([LateSource] if forced else [])
    for cls in misreadings:
        assert max(err(cls, 16)) > 100 * max(e16), cls.__name__


def test_separable_source_rows_integrate_the_profile():
    """Rows of a separable source against brute-force quadrature of
    (fx fy fz, B_r B_s B_t), and the partition-of-unity sum rule."""
    N, p = 5, 2
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, 0.1)
    src = maxwell.SeparableSource(comp=1, j=lambda t: 2.0 * t, fx=lambda x: x * x,
                                  fy=lambda y: np.cos(y), fz=lambda z: 1.0 + z)
    R = src.rows(prob, 1, 0.75)
    assert np.all(src.rows(prob, 0, 0.75) == 0)
    knots = bspline.open_uniform_knots(N, p)
    xs = (np.arange(4000) + 0.5) / 4000          # midpoint rule, fine grid
    V = bspline.basis(knots, p, xs) / 4000
    ref = 1.5 * np.einsum("k,j,i->kji", V.T @ (1.0 + xs), V.T @ np.cos(xs), V.T @ xs ** 2)
    np.testing.assert_allclose(R, ref, rtol=1e-6, atol=1e-9)
    # sum over all rows = j(t) * integral of the profile (partition of unity)
    total = 1.5 * (1.0 / 3.0) * np.sin(1.0) * 1.5
    assert R.sum() == pytest.approx(total, rel=1e-12)
