"""Why Newton from the previous time level fails with the harmonic mean.

With the harmonic mean, the conductivity of a face between a dry cell c and a
wet neighbour n is about 2 K(p_c): it grows with the dry cell's head as fast
as K itself.  The inflow K^AV (p_n - p_c) / h^2 then grows with p_c wherever
(p_n - p_c) K'(p_c) / K(p_c) > 1, and once h^2 / dt is small enough this
growth beats the storage term theta'(p_c) / dt: the diagonal of the Jacobian
(Section 3) is negative at the initial state.  The Newton direction from the
previous level then points away from the root, and the line search lets the
iterate slide down the merit function towards p -> -infinity, where Phi stays
bounded away from zero.  The scalar (one-cell) problem shows it with numbers
taken only from the residual (pinned elsewhere) and its central differences.
In 3-D the uniform mode of the top layer behaves like the one-cell problem
(horizontal differences vanish): along it the Jacobian is indefinite at the
512^3 spacing and the recipe's time step, and the steps fail the same way,
while a time step below theta' / (the inflow's growth) converges.
"""
import numpy as np
import pytest

import synth

H_C5 = 64.0 / 513.0        # grid spacing of the 512^3 cube
P0, P_TOP = synth.P_INIT, synth.P_TOP


def one_cell(dt, h=H_C5):
    return synth.Problem(nx=1, ny=1, nz=1, hx=h, hy=h, hz=h, mean=synth.HARMONIC, dt=dt)


def phi(orc, P, ks, p, th0):
    return orc.residual(P, ks, np.array([p]), th0)[0]


def dphi(orc, P, ks, p, th0, rel=1e-6):
    e = rel * abs(p)
    return (phi(orc, P, ks, p + e, th0) - phi(orc, P, ks, p - e, th0)) / (2 * e)


def bisect_root(orc, P, ks, lo, hi, th0):
    flo = phi(orc, P, ks, lo, th0)
    assert flo * phi(orc, P, ks, hi, th0) < 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = phi(orc, P, ks, mid, th0)
        if (fm < 0) == (flo < 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("dt", [0.3, 30.0])
def test_one_cell_newton_runs_away_from_the_root(orc, dt):
    """At the 512^3 spacing with the median K_s the one-cell residual has a
    root above p0, its slope at p0 is negative, and Newton with the line
    search drifts to ever lower heads without converging."""
    P = one_cell(dt)
    ks = np.array([synth.KS0])
    p0 = np.array([P0])
    th0 = orc.theta(P, p0)
    f0 = phi(orc, P, ks, P0, th0)
    assert f0 < 0  # the boundary feeds the cell: inflow exceeds storage at p0
    root = bisect_root(orc, P, ks, P0, 0.0, th0)
    assert P0 < root < 0.0
    # negative slope at p0, from central differences of the residual (and the
    # analytic Jacobian agrees with them)
    s0 = dphi(orc, P, ks, P0, th0)
    assert s0 < 0
    assert orc.jacobian(P, ks, p0).toarray()[0, 0] == pytest.approx(s0, rel=1e-5)
    # Phi stays negative everywhere below p0: no root on the side Newton goes to
    for p in np.geomspace(-P0, 1e9, 60):
        assert phi(orc, P, ks, -p, th0) < 0
    o = orc.Solver(P, synth.Options(precision=synth.FP64, amg_max_levels=1), ks)
    o.trace(400)
    p = p0.copy()
    st = o.step(p)
    assert st["status"] == orc.MAXITER
    u = o.iterate(1)[0]
    assert u < -1e6  # slid far below p0
    assert -f0 / s0 < 0  # the first Newton direction points down, away from the root
    ev = o.events()
    assert len(ev) == 200 and all(e["f_acc"] <= e["f0"] for e in ev)  # the merit function never rose


def test_one_cell_converges_below_the_critical_time_step(orc):
    """With dt below theta'(p0) / (the inflow's growth at p0) the slope at p0
    is positive and Newton reaches the root."""
    ks = np.array([synth.KS0])
    p0 = np.array([P0])
    th0 = orc.theta(one_cell(1.0), p0)
    theta_prime = orc.laws(one_cell(1.0), p0, ks)[1][0]
    growth = theta_prime / 1.0 - dphi(orc, one_cell(1.0), ks, P0, th0)  # d(inflow)/dp at p0
    assert growth > 0
    dt = 0.5 * theta_prime / growth
    P = one_cell(dt)
    assert dphi(orc, P, ks, P0, th0) > 0
    root = bisect_root(orc, P, ks, P0, 0.0, th0)
    o = orc.Solver(P, synth.Options(precision=synth.FP64, amg_max_levels=1, fnormtol=1e-12), ks)
    p = p0.copy()
    st = o.step(p)
    assert st["status"] == 0
    assert p[0] == pytest.approx(root, abs=1e-8)


def test_3d_harmonic_block_at_the_512_spacing(orc):
    """A 12^3 block at the 512^3 cube's spacing with that recipe's K_s
    statistics.  The uniform mode of the top layer (all top cells raised
    together; horizontal differences vanish, so it behaves like the one-cell
    problem) has v^T J v < 0 at the recipe's dt = 30 s: the Jacobian is
    indefinite along the direction the infiltration needs, GMRES with the SPD
    preconditioner does not converge and Newton ends at the iteration limit.
    At dt = 3 s the mode is positive and the steps converge."""
    r = synth.recipe("c5", n=12)
    P, ks, p0 = r.problem, r.ks(), r.p0()
    P.hx = P.hy = P.hz = H_C5
    r.options.precision = synth.FP64
    r.options.max_newton = 12
    v = np.zeros(P.n)
    v.reshape(P.nz, -1)[-1] = 1.0
    P.dt = 30.0
    assert v @ (orc.jacobian(P, ks, p0) @ v) < 0
    o = orc.Solver(P, r.options, ks)
    p = p0.copy()
    st = o.step(p)
    assert st["status"] == orc.MAXITER and st["linsolve_fails"] == st["newton_its"]
    P.dt = 3.0
    assert v @ (orc.jacobian(P, ks, p0) @ v) > 0
    o = orc.Solver(P, r.options, ks)
    p = p0.copy()
    for _ in range(3):
        assert o.step(p)["status"] == 0
