"""Pins of the oracle's constitutive laws, residual and Jacobian.

Each test checks the oracle against something other than its own formulas:
limits and special points of the laws, finite differences, the paper's own
printed expressions (Section 2.1 interior residual with its centred gravity
term; the expanded 3-D arithmetic Jacobian of Appendix B; the 1-D upstream
Jacobian of Appendix C), discrete conservation, the hydrostatic steady state
and closed-form spectra of constant-state Jacobians.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.helpers import all_dirichlet, box_problem, random_heads, random_ks

MEANS = [synth.ARITH, synth.UPSTREAM, synth.HARMONIC, synth.GEOMETRIC, synth.INTEGRAL]


def _P():
    return box_problem(4, 4, 4)


# ------------------------------------------------------------------ laws
def test_laws_special_points(orc):
    P = _P()
    # |p|^beta = alpha: theta is halfway between theta_r and theta_s
    p_half = -(P.alpha ** (1.0 / P.beta))
    th, dth, K, dK = orc.laws(P, np.array([p_half]), 1.0)
    assert th[0] == pytest.approx(0.5 * (P.theta_s + P.theta_r), rel=1e-14)
    # |p|^gamma = A: K is half of K_s
    p_k = -(P.A ** (1.0 / P.gamma))
    th, dth, K, dK = orc.laws(P, np.array([p_k]), 3.0)
    assert K[0] == pytest.approx(1.5, rel=1e-14)
    # saturated regime and the limits
    th, dth, K, dK = orc.laws(P, np.array([0.0, 2.0, -1e-9, -1e9]), 2.0)
    assert th[0] == P.theta_s and th[1] == P.theta_s and K[0] == 2.0 and K[1] == 2.0
    assert dth[0] == 0 and dK[0] == 0
    assert th[2] == pytest.approx(P.theta_s, rel=1e-12) and K[2] == pytest.approx(2.0, rel=1e-12)
    assert th[3] == pytest.approx(P.theta_r, rel=1e-9) and K[3] < 1e-30


def test_laws_monotone_and_derivatives_fd(orc):
    P = _P()
    p = -np.geomspace(0.5, 500.0, 400)
    th, dth, K, dK = orc.laws(P, p, 0.7)
    # wetter (larger p) means more water and more conductivity
    assert np.all(np.diff(th[::-1]) > 0) and np.all(np.diff(K[::-1]) > 0)
    assert np.all(dth > 0) and np.all(dK > 0)
    h = 1e-6 * np.abs(p)
    thp, _, Kp, _ = orc.laws(P, p + h, 0.7)
    thm, _, Km, _ = orc.laws(P, p - h, 0.7)
    eps = np.finfo(float).eps
    # truncation O(h^2) plus the rounding floor of the difference quotient
    assert np.all(np.abs((thp - thm) / (2 * h) - dth) <= 1e-6 * dth + 4 * eps * np.abs(th) / h)
    assert np.all(np.abs((Kp - Km) / (2 * h) - dK) <= 1e-6 * dK + 4 * eps * np.abs(K) / h)


def test_laws_continuity_at_zero(orc):
    P = _P()
    th, dth, K, dK = orc.laws(P, np.array([-1e-6, 0.0]), 1.0)
    assert abs(th[0] - th[1]) < 1e-12 and abs(K[0] - K[1]) < 1e-12
    assert dth[0] < 1e-12 and dK[0] < 1e-12  # C^1 since beta, gamma > 1


# -------------------------------------------------------------- residual
def paper_interior_residual(orc, P, ks, p, th_old, mean, mean_z=None):
    """Section 2.1 eq. (dynamic_of_the_problem), f = 0, written literally on the
    interior cells with the q's as printed (gravity: -K(p_{k+1})/(2 h_z) in
    q_{k+1/2} and -K(p_{k-1})/(2 h_z) in q_{k-1/2})."""
    nx, ny, nz = P.nx, P.ny, P.nz
    th, _, K, _ = orc.laws(P, p, ks)
    p3, K3 = p.reshape(nz, ny, nx), K.reshape(nz, ny, nx)
    ks3 = np.broadcast_to(ks, p.shape).reshape(nz, ny, nx)
    th3, tho3 = th.reshape(nz, ny, nx), th_old.reshape(nz, ny, nx)
    gt, gw = np.polynomial.legendre.leggauss(16)
    gt, gw = 0.5 * (gt + 1.0), 0.5 * gw

    def kav(KL, KU, pL, pU, ksL, ksU, m=mean):
        if m == synth.ARITH:
            return 0.5 * (KL + KU)
        if m == synth.HARMONIC:
            return 2 * KL * KU / (KL + KU)
        if m == synth.GEOMETRIC:
            return np.sqrt(KL * KU)
        if m == synth.INTEGRAL:  # average of K over [pL, pU] with the mean K_s
            kf = 0.5 * (ksL + ksU)
            psi = pL[None] + (pU - pL)[None] * gt[:, None, None, None]
            Kq = orc.laws(P, psi.ravel(), np.broadcast_to(kf[None], psi.shape).ravel())[2].reshape(psi.shape)
            return np.tensordot(gw, Kq, axes=1)
        return np.where(pU - pL >= 0, KU, KL)

    out = np.zeros((nz - 2, ny - 2, nx - 2))
    c = (slice(1, -1),) * 3
    for ax, h in ((2, P.hx), (1, P.hy), (0, P.hz)):
        up = [slice(1, -1)] * 3
        dn = [slice(1, -1)] * 3
        up[ax] = slice(2, None)
        dn[ax] = slice(0, -2)
        up, dn = tuple(up), tuple(dn)
        m = mean_z if (ax == 0 and mean_z is not None) else mean
        q_plus = -kav(K3[c], K3[up], p3[c], p3[up], ks3[c], ks3[up], m) * (p3[up] - p3[c]) / h**2
        q_minus = -kav(K3[dn], K3[c], p3[dn], p3[c], ks3[dn], ks3[c], m) * (p3[c] - p3[dn]) / h**2
        if ax == 0:
            q_plus = q_plus - K3[up] / (2 * h)
            q_minus = q_minus - K3[dn] / (2 * h)
        out += q_plus - q_minus
    out += (th3[c] - tho3[c]) / P.dt
    return out


@pytest.mark.parametrize("mean", MEANS)
def test_residual_equals_paper_interior_form(orc, mean):
    P = box_problem(7, 6, 9, mean=mean, dt=4.0)
    ks = random_ks(P, 1)
    p = random_heads(P.n, 2)
    th_old = orc.theta(P, random_heads(P.n, 3))
    F = orc.residual(P, ks, p, th_old).reshape(P.nz, P.ny, P.nx)[1:-1, 1:-1, 1:-1]
    ref = paper_interior_residual(orc, P, ks, p, th_old, mean)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(F - ref)) <= 1e-13 * scale


@pytest.mark.parametrize("mean", MEANS)
def test_conservation_noflux(orc, mean):
    """All faces no-flux: interior fluxes cancel pairwise, so sum Phi = sum (theta - theta_old)/dt."""
    bc = ((synth.NOFLUX,) * 6, (0.0,) * 6)
    P = box_problem(6, 5, 7, mean=mean, dt=3.0, bc=bc)
    ks = random_ks(P, 4)
    p = random_heads(P.n, 5, saturated_fraction=0.1)
    pold = random_heads(P.n, 6)
    th_old = orc.theta(P, pold)
    F = orc.residual(P, ks, p, th_old)
    storage = (orc.theta(P, p) - th_old) / P.dt
    flux_scale = np.max(np.abs(F - storage))
    assert flux_scale > 1e-6  # the fluxes are not trivially zero
    assert abs(F.sum() - storage.sum()) <= 1e-12 * flux_scale * P.n


@pytest.mark.parametrize("mean", MEANS)
def test_conservation_dirichlet_balance(orc, mean):
    """With Dirichlet faces the imbalance equals the net boundary flux, which
    is independent of the interior arrangement: perturbing heads of cells that
    touch no boundary leaves sum(Phi - storage) unchanged."""
    P = box_problem(6, 6, 6, mean=mean, bc=all_dirichlet())
    ks = random_ks(P, 7)
    p = random_heads(P.n, 8)
    th_old = orc.theta(P, p)
    F1 = orc.residual(P, ks, p, th_old) - (orc.theta(P, p) - th_old) / P.dt
    p2 = p.reshape(6, 6, 6).copy()
    p2[1:-1, 1:-1, 1:-1] += np.random.default_rng(9).uniform(-5, 5, (4, 4, 4))
    p2 = p2.ravel()
    F2 = orc.residual(P, ks, p2, th_old) - (orc.theta(P, p2) - th_old) / P.dt
    assert abs(F1.sum() - F2.sum()) <= 1e-11 * np.max(np.abs(F2)) * P.n


def test_hydrostatic_steady_state(orc):
    """p + z constant (no-flux sides and bottom, top held) is an exact steady state (arithmetic mean)."""
    P = box_problem(5, 4, 12, mean=synth.ARITH)
    ks = random_ks(P, 10, sigma=1.0)
    ztop = (P.nz + 1) * P.hz
    z = (np.arange(P.nz) + 1) * P.hz
    p = np.repeat(P.bc_value[5] + (ztop - z), P.nx * P.ny)
    th = orc.theta(P, p)
    F = orc.residual(P, ks, p, th)
    _, _, K, _ = orc.laws(P, p, ks)
    assert np.max(np.abs(F)) <= 1e-14 * np.max(K) / P.hz


# -------------------------------------------------------------- Jacobian
@pytest.mark.parametrize("mean", MEANS)
def test_jacobian_matches_finite_differences(orc, mean):
    P = box_problem(5, 4, 6, mean=mean, dt=2.0, bc=all_dirichlet())
    rng = np.random.default_rng(11)
    ks = random_ks(P, 12)
    # heads well separated so no upstream switch lies within the FD step
    p = -70 + 60 * rng.permutation(P.n) / P.n
    th_old = orc.theta(P, random_heads(P.n, 13))
    J = orc.jacobian(P, ks, p).toarray()
    Jfd = np.zeros_like(J)
    for j in range(P.n):
        h = 1e-6 * abs(p[j])
        e = np.zeros(P.n)
        e[j] = h
        Jfd[:, j] = (orc.residual(P, ks, p + e, th_old) - orc.residual(P, ks, p - e, th_old)) / (2 * h)
    scale = np.max(np.abs(J), axis=1, keepdims=True)
    assert np.max(np.abs(J - Jfd) / scale) <= 2e-6


def test_jacobian_paper_appendix_arithmetic(orc):
    """The expanded 3-D arithmetic-mean Jacobian entries printed in Appendix B."""
    P = box_problem(6, 5, 7, mean=synth.ARITH, dt=5.0)
    ks = np.full(P.n, synth.KS0)
    p = random_heads(P.n, 14)
    J = orc.jacobian(P, ks, p).tocsr()
    th, s1, K, K1 = orc.laws(P, p, ks)
    nx, ny = P.nx, P.ny
    hx2, hy2, hz2, hz = P.hx**2, P.hy**2, P.hz**2, P.hz
    errs = []
    for k in range(1, P.nz - 1):
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                c = i + nx * (j + ny * k)
                xm, xp, ym, yp, zm, zp = c - 1, c + 1, c - nx, c + nx, c - nx * ny, c + nx * ny
                diag = (s1[c] / P.dt + (K[xm] + K[xp] + 2 * K[c]) / (2 * hx2)
                        + (K[ym] + K[yp] + 2 * K[c]) / (2 * hy2) + (K[zm] + K[zp] + 2 * K[c]) / (2 * hz2)
                        + p[c] * (K1[c] / hx2 + K1[c] / hy2 + K1[c] / hz2)
                        - p[ym] * K1[c] / (2 * hy2) - p[zm] * K1[c] / (2 * hz2) - p[zp] * K1[c] / (2 * hz2)
                        - p[xm] * K1[c] / (2 * hx2) - p[xp] * K1[c] / (2 * hx2) - p[yp] * K1[c] / (2 * hy2))
                ref = {c: diag}
                for nb, h2 in ((xm, hx2), (xp, hx2), (ym, hy2), (yp, hy2)):
                    ref[nb] = -(K[nb] + K[c]) / (2 * h2) - p[nb] * K1[nb] / (2 * h2) + p[c] * K1[nb] / (2 * h2)
                ref[zm] = (-(K[zm] + K[c] - hz * K1[zm]) / (2 * hz2) - p[zm] * K1[zm] / (2 * hz2)
                           + p[c] * K1[zm] / (2 * hz2))
                ref[zp] = (-(K[zp] + K[c] + hz * K1[zp]) / (2 * hz2) - p[zp] * K1[zp] / (2 * hz2)
                           + p[c] * K1[zp] / (2 * hz2))
                for col, v in ref.items():
                    errs.append(abs(J[c, col] - v) / abs(diag))
    assert max(errs) <= 1e-13


def test_jacobian_paper_upstream_1d(orc):
    """The 1-D upstream tridiagonal Jacobian printed in Appendix C (Dirichlet ends)."""
    nz = 30
    bc = ((synth.NOFLUX,) * 4 + (synth.DIRICHLET, synth.DIRICHLET), (0,) * 4 + (-61.5, -20.7))
    P = box_problem(1, 1, nz, mean=synth.UPSTREAM, dt=0.1, L=(1.0, 1.0, 40.0), bc=bc)
    ks = np.full(nz, synth.KS0)
    rng = np.random.default_rng(15)
    p = -60 + 45 * rng.random(nz)
    J = orc.jacobian(P, ks, p).toarray()
    pe = np.concatenate([[-61.5], p, [-20.7]])  # with the boundary nodes
    _, s1, K, K1 = orc.laws(P, pe, np.full(nz + 2, synth.KS0))
    h, h2 = P.hz, P.hz**2
    for r in range(nz):
        i = r + 1
        up_lo = pe[i] - pe[i - 1] >= 0     # face (i-1, i): K_i if true
        up_hi = pe[i + 1] - pe[i] >= 0     # face (i, i+1): K_{i+1} if true
        zeta = (s1[i] / P.dt - pe[i - 1] / h2 * (K1[i] if up_lo else 0) - pe[i + 1] / h2 * (0 if up_hi else K1[i])
                + pe[i] / h2 * ((K1[i] if up_lo else 0) + (0 if up_hi else K1[i]))
                + ((K[i] if up_lo else K[i - 1]) + (K[i + 1] if up_hi else K[i])) / h2)
        assert J[r, r] == pytest.approx(zeta, rel=1e-13)
        if r + 1 < nz:
            xi = (-K1[i + 1] / (2 * h) - (K[i + 1] if up_hi else K[i]) / h2 + pe[i] / h2 * (K1[i + 1] if up_hi else 0)
                  - pe[i + 1] / h2 * (K1[i + 1] if up_hi else 0))
            assert J[r, r + 1] == pytest.approx(xi, rel=1e-12, abs=1e-15 * abs(zeta))
        if r > 0:
            eta = (K1[i - 1] / (2 * h) - (K[i] if up_lo else K[i - 1]) / h2 + pe[i] / h2 * (0 if up_lo else K1[i - 1])
                   - pe[i - 1] / h2 * (0 if up_lo else K1[i - 1]))
            assert J[r, r - 1] == pytest.approx(eta, rel=1e-12, abs=1e-15 * abs(zeta))


@pytest.mark.parametrize("mean", MEANS)
def test_constant_state_spectrum_closed_form(orc, mean):
    """Uniform head, homogeneous K_s, every face held at that head: J is a
    Kronecker sum of tridiagonal Toeplitz matrices whose eigenvalues are
    a + 2 sqrt(b c) cos(j pi / (n + 1))."""
    p0 = -40.0
    bc = ((synth.DIRICHLET,) * 6, (p0,) * 6)
    P = box_problem(4, 5, 6, mean=mean, dt=2.0, bc=bc)
    ks = np.full(P.n, synth.KS0)
    p = np.full(P.n, p0)
    J = orc.jacobian(P, ks, p).toarray()
    th, s1, K, K1 = orc.laws(P, np.array([p0]), synth.KS0)
    s1, K, K1 = s1[0], K[0], K1[0]
    ev = np.sort(np.linalg.eigvals(J).real)
    parts = []
    for n, h, grav in ((P.nx, P.hx, 0.0), (P.ny, P.hy, 0.0), (P.nz, P.hz, 1.0)):
        b = -K / h**2 - grav * K1 / (2 * h)  # coupling to the next index
        c = -K / h**2 + grav * K1 / (2 * h)  # coupling to the previous index
        j = np.arange(1, n + 1)
        parts.append(2 * K / h**2 + 2 * np.sqrt(b * c) * np.cos(j * math.pi / (n + 1)))
    lam = (s1 / P.dt + parts[0][:, None, None] + parts[1][None, :, None] + parts[2][None, None, :]).ravel()
    assert np.allclose(ev, np.sort(lam), rtol=1e-12, atol=0)


# ---------------------------------------------------------- auxiliary M
@pytest.mark.parametrize("mean", MEANS)
def test_auxiliary_symmetric_m_matrix_spd(orc, mean):
    P = box_problem(6, 5, 4, mean=mean, bc=all_dirichlet())
    ks = random_ks(P, 16)
    p = random_heads(P.n, 17, saturated_fraction=0.05)
    M = orc.auxiliary(P, ks, p)
    D = M.toarray()
    assert np.array_equal(D, D.T)  # bitwise symmetric
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0) and np.all(np.diag(D) > 0)
    # weakly diagonally dominant (equality for saturated interior cells, where theta' = 0)
    assert np.all(np.diag(D) >= -off.sum(axis=1) * (1 - 1e-14))
    assert np.linalg.eigvalsh(D).min() > 0
    # diffusion part equals J's symmetric frozen-coefficient part: at a
    # uniform head with uniform K_s, J - M is the gravity (skew-like) part
    bc = ((synth.DIRICHLET,) * 6, (-30.0,) * 6)
    P2 = box_problem(4, 4, 4, mean=mean, bc=bc)
    ks2 = np.full(P2.n, synth.KS0)
    p2 = np.full(P2.n, -30.0)
    Dm = (orc.jacobian(P2, ks2, p2) - orc.auxiliary(P2, ks2, p2)).toarray()
    assert np.allclose(Dm, -Dm.T, atol=1e-15 * np.abs(Dm).max())


@pytest.mark.parametrize("mean", MEANS)
def test_auxiliary_dflux_diagonal_is_the_diffusion_jacobian_diagonal(orc, mean):
    """With every face held (Dirichlet box) the two gravity derivative terms of a
    row cancel, so the diagonal of the flux-derivative auxiliary matrix must equal
    the Jacobian's; its off-diagonals are the frozen-coefficient ones."""
    P = box_problem(6, 5, 4, mean=mean, dt=3.0, bc=all_dirichlet())
    ks = random_ks(P, 18)
    p = random_heads(P.n, 19)
    J = orc.jacobian(P, ks, p)
    M = orc.auxiliary(P, ks, p)
    Md = orc.auxiliary(P, ks, p, dflux=True)
    assert np.allclose(Md.diagonal(), J.diagonal(), rtol=1e-13, atol=0)
    off = lambda A: (A - sp.diags(A.diagonal())).toarray()
    assert np.array_equal(off(Md), off(M))
    D = Md.toarray()
    assert np.array_equal(D, D.T)


# ------------------------------------------------------- interface means
def test_geometric_mean_between_harmonic_and_arithmetic(orc):
    """Section 2.1: K^G = sqrt(K_L K_U); the classical HM <= GM <= AM ordering."""
    rng = np.random.default_rng(21)
    for _ in range(20):
        pL, pU = rng.uniform(-80, -1, 2)
        kL, kU = synth.KS0 * np.exp(rng.normal(0, 2, 2))
        vals = {}
        for m in (synth.ARITH, synth.HARMONIC, synth.GEOMETRIC):
            P = _P()
            P.mean = m
            vals[m] = orc.face_mean(P, +1, pL, kL, pU, kU)[0]
        KL = orc.laws(_P(), np.array([pL]), kL)[2][0]
        KU = orc.laws(_P(), np.array([pU]), kU)[2][0]
        assert vals[synth.GEOMETRIC] ** 2 == pytest.approx(KL * KU, rel=1e-14)
        assert vals[synth.HARMONIC] <= vals[synth.GEOMETRIC] * (1 + 1e-15)
        assert vals[synth.GEOMETRIC] <= vals[synth.ARITH] * (1 + 1e-15)


def test_integral_mean_against_adaptive_quadrature(orc):
    """The integral mean of Section 2.1, (1/(p_U - p_L)) * integral of K over
    [p_L, p_U], against scipy's adaptive quadrature (the oracle's 16-point
    Gauss-Legendre rule is accurate to ~1e-6 across the saturation kink), its
    derivatives against central differences, the mean-value bounds, the
    equal-head limit K(p) and the symmetry in the two sides."""
    from scipy.integrate import quad
    P = _P()
    P.mean = synth.INTEGRAL
    ks = synth.KS0
    K = lambda x: orc.laws(P, np.array([x]), ks)[2][0]
    for pL, pU in ((-61.5, -20.7), (-40.0, 5.0), (-61.5, -1.0), (-30.0, -20.7), (-5.0, -70.0), (2.0, 4.0)):
        Kf, dL, dU = orc.face_mean(P, +1, pL, ks, pU, ks)
        ref = quad(K, pL, pU, epsabs=0, epsrel=1e-12, limit=200)[0] / (pU - pL)
        assert Kf == pytest.approx(ref, rel=2e-6)
        assert min(K(pL), K(pU)) * (1 - 1e-12) <= Kf <= max(K(pL), K(pU)) * (1 + 1e-12)
        h = 1e-5 * max(1.0, abs(pL))
        fdL = (orc.face_mean(P, +1, pL + h, ks, pU, ks)[0] - orc.face_mean(P, +1, pL - h, ks, pU, ks)[0]) / (2 * h)
        fdU = (orc.face_mean(P, +1, pL, ks, pU + h, ks)[0] - orc.face_mean(P, +1, pL, ks, pU - h, ks)[0]) / (2 * h)
        assert dL == pytest.approx(fdL, rel=1e-5, abs=1e-12 * Kf)
        assert dU == pytest.approx(fdU, rel=1e-5, abs=1e-12 * Kf)
        # seen from the other cell (direction -1) the same face gives the same mean
        Kr, dcr, dnr = orc.face_mean(P, -1, pU, ks, pL, ks)
        assert Kr == Kf and dcr == dU and dnr == dL
    Kf = orc.face_mean(P, +1, -33.0, ks, -33.0, ks)[0]
    assert Kf == pytest.approx(K(-33.0), rel=1e-14)


@pytest.mark.parametrize("mean,mean_z", [(synth.ARITH, synth.UPSTREAM), (synth.HARMONIC, synth.ARITH),
                                         (synth.UPSTREAM, synth.INTEGRAL)])
def test_per_direction_means(orc, mean, mean_z):
    """Section 2.1's combination of two means, one for the horizontal and one
    for the vertical direction: Phi equals the literal interior form with the
    per-axis means, and J matches central differences."""
    P = box_problem(6, 5, 7, mean=mean, dt=4.0)
    P.mean_vertical = mean_z
    ks = random_ks(P, 31)
    p = random_heads(P.n, 32)
    th_old = orc.theta(P, random_heads(P.n, 33))
    F = orc.residual(P, ks, p, th_old).reshape(P.nz, P.ny, P.nx)[1:-1, 1:-1, 1:-1]
    ref = paper_interior_residual(orc, P, ks, p, th_old, mean, mean_z)
    assert np.max(np.abs(F - ref)) <= 1e-12 * np.max(np.abs(ref))
    P2 = box_problem(4, 3, 5, mean=mean, dt=2.0, bc=all_dirichlet())
    P2.mean_vertical = mean_z
    rng = np.random.default_rng(34)
    ks2 = random_ks(P2, 35)
    p2 = -70 + 60 * rng.permutation(P2.n) / P2.n
    th2 = orc.theta(P2, random_heads(P2.n, 36))
    J = orc.jacobian(P2, ks2, p2).toarray()
    for j in range(P2.n):
        h = 1e-6 * abs(p2[j])
        e = np.zeros(P2.n)
        e[j] = h
        col = (orc.residual(P2, ks2, p2 + e, th2) - orc.residual(P2, ks2, p2 - e, th2)) / (2 * h)
        assert np.allclose(J[:, j], col, rtol=1e-5, atol=1e-7 * np.abs(J).max())
