"""Pins of the reference oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, values printed in the paper (tests/golden), invariants, special cases
that reduce to textbook results, and brute force.  None of these needs a GPU.
"""
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(20260207)


def _rand_points(n, a, rlo=1.8, rhi=30.0):
    r = RNG.uniform(rlo, rhi, n)
    th = RNG.uniform(0.15, np.pi - 0.15, n)
    return r, th


# ------------------------------------------------------------------ metric
@pytest.mark.parametrize("a", [0.0, 0.7, 0.9, 0.99])
def test_metric_inverse_and_determinant(a):
    """App. A: gamma^ij is the inverse of gamma_ij and det = rho^4 xi sin^2."""
    for r, th in zip(*_rand_points(20, a)):
        m = O.metric(a, r, th)
        g = np.array([[m[2], 0, m[5]], [0, m[3], 0], [m[5], 0, m[4]]])
        gi = np.array([[m[6], 0, m[9]], [0, m[7], 0], [m[9], 0, m[8]]])
        assert np.allclose(g @ gi, np.eye(3), atol=1e-13, rtol=0)
        rho2 = r * r + a * a * np.cos(th) ** 2
        xi = 1 + 2 * r / rho2
        assert np.isclose(np.linalg.det(g), rho2 ** 2 * xi * np.sin(th) ** 2, rtol=1e-12)
        assert np.isclose(m[10] ** 2, np.linalg.det(g), rtol=1e-12)
        # lapse / shift from the 4-metric: g_00 = -alpha^2 + beta_r beta^r
        # and beta_r = gamma_rr beta^r = 2r/rho^2 (Kerr-Schild g_0r)
        assert np.isclose(m[2] * m[1], 2 * r / rho2, rtol=1e-13)


def test_metric_schwarzschild_limit():
    """a -> 0: diagonal Kerr-Schild Schwarzschild metric (App. A, last line)."""
    for r, th in zip(*_rand_points(10, 0.0)):
        m = O.metric(0.0, r, th)
        s2 = np.sin(th) ** 2
        assert np.allclose(m[[2, 3, 4, 5]], [1 + 2 / r, r * r, r * r * s2, 0.0], rtol=1e-14, atol=0)
        assert np.isclose(m[0], 1 / np.sqrt(1 + 2 / r), rtol=1e-14)
        assert np.isclose(m[1], 2 / (r + 2), rtol=1e-14)


@pytest.mark.parametrize("a", [0.0, 0.9, 0.99])
def test_metric_derivatives_match_finite_differences(a):
    """Analytic d_r, d_theta of alpha, beta^r, gamma^ij (Sec. 2.2) vs central
    differences of the metric itself."""
    idx = [0, 1, 6, 7, 8, 9]
    for r, th in zip(*_rand_points(15, a)):
        d = O.metric_deriv(a, r, th)
        h = 2e-6
        for n, i in enumerate(idx):
            fr = (O.metric(a, r + h, th)[i] - O.metric(a, r - h, th)[i]) / (2 * h)
            ft = (O.metric(a, r, th + h)[i] - O.metric(a, r, th - h)[i]) / (2 * h)
            sc = max(1.0, abs(O.metric(a, r, th)[i]), abs(d[2 * n]), abs(d[2 * n + 1]))
            assert abs(d[2 * n] - fr) < 1e-8 * sc
            assert abs(d[2 * n + 1] - ft) < 1e-8 * sc


@pytest.mark.parametrize("k", [0, 1])
def test_metric_divided_differences(k):
    """The cancellation-free divided differences used by the discrete-gradient
    scheme equal the plain quotient of the metric for a finite step and the
    analytic derivative at the midpoint for a tiny one."""
    idx = [0, 1, 6, 7, 8, 9]
    for a in (0.0, 0.9, 0.99):
        for r, th in zip(*_rand_points(8, a)):
            dx = 0.05
            r1, t1 = (r + dx, th) if k == 0 else (r, th + dx)
            m0, m1 = O.metric(a, r, th), O.metric(a, r1, t1)
            plain = np.array([(m1[i] - m0[i]) / dx for i in idx])
            dd = O.metric_divdiff(a, k, r, th, r1, t1)
            assert np.allclose(dd, plain, rtol=1e-11, atol=1e-13)
            dx = 1e-8
            r1, t1 = (r + dx, th) if k == 0 else (r, th + dx)
            d = O.metric_deriv(a, r + (dx / 2 if k == 0 else 0), th + (dx / 2 if k == 1 else 0))
            dd = O.metric_divdiff(a, k, r, th, r1, t1)
            assert np.allclose(dd, d[[k, 2 + k, 4 + k, 6 + k, 8 + k, 10 + k]], rtol=1e-12,
                               atol=1e-14)


# --------------------------------------------------------- equations of motion
def _grad(fun, z, h=1e-6):
    g = np.zeros(6)
    for i in range(6):
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        g[i] = (fun(zp) - fun(zm)) / (2 * h)
    return g


@pytest.mark.parametrize("a", [0.0, 0.9, 0.995])
def test_neutral_rhs_is_hamiltonian_flow(a):
    """eqs. p1/p2: (dx/dt, du/dt) = (dH/du, -dH/dx) with H of eq. Ham (q=0)."""
    for _ in range(10):
        z = np.array([RNG.uniform(2, 20), RNG.uniform(0.2, 2.9), RNG.uniform(0, 6),
                      RNG.normal(), RNG.normal() * 2, RNG.normal() * 3])
        f = O.rhs(a, 0.0, z)
        g = _grad(lambda y: O.energy(a, y), z)
        assert np.allclose(f, np.r_[g[3:], -g[:3]], atol=2e-8, rtol=0)


@pytest.mark.parametrize("qm", [1.0, -1.0])
@pytest.mark.parametrize("a", [0.0, 0.7, 0.9])
def test_charged_wald_conserves_H_and_L(a, qm):
    """Sec. 3.1.3: in the Wald field H = -u_0 - (q/m) A_0 and
    L = u_phi + (q/m) A_phi are constants of the motion: their gradients are
    orthogonal to the flow F of eqs. p1-O2."""
    B0 = 2.0
    H = lambda y: O.energy(a, y) - qm * O.wald_potential(a, B0, y[0], y[1])[0]
    L = lambda y: y[5] + qm * O.wald_potential(a, B0, y[0], y[1])[3]
    for _ in range(8):
        z = np.array([RNG.uniform(2, 12), RNG.uniform(0.3, 2.8), 0.4,
                      RNG.normal(), RNG.normal(), RNG.normal() * 2])
        D, B = O.wald_fields(a, B0, z[0], z[1])
        f = O.rhs(a, qm, z, D, B)
        gH, gL = _grad(H, z), _grad(L, z)
        assert abs(gH @ f) < 1e-8 * max(np.abs(f).max() * np.abs(gH).max(), 1)
        assert abs(gL @ f) < 1e-8 * max(np.abs(f).max() * np.abs(gL).max(), 1)


@pytest.mark.parametrize("a,af", [(0.0, 0.0), (0.9, 0.9), (0.99, 0.99), (0.999, 0.0),
                                  (0.9, 0.5)])
def test_wald_field_is_curl_of_potential(a, af):
    """App. B.1: B^i = eta^ijk d_j A_k / sqrt(g); E_i = d_i A_0; E_phi = 0,
    with E_i = alpha D_i + sqrt(g) eta_ijk beta^j B^k (eq. Ei).  The
    potential may carry its own spin af (Sec. 3.3): curl and A_0 from the af
    potential, sqrt(g), alpha, beta, gamma from the spacetime's a."""
    B0, h = 1.3, 1e-6
    for r, th in zip(*_rand_points(10, a, 1.6, 15)):
        D, B = O.wald_fields(a, B0, r, th, a_field=af)
        A = lambda rr, tt: O.wald_potential(af, B0, rr, tt)
        dA_r = (A(r + h, th) - A(r - h, th)) / (2 * h)
        dA_t = (A(r, th + h) - A(r, th - h)) / (2 * h)
        m = O.metric(a, r, th)
        sg = m[10]
        assert np.isclose(B[0], dA_t[3] / sg, rtol=1e-7, atol=1e-9)
        assert np.isclose(B[1], -dA_r[3] / sg, rtol=1e-7, atol=1e-9)
        assert np.isclose(B[2], -dA_t[1] / sg, rtol=1e-7, atol=1e-9)
        Dl = np.array([[m[2], 0, m[5]], [0, m[3], 0], [m[5], 0, m[4]]]) @ D
        E = m[0] * Dl + sg * m[1] * np.array([0.0, -B[2], B[1]])
        assert np.allclose(E, [dA_r[0], dA_t[0], 0.0], rtol=1e-7, atol=1e-9)
    # the spin-a default is the af = a field
    assert np.array_equal(np.r_[O.wald_fields(a, B0, 3.0, 1.0)],
                          np.r_[O.wald_fields(a, B0, 3.0, 1.0, a_field=a)])


@pytest.mark.parametrize("a", [0.7, 0.999])
def test_schwarzschild_wald_start_in_kerr(a):
    """Sec. 3.3: a Kerr hole started with the a = 0 Wald field.  A_phi is
    B0 r^2 sin^2(theta) / 2 and A_0 = A_r = 0, so sqrt(g) B^r =
    B0 r^2 sin cos, sqrt(g) B^theta = -B0 r sin^2, B^phi = 0; the grid field
    E_i vanishes, D = -beta x B / alpha, and D_i B^i = 0 everywhere."""
    B0 = 1e3
    for r, th in zip(*_rand_points(12, a, 1.02 * _rplus(a), 20)):
        D, B = O.wald_fields(a, B0, r, th, a_field=0.0)
        m = O.metric(a, r, th)
        sg, s, c = m[10], np.sin(th), np.cos(th)
        assert np.isclose(B[0] * sg, B0 * r * r * s * c, rtol=1e-13, atol=1e-13 * B0)
        assert np.isclose(B[1] * sg, -B0 * r * s * s, rtol=1e-13)
        assert B[2] == 0.0
        Dl = np.array([[m[2], 0, m[5]], [0, m[3], 0], [m[5], 0, m[4]]]) @ D
        # (beta x B)_i = sqrt(g) eta_ijk beta^j B^k with beta = (beta^r, 0, 0)
        bxB = sg * m[1] * np.array([0.0, -B[2], B[1]])
        assert np.allclose(Dl, -bxB / m[0], rtol=1e-12, atol=1e-12 * B0)
        assert abs(Dl @ B) <= 1e-12 * np.linalg.norm(Dl) * np.linalg.norm(B) + 1e-300
    # and it differs from the Kerr Wald field of the same spacetime
    Dk, Bk = O.wald_fields(a, B0, 3.0, 1.0)
    D0, B0f = O.wald_fields(a, B0, 3.0, 1.0, a_field=0.0)
    assert not np.allclose(Bk, B0f, rtol=1e-3)


@pytest.mark.parametrize("a", [0.0, 0.9, 0.99])
def test_circular_orbits_are_equilibria(a):
    """Prograde equatorial circular orbits (Bardeen-Press-Teukolsky closed
    forms) with the Kerr-Schild u_r = (2rE - aL)/Delta are fixed points of
    the radial motion, rotate at Omega = 1/(r^1.5 + a) and have H = E."""
    for r in (8.0, 15.0, 40.0):
        Dn = r ** 0.75 * np.sqrt(r ** 1.5 - 3 * r ** 0.5 + 2 * a)
        E = (r ** 1.5 - 2 * r ** 0.5 + a) / Dn
        L = (r * r - 2 * a * r ** 0.5 + a * a) / Dn
        z = np.array([r, np.pi / 2, 0.0, (2 * r * E - a * L) / (r * r - 2 * r + a * a), 0.0, L])
        f = O.rhs(a, 0.0, z)
        assert abs(f[0]) < 1e-14 and abs(f[3]) < 1e-14 and abs(f[4]) < 1e-14
        assert np.isclose(f[2], 1 / (r ** 1.5 + a), rtol=1e-13)
        assert np.isclose(O.energy(a, z), E, rtol=1e-14)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9])
def test_isco_marks_radial_stability(a):
    """The radial motion at fixed u_phi is a one-degree-of-freedom
    Hamiltonian flow; its linearisation about a circular orbit has
    det(J) > 0 (stable) outside the ISCO and < 0 inside (BPT r_isco)."""
    Z1 = 1 + (1 - a * a) ** (1 / 3) * ((1 + a) ** (1 / 3) + (1 - a) ** (1 / 3))
    Z2 = np.sqrt(3 * a * a + Z1 * Z1)
    risco = 3 + Z2 - np.sqrt((3 - Z1) * (3 + Z1 + 2 * Z2))

    def detJ(r):
        Dn = r ** 0.75 * np.sqrt(r ** 1.5 - 3 * r ** 0.5 + 2 * a)
        E = (r ** 1.5 - 2 * r ** 0.5 + a) / Dn
        L = (r * r - 2 * a * r ** 0.5 + a * a) / Dn
        z = np.array([r, np.pi / 2, 0.0, (2 * r * E - a * L) / (r * r - 2 * r + a * a), 0.0, L])
        J = np.zeros((2, 2))
        for col, i in enumerate((0, 3)):
            h = 1e-6
            zp, zm = z.copy(), z.copy()
            zp[i] += h
            zm[i] -= h
            d = (O.rhs(a, 0, zp) - O.rhs(a, 0, zm)) / (2 * h)
            J[:, col] = d[[0, 3]]
        return np.linalg.det(J)

    assert detJ(risco * 1.02) > 0
    assert detJ(risco * 0.98) < 0


def _table_rows():
    rows = []
    with open(os.path.join(GOLD, "table1_neutral.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, a, E, r0, ur, uph = line.split()
                rows.append((name, float(a), float(E), float(r0), float(ur), float(uph)))
    return rows


@pytest.mark.parametrize("row", _table_rows(), ids=lambda r: r[0])
def test_table1_neutral_initial_energy(row):
    """Table tab:params (App. C): H(z^0) reproduces the printed E to the
    table's printed precision."""
    name, a, E, r0, ur, uph = row
    z = [r0, np.pi / 2, 0.0, ur, 0.0, uph]
    assert abs(O.energy(a, z) / E - 1) < 5e-9


def test_table1_rka8_angular_momentum():
    """Table tab:params RKA8 row: L = u_phi + (q/m) A_phi (Sec. 3.1.3, with
    the factor B0) equals the printed 5.0."""
    with open(os.path.join(GOLD, "table1_charged.txt")) as f:
        line = [l for l in f if l.strip() and not l.startswith("#")][0].split()
    a, B0, E, L, r0, th0, ur, ut, up = map(float, line[1:])
    A = O.wald_potential(a, B0, r0, th0)
    assert abs(up + A[3] - L) < 5e-5


# ------------------------------------------------------------------ pushers
ORBIT = (0.995, np.array([10.021533, np.pi / 2, 0.0, 0.201211, 0.0, 2.0]))
ORBIT2 = (0.995, np.array([4.376281, np.pi / 2, 0.0, 0.487625, 0.0, 1.82]))


def _evolve(stepfun, z, n):
    for _ in range(n):
        z = stepfun(z)
    return z


def test_rk4_is_fourth_order():
    """Sec. 2.2.1: global error of RK4 falls by 2^4 when dt halves."""
    a, z0 = ORBIT
    T = 8.0

    def run(dt):
        P = O.push_params(a, dt)
        return _evolve(lambda z: O.step_rk4(P, 0.0, z)[0], z0.copy(), int(round(T / dt)))

    ref = run(0.0125)
    e1 = np.abs(run(0.2) - ref).max()
    e2 = np.abs(run(0.1) - ref).max()
    assert 12 < e1 / e2 < 20


def test_imr_second_order_and_time_reversible():
    """Sec. 2.2.2: the implicit midpoint rule is second order and symmetric."""
    a, z0 = ORBIT
    T = 8.0

    def run(dt):
        P = O.push_params(a, dt, tol=1e-15, kmax=200)
        return _evolve(lambda z: O.step_imr(P, 0.0, z)[0], z0.copy(), int(round(T / dt)))

    ref = run(0.0125)
    e1 = np.abs(run(0.2) - ref).max()
    e2 = np.abs(run(0.1) - ref).max()
    assert 3.5 < e1 / e2 < 4.5
    P = O.push_params(a, 0.1, tol=1e-15, kmax=200)
    Pb = O.push_params(a, -0.1, tol=1e-15, kmax=200)
    z1 = O.step_imr(P, 0.0, z0)[0]
    zb = O.step_imr(Pb, 0.0, z1)[0]
    assert np.abs(zb - z0).max() < 1e-12


def test_imr_fixed_point_independent_of_guess():
    """Any starting guess converges to the same IMR solution (the property
    the learned guess relies on)."""
    a, z0 = ORBIT2
    P = O.push_params(a, 0.1, tol=1e-14, kmax=100)
    z_plain, k1, _ = O.step_imr(P, 0.0, z0)
    z_rk4 = O.step_rk4(P, 0.0, z0)[0]
    z_g, k2, _ = O.step_imr(P, 0.0, z0, guess=z_rk4)
    assert np.abs(z_plain - z_g).max() < 1e-13
    assert 0 < k2 < k1


def test_hamiltonian_scheme_conserves_energy_exactly():
    """Sec. 2.2.3 / App. D: the discrete-gradient scheme conserves H to
    round-off and keeps u_phi exactly constant (strong-field orbit a.995_2
    at the paper's dt = 0.1)."""
    a, z0 = ORBIT2
    # 1e-13: the rounding floor of the difference quotients at dt = 0.1
    P = O.push_params(a, 0.1, tol=1e-13, kmax=100)
    H0 = O.energy(a, z0)
    z = z0.copy()
    worst = 0.0
    for _ in range(400):
        z, k = O.step_ham(P, z)
        assert k > 0
        assert z[5] == z0[5]
        worst = max(worst, abs(O.energy(a, z) / H0 - 1))
    assert worst < 5e-14
    # RK4 at the same dt violates it by orders of magnitude more
    z = z0.copy()
    worst_rk = 0.0
    for _ in range(400):
        z = O.step_rk4(P, 0.0, z)[0]
        worst_rk = max(worst_rk, abs(O.energy(a, z) / H0 - 1))
    assert worst_rk > 1e3 * worst


def test_hamiltonian_scheme_second_order_and_reversible():
    a, z0 = ORBIT
    T = 8.0

    def run(dt):
        P = O.push_params(a, dt, tol=1e-13, kmax=200)
        return _evolve(lambda z: O.step_ham(P, z)[0], z0.copy(), int(round(T / dt)))

    ref = run(0.0125)
    e1 = np.abs(run(0.2) - ref).max()
    e2 = np.abs(run(0.1) - ref).max()
    assert 3.3 < e1 / e2 < 4.7
    P = O.push_params(a, 0.1, tol=1e-13, kmax=200)
    Pb = O.push_params(a, -0.1, tol=1e-13, kmax=200)
    z1 = O.step_ham(P, z0)[0]
    assert np.abs(O.step_ham(Pb, z1)[0] - z0).max() < 1e-12


def _c1_particles(n=64):
    return O.init_particles(O.INIT_ORBITS, 0.0, 7, n, 6.0, 20.0, np.pi / 4, 3 * np.pi / 4, 0.1)


@pytest.mark.parametrize("pusher,implicit", [(O.HYB1, O.HAM), (O.HYB2, O.HAM)])
def test_hybrid_threshold_limits_neutral(pusher, implicit):
    """The hybrid with an infinite threshold is RK4 and with a zero
    threshold is the implicit scheme, bit for bit."""
    base = _c1_particles()
    for thr, ref_pusher in ((np.inf, O.RK4), (-np.inf, implicit)):
        p1, p2 = base.copy(), base.copy()
        O.push(O.push_params(0.0, 0.05, pusher=pusher, thr=thr, r_min=2.0), p1)
        O.push(O.push_params(0.0, 0.05, pusher=ref_pusher, r_min=2.0), p2)
        assert np.array_equal(p1.state(), p2.state())


def test_hybrid_threshold_limits_charged():
    a, B0 = 0.9, 1.0
    base = O.init_particles(O.INIT_SHELL_ISO, a, 3, 64, 2.0, 10.0, 0.3, 2.8, 1.0)
    for thr, ref_pusher in ((np.inf, O.RK4), (-np.inf, O.IMR)):
        p1, p2 = base.copy(), base.copy()
        kw = dict(field_kind=O.FIELDS_WALD, B0=B0, r_min=1.44)
        O.push(O.push_params(a, 0.05, pusher=O.HYB2, thr=thr, **kw), p1)
        O.push(O.push_params(a, 0.05, pusher=ref_pusher, **kw), p2)
        assert np.array_equal(p1.state(), p2.state())


def test_hyb2_bounds_energy_violation():
    """Sec. 3.1.2: Hyb2 keeps |H - H0|/H0 below its threshold while RK4 alone
    exceeds it (a.995_2, dt = 0.05, threshold 1e-12 as in Table 2)."""
    a, z0 = ORBIT2
    thr = 1e-12
    p = O.Particles.from_state(z0, 0.0)
    p.H0[:] = O.energy(a, z0)
    q = p.copy()
    Ph = O.push_params(a, 0.05, pusher=O.HYB2, thr=thr, tol=1e-13, kmax=200)
    Pr = O.push_params(a, 0.05)
    worst_h = worst_r = 0.0
    n_impl = 0
    for _ in range(600):
        O.push(Ph, p)
        O.push(Pr, q)
        n_impl += int(p.flags[0] & O.IMPLICIT != 0)
        worst_h = max(worst_h, abs(O.energy(a, p.state()[0]) / p.H0[0] - 1))
        worst_r = max(worst_r, abs(O.energy(a, q.state()[0]) / p.H0[0] - 1))
    # below the threshold up to the implicit scheme's own round-off drift
    assert worst_h < thr + 1e-14
    assert worst_r > thr
    assert 0 < n_impl < 600


def test_charged_energy_budget_residual_is_rk4_local_error():
    """The charged switch quantity |e' - e - W|/|e| (reading for grid fields)
    falls like dt^5 for RK4 on a smooth field."""
    a, B0 = 0.9, 1.0
    z0 = np.array([5.0, 1.2, 0.0, 0.3, 0.4, 1.5])
    vals = []
    for dt in (0.04, 0.02):
        P = O.push_params(a, dt, field_kind=O.FIELDS_WALD, B0=B0)
        z1, W = O.step_rk4(P, 1.0, z0)
        e0 = O.energy(a, z0)
        vals.append(abs(O.energy(a, z1) - e0 - W) / abs(e0))
    assert 20 < vals[0] / vals[1] < 45


@pytest.mark.parametrize("dt", [0.05, 0.5, 1.0])
def test_newton_solves_the_same_midpoint_equation(dt):
    """The implicit midpoint equation (eq. imr1) has one solution near z^n:
    Newton's method (the solver Sec. 2.2.2 names) and the Picard iteration
    reach it to the stopping tolerance; Newton converges quadratically, in
    at most five iterations, where Picard needs many more as dt grows."""
    a, B0 = 0.9, 1.0
    rng = np.random.default_rng(31)
    kw = dict(field_kind=O.FIELDS_WALD, B0=B0, kmax=200, tol=1e-13)
    itp, itn = [], []
    for _ in range(12):
        z = np.array([rng.uniform(3, 12), rng.uniform(0.4, 2.7), 0.3, rng.normal(),
                      rng.normal(), rng.normal() * 2])
        qm = rng.choice([-1.0, 1.0])
        zp, ip, Wp = O.step_imr(O.push_params(a, dt, **kw), qm, z)
        zn, inn, Wn = O.step_imr(O.push_params(a, dt, solver=O.SOLVER_NEWTON, **kw), qm, z)
        assert ip > 0 and inn > 0
        assert np.all(np.abs(zp - zn) <= 2e-12 * np.maximum(np.abs(zp), 1))
        # the solution satisfies eq. imr1 itself
        f = O.rhs(a, qm, 0.5 * (z + zn), *O.wald_fields(a, B0, *(0.5 * (z + zn))[:2]))
        assert np.all(np.abs(zn - z - dt * f) <= 1e-12 * np.maximum(np.abs(zn), 1))
        itp.append(ip)
        itn.append(inn)
    assert max(itn) <= 5
    if dt >= 0.5:
        assert np.mean(itp) > 2.5 * np.mean(itn)


def test_nonfinite_state_is_removed_and_isolated():
    """A particle whose step gives a non-finite state is flagged and taken
    out (it then deposits nothing); the others step as without it."""
    base = _c1_particles(16)
    bad = base.copy()
    bad.ur[5] = np.nan
    bad.uph[9] = np.inf
    for pusher, thr in ((O.RK4, 0.0), (O.HYB2, 1e-15), (O.HAM, 0.0)):
        P = O.push_params(0.0, 0.05, pusher=pusher, thr=thr, r_min=2.0)
        p1, p2 = base.copy(), bad.copy()
        O.push(P, p1)
        O.push(P, p2)
        for k in (5, 9):
            assert p2.flags[k] == O.REMOVED | O.NONFINITE
        ok = np.ones(16, bool)
        ok[[5, 9]] = False
        assert np.array_equal(p1.state()[ok], p2.state()[ok])
        assert np.array_equal(p1.flags[ok], p2.flags[ok])


# --------------------------------------- own step lengths (Sec. 3.1.2, Table 2)
def _clocked(p):
    p = p.copy()
    p.t = np.zeros(p.n)
    return p


def test_particle_clocks_without_own_lengths_change_nothing():
    """Clocks with dt_impl = dt and no end: the same states and flags as the
    fixed-step push, and every clock is the running sum of dt."""
    base = _c1_particles()
    p1, p2 = base.copy(), _clocked(base)
    P = O.push_params(0.0, 0.05, pusher=O.HYB2, thr=1e-15, r_min=2.0)
    t = 0.0
    for _ in range(12):
        O.push(P, p1)
        O.push(P, p2)
        t += 0.05
    assert np.array_equal(p1.state(), p2.state()) and np.array_equal(p1.flags, p2.flags)
    assert np.all(p2.t[(p2.flags & O.ALIVE) != 0] == t)


def test_each_scheme_advances_by_its_own_step():
    """Table 2 pairs a Delta t_RK4 with a Delta t_Ham: a hybrid that always
    accepts is RK4 at dt (clock n dt), one that always rejects is the
    discrete-gradient scheme at dt_impl (clock n dt_impl), each checked
    against the single-step routines called with that step; a mixed run
    advances every clock by the step its scheme took."""
    base = _c1_particles(16)
    for thr, dt_used in ((np.inf, 0.5), (-np.inf, 1.0)):
        p = _clocked(base)
        P = O.push_params(0.0, 0.5, pusher=O.HYB2, thr=thr, r_min=2.0, dt_impl=1.0)
        z = base.state()
        for _ in range(3):
            O.push(P, p)
            for k in range(base.n):
                Q = O.push_params(0.0, dt_used, r_min=2.0)
                z[k] = O.step_rk4(Q, 0.0, z[k])[0] if thr > 0 else O.step_ham(Q, z[k])[0]
        assert np.array_equal(p.state(), z)
        assert np.all(p.t == 3 * dt_used)
    p = _clocked(_c1_particles())
    P = O.push_params(0.0, 0.5, pusher=O.HYB2, thr=1e-15, r_min=2.0, dt_impl=1.0)
    for _ in range(6):
        t0 = p.t.copy()
        O.push(P, p)
        alive = (p.flags & O.ALIVE) != 0
        impl = (p.flags & O.IMPLICIT) != 0
        assert np.all((p.t - t0)[alive & impl] == 1.0)
        assert np.all((p.t - t0)[alive & ~impl] == 0.5)
        assert impl[alive].any() and (~impl[alive]).any()


def test_clocks_stop_exactly_at_t_end():
    """With an end time the last step is clipped to the time left and lands
    on t_end; afterwards the particles stay put.  The clipped explicit step
    is RK4 with the remaining time as its step."""
    p = _clocked(_c1_particles(32))
    t_end = 2.3
    P = O.push_params(0.0, 0.5, pusher=O.HYB2, thr=1e-15, r_min=2.0, dt_impl=1.0, t_end=t_end)
    for _ in range(8):
        before, t0 = p.copy(), p.t.copy()
        O.push(P, p)
        alive = (p.flags & O.ALIVE) != 0
        last = alive & (t0 == 2.0) & ((p.flags & O.IMPLICIT) == 0)
        for k in np.nonzero(last)[0]:
            Q = O.push_params(0.0, t_end - 2.0, r_min=2.0)
            assert np.array_equal(p.state()[k], O.step_rk4(Q, 0.0, before.state()[k])[0])
    alive = (p.flags & O.ALIVE) != 0
    assert np.all(p.t[alive] == t_end)
    frozen = p.copy()
    O.push(P, p)
    assert np.array_equal(p.state(), frozen.state()) and np.array_equal(p.t, frozen.t)
    assert np.all(p.flags[alive] == O.ALIVE) and np.all(p.iters == 0)


def test_table2_hybrid_keeps_energy_in_a_tenth_of_the_steps():
    """Sec. 3.1.2 with the a.0 row of Table 2: Hyb2 (Delta t_RK4 = 0.5,
    Delta t_Ham = 1, threshold 1e-15) reaches t = 200 in at most 400 steps
    per particle, against 4000 for RK4 at 0.05, with a worst energy
    violation no larger than RK4's and at the 1e-14 level."""
    T = 200.0
    worst, steps = {}, {}
    for name, pusher, dt, dt_impl, thr in (("rk4", O.RK4, 0.05, 0.0, 0.0),
                                           ("hyb2", O.HYB2, 0.5, 1.0, 1e-15)):
        p = _clocked(_c1_particles())
        P = O.push_params(0.0, dt, pusher=pusher, thr=thr, r_min=2.0, dt_impl=dt_impl, t_end=T)
        n = 0
        while (p.t[(p.flags & O.ALIVE) != 0] < T).any():
            O.push(P, p)
            n += 1
        alive = (p.flags & O.ALIVE) != 0
        H = np.array([O.energy(0.0, z) for z in p.state()[alive]])
        worst[name] = np.max(np.abs(H - p.H0[alive]) / np.abs(p.H0[alive]))
        steps[name] = n
    assert steps["rk4"] == 4000 and steps["hyb2"] <= 400
    assert worst["hyb2"] <= worst["rk4"] and worst["hyb2"] < 1e-13


# ----------------------------------------------------------------- gather
def test_gather_exact_for_bilinear_densitized_fields():
    """The metric-weighted bilinear gather reproduces exactly any field
    whose sqrt(g) F is bilinear in (r, theta) on its sub-grid."""
    g = O.Grid(0.9, 12, 10, 1.3, 15.0)
    coef = RNG.normal(size=(6, 4))
    G = []
    for c in range(6):
        nT, nR = g.shape(c)
        R = (g.rh if c in (0, 4, 5) else g.rn)[:nR]
        T = (g.th if c in (1, 3, 5) else g.tn)[:nT]
        k = coef[c]
        G.append(k[0] + k[1] * R[None, :] + k[2] * T[:, None] + k[3] * R[None, :] * T[:, None])
    for _ in range(30):
        r, th = RNG.uniform(2.0, 13.0), RNG.uniform(0.4, 2.7)
        D, B = O.gather(g, G, r, th)
        sg = O.metric(0.9, r, th)[10]
        for c in range(6):
            k = coef[c]
            want = (k[0] + k[1] * r + k[2] * th + k[3] * r * th) / sg
            got = (D if c < 3 else B)[c % 3]
            assert abs(got - want) < 1e-12 * max(1, abs(want))


# ---------------------------------------------------------------- deposit
def test_deposit_weights_partition_and_flat_cic():
    """eqs. v1-v5: weights sum to one; with sqrt(g) = 1 they are the
    bilinear (cloud-in-cell) weights."""
    g = O.Grid(0.9, 10, 10, 1.3, 15.0)
    for _ in range(20):
        p, q = RNG.integers(0, 10), RNG.integers(0, 10)
        fr, ft = RNG.uniform(), RNG.uniform()
        r = g.rn[p] + fr * (g.rn[p + 1] - g.rn[p])
        th = g.tn[q] + ft * (g.tn[q + 1] - g.tn[q])
        W = O.dep_weights(g, r, th, int(p), int(q))
        assert abs(W.sum() - 1) < 1e-14 and (W >= 0).all()
        Wf = O.dep_weights(g, r, th, int(p), int(q), flat=True)
        fr = (r - g.rn[p]) / (g.rn[p + 1] - g.rn[p])
        ft = (th - g.tn[q]) / (g.tn[q + 1] - g.tn[q])
        cic = [(1 - fr) * (1 - ft), fr * (1 - ft), (1 - fr) * ft, fr * ft]
        assert np.allclose(Wf, cic, atol=1e-14, rtol=0)


def test_deposit_weights_converge_to_exact_subvolumes():
    """Brute force: the 4x4-point trapezoid sub-volumes agree with adaptive
    quadrature of sqrt(gamma) over the four sub-rectangles."""
    a = 0.99
    g = O.Grid(a, 6, 6, 1.03, 6.0)
    sg = lambda t, r: O.metric(a, r, t)[10]
    for (p, q) in ((0, 0), (2, 3), (5, 2)):
        r = g.rn[p] + 0.3 * (g.rn[p + 1] - g.rn[p])
        th = g.tn[q] + 0.7 * (g.tn[q + 1] - g.tn[q])
        W = O.dep_weights(g, r, th, p, q)
        V = lambda r0, r1, t0, t1: integrate.dblquad(sg, r0, r1, t0, t1, epsabs=1e-13)[0]
        ra, rb, ta, tb = g.rn[p], g.rn[p + 1], g.tn[q], g.tn[q + 1]
        Vs = np.array([V(r, rb, th, tb), V(ra, r, th, tb), V(r, rb, ta, th), V(ra, r, ta, th)])
        assert np.allclose(W, Vs / Vs.sum(), atol=3e-3, rtol=0)


def _lengths(g):
    Lr = np.r_[g.rh[0] - g.rn[0], np.diff(g.rh), g.rn[-1] - g.rh[-1]]
    dth = g.tn[1] - g.tn[0]
    Lt = np.r_[0.5 * dth, np.full(g.nth - 1, dth), 0.5 * dth]
    return Lr, Lt


def test_deposit_discrete_continuity_and_total_charge():
    """The deposited rho and J satisfy the discrete continuity equation to
    round-off at every node, also for moves that cross several cells, and
    the total deposited charge equals the total particle charge."""
    g = O.Grid(0.9, 16, 12, 1.3, 20.0)
    n = 500
    old = np.c_[RNG.uniform(2, 18, n), RNG.uniform(0.1, 3.0, n), RNG.uniform(0, 6, n)]
    new = old + np.c_[RNG.uniform(-1.5, 1.5, n), RNG.uniform(-0.3, 0.3, n), RNG.uniform(-1, 1, n)]
    new[:, 0] = np.clip(new[:, 0], 1.31, 19.9)
    new[:, 1] = np.clip(new[:, 1], g.th0 + 1e-9, np.pi - g.th0 - 1e-9)
    qw = RNG.choice([-1.0, 1.0], n) * RNG.uniform(0.5, 2, n)
    dt = 0.5
    rho0 = O.deposit(g, dt, old, old, qw)[0]
    rho1, Jr, Jt, Jp = O.deposit(g, dt, old, new, qw)
    Lr, Lt = _lengths(g)
    res = (rho1 - rho0) / dt
    # divergence of the densitized current with dual lengths; the edge
    # fluxes outside the grid are zero
    Jr_p = np.zeros((g.nth + 1, g.nr + 2))
    Jr_p[:, 1:-1] = Jr
    Jt_p = np.zeros((g.nth + 2, g.nr + 1))
    Jt_p[1:-1, :] = Jt
    res += (Jr_p[:, 1:] - Jr_p[:, :-1]) / Lr[None, :]
    res += (Jt_p[1:, :] - Jt_p[:-1, :]) / Lt[:, None]
    assert np.abs(res).max() < 1e-12 * np.abs(rho1).max() / dt
    Q = (rho1 * 2 * np.pi * Lr[None, :] * Lt[:, None]).sum()
    assert abs(Q - qw.sum()) < 1e-12 * np.abs(qw).sum()


def _paper_particles(g, n, seed):
    rng = np.random.default_rng(seed)
    z = np.c_[rng.uniform(g.rn[0], g.rn[-1], n), rng.uniform(g.th0, np.pi - g.th0, n),
              rng.uniform(0, 6, n), rng.normal(0, 1, (n, 3))]
    qw = rng.choice([-1.0, 1.0], n) * rng.uniform(0.5, 2, n)
    return z, qw


def test_paper_current_carries_each_particles_charge_flux():
    """Sec. 2.3 (paper mode): summed over its subgrid with the dual volumes,
    every component gives the total q w dx^i/dt with dx^i/dt of eq. p1 (the
    weights are a partition of unity on every subgrid, positions off a half
    subgrid included), and rho gives the total charge."""
    a = 0.9
    g = O.Grid(a, 16, 12, 1.3, 20.0)
    z, qw = _paper_particles(g, 400, 11)
    rho, Jr, Jt, Jp = O.deposit_paper(g, z, qw)
    xdot = np.array([O.rhs(a, 0.0, zk)[:3] for zk in z])
    Lr, Lt = _lengths(g)
    dth = g.tn[1] - g.tn[0]
    tp = 2 * np.pi
    assert np.isclose((rho * tp * Lr[None, :] * Lt[:, None]).sum(), qw.sum(), rtol=1e-13)
    assert np.isclose((Jr * tp * np.diff(g.rn)[None, :] * Lt[:, None]).sum(), qw @ xdot[:, 0],
                      rtol=1e-12)
    assert np.isclose((Jt * tp * Lr[None, :] * dth).sum(), qw @ xdot[:, 1], rtol=1e-12)
    assert np.isclose((Jp * tp * Lr[None, :] * Lt[:, None]).sum(), qw @ xdot[:, 2], rtol=1e-12)


def test_paper_current_of_a_particle_on_a_subgrid_point():
    """A particle sitting on a J^r point (r_{i+1/2}, theta_j) gives all its
    J^r to that point; on a J^theta point (r_i, theta_{j+1/2}) all its
    J^theta; it moves with dx^i/dt = alpha gamma^ij u_j / Gamma - beta^i."""
    a = 0.7
    g = O.Grid(a, 10, 8, 1.8, 12.0)
    i, j = 4, 3
    u = np.array([0.3, -0.5, 1.1])
    for pos, comp in (((g.rh[i], g.tn[j]), 0), ((g.rn[i], g.th[j]), 1)):
        z = np.r_[pos, 0.0, u]
        rho, Jr, Jt, Jp = O.deposit_paper(g, z[None], [1.0])
        m = O.metric(a, pos[0], pos[1])
        gi = np.array([[m[6], 0, m[9]], [0, m[7], 0], [m[9], 0, m[8]]])
        Gam = np.sqrt(1 + u @ gi @ u)
        v = m[0] * gi @ u / Gam - np.array([m[1], 0, 0])
        J = (Jr, Jt)[comp]
        k = np.unravel_index(np.abs(J).argmax(), J.shape)
        assert k == (j, i)
        Lr, Lt = _lengths(g)
        vol = (2 * np.pi * (g.rn[i + 1] - g.rn[i]) * Lt[j] if comp == 0
               else 2 * np.pi * Lr[i] * (g.tn[1] - g.tn[0]))
        assert np.isclose(J[j, i] * vol, v[comp], rtol=1e-13)
        others = np.delete(J.ravel(), np.ravel_multi_index((j, i), J.shape))
        assert np.abs(others).max() <= 1e-15 * abs(J[j, i])


def _stream_field(g, rng):
    """D with zero discrete divergence at every interior node: the densitized
    components are differences of one potential A on the cell centres."""
    A = rng.normal(size=(g.nth + 2, g.nr + 2))  # centres, with a ghost ring
    dth = g.tn[1] - g.tn[0]
    Lr, _ = _lengths(g)
    Dr = g.zeros(0)
    Dt = g.zeros(1)
    # sqrt(g) D^r at (i+1/2, j) = (A[j+1/2] - A[j-1/2]) / dth,
    # sqrt(g) D^th at (i, j+1/2) = -(A[i+1/2] - A[i-1/2]) / Lr_i
    Dr[:, :] = (A[1:, 1:-1] - A[:-1, 1:-1]) / dth
    Dt[:, :] = -(A[1:-1, 1:] - A[1:-1, :-1]) / Lr[None, :]
    return [g.densitize(0, Dr, -1), g.densitize(1, Dt, -1), g.zeros(6)]


def test_cleaning_converged_removes_the_gauss_residual():
    """Sec. 2.4, eq. phi: the cleaned D satisfies Gauss's law at every
    interior node once the Jacobi iteration has converged (the residual is
    measured by the independent om_gauss_residual); more sweeps, smaller
    residual; B is not touched."""
    a = 0.9
    g = O.Grid(a, 10, 8, 1.3, 10.0)
    D, B = O.wald_grid(g, 1.0)
    z, qw = _paper_particles(g, 300, 12)
    rho = O.deposit_paper(g, z, qw)[0]
    G0 = np.abs(O.gauss_residual(g, D, rho)).max()
    res = []
    for iters in (50, 500, 5000):
        Dc, phi = O.div_clean(g, D, rho, iters)
        res.append(np.abs(O.gauss_residual(g, Dc, rho)).max())
        assert np.all(phi[0] == 0) and np.all(phi[-1] == 0)
        assert np.all(phi[:, 0] == 0) and np.all(phi[:, -1] == 0)
    assert res[0] < G0 and res[1] < res[0] and res[2] < res[1]
    assert res[2] < 1e-10 * G0


def test_cleaning_keeps_a_field_that_obeys_gauss():
    """A divergence-free D with rho = 0 (discrete Gauss holds at every
    interior node) comes back unchanged up to round-off."""
    a = 0.5
    g = O.Grid(a, 12, 10, 1.9, 15.0)
    D = _stream_field(g, np.random.default_rng(13))
    rho = g.zeros(6)
    assert np.abs(O.gauss_residual(g, D, rho)).max() < 1e-12 * max(np.abs(x).max() for x in D)
    Dc, phi = O.div_clean(g, D, rho, 500)
    assert np.abs(phi).max() < 1e-10
    scale = max(np.abs(x).max() for x in D)
    for c in range(3):
        assert np.allclose(Dc[c], D[c], rtol=0, atol=1e-10 * scale)


def test_paper_mode_step_breaks_gauss_and_cleaning_restores_it():
    """Sec. 2.4: the paper's own current is not charge-conserving, so Gauss's
    law drifts over paper-mode steps (the conserving deposit keeps it); the
    paper's schedule (every 25 steps, 500 Jacobi sweeps) pulls it back."""
    a = 0.9
    g = O.Grid(a, 12, 10, 0.9 * _rplus(a), 12.0)
    D, B = O.wald_grid(g, 1.0)
    dt = 0.2 * min(np.diff(g.rn).min(), g.rn[0] * (g.tn[1] - g.tn[0]))
    # shell far enough from both radial ends that no particle is removed (a
    # removal takes its charge away without a current)
    p0 = O.init_particles(O.INIT_SHELL_MJ, a, 5, 600, 4.0, 10.0, 0.2, 2.9, 0.3, w=0.05)
    out = {}
    for mode in (O.DEPOSIT_CONSERVING, O.DEPOSIT_PAPER):
        F = O.Fields.uniform_levels(g, D, B)
        p = p0.copy()
        st = p.state()
        alive = np.ones(p.n, np.int32)
        F.rho[:] = O.deposit(g, dt, st[:, :3], st[:, :3], p.qm * p.w)[0]
        if mode == O.DEPOSIT_PAPER:
            rho, Jr, Jt, Jp = O.deposit_paper(g, st, p.qm * p.w, alive)
            F.Jprev[0][:], F.Jprev[1][:], F.Jprev[2][:] = Jr, Jt, Jp
        P = O.push_params(a, dt, field_kind=O.FIELDS_GRID, r_min=_rplus(a), r_max=12.0,
                          th_lo=g.th0, th_hi=np.pi - g.th0, deposit_mode=mode)
        G0 = np.abs(O.gauss_residual(g, F.Dn, F.rho)).max()
        for _ in range(25):
            O.pic_step(P, g, F, p)
        assert np.all(p.flags & O.ALIVE)
        out[mode] = (G0, np.abs(O.gauss_residual(g, F.Dn, F.rho)).max(), F)
    G0, Gc, _ = out[O.DEPOSIT_CONSERVING]
    assert abs(Gc - G0) < 1e-10 * max(G0, 1.0)
    G0p, Gp, F = out[O.DEPOSIT_PAPER]
    assert Gp > 100 * abs(Gc - G0) and Gp > 1e-6
    Dc, _ = O.div_clean(g, F.Dn, F.rho, 500)
    assert np.abs(O.gauss_residual(g, Dc, F.rho)).max() < 0.05 * Gp


# ------------------------------------------------------------------ Maxwell
def _rplus(a):
    return 1 + np.sqrt(1 - a * a)


def test_fdtd_preserves_divB_and_gauss_with_particles():
    """Yee staggering keeps div B constant (Sec. 2.1); with the conserving
    current the Gauss residual of the integer chain stays constant too."""
    a = 0.9
    g = O.Grid(a, 20, 20, 0.9 * _rplus(a), 12.0)
    D, B = O.wald_grid(g, 1.0)
    F = O.Fields.uniform_levels(g, D, B)
    dt = 0.2 * min(np.diff(g.rn).min(), g.rn[0] * (g.tn[1] - g.tn[0]))
    P = O.push_params(a, dt, field_kind=O.FIELDS_GRID, r_min=_rplus(a), r_max=12.0,
                      th_lo=g.th0, th_hi=np.pi - g.th0)
    p = O.init_particles(O.INIT_SHELL_MJ, a, 5, 1000, 2.5, 10.0, 0.2, 2.9, 0.3, w=0.05)
    st = p.state()
    F.rho[:] = O.deposit(g, dt, st[:, :3], st[:, :3], p.qm * p.w)[0]
    G0, dB0 = O.gauss_residual(g, F.Dn, F.rho), O.div_B(g, F.Bn)
    for _ in range(15):
        O.pic_step(P, g, F, p)
    G1, dB1 = O.gauss_residual(g, F.Dn, F.rho), O.div_B(g, F.Bn)
    assert np.abs(dB1 - dB0).max() < 1e-11 * np.abs(dB0).max()
    assert np.abs(G1 - G0).max() < 1e-11 * max(np.abs(G0).max(), np.abs(F.rho).max())


def test_kerr_wald_is_stationary_to_second_order():
    """The Kerr Wald field (App. B.1, E_theta reading) is an exact stationary
    vacuum solution: outside the horizon it stays put to O(h^2)."""
    a, T = 0.9, 2.0
    errs = []
    for N in (24, 48):
        g = O.Grid(a, N, N, 0.9 * _rplus(a), 12.0)
        D, B = O.wald_grid(g, 1.0)
        F = O.Fields.uniform_levels(g, D, B)
        dt0 = 0.3 * min(np.diff(g.rn).min(), g.rn[0] * (g.tn[1] - g.tn[0]))
        steps = int(np.ceil(T / dt0))
        P = O.push_params(a, T / steps)
        for _ in range(steps):
            O.pic_step(P, g, F, None)
        e = []
        for lev, ref, cs in ((F.Bn, B, (3, 4, 5)), (F.Dn, D, (0, 1, 2))):
            for k, c in enumerate(cs):
                nT, nR = g.shape(c)
                R = (g.rh if c in (0, 4, 5) else g.rn)[:nR]
                Th = (g.th if c in (1, 3, 5) else g.tn)[:nT]
                mk = (R[None] > 3) & (R[None] < 7) & (Th[:, None] > 0.4) & (Th[:, None] < np.pi - 0.4)
                e.append(np.abs(lev[k] - ref[k])[mk].max() / np.abs(ref[k][mk]).max())
        errs.append(np.array(e))
    assert (errs[0] < 1e-2).all()
    assert (errs[0] / errs[1] > 3.0).all()


def test_split_monopole_divergence_free():
    g = O.Grid(0.9, 32, 32, 1.29, 20.0)
    D, B = O.split_monopole_grid(g, 1.0, 1e3)
    assert np.abs(O.div_B(g, B)).max() < 1e-12 * np.abs(g.densitize(3, B[0])).max()
    # far from the sheet, B^r -> 4 B0 sin(theta)/sqrt(g) (monopole of Psi)
    j = 3
    sg = np.array([O.metric(0.9, g.rn[i], g.th[j])[10] for i in range(g.nr + 1)])
    assert np.allclose(B[0][j] * sg, -4 * np.sin(g.th[j]), rtol=2e-3)


def test_poynting_vanishes_for_static_schwarzschild_wald():
    """a = 0 Wald vacuum carries no energy flux: P_BZ -> 0 with resolution."""
    vals = []
    for N in (16, 32):
        g = O.Grid(0.0, N, N, 1.8, 12.0)
        D, B = O.wald_grid(g, 1.0)
        vals.append(np.abs(O.poynting(g, D, B)[N // 2]))
    assert vals[1] < vals[0] / 3 or vals[1] < 1e-14


def _fields_for_EH(a, r, th, EH):
    """D^i, B^i (contravariant, plain) whose electric and magnetic fields
    E_i, H_i (covariant) are the given EH = (E_r, E_th, E_ph, H_r, H_th, H_ph)
    at (r, th): the constitutive relations of eq. Ei and its H analogue,
    E_i = alpha gamma_ij D^j + e_ijk beta^j B^k and
    H_i = alpha gamma_ij B^j - e_ijk beta^j D^k with e_ijk = sqrt(gamma)
    eta_ijk (eta_{r th ph} = +1) and beta = (beta^r, 0, 0), inverted as one
    6 x 6 linear system."""
    m = O.metric(a, r, th)
    alpha, betar, sg = m[0], m[1], m[10]
    gam = np.array([[m[2], 0, m[5]], [0, m[3], 0], [m[5], 0, m[4]]])
    X = np.zeros((3, 3))          # (beta x V)_i = X_ik V^k
    X[1, 2] = -sg * betar         # e_{th r ph} beta^r V^ph
    X[2, 1] = sg * betar          # e_{ph r th} beta^r V^th
    M = np.block([[alpha * gam, X], [-X, alpha * gam]])
    sol = np.linalg.solve(M, np.asarray(EH, np.float64))
    return sol[:3], sol[3:]


def _target_EH(r, th):
    """Smooth E_i, H_i with E_th H_ph and E_ph H_th both of order one."""
    s, c = np.sin(th), np.cos(th)
    return (0.0, s * s * (1 + 0.3 * c) * r / (r + 1), 0.6 * s ** 3 / (1 + 0.1 * r),
            0.0, 0.9 * s * s * (1 + 0.5 * c) * np.sqrt(r) / 3, s * s * (0.7 + 0.2 * np.cos(2 * th)) * np.exp(-r / 10))


def test_poynting_luminosity_of_prescribed_fields():
    """Eq. Pbz read as P(r) = (1/2) int (E_th H_ph - E_ph H_th) dtheta (the
    factor 2 pi / 4 pi of the phi integral and the Gaussian Poynting vector):
    D and B are built on every Yee point from prescribed smooth E_i, H_i by
    inverting the constitutive relations, and the oracle's luminosity at
    interior radii converges at second order to the integral of the
    prescribed fields, positive for an outgoing flux.  A wrong factor, sign,
    or an average taken from the wrong Yee points fails this."""
    a = 0.9
    i_frac = 0.5  # the radius r_{N/2}, common to every resolution
    errs, vals = [], []
    for N in (24, 48, 96):
        g = O.Grid(a, N, N, 1.9, 12.0)
        D = [g.zeros(c) for c in range(3)]
        B = [g.zeros(3 + c) for c in range(3)]
        # Yee points of each component (row = theta index, column = r index)
        pts = {0: (g.rh, g.tn), 1: (g.rn, g.th), 2: (g.rn, g.tn),
               3: (g.rn, g.th), 4: (g.rh, g.tn), 5: (g.rh, g.th)}
        for c in range(6):
            rr, tt = pts[c]
            arr = D[c] if c < 3 else B[c - 3]
            for j, t in enumerate(tt):
                for i, r in enumerate(rr):
                    d, b = _fields_for_EH(a, r, t, _target_EH(r, t))
                    arr[j, i] = d[c] if c < 3 else b[c - 3]
        P = O.poynting(g, D, B)
        i = int(i_frac * N)
        r = g.rn[i]

        def flux(t):
            E = _target_EH(r, t)
            return 0.5 * (E[1] * E[5] - E[2] * E[4])
        exact, _ = integrate.quad(flux, g.th0, np.pi - g.th0, epsabs=1e-14, epsrel=1e-13)
        # both terms matter: the second is a sizeable fraction of the first
        t1, _ = integrate.quad(lambda t: 0.5 * _target_EH(r, t)[1] * _target_EH(r, t)[5],
                               g.th0, np.pi - g.th0)
        assert 0.2 < (t1 - exact) / t1 < 0.9
        errs.append(abs(P[i] - exact) / abs(exact))
        vals.append((P[i], exact))
    assert all(p > 0 and e > 0 for p, e in vals)
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


# ------------------------------------------------------ pair injection
def _inj_params(r0=2.0, r1=6.0, mult=3.0, density=5.0, theta=0.5, seed=99):
    return O.InjectParams(r0, r1, mult, density, theta, seed)


def _inj_cells(g, r0, r1):
    return [(p, q) for q in range(g.nth) for p in range(g.nr) if r0 <= g.rh[p] <= r1]


def test_injection_adds_the_goldreich_julian_charge_of_the_volume():
    """Sec. 3.3 into electrovacuum (the a = 0 Wald start in Kerr): one
    co-located e+/e- pair per cell of the injection shell, inside its cell,
    carrying density * n_GJ * V_cell.  For this field Omega . B =
    Omega_H B0 r^2 sin(theta) / sqrt(g), so the total injected weight is
    density Omega_H B0 / 2 times the coordinate integral of r^2 sin(theta)
    over the shell's cells (sqrt(g) cancels); a = 0 injects nothing."""
    a, B0 = 0.9, 1.0
    g = O.Grid(a, 48, 40, 1.3, 12.0)
    D, B = O.wald_grid(g, B0, a_field=0.0)
    I = _inj_params()
    q = O.inject(g, I, 0, B, O.Particles(0), 10 ** 6)
    cells = _inj_cells(g, I.r0, I.r1)
    assert q.n == 2 * len(cells)
    assert np.array_equal(q.qm, np.tile([1.0, -1.0], len(cells)))
    assert np.array_equal(q.r[0::2], q.r[1::2]) and np.array_equal(q.th[0::2], q.th[1::2])
    for k, (p, qq) in enumerate(cells):
        assert g.rn[p] <= q.r[2 * k] <= g.rn[p + 1] and g.tn[qq] <= q.th[2 * k] <= g.tn[qq + 1]
    rp = 1 + np.sqrt(1 - a * a)
    ps = sorted({p for p, _ in cells})
    ra, rb = g.rn[ps[0]], g.rn[ps[-1] + 1]
    shell = (rb ** 3 - ra ** 3) / 3 * 2 * np.cos(g.th0)
    want = I.density * (a / (2 * rp)) * B0 / 2 * shell
    assert np.isclose(q.w.sum(), want, rtol=2e-3)
    g0 = O.Grid(0.0, 48, 40, 2.1, 12.0)
    D0, B0s = O.wald_grid(g0, B0)
    assert O.inject(g0, I, 0, B0s, O.Particles(0), 10 ** 6).n == 0


def test_injection_stops_at_the_multiplicity_and_respects_room():
    """A cell holding density * n_GJ >= mult * n_GJ gets no second pair; with
    mult above density it does.  With room for k pairs the first k eligible
    cells in index order get them."""
    a = 0.9
    g = O.Grid(a, 24, 20, 1.3, 12.0)
    D, B = O.wald_grid(g, 1.0, a_field=0.0)
    q1 = O.inject(g, _inj_params(mult=3.0, density=5.0), 0, B, O.Particles(0), 10 ** 6)
    ncell = len(_inj_cells(g, 2.0, 6.0))
    assert q1.n == 2 * ncell
    assert O.inject(g, _inj_params(mult=3.0, density=5.0), 1, B, q1, 10 ** 6).n == q1.n
    q2 = O.inject(g, _inj_params(mult=10.0, density=5.0), 1, B, q1, 10 ** 6)
    assert q2.n == 2 * q1.n
    # the second injection draws from another seed: new positions
    assert not np.array_equal(q2.r[q1.n:], q1.r)
    q3 = O.inject(g, _inj_params(), 0, B, O.Particles(0), 11)
    assert q3.n == 10 and np.array_equal(q3.r, q1.r[:10])


def test_injected_momenta_are_maxwell_juettner():
    """The FIDO Lorentz factors of the injected particles average
    3 Theta + K_1(1/Theta) / K_2(1/Theta) (relativistic Maxwell-Juettner)."""
    from scipy.special import kv
    a = 0.9
    g = O.Grid(a, 96, 80, 1.3, 12.0)
    D, B = O.wald_grid(g, 1.0, a_field=0.0)
    theta = 0.5
    q = O.inject(g, _inj_params(r0=2.0, r1=10.0, theta=theta), 3, B, O.Particles(0), 10 ** 6)
    assert q.n > 5000
    gam = []
    for z in q.state():
        m = O.metric(a, z[0], z[1])
        gi = np.array([[m[6], 0, m[9]], [0, m[7], 0], [m[9], 0, m[8]]])
        gam.append(np.sqrt(1 + z[3:] @ gi @ z[3:]))
    want = 3 * theta + kv(1, 1 / theta) / kv(2, 1 / theta)
    assert abs(np.mean(gam) / want - 1) < 0.02


# ------------------------------------------------------------ initial data
def test_splitmix64_reference_outputs():
    """The counter-based generator is SplitMix64: from state 0 it yields the
    generator's published first outputs (top 53 bits)."""
    with open(os.path.join(GOLD, "splitmix64_seed0.txt")) as f:
        vals = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    for k, v in enumerate(vals):
        assert int(O.uniform(0, k) * 2 ** 53) == v >> 11


def test_shell_sampling_is_uniform_in_proper_volume():
    """Positions follow sqrt(gamma) dr dtheta (proper volume): the share of
    particles below r_mid matches the volume ratio from quadrature."""
    a, r0, r1, t0, t1 = 0.9, 2.0, 30.0, np.pi / 200, np.pi - np.pi / 200
    n = 40000
    p = O.init_particles(O.INIT_SHELL_ISO, a, 11, n, r0, r1, t0, t1, 1.0)
    sg = lambda t, r: O.metric(a, r, t)[10]
    for rm in (5.0, 12.0):
        frac = integrate.dblquad(sg, r0, rm, t0, t1)[0] / integrate.dblquad(sg, r0, r1, t0, t1)[0]
        got = (p.r < rm).mean()
        assert abs(got - frac) < 4 * np.sqrt(frac * (1 - frac) / n)
    tm = 0.8
    frac = integrate.dblquad(sg, r0, r1, t0, tm)[0] / integrate.dblquad(sg, r0, r1, t0, t1)[0]
    assert abs((p.th < tm).mean() - frac) < 4 * np.sqrt(frac * (1 - frac) / n)
    # |u| uniform on [0, 1] in the FIDO frame: Gamma = sqrt(1 + |u|^2)
    m = np.array([O.metric(a, r, t) for r, t in zip(p.r[:2000], p.th[:2000])])
    u2 = (m[:, 6] * p.ur[:2000] ** 2 + m[:, 7] * p.uth[:2000] ** 2 + m[:, 8] * p.uph[:2000] ** 2
          + 2 * m[:, 9] * p.ur[:2000] * p.uph[:2000])
    assert abs(np.sqrt(u2).mean() - 0.5) < 0.02
    assert set(np.unique(p.qm)) == {-1.0, 1.0}


def test_maxwell_juettner_mean_lorentz_factor():
    """Maxwell-Juettner at Theta: <gamma> = K1(1/Theta)/K2(1/Theta) + 3 Theta."""
    a, theta, n = 0.99, 0.1, 40000
    p = O.init_particles(O.INIT_SHELL_MJ, a, 5, n, 1.2, 18.0, 0.1, 3.0, theta)
    m = np.array([O.metric(a, r, t) for r, t in zip(p.r, p.th)])
    u2 = (m[:, 6] * p.ur ** 2 + m[:, 7] * p.uth ** 2 + m[:, 8] * p.uph ** 2
          + 2 * m[:, 9] * p.ur * p.uph)
    gam = np.sqrt(1 + u2)
    want = special.kn(1, 1 / theta) / special.kn(2, 1 / theta) + 3 * theta
    assert abs(gam.mean() - want) < 4 * gam.std() / np.sqrt(n)
    # pairs share their position and carry opposite charge
    assert np.array_equal(p.r[0::2], p.r[1::2])
    assert (p.qm[0::2] == 1).all() and (p.qm[1::2] == -1).all()


# ---------------------------------------------------------------------- MLP
def test_mlp_gradient_matches_finite_differences():
    """Backward pass of the guess network vs central differences of its
    FP64 loss."""
    theta = RNG.normal(size=O.NPARAM) * 0.2
    X = RNG.normal(size=(7, 14))
    T = RNG.normal(size=(7, 6))
    loss, g = O.mlp_loss_grad(theta, X, T)
    idx = RNG.choice(O.NPARAM, 60, replace=False)
    for i in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (O.mlp_loss_grad(tp, X, T)[0] - O.mlp_loss_grad(tm, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1, abs(fd))
    Y = O.mlp_forward(theta, X)
    assert np.isclose(((Y - T) ** 2).mean(), loss, rtol=1e-14)
