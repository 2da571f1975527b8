"""Single-cell pins of the FP64 oracle: lattice, equilibria and the operator K_lambda.

Each expected value comes from the paper's definitions or from mathematics
independent of the oracle's code: closed-form moments derived by hand from
eq. phi / feq / f_star / geq, textbook lattice weights (tests/golden), the
idempotency and orthogonality of eq. K stated after eq. def_ustar, local
conservation of J_loc and the lambda -> 0 limit eq. lim_projection.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
RNG = np.random.default_rng(12345)


def _moments(D, pops):
    c, _ = O.lattice(D)
    c = c[:, :D].astype(np.float64)
    m0 = pops.sum()
    m1 = c.T @ pops
    m2 = np.einsum("ia,ib,i->ab", c, c, pops)
    return m0, m1, m2


def test_weights_match_golden():
    table = {}
    with open(os.path.join(HERE, "golden", "lattice_weights.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lat, c2, w = line.split()
            table[(lat, int(c2))] = float(Fraction(w))
    for D, name in ((2, "D2Q9"), (3, "D3Q27")):
        c, w = O.lattice(D)
        assert len(w) == (9 if D == 2 else 27)
        for i in range(len(w)):
            assert w[i] == pytest.approx(table[(name, int((c[i] ** 2).sum()))], rel=1e-15)
            # opposite direction is Q-1-i
            assert np.array_equal(c[len(w) - 1 - i], -c[i])
        # rest equilibrium at P0/rho = 1/3 equals the weights
        feq = O.feq_cell(D, 1.0, [0.0] * D, 1.0 / 3.0)
        assert np.allclose(feq, w, rtol=1e-15, atol=0)


def test_psi_moments():
    """sum_c Psi = 1, sum_c c Psi = xi, sum_c c^2 Psi = zeta (eq. phi)."""
    for _ in range(50):
        xi, zeta = RNG.uniform(-1, 1), RNG.uniform(0, 1)
        ps = {c: O.psi(c, xi, zeta) for c in (-1, 0, 1)}
        assert sum(ps.values()) == pytest.approx(1.0, abs=1e-15)
        assert sum(c * p for c, p in ps.items()) == pytest.approx(xi, abs=1e-15)
        assert sum(c * c * p for c, p in ps.items()) == pytest.approx(zeta, abs=1e-15)


@pytest.mark.parametrize("D", [2, 3])
def test_feq_and_fstar_moments(D):
    """rho, rho u and rho u u + P0 I for f^eq (eq. feq); diagonal
    rho zeta* for f* (eq. f_star) with the off-diagonal rho u*_a u*_b."""
    for _ in range(30):
        rho = RNG.uniform(0.05, 2.5)
        u = RNG.uniform(-0.2, 0.2, D)
        theta = RNG.uniform(0.01, 0.3)
        f = O.feq_cell(D, rho, u, theta)
        m0, m1, m2 = _moments(D, f)
        assert m0 == pytest.approx(rho, rel=1e-14)
        assert np.allclose(m1, rho * u, rtol=1e-13, atol=1e-15)
        P = rho * np.outer(u, u) + rho * theta * np.eye(D)
        assert np.allclose(m2, P, rtol=1e-13, atol=1e-15)
        # lattice third moment c^3 = c: sum c_a^3 f = rho u_a
        c, _ = O.lattice(D)
        assert np.allclose((c[:, :D] ** 3).T @ f, rho * u, rtol=1e-13, atol=1e-15)
        # shifted equilibrium with a diagonal correction
        us = u + RNG.uniform(-0.05, 0.05, D)
        Phi = RNG.uniform(-0.01, 0.01, D)
        zeta = theta + us * us + Phi / rho
        fs = O.product_cell(D, rho, us, zeta)
        m0, m1, m2 = _moments(D, fs)
        assert m0 == pytest.approx(rho, rel=1e-14)
        assert np.allclose(m1, rho * us, rtol=1e-13, atol=1e-15)
        expect = rho * np.outer(us, us)
        expect[np.diag_indices(D)] = rho * zeta
        assert np.allclose(m2, expect, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("D", [2, 3])
def test_geq_moments(D):
    """The moments of eq. geq.  From O_a A = theta dA/du_a + u_a A and
    E = (3/2)RT + |u|^2/2, worked by hand:
      sum g = rho E,
      sum c_a g = rho O_a E = u_a (rho E + P0),
      sum c_a c_b g = rho O_a O_b E = rho u_a u_b (E + 2 theta)         (a != b),
      sum c_a^2 g = rho O_a^2 E = rho (theta^2 + theta E + 2 theta u_a^2 + u_a^2 E)."""
    for _ in range(30):
        rho = RNG.uniform(0.05, 2.5)
        u = RNG.uniform(-0.2, 0.2, D)
        RT = RNG.uniform(0.01, 0.05)
        theta = RT / (1.0 - RNG.uniform(0.0, 0.7))
        g = O.geq_cell(D, rho, u, RT, theta)
        E = 1.5 * RT + 0.5 * (u * u).sum()
        m0, m1, m2 = _moments(D, g)
        assert m0 == pytest.approx(rho * E, rel=1e-13)
        assert np.allclose(m1, u * (rho * E + rho * theta), rtol=1e-12, atol=1e-16)
        for a in range(D):
            for b in range(D):
                if a == b:
                    ex = rho * (theta ** 2 + theta * E + 2 * theta * u[a] ** 2 + u[a] ** 2 * E)
                else:
                    ex = rho * u[a] * u[b] * (E + 2 * theta)
                assert m2[a, b] == pytest.approx(ex, rel=1e-12, abs=1e-16)


def test_d3q27_sums_to_d2q9():
    """At cell level, summing D3Q27 over c_z with u_z = 0 gives D2Q9."""
    c3, _ = O.lattice(3)
    c2, _ = O.lattice(2)
    for _ in range(20):
        rho = RNG.uniform(0.05, 2.5)
        u = list(RNG.uniform(-0.2, 0.2, 2))
        RT = RNG.uniform(0.01, 0.05)
        theta = RT * RNG.uniform(1.0, 3.0)
        f3 = O.feq_cell(3, rho, u + [0.0], theta)
        g3 = O.geq_cell(3, rho, u + [0.0], RT, theta)
        f2 = O.feq_cell(2, rho, u, theta)
        g2 = O.geq_cell(2, rho, u, RT, theta)
        for i in range(9):
            sel = np.all(c3[:, :2] == c2[i, :2], axis=1)
            assert f3[sel].sum() == pytest.approx(f2[i], rel=1e-13, abs=1e-17)
            assert g3[sel].sum() == pytest.approx(g2[i], rel=1e-13, abs=1e-17)


def _random_state(D):
    rho = RNG.uniform(0.3, 2.0)
    u = RNG.uniform(-0.1, 0.1, D)
    RT = RNG.uniform(0.1, 0.3)
    Q = 9 if D == 2 else 27
    J = RNG.uniform(-1, 1, Q) * 0.004
    J -= J.mean()  # local mass conservation: sum J = 0
    return rho, u, RT, J


def test_kop_idempotent_and_orthogonal():
    """K(K(J)) = K(J) and K(J - K(J)) = 0 (text after eq. def_ustar)."""
    worst = 0.0
    for _ in range(300):
        rho, u, RT, J = _random_state(3)
        lam = RNG.uniform(0.1, 1.5)
        K = O.kop(3, rho, u, RT, J, lam)
        KK = O.kop(3, rho, u, RT, K, lam)
        Korth = O.kop(3, rho, u, RT, J - K, lam)
        scale = np.abs(K).max()
        worst = max(worst, np.abs(KK - K).max() / scale, np.abs(Korth).max() / scale)
    assert worst < 1e-11


def test_kop_local_part_conserves():
    """J_loc = J - K(J) conserves mass, momentum and kinetic energy."""
    c, _ = O.lattice(3)
    c = c.astype(np.float64)
    for _ in range(200):
        rho, u, RT, J = _random_state(3)
        lam = RNG.uniform(0.1, 1.5)
        Jl = J - O.kop(3, rho, u, RT, J, lam)
        # K is a difference of two equilibria of size rho divided by lambda:
        # its rounding floor is about 1e-16 rho/lambda per entry.
        tol = 1e-13 * rho / lam
        assert abs(Jl.sum()) < tol
        assert np.abs(c.T @ Jl).max() < tol
        assert abs(((c * c).sum(1) * Jl).sum()) < 10 * tol


def test_kop_linear_limit():
    """K_lambda -> (1/rho) df^eq/du . F + (2/(3 rho)) df^eq/dRT Qt as
    lambda -> 0 (eq. lim_projection), with an O(lambda) remainder."""
    c, _ = O.lattice(3)
    c = c.astype(np.float64)
    rho, u, RT, J = _random_state(3)
    F = c.T @ J
    Qt = 0.5 * (((c - u) ** 2).sum(1) * J).sum()

    def feq(uu, rt):
        return O.feq_cell(3, rho, uu, rt)  # kinetic Maxwellian, P0 = rho RT

    h = 1e-5
    lin = np.zeros(27)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        lin += (feq(u + e, RT) - feq(u - e, RT)) / (2 * h) * F[a] / rho
    lin += (feq(u, RT + h) - feq(u, RT - h)) / (2 * h) * 2.0 * Qt / (3.0 * rho)
    errs = []
    for lam in (1e-1, 1e-2, 1e-3):
        K = O.kop(3, rho, u, RT, J, lam)
        errs.append(np.abs(K - lin).max() / np.abs(lin).max())
    assert errs[1] < errs[0] / 7 and errs[2] < errs[1] / 7
    assert 8 < errs[0] / errs[1] < 12


def test_stencils_exact_and_second_order():
    """The isotropic gradient is exact on quadratics, the Laplacian on
    cubics (checked away from the periodic seam), and on sin(kx) they give
    sin(k) cos(kx) and 2(cos k - 1) sin(kx) respectively."""
    for D, shape in ((2, (1, 24, 20)), (3, (14, 12, 10))):
        nz, ny, nx = shape
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        X = [x.astype(float), y.astype(float), z.astype(float)]
        for _ in range(5):
            co = RNG.uniform(-1, 1, 10)
            phi = co[0] + co[1] * X[0] + co[2] * X[1] + co[3] * X[0] * X[1] + co[4] * X[0] ** 2 + co[5] * X[1] ** 2
            dphi = [co[1] + co[3] * X[1] + 2 * co[4] * X[0], co[2] + co[3] * X[0] + 2 * co[5] * X[1]]
            lphi = 2 * co[4] + 2 * co[5] + 0 * X[0]
            if D == 3:
                phi = phi + co[6] * X[2] + co[7] * X[2] ** 2 + co[8] * X[0] * X[2]
                dphi[0] = dphi[0] + co[8] * X[2]
                dphi[1] = dphi[1] + 0 * X[2]
                dphi.append(co[6] + 2 * co[7] * X[2] + co[8] * X[0])
                lphi = lphi + 2 * co[7]
            grad, lap = O.stencils(D, shape, phi)
            inner = (slice(1, -1) if D == 3 else slice(None), slice(1, -1), slice(1, -1))
            for a in range(D):
                assert np.allclose(grad[a][inner], dphi[a][inner], atol=1e-11)
            assert np.allclose(lap[inner], lphi[inner], atol=1e-11)
            # Laplacian exact on a cubic too
            cub = X[0] ** 3 - 2 * X[1] ** 3
            _, lap3 = O.stencils(D, shape, cub)
            assert np.allclose(lap3[inner], (6 * X[0] - 12 * X[1])[inner], atol=1e-9)
        # sines along each axis (periodic)
        for a in range(D):
            n = shape[2 - a]
            k = 2 * np.pi * 3 / n
            phi = np.sin(k * X[a])
            grad, lap = O.stencils(D, shape, phi)
            assert np.allclose(grad[a], np.sin(k) * np.cos(k * X[a]), atol=1e-13)
            for b in range(D):
                if b != a:
                    assert np.allclose(grad[b], 0, atol=1e-13)
            assert np.allclose(lap, 2 * (np.cos(k) - 1) * phi, atol=1e-13)
