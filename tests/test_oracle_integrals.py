"""Pins of the oracle's flat-cell integrals (the integrals of eqs. (BEM2),
(BEM3) per unit density; the paper leaves its closed forms unpublished).

Each pin is independent of the closed form: numerical quadrature in polar
coordinates, exact subdivision identities, the classical rectangle solid angle,
the disk limit, the far-field monopole limit, finite differences and
rotation/reflection equivariance."""
import numpy as np
import pytest

RNG = np.random.default_rng(1234)


def _polar_quad(a, b, c, r, n=96):
    """IV and IE by Gauss-Legendre quadrature in polar coordinates about the
    foot point of r, with s = |h| sinh(tau) so every integrand is smooth."""
    a, b, c, r = (np.asarray(v, float) for v in (a, b, c, r))
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm)
    h = nrm @ (r - a)
    rho = r - h * nrm
    x, w = np.polynomial.legendre.leggauss(n)
    IV = 0.0
    IE = np.zeros(3)
    for p, q in ((a, b), (b, c), (c, a)):
        dp, dq = p - rho, q - rho
        lp = np.linalg.norm(dp)
        if lp < 1e-300:
            continue
        u = dp / lp
        v = np.cross(nrm, u)
        thq = np.arctan2(dq @ v, dq @ u)
        if abs(np.sin(thq)) < 1e-15 and abs(thq) < 1.0:
            continue
        th = 0.5 * thq * (x + 1)
        wt = 0.5 * thq * w
        d = np.cos(th)[:, None] * u + np.sin(th)[:, None] * v          # ray directions
        # ray rho + s d meets line p + t (q - p): solve in the plane
        e = q - p
        # 2x2 system in (u, v) coordinates
        du, dv = d @ u, d @ v
        eu, ev = e @ u, e @ v
        pu, pv = dp @ u, dp @ v
        det = du * (-ev) - dv * (-eu)
        smax = (pu * (-ev) - pv * (-eu)) / det
        tmax = np.arcsinh(smax / abs(h))
        tau = 0.5 * tmax[:, None] * (x[None, :] + 1)
        wtau = 0.5 * tmax[:, None] * w[None, :]
        s = abs(h) * np.sinh(tau)
        ch = np.cosh(tau)
        R = abs(h) * ch
        jac = abs(h) * ch * s                                         # ds * s
        # IV: s/R ds ; IE: s (r - r')/R^3 ds,  r - r' = h n - s d
        IV += np.sum(wt[:, None] * wtau * jac / R)
        f3 = jac / R ** 3
        IE += np.sum((wt[:, None] * wtau * f3)[..., None] *
                     (h * nrm[None, None, :] - s[..., None] * d[:, None, :]), axis=(0, 1))
    return IV, IE


def _direct_quad(a, b, c, r, n=64):
    """IV and IE by a tensor Gauss-Legendre rule on the collapsed square
    (u, v(1 - u)); accurate when r is well away from the cell."""
    a, b, c, r = (np.asarray(v, float) for v in (a, b, c, r))
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w) * (1 - U)
    P = a + U[..., None] * (b - a) + (V * (1 - U))[..., None] * (c - a)
    J = np.linalg.norm(np.cross(b - a, c - a))
    d = r - P
    R = np.linalg.norm(d, axis=-1)
    return J * np.sum(W / R), J * np.sum((W / R ** 3)[..., None] * d, axis=(0, 1))


def _rand_tri():
    a = RNG.normal(size=3)
    b = a + RNG.normal(size=3)
    c = a + RNG.normal(size=3)
    return a, b, c


@pytest.mark.parametrize("dist", [3e-3, 3e-2, 0.3, 1.0, 3.0, 30.0, 300.0])
def test_closed_form_matches_polar_quadrature(orc, dist):
    for _ in range(4):
        a, b, c = _rand_tri()
        cen = (a + b + c) / 3
        D = max(np.linalg.norm(b - a), np.linalg.norm(c - b), np.linalg.norm(a - c))
        d = RNG.normal(size=3)
        r = cen + dist * D * d / np.linalg.norm(d)
        iv, ie = orc.tri_integrals(a, b, c, r)
        if dist >= 3.0:
            qv, qe = _direct_quad(a, b, c, r)
        else:
            qv, qe = _polar_quad(a, b, c, r, n=128 if dist < 0.1 else 96)
        assert abs(iv - qv) <= 1e-11 * abs(qv)
        assert np.linalg.norm(ie - qe) <= 1e-10 * np.linalg.norm(qe)


def test_near_plane_inside_and_outside(orc):
    # points 1e-6 D above/below the interior and just beside the cell
    a, b, c = np.array([0, 0, 0.]), np.array([1, 0, 0.]), np.array([0.2, 0.9, 0.])
    for r in ([0.3, 0.3, 1e-6], [0.3, 0.3, -1e-6], [1.0, 1.0, 1e-4], [-0.5, 0.2, 3e-5]):
        iv, ie = orc.tri_integrals(a, b, c, r)
        qv, qe = _polar_quad(a, b, c, r, n=160)
        assert abs(iv - qv) <= 1e-10 * abs(qv)
        assert np.linalg.norm(ie - qe) <= 1e-9 * np.linalg.norm(qe)
    # normal component just above/below the interior tends to +-2 pi
    _, up = orc.tri_integrals(a, b, c, [0.3, 0.3, 1e-9])
    _, dn = orc.tri_integrals(a, b, c, [0.3, 0.3, -1e-9])
    assert abs(up[2] - 2 * np.pi) < 1e-7 and abs(dn[2] + 2 * np.pi) < 1e-7
    # principal value exactly in the plane (self term): normal part 0
    _, pv = orc.tri_integrals(a, b, c, [0.3, 0.3, 0.0])
    assert pv[2] == 0.0


def test_midpoint_subdivision_additivity(orc):
    """Exact identity: the integral over a cell equals the sum over its four
    midpoint sub-triangles."""
    for _ in range(20):
        a, b, c = _rand_tri()
        r = RNG.normal(size=3) * 2
        ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
        iv, ie = orc.tri_integrals(a, b, c, r)
        sv, se = 0.0, np.zeros(3)
        for t in ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)):
            v_, e_ = orc.tri_integrals(*t, r)
            sv += v_
            se += e_
        assert abs(iv - sv) <= 1e-13 * abs(iv)
        assert np.linalg.norm(ie - se) <= 1e-12 * np.linalg.norm(ie)


@pytest.mark.parametrize("A,B,h", [(1.0, 2.0, 0.5), (0.3, 0.1, 2.0), (5.0, 5.0, 1e-3)])
def test_rectangle_solid_angle_above_corner(orc, A, B, h):
    """Rectangle [0,A]x[0,B] split into two triangles; at (0,0,h) the solid
    angle is atan(AB / (h sqrt(A^2 + B^2 + h^2))); so is the normal part of IE,
    and the on-axis field of the charged rectangle is sigma Omega / (4 pi eps0)."""
    p = [np.array(v, float) for v in ([0, 0, 0], [A, 0, 0], [A, B, 0], [0, B, 0])]
    r = np.array([0, 0, h])
    tot = np.zeros(3)
    for t in ((p[0], p[1], p[2]), (p[0], p[2], p[3])):
        tot += orc.tri_integrals(*t, r)[1]
    om = np.arctan(A * B / (h * np.sqrt(A * A + B * B + h * h)))
    assert abs(tot[2] - om) <= 1e-13 * om


def test_polygonal_disk_converges_to_disk_field(orc):
    """Regular n-gon fan of radius R: on-axis normal field -> 2 pi (1 - h /
    sqrt(h^2 + R^2)) (the charged disk) with an O(n^-2) error."""
    R, h = 1.0, 0.7
    exact = 2 * np.pi * (1 - h / np.hypot(h, R))
    errs = []
    for n in (64, 128, 256):
        th = 2 * np.pi * np.arange(n + 1) / n
        tot = 0.0
        for k in range(n):
            a = np.zeros(3)
            b = np.array([R * np.cos(th[k]), R * np.sin(th[k]), 0])
            c = np.array([R * np.cos(th[k + 1]), R * np.sin(th[k + 1]), 0])
            tot += orc.tri_integrals(a, b, c, [0, 0, h])[1][2]
        errs.append(abs(tot - exact))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.02)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.02)


def test_far_field_monopole_limit(orc):
    for _ in range(10):
        a, b, c = _rand_tri()
        area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
        cen = (a + b + c) / 3
        d = RNG.normal(size=3)
        d /= np.linalg.norm(d)
        for R in (1e2, 1e3):
            r = cen + R * d
            iv, ie = orc.tri_integrals(a, b, c, r)
            mono = area * (r - cen) / R ** 3
            # the dipole term vanishes about the centroid: error O((D/R)^2)
            assert np.linalg.norm(ie - mono) <= 10 / R ** 2 * np.linalg.norm(mono)
            assert abs(iv - area / R) <= 10 / R ** 2 * area / R


def test_field_is_minus_gradient_of_potential(orc):
    for _ in range(10):
        a, b, c = _rand_tri()
        r = RNG.normal(size=3) * 1.5
        h = 1e-6
        g = np.array([(orc.tri_integrals(a, b, c, r + h * e)[0] - orc.tri_integrals(a, b, c, r - h * e)[0]) / (2 * h)
                      for e in np.eye(3)])
        ie = orc.tri_integrals(a, b, c, r)[1]
        assert np.linalg.norm(ie + g) <= 1e-7 * np.linalg.norm(ie)


def test_jacobian_fd_symmetric_traceless(orc):
    for _ in range(10):
        a, b, c = _rand_tri()
        r = RNG.normal(size=3) * 1.5
        G = orc.tri_grad(a, b, c, r)
        h = 1e-6
        Gfd = np.stack([(orc.tri_integrals(a, b, c, r + h * e)[1] - orc.tri_integrals(a, b, c, r - h * e)[1]) / (2 * h)
                        for e in np.eye(3)], axis=1)
        sc = np.abs(G).max()
        assert np.abs(G - Gfd).max() <= 1e-6 * sc
        assert np.abs(G - G.T).max() <= 1e-12 * sc        # Hessian of -IV
        assert abs(np.trace(G)) <= 1e-12 * sc             # Laplace off the cell


def test_jacobian_near_edge_line(orc):
    """Close to an edge line (stable differencing branch) the Jacobian still
    matches finite differences."""
    a, b, c = np.array([0, 0, 0.]), np.array([1, 0, 0.]), np.array([0.3, 0.8, 0.])
    for r in ([1.5, 1e-4, 1e-4], [-0.7, -2e-5, 3e-5], [0.5, -1e-3, 2e-3]):
        r = np.asarray(r)
        G = orc.tri_grad(a, b, c, r)
        h = 1e-9
        Gfd = np.stack([(orc.tri_integrals(a, b, c, r + h * e)[1] - orc.tri_integrals(a, b, c, r - h * e)[1]) / (2 * h)
                        for e in np.eye(3)], axis=1)
        assert np.abs(G - Gfd).max() <= 1e-4 * np.abs(G).max()


def test_rotation_and_reflection_equivariance(orc):
    for _ in range(10):
        a, b, c = _rand_tri()
        r = RNG.normal(size=3) * 2
        Q, _ = np.linalg.qr(RNG.normal(size=(3, 3)))
        for M in (Q, Q @ np.diag([1, 1, -1])):
            iv, ie = orc.tri_integrals(a, b, c, r)
            iv2, ie2 = orc.tri_integrals(M @ a, M @ b, M @ c, M @ r)
            assert abs(iv2 - iv) <= 1e-13 * abs(iv)
            assert np.linalg.norm(ie2 - M @ ie) <= 1e-12 * np.linalg.norm(ie)
            # reversing the vertex order (flipping the normal) leaves IE unchanged
            ie3 = orc.tri_integrals(a, c, b, r)[1]
            assert np.linalg.norm(ie3 - ie) <= 1e-12 * np.linalg.norm(ie)
