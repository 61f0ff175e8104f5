"""Pins of the oracle's direct pairwise field (eq. (nbody) with Plummer
softening): the point-charge formula, Newton's third law, Gauss's law through
closed boxes, the divergence of the softened field, and the nearest
opposite-species search used by recombination."""
import numpy as np
import pytest

RNG = np.random.default_rng(77)


def test_point_charge(orc):
    k = orc.constants()
    q = np.array([3.2e-19])
    xs = np.array([[0.1, -0.2, 0.3]])
    for soft in (0.0, 1e-7):
        r = np.array([[0.1 + 1e-6, -0.2 - 2e-6, 0.3 + 0.5e-6]])
        E, V = orc.pair_field(r, xs, q, soft, want_v=True)
        d = r[0] - xs[0]
        S2 = d @ d + soft ** 2
        assert np.allclose(E[0], k["k_e"] * q[0] * d / S2 ** 1.5, rtol=1e-15, atol=0)
        assert V[0] == pytest.approx(k["k_e"] * q[0] / np.sqrt(S2), rel=1e-15)


def test_newton_third_law(orc):
    n = 300
    x = RNG.normal(size=(n, 3)) * 1e-5
    q = RNG.choice([-1.0, 1.0], size=n) * 1.602176634e-19
    for soft in (0.0, 1e-7):
        E = orc.pair_field(x, x, q, soft, tgt_is_src=True)
        F = q[:, None] * E
        scale = np.abs(F).sum(axis=0)
        assert np.all(np.abs(F.sum(axis=0)) <= 1e-13 * scale)


def _box_flux(orc, xs, q, soft, lo, hi, n=48):
    xg, wg = np.polynomial.legendre.leggauss(n)
    flux = 0.0
    for ax in range(3):
        o1, o2 = [k for k in range(3) if k != ax]
        for side, sgn in ((lo[ax], -1.0), (hi[ax], 1.0)):
            u = lo[o1] + (hi[o1] - lo[o1]) * 0.5 * (xg + 1)
            v = lo[o2] + (hi[o2] - lo[o2]) * 0.5 * (xg + 1)
            U, Vv = np.meshgrid(u, v, indexing="ij")
            P = np.zeros(U.shape + (3,))
            P[..., ax] = side
            P[..., o1] = U
            P[..., o2] = Vv
            E = orc.pair_field(P.reshape(-1, 3), xs, q, soft).reshape(U.shape + (3,))
            W = np.outer(wg, wg) * 0.25 * (hi[o1] - lo[o1]) * (hi[o2] - lo[o2])
            flux += sgn * np.sum(W * E[..., ax])
    return flux


def test_gauss_law_flux_through_boxes(orc):
    """Flux of E through a closed box = Q_enclosed / eps0 (charges well inside
    or well outside, many softening lengths from the faces)."""
    k = orc.constants()
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.2, 0.9])
    inside = RNG.uniform(-0.4, 0.4, size=(6, 3))
    outside = RNG.uniform(-0.5, 0.5, size=(5, 3)) + np.array([3.0, 0.0, 0.0])
    xs = np.concatenate([inside, outside])
    q = RNG.normal(size=11)
    flux = _box_flux(orc, xs, q, 1e-6, lo, hi)
    assert flux == pytest.approx(q[:6].sum() / k["eps0"], rel=1e-9)


def test_divergence_of_softened_field(orc):
    """div E = 3 k_e sum_j q_j s^2 / (r^2 + s^2)^{5/2} (finite differences)."""
    k = orc.constants()
    s = 0.3
    xs = RNG.normal(size=(4, 3))
    q = RNG.normal(size=4)
    for _ in range(5):
        r = RNG.normal(size=3)
        h = 1e-5
        div = 0.0
        for ax in range(3):
            e = np.zeros(3)
            e[ax] = h
            Ep = orc.pair_field(r + e, xs, q, s)[0]
            Em = orc.pair_field(r - e, xs, q, s)[0]
            div += (Ep[ax] - Em[ax]) / (2 * h)
        d2 = np.sum((r - xs) ** 2, axis=1)
        exact = 3 * k["k_e"] * np.sum(q * s * s / (d2 + s * s) ** 2.5)
        assert div == pytest.approx(exact, rel=1e-6, abs=1e-9 * k["k_e"])


def test_nearest_opposite_species(orc):
    # electrons (0) find cations (1) and vice versa; anions (2) are ignored;
    # equal distances resolve to the lower source index
    x = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 0.5, 0], [0, 0.4, 0.0], [5, 5, 5]], float)
    sp = np.array([0, 1, 1, 2, 0, 1], np.int8)
    q = np.where(sp == 1, 1.0, -1.0)
    E, nn, d2 = orc.pair_field(x, x, q, 0.0, tgt_is_src=True, sp_t=sp, sp_s=sp)
    assert nn[0] == 1 and d2[0] == 1.0           # tie between 1 and 2 -> lower index
    assert nn[1] == 0 and d2[1] == 1.0           # cation 1: electrons 0 (d=1), 4 (d^2=1.16)
    assert nn[2] == 0
    assert nn[3] == -1 and np.isinf(d2[3])       # anion: no partner
    assert nn[4] == 1 and d2[4] == pytest.approx(1.16)
    assert nn[5] == 4
