"""Pins of the oracle's static field map (section 3.3.1: field on a uniform
3D grid, interpolated at the particles) and Shockley-Ramo currents (section
3.5, eq. (ramo))."""
import numpy as np
import pytest

from paper_2110_09214_amd import workloads as W


def _linear_map(lo, h, n, A, b):
    nx, ny, nz = n
    gx, gy, gz = (lo[k] + h[k] * np.arange(n[k]) for k in range(3))
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    P = np.stack([X, Y, Z], -1)
    return P @ A.T + b


def test_trilinear_reproduces_linear_fields(orc):
    """Trilinear interpolation is exact for any affine field."""
    rng = np.random.default_rng(1)
    lo, h, n = (-1e-3, 2e-4, -3e-4), (1e-4, 5e-5, 2e-4), (7, 5, 4)
    A, b = rng.normal(size=(3, 3)) * 1e6, rng.normal(size=3) * 1e3
    Emap = _linear_map(lo, h, n, A, b)
    hi = [lo[k] + h[k] * (n[k] - 1) for k in range(3)]
    x = rng.uniform(lo, hi, size=(500, 3))
    got = orc.trilinear(Emap, lo, h, x)
    ref = x @ A.T + b
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_trilinear_nodes_and_clamping(orc):
    rng = np.random.default_rng(2)
    lo, h, n = (0.0, 0.0, 0.0), (1.0, 2.0, 0.5), (4, 3, 5)
    Emap = rng.normal(size=(n[2], n[1], n[0], 3))
    idx = np.array([[0, 0, 0], [3, 2, 4], [1, 2, 3], [2, 0, 1]])
    x = idx * np.array(h)
    got = orc.trilinear(Emap, lo, h, x)
    assert np.array_equal(got, Emap[idx[:, 2], idx[:, 1], idx[:, 0]])
    # outside the box: the value at the nearest boundary point
    out = np.array([[-5.0, 1.0, 1.0], [10.0, 7.0, -1.0]])
    clamped = np.clip(out, 0.0, [3.0, 4.0, 2.0])
    assert np.allclose(orc.trilinear(Emap, lo, h, out), orc.trilinear(Emap, lo, h, clamped), rtol=0, atol=1e-15)


def test_field_map_of_a_capacitor(orc):
    """Between 1 cm plates 1 mm apart (0 V / -500 V) the mapped field near the
    centre is the uniform capacitor field, and the interpolated field between
    nodes agrees with a direct evaluation."""
    m = W.parallel_plate_mesh(n=16)
    sig, _ = orc.bem_solve(m)
    lo, h, n = (-1e-3, -1e-3, 0.1e-3), (5e-4, 5e-4, 1e-4), (5, 5, 9)
    Emap = orc.field_map(m, sig, lo, h, n)
    assert Emap.shape == (9, 5, 5, 3)
    ez = Emap[..., 2]
    assert np.abs(ez / 5e5 - 1.0).max() < 2e-3
    x = np.random.default_rng(3).uniform((-1e-3, -1e-3, 0.1e-3), (1e-3, 1e-3, 0.9e-3), size=(50, 3))
    direct = orc.panel_field(x, m.a, m.b, m.c, sig)
    assert np.abs(orc.trilinear(Emap, lo, h, x) - direct).max() < 2e-3 * 5e5


def _weighting_problem(orc):
    m = W.parallel_plate_mesh(n=16, v_bottom=0.0, v_top=1.0)
    sig_w, _ = orc.bem_solve(m)
    return m, sig_w


def test_ramo_uniform_weighting_field(orc):
    """Parallel plates, read-out = top plate at 1 V: near the centre E_w =
    -z/d, so i = -q v_z / d for every particle; species are summed apart."""
    m, sig_w = _weighting_problem(orc)
    rng = np.random.default_rng(4)
    x = rng.uniform((-5e-4, -5e-4, 2e-4), (5e-4, 5e-4, 8e-4), size=(300, 3))
    v = rng.normal(size=(300, 3)) * 1e5
    sp = rng.integers(0, 3, size=300).astype(np.int8)
    q = np.where(sp == 1, W.E_CHARGE, -W.E_CHARGE)
    Ew = orc.panel_field(x, m.a, m.b, m.c, sig_w)
    cur, terms = orc.induced_current(Ew, v, q, sp)
    ideal = -q * v[:, 2] / 1e-3
    assert np.abs(terms - ideal).max() < 3e-3 * np.abs(ideal).max()
    assert cur.sum() == pytest.approx(terms.sum(), rel=1e-12)
    for s in range(3):
        assert cur[s] == pytest.approx(terms[sp == s].sum(), rel=1e-12)


def test_ramo_charge_integral_equals_weighting_potential_change(orc):
    """Along any path, int i dt = -q (V_w(end) - V_w(start)) because
    E_w = -grad V_w (Shockley's theorem); integrated with Simpson's rule
    over a straight, uniformly travelled path."""
    m, sig_w = _weighting_problem(orc)
    a, b = np.array([-3e-4, 2e-4, 1.5e-4]), np.array([4e-4, -1e-4, 8.5e-4])
    T = 1e-9
    k = 400
    t = np.linspace(0.0, T, k + 1)
    x = a + (b - a) * (t / T)[:, None]
    v = np.broadcast_to((b - a) / T, x.shape)
    q = -W.E_CHARGE
    Ew = orc.panel_field(x, m.a, m.b, m.c, sig_w)
    _, terms = orc.induced_current(Ew, v, np.full(k + 1, q), np.zeros(k + 1, np.int8))
    wts = np.ones(k + 1)
    wts[1:-1:2], wts[2:-1:2] = 4.0, 2.0
    charge = (T / k / 3.0) * (wts * terms).sum()
    _, V = orc.panel_field(np.stack([a, b]), m.a, m.b, m.c, sig_w, want_v=True)
    assert charge == pytest.approx(-q * (V[1] - V[0]), rel=1e-8)
