"""Pins of the oracle's adjoint of the field evaluation, L = sum_i w_i . E(x_i):
central finite differences in sigma (exact up to rounding: L is linear in
sigma) and in the particle positions, for panels and for point charges, with
separate and shared target/source sets."""
import numpy as np
import pytest

from paper_2110_09214_amd import workloads as W

RNG = np.random.default_rng(31)


def _loss(orc, x, mesh, sig, xs, q, soft, w, tgt_is_src):
    E = np.zeros_like(x)
    if mesh is not None:
        E += orc.panel_field(x, mesh.a, mesh.b, mesh.c, sig)
    if xs is not None:
        E += orc.pair_field(x, x if tgt_is_src else xs, q, soft, tgt_is_src=tgt_is_src)
    return float(np.sum(w * E))


@pytest.fixture(scope="module")
def small():
    m = W.parallel_plate_mesh(n=4, half=1e-3, gap=0.5e-3)
    sig = RNG.normal(size=m.n) * 1e-6
    x = RNG.uniform([-1e-3, -1e-3, 0.05e-3], [1e-3, 1e-3, 0.45e-3], size=(12, 3))
    w = RNG.normal(size=(12, 3))
    return m, sig, x, w


def test_panel_sigma_gradient_is_exact_linear(orc, small):
    m, sig, x, w = small
    gs, _ = orc.panel_backward(x, m, sig, w, want_x=False)
    for k in (0, 5, 17, m.n - 1):
        e = np.zeros(m.n)
        e[k] = 1.0
        d = _loss(orc, x, m, e, None, None, 0, w, False)   # L linear: dL/dsigma_k = L(e_k)
        assert gs[k] == pytest.approx(d, rel=1e-12)
        h = 1e-3 * np.abs(sig).max()
        fd = (_loss(orc, x, m, sig + h * e, None, None, 0, w, False) -
              _loss(orc, x, m, sig - h * e, None, None, 0, w, False)) / (2 * h)
        assert gs[k] == pytest.approx(fd, rel=1e-7)


def test_panel_position_gradient_fd(orc, small):
    m, sig, x, w = small
    _, gx = orc.panel_backward(x, m, sig, w, want_sigma=False)
    for i in (0, 3, 11):
        for ax in range(3):
            h = 1e-6 * 1e-3
            xp, xm = x.copy(), x.copy()
            xp[i, ax] += h
            xm[i, ax] -= h
            fd = (_loss(orc, xp, m, sig, None, None, 0, w, False) - _loss(orc, xm, m, sig, None, None, 0, w, False)) / (2 * h)
            assert gx[i, ax] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(gx).max())


@pytest.mark.parametrize("tgt_is_src", [False, True])
def test_pair_position_gradient_fd(orc, tgt_is_src):
    n = 40
    xs = RNG.normal(size=(n, 3)) * 1e-5
    q = RNG.choice([-1.0, 1.0], size=n) * 1.6e-19
    xt = xs if tgt_is_src else RNG.normal(size=(25, 3)) * 1e-5
    w = RNG.normal(size=xt.shape)
    soft = 1e-7
    gt, gs = orc.pair_backward(xt, xs, q, soft, w, tgt_is_src=tgt_is_src)

    def L(xt_, xs_):
        return float(np.sum(w * orc.pair_field(xt_, xs_ if not tgt_is_src else xt_, q, soft, tgt_is_src=tgt_is_src)))

    h = 1e-6 * 1e-5
    for i in (0, 7, 19):
        for ax in range(3):
            xp, xm = xt.copy(), xt.copy()
            xp[i, ax] += h
            xm[i, ax] -= h
            fd = (L(xp, xs) - L(xm, xs)) / (2 * h)
            assert gt[i, ax] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(gt).max())
    if not tgt_is_src:
        for j in (1, 30):
            for ax in range(3):
                sp, sm = xs.copy(), xs.copy()
                sp[j, ax] += h
                sm[j, ax] -= h
                fd = (L(xt, sp) - L(xt, sm)) / (2 * h)
                assert gs[j, ax] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(gs).max())


def test_fd_particle_helper_matches_analytic_adjoint(orc, small):
    """The re-summing finite difference used at full size agrees with the
    analytic adjoint (cells + pairwise, targets = sources)."""
    m, sig, _, _ = small
    rng = np.random.default_rng(8)
    n = 30
    x = rng.uniform([-1e-3, -1e-3, 0.05e-3], [1e-3, 1e-3, 0.45e-3], size=(n, 3))
    q = rng.choice([-1.0, 1.0], size=n) * 1.6e-19
    w = rng.normal(size=(n, 3))
    soft = 1e-7
    gp, _ = orc.pair_backward(x, x, q, soft, w, tgt_is_src=True)
    _, gc = orc.panel_backward(x, m, sig, w, want_sigma=False)
    g = gp + gc
    for i in (0, 13, 29):
        for ax in range(3):
            fd = orc.fd_particle(x, q, w, soft, m, sig, i, ax, 1e-10)
            assert fd == pytest.approx(g[i, ax], rel=1e-6, abs=1e-10 * np.abs(g).max())
