"""GPU parity of bem_influence (section 3.3.2, eqs. (potpart), (fldpart),
(BEMpotpart), (BEMfldpart)) against the oracle: cell-averaged potential and
field of point charges and the modified left-hand side, on a mesh with ed and
dd cells, and on sampled cells of the GEM cell with a space-charge cloud."""
import numpy as np
import pytest
import torch

from paper_2110_09214_amd import binding as B
from paper_2110_09214_amd import workloads as W
from gpu_helpers import bind, dev, host, rel_l2

pytestmark = pytest.mark.gpu

TOL = {B.OBEM_FP64: 1e-12, B.OBEM_MIXED: 1e-5}


def _slab_charges(m, n, seed):
    """Charges of both signs between the plates (ragged count), plus charges
    a fraction of a cell diameter above sampled cells (closed-form zone)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform([-4.5e-3, -4.5e-3, 0.05e-3], [4.5e-3, 4.5e-3, 0.95e-3], size=(n, 3))
    cen = (m.a + m.b + m.c) / 3
    nrm = np.cross(m.b - m.a, m.c - m.a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    diam = np.max([np.linalg.norm(m.a - m.b, axis=1), np.linalg.norm(m.b - m.c, axis=1),
                   np.linalg.norm(m.c - m.a, axis=1)], axis=0)
    pick = rng.choice(m.n, 64, replace=False)
    xn = cen[pick] + nrm[pick] * (diam[pick] * rng.uniform(0.05, 2.0, size=64))[:, None]
    x = np.concatenate([x, xn])
    q = W.E_CHARGE * rng.choice([-1.0, 1.0], size=x.shape[0]) * rng.uniform(0.5, 2.0, size=x.shape[0])
    return x, q


@pytest.mark.parametrize("prec", [B.OBEM_FP64, B.OBEM_MIXED])
@pytest.mark.parametrize("n_s", [1, 255, 5000])
def test_influence_against_oracle(ctx, orc, prec, n_s):
    m = W.plates_with_slab_mesh(n=12)
    x, q = _slab_charges(m, n_s, seed=11 + n_s)
    ref_rhs, ref_v, ref_e = orc.influence(m, m.rhs, x, q)
    bm = bind(ctx, m)
    rhs_out, vb, eb = B.bem_influence(ctx, bm, dev(m.rhs), dev(x), dev(q), prec, want_bar=True)
    ev, ee = rel_l2(host(vb), ref_v), rel_l2(host(eb), ref_e)
    print("influence", prec, n_s, "Vbar", ev, "Ebar", ee)
    tol = TOL[prec]
    assert max(ev, ee) <= tol
    # rhs_out = rhs - shift, rounded once on each side: the error is the shift's
    # error plus a few ulps of rhs (the shift can be far below one ulp of rhs)
    r = host(rhs_out)
    for rows in (m.kind == 0, m.kind == 1):
        err = np.linalg.norm(r[rows] - ref_rhs[rows])
        bound = tol * np.linalg.norm(m.rhs[rows] - ref_rhs[rows]) + 4 * 2.0 ** -52 * np.linalg.norm(m.rhs[rows])
        print("  rows", rows.sum(), "err", err, "bound", bound)
        assert err <= bound


def test_no_charges_leaves_rhs(ctx):
    m = W.plates_with_slab_mesh(n=6)
    bm = bind(ctx, m)
    rhs = dev(m.rhs)
    out, vb, eb = B.bem_influence(ctx, bm, rhs, None, None, B.OBEM_MIXED, want_bar=True)
    assert torch.equal(out, rhs)
    assert float(vb.abs().max()) == 0.0 and float(eb.abs().max()) == 0.0
    # in place
    r2 = rhs.clone()
    B.bem_influence(ctx, bm, r2, dev(np.array([[0.0, 0.0, 5e-4]])), dev(np.array([1e-15])), B.OBEM_FP64,
                    rhs_out=r2)
    ref = B.bem_influence(ctx, bm, rhs, dev(np.array([[0.0, 0.0, 5e-4]])), dev(np.array([1e-15])), B.OBEM_FP64)
    assert torch.equal(r2, ref)


def test_solve_with_influence_against_oracle(ctx, orc):
    """sigma from the influenced left-hand side (charge-up, section 3.3.2)."""
    m = W.plates_with_slab_mesh(n=12)
    x, q = _slab_charges(m, 3000, seed=21)
    q = q * 1e5  # enough charge to move sigma visibly
    rhs_ref, _, _ = orc.influence(m, m.rhs, x, q)
    sig_ref, _ = orc.bem_solve(m, rhs_ref)
    sig0, _ = orc.bem_solve(m, m.rhs)
    bm = bind(ctx, m)
    rhs = B.bem_influence(ctx, bm, dev(m.rhs), dev(x), dev(q), B.OBEM_FP64)
    sig, info = B.bem_solve_charges(ctx, bm, rhs)
    s = host(sig)
    print("solve with influence", rel_l2(s, sig_ref), "change from charges", rel_l2(sig0, sig_ref))
    assert rel_l2(sig0, sig_ref) > 3e-3
    assert rel_l2(s, sig_ref) <= 1e-10


@pytest.fixture(scope="module")
def gem_case(orc):
    """40,776 cells x 1M charges of the space-charge cloud; 24 sampled cells
    (the nearest to the cloud, and random ones) with their oracle values."""
    m = W.gem_cell_mesh()
    x, q, _ = W.space_charge_cloud(500_000, 500_000)
    cen = (m.a + m.b + m.c) / 3
    d = np.linalg.norm(cen - np.array([0, 0, 220e-6]), axis=1)
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([np.argsort(d)[:12], rng.choice(m.n, 12, replace=False)]))
    sub = W.Mesh(a=m.a[rows], b=m.b[rows], c=m.c[rows], kind=m.kind[rows], eps1=m.eps1[rows], eps2=m.eps2[rows],
                 rhs=m.rhs[rows])
    return m, x, q, rows, sub, orc.influence(sub, sub.rhs, x, q)


@pytest.mark.parametrize("prec", [B.OBEM_FP64, B.OBEM_MIXED])
def test_gem_cell_influence_sampled_rows(ctx, gem_case, prec):
    m, x, q, rows, sub, (ref_rhs, ref_v, ref_e) = gem_case
    bm = bind(ctx, m)
    rhs_out, vb, eb = B.bem_influence(ctx, bm, dev(m.rhs), dev(x), dev(q), prec, want_bar=True)
    v, e, r = host(vb)[rows], host(eb)[rows], host(rhs_out)[rows]
    ev = np.abs(v - ref_v).max() / np.abs(ref_v).max()
    ee = np.linalg.norm(e - ref_e, axis=1).max() / np.linalg.norm(ref_e, axis=1).max()
    er = np.abs((sub.rhs - r) - (sub.rhs - ref_rhs)).max() / np.abs(sub.rhs - ref_rhs).max()
    print("gem influence", prec, "Vbar", ev, "Ebar", ee, "rhs shift", er)
    assert max(ev, ee, er) <= TOL[prec]
    assert np.isfinite(host(rhs_out)).all()


def test_influence_invalid_arguments(ctx):
    m = W.plates_with_slab_mesh(n=4)
    bm = bind(ctx, m)
    rhs = dev(m.rhs)
    x0, x1, x2 = (dev(np.zeros(3)) for _ in range(3))
    q = dev(np.ones(3))
    with pytest.raises(B.ObemError):
        ctx.check(ctx.lib.bem_influence(ctx.h, bm.h, 3, None, None, None, None, rhs.data_ptr(), rhs.data_ptr(),
                                        B.OBEM_FP64, None, None, None, None))
    with pytest.raises(B.ObemError):
        ctx.check(ctx.lib.bem_influence(ctx.h, bm.h, 3, x0.data_ptr(), x1.data_ptr(), x2.data_ptr(), q.data_ptr(),
                                        rhs.data_ptr(), rhs.data_ptr(), 7, None, None, None, None))
    eb = torch.empty(m.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.ObemError):
        ctx.check(ctx.lib.bem_influence(ctx.h, bm.h, 0, None, None, None, None, rhs.data_ptr(), rhs.data_ptr(),
                                        B.OBEM_FP64, None, eb.data_ptr(), None, None))
    # the context stays usable
    out = B.bem_influence(ctx, bm, rhs, None, None)
    assert torch.equal(out, rhs)
