"""GPU parity of bem_solve_charges (eq. (matrixBEM)) against the oracle's
assembly + LAPACK solve, and residual / Dirichlet-row properties at the full
GEM-cell size."""
import numpy as np
import pytest
import torch

from paper_2110_09214_amd import binding as B
from paper_2110_09214_amd import workloads as W
from gpu_helpers import bind, dev, host, rel_l2

pytestmark = pytest.mark.gpu


def _check_against_oracle(ctx, orc, m, tol_sigma):
    sig_ref, A = orc.bem_solve(m)
    bm = bind(ctx, m)
    sig, info = B.bem_solve_charges(ctx, bm, dev(m.rhs), max_refine=3)
    s = host(sig)
    err = rel_l2(s, sig_ref)
    # backward error of the GPU sigma against the oracle's matrix
    r = orc.residual_dense(A, s, m.rhs)
    berr = np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(s).max() + np.abs(m.rhs).max())
    print(m.name, m.n, "sigma rel", err, "info", info, "berr vs oracle A", berr)
    assert info["backward_error"] <= 1e-15
    assert berr <= 1e-13
    assert err <= tol_sigma
    return bm, sig


def test_parallel_plates_solve(ctx, orc):
    m = W.parallel_plate_mesh()
    bm, sig = _check_against_oracle(ctx, orc, m, 1e-10)
    # Dirichlet rows reproduced by the GPU evaluation at every centroid (FP64)
    g = bm.geometry()
    _, V = B.field_eval(ctx, bm, sig, None, None, g["centroid"].contiguous(), 0.0, B.OBEM_FP64, want_v=True)
    assert np.abs(host(V) - m.rhs).max() <= 1e-11 * 500.0
    # the cached factors are reused for a new right-hand side
    rhs2 = m.rhs * 0.5 + 7.0
    sig2, info2 = B.bem_solve_charges(ctx, bm, dev(rhs2))
    sref, _ = orc.bem_solve(m, rhs2, A=orc.bem_matrix(m))
    assert rel_l2(host(sig2), sref) <= 1e-10


def test_dielectric_slab_solve(ctx, orc):
    m = W.plates_with_slab_mesh(n=12)
    bm, sig = _check_against_oracle(ctx, orc, m, 1e-10)
    # the field the GPU evaluates from its own sigma meets the slab closed form
    E = host(B.field_eval(ctx, bm, sig, None, None, dev(np.array([[0, 0, 0.7e-3], [0, 0, 0.2e-3]])), 0.0,
                          B.OBEM_FP64))
    ev = 500.0 / (0.4e-3 / 3 + 0.6e-3)
    assert E[0, 2] == pytest.approx(ev, rel=3e-4)
    assert E[1, 2] == pytest.approx(ev / 3, rel=3e-4)


def test_gem_cell_solve_full_size(ctx, orc):
    """~40k cells: matrix-free oracle residual rows of the GPU sigma and the
    Dirichlet rows reproduced at sampled ed centroids."""
    m = W.gem_cell_mesh()
    bm = bind(ctx, m)
    sig, info = B.bem_solve_charges(ctx, bm, dev(m.rhs), max_refine=3)
    s = host(sig)
    print("gem solve info", info)
    assert info["backward_error"] <= 1e-15
    rng = np.random.default_rng(2)
    rows = np.concatenate([rng.choice(np.nonzero(m.kind == 0)[0], 12, replace=False),
                           rng.choice(np.nonzero(m.kind == 1)[0], 12, replace=False)])
    res, absr = orc.bem_residual_rows(m, s, m.rhs, rows)
    rel = np.abs(res) / (absr * np.abs(s).max() + np.abs(m.rhs[rows]))
    print("gem residual rows", rel.max())
    assert rel.max() <= 1e-13
    ed = rows[:12]
    g = bm.geometry()
    _, V = B.field_eval(ctx, bm, sig, None, None, g["centroid"][torch.as_tensor(ed, device="cuda")].contiguous(),
                        0.0, B.OBEM_FP64, want_v=True)
    assert np.abs(host(V) - m.rhs[ed]).max() <= 1e-9 * 3000.0


def test_singular_mesh_is_reported(ctx):
    m = W.parallel_plate_mesh(n=4)
    m2 = W.Mesh.concat([m, W.Mesh(a=m.a[:1], b=m.b[:1], c=m.c[:1], kind=m.kind[:1], eps1=m.eps1[:1],
                                  eps2=m.eps2[:1], rhs=m.rhs[:1])])
    bm = bind(ctx, m2)
    with pytest.raises(B.ObemError) as e:
        B.bem_solve_charges(ctx, bm, dev(m2.rhs))
    assert e.value.status == -4
    # the context stays usable
    bm2 = bind(ctx, m)
    sig, info = B.bem_solve_charges(ctx, bm2, dev(m.rhs))
    assert info["backward_error"] <= 1e-15


def test_invalid_arguments(ctx):
    m = W.parallel_plate_mesh(n=2)
    bm = bind(ctx, m)
    with pytest.raises(B.ObemError) as e:
        ctx.check(ctx.lib.bem_solve_charges(ctx.h, bm.h, None, None, 1, None))
    assert e.value.status == -1
    host_rhs = np.ascontiguousarray(m.rhs)
    out = torch.empty(m.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.ObemError):
        ctx.check(ctx.lib.bem_solve_charges(ctx.h, bm.h, host_rhs.ctypes.data, out.data_ptr(), 1, None))
    with pytest.raises(B.ObemError):
        B.field_eval(ctx, None, None, None, None, dev(np.zeros((4, 3))), -1.0, B.OBEM_FP64)


def test_adjoint_solve_against_oracle(ctx, orc):
    """g_rhs = A^{-T} g_sigma on the plates-with-slab mesh (ed and dd rows)."""
    m = W.plates_with_slab_mesh(n=12)
    A = orc.bem_matrix(m)
    g = np.random.default_rng(5).normal(size=m.n)
    ref = orc.bem_solve_adjoint(m, g, A=A)
    bm = bind(ctx, m)
    lam, info = B.bem_solve_charges_adjoint(ctx, bm, dev(g))
    print("adjoint solve", rel_l2(host(lam), ref), info)
    assert info["backward_error"] <= 1e-15
    assert rel_l2(host(lam), ref) <= 1e-10


def test_voltage_gradient_through_solve_and_field(ctx):
    """End to end: L = w . E(x; sigma(V)) -- dL/dV of the top plate (sum of
    g_rhs over its cells) equals the exact difference of L (linear in V)."""
    from paper_2110_09214_amd.autograd import field, solve_charges

    m = W.parallel_plate_mesh(n=8, half=1e-3, gap=0.5e-3)
    bm = bind(ctx, m)
    rng = np.random.default_rng(6)
    x = dev(rng.uniform([-5e-4, -5e-4, 1e-4], [5e-4, 5e-4, 4e-4], size=(50, 3)))
    w = dev(rng.normal(size=(50, 3)))
    top = dev((m.a[:, 2] > 1e-4).astype(np.float64))
    v = torch.tensor(-500.0, dtype=torch.float64, device="cuda", requires_grad=True)
    rhs = top * v
    sig = solve_charges(ctx, bm, rhs)
    L = (field(ctx, bm, sig, None, None, x, 0.0, B.OBEM_FP64) * w).sum()
    L.backward()
    with torch.no_grad():
        def Lv(vv):
            s, _ = B.bem_solve_charges(ctx, bm, top * vv)
            return float((B.field_eval(ctx, bm, s, None, None, x, 0.0, B.OBEM_FP64) * w).sum())
        d = (Lv(-400.0) - Lv(-600.0)) / 200.0
    assert float(v.grad) == pytest.approx(d, rel=1e-9)


def test_double_gem_solve_beyond_2_31_elements(ctx, orc):
    """60,752 cells (n^2 = 3.7e9 matrix elements, the 64-bit factor / inverse /
    product path): backward error, sampled residual rows of the oracle's
    matrix, and the transposed (adjoint) solve on the same factors."""
    m = W.double_gem_mesh()
    assert m.n * m.n >= 2 ** 31
    bm = bind(ctx, m)
    sig, info = B.bem_solve_charges(ctx, bm, dev(m.rhs), max_refine=3)
    s = host(sig)
    print("double GEM solve", m.n, info)
    assert info["backward_error"] <= 1e-15
    rng = np.random.default_rng(4)
    rows = np.concatenate([rng.choice(np.nonzero(m.kind == 0)[0], 8, replace=False),
                           rng.choice(np.nonzero(m.kind == 1)[0], 8, replace=False)])
    res, absr = orc.bem_residual_rows(m, s, m.rhs, rows)
    rel = np.abs(res) / (absr * np.abs(s).max() + np.abs(m.rhs[rows]))
    print("double GEM residual rows", rel.max())
    assert rel.max() <= 1e-13
    g = np.random.default_rng(5).normal(size=m.n)
    lam, info_t = B.bem_solve_charges_adjoint(ctx, bm, dev(g))
    print("double GEM adjoint", info_t)
    assert info_t["backward_error"] <= 1e-15
    bm.release()


def test_degenerate_cells_rejected_at_bind(ctx):
    """A zero-area cell or a non-finite vertex is rejected (OBEM_EINVAL) and
    the partially bound mesh is released; the context stays usable."""
    m = W.parallel_plate_mesh(n=4)
    for mutate in ("flat", "nan"):
        a, b, c = m.a.copy(), m.b.copy(), m.c.copy()
        if mutate == "flat":
            c[3] = a[3] + 0.5 * (b[3] - a[3])   # collinear vertices
        else:
            b[5, 1] = np.nan
        bad = W.Mesh(a=a, b=b, c=c, kind=m.kind, eps1=m.eps1, eps2=m.eps2, rhs=m.rhs)
        with pytest.raises(B.ObemError) as e:
            bind(ctx, bad)
        assert e.value.status == -1
    bm = bind(ctx, m)
    sig, info = B.bem_solve_charges(ctx, bm, dev(m.rhs))
    assert info["backward_error"] <= 1e-15
