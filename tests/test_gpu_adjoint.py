"""GPU parity of field_eval_backward (adjoint of L = sum_t w_t . E(x_t))
against the oracle's analytic gradient, its re-summing finite differences
and the GPU forward itself."""
import numpy as np
import pytest
import torch

from paper_2110_09214_amd import binding as B
from paper_2110_09214_amd import workloads as W
from gpu_helpers import bind, dev, host, rel_l2, synthetic_sigma

pytestmark = pytest.mark.gpu
# gradients: relative L2 <= 1e-4 against the FP64 reference in mixed mode (the
# adjoint's contract), FP64 mode limited by the FP64 rounding of 1/d^3 sums
TOL = {B.OBEM_FP64: 1e-11, B.OBEM_MIXED: 1e-4}


@pytest.mark.parametrize("prec", [B.OBEM_FP64, B.OBEM_MIXED])
def test_pairwise_adjoint_shared(ctx, orc, prec):
    rng = np.random.default_rng(1)
    x, q, _ = W.gaussian_clouds(1100, 900, (0, 0, 2e-5), (0, 0, 0), 5e-5, rng)
    w = rng.normal(size=x.shape)
    g_ref, _ = orc.pair_backward(x, x, q, 1e-7, w, tgt_is_src=True)
    _, gt, _ = B.field_eval_backward(ctx, None, None, dev(x), dev(q), dev(x), 1e-7, dev(w), prec, tgt_is_src=True)
    err = rel_l2(host(gt), g_ref)
    print("pair bwd shared", prec, err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [B.OBEM_FP64, B.OBEM_MIXED])
@pytest.mark.parametrize("soft", [0.0, 1e-7])
def test_pairwise_adjoint_separate(ctx, orc, prec, soft):
    rng = np.random.default_rng(2)
    xs = rng.normal(size=(1537, 3)) * 1e-4
    q = rng.choice([-1.0, 1.0], size=1537) * W.E_CHARGE
    xt = rng.normal(size=(701, 3)) * 1e-4
    w = rng.normal(size=xt.shape)
    gt_ref, gs_ref = orc.pair_backward(xt, xs, q, soft, w)
    _, gt, gs = B.field_eval_backward(ctx, None, None, dev(xs), dev(q), dev(xt), soft, dev(w), prec)
    assert rel_l2(host(gt), gt_ref) <= TOL[prec]
    assert rel_l2(host(gs), gs_ref) <= TOL[prec]


@pytest.mark.parametrize("prec", [B.OBEM_FP64, B.OBEM_MIXED])
def test_cell_adjoint_parallel_plates(ctx, orc, prec):
    m = W.parallel_plate_mesh(n=16)
    sig = synthetic_sigma(m, seed=3) * 50
    rng = np.random.default_rng(4)
    x = rng.uniform([-6e-3, -6e-3, -0.3e-3], [6e-3, 6e-3, 1.3e-3], size=(1300, 3))
    x[:100, 2] = 2e-6          # near the lower plate: FP64 closed-form Jacobian
    w = rng.normal(size=x.shape)
    gs_ref, gx_ref = orc.panel_backward(x, m, sig, w)
    bm = bind(ctx, m)
    gs, gx, _ = B.field_eval_backward(ctx, bm, dev(sig), None, None, dev(x), 0.0, dev(w), prec)
    e1, e2 = rel_l2(host(gs), gs_ref), rel_l2(host(gx), gx_ref)
    print("cell bwd", prec, e1, e2)
    assert e1 <= TOL[prec]
    assert e2 <= TOL[prec]


def test_adjoint_matches_gpu_forward_fd(ctx):
    """Self-consistency: FP64 adjoint vs central differences of the FP64
    forward at a small size (L is linear in sigma, exact up to rounding)."""
    m = W.parallel_plate_mesh(n=8, half=1e-3, gap=0.5e-3)
    sig = synthetic_sigma(m, seed=5) * 10
    rng = np.random.default_rng(6)
    x, q, _ = W.gaussian_clouds(60, 60, (0, 0, 2.5e-4), (0, 0, 2.3e-4), 5e-5, rng)
    w = rng.normal(size=x.shape)
    bm = bind(ctx, m)
    X, Q, Wt, S = dev(x), dev(q), dev(w), dev(sig)
    gs, gt, _ = B.field_eval_backward(ctx, bm, S, X, Q, X, 1e-7, Wt, B.OBEM_FP64, tgt_is_src=True)
    gs, gt = host(gs), host(gt)

    def L(xx, ss):
        E = B.field_eval(ctx, bm, ss, xx, Q, xx, 1e-7, B.OBEM_FP64, tgt_is_src=True)
        return float((E * Wt).sum())

    def L_cells(ss):
        E = B.field_eval(ctx, bm, ss, None, None, X, 0.0, B.OBEM_FP64)
        return float((E * Wt).sum())

    for k in (0, 33, 200):
        e = torch.zeros_like(S)
        e[k] = 1.0
        assert L_cells(e) == pytest.approx(gs[k], rel=1e-10)     # L is affine in sigma
    for i, ax in ((0, 0), (77, 2), (119, 1)):
        h = 1e-6 * 5e-5
        xp, xm = X.clone(), X.clone()
        xp[i, ax] += h
        xm[i, ax] -= h
        fd = (L(xp, S) - L(xm, S)) / (2 * h)
        assert fd == pytest.approx(gt[i, ax], rel=1e-4, abs=1e-6 * np.abs(gt).max())


def test_adjoint_1M_charges_49k_cells(ctx, orc):
    """1M particles (targets = sources) and the refined GEM mesh (~50k cells),
    mixed precision: 64 sampled charge-gradient components against the
    oracle's analytic gradient and 64 position components against the
    oracle's re-summing central differences (h = 1e-6 relative)."""
    geo = W.gem_cell_refined_geometry()
    m = W.gem_cell_mesh(geo)
    sig = synthetic_sigma(m, seed=7)
    x, q, sp, w = W.adjoint_workload()
    bm = bind(ctx, m)
    gs, gt, _ = B.field_eval_backward(ctx, bm, dev(sig), dev(x), dev(q), dev(x), 1e-7, dev(w), B.OBEM_MIXED,
                                      tgt_is_src=True)
    gs, gt = host(gs), host(gt)
    rng = np.random.default_rng(3)
    ks = rng.choice(m.n, 64, replace=False)
    sub = W.Mesh(a=m.a[ks], b=m.b[ks], c=m.c[ks], kind=m.kind[ks], eps1=m.eps1[ks], eps2=m.eps2[ks], rhs=m.rhs[ks])
    gs_ref, _ = orc.panel_backward(x, sub, sig[ks], w, want_x=False)
    e_sig = rel_l2(gs[ks], gs_ref)
    comps = [(int(rng.integers(len(x))), int(rng.integers(3))) for _ in range(64)]
    fd = np.array([orc.fd_particle(x, q, w, 1e-7, m, sig, i, ax, 1e-6 * 5e-5) for i, ax in comps])
    got = np.array([gt[i, ax] for i, ax in comps])
    e_x = rel_l2(got, fd)
    print("1M-charge adjoint: sigma", e_sig, "x", e_x)
    assert e_sig <= 1e-4
    assert e_x <= 1e-4


def test_autograd_function(ctx):
    """FieldEval's gradients equal field_eval_backward's (separate sources:
    sigma, target and source positions)."""
    from paper_2110_09214_amd.autograd import field

    m = W.parallel_plate_mesh(n=8, half=1e-3, gap=0.5e-3)
    rng = np.random.default_rng(9)
    sig = dev(synthetic_sigma(m, seed=9)).requires_grad_(True)
    xs = dev(rng.normal(size=(300, 3)) * 5e-5 + np.array([0, 0, 2.5e-4])).requires_grad_(True)
    xt = dev(rng.normal(size=(200, 3)) * 5e-5 + np.array([0, 0, 2.5e-4])).requires_grad_(True)
    q = dev(rng.choice([-1.0, 1.0], size=300) * W.E_CHARGE)
    w = dev(rng.normal(size=(200, 3)))
    bm = bind(ctx, m)
    E = field(ctx, bm, sig, xs, q, xt, 1e-7, B.OBEM_FP64)
    (E * w).sum().backward()
    gs, gt, gsrc = B.field_eval_backward(ctx, bm, sig.detach(), xs.detach(), q, xt.detach(), 1e-7, w, B.OBEM_FP64)
    assert torch.allclose(sig.grad, gs, rtol=1e-12, atol=0)
    assert torch.allclose(xt.grad, gt, rtol=1e-12, atol=0)
    assert torch.allclose(xs.grad, gsrc, rtol=1e-12, atol=0)
