"""field_eval_noalloc (the allocation-free variant of field_eval, for callers
that cannot allocate) against field_eval through the C ABI: two calls in a
row on one context, the second with a smaller input, with cells and charges
in both precisions (the mixed one large enough for the pair-once
evaluation), the largest call (OBEM_NOALLOC_MAX_POINTS charges in a 40,776-cell
mesh), then the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2110_09214_amd import binding as B
from paper_2110_09214_amd import workloads as W
from gpu_helpers import bind, dev, host, rel_l2, synthetic_sigma

pytestmark = pytest.mark.gpu

TOL = {B.OBEM_FP64: 1e-12, B.OBEM_MIXED: 1e-5}


def _noalloc(ctx, bm, sig, xs, q, xt, soft, prec, tgt_is_src):
    lib = ctx.lib
    n_t = xt.shape[0]
    n_s = 0 if xs is None else xs.shape[0]
    E = [torch.empty(n_t, dtype=torch.float64, device="cuda") for _ in range(3)]
    cols_t = [xt[:, k].contiguous() for k in range(3)]
    cols_s = [xs[:, k].contiguous() for k in range(3)] if n_s else [None] * 3
    p = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    flags = B.OBEM_TGT_IS_SRC if tgt_is_src else 0
    st = lib.field_eval_noalloc(ctx.h, bm.h if bm is not None else None, p(sig), C.c_int64(n_s), *map(p, cols_s),
                                p(q), C.c_int64(n_t), *map(p, cols_t), C.c_double(soft), C.c_int(prec),
                                C.c_uint(flags), *map(p, E), None)
    return st, torch.stack(E, 1)


@pytest.mark.parametrize("prec", [B.OBEM_MIXED, B.OBEM_FP64])
def test_noalloc_matches_field_eval_twice(ctx, prec):
    m = W.parallel_plate_mesh(n=16)
    bm = bind(ctx, m)
    sig = dev(synthetic_sigma(m))
    rng = np.random.default_rng(21)
    for n in (9000, 3001):                       # second call smaller
        x = rng.normal(size=(n, 3)) * 2e-4 + np.array([0, 0, 5e-4])
        q = rng.choice([-1.0, 1.0], size=n) * W.E_CHARGE
        X, Q = dev(x), dev(q)
        st, E0 = _noalloc(ctx, bm, sig, X, Q, X, 1e-7, prec, True)
        assert st == 0, ctx.lib.obem_last_error(ctx.h)
        E1 = B.field_eval(ctx, bm, sig, X, Q, X, 1e-7, prec, tgt_is_src=True)
        err = rel_l2(host(E0), host(E1))
        print(f"noalloc prec {prec} n {n}: rel L2 vs field_eval {err:.3g}")
        assert err <= TOL[prec]
    # separate targets, no cells
    xt = dev(rng.normal(size=(700, 3)) * 2e-4)
    st, E0 = _noalloc(ctx, None, None, X, Q, xt, 1e-7, prec, False)
    assert st == 0
    E1 = B.field_eval(ctx, None, None, X, Q, xt, 1e-7, prec)
    assert rel_l2(host(E0), host(E1)) <= TOL[prec]


@pytest.mark.parametrize("prec", [B.OBEM_MIXED, B.OBEM_FP64])
def test_noalloc_at_the_limit(ctx, prec):
    """OBEM_NOALLOC_MAX_POINTS charges (targets = sources) in the 40,776-cell
    GEM cell: the workspace of the largest call fits the static array."""
    m = W.gem_cell_mesh()
    bm = bind(ctx, m)
    sig = dev(synthetic_sigma(m))
    n = 16384
    rng = np.random.default_rng(23)
    x = rng.normal(size=(n, 3)) * 3e-5 + np.array([0, 0, 2e-4])
    q = rng.choice([-1.0, 1.0], size=n) * W.E_CHARGE
    X, Q = dev(x), dev(q)
    st, E0 = _noalloc(ctx, bm, sig, X, Q, X, 1e-7, prec, True)
    assert st == 0, ctx.lib.obem_last_error(ctx.h)
    E1 = B.field_eval(ctx, bm, sig, X, Q, X, 1e-7, prec, tgt_is_src=True)
    err = rel_l2(host(E0), host(E1))
    print(f"noalloc at the limit, prec {prec}: rel L2 vs field_eval {err:.3g}")
    assert err <= TOL[prec]


def test_noalloc_rejects_sizes_beyond_the_limit(ctx):
    n = 16385
    X = dev(np.zeros((n, 3)))
    Q = dev(np.zeros(n))
    st, _ = _noalloc(ctx, None, None, X, Q, X, 1e-7, B.OBEM_MIXED, True)
    assert st == -1                              # OBEM_EINVAL, before any launch
    assert b"16384" in ctx.lib.obem_last_error(ctx.h)
