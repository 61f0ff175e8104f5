"""Small calls of every oracle entry point, for the sanitizer build test:
`run(path)` writes the results to an .npz.  Run as a script it uses the
oracle library named by OBEM_ORACLE_LIB (the sanitized build)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(path):
    import oracle as O
    from paper_2110_09214_amd import workloads as W

    out = {}
    rng = np.random.default_rng(3)
    a, b, c = np.array([0.0, 0, 0]), np.array([1e-4, 0, 0]), np.array([0.3e-4, 0.8e-4, 0])
    r = np.array([0.2e-4, 0.3e-4, 0.4e-4])
    out["iv"], out["ie"] = O.tri_integrals(a, b, c, r)
    out["grad"] = O.tri_grad(a, b, c, r)
    m = W.plates_with_slab_mesh(n=4, half=1e-3, gap=1e-3, t=0.4e-3)
    nrm, area, cen, diam = O.tri_geometry(m.a, m.b, m.c)
    out["area"] = area
    sig, A = O.bem_solve(m)
    out["sigma"] = sig
    out["resid"], out["resid_abs"] = O.bem_residual_rows(m, sig, m.rhs, np.arange(0, m.n, 7))
    x = rng.uniform([-8e-4, -8e-4, 5e-4], [8e-4, 8e-4, 9e-4], size=(300, 3))
    q = rng.choice([-1.0, 1.0], size=300) * W.E_CHARGE
    sp = (q > 0).astype(np.int8)
    out["Ep"], out["Vp"] = O.panel_field(x, m.a, m.b, m.c, sig, want_v=True)
    out["Eq"], out["Vq"], out["nn"], out["d2"] = O.pair_field(x, x, q, 1e-7, tgt_is_src=True, want_v=True,
                                                             sp_t=sp, sp_s=sp)
    w = rng.normal(size=(300, 3))
    gs, gx = O.panel_backward(x, m, sig, w)
    out["gs"], out["gx"] = gs, gx
    out["gpair"], _ = O.pair_backward(x, x, q, 1e-7, w, tgt_is_src=True)
    out["fd"] = O.fd_particle(x, q, w, 1e-7, m, sig, 5, 2, 1e-9)
    out["infl"], out["vbar"], out["ebar"] = O.influence(m, m.rhs, x, q)
    out["adj"] = O.bem_solve_adjoint(m, rng.normal(size=m.n), A=A)
    out["philox"] = O.philox4x32_10(np.array([1, 2, 3, 4], np.uint32), np.array([5, 6], np.uint32))
    gas = W.synthetic_ar_co2(anisotropic=True, penning_prob=0.574, penning_level=12.5)
    out["numax"] = O.nu_max_electron(gas)
    out["xs"] = np.array([O.xs_at(gas, k, e) for k in range(5) for e in (0.005, 1.0, 20.0, 2000.0)])
    out["aniso"] = np.array([O.aniso_cos(xi, R) for xi in (0.0, 0.5, 0.9) for R in (0.1, 0.5, 0.9)])
    # three tracking steps of both steppers on a cloud above the slab
    for stepper, dt in ((0, 1e-12), (2, 25e-15)):
        n = 200
        xs = rng.normal(size=(n, 3)) * 3e-5 + np.array([0, 0, 6e-4])
        eps = rng.uniform(1.0, 60.0, n)
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        spc = (np.arange(n) % 3 == 0).astype(np.int8)
        v *= np.where(spc == 0, np.sqrt(2 * eps * W.E_CHARGE / W.M_ELECTRON), 300.0)[:, None]
        state = dict(x=xs, v=v, species=spc, id=np.arange(n, dtype=np.int64), next_id=n)
        counts = np.zeros(m.n, np.int64)
        s = sig.copy()
        for k in range(3):
            p = dict(dt=dt, step=k, seed=5, max_coll=64, max_ion_per_step=4, ion_v_cap=2e4,
                     box_lo=(-1e-3, -1e-3, 0.0), box_hi=(1e-3, 1e-3, 1e-3), soft=1e-7, r_rec=1e-6, capacity=5000,
                     stepper=stepper)
            state, s, counts, st, _ = O.track_step(state, m, s, gas, p, counts, rhs0=m.rhs, area=area, A=A,
                                                   resolve=k > 0)
        out[f"track{stepper}_x"] = state["x"]
        out[f"track{stepper}_id"] = state["id"]
        out[f"track{stepper}_counts"] = counts
    np.savez(path, **out)


if __name__ == "__main__":
    run(sys.argv[1])
