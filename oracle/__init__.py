"""CPU oracle for the space-charge field path (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library (paper_2110_09214_amd) neither imports it
nor shares code with it.

The arithmetic lives in oracle.c (plain C, FP64 inputs, long-double
accumulation, brute force over all pairs); this module wraps it with numpy and
adds the steps that are plain bookkeeping: the dense LU solve of the
collocation system (a library routine), the recombination matching, the
compaction with deterministic ids and the charging-up counts.

Paper: OuroborosBEM, arXiv 2110.09214.  Each function names the passage it
follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no fast-math; OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_sanitized(out_path: str) -> str:
    """Compile oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts) into out_path, for the sanitizer test."""
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", _SRC, "-o",
           out_path, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("OBEM_ORACLE_LIB")     # a sanitizer build (tests only)
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        _lib = C.CDLL(path)
    return _lib


_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------------------
# constants
# ---------------------------------------------------------------------------
def constants() -> dict:
    out = np.zeros(6)
    lib().oc_constants(_p(out))
    return dict(eps0=out[0], k_e=out[1], e=out[2], m_e=out[3], k_B=out[4], u=out[5])


# ---------------------------------------------------------------------------
# cell integrals (eqs. BEM2 / BEM3 per unit density)
# ---------------------------------------------------------------------------
def tri_integrals(a, b, c, r):
    """(IV, IE[3]) of one flat triangle at point r."""
    a, b, c, r = (_f64(v, (3,)) for v in (a, b, c, r))
    iv = np.zeros(1)
    ie = np.zeros(3)
    lib().oc_tri_integrals(_p(a), _p(b), _p(c), _p(r), _p(iv), _p(ie))
    return iv[0], ie


def tri_grad(a, b, c, r):
    """G[j, k] = d IE_j / d r_k."""
    a, b, c, r = (_f64(v, (3,)) for v in (a, b, c, r))
    g = np.zeros(9)
    lib().oc_tri_grad(_p(a), _p(b), _p(c), _p(r), _p(g))
    return g.reshape(3, 3)


def tri_geometry(a, b, c):
    """normal (N,3), area (N,), centroid (N,3), diameter (N,) = longest edge."""
    a, b, c = (_f64(v) for v in (a, b, c))
    N = a.shape[0]
    nrm = np.zeros((N, 3)); area = np.zeros(N); cen = np.zeros((N, 3)); diam = np.zeros(N)
    lib().oc_tri_geometry(C.c_int64(N), _p(a), _p(b), _p(c), _p(nrm), _p(area), _p(cen), _p(diam))
    return nrm, area, cen, diam


# ---------------------------------------------------------------------------
# field evaluation
# ---------------------------------------------------------------------------
def panel_field(x, a, b, c, sigma, want_v=False):
    """E (n,3) [and V (n,)] at points x from cells with constant sigma,
    eqs. (BEM2), (BEM3)."""
    x = _f64(x).reshape(-1, 3)
    a, b, c, sigma = _f64(a), _f64(b), _f64(c), _f64(sigma)
    E = np.zeros((x.shape[0], 3))
    V = np.zeros(x.shape[0]) if want_v else None
    lib().oc_panel_field(C.c_int64(x.shape[0]), _p(x), C.c_int64(a.shape[0]), _p(a), _p(b), _p(c),
                         _p(sigma), _p(E), _p(V))
    return (E, V) if want_v else E


def pair_field(xt, xs, q, soft, tgt_is_src=False, want_v=False, sp_t=None, sp_s=None):
    """Direct pairwise field, eq. (nbody), Plummer softening `soft`.  With
    species arrays also returns (nn_idx, nn_d2): nearest opposite-species
    source (electron <-> cation) for each target."""
    xt = _f64(xt).reshape(-1, 3)
    xs = _f64(xs).reshape(-1, 3)
    q = _f64(q)
    nt = xt.shape[0]
    E = np.zeros((nt, 3))
    V = np.zeros(nt) if want_v else None
    want_nn = sp_t is not None
    nn = np.full(nt, -1, np.int64) if want_nn else None
    d2 = np.full(nt, np.inf) if want_nn else None
    spt = np.ascontiguousarray(sp_t, np.int8) if want_nn else None
    sps = np.ascontiguousarray(sp_s, np.int8) if want_nn else None
    lib().oc_pair_field(C.c_int64(nt), _p(xt), C.c_int64(xs.shape[0]), _p(xs), _p(q), C.c_double(soft),
                        C.c_int(1 if tgt_is_src else 0), _p(E), _p(V), _p(spt), _p(sps), _p(nn), _p(d2))
    out = [E]
    if want_v:
        out.append(V)
    if want_nn:
        out += [nn, d2]
    return out[0] if len(out) == 1 else tuple(out)


def field(x_t, mesh, sigma, xs, q, soft, tgt_is_src=False, want_v=False):
    """Total field: panels + point charges (either part may be absent)."""
    x_t = _f64(x_t).reshape(-1, 3)
    E = np.zeros_like(x_t)
    V = np.zeros(x_t.shape[0])
    if mesh is not None:
        r = panel_field(x_t, mesh.a, mesh.b, mesh.c, sigma, want_v=True)
        E += r[0]
        V += r[1]
    if xs is not None and len(q):
        r = pair_field(x_t, xs, q, soft, tgt_is_src=tgt_is_src, want_v=True)
        E += r[0]
        V += r[1]
    return (E, V) if want_v else E


# ---------------------------------------------------------------------------
# collocation system, eq. (matrixBEM)
# ---------------------------------------------------------------------------
def bem_matrix(mesh):
    N = mesh.n
    A = np.zeros((N, N))
    lib().oc_bem_assemble(C.c_int64(N), _p(_f64(mesh.a)), _p(_f64(mesh.b)), _p(_f64(mesh.c)),
                          _p(np.ascontiguousarray(mesh.kind, np.int8)), _p(_f64(mesh.eps1)),
                          _p(_f64(mesh.eps2)), _p(A))
    return A


def residual_dense(A, x, b):
    """b - A x with long-double accumulation."""
    A, x, b = _f64(A), _f64(x), _f64(b)
    r = np.zeros_like(b)
    lib().oc_residual_dense(C.c_int64(b.shape[0]), _p(A), _p(x), _p(b), _p(r))
    return r


def bem_solve(mesh, rhs=None, A=None, refine=2):
    """sigma solving eq. (matrixBEM) by LU (numpy/LAPACK dgesv) plus
    iterative refinement with an extended-precision residual.  Returns
    (sigma, A)."""
    if A is None:
        A = bem_matrix(mesh)
    b = _f64(mesh.rhs if rhs is None else rhs)
    sig = np.linalg.solve(A, b)
    for _ in range(refine):
        sig = sig + np.linalg.solve(A, residual_dense(A, sig, b))
    return sig, A


def bem_residual_rows(mesh, sigma, rhs, rows):
    """Matrix-free r_i = rhs_i - sum_j A_ij sigma_j (A regenerated row by row)
    and sum_j |A_ij| for the listed rows."""
    rows = np.ascontiguousarray(rows, np.int64)
    res = np.zeros(rows.shape[0])
    absr = np.zeros(rows.shape[0])
    lib().oc_bem_residual_rows(C.c_int64(mesh.n), _p(_f64(mesh.a)), _p(_f64(mesh.b)), _p(_f64(mesh.c)),
                               _p(np.ascontiguousarray(mesh.kind, np.int8)), _p(_f64(mesh.eps1)),
                               _p(_f64(mesh.eps2)), _p(_f64(sigma)), _p(_f64(rhs)), C.c_int64(rows.shape[0]),
                               _p(rows), _p(res), _p(absr))
    return res, absr


# ---------------------------------------------------------------------------
# adjoint (not in the paper): L = sum_i w_i . E(x_i)
# ---------------------------------------------------------------------------
def panel_backward(x, mesh, sigma, w, want_sigma=True, want_x=True):
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    gs = np.zeros(mesh.n) if want_sigma else None
    gx = np.zeros_like(x) if want_x else None
    lib().oc_panel_backward(C.c_int64(x.shape[0]), _p(x), C.c_int64(mesh.n), _p(_f64(mesh.a)),
                            _p(_f64(mesh.b)), _p(_f64(mesh.c)), _p(_f64(sigma)), _p(w), _p(gs), _p(gx))
    return gs, gx


def pair_backward(xt, xs, q, soft, w, tgt_is_src=False):
    xt = _f64(xt).reshape(-1, 3)
    xs = _f64(xs).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    gt = np.zeros_like(xt)
    gs = None if tgt_is_src else np.zeros_like(xs)
    lib().oc_pair_backward(C.c_int64(xt.shape[0]), _p(xt), C.c_int64(xs.shape[0]), _p(xs), _p(_f64(q)),
                           C.c_double(soft), C.c_int(1 if tgt_is_src else 0), _p(w), _p(gt), _p(gs))
    return gt, gs


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


# ---------------------------------------------------------------------------
# transport step
# ---------------------------------------------------------------------------
class _Gas(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("e_min", C.c_double), ("e_max", C.c_double),
                ("xs", C.c_void_p), ("thr", C.c_double * 5), ("density", C.c_double),
                ("temperature", C.c_double), ("m_gas", C.c_double), ("m_cation", C.c_double),
                ("m_anion", C.c_double), ("ion_xs_iso", C.c_double), ("ion_xs_back", C.c_double),
                ("xi", C.c_void_p), ("penning_prob", C.c_double), ("penning_level", C.c_double)]


class _Step(C.Structure):
    _fields_ = [("dt", C.c_double), ("step", C.c_uint32), ("seed", C.c_uint64), ("max_coll", C.c_int32),
                ("max_ion_per_step", C.c_int32), ("ion_v_cap", C.c_double), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3)]


def _gas_struct(gas):
    xs = np.ascontiguousarray(gas.xs, np.float64)
    xi = None if getattr(gas, "xi", None) is None else np.ascontiguousarray(gas.xi, np.float64)
    g = _Gas(n_nodes=xs.shape[1], e_min=gas.e_min, e_max=gas.e_max, xs=xs.ctypes.data,
             density=gas.density, temperature=gas.temperature, m_gas=gas.m_gas, m_cation=gas.m_cation,
             m_anion=gas.m_anion, ion_xs_iso=gas.ion_xs_iso, ion_xs_back=gas.ion_xs_back,
             xi=None if xi is None else xi.ctypes.data, penning_prob=float(getattr(gas, "penning_prob", 0.0)),
             penning_level=float(getattr(gas, "penning_level", 0.0)))
    for k in range(5):
        g.thr[k] = float(gas.thresholds[k])
    return g, (xs, xi)


def nu_max_electron(gas):
    g, keep = _gas_struct(gas)
    lib().oc_nu_max_electron.restype = C.c_double
    return lib().oc_nu_max_electron(C.byref(g))


def xs_at(gas, k, eps):
    """Cross section k at energy eps (eV): linear in the normalised lethargy of
    eq. (leth) between nodes."""
    g, keep = _gas_struct(gas)
    lib().oc_xs_at.restype = C.c_double
    return lib().oc_xs_at(C.byref(g), C.c_int(k), C.c_double(eps))


COUNTER_NAMES = ["elastic", "exc1", "exc2", "ionisation", "attachment", "null", "ion_collisions",
                 "rate_overflow", "flight_cap", "children_dropped", "penning"]


def mc_step(x, v, species, ids, E, gas, params, mesh=None, skip=None):
    """One constant-field step with null-collision MC for every particle.
    Arrays are updated in place (x, v, species); returns (status, hit,
    n_child, child_x, child_v, counters)."""
    n = x.shape[0]
    mi = int(params["max_ion_per_step"])
    g, keep = _gas_struct(gas)
    p = _Step(dt=params["dt"], step=params["step"], seed=params["seed"], max_coll=params["max_coll"],
              max_ion_per_step=mi, ion_v_cap=params["ion_v_cap"])
    for k in range(3):
        p.box_lo[k] = params["box_lo"][k]
        p.box_hi[k] = params["box_hi"][k]
    status = np.zeros(n, np.int8)
    hit = np.zeros(n, np.int64)
    n_child = np.zeros(n, np.int32)
    child_x = np.zeros((max(n, 1) * mi * 2, 3))
    child_v = np.zeros((max(n, 1) * mi * 2, 3))
    counters = np.zeros(len(COUNTER_NAMES), np.int64)
    if mesh is not None:
        a, b, c = _f64(mesh.a), _f64(mesh.b), _f64(mesh.c)
        N = mesh.n
    else:
        a = b = c = np.zeros((1, 3))
        N = 0
    sk = None if skip is None else np.ascontiguousarray(skip, np.uint8)
    lib().oc_mc_step(C.c_int64(n), _p(x), _p(v), _p(species), _p(ids), _p(_f64(E)), _p(sk), C.byref(g),
                     C.byref(p), C.c_int64(N), _p(a), _p(b), _p(c), _p(status), _p(hit), _p(n_child),
                     _p(child_x), _p(child_v), _p(counters))
    return status, hit, n_child, child_x.reshape(max(n, 1), mi, 2, 3), child_v.reshape(max(n, 1), mi, 2, 3), counters


def _step_struct(params):
    p = _Step(dt=params["dt"], step=params["step"], seed=params["seed"], max_coll=params["max_coll"],
              max_ion_per_step=int(params["max_ion_per_step"]), ion_v_cap=params["ion_v_cap"])
    for k in range(3):
        p.box_lo[k] = params["box_lo"][k]
        p.box_hi[k] = params["box_hi"][k]
    return p


def _mesh_arrays(mesh):
    if mesh is not None:
        return _f64(mesh.a), _f64(mesh.b), _f64(mesh.c), mesh.n
    z = np.zeros((1, 3))
    return z, z, z, 0


def aniso_cos(xi, R):
    """cos theta of eq. (anisotrop) for anisotropy xi and uniform R."""
    lib().oc_aniso_cos.restype = C.c_double
    return lib().oc_aniso_cos(C.c_double(xi), C.c_double(R))


def flight(x, v, species, E, gas, params, tau, status, hit, mesh=None, skip=None):
    """Flight of duration tau (constant acceleration qE/m, E None = straight
    drift) for live particles, with absorption and world-box tests; x, v,
    status, hit updated in place (section 3.3.5 steppers)."""
    n = x.shape[0]
    g, keep = _gas_struct(gas)
    p = _step_struct(params)
    a, b, c, N = _mesh_arrays(mesh)
    sk = None if skip is None else np.ascontiguousarray(skip, np.uint8)
    Ep = None if E is None else _f64(E)
    lib().oc_flight(C.c_int64(n), _p(x), _p(v), _p(species), _p(Ep), _p(sk), C.byref(g), C.byref(p),
                    C.c_double(tau), C.c_int64(N), _p(a), _p(b), _p(c), _p(status), _p(hit))


def collide_step(x, v, species, ids, gas, params, status, skip=None):
    """Per-step collision test of section 3.4.2 for live particles (in place);
    returns (n_child, child_x, child_v, counters)."""
    n = x.shape[0]
    mi = int(params["max_ion_per_step"])
    g, keep = _gas_struct(gas)
    p = _step_struct(params)
    n_child = np.zeros(n, np.int32)
    child_x = np.zeros((max(n, 1) * mi * 2, 3))
    child_v = np.zeros((max(n, 1) * mi * 2, 3))
    counters = np.zeros(len(COUNTER_NAMES), np.int64)
    sk = None if skip is None else np.ascontiguousarray(skip, np.uint8)
    lib().oc_collide_step(C.c_int64(n), _p(x), _p(v), _p(species), _p(ids), _p(sk), C.byref(g), C.byref(p),
                          _p(status), _p(n_child), _p(child_x), _p(child_v), _p(counters))
    return n_child, child_x.reshape(max(n, 1), mi, 2, 3), child_v.reshape(max(n, 1), mi, 2, 3), counters


def recombine(species, ids, nn_idx, nn_d2, r_rec):
    """Two-body electron-cation recombination (section 3.4.3, eq. (distRecomb)
    with the radius given as a parameter): every electron proposes to its
    nearest cation if within r_rec; each cation accepts its nearest proposer
    (ties to the lower id); accepted pairs are removed.  Returns a bool mask of
    removed particles."""
    n = species.shape[0]
    dead = np.zeros(n, bool)
    best = {}
    for e in np.nonzero((species == 0) & (nn_idx >= 0) & (nn_d2 <= r_rec * r_rec))[0]:
        cidx = int(nn_idx[e])
        key = (nn_d2[e], int(ids[e]))
        if cidx not in best or key < best[cidx][0]:
            best[cidx] = (key, int(e))
    for cidx, (_, e) in best.items():
        dead[cidx] = True
        dead[e] = True
    return dead


def track_step(state, mesh, sigma, gas, params, dd_counts, rhs0=None, area=None, A=None, resolve=False,
               with_influence=False, field_map=None):
    """One tracking step, in the order: (re-)solve for sigma if charge was
    deposited (eq. (charge-up)), with with_influence after moving the
    particles' influence onto the left-hand side (section 3.3.2), field at the
    start positions (panels + pairwise), recombination, constant-field
    flights with null-collision MC and absorption, compaction with appended
    children, charging-up counts.  field_map = (Emap, lo, h): the static
    option (section 3.3.1), the field of the set-up interpolated in the map
    instead of summed over the cells.

    params["stepper"] selects the transport (section 3.3.5 and 3.4.2): 0 =
    constant-field flights with null collisions (above); 1 = Euler (one
    constant-field flight over dt in the start field) and 2 = PEFRL (4 force
    evaluations at the intermediate positions, field of the set-up plus the
    charges still alive, at those positions), both followed by the per-step
    collision test.  The start-of-step field evaluation gives the
    recombination partners in every mode.

    state: dict with x (n,3), v (n,3), species (n,) int8, id (n,) int64,
    next_id int.  Returns (new_state, sigma, stats)."""
    x = state["x"].copy()
    v = state["v"].copy()
    sp = state["species"].copy()
    ids = state["id"].copy()
    e = constants()["e"]
    q = np.where(sp == 1, e, -e).astype(np.float64)
    if resolve:
        dd = mesh.kind == 1
        rhs = np.array(rhs0, np.float64)
        rhs[dd] += e * dd_counts[dd] / area[dd]
        if with_influence and x.shape[0]:
            rhs, _, _ = influence(mesh, rhs, x, q)
        sigma, _ = bem_solve(mesh, rhs, A=A)
    n = x.shape[0]
    stats = {}
    if n:
        E_pair, nn, d2 = pair_field(x, x, q, params["soft"], tgt_is_src=True, sp_t=sp, sp_s=sp)
        if field_map is not None:
            E = E_pair + trilinear(field_map[0], field_map[1], field_map[2], x)
        else:
            E = E_pair + (panel_field(x, mesh.a, mesh.b, mesh.c, sigma) if mesh is not None else 0.0)
        dead = recombine(sp, ids, nn, d2, params["r_rec"])
    else:
        E = np.zeros((0, 3))
        dead = np.zeros(0, bool)
    stepper = int(params.get("stepper", 0))
    if stepper == 0:
        status, hit, n_child, cx, cv, counters = mc_step(x, v, sp, ids, E, gas, params, mesh, skip=dead)
    else:
        status = np.zeros(n, np.int8)
        hit = np.full(n, -1, np.int64)
        if stepper == 1:
            flight(x, v, sp, E, gas, params, params["dt"], status, hit, mesh, skip=dead)
        else:
            _pefrl(x, v, sp, q, dead, status, hit, gas, params, mesh, sigma, field_map)
        n_child, cx, cv, counters = collide_step(x, v, sp, ids, gas, params, status, skip=dead)
    stats["recombined"] = int(dead.sum())
    stats["absorbed"] = int((status == 1).sum())
    stats["left"] = int((status == 2).sum())
    stats.update({k: int(val) for k, val in zip(COUNTER_NAMES, counters)})
    # charging-up: integer elementary-charge counts per dd cell (eq. (charge-up))
    new_counts = dd_counts.copy()
    for i in np.nonzero(status == 1)[0]:
        h = int(hit[i])
        if mesh.kind[h] == 1:
            new_counts[h] += 1 if sp[i] == 1 else -1
    keep = (~dead) & (status == 0)
    # compaction: survivors in id order, then children in parent order
    out_x = [x[keep]]
    out_v = [v[keep]]
    out_sp = [sp[keep]]
    out_id = [ids[keep]]
    n_surv = int(keep.sum())
    cap = int(params["capacity"])
    room = max(0, cap - n_surv)
    chx, chv, chs = [], [], []
    for i in np.nonzero(n_child > 0)[0]:
        for k in range(int(n_child[i])):
            for s in (0, 1):
                chx.append(cx[i, k, s]); chv.append(cv[i, k, s]); chs.append(s)
    n_new = len(chs)
    take = min(room, n_new)
    stats["children_dropped"] = stats.get("children_dropped", 0) + (n_new - take)
    nid = int(state["next_id"])
    if take:
        out_x.append(np.array(chx[:take]).reshape(-1, 3))
        out_v.append(np.array(chv[:take]).reshape(-1, 3))
        out_sp.append(np.array(chs[:take], np.int8))
        out_id.append(nid + np.arange(take, dtype=np.int64))
    new_state = dict(x=np.concatenate(out_x), v=np.concatenate(out_v), species=np.concatenate(out_sp),
                     id=np.concatenate(out_id), next_id=nid + take)
    stats["n_live"] = new_state["x"].shape[0]
    stats["children"] = take
    return new_state, sigma, new_counts, stats, E


# Position-extended Forest-Ruth-like integrator (Omelyan, Mryglod, Folk,
# Comput. Phys. Commun. 146 (2002) 188), the PEFRL of section 3.3.5.
PEFRL_XI = 0.1786178958448091
PEFRL_LAMBDA = -0.2123418310626054
PEFRL_CHI = -0.06626458266981849


def _pefrl(x, v, sp, q, dead, status, hit, gas, params, mesh, sigma, field_map):
    """One PEFRL step in place: drifts (straight, absorption and box tested)
    and kicks q E(x) / m with E re-evaluated after each drift from the set-up
    (cells or map) and the charges not yet removed, at their current
    positions."""
    dt = params["dt"]
    masses = np.array([constants()["m_e"], gas.m_cation, gas.m_anion])
    drifts = [PEFRL_XI, PEFRL_CHI, 1.0 - 2.0 * (PEFRL_CHI + PEFRL_XI), PEFRL_CHI, PEFRL_XI]
    kicks = [0.5 * (1.0 - 2.0 * PEFRL_LAMBDA), PEFRL_LAMBDA, PEFRL_LAMBDA, 0.5 * (1.0 - 2.0 * PEFRL_LAMBDA)]
    for s_, cd in enumerate(drifts):
        flight(x, v, sp, None, gas, params, cd * dt, status, hit, mesh, skip=dead)
        if s_ == len(kicks):
            break
        live = (~dead) & (status == 0)
        qm = np.where(live, q, 0.0)
        E = pair_field(x, x, qm, params["soft"], tgt_is_src=True)
        if field_map is not None:
            E = E + trilinear(field_map[0], field_map[1], field_map[2], x)
        elif mesh is not None:
            E = E + panel_field(x, mesh.a, mesh.b, mesh.c, sigma)
        acc = (q / masses[sp])[:, None] * E
        v[live] += kicks[s_] * dt * acc[live]


def fd_particle(x, q, w, soft, mesh, sigma, m, axis, h):
    """Central difference of L = sum_i w_i . E(x_i) in coordinate `axis` of
    particle m (targets = sources), re-summing only the terms involving m."""
    x = _f64(x).reshape(-1, 3)
    w = _f64(w).reshape(-1, 3)
    if mesh is not None:
        a, b, c, N, sg = _f64(mesh.a), _f64(mesh.b), _f64(mesh.c), mesh.n, _f64(sigma)
    else:
        a = b = c = np.zeros((1, 3))
        N, sg = 0, np.zeros(1)
    lib().oc_fd_particle.restype = C.c_double
    return lib().oc_fd_particle(C.c_int64(x.shape[0]), _p(x), _p(_f64(q)), _p(w), C.c_double(soft), C.c_int64(N),
                                _p(a), _p(b), _p(c), _p(sg), C.c_int64(m), C.c_int(axis), C.c_double(h))


def bem_solve_adjoint(mesh, g_sigma, A=None, refine=2):
    """lambda with A^T lambda = g_sigma (LAPACK dgesv on A^T plus refinement
    with a long-double residual): the gradient with respect to the
    left-hand side of eq. (matrixBEM)."""
    if A is None:
        A = bem_matrix(mesh)
    At = np.ascontiguousarray(A.T)
    g = _f64(g_sigma)
    lam = np.linalg.solve(At, g)
    for _ in range(refine):
        lam = lam + np.linalg.solve(At, residual_dense(At, lam, g))
    return lam


def influence(mesh, rhs, x, q):
    """Left-hand side modified by the charges q at x (eqs. potpart, fldpart,
    BEMpotpart, BEMfldpart); returns (rhs_out, Vbar (N,), Ebar (N,3))."""
    x = _f64(x).reshape(-1, 3)
    N = mesh.n
    out = np.zeros(N)
    vb = np.zeros(N)
    eb = np.zeros((N, 3))
    lib().oc_influence(C.c_int64(N), _p(_f64(mesh.a)), _p(_f64(mesh.b)), _p(_f64(mesh.c)),
                       _p(np.ascontiguousarray(mesh.kind, np.int8)), _p(_f64(mesh.eps1)), _p(_f64(mesh.eps2)),
                       _p(_f64(rhs)), C.c_int64(x.shape[0]), _p(x), _p(_f64(q)), _p(out), _p(vb), _p(eb))
    return out, vb, eb


# --------------------------------------------------------------------------
# Static field option (section 3.3.1): field of the cells on a uniform 3D
# grid, computed once, and trilinear interpolation at the particles.
# --------------------------------------------------------------------------
def field_map(mesh, sigma, lo, h, n):
    """Cell field (eq. (BEM3)) at the nodes lo + (i, j, k) h of a uniform grid
    with n = (nx, ny, nz) nodes; returns E with shape (nz, ny, nx, 3)."""
    nx, ny, nz = (int(v) for v in n)
    gx = lo[0] + h[0] * np.arange(nx)
    gy = lo[1] + h[1] * np.arange(ny)
    gz = lo[2] + h[2] * np.arange(nz)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    E = panel_field(pts, mesh.a, mesh.b, mesh.c, sigma)
    return E.reshape(nz, ny, nx, 3)


def trilinear(Emap, lo, h, x):
    """Trilinear interpolation of the node values Emap (nz, ny, nx, 3) at the
    points x (n, 3).  Reading: the paper leaves points outside the grid open;
    they are clamped onto the grid box (the field of the nearest boundary
    point)."""
    x = _f64(x).reshape(-1, 3)
    nz, ny, nx = Emap.shape[:3]
    size = np.array([nx, ny, nz])
    u = (x - np.asarray(lo, np.float64)) / np.asarray(h, np.float64)
    u = np.clip(u, 0.0, size - 1.0)
    i0 = np.minimum(np.floor(u).astype(np.int64), size - 2)
    f = u - i0
    out = np.zeros((x.shape[0], 3))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) *
                     (f[:, 2] if dz else 1 - f[:, 2]))
                out += w[:, None] * Emap[i0[:, 2] + dz, i0[:, 1] + dy, i0[:, 0] + dx]
    return out


# --------------------------------------------------------------------------
# Signal induction (section 3.5, eq. (ramo))
# --------------------------------------------------------------------------
def induced_current(Ew, v, q, species):
    """Shockley-Ramo current i = sum_p q_p v_p . E_w(x_p) split by species
    (electrons, cations, anions), given the weighting field Ew (n, 3) at the
    particles.  Returns (currents[3], per-particle terms)."""
    terms = q * np.einsum("ij,ij->i", _f64(v).reshape(-1, 3), _f64(Ew).reshape(-1, 3))
    cur = np.array([terms[species == s].sum() for s in (0, 1, 2)])
    return cur, terms
