"""ctypes binding of libobem (C ABI in include/obem.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions take torch tensors on the GPU (float64, int8, int64 as
the header states), contiguous, and pass their data pointers.  The library is
loaded on first use; if it has not been built, or the process has no GPU, the
calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libobem.so")

OBEM_FP64 = 0
OBEM_MIXED = 1
OBEM_TGT_IS_SRC = 1
OBEM_WANT_V = 2

STATUS = {0: "OBEM_OK", -1: "OBEM_EINVAL", -2: "OBEM_ENOMEM", -3: "OBEM_EDEVICE", -4: "OBEM_ESINGULAR",
          -5: "OBEM_ENOCONV", -6: "OBEM_ECAPACITY", -7: "OBEM_ESTATE"}


class ObemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Mesh_t(C.Structure):
    _fields_ = [("n_panels", C.c_int64)] + [(n, C.c_void_p) for n in
                                            ("ax", "ay", "az", "bx", "by", "bz", "cx", "cy", "cz", "kind",
                                             "eps_r1", "eps_r2")]


class SolveInfo_t(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("backward_error", C.c_double), ("residual_inf", C.c_double)]


class Particles_t(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("n_live", C.c_int64), ("next_id", C.c_int64)] + [
        (n, C.c_void_p) for n in ("x", "y", "z", "vx", "vy", "vz", "species", "id")]


class Gas_t(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("e_min", C.c_double), ("e_max", C.c_double), ("xs", C.c_void_p),
                ("thr", C.c_double * 5), ("density", C.c_double), ("temperature", C.c_double),
                ("m_gas", C.c_double), ("m_cation", C.c_double), ("m_anion", C.c_double),
                ("ion_xs_iso", C.c_double), ("ion_xs_back", C.c_double), ("xi", C.c_void_p),
                ("penning_prob", C.c_double), ("penning_level", C.c_double)]


class StepParams_t(C.Structure):
    _fields_ = [("dt", C.c_double), ("step", C.c_uint32), ("seed", C.c_uint64), ("max_coll", C.c_int32),
                ("max_ion_per_step", C.c_int32), ("ion_v_cap", C.c_double), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3), ("soft", C.c_double), ("r_rec", C.c_double),
                ("precision", C.c_int), ("resolve", C.c_int32), ("influence", C.c_int32),
                ("rhs0", C.c_void_p), ("stepper", C.c_int32), ("map", C.c_void_p), ("field_out", C.c_void_p)]


class FieldMap_t(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("lo", C.c_double * 3),
                ("h", C.c_double * 3), ("ex", C.c_void_p), ("ey", C.c_void_p), ("ez", C.c_void_p)]


class StepStats_t(C.Structure):
    _fields_ = [("n_live", C.c_int64), ("recombined", C.c_int64), ("absorbed", C.c_int64),
                ("left_world", C.c_int64), ("children", C.c_int64), ("children_dropped", C.c_int64),
                ("real_collisions", C.c_int64 * 5), ("null_collisions", C.c_int64),
                ("ion_collisions", C.c_int64), ("rate_overflow", C.c_int64), ("flight_cap", C.c_int64),
                ("dd_charge_deposited", C.c_int64), ("penning", C.c_int64)]


SYMBOLS = ["obem_create", "obem_destroy", "obem_last_error", "obem_constants", "obem_profile_enable",
           "obem_profile_read", "obem_profile_work", "obem_mesh_bind",
           "obem_mesh_release", "obem_mesh_geometry", "bem_solve_charges", "bem_solve_charges_adjoint", "bem_influence",
           "field_eval", "field_eval_noalloc", "field_eval_backward", "field_map_build", "field_map_eval", "induced_current", "track_step"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libobem.so and declare its signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2110_09214_amd.build`")
    lib = C.CDLL(path)
    vp, i64, d, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
    lib.obem_create.argtypes = [C.POINTER(vp), i32, vp]
    lib.obem_destroy.argtypes = [vp]
    lib.obem_last_error.argtypes = [vp]
    lib.obem_last_error.restype = C.c_char_p
    lib.obem_constants.argtypes = [vp]
    lib.obem_constants.restype = None
    lib.obem_profile_enable.argtypes = [vp, i32]
    lib.obem_profile_read.argtypes = [vp, i32, vp, vp, vp, C.POINTER(C.c_int)]
    lib.obem_profile_work.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    lib.obem_mesh_bind.argtypes = [vp, C.POINTER(Mesh_t), C.POINTER(vp)]
    lib.obem_mesh_release.argtypes = [vp, vp]
    lib.obem_mesh_geometry.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.bem_solve_charges.argtypes = [vp, vp, vp, vp, i32, C.POINTER(SolveInfo_t)]
    lib.bem_solve_charges_adjoint.argtypes = [vp, vp, vp, vp, i32, C.POINTER(SolveInfo_t)]
    lib.bem_influence.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.field_map_build.argtypes = [vp, vp, vp, C.POINTER(FieldMap_t), i32]
    lib.field_map_eval.argtypes = [vp, C.POINTER(FieldMap_t), i64, vp, vp, vp, vp, vp, vp]
    lib.induced_current.argtypes = [vp, vp, vp, C.POINTER(FieldMap_t), i64, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.field_eval.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, d, i32, C.c_uint, vp, vp, vp, vp]
    lib.field_eval_noalloc.argtypes = lib.field_eval.argtypes
    lib.field_eval_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, d, i32, C.c_uint,
                                        vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.track_step.argtypes = [vp, vp, C.POINTER(Particles_t), C.POINTER(Gas_t), C.POINTER(StepParams_t), vp, vp,
                               C.POINTER(StepStats_t)]
    for name in SYMBOLS:
        if name not in ("obem_last_error", "obem_constants"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def obem_constants():
    out = (C.c_double * 6)()
    load().obem_constants(out)
    return dict(eps0=out[0], k_e=out[1], e=out[2], m_e=out[3], k_B=out[4], u=out[5])


def _ptr(t, dtype=torch.float64, n=None, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return C.c_void_p(t.data_ptr())


class Context:
    """One obem context on a GPU, launching on torch's current stream of that
    device at creation time."""

    def __init__(self, device: int = 0):
        lib = load()
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib.obem_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise ObemError(st, "obem_create failed (is this a gfx950 GPU?)")
        self.h = h
        self.lib = lib

    def check(self, st):
        if st != 0:
            raise ObemError(st, self.lib.obem_last_error(self.h).decode())
        return st

    def profile(self, enable: bool = True):
        """Enable or disable per-kernel event timing on this context."""
        self.check(self.lib.obem_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self):
        """{name: (total ms, launches)} since the last read (synchronises)."""
        m = 64
        names = C.create_string_buffer(32 * m)
        ms = (C.c_double * m)()
        cnt = (C.c_int64 * m)()
        n = C.c_int()
        self.check(self.lib.obem_profile_read(self.h, m, names, ms, cnt, C.byref(n)))
        raw = names.raw
        return {raw[32 * k:32 * k + 32].split(b"\0")[0].decode(): (ms[k], cnt[k]) for k in range(n.value)}

    def profile_work(self):
        """(directed terms, pair-once pairs) of the forward pairwise kernels
        since the last read (synchronises)."""
        d, o = C.c_int64(), C.c_int64()
        self.check(self.lib.obem_profile_work(self.h, C.byref(d), C.byref(o)))
        return d.value, o.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.obem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BoundMesh:
    """obem_mesh_bind of a mesh given as GPU tensors: a, b, c (N, 3) float64
    (split into SoA here), kind (N,) int8, eps1 / eps2 (N,) float64."""

    def __init__(self, ctx: Context, a, b, c, kind, eps1=None, eps2=None):
        self.ctx = ctx
        self.n = int(a.shape[0])
        cols = [t[:, k].contiguous() for t in (a, b, c) for k in range(3)]
        self._keep = cols + [kind, eps1, eps2]
        m = Mesh_t(self.n, *[_ptr(t, name="vertex") for t in cols], _ptr(kind, torch.int8, self.n, "kind"),
                   _ptr(eps1, n=self.n, name="eps1"), _ptr(eps2, n=self.n, name="eps2"))
        h = C.c_void_p()
        ctx.check(ctx.lib.obem_mesh_bind(ctx.h, C.byref(m), C.byref(h)))
        self.h = h

    def geometry(self):
        dev = self._keep[0].device
        out = [torch.empty(self.n, dtype=torch.float64, device=dev) for _ in range(5)]
        self.ctx.check(self.ctx.lib.obem_mesh_geometry(self.ctx.h, self.h, *[_ptr(t) for t in out]))
        return dict(area=out[0], centroid=torch.stack(out[1:4], 1), diameter=out[4])

    def release(self):
        if getattr(self, "h", None) and self.ctx.h:
            self.ctx.lib.obem_mesh_release(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def bem_solve_charges(ctx: Context, mesh: BoundMesh, rhs, sigma_out=None, max_refine=3, want_info=True):
    n = mesh.n
    if sigma_out is None:
        sigma_out = torch.empty(n, dtype=torch.float64, device=rhs.device)
    info = SolveInfo_t()
    ctx.check(ctx.lib.bem_solve_charges(ctx.h, mesh.h, _ptr(rhs, n=n, name="rhs"), _ptr(sigma_out, n=n),
                                        max_refine, C.byref(info) if want_info else None))
    return sigma_out, (dict(iterations=info.iterations, backward_error=info.backward_error,
                            residual_inf=info.residual_inf) if want_info else None)


def bem_solve_charges_adjoint(ctx: Context, mesh: BoundMesh, g_sigma, g_rhs=None, max_refine=3, want_info=True):
    """g_rhs = A^{-T} g_sigma (gradient with respect to the left-hand side of
    the collocation system)."""
    n = mesh.n
    if g_rhs is None:
        g_rhs = torch.empty(n, dtype=torch.float64, device=g_sigma.device)
    info = SolveInfo_t()
    ctx.check(ctx.lib.bem_solve_charges_adjoint(ctx.h, mesh.h, _ptr(g_sigma, n=n, name="g_sigma"),
                                                _ptr(g_rhs, n=n), max_refine, C.byref(info) if want_info else None))
    return g_rhs, (dict(iterations=info.iterations, backward_error=info.backward_error,
                        residual_inf=info.residual_inf) if want_info else None)


def _soa(x):
    return [x[:, k].contiguous() for k in range(3)]


def bem_influence(ctx: Context, mesh: BoundMesh, rhs, xs, q, precision=OBEM_MIXED, rhs_out=None, want_bar=False):
    """Left-hand side of the collocation system with the influence of the
    point charges q at xs (n_s, 3) moved onto it (section 3.3.2).  Returns
    rhs_out, or (rhs_out, Vbar, Ebar (n, 3)) with want_bar."""
    n = mesh.n
    n_s = 0 if xs is None else int(xs.shape[0])
    sx = _soa(xs) if n_s else [None] * 3
    if rhs_out is None:
        rhs_out = torch.empty(n, dtype=torch.float64, device=rhs.device)
    vb = eb = None
    if want_bar:
        vb = torch.empty(n, dtype=torch.float64, device=rhs.device)
        eb = [torch.empty(n, dtype=torch.float64, device=rhs.device) for _ in range(3)]
    ctx.check(ctx.lib.bem_influence(ctx.h, mesh.h, n_s, *[_ptr(a, n=n_s) for a in sx],
                                    _ptr(q, n=n_s, name="q") if n_s else None, _ptr(rhs, n=n, name="rhs"),
                                    _ptr(rhs_out, n=n), int(precision), _ptr(vb, n=n),
                                    *([_ptr(a, n=n) for a in eb] if want_bar else [None] * 3)))
    if want_bar:
        return rhs_out, vb, torch.stack(eb, dim=1)
    return rhs_out


def field_eval(ctx: Context, mesh, sigma, xs, q, xt, soft, precision=OBEM_MIXED, tgt_is_src=False, want_v=False,
               out=None):
    """E (n_t, 3) [, V (n_t,)] at targets xt (n_t, 3) from the cells of `mesh`
    (BoundMesh or None) with charge densities sigma and the point charges q at
    xs (n_s, 3) (None for none)."""
    n_t = int(xt.shape[0])
    n_s = 0 if xs is None else int(xs.shape[0])
    tx = _soa(xt)
    sx = _soa(xs) if n_s else [None] * 3
    dev = xt.device
    E = [torch.empty(n_t, dtype=torch.float64, device=dev) for _ in range(3)] if out is None else out
    V = torch.empty(n_t, dtype=torch.float64, device=dev) if want_v else None
    flags = (OBEM_TGT_IS_SRC if tgt_is_src else 0) | (OBEM_WANT_V if want_v else 0)
    ctx.check(ctx.lib.field_eval(ctx.h, mesh.h if mesh is not None else None,
                                 _ptr(sigma) if mesh is not None else None, n_s, *[_ptr(t) for t in sx],
                                 _ptr(q) if n_s else None, n_t, *[_ptr(t) for t in tx], float(soft), int(precision),
                                 flags, *[_ptr(t) for t in E], _ptr(V)))
    Et = torch.stack(E, 1)
    return (Et, V) if want_v else Et


def field_eval_noalloc(ctx: Context, mesh, sigma, xs, q, xt, soft, precision=OBEM_MIXED, tgt_is_src=False,
                       want_v=False, out=None):
    """field_eval through the allocation-free entry point (at most
    OBEM_NOALLOC_MAX_POINTS targets and sources; the library's workspace comes
    from its static scratch array).  Pass `out` (three n_t device tensors) for
    a call that allocates nothing on the Python side either."""
    n_t = int(xt.shape[0])
    n_s = 0 if xs is None else int(xs.shape[0])
    tx = _soa(xt)
    sx = _soa(xs) if n_s else [None] * 3
    dev = xt.device
    E = [torch.empty(n_t, dtype=torch.float64, device=dev) for _ in range(3)] if out is None else out
    V = torch.empty(n_t, dtype=torch.float64, device=dev) if want_v else None
    flags = (OBEM_TGT_IS_SRC if tgt_is_src else 0) | (OBEM_WANT_V if want_v else 0)
    ctx.check(ctx.lib.field_eval_noalloc(ctx.h, mesh.h if mesh is not None else None,
                                         _ptr(sigma) if mesh is not None else None, n_s, *[_ptr(t) for t in sx],
                                         _ptr(q) if n_s else None, n_t, *[_ptr(t) for t in tx], float(soft),
                                         int(precision), flags, *[_ptr(t) for t in E], _ptr(V)))
    Et = torch.stack(E, 1)
    return (Et, V) if want_v else Et


def field_eval_backward(ctx: Context, mesh, sigma, xs, q, xt, soft, gE, precision=OBEM_MIXED, tgt_is_src=False,
                        want_sigma=True, want_t=True, want_s=True):
    """Adjoint of field_eval for L = sum gE . E: returns (g_sigma, g_t (n_t,3),
    g_s (n_s,3)); entries not requested are None."""
    n_t = int(xt.shape[0])
    n_s = 0 if xs is None else int(xs.shape[0])
    dev = xt.device
    tx = _soa(xt)
    sx = _soa(xs) if n_s else [None] * 3
    g = _soa(gE)
    gs = torch.empty(mesh.n, dtype=torch.float64, device=dev) if (mesh is not None and want_sigma) else None
    gt = [torch.empty(n_t, dtype=torch.float64, device=dev) for _ in range(3)] if want_t else [None] * 3
    gsrc = ([torch.empty(n_s, dtype=torch.float64, device=dev) for _ in range(3)]
            if (want_s and n_s and not tgt_is_src) else [None] * 3)
    flags = OBEM_TGT_IS_SRC if tgt_is_src else 0
    ctx.check(ctx.lib.field_eval_backward(ctx.h, mesh.h if mesh is not None else None,
                                          _ptr(sigma) if mesh is not None else None, n_s, *[_ptr(t) for t in sx],
                                          _ptr(q) if n_s else None, n_t, *[_ptr(t) for t in tx], float(soft),
                                          int(precision), flags, *[_ptr(t) for t in g], _ptr(gs),
                                          *[_ptr(t) for t in gt], *[_ptr(t) for t in gsrc]))
    return (gs, torch.stack(gt, 1) if want_t else None,
            torch.stack(gsrc, 1) if gsrc[0] is not None else None)


class Particles:
    """Device SoA particle buffers of a fixed capacity (obem_particles)."""

    def __init__(self, capacity, device, x=None, v=None, species=None, ids=None, next_id=None):
        self.capacity = int(capacity)
        f = dict(dtype=torch.float64, device=device)
        self.cols = [torch.zeros(self.capacity, **f) for _ in range(6)]
        self.species = torch.zeros(self.capacity, dtype=torch.int8, device=device)
        self.id = torch.zeros(self.capacity, dtype=torch.int64, device=device)
        self.n_live = 0
        self.next_id = 0
        if x is not None:
            n = int(x.shape[0])
            if n > self.capacity:
                raise ValueError("more particles than capacity")
            for k in range(3):
                self.cols[k][:n] = x[:, k]
                if v is not None:
                    self.cols[3 + k][:n] = v[:, k]
            self.species[:n] = species
            self.id[:n] = ids if ids is not None else torch.arange(n, device=device)
            self.n_live = n
            self.next_id = int(next_id if next_id is not None else n)

    def struct(self):
        return Particles_t(self.capacity, self.n_live, self.next_id, *[_ptr(t) for t in self.cols],
                           _ptr(self.species, torch.int8), _ptr(self.id, torch.int64))

    def state(self):
        n = self.n_live
        return dict(x=torch.stack([c[:n] for c in self.cols[:3]], 1), v=torch.stack([c[:n] for c in self.cols[3:]], 1),
                    species=self.species[:n].clone(), id=self.id[:n].clone(), next_id=self.next_id)


def gas_struct(gas, device):
    """obem_gas from a workloads.GasTables; returns (struct, keep-alive tensors)."""
    xs = torch.as_tensor(gas.xs, dtype=torch.float64, device=device).contiguous()
    xi = None
    if getattr(gas, "xi", None) is not None:
        xi = torch.as_tensor(gas.xi, dtype=torch.float64, device=device).contiguous()
    g = Gas_t(xs.shape[1], gas.e_min, gas.e_max, _ptr(xs), (C.c_double * 5)(*[float(t) for t in gas.thresholds]),
              gas.density, gas.temperature, gas.m_gas, gas.m_cation, gas.m_anion, gas.ion_xs_iso, gas.ion_xs_back,
              _ptr(xi), float(getattr(gas, "penning_prob", 0.0)), float(getattr(gas, "penning_level", 0.0)))
    return g, (xs, xi)


class FieldMap:
    """Uniform-grid field map (obem_field_map) with its device arrays:
    nodes lo + (i, j, k) h, n = (nx, ny, nz)."""

    def __init__(self, lo, h, n, device="cuda"):
        self.lo, self.h, self.n = tuple(float(v) for v in lo), tuple(float(v) for v in h), tuple(int(v) for v in n)
        m = self.n[0] * self.n[1] * self.n[2]
        self.e = [torch.zeros(m, dtype=torch.float64, device=device) for _ in range(3)]
        self.s = FieldMap_t(self.n[0], self.n[1], self.n[2], (C.c_double * 3)(*self.lo), (C.c_double * 3)(*self.h),
                            *[C.c_void_p(t.data_ptr()) for t in self.e])

    def values(self):
        """(nz, ny, nx, 3) tensor of the node values."""
        nx, ny, nz = self.n
        return torch.stack(self.e, 1).reshape(nz, ny, nx, 3)


def field_map_build(ctx: Context, mesh: BoundMesh, sigma, fmap: FieldMap, precision=OBEM_MIXED):
    ctx.check(ctx.lib.field_map_build(ctx.h, mesh.h, _ptr(sigma, n=mesh.n, name="sigma"), C.byref(fmap.s),
                                      int(precision)))
    return fmap


def field_map_eval(ctx: Context, fmap: FieldMap, x, out=None):
    n = int(x.shape[0])
    xs = _soa(x)
    out = out if out is not None else [torch.empty(n, dtype=torch.float64, device=x.device) for _ in range(3)]
    ctx.check(ctx.lib.field_map_eval(ctx.h, C.byref(fmap.s), n, *[_ptr(a, n=n) for a in xs],
                                     *[_ptr(a, n=n) for a in out]))
    return torch.stack(out, 1)


def induced_current(ctx: Context, x, v, species, mesh: BoundMesh = None, sigma_w=None, fmap: FieldMap = None,
                    precision=OBEM_MIXED, want_terms=False):
    """Shockley-Ramo currents [electrons, cations, anions] (A) induced on the
    electrode whose weighting field is the cell field of sigma_w, or fmap."""
    n = int(x.shape[0])
    xs, vs = _soa(x), _soa(v)
    cur = (C.c_double * 3)()
    terms = torch.empty(n, dtype=torch.float64, device=x.device) if want_terms else None
    ctx.check(ctx.lib.induced_current(ctx.h, mesh.h if mesh is not None else None,
                                      _ptr(sigma_w, n=mesh.n, name="sigma_w") if mesh is not None else None,
                                      C.byref(fmap.s) if fmap is not None else None, n,
                                      *[_ptr(a, n=n) for a in xs], *[_ptr(a, n=n) for a in vs],
                                      _ptr(species, torch.int8, n=n, name="species"), int(precision), cur,
                                      _ptr(terms, n=n)))
    c = [cur[0], cur[1], cur[2]]
    return (c, terms) if want_terms else c


def track_step(ctx: Context, mesh: BoundMesh, parts: Particles, gas_s, params: dict, dd_counts, sigma, rhs0=None,
               fmap: FieldMap = None, field_out=None):
    """One tracking step (obem track_step); field_out (3 x n_live device
    doubles) receives the field at the start positions."""
    p = StepParams_t(params["dt"], params["step"], params["seed"], params["max_coll"], params["max_ion_per_step"],
                     params["ion_v_cap"], (C.c_double * 3)(*params["box_lo"]), (C.c_double * 3)(*params["box_hi"]),
                     params["soft"], params["r_rec"], int(params.get("precision", OBEM_MIXED)),
                     int(params.get("resolve", 0)), int(params.get("influence", 0)),
                     _ptr(rhs0) if rhs0 is not None else None, int(params.get("stepper", 0)),
                     C.cast(C.pointer(fmap.s), C.c_void_p) if fmap is not None else None,
                     _ptr(field_out, n=3 * parts.n_live, name="field_out") if field_out is not None else None)
    ps = parts.struct()
    stats = StepStats_t()
    st = ctx.lib.track_step(ctx.h, mesh.h if mesh is not None else None, C.byref(ps), C.byref(gas_s), C.byref(p),
                            _ptr(dd_counts, torch.int64, name="dd_counts") if dd_counts is not None else None,
                            _ptr(sigma) if sigma is not None else None, C.byref(stats))
    if st not in (0, -6):
        ctx.check(st)
    parts.n_live = ps.n_live
    parts.next_id = ps.next_id
    out = {k: getattr(stats, k) for k, _ in StepStats_t._fields_ if k != "real_collisions"}
    out["real_collisions"] = list(stats.real_collisions)
    out["status"] = st
    return out
