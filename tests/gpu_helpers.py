"""Shared helpers of the GPU parity tests."""
import numpy as np
import torch

from paper_2110_09214_amd import binding as B


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def bind(ctx, mesh):
    return B.BoundMesh(ctx, dev(mesh.a), dev(mesh.b), dev(mesh.c), dev(mesh.kind, torch.int8), dev(mesh.eps1),
                       dev(mesh.eps2))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def synthetic_sigma(mesh, seed=0):
    """Smooth, sign-changing charge densities (C/m^2) of realistic magnitude;
    an input for field parity only (no solve involved)."""
    c = (mesh.a + mesh.b + mesh.c) / 3
    rng = np.random.default_rng(seed)
    k = rng.normal(size=(3, 3)) / 1e-4
    s = np.sin(c @ k[0]) + 0.5 * np.cos(c @ k[1]) + 0.2
    return 1e-6 * np.where(mesh.kind == 0, s, 0.3 * s)
