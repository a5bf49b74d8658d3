"""Helpers of the GPU tests: run the library through the C ABI and compare with the oracle."""
import numpy as np


def context(mesh, **opts):
    from paper_2108_03991_amd import slim
    ctx = slim.Context(0)
    ctx.set_mesh(mesh.verts, mesh.tris, mesh.obj, mesh.n_obj)
    lay = ctx.build(**opts)
    return ctx, lay


def run_parts(ctx, lay, prec, x):
    import torch
    ne, nt = lay.n_e, lay.n_t
    dev = 'cuda'
    xt = torch.tensor(x, dtype=torch.complex128, device=dev)
    y = torch.zeros_like(xt)
    e = torch.zeros(ne, dtype=torch.complex128, device=dev)
    g = torch.zeros_like(e)
    a = torch.zeros_like(e)
    phi = torch.zeros(nt, dtype=torch.complex128, device=dev)
    ctx.matvec_parts(prec, xt, y, e, g, a, phi)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in dict(y=y, e=e, g=g, a=a, phi=phi).items()}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
