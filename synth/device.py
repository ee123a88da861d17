"""Large seeded synthetic fields generated on the device with torch (inputs
only, no correlation arithmetic): unit-variance Gaussian noise smoothed by a
periodic box filter along x, y and z, member-major (M, nx*ny*nz).

Used where a field is too large to draw on the host in reasonable time (the
180-member 640 x 704 x 64 ensemble shape). The values depend on torch's
device generator, so they are reproducible per seed on one software stack,
not across stacks; tests that use them compare the library with the oracle
on the very values drawn.
"""
from __future__ import annotations


def smooth_field_torch(M, nx, ny, nz, seed, device="cuda", dtype=None, width=5, chunk=8):
    import torch

    dtype = torch.float32 if dtype is None else dtype
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty((M, nx * ny * nz), dtype=dtype, device=device)
    half = width // 2
    scale = float(width) ** 1.5  # the box mean of width^3 unit normals has variance 1 / width^3
    for m0 in range(0, M, chunk):
        m1 = min(M, m0 + chunk)
        w = torch.randn((m1 - m0, nz, ny, nx), generator=g, device=device, dtype=torch.float32)
        for dim in (3, 2, 1):
            acc = w.clone()
            for s in range(1, half + 1):
                acc += torch.roll(w, s, dims=dim)
                acc += torch.roll(w, -s, dims=dim)
            w = acc / width
            del acc
        out[m0:m1] = (w * scale).reshape(m1 - m0, -1).to(dtype)
        del w
    return out
