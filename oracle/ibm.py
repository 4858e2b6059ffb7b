"""Immersed-boundary coupling, FP64 (test infrastructure only).

The paper cites the immersed-boundary method as prior art (Sec. I) without
giving a kernel; the delta here is Peskin's published 4-point function
  phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8        |r| <= 1
           (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8       1 <= |r| <= 2
           0                                              otherwise,
with the 3D weight the product over the three axes.  The stencil of a
point X covers lattice nodes floor(X_d) - 1 + k, k = 0..3, wrapped
periodically.

Pins (tests/test_oracle_ibm.py): partition of unity, zero first moment and
sum of squares 3/8 for any offset; linear fields interpolated exactly;
spreading conserves the total; spreading and interpolation are adjoint.
"""

import torch

DT = torch.float64


def peskin4(r):
    """Peskin 4-point kernel, elementwise."""
    a = r.abs()
    near = a <= 1.0
    mid = (a > 1.0) & (a <= 2.0)
    one = torch.ones_like(a)
    # each square root only sees the range where its branch is used, so the
    # unselected branch never produces an infinite derivative under autograd
    s_in = torch.sqrt(torch.where(near, 1.0 + 4.0 * a - 4.0 * a * a, one))
    s_out = torch.sqrt(torch.where(mid, -7.0 + 12.0 * a - 4.0 * a * a, one))
    inner = (3.0 - 2.0 * a + s_in) / 8.0
    outer = (5.0 - 2.0 * a - s_out) / 8.0
    return torch.where(near, inner, torch.where(mid, outer, torch.zeros_like(a)))


def stencil(X, dims):
    """Stencil indices and 1D weights of points X [N, 3] (x, y, z) on a
    periodic lattice of size dims = (nx, ny, nz).

    Returns (idx [3][N, 4] int64 wrapped node indices per axis,
             wts [3][N, 4] float64 weights per axis,
             base [N, 3] int64 unwrapped stencil base floor(X) - 1)."""
    fl = torch.floor(X)
    base = fl.to(torch.int64) - 1
    r = X - fl
    idx, wts = [], []
    k = torch.arange(4, dtype=torch.int64)
    for d in range(3):
        n = int(dims[d])
        i = base[:, d:d + 1] + k.unsqueeze(0)
        idx.append(torch.remainder(i, n))
        dist = r[:, d:d + 1] + 1.0 - k.to(DT).unsqueeze(0)
        wts.append(peskin4(dist))
    return idx, wts, base


def weights3(wts):
    """Tensor-product weights [N, 4(z), 4(y), 4(x)]."""
    wx, wy, wz = wts
    return wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]


def interpolate(field, X):
    """U(X_b) = sum_x field(x) delta4(x - X_b).  field: [k, z, y, x];
    returns [N, k]."""
    nz, ny, nx = field.shape[-3:]
    idx, wts, _ = stencil(X, (nx, ny, nz))
    ix, iy, iz = idx
    g = field[:, iz[:, :, None, None], iy[:, None, :, None], ix[:, None, None, :]]
    w = weights3(wts)
    return (g * w.unsqueeze(0)).sum((-1, -2, -3)).transpose(0, 1)


def spread(values, X, dims):
    """field(x) = sum_b values_b delta4(x - X_b).  values: [N, k];
    returns [k, z, y, x] for dims = (nx, ny, nz)."""
    nx, ny, nz = (int(d) for d in dims)
    idx, wts, _ = stencil(X, (nx, ny, nz))
    ix, iy, iz = idx
    w = weights3(wts)                                     # [N,4,4,4]
    flat = (iz[:, :, None, None] * ny + iy[:, None, :, None]) * nx + ix[:, None, None, :]
    flat = flat.reshape(-1)
    k = values.shape[1]
    contrib = (values[:, :, None, None, None] * w[:, None]).permute(1, 0, 2, 3, 4).reshape(k, -1)
    out = torch.zeros(k, nx * ny * nz, dtype=values.dtype)
    out = out.index_add(1, flat, contrib)
    return out.view(k, nz, ny, nx)


def tile_of(X, dims, tile=8):
    """Index of the tile (edge `tile`) holding the node floor(X), wrapped
    periodically; tiles are numbered x fastest."""
    nx, ny, nz = (int(d) for d in dims)
    fl = torch.floor(X).to(torch.int64)
    cx = torch.remainder(fl[:, 0], nx) // tile
    cy = torch.remainder(fl[:, 1], ny) // tile
    cz = torch.remainder(fl[:, 2], nz) // tile
    tx = (nx + tile - 1) // tile
    ty = (ny + tile - 1) // tile
    return (cz * ty + cy) * tx + cx
