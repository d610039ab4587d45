"""Seeded synthetic inputs: random SU(3) gauge links, Gaussian and point sources,
random gauge transformations.

This module holds none of the solver's arithmetic.  It only draws inputs, in
the canonical layout shared by the oracle and the GPU library:

  links   U[mu][t][z][y][x][a][b]   complex128   (mu = 0..3 is the paper's mu = 1..4)
  spinor  psi[t][z][y][x][colour][spin] complex128

Recipe for the links (the paper states no gauge ensemble; these stand in for
it): for every link draw X, Y with independent N(0,1) entries, Z = X + iY,
H = (Z + Z^dagger)/2 minus (tr H / 3) * 1, and U = exp(i eps H), an exact SU(3)
matrix.  eps = 0.3 gives a plaquette near 0.6, close to production ensembles;
eps = 0.5 gives a rougher field.  Sources draw Re and Im of every component
from N(0,1).

Random numbers come from torch's generator on the requested device: the CPU
generator for the lattices the oracle handles, the device generator for the
large benchmark lattice (drawn where it is used, in HBM).  A given
(seed, device) pair always yields the same field.
"""
import math

import torch

# links are drawn in chunks of this many 3x3 matrices; part of the recipe
# (changing it changes the field drawn for a seed)
CHUNK = 1 << 20


def lattice_shape(dims):
    """dims = (Lx, Ly, Lz, Lt) -> array shape (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = dims
    return (Lt, Lz, Ly, Lx)


def _matmul3(A, B):
    # batched 3x3 complex product written out as a broadcast sum
    return (A.unsqueeze(-1) * B.unsqueeze(-3)).sum(-2)


def _expm_i(H, eps):
    """exp(i eps H) for a batch of Hermitian 3x3 H: Taylor series of degree 18
    after scaling by 2^-s, then s squarings."""
    A = (1j * eps) * H
    nrm = torch.linalg.matrix_norm(A, ord="fro").max().item() if A.numel() else 0.0
    s = max(0, int(math.ceil(math.log2(max(nrm, 1e-300) / 0.25)))) if nrm > 0.25 else 0
    A = A / (2.0 ** s)
    eye = torch.eye(3, dtype=A.dtype, device=A.device).expand_as(A)
    term = eye.clone()
    out = eye.clone()
    for k in range(1, 19):
        term = _matmul3(term, A) / k
        out = out + term
    for _ in range(s):
        out = _matmul3(out, out)
    return out


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def random_su3(n, eps, seed, device="cpu"):
    """n random SU(3) matrices exp(i eps H), H traceless Hermitian with Gaussian entries."""
    device = torch.device(device)
    g = _gen(seed, device)
    out = torch.empty((n, 3, 3), dtype=torch.complex128, device=device)
    for lo in range(0, n, CHUNK):
        m = min(CHUNK, n - lo)
        X = torch.randn((m, 3, 3), generator=g, dtype=torch.float64, device=device)
        Y = torch.randn((m, 3, 3), generator=g, dtype=torch.float64, device=device)
        Z = torch.complex(X, Y)
        H = 0.5 * (Z + Z.conj().transpose(-1, -2))
        tr = H.diagonal(dim1=-2, dim2=-1).sum(-1) / 3.0
        H = H - tr[:, None, None] * torch.eye(3, dtype=H.dtype, device=device)
        out[lo:lo + m] = _expm_i(H, eps)
        del X, Y, Z, H
    return out


def su3_links(dims, eps, seed, device="cpu"):
    """Gauge links U[4][Lt][Lz][Ly][Lx][3][3] (complex128), links exp(i eps H)."""
    shp = lattice_shape(dims)
    V = math.prod(shp)
    return random_su3(4 * V, eps, seed, device).reshape((4,) + shp + (3, 3))


def unit_links(dims, device="cpu"):
    """The free field U = 1."""
    shp = lattice_shape(dims)
    U = torch.zeros((4,) + shp + (3, 3), dtype=torch.complex128, device=device)
    U[..., 0, 0] = 1
    U[..., 1, 1] = 1
    U[..., 2, 2] = 1
    return U


def gauge_transform(dims, seed, device="cpu"):
    """A random SU(3) matrix per site, Omega[Lt][Lz][Ly][Lx][3][3] (eps = 1)."""
    shp = lattice_shape(dims)
    return random_su3(math.prod(shp), 1.0, seed, device).reshape(shp + (3, 3))


def gaussian_spinor(dims, seed, device="cpu", batch=None):
    """Gaussian complex spinor psi[t][z][y][x][3][4], Re and Im ~ N(0,1)."""
    shp = lattice_shape(dims)
    lead = (batch,) if batch else ()
    g = _gen(seed, torch.device(device))
    re = torch.randn(lead + shp + (3, 4), generator=g, dtype=torch.float64, device=device)
    im = torch.randn(lead + shp + (3, 4), generator=g, dtype=torch.float64, device=device)
    return torch.complex(re, im)


def point_source(dims, colour, spin, site=(0, 0, 0, 0), device="cpu"):
    """delta_{n,site} delta_{colour,c} delta_{spin,s}; site = (x, y, z, t)."""
    shp = lattice_shape(dims)
    psi = torch.zeros(shp + (3, 4), dtype=torch.complex128, device=device)
    x, y, z, t = site
    psi[t, z, y, x, colour, spin] = 1.0
    return psi
