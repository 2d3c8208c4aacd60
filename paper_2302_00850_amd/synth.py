"""Seeded synthetic inputs for the Wilson-Dirac hot path.

This module only *draws* inputs: SU(3) gauge links, Gaussian and point
sources, random gauge transformations.  It holds none of the operator or
solver arithmetic, so it can feed both the FP64 CPU oracle and the HIP path.

Canonical layouts (complex128, row-major):
  gauge   U[Lt][Lz][Ly][Lx][mu][a][b]        mu = 0,1,2,3 = x,y,z,t
  spinor  psi[nrhs][Lt][Lz][Ly][Lx][spin][colour]

Recipe (the lattice workloads of the paper's CG benchmark are unspecified;
these stand in for them):
  * Haar SU(3): a 3x3 matrix of complex Gaussians (Re, Im ~ N(0,1)), QR with
    a positive real diagonal of R (the Mezzadri phase fix; Gram-Schmidt on
    the columns produces exactly that factor), then divided by the principal
    cube root of its determinant.
  * mixed link U = proj_SU3(1 + mix*(U_haar - 1)), proj_SU3 = polar factor
    (Newton iteration W <- (W + W^-H)/2), determinant phase removed with the
    principal cube root, then rows re-orthonormalised with row 2 rebuilt as
    conj(row0 x row1) so the stored link is SU(3) to rounding.
  * draw order: for each timeslice t, the Re parts of all that slice's
    Haar seeds (z, y, x, mu, 3, 3 order) then their Im parts; afterwards the
    sources.  One numpy Generator (PCG64, ``default_rng(seed)``) per field set.
  * complex Gaussian spinor entries: Re, Im ~ N(0, 1/2), so E|z|^2 = 1.
"""
from __future__ import annotations

import numpy as np
import torch

C128 = torch.complex128


def _vdot(a, b):
    """sum_i conj(a_i) b_i over the last axis."""
    return (a.conj() * b).sum(-1)


def _normalise(v):
    return v / torch.sqrt((v.real ** 2 + v.imag ** 2).sum(-1, keepdim=True))


def _cross(a, b):
    a0, a1, a2 = a[..., 0], a[..., 1], a[..., 2]
    b0, b1, b2 = b[..., 0], b[..., 1], b[..., 2]
    return torch.stack([a1 * b2 - a2 * b1, a2 * b0 - a0 * b2, a0 * b1 - a1 * b0], -1)


def _det3(m):
    return (m[..., 0, :] * _cross(m[..., 1, :], m[..., 2, :])).sum(-1)


def _inv3(m):
    """Inverse of a stack of 3x3 complex matrices by the adjugate."""
    r0, r1, r2 = m[..., 0, :], m[..., 1, :], m[..., 2, :]
    # columns of the adjugate are the cross products of row pairs
    adj_t = torch.stack([_cross(r1, r2), _cross(r2, r0), _cross(r0, r1)], -2)
    det = (r0 * adj_t[..., 0, :]).sum(-1)
    return adj_t.transpose(-1, -2) / det[..., None, None]


def _remove_det_phase(m):
    det = _det3(m)
    ph = torch.exp(-1j * torch.angle(det) / 3.0)
    return m * ph[..., None, None]


def haar_su3(z: torch.Tensor) -> torch.Tensor:
    """Map complex Gaussian 3x3 matrices z to Haar-distributed SU(3)."""
    c0, c1, c2 = z[..., :, 0], z[..., :, 1], z[..., :, 2]
    q0 = _normalise(c0)
    c1 = c1 - q0 * _vdot(q0, c1)[..., None]
    q1 = _normalise(c1)
    c2 = c2 - q0 * _vdot(q0, c2)[..., None] - q1 * _vdot(q1, c2)[..., None]
    q2 = _normalise(c2)
    q = torch.stack([q0, q1, q2], -1)
    return _remove_det_phase(q)


def reunitarise_rows(w: torch.Tensor) -> torch.Tensor:
    """Gram-Schmidt on rows 0 and 1; row 2 = conj(row0 x row1)."""
    r0 = _normalise(w[..., 0, :])
    r1 = w[..., 1, :]
    r1 = _normalise(r1 - r0 * _vdot(r0, r1)[..., None])
    r2 = _cross(r0, r1).conj()
    return torch.stack([r0, r1, r2], -2)


def proj_su3(w: torch.Tensor, newton_steps: int = 10) -> torch.Tensor:
    """Nearest-unitary (polar) projection, det phase removed, rows re-orthonormalised."""
    for _ in range(newton_steps):
        w = 0.5 * (w + _inv3(w).conj().transpose(-1, -2))
    return reunitarise_rows(_remove_det_phase(w))


def _check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or min(dims) <= 0:
        raise ValueError(f"dims must be four positive ints (Lx,Ly,Lz,Lt), got {dims}")
    return dims


class Synth:
    """One seeded stream of synthetic fields.

    rng="numpy" (default): numpy PCG64 draws, identical on every machine.
    rng="torch": draws from a torch.Generator on `device` (fast for 10^7-site
    lattices; reproducible for a given device type, not across them).
    """

    def __init__(self, seed: int = 0, device="cpu", rng: str = "numpy"):
        self.device = torch.device(device)
        self.kind = rng
        if rng == "numpy":
            self.rng = np.random.default_rng(seed)
        elif rng == "torch":
            self.gen = torch.Generator(device=self.device)
            self.gen.manual_seed(seed)
        else:
            raise ValueError("rng must be 'numpy' or 'torch'")

    def _complex_normal(self, shape, std):
        if self.kind == "torch":
            re = torch.randn(shape, generator=self.gen, dtype=torch.float64, device=self.device)
            im = torch.randn(shape, generator=self.gen, dtype=torch.float64, device=self.device)
            return torch.complex(re, im) * std
        re = self.rng.standard_normal(shape)
        im = self.rng.standard_normal(shape)
        z = torch.complex(torch.from_numpy(re), torch.from_numpy(im)).to(self.device)
        return z * std

    def gauge(self, dims, mix: float = 0.3) -> torch.Tensor:
        """U = proj_SU3(1 + mix (U_haar - 1)), shape (Lt,Lz,Ly,Lx,4,3,3)."""
        lx, ly, lz, lt = _check_dims(dims)
        out = torch.empty((lt, lz, ly, lx, 4, 3, 3), dtype=C128, device=self.device)
        eye = torch.eye(3, dtype=C128, device=self.device)
        for t in range(lt):
            z = self._complex_normal((lz, ly, lx, 4, 3, 3), 1.0)
            u = haar_su3(z)
            out[t] = proj_su3(eye + mix * (u - eye))
        return out

    def haar_field(self, dims) -> torch.Tensor:
        """One Haar SU(3) matrix per site, shape (Lt,Lz,Ly,Lx,3,3) (gauge transforms)."""
        lx, ly, lz, lt = _check_dims(dims)
        z = self._complex_normal((lt, lz, ly, lx, 3, 3), 1.0)
        return haar_su3(z)

    def gaussian_spinor(self, dims, nrhs: int = 1) -> torch.Tensor:
        """Complex Gaussian spinors with E|z|^2 = 1, shape (nrhs,Lt,Lz,Ly,Lx,4,3)."""
        lx, ly, lz, lt = _check_dims(dims)
        return self._complex_normal((nrhs, lt, lz, ly, lx, 4, 3), np.sqrt(0.5))


    def momenta(self, dims) -> torch.Tensor:
        """Traceless Hermitian Gaussian matrices per link with density exp(-Tr P^2 / 2),
        shape (Lt,Lz,Ly,Lx,4,3,3): diagonal entries of variance 1, off-diagonal real and
        imaginary parts of variance 1/2, then the trace removed."""
        lx, ly, lz, lt = _check_dims(dims)
        z = self._complex_normal((lt, lz, ly, lx, 4, 3, 3), np.sqrt(0.5))
        h = (z + z.conj().transpose(-1, -2)) * np.sqrt(0.5)
        tr = torch.diagonal(h, dim1=-2, dim2=-1).sum(-1)
        eye = torch.eye(3, dtype=C128, device=self.device)
        return h - tr[..., None, None] / 3 * eye


def unit_gauge(dims, device="cpu") -> torch.Tensor:
    lx, ly, lz, lt = _check_dims(dims)
    u = torch.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=C128, device=device)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def point_sources(dims, device="cpu") -> torch.Tensor:
    """The 12 spin-colour point sources at the origin; source q = 3*spin + colour."""
    lx, ly, lz, lt = _check_dims(dims)
    b = torch.zeros((12, lt, lz, ly, lx, 4, 3), dtype=C128, device=device)
    for q in range(12):
        b[q, 0, 0, 0, 0, q // 3, q % 3] = 1.0
    return b


def bc_phases(theta=(0.0, 0.0, 0.0, np.pi)) -> np.ndarray:
    """Boundary phases e^{i theta_mu} as a (4, 2) float64 array of (re, im)."""
    th = np.asarray(theta, dtype=np.float64)
    ph = np.stack([np.cos(th), np.sin(th)], -1)
    ph[np.abs(ph) < 1e-15] = 0.0  # theta = pi gives exactly (-1, 0)
    return ph
