"""Seeded synthetic inputs for the spherical-shell diffusion workloads.

This module is shared by the tests, the benchmark and the smoke check: it
builds meshes, initial fields, boundary data and magnetic fields, and nothing
else.  It holds none of the method's arithmetic (no operator, no time
stepping, no time-step limit); both the GPU path and the CPU oracle receive
the arrays it returns as plain inputs.

The paper's workloads are production MAS relaxations on non-uniform
spherical grids of 3.4 M and 22.8 M points with a dipole-plus-active-region
or an observed radial surface field (Sec. 3.2).  Those runs are not
available, so the fields below stand in for them with the same structure:
a radially stretched shell, a tilted dipole direction field, smooth large
scale variation plus grid-scale noise (the oscillations the time-step limit
is meant to control, Sec. 4.1), and a sharp transition-region-like jump in
temperature for the preconditioner workload.

Index convention everywhere: linear index ((c*nr + i)*nt + j)*np + k with
i the radial, j the colatitude and k the (periodic) longitude cell; the
longitude index is fastest.  Corner arrays are [3][nr+1][nt+1][np] in the
(r, theta, phi) unit-vector basis.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Mesh:
    """Cell-face coordinates of a spherical (r, theta, phi) shell mesh."""

    r_faces: np.ndarray  # (nr+1,) increasing
    t_faces: np.ndarray  # (nt+1,) increasing, 0 .. pi
    p_faces: np.ndarray  # (np+1,) increasing, one full period

    @property
    def shape(self):
        return (len(self.r_faces) - 1, len(self.t_faces) - 1, len(self.p_faces) - 1)

    @property
    def ncells(self):
        nr, nt, np_ = self.shape
        return nr * nt * np_


def shell_mesh(nr: int, nt: int, np_: int, r_in: float = 1.0, r_out: float = 2.5,
               stretch: float = 1.02) -> Mesh:
    """Shell r in [r_in, r_out] with geometric radial stretch; uniform theta on
    [0, pi] and uniform periodic phi on [0, 2 pi)."""
    if nr < 1 or nt < 2 or np_ < 3:
        raise ValueError("need nr>=1, nt>=2, np>=3")
    if stretch == 1.0:
        r = np.linspace(r_in, r_out, nr + 1)
    else:
        dr0 = (r_out - r_in) * (stretch - 1.0) / (stretch ** nr - 1.0)
        r = r_in + dr0 * (stretch ** np.arange(nr + 1) - 1.0) / (stretch - 1.0)
        r[-1] = r_out
    t = np.linspace(0.0, math.pi, nt + 1)
    p = np.linspace(0.0, 2.0 * math.pi, np_ + 1)
    return Mesh(np.ascontiguousarray(r), np.ascontiguousarray(t), np.ascontiguousarray(p))


def _mid(a):
    return 0.5 * (a[1:] + a[:-1])


def cell_centres(mesh: Mesh):
    """Midpoints of the face coordinates, one 1-D array per direction."""
    return _mid(mesh.r_faces), _mid(mesh.t_faces), _mid(mesh.p_faces)


# ----------------------------------------------------------------------------
# smooth seeded random fields
# ----------------------------------------------------------------------------

class SmoothField:
    """S(x) = sum_n a_n cos(k_n . x + psi_n) over 16 random waves with |k|~3,
    x the Cartesian position; smooth across the poles and periodic in phi.
    Normalised by the maximum over the grid it is first evaluated on."""

    NWAVES = 16

    def __init__(self, seed: int):
        self.rng = np.random.default_rng(seed)
        g = self.rng.standard_normal((self.NWAVES, 3))
        self.k = g * math.sqrt(3.0)
        self.a = self.rng.standard_normal(self.NWAVES)
        self.psi = self.rng.uniform(0.0, 2.0 * math.pi, self.NWAVES)

    def raw(self, r, t, p):
        """Unnormalised value on the tensor grid r (n1,), t (n2,), p (n3,)."""
        r = np.asarray(r, float)[:, None, None]
        st, ct = np.sin(t)[None, :, None], np.cos(t)[None, :, None]
        sp, cp = np.sin(p)[None, None, :], np.cos(p)[None, None, :]
        out = np.zeros((r.shape[0], st.shape[1], sp.shape[2]))
        x, y, z = r * st * cp, r * st * sp, r * ct * np.ones_like(cp)
        for n in range(self.NWAVES):
            out += self.a[n] * np.cos(self.k[n, 0] * x + self.k[n, 1] * y
                                      + self.k[n, 2] * z + self.psi[n])
        return out


def _raw_device(sf, r, t, p, torch, device):
    """SmoothField.raw evaluated with torch on `device` (FP64): the same
    waves, for grids too large to build in numpy in reasonable time."""
    f64 = torch.float64
    r = torch.as_tensor(np.asarray(r, float), dtype=f64, device=device)[:, None, None]
    t = torch.as_tensor(np.asarray(t, float), dtype=f64, device=device)
    p = torch.as_tensor(np.asarray(p, float), dtype=f64, device=device)
    st, ct = torch.sin(t)[None, :, None], torch.cos(t)[None, :, None]
    sp, cp = torch.sin(p)[None, None, :], torch.cos(p)[None, None, :]
    x, y, z = r * st * cp, r * st * sp, r * ct * torch.ones_like(cp)
    out = torch.zeros((r.shape[0], st.shape[1], sp.shape[2]), dtype=f64, device=device)
    for n in range(sf.NWAVES):
        out += float(sf.a[n]) * torch.cos(float(sf.k[n, 0]) * x + float(sf.k[n, 1]) * y
                                          + float(sf.k[n, 2]) * z + float(sf.psi[n]))
    return out


def _smooth_on(seed, mesh, extra_r=()):
    """Field at cell centres and at the listed extra radii (for boundary
    data), normalised together so max |S| over the cells is 1; also returns
    the generator so further draws (noise) continue its stream."""
    rc, tc, pc = cell_centres(mesh)
    sf = SmoothField(seed)
    cells = sf.raw(rc, tc, pc)
    scale = 1.0 / np.max(np.abs(cells))
    faces = [sf.raw(np.array([r]), tc, pc)[0] * scale for r in extra_r]
    return cells * scale, faces, sf.rng


def noise(rng, shape):
    return rng.uniform(-1.0, 1.0, shape)


# ----------------------------------------------------------------------------
# magnetic field direction at the cell corners
# ----------------------------------------------------------------------------

def dipole_corners(mesh: Mesh, tilt_deg: float = 10.0):
    """Tilted dipole B ~ (3 (m.rhat) rhat - m)/r^3 at the corners
    (r_faces[ic], t_faces[jc], p_faces[kc]), components in the local
    (rhat, thetahat, phihat) basis.  Shape [3][nr+1][nt+1][np]."""
    R, T, P = mesh.r_faces, mesh.t_faces, mesh.p_faces[:-1]
    a = math.radians(tilt_deg)
    m = np.array([math.sin(a), 0.0, math.cos(a)])
    st, ct = np.sin(T)[None, :, None], np.cos(T)[None, :, None]
    sp, cp = np.sin(P)[None, None, :], np.cos(P)[None, None, :]
    rhat = np.stack(np.broadcast_arrays(st * cp, st * sp, ct * np.ones_like(cp)))
    that = np.stack(np.broadcast_arrays(ct * cp, ct * sp, -st * np.ones_like(cp)))
    phat = np.stack(np.broadcast_arrays(-sp * np.ones_like(st), cp * np.ones_like(st),
                                        np.zeros_like(st * cp)))
    mr = m[0] * rhat[0] + m[1] * rhat[1] + m[2] * rhat[2]          # (1, nt+1, np)
    r3 = (R ** 3)[:, None, None]
    out = np.empty((3, len(R), len(T), len(P)))
    # B . e = (3 (m.rhat)(rhat.e) - m.e) / r^3
    out[0] = (3.0 * mr - mr) / r3
    out[1] = (-(m[0] * that[0] + m[1] * that[1] + m[2] * that[2])) / r3
    out[2] = (-(m[0] * phat[0] + m[1] * phat[1] + m[2] * phat[2])) / r3
    return np.ascontiguousarray(out)


def uniform_direction_corners(mesh: Mesh, comp: int):
    """Unit field along one local basis vector (0 r, 1 theta, 2 phi)."""
    nr, nt, np_ = mesh.shape
    out = np.zeros((3, nr + 1, nt + 1, np_))
    out[comp] = 1.0
    return out


# ----------------------------------------------------------------------------
# workload recipes
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One split parabolic operator's inputs."""
    mesh: Mesh
    op: str                 # "iso7", "viscv" (vector viscosity) or "aligned"
    ncomp: int
    u: np.ndarray           # (ncomp, nr, nt, np) initial field
    ub_in: np.ndarray       # (ncomp, nt, np) Dirichlet data at r_in
    ub_out: np.ndarray      # (ncomp, nt, np) Dirichlet data at r_out
    T0: np.ndarray | None   # (nr, nt, np) lagged temperature, or None
    scale: float            # kappa0 or nu
    expo: float             # 2.5 for Spitzer, 0 for constant
    B: np.ndarray | None    # corner field (aligned operator only)
    bc_in: str = "dirichlet"
    bc_out: str = "dirichlet"
    name: str = ""
    w: np.ndarray | None = None    # (nr, nt, np) weight of F = (1/w) div(...)
    fc: np.ndarray | None = None   # (nr,) radial profile of the coefficient
    Tc: float = 0.0                # low-temperature threshold of f_m (0: none)


def heat_iso(nr=32, nt=32, np_=64, seed=101, stretch=1.02):
    """Scalar heat equation with kappa = kappa0 T^{5/2}, T = 1 + 0.5 S,
    Dirichlet T at both radial boundaries (the small 32x32x64 workload)."""
    mesh = shell_mesh(nr, nt, np_, stretch=stretch)
    s, (s_in, s_out), _ = _smooth_on(seed, mesh, (mesh.r_faces[0], mesh.r_faces[-1]))
    T = 1.0 + 0.5 * s
    return Problem(mesh, "iso7", 1, T[None].copy(), (1.0 + 0.5 * s_in)[None].copy(),
                   (1.0 + 0.5 * s_out)[None].copy(), T.copy(), 1.0, 2.5, None,
                   name=f"heat_iso_{nr}x{nt}x{np_}")


def conduction(nr=151, nt=301, np_=400, seed=201, noise_amp=0.01, stretch=1.02):
    """Field-aligned Spitzer conduction: T = 1 + 0.5 S + 0.01 eta, lagged
    kappa from the same T, tilted-dipole direction field, Dirichlet T."""
    mesh = shell_mesh(nr, nt, np_, stretch=stretch)
    s, (s_in, s_out), rng = _smooth_on(seed, mesh, (mesh.r_faces[0], mesh.r_faces[-1]))
    T = 1.0 + 0.5 * s + noise_amp * noise(rng, s.shape)
    return Problem(mesh, "aligned", 1, T[None].copy(), (1.0 + 0.5 * s_in)[None].copy(),
                   (1.0 + 0.5 * s_out)[None].copy(), T.copy(), 1.0, 2.5,
                   dipole_corners(mesh), name=f"conduction_{nr}x{nt}x{np_}")


def viscosity(nr=151, nt=301, np_=400, seed=202, noise_amp=0.01, nu=1e-3, stretch=1.02,
              vector=False):
    """Artificial viscosity nu Lap v on three velocity components,
    v_c = 0.1 S(seed+c) + 0.01 eta_c, Dirichlet v at both radial boundaries.
    vector: the components are the spherical (v_r, v_theta, v_phi) of one
    vector field (operator "viscv"); else three scalars ("iso7")."""
    mesh = shell_mesh(nr, nt, np_, stretch=stretch)
    u, ui, uo = [], [], []
    for c in range(3):
        s, (s_in, s_out), rng = _smooth_on(seed + c, mesh, (mesh.r_faces[0], mesh.r_faces[-1]))
        u.append(0.1 * s + noise_amp * noise(rng, s.shape))
        ui.append(0.1 * s_in)
        uo.append(0.1 * s_out)
    return Problem(mesh, "viscv" if vector else "iso7", 3, np.stack(u), np.stack(ui),
                   np.stack(uo), None, nu, 0.0, None,
                   name=f"viscosity{'_vec' if vector else ''}_{nr}x{nt}x{np_}")


def viscosity_device(nr, nt, np_, torch, device, seed=202, noise_amp=0.01, nu=1e-3,
                     stretch=1.02, vector=True):
    """viscosity() with the smooth fields evaluated by torch on `device`
    (same waves and noise stream; values equal to rounding).  u, ub_in and
    ub_out are device tensors.  For the largest grids."""
    mesh = shell_mesh(nr, nt, np_, stretch=stretch)
    rc, tc, pc = cell_centres(mesh)
    u = torch.empty((3, nr, nt, np_), dtype=torch.float64, device=device)
    ui = torch.empty((3, nt, np_), dtype=torch.float64, device=device)
    uo = torch.empty_like(ui)
    for c in range(3):
        sf = SmoothField(seed + c)
        cells = _raw_device(sf, rc, tc, pc, torch, device)
        scale = 1.0 / float(cells.abs().max())
        u[c] = 0.1 * scale * cells
        u[c] += noise_amp * torch.as_tensor(noise(sf.rng, cells.shape), device=device)
        ui[c] = 0.1 * scale * _raw_device(sf, [mesh.r_faces[0]], tc, pc, torch, device)[0]
        uo[c] = 0.1 * scale * _raw_device(sf, [mesh.r_faces[-1]], tc, pc, torch, device)[0]
        del cells
    return Problem(mesh, "viscv" if vector else "iso7", 3, u, ui, uo, None, nu, 0.0, None,
                   name=f"viscosity{'_vec' if vector else ''}_{nr}x{nt}x{np_}")


def transition_region(nr=151, nt=301, np_=400, seed=401, i_tr0=12.0, i_amp=3.0,
                      width=5.0, stretch=1.02):
    """Conduction with a sharp transition-region-like jump: T rises from 0.02
    to 1 over `width` radial cells starting at i_tr(theta, phi) =
    i_tr0 + i_amp * S(seed) on the inner surface."""
    mesh = shell_mesh(nr, nt, np_, stretch=stretch)
    _, tc, pc = cell_centres(mesh)
    sf = SmoothField(seed)
    s2 = sf.raw(np.array([mesh.r_faces[0]]), tc, pc)[0]
    s2 = s2 / np.max(np.abs(s2))
    itr = i_tr0 + i_amp * s2
    x = (np.arange(nr)[:, None, None] - itr[None]) / width
    x = np.clip(x, 0.0, 1.0)
    T = 0.02 + 0.98 * (3.0 * x * x - 2.0 * x ** 3)
    ub_in = T[0][None].copy()
    ub_out = T[-1][None].copy()
    return Problem(mesh, "aligned", 1, T[None].copy(), ub_in, ub_out, T.copy(), 1.0, 2.5,
                   dipole_corners(mesh), name=f"transition_{nr}x{nt}x{np_}")


def random_field(shape, seed):
    """Plain N(0,1) array (for symmetry / parity probes)."""
    return np.random.default_rng(seed).standard_normal(shape)
