"""Shared test utilities: small custom workloads and statistical comparisons."""
import numpy as np

from synth import physics as ph
from synth import workloads as W


def slab_workload(layers, e_kev=60.0, n_hist=100_000, seed=11, rayleigh=True, nxy=4,
                  dz=0.5, dxy=0.5):
    """Pencil beam along +z through slabs: layers = [(material, rho, n_vox_z)]."""
    mats = []
    for m, _, _ in layers:
        if m not in mats:
            mats.append(m)
    nz = sum(n for _, _, n in layers)
    mat = np.zeros((nz, nxy, nxy), np.uint8)
    rho = np.zeros((nz, nxy, nxy), np.float32)
    z = 0
    for m, r, n in layers:
        mat[z:z + n] = mats.index(m)
        rho[z:z + n] = r
        z += n
    g = dict(nx=nxy, ny=nxy, nz=nz, dx=dxy, dy=dxy, dz=dz, ox=0.0, oy=0.0, oz=0.0)
    c = nxy * dxy / 2.0
    geo = dict(kind="pencil", src=(c, c, 0.0), dir=(0.0, 0.0, 1.0))
    return W.Workload("slab", g, mat, rho, mats, rayleigh, np.array([e_kev]), 0.0,
                      np.array([1.0]), geo, seed, n_hist)


def random_phantom(shape, n_mat, seed, rayleigh=True, n_hist=10_000, cone=True, dxyz=1.0):
    rng = np.random.default_rng(seed)
    names = ["water", "cortical_bone", "lung", "air", "soft_tissue", "brain"][:n_mat]
    nz, ny, nx = shape
    mat = rng.integers(0, n_mat, shape).astype(np.uint8)
    dens = np.array([ph.MATERIALS[m][0] for m in names])
    rho = (dens[mat] * rng.uniform(0.9, 1.1, shape)).astype(np.float32)
    g = dict(nx=nx, ny=ny, nz=nz, dx=dxyz, dy=dxyz, dz=dxyz,
             ox=-nx * dxyz / 2, oy=-ny * dxyz / 2, oz=-nz * dxyz / 2)
    lo, w = ph.kramers_spectrum(100)
    if cone:
        geo = dict(kind="cone", sad=30.0, iso=(0.0, 0.0, 0.0), a0=-3.0, a1=3.0, b0=-2.0,
                   b1=2.0, nproj=8, arc_deg=360.0, phi0_deg=0.0)
    else:
        geo = dict(kind="pencil", src=(0.1, 0.2, -nz * dxyz), dir=(0.05, 0.02, 1.0))
    return W.Workload("rand", g, mat, rho, names, rayleigh, lo, 1.0, w, geo, seed, n_hist)


def frac_within(d1, s1, d2, s2, mask, k=3.0):
    """Fraction of masked voxels with |d1-d2| <= k sqrt(s1^2 + s2^2)."""
    diff = np.abs(d1[mask] - d2[mask])
    tol = k * np.sqrt(s1[mask] ** 2 + s2[mask] ** 2)
    return float(np.mean(diff <= tol))
