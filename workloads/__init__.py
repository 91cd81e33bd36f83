"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: voxel material maps, random field
states and source parameters.  It contains none of the method's
arithmetic (no basis functions, no Gram matrices, no solves) and imports
nothing from the oracle or from the GPU package, so both sides can draw
identical inputs from it without sharing any implementation.

The paper's head model comes from an MRI scan that is not available
(section "Incorporating non-regular material data ...": 29 slices of
532x565 pixels with air / tissue / skull classes).  The generators below
stand in for it with the same three-class air / skull-like / tissue-like
structure:

* ``blob_map``   -- three classes from the tertiles of wrapped, Gaussian
  filtered white noise (64^3 voxels in the 64^3 workload);
* ``shell_map``  -- nested ellipsoidal shells, air outside, a thin
  skull-like shell, tissue-like interior, with +-5% per-voxel noise.

All randomness uses ``numpy.random.default_rng(seed)`` (PCG64) and is
evaluated in float64 at voxel centres ``(v + 1/2) / V``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Free-space wave impedance in ohm; converts a conductivity in S/m into
# the non-dimensional form used with c0 = 1, eps = eps_r, mu = mu_r and a
# unit length of L = 1 m:  sigma_nd = Z0 * L * sigma.
Z0_OHM = 376.730313668


def sigma_to_nd(sigma_s_per_m, length_m: float = 1.0):
    """Conductivity in S/m -> non-dimensional conductivity."""
    return np.asarray(sigma_s_per_m, dtype=np.float64) * (Z0_OHM * length_m)


@dataclasses.dataclass
class VoxelMaterial:
    """A voxel material map, arrays shaped (Vz, Vy, Vx), x fastest."""

    eps_r: np.ndarray
    mu_r: np.ndarray
    sigma: np.ndarray  # S/m

    @property
    def shape(self):
        return self.eps_r.shape

    @property
    def sigma_nd(self) -> np.ndarray:
        return sigma_to_nd(self.sigma)


@dataclasses.dataclass
class DipoleSource:
    """Gaussian-modulated sine point dipole.

    amp * sin(2 pi f0 (t - t0)) * exp(-((t - t0) / width)^2), pointing
    along field component ``comp`` (0 = x, 1 = y, 2 = z), located at ``xs``.
    """

    xs: tuple = (0.5, 0.5, 0.5)
    comp: int = 0
    amp: float = 1.0
    f0: float = 2.0
    t0: float = 0.5
    width: float = 0.2


def uniform_material(V: int = 1, eps_r: float = 1.0, mu_r: float = 1.0,
                     sigma: float = 0.0) -> VoxelMaterial:
    shape = (V, V, V)
    return VoxelMaterial(np.full(shape, float(eps_r)), np.full(shape, float(mu_r)),
                         np.full(shape, float(sigma)))


def _voxel_centres(V: int) -> np.ndarray:
    return (np.arange(V, dtype=np.float64) + 0.5) / V


def blob_map(V: int, seed: int, blur_vox: float = 4.0,
             classes=((1.0, 0.0), (15.0, 0.02), (50.0, 0.5))) -> VoxelMaterial:
    """Three-class blob map: tertiles of wrapped Gaussian-filtered noise.

    ``classes`` lists (eps_r, sigma[S/m]) from the lowest to the highest
    tertile; mu_r = 1 everywhere.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((V, V, V))
    g = gaussian_filter(noise, sigma=blur_vox, mode="wrap")
    t1, t2 = np.quantile(g, [1.0 / 3.0, 2.0 / 3.0])
    cls = np.where(g <= t1, 0, np.where(g <= t2, 1, 2))
    eps_tab = np.array([c[0] for c in classes], dtype=np.float64)
    sig_tab = np.array([c[1] for c in classes], dtype=np.float64)
    return VoxelMaterial(eps_tab[cls], np.ones((V, V, V)), sig_tab[cls])


def shell_map(V: int, seed: int) -> VoxelMaterial:
    """Nested ellipsoidal shells: air / skull-like shell / tissue-like core."""
    rng = np.random.default_rng(seed)
    centre = 0.5 + rng.uniform(-0.02, 0.02, size=3)
    outer = np.array([rng.uniform(0.34, 0.40), rng.uniform(0.36, 0.42),
                      rng.uniform(0.34, 0.40)])
    thick = rng.uniform(0.03, 0.05)
    eps_skull = rng.uniform(12.0, 18.0)
    sig_skull = rng.uniform(0.01, 0.05)
    eps_tissue = rng.uniform(40.0, 60.0)
    sig_tissue = rng.uniform(0.3, 0.7)
    inner = outer - thick

    c = _voxel_centres(V)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r_out = ((x - centre[0]) / outer[0]) ** 2 + ((y - centre[1]) / outer[1]) ** 2 \
        + ((z - centre[2]) / outer[2]) ** 2
    r_in = ((x - centre[0]) / inner[0]) ** 2 + ((y - centre[1]) / inner[1]) ** 2 \
        + ((z - centre[2]) / inner[2]) ** 2
    tissue = r_in <= 1.0
    skull = (r_out <= 1.0) & ~tissue
    eps = np.ones((V, V, V))
    sig = np.zeros((V, V, V))
    eps[skull] = eps_skull
    sig[skull] = sig_skull
    eps[tissue] = eps_tissue
    sig[tissue] = sig_tissue
    solid = skull | tissue
    # +-5% uniform per-voxel noise on eps_r and sigma of non-air voxels.
    ne = rng.uniform(-0.05, 0.05, size=(V, V, V))
    ns = rng.uniform(-0.05, 0.05, size=(V, V, V))
    eps = np.where(solid, eps * (1.0 + ne), eps)
    sig = np.where(solid, sig * (1.0 + ns), sig)
    return VoxelMaterial(eps, np.ones((V, V, V)), sig)


def random_fields(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Six random coefficient arrays (E1,E2,E3,H1,H2,H3), shape (6,n,n,n).

    The entries are standard normal; boundary rows are *not* zeroed here.
    """
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((6, n, n, n))


def random_material(V: int, seed: int, eps_range=(1.0, 60.0), mu_range=(0.8, 1.5),
                    sig_range=(0.0, 0.7)) -> VoxelMaterial:
    """Independent per-voxel uniform material (stress test for parity)."""
    rng = np.random.default_rng(seed)
    shape = (V, V, V)
    return VoxelMaterial(rng.uniform(*eps_range, size=shape), rng.uniform(*mu_range, size=shape),
                         rng.uniform(*sig_range, size=shape))


@dataclasses.dataclass
class Workload:
    name: str
    N: int
    p: int
    material: VoxelMaterial
    dt: float
    steps: int
    source: Optional[DipoleSource]
    initial: str  # "mms" (manufactured solution) or "zero"


def make(name: str) -> Workload:
    """The named synthetic workloads.

    * ``mms16``      -- 16^3 elements, p=2, eps=mu=1, sigma=0, manufactured
                        initial state, dt=1e-3, 10 steps.
    * ``blob64``     -- 64^3 p=2 three-class blob map (seed 2), centred
                        dipole, 100 steps of dt=1/128.
    * ``shell128``   -- 128^3 p=3 on a 256^3 shell map (seed 3), dipole at
                        (0.5,0.5,0.04) in air, 200 steps of dt=1/256.
    * ``shell256``   -- 256^3 p=2 on a 256^3 shell map (seed 4), 50 steps
                        of dt=1/512.
    * ``shell32``    -- 32^3 p=2 sub-run on the seed-4 shell map (for the
                        oracle comparison of the 256^3 workload).
    """
    if name == "mms16":
        return Workload(name, 16, 2, uniform_material(1), 1e-3, 10, None, "mms")
    if name == "blob64":
        return Workload(name, 64, 2, blob_map(64, 2), 1.0 / 128, 100,
                        DipoleSource(xs=(0.5, 0.5, 0.5)), "zero")
    if name == "shell128":
        return Workload(name, 128, 3, shell_map(256, 3), 1.0 / 256, 200,
                        DipoleSource(xs=(0.5, 0.5, 0.04)), "zero")
    if name == "shell256":
        return Workload(name, 256, 2, shell_map(256, 4), 1.0 / 512, 50,
                        DipoleSource(xs=(0.5, 0.5, 0.04)), "zero")
    if name == "shell32":
        return Workload(name, 32, 2, shell_map(256, 4), 1.0 / 512, 50,
                        DipoleSource(xs=(0.5, 0.5, 0.04)), "zero")
    raise KeyError(name)
