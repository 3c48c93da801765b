"""Seeded synthetic inputs for the 3D frequency-domain Helmholtz hot path.

This module only *generates inputs*: velocity models on the computational grid
(absorbing layer included), grid/layer parameters, frequencies and on-node
source/receiver positions.  It contains none of the method's arithmetic (no
operator, solver, misfit or gradient) and imports neither the FP64 oracle nor
the HIP library, so both sides can be fed from the same seeded draws.

Conventions
-----------
* Arrays are C-ordered ``[nx][ny][nz]`` with z (depth) fastest; grid sizes
  always include the absorbing layer of ``npml`` nodes on each of the 6 faces.
* ``m = 1/v**2`` (slowness squared, s^2/m^2) is the model the operator takes;
  ``omega = 2*pi*freq``.
* Velocity is built on the interior and extended into the layer by copying
  the nearest interior value along the face normal (the paper's extension of
  medium parameters into the layer, Preamble, rectangular-domain paragraph).
* Each named workload seeds ``numpy.random.default_rng(170309268 + k)``.

The paper's own field models (public benchmark earth models) are not
reproduced; the layered / random / salt-body models here are synthetic
stand-ins with the sizes, frequencies and velocity ranges of its workloads.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy import ndimage

SEED_BASE = 170309268

# Compact 27-point weights (w1, w2, w3, wm1, wm2, wm3, wm4) used by the
# large-grid workload.  They are plain input numbers here; the oracle-side
# script ``oracle/fit_weights27.py`` reproduces them by a bounded (all
# weights >= 0) least-squares fit of the plane-wave phase velocity over 4-40
# points per wavelength, under w1+w2+w3 = 1 and wm1+6wm2+12wm3+8wm4 = 1
# (max phase-velocity error 0.4 % over that range).
W27_DEFAULT = (
    0.04691172072150582,
    0.8230006108925432,
    0.13008766838595098,
    0.47400425837948634,
    0.08384248576900874,
    0.0019117355828781614,
    1.4904158307892655e-12,
)

# Off-grid source / receiver interpolation: Kaiser-windowed sinc of half-width
# 4 nodes with window shape b, as printed by ``python -m oracle.fit_kaiser``
# (spectral error below 0.9 % up to three points per wavelength).
SINC_RADIUS = 4
SINC_KAISER_B = 4.058383564340161


@dataclass
class Workload:
    """One synthetic Helmholtz problem family (shared m, one or more sources)."""

    name: str
    n: tuple
    h: float
    npml: int
    freq: float
    v: np.ndarray  # velocity on the full grid, float64, shape n
    src: np.ndarray  # int32 (nsrc, 3) on-node source positions
    rec: np.ndarray  # int32 (nrec, 3) on-node receiver positions
    stencil: str = "7pt"  # "7pt" | "27pt"
    dtype: str = "c64"  # "c64" | "c128"
    pml_R: float = 1e-3
    v_true: Optional[np.ndarray] = None  # model that synthesises observed data
    w27: tuple = (1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0)
    solver: dict = field(default_factory=dict)

    @property
    def omega(self) -> float:
        return 2.0 * np.pi * self.freq

    @property
    def m(self) -> np.ndarray:
        return 1.0 / self.v ** 2

    @property
    def m_true(self) -> Optional[np.ndarray]:
        return None if self.v_true is None else 1.0 / self.v_true ** 2

    @property
    def v_ref(self) -> float:
        vv = self.v if self.v_true is None else np.maximum(self.v, self.v_true)
        return float(vv.max())

    @property
    def N(self) -> int:
        return int(np.prod(self.n))


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def interior_shape(n, npml):
    return tuple(int(a) - 2 * npml for a in n)


def edge_extend(v_int: np.ndarray, npml: int) -> np.ndarray:
    """Pad an interior model into the absorbing layer by nearest-value copy."""
    if npml == 0:
        return np.ascontiguousarray(v_int, dtype=np.float64)
    return np.pad(np.asarray(v_int, dtype=np.float64), npml, mode="edge")


def surface_positions(n, npml, counts, depth_index=None):
    """On-node positions of a regular (cx x cy) array on a constant-z plane.

    Node j of c along an axis with n_int interior nodes sits at
    ``npml + floor((j + 1/2) * n_int / c)`` (cell-centred sampling of the
    interior), on plane ``k = depth_index`` (default: first interior plane).
    """
    nx, ny, nz = n
    cx, cy = counts
    k = npml if depth_index is None else depth_index
    nix, niy = nx - 2 * npml, ny - 2 * npml
    xs = npml + np.floor((np.arange(cx) + 0.5) * nix / cx).astype(np.int64)
    ys = npml + np.floor((np.arange(cy) + 0.5) * niy / cy).astype(np.int64)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), np.full(X.size, k)], axis=1)
    return pos.astype(np.int32)


def layered_velocity(shape_int, nlayers, vmin, vmax, smooth_cells):
    """Depth (z) layers with velocities linspace(vmin, vmax), smoothed in z."""
    nz = shape_int[2]
    vals = np.linspace(vmin, vmax, nlayers)
    idx = np.minimum((np.arange(nz) * nlayers) // max(nz, 1), nlayers - 1)
    prof = vals[idx].astype(np.float64)
    if smooth_cells > 0:
        prof = ndimage.gaussian_filter1d(prof, smooth_cells, mode="nearest")
    return np.broadcast_to(prof, shape_int).copy()


def gaussian_random_field(rng, shape, sigma_cells):
    """Unit-std Gaussian field: white noise filtered with a Gaussian kernel."""
    w = rng.standard_normal(shape)
    f = ndimage.gaussian_filter(w, sigma_cells, mode="wrap")
    f = f - f.mean()
    s = f.std()
    return f / (s if s > 0 else 1.0)


def constant_workload(n, h, npml, freq, v0=2000.0, src=None, name="constant",
                      dtype="c128"):
    v = np.full(tuple(n), float(v0))
    if src is None:
        src = np.array([[n[0] // 2, n[1] // 2, n[2] // 2]], dtype=np.int32)
    return Workload(name=name, n=tuple(n), h=h, npml=npml, freq=freq, v=v,
                    src=np.asarray(src, dtype=np.int32),
                    rec=np.zeros((0, 3), np.int32), dtype=dtype)


def layered_random_workload(n, h, npml, freq, nsrc_xy=(4, 4), nrec_xy=(4, 4),
                            seed=0, vmin=1500.0, vmax=4500.0, nlayers=6,
                            pert=0.05, corr_sigma=5.0, smooth_z=2.0,
                            name="layered_random", dtype="c64"):
    """Layered background times (1 + pert*xi), xi a smooth unit-std field."""
    rng = np.random.default_rng(seed)
    si = interior_shape(n, npml)
    vb = layered_velocity(si, nlayers, vmin, vmax, smooth_z)
    xi = gaussian_random_field(rng, si, corr_sigma)
    v = edge_extend(vb * (1.0 + pert * xi), npml)
    return Workload(name=name, n=tuple(n), h=h, npml=npml, freq=freq, v=v,
                    src=surface_positions(n, npml, nsrc_xy),
                    rec=surface_positions(n, npml, nrec_xy), dtype=dtype)


# ----------------------------------------------------------------------------
# the five named workloads
# ----------------------------------------------------------------------------

def c1_small():
    """32^3, h=10 m, layer 8, 5 Hz, 2000 m/s + 10 % Gaussian bump (sigma 4
    cells) at the centre, one centred source, complex128, GMRES(20)."""
    n, npml = (32, 32, 32), 8
    I, J, K = np.meshgrid(*[np.arange(a, dtype=np.float64) for a in n],
                          indexing="ij")
    r2 = (I - 16) ** 2 + (J - 16) ** 2 + (K - 16) ** 2
    v = 2000.0 * (1.0 + 0.10 * np.exp(-r2 / (2 * 4.0 ** 2)))
    v = edge_extend(v[npml:-npml, npml:-npml, npml:-npml], npml)
    return Workload(name="c1_32cube_7pt_c128", n=n, h=10.0, npml=npml,
                    freq=5.0, v=v, src=np.array([[16, 16, 16]], np.int32),
                    rec=np.zeros((0, 3), np.int32), dtype="c128",
                    solver=dict(method="gmres", restart=20, tol=1e-6,
                                max_cycles=200))


def c2_layered(n=(128, 128, 128), nsrc_xy=(4, 4)):
    """128^3, h=12.5 m, layer 15, 8 Hz; 6 depth layers 1500-4500 m/s smoothed
    in z (sigma 2 cells) times (1 + 0.05 xi), xi with correlation length 10
    cells; 16 sources on a 4x4 array on the top interior plane."""
    npml = 15
    w = layered_random_workload(n, 12.5, npml, 8.0, nsrc_xy=nsrc_xy,
                                nrec_xy=(4, 4), seed=SEED_BASE + 2,
                                name="c2_128cube_layered_16src", dtype="c64")
    w.solver = dict(method="fgmres_ml", restart=5, tol=1e-6, max_cycles=30,
                    ks_o=3, ks_i=5, kc_o=3, kc_i=5, levels=3)
    return w


def c3_fwi(n=(96, 96, 96), nsrc_xy=(8, 8), nrec_xy=(48, 48)):
    """96^3 FWI gradient case: h=30 m, 5 Hz, layer 10; true model = 6 smoothed
    layers 1500-4500 m/s with a 1 km-radius sphere at the centre at 0.85x
    velocity (sharp edge); starting model = the layered background smoothed
    with sigma 6 cells; 64 sources (8x8) and 48x48 receivers on the top
    interior plane."""
    npml, h = 10, 30.0
    si = interior_shape(n, npml)
    vb = layered_velocity(si, 6, 1500.0, 4500.0, 2.0)
    c = [(a - 1) / 2.0 for a in si]
    I, J, K = np.meshgrid(*[np.arange(a, dtype=np.float64) for a in si],
                          indexing="ij")
    r = h * np.sqrt((I - c[0]) ** 2 + (J - c[1]) ** 2 + (K - c[2]) ** 2)
    vt = np.where(r <= 1000.0, 0.85 * vb, vb)
    v0 = ndimage.gaussian_filter(vb, 6.0, mode="nearest")
    return Workload(name="c3_96cube_fwi_64src", n=tuple(n), h=h, npml=npml,
                    freq=5.0, v=edge_extend(v0, npml),
                    v_true=edge_extend(vt, npml),
                    src=surface_positions(n, npml, nsrc_xy),
                    rec=surface_positions(n, npml, nrec_xy), dtype="c64",
                    solver=dict(method="fgmres_ml", restart=5, tol=1e-6,
                                max_cycles=30, ks_o=3, ks_i=5, kc_o=3,
                                kc_i=5, levels=3))


def c4_problem_params(count=256, seed=SEED_BASE + 4, lo=48, hi=160):
    """Sizes and frequencies of the uneven batch: each dim ~ U{lo..hi}, redrawn
    until max/min <= 2; f ~ U[3,12] Hz; h = 1500/(8 f) (8 points per
    wavelength at 1500 m/s); layer 8.  Returns a list of dicts (no arrays)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        while True:
            dims = rng.integers(lo, hi + 1, size=3)
            if dims.max() <= 2 * dims.min():
                break
        f = float(rng.uniform(3.0, 12.0))
        out.append(dict(n=tuple(int(d) for d in dims), freq=f,
                        h=1500.0 / (8.0 * f), npml=8,
                        seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def c4_problem(p, sigma_cells=6.0):
    """One member of the uneven batch: smooth random velocity in 1500..4500."""
    rng = np.random.default_rng(p["seed"])
    si = interior_shape(p["n"], p["npml"])
    f = ndimage.gaussian_filter(rng.standard_normal(si).astype(np.float32),
                                sigma_cells, mode="nearest").astype(np.float64)
    lo, hi = f.min(), f.max()
    v = 1500.0 + 3000.0 * (f - lo) / (hi - lo if hi > lo else 1.0)
    n = p["n"]
    npml = p["npml"]
    src = np.array([[n[0] // 2, n[1] // 2, npml + 2]], np.int32)
    return Workload(name="c4_member", n=n, h=p["h"], npml=npml,
                    freq=p["freq"], v=edge_extend(v, npml), src=src,
                    rec=np.zeros((0, 3), np.int32), dtype="c64",
                    solver=dict(method="fgmres_ml", restart=5, tol=1e-6,
                                max_cycles=30, ks_o=3, ks_i=5, kc_o=3,
                                kc_i=5, levels=3))


def c5_salt(n=(320, 320, 160), nsrc_xy=(2, 4), rec_every=1):
    """320x320x160, h=15 m, 10 Hz, layer 10, 27-point stencil: 5 smoothed
    layers 1500-3500 m/s with an ellipsoidal 4500 m/s body (centre at
    (1/2, 1/2, 0.55) of the interior, semi-axes (0.30, 0.25, 0.20) of the
    extent, sharp edge).  The inversion model is that model smoothed with
    sigma 4 cells; observed data come from the sharp model.  8 sources on a
    2x4 array; receivers on every interior node of the top interior plane."""
    npml, h = 10, 15.0
    si = interior_shape(n, npml)
    vb = layered_velocity(si, 5, 1500.0, 3500.0, 2.0)
    g = [np.arange(a, dtype=np.float64) / max(a - 1, 1) for a in si]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    e = ((X - 0.5) / 0.30) ** 2 + ((Y - 0.5) / 0.25) ** 2 + \
        ((Z - 0.55) / 0.20) ** 2
    vt = np.where(e <= 1.0, 4500.0, vb)
    v0 = ndimage.gaussian_filter(vt, 4.0, mode="nearest")
    nr = (si[0] // rec_every, si[1] // rec_every)
    return Workload(name="c5_320x320x160_27pt_8src", n=tuple(n), h=h,
                    npml=npml, freq=10.0, v=edge_extend(v0, npml),
                    v_true=edge_extend(vt, npml),
                    src=surface_positions(n, npml, nsrc_xy),
                    rec=surface_positions(n, npml, nr), stencil="27pt",
                    dtype="c64", w27=W27_DEFAULT,
                    solver=dict(method="fgmres_ml", restart=5, tol=1e-6,
                                max_cycles=30, ks_o=3, ks_i=5, kc_o=3,
                                kc_i=5, levels=3))


def random_complex(rng, shape, dtype=np.complex128):
    """Standard complex normal entries (re, im each unit variance)."""
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return z.astype(dtype)
