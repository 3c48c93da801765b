"""Least-squares fit of compact 27-point stencil weights (TEST INFRASTRUCTURE).

The paper uses the compact 27-point mixed-grid stencil but does not print its
weights.  That stencil's own reference chooses them by minimising the
phase-velocity error of plane waves over a range of grid sampling and
propagation angles, under the consistency constraints w1 + w2 + w3 = 1 and
wm1 + 6 wm2 + 12 wm3 + 8 wm4 = 1.  Here all weights are also kept
non-negative (bounded fit), which keeps the mass matrix diagonally
dominant.  This script performs such a fit with the oracle's closed-form
plane-wave symbol and prints the seven numbers; the workload generator
stores the result as plain input literals.

Normalised phase velocity of the interior row for wavenumber k = |k| n:
``v_num / v = sqrt(-S(k) / W(k)) / (|k| h)`` in units where m h^2 = 1, with
S the Laplacian symbol and W the mass symbol; the fit samples 1/G in
[1/40, 1/4] (G = points per wavelength) and directions over one octant.

Run: ``python -m oracle.fit_weights27``
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import least_squares

from .operators import symbol27


def _unpack(p):
    w1, w2, wm2, wm3, wm4 = p
    return (w1, w2, 1.0 - w1 - w2, 1.0 - 6 * wm2 - 12 * wm3 - 8 * wm4,
            wm2, wm3, wm4)


def phase_velocity_error(w27, inv_g, theta, phi):
    h = 1.0
    err = []
    for ig in inv_g:
        kmag = 2 * np.pi * ig / h
        for th in theta:
            for ph in phi:
                kv = (kmag * np.sin(th) * np.cos(ph),
                      kmag * np.sin(th) * np.sin(ph), kmag * np.cos(th))
                lap = symbol27(kv, h, w27, 0.0)
                mass = symbol27(kv, h, w27, 1.0) - lap
                ratio = -lap / mass
                vn = np.sqrt(max(ratio, 0.0)) / kmag
                err.append(vn - 1.0)
    return np.array(err)


def fit(n_g=25, n_ang=7):
    inv_g = np.linspace(1.0 / 40.0, 1.0 / 4.0, n_g)
    theta = np.linspace(0.0, np.pi / 2, n_ang)
    phi = np.linspace(0.0, np.pi / 4, n_ang)
    p0 = np.array([0.6, 0.3, 0.05, 0.002, 0.0])
    res = least_squares(lambda p: phase_velocity_error(_unpack(p), inv_g,
                                                       theta, phi),
                        p0, bounds=(np.zeros(5), np.array([1.0, 1.0, 0.1, 0.1, 0.1])),
                        xtol=1e-14, ftol=1e-14, gtol=1e-14)
    w = _unpack(res.x)
    return w, float(np.abs(res.fun).max())


if __name__ == "__main__":
    w, emax = fit()
    print("w27 =", tuple(float(v) for v in w))
    print("max |v_num/v - 1| over the fit range:", emax)
