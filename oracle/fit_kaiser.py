"""Kaiser window shape of the off-grid source / receiver interpolation
(TEST INFRASTRUCTURE).

The paper interpolates sources and receivers with Kaiser-windowed sincs but
prints neither the half-width nor the window shape.  Its reference chooses the
shape b for a half-width r so that the interpolator's spectrum stays closest
to 1 up to a maximum wavenumber; this script performs that choice with the
oracle's own spectral-error measure (oracle.interp.spectral_error, a
golden-section search) for r = 4 and kmax = 2 pi / 3 (three points per
wavelength) and prints b; the workload generator stores it as a plain input
literal.

Run: ``python -m oracle.fit_kaiser``
"""
from __future__ import annotations

import numpy as np

from .interp import fit_kaiser_b, spectral_error

RADIUS = 4
KMAX = 2.0 * np.pi / 3.0


def main():
    b = fit_kaiser_b(RADIUS, KMAX)
    print(f"radius {RADIUS}, kmax {KMAX:.6f}: b = {float(b)!r}, spectral error {spectral_error(RADIUS, b, KMAX):.3e}")


if __name__ == "__main__":
    main()
