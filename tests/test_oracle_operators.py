"""Pins of the oracle's discrete Helmholtz operators against closed forms,
independent constructions and invariants (CPU only)."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import fwi, krylov


def _rand_grid(rng, n=(10, 11, 12), npml=3, f=5.0, h=10.0):
    g = ops.make_grid(n, h, npml, 2 * np.pi * f, 2600.0)
    m = 1.0 / (2000.0 + 600.0 * rng.random(g.n)) ** 2
    return g, m


def _cplx(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


W27_TEST = (0.55, 0.3, 0.15, 0.62, 0.06, 0.0025, -0.001)


def _w27_valid(w):
    w = list(w)
    w[3] = 1.0 - 6 * w[4] - 12 * w[5] - 8 * w[6]
    w[0] = 1.0 - w[1] - w[2]
    return tuple(w)


def test_apply7_matches_kronecker_assembly():
    """Stencil slicing equals the Kronecker-sum sparse matrix built from the
    1D tridiagonal factors (independent construction), forward and H^H."""
    rng = np.random.default_rng(1)
    g, m = _rand_grid(rng)
    H = ops.assemble7(g, m)
    x, y = _cplx(rng, g.n), _cplx(rng, g.n)
    hx = H @ x.ravel()
    assert np.abs(hx - ops.apply7(g, m, x).ravel()).max() <= 1e-14 * np.abs(hx).max()
    hy = H.conj().T @ y.ravel()
    assert np.abs(hy - ops.apply7(g, m, y, True).ravel()).max() <= 1e-14 * np.abs(hy).max()


def test_laplacian_dirichlet_sine_modes():
    """Without a layer (sigma = 0), the discrete sine modes are eigenvectors
    of the zero-Dirichlet 7-point Laplacian with eigenvalue
    -(4/h^2) sum_a sin^2(pi p_a / (2 (n_a + 1)))."""
    n, h = (9, 10, 12), 7.0
    g = ops.make_grid(n, h, 0, 1.0, 1.0)
    grids = np.meshgrid(*[np.arange(a) for a in n], indexing="ij")
    for p in [(1, 1, 1), (2, 5, 3), (9, 1, 12)]:
        u = np.ones(n)
        lam = 0.0
        for a in range(3):
            u = u * np.sin(np.pi * p[a] * (grids[a] + 1) / (n[a] + 1))
            lam -= 4.0 / h ** 2 * np.sin(np.pi * p[a] / (2 * (n[a] + 1))) ** 2
        Lu = ops.laplacian7(g, u.astype(complex))
        assert np.abs(Lu - lam * u).max() <= 1e-13 * abs(lam)


def _manufactured_error(nn):
    L = 1.0
    h = L / (nn + 1)
    g = ops.make_grid((nn, nn, nn), h, 0, 3.0, 1.0)
    xs = (np.arange(nn) + 1) * h
    X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
    u = np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(np.pi * Z) * np.exp(0.3 * X)
    # exact Laplacian
    ux = np.exp(0.3 * X) * ((0.09 - np.pi ** 2) * np.sin(np.pi * X)
                            + 0.6 * np.pi * np.cos(np.pi * X))
    lap = ux * np.sin(2 * np.pi * Y) * np.sin(np.pi * Z) \
        - (4 * np.pi ** 2 + np.pi ** 2) * u
    m = 0.7 + 0.2 * X * Y
    exact = lap + g.omega ** 2 * m * u
    err = ops.apply7(g, m, u) - exact
    return np.sqrt(np.mean(np.abs(err) ** 2))


def test_apply7_manufactured_second_order():
    """Apply H to a smooth u that vanishes on the Dirichlet boundary: the
    error against the exact Laplacian + omega^2 m u is O(h^2)."""
    e1, e2 = _manufactured_error(15), _manufactured_error(31)
    assert 3.6 < e1 / e2 < 4.4


def _layer_error(n):
    """1D stretched operator (1/s) d/dx ((1/s) du/dx) against the exact
    expression u''/s^2 - s' u'/s^3 for an analytic complex stretch s(x)."""
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    s = lambda t: 1.0 + 0.8j * t ** 2 + 0.1 * t
    ds = lambda t: 1.6j * t + 0.1
    u = np.sin(np.pi * x) * np.exp(x)
    du = np.exp(x) * (np.sin(np.pi * x) + np.pi * np.cos(np.pi * x))
    d2u = np.exp(x) * ((1 - np.pi ** 2) * np.sin(np.pi * x)
                       + 2 * np.pi * np.cos(np.pi * x))
    exact = d2u / s(x) ** 2 - ds(x) * du / s(x) ** 3
    cp, cm = ops.coeffs_from_stretch(h, s(x), s(x + h / 2), s(x - h / 2))
    z = np.zeros(1, complex)
    g = ops.make_grid((n, 1, 1), h, 0, 1.0, 1.0)
    Lu = ops.laplacian7(g, u.reshape(n, 1, 1).astype(complex),
                        coeffs=[(cp, cm), (z, z), (z, z)]).ravel()
    return np.sqrt(np.mean(np.abs(Lu - exact) ** 2))


def test_layer_operator_second_order():
    e1, e2 = _layer_error(63), _layer_error(127)
    assert 3.6 < e1 / e2 < 4.4


def test_layer_profile_shape():
    """sigma vanishes on the interior nodes and grows quadratically to
    sigma_max at the outer grid node; Im(s) > 0 in the layer."""
    g = ops.make_grid((40, 30, 20), 10.0, 6, 2 * np.pi * 4.0, 3000.0)
    smax = 3 * 3000.0 * np.log(1e3) / (2 * 6 * 10.0)
    for a in range(3):
        n = g.n[a]
        i = np.arange(n)
        sig = ops.layer_sigma(g, a, i)
        assert np.all(sig[6:n - 6] == 0.0)
        assert np.isclose(sig[0], smax) and np.isclose(sig[-1], smax)
        assert np.isclose(ops.layer_sigma(g, a, 3.0), smax / 4)
        assert np.all(np.imag(ops.stretch(g, a, i[:6])) > 0)


def _stretched_row_error(scale):
    """RMS error of the oracle's 1D layer rows (axis_coeffs: stretches at the
    node and at the half nodes i +- 1/2) against the continuous operator
    (1/s) d/dx ((1/s) du/dx) = u''/s^2 - s' u'/s^3, with s(x) = 1 + i
    sigma(x)/omega written here in physical coordinates: a layer of fixed
    width Lp = npml h on both ends of [0, 1], sigma = sigma_max (depth/Lp)^2,
    sigma_max = 3 v ln(1/R) / (2 Lp)."""
    npml, nint = 8 * scale, 24 * scale
    n = nint + 2 * npml
    h = 1.0 / (n - 1)
    omega, vref = 2 * np.pi * 3.0, 2.0
    g = ops.make_grid((n, 3, 3), h, npml, omega, vref)
    cp, cm = ops.axis_coeffs(g, 0)
    x = np.arange(n) * h
    Lp = npml * h
    smax = 3 * vref * np.log(1.0 / g.R) / (2 * Lp)
    depth = np.maximum(0.0, np.maximum(Lp - x, x - (1.0 - Lp)))
    sig = smax * (depth / Lp) ** 2
    dsig = np.where(x < Lp, -2 * smax * (Lp - x) / Lp ** 2,
                    np.where(x > 1.0 - Lp, 2 * smax * (x - (1.0 - Lp)) / Lp ** 2, 0.0))
    s, ds = 1 + 1j * sig / omega, 1j * dsig / omega
    k = 2.3
    u = np.exp(1j * k * x) * (1 + x)
    du = np.exp(1j * k * x) * (1j * k * (1 + x) + 1)
    d2u = np.exp(1j * k * x) * (-k * k * (1 + x) + 2j * k)
    exact = d2u / s ** 2 - ds * du / s ** 3
    Lu = cp[1:-1] * (u[2:] - u[1:-1]) - cm[1:-1] * (u[1:-1] - u[:-2])
    return np.sqrt(np.mean(np.abs(Lu - exact[1:-1]) ** 2))


def test_layer_rows_converge_to_the_stretched_operator():
    """The grid's own layer rows converge to the continuous stretched
    operator (Preamble: d/dx -> (1/eta) d/dx).  sigma'' jumps where the layer
    starts, so the RMS order is about 1.5; stretches taken at the nodes
    i +- 1 or i instead of the half nodes leave an O(1) error (about 15 here)."""
    e = [_stretched_row_error(s) for s in (2, 4, 8)]
    assert e[2] < 0.05
    assert e[0] / e[1] > 2.5 and e[1] / e[2] > 2.5


def test_layer_reflection_coefficient_and_coarse_rediscretisation():
    """(i) The damping profile integrates to the nominal normal-incidence
    reflection: exp(-(2/v_ref) int_0^Lp sigma dx) = R (continuous layer
    theory; pins sigma_max and the quadratic profile in fine-grid units).
    (ii) The coarse level of a grid (coarse node I at fine node 2I, spacing
    2h, profile at fine coordinates 2I and 2I +- 1) has the layer rows of the
    same physical problem discretised directly at spacing 2h."""
    from oracle import mlgmres  # noqa: F401  (coarsening lives with the hierarchy)
    g = ops.make_grid((61, 41, 33), 12.5, 10, 2 * np.pi * 6.0, 3200.0)
    t = np.linspace(0.0, 10.0, 200001)
    integral = np.trapezoid(ops.layer_sigma(g, 0, t), t) * g.h
    assert abs(np.exp(-2.0 * integral / g.v_ref) - g.R) <= 1e-8
    gc = ops.coarsen(g)
    direct = ops.make_grid(gc.n, 2 * g.h, 5, g.omega, g.v_ref)
    for a in range(3):
        for c_coarse, c_direct in zip(ops.axis_coeffs(gc, a), ops.axis_coeffs(direct, a)):
            assert np.allclose(c_coarse, c_direct, rtol=1e-13, atol=0.0)


def test_adjoint_identity_7pt():
    """<H x, y> = <x, H^H y> (paper's adjoint test), random complex x, y, with
    and without zeroing in the layer and on the original boundary."""
    rng = np.random.default_rng(2)
    g, m = _rand_grid(rng, n=(14, 13, 15), npml=4)
    for zero in (False, True):
        x, y = _cplx(rng, g.n), _cplx(rng, g.n)
        if zero:
            k = g.npml + 1
            for v in (x, y):
                mask = np.zeros(g.n, bool)
                mask[k:-k, k:-k, k:-k] = True
                v[~mask] = 0
        hx = ops.apply7(g, m, x)
        hy = ops.apply7(g, m, y, adjoint=True)
        a, b = np.vdot(y, hx), np.vdot(hy, x)
        assert abs(a - b) / (np.linalg.norm(hx) * np.linalg.norm(y)) <= 1e-12


def test_apply27_matches_assembly_and_adjoint():
    rng = np.random.default_rng(3)
    g, m = _rand_grid(rng, n=(11, 10, 12), npml=3)
    w = _w27_valid(W27_TEST)
    H = ops.assemble27(g, m, w)
    x, y = _cplx(rng, g.n), _cplx(rng, g.n)
    hx = H @ x.ravel()
    assert np.abs(hx - ops.apply27(g, m, x, w).ravel()).max() <= 1e-14 * np.abs(hx).max()
    hy = H.conj().T @ y.ravel()
    assert np.abs(hy - ops.apply27(g, m, y, w, True).ravel()).max() <= 1e-14 * np.abs(hy).max()
    a = np.vdot(y, ops.apply27(g, m, x, w))
    b = np.vdot(ops.apply27(g, m, y, w, True), x)
    assert abs(a - b) / (np.linalg.norm(hx) * np.linalg.norm(y)) <= 1e-12


def test_interior27_mask_by_brute_force():
    """Rows that take the compact 27-point Laplacian: the node and all 26
    neighbours lie where no axis is damped (sigma = 0), checked node by node
    and offset by offset on a small grid (on a coarse level too).  On those
    rows every 7-point layer coefficient is the undamped 1/h^2."""
    g0 = ops.make_grid((13, 11, 12), 10.0, 3, 2 * np.pi * 5.0, 2600.0)
    for g in (g0, ops.coarsen(ops.make_grid((25, 21, 23), 5.0, 6, 2 * np.pi * 5.0, 2600.0))):
        mask = ops.interior27_mask(g)
        brute = np.zeros(g.n, bool)
        for p in np.ndindex(*g.n):
            ok = True
            for d in ops.offsets27():
                for a in range(3):
                    if ops.layer_sigma(g, a, p[a] + d[a]) != 0.0:
                        ok = False
            brute[p] = ok
        assert np.array_equal(mask, brute)
        assert brute.any() and not brute.all()
        coeffs = [ops.axis_coeffs(g, a) for a in range(3)]
        for p in zip(*np.nonzero(mask)):
            for a in range(3):
                for c in coeffs[a]:
                    assert c[p[a]] == 1.0 / g.h ** 2


def test_apply27_reduces_to_7pt():
    """w = (1,0,0), wm = (1,0,0,0) gives exactly the 7-point operator."""
    rng = np.random.default_rng(4)
    g, m = _rand_grid(rng)
    x = _cplx(rng, g.n)
    for adj in (False, True):
        a = ops.apply27(g, m, x, (1, 0, 0, 1, 0, 0, 0), adj)
        b = ops.apply7(g, m, x, adj)
        assert np.abs(a - b).max() <= 1e-15 * np.abs(b).max()


def test_apply27_plane_wave_symbol():
    """On rows whose whole 27-point neighbourhood is interior, H exp(i k.x) =
    symbol(k) exp(i k.x), the closed-form cosine sum."""
    n, h, npml = (14, 14, 14), 12.0, 3
    g = ops.make_grid(n, h, npml, 2 * np.pi * 6.0, 2500.0)
    m0 = 1 / 2300.0 ** 2
    m = np.full(n, m0)
    w = _w27_valid(W27_TEST)
    kv = (0.11, -0.07, 0.05)
    X = np.meshgrid(*[np.arange(a) * h for a in n], indexing="ij")
    u = np.exp(1j * (kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2]))
    Hu = ops.apply27(g, m, u, w)
    sym = ops.symbol27(kv, h, w, g.omega ** 2 * m0)
    inner = ops.interior27_mask(g)
    inner[[0, -1], :, :] = False
    inner[:, [0, -1], :] = False
    inner[:, :, [0, -1]] = False
    # rows whose mass neighbourhood is also inside the grid
    assert inner.sum() > 0
    assert np.abs(Hu[inner] - sym * u[inner]).max() <= 1e-12 * abs(sym)


def test_laplacian27_exact_on_quadratics():
    """Every L_i is exact on quadratics, so L27 = w1 L1 + w2 L2 + w3 L3 with
    w1+w2+w3 = 1 reproduces the exact Laplacian of x^2, yz, ... at interior
    rows; the 27-point mass weights sum to one (A 1 = 1 in the interior)."""
    n, h, npml = (12, 12, 12), 3.0, 2
    g = ops.make_grid(n, h, npml, 1.0, 1.0)
    w = _w27_valid(W27_TEST)
    X = np.meshgrid(*[np.arange(a) * h for a in n], indexing="ij")
    inner = ops.interior27_mask(g)
    lw = ops.laplacian27_weights(w, h)
    for u, lap in [(X[0] ** 2, 2.0), (X[1] * X[2], 0.0),
                   (X[0] ** 2 + 3 * X[2] ** 2 - X[0] * X[1], 8.0)]:
        Lu = ops.stencil27(u.astype(complex), lw)
        assert np.abs(Lu[inner] - lap).max() <= 1e-9 * (1 + np.abs(u).max() / h ** 2)
    A1 = ops.stencil27(np.ones(n, complex), ops.mass27_weights(w))
    assert np.abs(A1[1:-1, 1:-1, 1:-1] - 1.0).max() <= 1e-14


def _green_error(n, npml, ppw, tol=1e-9):
    v0, f = 2000.0, 5.0
    h = v0 / (f * ppw)
    g = ops.make_grid((n, n, n), h, npml, 2 * np.pi * f, v0)
    m = np.full(g.n, 1 / v0 ** 2)
    c = n // 2
    q = fwi.point_source(g, (c, c, c))
    u, info = krylov.gmres(lambda v: ops.apply7(g, m, v), q, k=30,
                           cycles=2000, tol=tol)
    assert info["relres"] <= tol
    I, J, K = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    r = h * np.sqrt((I - c) ** 2 + (J - c) ** 2 + (K - c) ** 2)
    kap = 2 * np.pi * f / v0
    G = -np.exp(1j * kap * r) / (4 * np.pi * np.maximum(r, 1e-30))
    rmax = (n - 2 * npml) // 2 - 1
    sel = (r >= 4 * h) & (r <= rmax * h)
    return np.linalg.norm((u - G)[sel]) / np.linalg.norm(G[sel])


@pytest.mark.slow
def test_green_function_3d_with_layer():
    """Constant velocity, on-node unit source q = e_s/h^3: the solution
    approaches -exp(i kappa r)/(4 pi r) in an annulus 4 <= r/h <= r_max
    (paper's 3D analytic comparison, Validation section; the sign follows
    from (Laplacian + kappa^2) G = delta with the outgoing condition).  The
    same interior with no absorbing layer (Dirichlet walls reflect) is far
    off, and the wrong-sign solution is off by ~200 %."""
    e_layer = _green_error(32, 6, 24)
    assert e_layer < 0.02
    e_wall = _green_error(20, 0, 24)
    assert e_wall > 5 * e_layer


def test_default_27pt_weights_constraints_and_dispersion():
    """The 27-point weights of the large-grid workload satisfy both sum
    constraints and keep the interior phase-velocity error below 0.5 % from
    4 to 40 points per wavelength (all directions of one octant)."""
    import workloads
    from oracle.fit_weights27 import phase_velocity_error
    w = workloads.W27_DEFAULT
    assert abs(w[0] + w[1] + w[2] - 1.0) <= 1e-12
    assert abs(w[3] + 6 * w[4] + 12 * w[5] + 8 * w[6] - 1.0) <= 1e-12
    err = phase_velocity_error(w, np.linspace(1 / 40, 1 / 4, 13),
                               np.linspace(0, np.pi / 2, 5),
                               np.linspace(0, np.pi / 4, 5))
    assert np.abs(err).max() < 5e-3
    # the plain 7-point scheme is much worse at 4 points per wavelength
    err7 = phase_velocity_error((1, 0, 0, 1, 0, 0, 0), [0.25], [0.0], [0.0])
    assert abs(err7[0]) > 0.05
