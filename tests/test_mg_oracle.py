"""Pins of the multigrid oracle (section 2.7 and the divergence cleaning of
section 2.2) against closed forms, exact discrete solutions and the
mathematics of the operators, independent of the oracle's own code."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import mg

CART, CYL, SPH = mg.CART, mg.CYL, mg.SPH
D, N, PER, ROB = mg.DIRICHLET, mg.NEUMANN, mg.PERIODIC, mg.ROBIN


def prob(ndim, coord, n, xmin, xmax, bc, **kw):
    n = list(n) + [1] * (3 - len(n))
    xmin, xmax = list(xmin) + [0] * (3 - len(xmin)), list(xmax) + [1] * (3 - len(xmax))
    dx = [(xmax[a] - xmin[a]) / n[a] for a in range(3)]
    bc = list(bc) + [[N, N]] * (3 - len(bc))
    p = dict(ndim=ndim, coord=coord, n=n, xmin=xmin, dx=dx, bc=bc)
    p.update(kw)
    return p


# ------------------------------------------------------------- operators

def test_cartesian_laplacian_is_exact_on_quadratics():
    """The 7-point Laplacian of a quadratic is its exact Laplacian."""
    p = prob(3, CART, (8, 6, 4), (0, 0, 0), (1, 2, 1), [[D, D]] * 3)
    x, y, z = mg.centres(p)
    u = x * x + 2 * y * y - z * z + x * y - 3 * y * z + x
    L = mg.interior(p, mg.apply(p, np.ascontiguousarray(u)))
    np.testing.assert_allclose(L, 4.0, rtol=0, atol=1e-11)


def test_radial_operators_closed_forms():
    """Cylindrical: the radial operator is exact on R^2 (Lap = 4).
    Spherical: on r^2 it gives 6 + dr^2 / (2 r^2) exactly, and the polar
    operator on cos(theta) gives -2 cos(theta) / r^2 times
    2 sin(dth/2) sin(dth) / dth^2 (both by summing the telescoping
    face fluxes in closed form)."""
    p = prob(2, CYL, (16, 8), (0.0, -1), (2.0, 1), [[N, N], [N, N]])
    R, z, _ = mg.centres(p)
    L = mg.interior(p, mg.apply(p, np.ascontiguousarray(R * R)))
    np.testing.assert_allclose(L, 4.0, rtol=1e-13)
    p = prob(2, SPH, (16, 12), (0.5, 0.2), (2.5, math.pi - 0.2), [[N, N], [N, N]])
    r, th, _ = mg.centres(p)
    dr, dth = p["dx"][0], p["dx"][1]
    L = mg.interior(p, mg.apply(p, np.ascontiguousarray(r * r)))
    ri = mg.interior(p, r)
    np.testing.assert_allclose(L, 6.0 + dr * dr / (2 * ri * ri), rtol=1e-13)
    L = mg.interior(p, mg.apply(p, np.ascontiguousarray(np.cos(th))))
    thi = mg.interior(p, th)
    fac = 2 * math.sin(dth / 2) * math.sin(dth) / dth ** 2
    np.testing.assert_allclose(L, -2 * np.cos(thi) / ri ** 2 * fac, rtol=1e-12, atol=1e-13)


def test_azimuthal_second_difference_sign():
    """The azimuthal term is a centred second difference (u+ - 2u + u-): on
    cos(phi) in 3D spherical coordinates it gives
    -cos(phi) (2 - 2 cos dphi) / (r sin(theta) dphi)^2."""
    p = prob(3, SPH, (4, 4, 16), (1.0, 1.0, 0.0), (1.4, 1.4, 2 * math.pi), [[N, N], [N, N], [PER, PER]])
    r, th, ph = mg.centres(p)
    dph = p["dx"][2]
    L = mg.interior(p, mg.apply(p, np.ascontiguousarray(np.cos(ph))))
    ri, thi, phi = (mg.interior(p, a) for a in (r, th, ph))
    ex = -np.cos(phi) * (2 - 2 * math.cos(dph)) / (ri * np.sin(thi) * dph) ** 2
    np.testing.assert_allclose(L, ex, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------ transfer operators

@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_kwak_prolongation_reproduces_linear_fields(ndim):
    """The printed 2D weights (2, 1, 1)/4 toward the child's side, and the
    1D / 3D weights of the same construction, interpolate linear functions
    exactly (coarse ghosts set to the function)."""
    n = [8, 8, 8][:ndim]
    p = prob(ndim, CART, n, [0] * ndim, [1] * ndim, [[D, D]] * ndim)
    xc = mg.centres(p, level=mg.make_desc(p).levels - 2)
    xf = mg.centres(p)
    lin = lambda X: 0.3 + 1.7 * X[0] - (0.9 * X[1] if ndim > 1 else 0) + (0.4 * X[2] if ndim > 2 else 0)
    fine = mg.prolong(p, mg.make_desc(p).levels - 1, np.ascontiguousarray(lin(xc)))
    np.testing.assert_allclose(mg.interior(p, fine), mg.interior(p, lin(xf)), rtol=0, atol=1e-14)


def test_kwak_weights_printed_in_2d():
    """A coarse delta: each child of its cell gets 2/4, each child of a face
    neighbour that faces it 1/4, diagonal neighbours nothing."""
    p = prob(2, CART, (8, 8), (0, 0), (1, 1), [[D, D]] * 2)
    top = mg.make_desc(p).levels - 1
    c = np.zeros(mg.shape(p, top - 1))
    c[0, 3, 3] = 1.0  # coarse interior cell (2, 2)
    f = mg.interior(p, mg.prolong(p, top, c))[0]
    # children of coarse cell (2,2): fine (4..5, 4..5)
    np.testing.assert_allclose(f[4:6, 4:6], 0.5)
    # children of (3,2) facing (2,2): fine i = 6, j = 4..5
    np.testing.assert_allclose(f[4:6, 6], 0.25)
    np.testing.assert_allclose(f[4:6, 7], 0.0)
    np.testing.assert_allclose(f[6, 6], 0.0)
    assert abs(f.sum() - 4 * 0.5 - 8 * 0.25) < 1e-15


def test_piecewise_constant_restriction_is_the_mean_of_children():
    p = prob(3, CART, (8, 8, 4), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
    top = mg.make_desc(p).levels - 1
    rng = np.random.default_rng(3)
    f = rng.standard_normal(mg.shape(p))
    c = mg.interior(p, mg.restrict(p, top, np.ascontiguousarray(f)))
    fi = mg.interior(p, f)
    ex = fi.reshape(2, 2, 4, 2, 4, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(c, ex, rtol=0, atol=1e-15)


# ------------------------------------------------------------------ solver

def operator_matrix(p, a=None):
    """The discrete operator (with its boundary conditions) as a sparse
    matrix, column by column from the oracle's own apply."""
    shp = mg.shape(p)
    inner = mg.interior(p, np.arange(np.prod(shp)).reshape(shp)).ravel()
    cols = []
    for k in inner:
        e = np.zeros(np.prod(shp))
        e[k] = 1.0
        u = np.ascontiguousarray(e.reshape(shp))
        mg.fill_ghosts(p, u)
        cols.append(mg.interior(p, mg.apply(p, u, a)).ravel())
    return sp.csc_matrix(np.array(cols).T)


@pytest.mark.parametrize("coord", [CART, CYL, SPH])
def test_multigrid_reaches_the_discrete_solution(coord):
    """FAS-FMG + V-cycles converge to the exact solution of the discrete
    linear system (direct sparse solve) on 2D grids with Dirichlet, Neumann
    and Robin faces; each V-cycle cuts the residual by a factor > 5 (> 1.6
    in spherical coordinates, whose anisotropy near the inner radius slows
    point smoothers, as section 2.7 notes)."""
    if coord == CART:
        p = prob(2, CART, (16, 16), (0, 0), (1, 1), [[D, D], [N, D]])
    elif coord == CYL:
        p = prob(2, CYL, (16, 16), (0.0, -1), (2.0, 1), [[N, D], [D, D]])
    else:
        p = prob(2, SPH, (16, 16), (0.5, 0.0), (4.5, math.pi), [[D, ROB], [N, N]])
    x, y, _ = mg.centres(p)
    f = np.ascontiguousarray(np.exp(-((x - 1.0) ** 2 + (y - 0.3) ** 2) * 4) - 0.2)
    u = np.zeros(mg.shape(p))
    res = mg.solve(p, u, f, tol=1e-13, max_cycles=40)
    assert res[-1] <= 1e-13
    A = operator_matrix(p)
    ex = spla.spsolve(A, mg.interior(p, f).ravel())
    np.testing.assert_allclose(mg.interior(p, u).ravel(), ex, rtol=0, atol=1e-11 * np.abs(ex).max())
    rates = res[2:-1] / res[1:-2]
    assert rates.max() < (0.6 if coord == SPH else 0.2), rates


def test_second_order_convergence_and_cycle_rate_3d():
    """3D Poisson with a manufactured solution: error O(h^2); the residual
    drops by a steady factor of about 10 per V(2,2)-cycle (> 6.5 asserted)."""
    errs = []
    for n in (16, 32):
        p = prob(3, CART, (n, n, n), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
        x, y, z = mg.centres(p)
        ue = np.sin(math.pi * x) * np.sin(2 * math.pi * y) * np.sin(math.pi * z)
        f = np.ascontiguousarray(-6 * math.pi ** 2 * ue)
        u = np.zeros(mg.shape(p))
        res = mg.solve(p, u, f, tol=1e-11, max_cycles=30)
        assert res[-1] <= 1e-11
        assert (res[2:] / res[1:-1]).max() < 0.15
        errs.append(np.abs(mg.interior(p, u) - mg.interior(p, ue)).max())
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_robin_face_gives_the_exterior_potential():
    """Spherical 1D: a uniform ball (rho = 1 for r < 1/2) on [0, 4] with the
    Robin outer face d(r u)/dr = 0: the solution approaches the exact
    potential (-rho (3R^2 - r^2)/6 inside, -rho R^3 / (3 r) outside) at
    second order."""
    errs = []
    for n in (64, 128):
        p = prob(1, SPH, (n,), (0.0,), (4.0,), [[N, ROB]])
        r, _, _ = mg.centres(p)
        R = 0.5
        f = np.ascontiguousarray(np.where(r < R, 1.0, 0.0))
        ue = np.where(r < R, -(3 * R * R - r * r) / 6.0, -R ** 3 / (3 * r))
        u = np.zeros(mg.shape(p))
        res = mg.solve(p, u, f, tol=1e-13, max_cycles=60)
        assert res[-1] <= 1e-13
        errs.append(np.abs(mg.interior(p, u) - mg.interior(p, ue)).max())
    assert errs[1] < 1e-3 and errs[0] / errs[1] > 3.0


def test_nonlinear_conformal_factor_equation():
    """The static conformal-factor equation of section 2.6 in deviation form,
    Lap(d) = -2 pi U / (1 + d) (p = -1, c = 1), with U a smooth blob and a
    Robin outer face: Newton-Gauss-Seidel multigrid drives the nonlinear
    residual to 1e-12, and the result satisfies the equation as evaluated
    independently (discrete operator on the solution).  Four red-black
    sweeps each way: spherical grids are strongly anisotropic for point
    smoothers (section 2.7)."""
    p = prob(2, SPH, (32, 16), (0.0, 0.0), (8.0, math.pi), [[N, ROB], [N, N]], power=-1, offset=1.0, pre=4,
             post=4)
    r, th, _ = mg.centres(p)
    U = np.ascontiguousarray(0.05 * np.exp(-r * r) * (1 + 0.3 * np.cos(th) ** 2))
    a = np.ascontiguousarray(-2 * math.pi * U)
    f = np.zeros(mg.shape(p))
    u = np.zeros(mg.shape(p))
    res = mg.solve(p, u, f, a, tol=1e-12, max_cycles=100)
    assert res[-1] <= 1e-12
    mg.fill_ghosts(p, u)
    lap = mg.apply(p, u)  # without the nonlinear term
    np.testing.assert_allclose(mg.interior(p, lap), mg.interior(p, -2 * math.pi * U / (1 + u)), rtol=0, atol=1e-11)
    assert mg.interior(p, u).min() > 0.0  # psi > 1 for positive energy density


# --------------------------------------------------- divergence cleaning

def test_cleaning_removes_a_gradient_and_keeps_a_curl():
    """q = grad(phi) + curl(A) in a box (phi = 0 on its faces): one cleaning (solve
    Lap(Phi) = div q, q -= grad Phi) leaves q close to curl(A): the error
    and the remaining divergence are O(h^2) of the removed part."""
    out = []
    for n in (16, 32):
        p = prob(3, CART, (n, n, n), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
        x, y, z = mg.centres(p)
        s = np.sin
        phi = s(math.pi * x) * s(math.pi * y) * s(math.pi * z)
        gphi = [math.pi * np.cos(math.pi * x) * s(math.pi * y) * s(math.pi * z),
                math.pi * s(math.pi * x) * np.cos(math.pi * y) * s(math.pi * z),
                math.pi * s(math.pi * x) * s(math.pi * y) * np.cos(math.pi * z)]
        # A = (0, 0, sin(2 pi x) sin(2 pi y)) -> curl A = (dAz/dy, -dAz/dx, 0)
        curl = [2 * math.pi * s(2 * math.pi * x) * np.cos(2 * math.pi * y),
                -2 * math.pi * np.cos(2 * math.pi * x) * s(2 * math.pi * y), 0 * x]
        q = np.ascontiguousarray(np.stack([gphi[i] + curl[i] for i in range(3)]))
        div0 = mg.divergence(p, q)
        u = np.zeros(mg.shape(p))
        res = mg.solve(p, u, np.ascontiguousarray(div0), tol=1e-12, max_cycles=40)
        assert res[-1] <= 1e-12
        mg.fill_ghosts(p, u)
        mg.subtract_gradient(p, u, q)
        err = max(np.abs(mg.interior(p, q[i]) - mg.interior(p, curl[i])).max() for i in range(3))
        # divergence away from the boundary layer (q's ghosts keep the
        # uncleaned field)
        inner = (slice(2, -2),) * 3
        out.append((err, np.abs(div0[inner]).max(), np.abs(mg.divergence(p, q)[inner]).max()))
    assert out[0][0] / out[1][0] > 3.5       # the gradient part is removed at second order
    assert out[1][2] < 0.05 * out[1][1]       # divergence reduced well below the initial one
    assert out[0][2] / out[1][2] > 3.5       # and what remains is a second-order truncation error


# ----------------------------------------- xCFC vector and A^2 equations

def test_vector_operator_exact_on_quadratics():
    """Lap X^i + (1/3) d_i d_j X^j of quadratic X equals its exact value
    (second differences and the four-point mixed difference are exact on
    quadratics) away from the boundary layer: here (4 + 7/3, 4 + 8/3, 2/3)."""
    p = prob(3, CART, (8, 6, 6), (0, 0, 0), (1, 1.5, 1), [[D, D]] * 3)
    x, y, z = mg.centres(p)
    X = np.ascontiguousarray(np.stack([x * x + 3 * x * y - y * z + z * z,
                                       2 * y * y - x * z + x * y,
                                       z * z + 4 * x * z - x * x + y * z]))
    L = mg.vapply(p, X)
    inner = (slice(2, -2),) * 3
    for i, v in enumerate((4 + 7 / 3, 4 + 8 / 3, 2 / 3)):
        np.testing.assert_allclose(L[i][inner], v, rtol=0, atol=1e-10)


def test_vector_operator_discrete_symbol_on_periodic_modes():
    """On a periodic box every cell, corners and edges across the wrap
    included, gives the discrete symbol of the operator: a second
    difference multiplies a mode by -4 sin^2(k h / 2) / h^2 and the
    four-point mixed difference is the product of two centred first
    differences (factor sin(k h) / h each)."""
    p = prob(3, CART, (8, 12, 8), (0, 0, 0), (1, 1, 1), [[PER, PER]] * 3)
    x, y, z = mg.centres(p)
    hx, hy, hz = p["dx"][:3]
    kx, ky, kz = 2 * math.pi, 4 * math.pi, 2 * math.pi
    sx, sy, sz = (4 * math.sin(k * h / 2) ** 2 / h ** 2 for k, h in ((kx, hx), (ky, hy), (kz, hz)))
    cx, cy, cz = (math.sin(k * h) / h for k, h in ((kx, hx), (ky, hy), (kz, hz)))
    S, C = np.sin, np.cos
    X0 = S(kx * x) * S(ky * y)
    X1 = C(kx * x) * C(ky * y) * C(kz * z)
    X2 = C(kx * x) * S(kz * z)
    L0 = -(sx + sy) * X0 + (-sx * X0 + cx * cy * S(kx * x) * S(ky * y) * C(kz * z)
                            - cx * cz * S(kx * x) * C(kz * z)) / 3
    L1 = -(sx + sy + sz) * X1 + (cx * cy * C(kx * x) * C(ky * y) - sy * X1) / 3
    L2 = -(sx + sz) * X2 + (cy * cz * C(kx * x) * S(ky * y) * S(kz * z) - sz * X2) / 3
    L = mg.vapply(p, np.ascontiguousarray(np.stack([X0, X1, X2])))
    for i, ex in enumerate((L0, L1, L2)):
        np.testing.assert_allclose(mg.interior(p, L[i]), mg.interior(p, ex), rtol=0, atol=1e-9)


def vector_operator_matrix(p):
    shp = (3,) + mg.shape(p)
    inner = np.stack([mg.interior(p, c) for c in np.arange(np.prod(shp)).reshape(shp)]).ravel()
    cols = []
    for k in inner:
        e = np.zeros(np.prod(shp))
        e[k] = 1.0
        L = mg.vapply(p, np.ascontiguousarray(e.reshape(shp)))
        cols.append(np.stack([mg.interior(p, c) for c in L]).ravel())
    return sp.csc_matrix(np.array(cols).T)


def test_vector_multigrid_reaches_the_discrete_solution():
    """The four-colour Newton-Gauss-Seidel FAS cycles reach the exact
    solution of the discrete vector system (direct sparse solve) on a 2D
    grid with Dirichlet x faces and periodic y faces."""
    p = prob(2, CART, (16, 16), (0, 0), (1, 1), [[D, D], [PER, PER]])
    x, y, _ = mg.centres(p)
    f = np.ascontiguousarray(np.stack([np.exp(-((x - 0.4) ** 2 + (y - 0.5) ** 2) * 20),
                                       np.cos(2 * math.pi * y) * x * (1 - x), 0.3 + 0 * x]))
    X = np.zeros((3,) + mg.shape(p))
    res = mg.vsolve(p, X, f, tol=1e-12, max_cycles=60)
    assert res[-1] <= 1e-12
    ex = spla.spsolve(vector_operator_matrix(p), np.stack([mg.interior(p, c) for c in f]).ravel())
    got = np.stack([mg.interior(p, c) for c in X]).ravel()
    np.testing.assert_allclose(got, ex, rtol=0, atol=1e-10 * np.abs(ex).max())
    assert (res[2:] / res[1:-1]).max() < 0.3


def test_vector_equation_second_order_3d():
    """X = phi (1, 2, -1), phi = sin(pi x) sin(pi y) sin(pi z) vanishing on
    the faces of the unit box: L(X)^i = -3 pi^2 X^i + (1/3) d_i (sum_b c_b
    d_b phi) in closed form; the multigrid solution converges to X at
    second order and each V-cycle cuts the residual by > 4."""
    errs = []
    c = (1.0, 2.0, -1.0)
    for n in (8, 16):
        p = prob(3, CART, (n, n, n), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
        x, y, z = mg.centres(p)
        S, C, pi = np.sin, np.cos, math.pi
        phi = S(pi * x) * S(pi * y) * S(pi * z)
        # second derivatives d_i d_b phi
        H = [[-pi * pi * phi, pi * pi * C(pi * x) * C(pi * y) * S(pi * z), pi * pi * C(pi * x) * S(pi * y) * C(pi * z)],
             [None, -pi * pi * phi, pi * pi * S(pi * x) * C(pi * y) * C(pi * z)],
             [None, None, -pi * pi * phi]]
        for i in range(3):
            for b in range(i):
                H[i][b] = H[b][i]
        f = np.ascontiguousarray(np.stack([-3 * pi * pi * c[i] * phi + sum(c[b] * H[i][b] for b in range(3)) / 3
                                           for i in range(3)]))
        X = np.zeros((3,) + mg.shape(p))
        res = mg.vsolve(p, X, f, tol=1e-11, max_cycles=40)
        assert res[-1] <= 1e-11
        assert (res[2:] / res[1:-1]).max() < 0.25
        errs.append(max(np.abs(mg.interior(p, X[i]) - c[i] * mg.interior(p, phi)).max() for i in range(3)))
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_xcfc_aij_of_a_linear_field():
    """For X^b = sum_a M_ba x^a + const, A~^ab = M_ab + M_ba - (2/3) tr(M)
    delta^ab exactly (centred differences), traceless, and A~_ij A~^ij is
    the sum of its squares; six components in the order xx yy zz xy xz yz."""
    p = prob(3, CART, (6, 6, 6), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
    x, y, z = mg.centres(p)
    M = np.array([[0.3, -1.0, 2.0], [0.5, 1.2, -0.7], [0.1, 0.4, -0.9]])
    xs = (x, y, z)
    X = np.ascontiguousarray(np.stack([sum(M[b, a] * xs[a] for a in range(3)) + b for b in range(3)]))
    A6, a2 = mg.xcfc_aij(p, X)
    A = M + M.T - 2.0 / 3.0 * np.trace(M) * np.eye(3)
    inner = (slice(2, -2),) * 3
    for q, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        np.testing.assert_allclose(A6[q][inner], A[i, j], rtol=0, atol=1e-12)
    np.testing.assert_allclose(A6[0][inner] + A6[1][inner] + A6[2][inner], 0.0, atol=1e-12)
    np.testing.assert_allclose(a2[inner], (A * A).sum(), rtol=1e-13)


def test_xcfc_shift_source_closed_form():
    """16 pi w S_i + 2 A~^ij d_j w for w linear (exact centred gradient),
    a uniform S and arbitrary symmetric A~ per cell."""
    p = prob(3, CART, (6, 4, 4), (0, 0, 0), (1.5, 1, 1), [[D, D]] * 3)
    x, y, z = mg.centres(p)
    g = np.array([0.7, -0.2, 0.4])
    w = np.ascontiguousarray(0.9 + g[0] * x + g[1] * y + g[2] * z)
    S = np.ascontiguousarray(np.stack([0.1 + 0 * x, -0.3 + 0 * x, 0.05 + 0 * x]))
    rng = np.random.default_rng(3)
    A6 = np.ascontiguousarray(rng.standard_normal((6,) + x.shape))
    full = [[0, 3, 4], [3, 1, 5], [4, 5, 2]]
    out = mg.xcfc_beta_rhs(p, w, S, A6)
    for i in range(3):
        ex = 16 * math.pi * w * S[i] + 2 * sum(A6[full[i][j]] * g[j] for j in range(3))
        np.testing.assert_allclose(mg.interior(p, out[i]), mg.interior(p, ex), rtol=1e-13, atol=1e-13)


def test_conformal_factor_equation_with_the_aij_term():
    """The conformal-factor equation with both source terms of section 2.6
    in deviation form, Lap(d) = -2 pi U / (1 + d) - (1/8) A2 (1 + d)^-7
    (p = -1, q = -7, c = 1): for a manufactured d (zero on the faces) the
    multigrid solution converges to it at second order, so both non-linear
    terms and their Newton derivatives enter with the right sign and power."""
    errs = []
    for n in (16, 32):
        p = prob(2, CART, (n, n), (0, 0), (1, 1), [[D, D]] * 2, power=-1, power2=-7, offset=1.0)
        x, y, _ = mg.centres(p)
        pi = math.pi
        d = 0.4 * np.sin(pi * x) * np.sin(pi * y)
        U = 0.3 * (1 + x * y)
        A2 = 2.0 + np.cos(3 * x) * np.sin(2 * y)
        a = np.ascontiguousarray(-2 * pi * U)
        a2 = np.ascontiguousarray(-A2 / 8)
        f = np.ascontiguousarray(-2 * pi * pi * d - a / (1 + d) - a2 * (1 + d) ** -7)
        u = np.zeros(mg.shape(p))
        res = mg.solve(p, u, f, a, tol=1e-12, max_cycles=40, a2=a2)
        assert res[-1] <= 1e-12
        errs.append(np.abs(mg.interior(p, u) - mg.interior(p, d)).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_vector_sweep_is_jacobi_within_each_of_four_colours():
    """One vector smoothing sweep equals, colour by colour in the order
    (i mod 2, j mod 2) = (0,0), (1,0), (0,1), (1,1), a simultaneous Newton
    update of that colour's cells, X -= (L(X) - f) / diag, with the operator's
    analytic diagonal -2 sum_a 1/h_a^2 - (2/3)/h_i^2 (component i active): the
    mixed stencil couples diagonal neighbours, so two colours do not
    suffice.  Both axes mirror here, so at the corners the mixed difference
    of one component reads the cell's own other component, which the
    simultaneous update takes from before the cell's update."""
    p = prob(2, CART, (8, 6), (0, 0), (1, 1.5), [[D, N], [D, N]])
    rng = np.random.default_rng(5)
    shp = (3,) + mg.shape(p)
    X = np.ascontiguousarray(rng.standard_normal(shp))
    f = np.ascontiguousarray(rng.standard_normal(shp))
    got = mg.vsmooth(p, X.copy(), f, sweeps=1)
    h = p["dx"]
    diag = [-2 * (1 / h[0] ** 2 + 1 / h[1] ** 2) - (2 / 3) / h[i] ** 2 if i < 2 else -2 * (1 / h[0] ** 2 + 1 / h[1] ** 2)
            for i in range(3)]
    ref = X.copy()
    jj, ii = np.meshgrid(np.arange(shp[2]) - 1, np.arange(shp[3]) - 1, indexing="ij")
    for col in range(4):
        mask = ((ii % 2) == (col & 1)) & ((jj % 2) == (col >> 1))
        mask[0, :] = mask[-1, :] = False
        mask[:, 0] = mask[:, -1] = False
        L = mg.vapply(p, np.ascontiguousarray(ref))
        for i in range(3):
            ref[i, 0][mask] -= (L[i, 0][mask] - f[i, 0][mask]) / diag[i]
    for i in range(3):
        np.testing.assert_allclose(mg.interior(p, got[i]), mg.interior(p, ref[i]), rtol=1e-12, atol=1e-12)


def test_smoother_takes_a_newton_step_on_both_nonlinear_terms():
    """With a negligible Laplacian (huge cells) each cell's equation is
    -a (u+1)^-1 - a2 (u+1)^-7 = f, and one sweep is exactly one Newton step
    on it, derivative a (u+1)^-2 + 7 a2 (u+1)^-8 included."""
    p = prob(2, CART, (4, 4), (0, 0), (4e6, 4e6), [[N, N], [N, N]], power=-1, power2=-7, offset=1.0)
    rng = np.random.default_rng(9)
    shp = mg.shape(p)
    u = np.ascontiguousarray(0.2 + 0.1 * rng.random(shp))
    a = np.ascontiguousarray(-1.0 - rng.random(shp))
    a2 = np.ascontiguousarray(-0.5 - rng.random(shp))
    f = np.ascontiguousarray(rng.random(shp))
    w = 1 + u
    g = -a / w - a2 * w ** -7 - f
    dg = a / w ** 2 + 7 * a2 * w ** -8
    ex = u - g / dg
    got = mg.smooth(p, u.copy(), f, a, sweeps=1, a2=a2)
    np.testing.assert_allclose(mg.interior(p, got), mg.interior(p, ex), rtol=1e-9)


def _xcfc_manufactured():
    """Closed forms of a smooth xCFC configuration on [-1, 1]^3 (all fields
    vanish, or psi and alpha psi equal 1, on the faces): X, psi and
    alpha psi chosen; S~_i, U~ and S~ follow from the X, psi and alpha
    equations of section 2.6; the shift source in closed form too."""
    import sympy as sy
    x, y, z = sy.symbols("x y z")
    c = (x, y, z)
    b = sy.cos(sy.pi * x / 2) * sy.cos(sy.pi * y / 2) * sy.cos(sy.pi * z / 2)
    psi = 1 + sy.Rational(1, 10) * b
    ap = 1 - sy.Rational(3, 20) * b
    X = [sy.Rational(1, 20) * b * (1 + x / 2), -sy.Rational(3, 100) * b * (1 - 2 * y / 5 + z / 5),
         sy.Rational(1, 50) * b * (1 + 3 * x * y / 10)]
    lap = lambda f: sum(sy.diff(f, v, 2) for v in c)  # noqa: E731
    div = sum(sy.diff(X[i], c[i]) for i in range(3))
    S = [(lap(X[i]) + sy.diff(div, c[i]) / 3) / (8 * sy.pi) for i in range(3)]
    A = [[sy.diff(X[j], c[i]) + sy.diff(X[i], c[j]) - (sy.Rational(2, 3) * div if i == j else 0) for j in range(3)]
         for i in range(3)]
    A2 = sum(A[i][j] ** 2 for i in range(3) for j in range(3))
    U = -(lap(psi) + A2 / 8 * psi ** -7) * psi / (2 * sy.pi)
    St = ((lap(ap) / ap - sy.Rational(7, 8) * A2 * psi ** -8) * psi ** 2 / (2 * sy.pi) - U) / 2
    w = ap / psi * psi ** -6
    fb = [16 * sy.pi * w * S[i] + 2 * sum(A[i][j] * sy.diff(w, c[j]) for j in range(3)) for i in range(3)]
    f = lambda e: sy.lambdify(c, e, "numpy")  # noqa: E731
    return dict(psi=f(psi), alpha=f(ap / psi), X=[f(e) for e in X], S=[f(e) for e in S], U=f(U),
                P=f(St / psi ** 6), fb=[f(e) for e in fb])


def test_xcfc_sequence_converges_to_a_manufactured_metric():
    """The oracle's xCFC sequence (steps 1 to 6 of section 2.6) with sources
    manufactured from a chosen X, psi and alpha psi returns them at second
    order; the shift converges at second order to the discrete solution of
    its equation with the closed-form source, so every coefficient of the
    sequence (8 pi S~, A~^ij, the A2 terms of both scalar equations, the
    16 pi w S~ and A~ grad w terms) enters with the right sign and factor."""
    M = _xcfc_manufactured()
    errs = []
    for n in (16, 32):
        base = dict(ndim=3, coord=CART, n=[n] * 3, xmin=[-1.0] * 3, dx=[2.0 / n] * 3, bc=[[D, D]] * 3)
        pv = dict(base)
        ps = dict(base, power=-1, power2=-7, offset=1.0)
        pa = dict(base, power=1, offset=1.0)
        x, y, z = mg.centres(pv)
        ev = lambda fn: np.ascontiguousarray(np.broadcast_to(fn(x, y, z), x.shape), dtype=np.float64)  # noqa: E731
        U = ev(M["U"])
        S = np.ascontiguousarray(np.stack([ev(e) for e in M["S"]]))
        P = ev(M["P"])
        X = np.zeros((3,) + x.shape)
        beta = np.zeros((3,) + x.shape)
        up, ua = np.zeros(x.shape), np.zeros(x.shape)
        psi, alpha, cyc = mg.xcfc_solve(pv, ps, pa, U, S, lambda ps_: ps_ ** 6 * P, X, up, ua, beta, tol=1e-12)
        assert max(cyc) < 60
        bref = np.zeros((3,) + x.shape)
        mg.vsolve(pv, bref, np.ascontiguousarray(np.stack([ev(e) for e in M["fb"]])), tol=1e-12, max_cycles=60)
        I = lambda a: mg.interior(pv, a)  # noqa: E731
        errs.append((max(np.abs(I(X[i]) - I(ev(M["X"][i]))).max() for i in range(3)),
                     np.abs(I(psi) - I(ev(M["psi"]))).max(), np.abs(I(alpha) - I(ev(M["alpha"]))).max(),
                     max(np.abs(I(beta[i]) - I(bref[i])).max() for i in range(3)),
                     max(np.abs(I(bref[i])).max() for i in range(3))))
    for q in range(4):
        assert 3.3 < errs[0][q] / errs[1][q] < 4.7, (q, errs)
    assert errs[1][3] < 0.05 * errs[1][4]  # the shift itself is not small


def test_periodic_axes_keep_an_even_count_on_every_level():
    """With an odd number of cells on a periodic axis the two cells beside
    the wrap would share a colour: the hierarchy stops before that level
    (12 periodic cells: 12, 6; not 3) and refuses it when asked for."""
    p = prob(2, CART, (12, 16), (0, 0), (1, 1), [[PER, PER], [D, D]])
    assert mg.make_desc(p).levels == 2
    assert mg.make_desc(dict(p, bc=[[D, D], [D, D], [N, N]])).levels == 3
    with pytest.raises(ValueError):
        mg.make_desc(dict(p, levels=3))


def test_metric_update_of_a_tov_star():
    """Re-solving the metric of a static TOV star (2D spherical, Robin outer
    face) from its conserved variables, starting from the flat metric:
    psi and alpha approach the TOV metric at second order on the interior
    and on both ghost layers (centre mirror, polar axis, Robin falloff), and
    the primitives recovered on the new metric approach the star's."""
    import oracle as og
    import workloads as W
    errs = []
    for nr, nth in ((48, 8), (96, 16)):
        hp, pr, met = W.magnetised_star_2d(nr, nth, b_peak=1e-12)
        pr = og.fill_ghosts(hp, np.ascontiguousarray(pr))
        q = og.prim2con(hp, pr, met)
        m = met.copy()
        m[0] = 1.0
        m[1] = 1.0
        base = dict(ndim=2, coord=SPH, n=[nr, nth, 1], xmin=[0.0, 0.0, 0.0], dx=[hp["dx"][0], math.pi / nth, 1.0],
                    bc=[[N, ROB], [N, N], [N, N]], pre=4, post=4)
        qc, prim, flags, nf, cyc = mg.metric_update(hp, dict(base, power=-1, offset=1.0),
                                                    dict(base, power=1, offset=1.0), q, pr, m, tol=1e-12,
                                                    max_cycles=300)
        assert nf == 0 and max(cyc) < 300
        g = hp["ng"]
        inner = (0, slice(g, g + nth), slice(g, g + nr))
        ghost = (0, slice(0, g + nth + g), slice(0, g + nr + g))
        rho_i = np.abs(prim[0][inner] - pr[0][inner]).max() / pr[0].max()
        errs.append((np.abs(m[0][ghost] - met[0][ghost]).max(), np.abs(m[1][ghost] - met[1][ghost]).max(), rho_i))
    assert errs[1][0] < 4e-4 and errs[1][1] < 6e-4
    for k in range(3):
        assert errs[0][k] / errs[1][k] > 2.5, errs


def test_stilde_is_the_same_scalar_in_every_coordinate_system():
    """S~ = psi^6 (rho h W^2 v^2 + 3 p) is a scalar: one uniform flow
    (W v = (0.3, -0.2, 0.4) in Cartesian components) written in cylindrical
    (R, z, phi) and spherical (r, theta, phi) contravariant components by
    the coordinate Jacobian gives the Cartesian value in every cell."""
    import workloads as W
    V = np.array([0.3, -0.2, 0.4])
    psi0, rho0, p0, gam = 1.1, 0.7, 0.2, 5.0 / 3.0
    ex = psi0 ** 6 * ((rho0 + gam / (gam - 1) * p0) * psi0 ** 4 * (V @ V) + 3 * p0)
    for coord in (W.CYL, W.SPH):
        if coord == W.CYL:
            hp = W.grid(3, coord, [6, 5, 8], [0.5, -1.0, 0.0], [2.0, 1.0, 2 * math.pi], [[W.OUTFLOW] * 2] * 3,
                        gamma=gam)
        else:
            hp = W.grid(3, coord, [6, 5, 8], [0.5, 0.3, 0.0], [2.0, math.pi - 0.3, 2 * math.pi],
                        [[W.OUTFLOW] * 2] * 3, gamma=gam)
        a, b, c = W.centres(hp)
        pr = W.empty_prim(hp)
        pr[0], pr[4] = rho0, p0
        if coord == W.CYL:
            R, phi = a, c
            x, y = R * np.cos(phi), R * np.sin(phi)
            pr[1] = (x * V[0] + y * V[1]) / R
            pr[2] = V[2] + 0 * R
            pr[3] = (x * V[1] - y * V[0]) / R ** 2
        else:
            r, th, phi = a, b, c
            pr[1] = np.sin(th) * np.cos(phi) * V[0] + np.sin(th) * np.sin(phi) * V[1] + np.cos(th) * V[2]
            pr[2] = (np.cos(th) * np.cos(phi) * V[0] + np.cos(th) * np.sin(phi) * V[1] - np.sin(th) * V[2]) / r
            pr[3] = (-np.sin(phi) * V[0] + np.cos(phi) * V[1]) / (r * np.sin(th))
        St = mg.fluid_stilde_curvilinear(hp, np.full(a.shape, psi0), pr)
        np.testing.assert_allclose(St, ex, rtol=1e-13)


def test_cartesian_robin_faces_give_the_exterior_potential():
    """A uniform ball (rho = 1, R = 1/2) at the centre of a Cartesian box
    [-2, 2]^3 with the condition u + x.grad u = 0 on every face (section
    2.6; ghost rule exact for a 1/r fall-off): the solution approaches the
    exact potential of the ball (-rho (3R^2 - r^2)/6 inside, -rho R^3/(3r)
    outside) at second order; with Dirichlet faces it does not."""
    errs, errd = [], []
    for n in (16, 32):
        for kind, out in ((ROB, errs), (D, errd)):
            p = prob(3, CART, (n, n, n), (-2, -2, -2), (2, 2, 2), [[kind, kind]] * 3)
            x, y, z = mg.centres(p)
            r = np.sqrt(x * x + y * y + z * z)
            R = 0.5
            # cell-averaged ball (8^3 sub-samples) keeps the source smooth in n
            f = np.zeros_like(r)
            h = p["dx"][0]
            sub = (np.arange(8) + 0.5) / 8 - 0.5
            for sx in sub:
                for sy in sub:
                    for sz in sub:
                        f += ((x + sx * h) ** 2 + (y + sy * h) ** 2 + (z + sz * h) ** 2 < R * R)
            f = np.ascontiguousarray(f / 512.0)
            ue = np.where(r < R, -(3 * R * R - r * r) / 6.0, -R ** 3 / (3 * r))
            u = np.zeros(mg.shape(p))
            res = mg.solve(p, u, f, tol=1e-12, max_cycles=60)
            assert res[-1] <= 1e-12
            out.append(np.abs(mg.interior(p, u) - mg.interior(p, ue)).max())
    assert errs[0] / errs[1] > 3.0, errs
    assert errd[1] > 10 * errs[1], (errs, errd)


def test_extend_reproduces_a_monopole_on_cartesian_robin_faces():
    """Extending u = 1/r from the interior of a Cartesian grid to two ghost
    layers by the Robin rule reproduces 1/r on every ghost cell, edges and
    corners included (the per-axis factors telescope)."""
    import workloads as W
    hp = W.grid(3, W.CART, [8, 6, 4], [0.5, -1.0, 0.3], [2.5, 1.4, 1.9], [[W.OUTFLOW] * 2] * 3)
    p = dict(ndim=3, coord=CART, n=[8, 6, 4], xmin=[0.5, -1.0, 0.3], dx=list(hp["dx"]), bc=[[ROB, ROB]] * 3)
    x, y, z = mg.centres(p)
    u = 1.0 / np.sqrt(x * x + y * y + z * z)
    X, Y, Z = W.centres(hp)
    np.testing.assert_allclose(mg.extend(hp, p, u), 1.0 / np.sqrt(X * X + Y * Y + Z * Z), rtol=1e-14)


def test_cylindrical_robin_faces_give_the_exterior_potential():
    """A Gaussian mass (rho = exp(-r^2/s^2), s = 0.3) in a cylindrical
    (R, z) box [0, 2] x [-2, 2] with the condition u + R du/dR + z du/dz = 0
    on the outer R face and both z faces: the solution converges at second
    order to its exact potential -M erf(r/s) / (4 pi r), M = pi^(3/2) s^3
    (ratios 3.7-4.0 from 16 to 128 cells); Dirichlet faces do not converge."""
    from scipy.special import erf
    out = {}
    for kind in (ROB, D):
        errs = []
        for n in (32, 64):
            p = prob(2, CYL, (n // 2, n), (0.0, -2.0), (2.0, 2.0), [[N, kind], [kind, kind]])
            R_, z, _ = mg.centres(p)
            r = np.sqrt(R_ * R_ + z * z)
            s = 0.3
            f = np.ascontiguousarray(np.exp(-r * r / s ** 2))
            ue = -math.pi ** 1.5 * s ** 3 / (4 * math.pi * r) * erf(r / s)
            u = np.zeros(mg.shape(p))
            res = mg.solve(p, u, f, tol=1e-12, max_cycles=80)
            assert res[-1] <= 1e-12
            errs.append(np.abs(mg.interior(p, u) - mg.interior(p, ue)).max())
        out[kind] = errs
    assert out[ROB][0] / out[ROB][1] > 3.5, out
    assert out[D][1] > 10 * out[ROB][1], out


def _cartesian_field(kind):
    """A smooth vector field V(x, y, z) (axisymmetric about z for the
    curvilinear cases, equatorially symmetric where a grid needs it,
    vanishing on the outer faces used below) with L(V) = Lap V +
    (1/3) grad div V and A~_ij = d_i V_j + d_j V_i - (2/3) delta_ij div V in
    closed form (Cartesian components, sympy)."""
    import sympy as sy
    x, y, z = sy.symbols("x y z", real=True)
    c = (x, y, z)
    R2 = x * x + y * y
    if kind == "cart":
        B = (1 - x * x) ** 2 * (1 - y * y) ** 2 * (1 - z * z) ** 2
        V = [B * (1 + z * z) * (x + 0.5), B * y * (2 - z * z), B * z * (1 + x * y)]
    elif kind == "cyl":
        B = (1 - R2 / 4) ** 2 * (1 - z * z / 4) ** 2
        f1, f2, f3 = B * (1 + z / 3), B * (1 + R2 / 5 - z), B * (2 - R2 / 3)
        V = [f1 * x - f3 * y, f1 * y + f3 * x, f2]
    else:
        B = (1 - (R2 + z * z) / 4) ** 2
        g1, g2, g3 = B * (1 + z * z / 2), B * (1 - R2 / 3), B * (1 + R2 / 4 + z * z)
        V = [g1 * x - g3 * y, g1 * y + g3 * x, g2 * z]
    div = sum(sy.diff(V[i], c[i]) for i in range(3))
    Lv = [sum(sy.diff(V[i], v, 2) for v in c) + sy.diff(div, c[i]) / 3 for i in range(3)]
    A = [[sy.diff(V[j], c[i]) + sy.diff(V[i], c[j]) - (sy.Rational(2, 3) * div if i == j else 0) for j in range(3)]
         for i in range(3)]
    f = lambda e: sy.lambdify(c, e, "numpy")  # noqa: E731
    return [f(e) for e in V], [f(e) for e in Lv], [[f(A[i][j]) for j in range(3)] for i in range(3)]


def _orthonormal(kind, p, F):
    """Cartesian vector (list of three callables) at the cell centres of p,
    in the grid's orthonormal components (axisymmetric grids: the phi = 0
    half-plane, x = R or r sin(theta), y = 0)."""
    a, b, cz = mg.centres(p)
    if kind == "cart":
        return [np.broadcast_to(F[i](a, b, cz), a.shape) for i in range(3)]
    if kind == "cyl":
        X, Z = a, b
        v = [np.broadcast_to(F[i](X, 0 * X, Z), X.shape) for i in range(3)]
        return [v[0], v[2], v[1]]  # (R, z, phi) = (x, z, y) on phi = 0
    r, th = a, b
    X, Z = r * np.sin(th), r * np.cos(th)
    v = [np.broadcast_to(F[i](X, 0 * X, Z), X.shape) for i in range(3)]
    return [v[0] * np.sin(th) + v[2] * np.cos(th), v[0] * np.cos(th) - v[2] * np.sin(th), v[1]]


VGRIDS = {
    # half box with the symmetry plane z = 0 (Neumann: V_z odd, V_x, V_y even)
    "cart": lambda n: prob(3, CART, (n, n, n // 2), (-1, -1, 0), (1, 1, 1), [[D, D], [D, D], [N, D]]),
    # (R, z): axis R = 0 (V_R, V_phi odd), Dirichlet outer faces
    "cyl": lambda n: prob(2, CYL, (n, 2 * n), (0.0, -2.0), (2.0, 2.0), [[N, D], [D, D]]),
    # (r, theta) on [0, 2] x [0, pi/2]: centre, polar axis, equator, Dirichlet at r = 2
    "sph": lambda n: prob(2, SPH, (n, n // 2), (0.0, 0.0), (2.0, math.pi / 2), [[N, D], [N, N]], pre=4, post=4),
}


@pytest.mark.parametrize("kind", ["cart", "cyl", "sph"])
def test_vector_equations_in_three_coordinate_systems(kind):
    """A manufactured solution built in Cartesian coordinates (sympy) and
    written in the grid's orthonormal components: the discrete vector
    solution converges to it at second order in Cartesian (with a symmetry
    plane), cylindrical and spherical coordinates, which checks every
    connection term, the corner weights and the per-component parity of
    every face kind (centre, axis, equator, symmetry plane)."""
    V, Lv, _ = _cartesian_field(kind)
    errs = []
    for n in (16, 32):
        p = VGRIDS[kind](n)
        f = np.ascontiguousarray(np.stack(_orthonormal(kind, p, Lv)))
        ex = _orthonormal(kind, p, V)
        X = np.zeros((3,) + mg.shape(p))
        res = mg.vsolve(p, X, f, tol=1e-10 * np.abs(f).max(), max_cycles=400)
        assert res[-1] <= 1e-10 * np.abs(f).max(), (len(res), res[-1])
        errs.append(max(np.abs(mg.interior(p, X[i]) - mg.interior(p, ex[i])).max() for i in range(3)))
    # (Cartesian 16 -> 32 is still pre-asymptotic: 3.2, then order 1.84 to 48)
    assert 3.0 < errs[0] / errs[1] < 4.7, errs


@pytest.mark.parametrize("kind", ["cyl", "sph"])
def test_xcfc_aij_in_curvilinear_components(kind):
    """A~ from the orthonormal components of a field in cylindrical or
    spherical coordinates (with the connection terms) converges at second
    order to the Cartesian A~_ij of the same field projected on the
    orthonormal frame, and A~_ij A~^ij to its (frame-independent) value."""
    V, _, A = _cartesian_field(kind)
    errs = []
    for n in (32, 64):
        p = VGRIDS[kind](n)
        X = np.ascontiguousarray(np.stack(_orthonormal(kind, p, V)))
        A6, a2 = mg.xcfc_aij(p, X)
        inner = (Ellipsis, slice(2, -2), slice(2, -2))
        # the Cartesian tensor at the centres, then its components on the
        # grid's orthonormal frame (E_R, E_z, E_phi) or (E_r, E_theta, E_phi)
        a_, b_, _ = mg.centres(p)
        if kind == "cyl":
            pts = (a_, 0 * a_, b_)
            E = [(1.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0)]
            frame = [[np.full(a_.shape, e[q]) for q in range(3)] for e in E]
        else:
            r, th = a_, b_
            pts = (r * np.sin(th), 0 * r, r * np.cos(th))
            frame = [[np.sin(th), 0 * r, np.cos(th)], [np.cos(th), 0 * r, -np.sin(th)], [0 * r, 1 + 0 * r, 0 * r]]
        T = [[np.broadcast_to(A[i][j](*pts), a_.shape) for j in range(3)] for i in range(3)]
        proj = [[sum(frame[u][i] * T[i][j] * frame[v][j] for i in range(3) for j in range(3)) for v in range(3)]
                for u in range(3)]
        e = 0.0
        for q, (u, v) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
            e = max(e, np.abs(A6[q][inner] - proj[u][v][inner]).max())
        e2 = np.abs(a2[inner] - sum(T[i][j] ** 2 for i in range(3) for j in range(3))[inner]).max()
        errs.append((e, e2))
    for k in range(2):
        assert errs[0][k] / errs[1][k] > 3.3, errs


def test_shift_source_uses_the_orthonormal_gradient():
    """16 pi w S_i + 2 A~^ij grad_j w in spherical coordinates: for
    w = 1 + 0.2 z (z = r cos(theta)) the orthonormal gradient is
    (0.2 cos(theta), -0.2 sin(theta), 0); the discrete source converges to
    the closed form at second order (the theta derivative carries 1/r)."""
    errs = []
    for n in (32, 64):
        p = VGRIDS["sph"](n)
        r, th, _ = mg.centres(p)
        w = np.ascontiguousarray(1.0 + 0.2 * r * np.cos(th))
        S = np.ascontiguousarray(np.stack([0.1 + 0 * r, -0.05 + 0 * r, 0.02 + 0 * r]))
        rng = np.random.default_rng(4)
        A6 = np.ascontiguousarray(np.broadcast_to(rng.standard_normal((6, 1, 1, 1)), (6,) + r.shape))
        g = [0.2 * np.cos(th), -0.2 * np.sin(th), 0 * r]
        full = [[0, 3, 4], [3, 1, 5], [4, 5, 2]]
        out = mg.xcfc_beta_rhs(p, w, S, A6)
        e = 0.0
        for i in range(3):
            ex = 16 * math.pi * w * S[i] + 2 * sum(A6[full[i][j]] * g[j] for j in range(3))
            e = max(e, np.abs(mg.interior(p, out[i]) - mg.interior(p, ex)).max())
        errs.append(e)
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


# ------------------------------------------------ line relaxation smoother

def _lines(p, ax, col):
    """Interior flat indices (k, j, i order) of each line of colour col
    along axis ax: transverse axes coloured by index parity (bit 0 the
    lower transverse axis, bit 1 the upper)."""
    nd = p["ndim"]
    shp = tuple(p["n"][a] for a in (2, 1, 0))
    idx = np.arange(int(np.prod(shp))).reshape(shp)
    b1, b2 = (1 if ax == 0 else 0), (1 if ax == 2 else 2)
    lines = {}
    for kk in range(shp[0]):
        for jj in range(shp[1]):
            for ii in range(shp[2]):
                c = [ii, jj, kk]
                p1 = c[b1] & 1 if b1 < nd else 0
                p2 = c[b2] & 1 if b2 < nd else 0
                if (p1 | (p2 << 1)) == col:
                    lines.setdefault(tuple(c[b] for b in range(3) if b != ax), []).append(idx[kk, jj, ii])
    return [np.array(sorted(v)) for v in lines.values()]


def _block_gauss_seidel(p, residual, jacobian, u, sweeps, ncomp=1):
    """Line sweeps from their definition: per active non-periodic axis, per
    colour, per line (per component) one Newton step u_I += J_II^-1 r_I with
    the full residual r and the Jacobian block of the line's unknowns."""
    nd = p["ndim"]
    nc = int(np.prod(p["n"]))
    for _ in range(sweeps):
        for ax in range(nd):
            if p["bc"][ax][0] == PER:
                continue
            for col in range(1 << (nd - 1)):
                for I0 in _lines(p, ax, col):
                    for q in range(ncomp):
                        I = I0 + q * nc
                        r = residual(u)
                        u[I] += np.linalg.solve(jacobian(u)[np.ix_(I, I)], r[I])
    return u


LINE_SCALAR = {
    "sph2d_robin": prob(2, SPH, (8, 6), (0, 0), (30, math.pi / 2), [[N, ROB], [N, N]]),
    "cyl2d_robin": prob(2, CYL, (6, 8), (0, -1), (2, 1), [[N, ROB], [ROB, D]]),
    "cart3d_periodic": prob(3, CART, (4, 4, 6), (0, 0, 0), (1, 1, 1), [[D, N], [PER, PER], [ROB, D]]),
    "sph3d_shell": prob(3, SPH, (4, 4, 4), (0.5, 0.3, 0), (2.5, math.pi - 0.3, 2 * math.pi),
                        [[D, ROB], [N, D], [PER, PER]]),
    "psi_sph2d": prob(2, SPH, (8, 6), (0, 0), (30, math.pi / 2), [[N, ROB], [N, N]], power=-1, power2=-7,
                      offset=1.0),
}


@pytest.mark.parametrize("case", sorted(LINE_SCALAR))
def test_line_smoother_is_block_gauss_seidel_over_lines(case):
    """Two line-relaxation sweeps equal block Gauss-Seidel over the lines
    of the assembled operator (its matrix built column by column from the
    point operator with the boundary rule, the nonlinear terms' derivative
    added on the diagonal): the Jacobian blocks, the line ordering and the
    boundary folds all follow from the operator itself."""
    p = LINE_SCALAR[case]
    rng = np.random.default_rng(5)
    sh = mg.shape(p)
    u0 = rng.standard_normal(sh) * 0.1
    f = rng.standard_normal(sh)
    nl = p.get("power", 0) != 0
    a = rng.random(sh) * 0.1 if nl else None
    a2 = rng.random(sh) * 0.1 if nl else None
    A = operator_matrix(p).toarray()
    ai, a2i = (mg.interior(p, a).ravel(), mg.interior(p, a2).ravel()) if nl else (0.0, 0.0)
    c, q = p.get("offset", 0.0), p.get("power2", 0)

    def nonlin(v, deriv):
        w = v + c
        if not nl:
            return 0.0 * v
        return (-ai / (w * w) + a2i * q * w ** (q - 1)) if deriv else (ai / w + a2i * w ** q)

    fi = mg.interior(p, f).ravel()
    ref = _block_gauss_seidel(p, lambda v: fi - (A @ v - nonlin(v, False)),
                              lambda v: A - np.diag(nonlin(v, True)), mg.interior(p, u0).ravel().copy(), 2)
    got = mg.interior(p, mg.line_smooth(p, u0.copy(), f, a, sweeps=2, a2=a2)).ravel()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


LINE_VECTOR = {
    "sph2d_eq": prob(2, SPH, (8, 6), (0, 0), (2, math.pi / 2), [[N, D], [N, N]]),
    "sph2d_shell": prob(2, SPH, (6, 8), (0.5, 0), (2.5, math.pi), [[D, D], [N, N]]),
    "cyl2d": prob(2, CYL, (6, 8), (0, -2), (2, 2), [[N, D], [D, D]]),
    "cart3d_ragged": prob(3, CART, (4, 6, 4), (0, 0, 0), (1.2, 2.0, 0.6), [[PER, PER], [N, D], [D, D]]),
    "cart1d": prob(1, CART, (8,), (0,), (1,), [[D, N]]),
}


@pytest.mark.parametrize("case", sorted(LINE_VECTOR))
def test_vector_line_smoother_is_block_gauss_seidel(case):
    """Two vector line sweeps equal block Gauss-Seidel over (line,
    component) blocks of the assembled vector operator, components of a
    line in order: the 4/3 weight of the component along the line, the
    mirror signs folded at the boundaries and the orthonormal connection
    terms on the diagonal all follow from the operator."""
    p = LINE_VECTOR[case]
    rng = np.random.default_rng(6)
    sh = (3,) + mg.shape(p)
    X0, f = rng.standard_normal(sh), rng.standard_normal(sh)
    A = vector_operator_matrix(p).toarray()
    fi = np.concatenate([mg.interior(p, f[q]).ravel() for q in range(3)])
    x = np.concatenate([mg.interior(p, X0[q]).ravel() for q in range(3)])
    ref = _block_gauss_seidel(p, lambda v: fi - A @ v, lambda v: A, x, 2, ncomp=3)
    got = mg.vline_smooth(p, X0.copy(), f, sweeps=2)
    g = np.concatenate([mg.interior(p, got[q]).ravel() for q in range(3)])
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("coord", [CART, CYL, SPH])
def test_one_line_sweep_solves_a_linear_1d_problem(coord):
    """In 1D the only line is the whole grid: one sweep solves a linear
    equation (p = 1 here) to rounding."""
    p = prob(1, coord, (32,), (0.0,), (4.0,), [[N if coord != CART else D, ROB]], power=1, offset=1.0)
    rng = np.random.default_rng(7)
    sh = mg.shape(p)
    u, f, a = rng.standard_normal(sh), rng.standard_normal(sh), rng.random(sh)
    mg.line_smooth(p, u, f, a, sweeps=1)
    L = mg.interior(p, mg.apply(p, u, a))
    assert np.abs(mg.interior(p, f) - L).max() <= 1e-12 * np.abs(L).max()


def test_line_relaxation_cycles_reach_the_discrete_solution_on_anisotropic_cells():
    """FAS cycles with line relaxation on the spherical layout of the paper's
    2D rotating-star runs, coarsened (64 x 16 on [0, 30] x [0, pi/2]: cells
    from r dtheta / dr = 0.05 at the centre to 26 at r = 30) reach the
    direct sparse solution of the discrete system; each V(2,2)-cycle cuts
    the residual by more than 5 until the rounding floor of this grid
    (about 1e-11) is near, where point relaxation (section 2.7's smoother,
    which the paper notes slows down on such grids) has not converged after
    three times as many cycles."""
    p = prob(2, SPH, (64, 16), (0.0, 0.0), (30.0, math.pi / 2), [[N, ROB], [N, N]], smoother=1)
    x, y, _ = mg.centres(p)
    f = np.ascontiguousarray(np.exp(-(x / 6) ** 2) * (1 + 0.5 * np.cos(y) ** 2))
    u = np.zeros(mg.shape(p))
    res = mg.solve(p, u, f, tol=1e-11, max_cycles=60)
    assert res[-1] <= 1e-11
    A = operator_matrix(p)
    ex = spla.spsolve(A, mg.interior(p, f).ravel())
    np.testing.assert_allclose(mg.interior(p, u).ravel(), ex, rtol=0, atol=1e-10 * np.abs(ex).max())
    rates = np.array([res[c + 1] / res[c] for c in range(1, len(res) - 1) if res[c] > 1e-8])
    assert len(rates) >= 5 and rates.max() < 0.2, rates
    up = np.zeros(mg.shape(p))
    resp = mg.solve(dict(p, smoother=0), up, f, tol=1e-11, max_cycles=3 * (len(res) - 1))
    assert resp[-1] > 1e3 * 1e-11, resp[-1]
