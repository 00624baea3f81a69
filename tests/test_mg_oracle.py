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
