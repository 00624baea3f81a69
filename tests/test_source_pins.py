"""Pins of the oracle's gravitational source terms (section 2.1, the momentum
and energy sources with the extrinsic curvature and the shift) against an
independent construction from the 4-metric.

For a stationary space-time (psi, alpha, beta^i independent of t) the
covariant conservation law, written with partial derivatives of the full
4-metric g_mu_nu, gives the sources directly:
    momentum:  sqrt(-g)/sqrt(ref) * 1/2 T^{mu nu} d_j g_{mu nu}
    energy:    sqrt(-g)/sqrt(ref) * (T^{mu 0} d_mu alpha - alpha T^{mu nu} Gamma^0_{mu nu})
(sqrt(-g)/sqrt(ref) = alpha psi^6).  In curvilinear coordinates the paper
moves the flat-metric part Gamma^_{l i j} F^i_l of the momentum divergence
into the geometric source, so the gravitational momentum source is the
expression above minus Gamma^l_{ij} F^i_l with the point Christoffel symbols
of the reference metric and the densitised flux F^i_l = alpha psi^6 T^i_l.
The 4-metric, its derivatives and Christoffel symbols come from sympy; the
stress tensor from plain tensor algebra of the primitives.  The extrinsic
curvature of a stationary metric follows from the ADM evolution equation
with d_t gamma_ij = 0: K_ij = (D_i beta_j + D_j beta_i) / (2 alpha), D the
covariant derivative of gamma_ij = psi^4 ref_ij (3-Christoffels from sympy).

The oracle evaluates the same sources with centred differences of
cell-centred metric arrays; at spacings h and h/2 the Richardson
combination (4 s(h/2) - s(h)) / 3 removes the O(h^2) term.  Cases:
  - a general metric (psi, alpha, beta varying, beta not divergence free)
    with K_ij supplied exactly, Cartesian and spherical;
  - a rotating shift (divergence free, tangent to the level sets of psi) with
    K_ij taken from the shift by the oracle's own CFC relation under maximal
    slicing, which is exact for such a stationary metric.
A set of mutant oracles, each compiled from the oracle's source with one
planted mistake (the sign of the K_ij beta^i beta^j term, the index order of
D^_i beta^k, the Christoffel index in D^_i beta^k, the 1/2 of the d psi
term, the factor 2 of the K_ij beta^j term), must fail the same pin.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest
import sympy as sy

import oracle
import workloads as W

GAMMA = 5.0 / 3.0
X1, X2, X3 = sy.symbols("x1 x2 x3", real=True)
XS = (X1, X2, X3)


def ref_metric_sym(coord):
    if coord == W.SPH:
        return [sy.Integer(1), X1 ** 2, (X1 * sy.sin(X2)) ** 2]
    return [sy.Integer(1), sy.Integer(1), sy.Integer(1)]


def metric_case(name):
    """psi, alpha, beta^i (coordinate components) as sympy expressions."""
    if name == "cart_general":
        psi = 1 + sy.Rational(1, 10) * sy.exp(-(X1 ** 2 + 2 * X2 ** 2 + X3 ** 2) / 3) + sy.Rational(1, 50) * X1 * X3
        alpha = sy.Rational(7, 10) + sy.Rational(1, 10) * sy.cos(X1 + X2) + sy.Rational(1, 20) * X3
        beta = [sy.Rational(1, 10) * sy.sin(X2 + X3), sy.Rational(1, 8) * X1 * X3, sy.Rational(1, 12) * (X1 + X2 ** 2)]
        return W.CART, (0.3, -0.2, 0.4), psi, alpha, beta
    if name == "sph_general":
        psi = 1 + sy.Rational(1, 10) / (1 + X1 ** 2) + sy.Rational(1, 40) * sy.cos(X2) * sy.sin(X3)
        alpha = sy.Rational(3, 4) - sy.Rational(1, 10) / (1 + X1) + sy.Rational(1, 30) * sy.sin(X2) ** 2
        beta = [sy.Rational(1, 10) * sy.sin(X2) / (1 + X1), sy.Rational(1, 20) * sy.cos(X2) / X1,
                sy.Rational(1, 15) / (1 + X1 ** 2) + sy.Rational(1, 50) * sy.cos(X3)]
        return W.SPH, (1.3, 0.9, 0.7), psi, alpha, beta
    if name == "cart_rotating":
        rho2 = X1 ** 2 + X2 ** 2
        psi = 1 + sy.Rational(1, 8) * sy.exp(-(rho2 + 2 * X3 ** 2) / 4)
        alpha = sy.Rational(7, 10) + sy.Rational(1, 10) * sy.cos(X1 - X3) + sy.Rational(1, 20) * X2
        om = sy.Rational(1, 5) / (1 + rho2 + X3 ** 2)
        beta = [-om * X2, om * X1, sy.Integer(0)]
        return W.CART, (0.35, -0.25, 0.3), psi, alpha, beta
    if name == "sph_rotating":
        psi = 1 + sy.Rational(1, 6) / (1 + X1 ** 2) + sy.Rational(1, 30) * sy.cos(X2) ** 2
        alpha = sy.Rational(3, 4) - sy.Rational(1, 10) / (1 + X1) + sy.Rational(1, 40) * sy.cos(X3)
        beta = [sy.Integer(0), sy.Integer(0), sy.Rational(1, 5) / (1 + X1 ** 3) * (1 + sy.sin(X2) ** 2)]
        return W.SPH, (1.4, 1.1, 0.6), psi, alpha, beta
    raise KeyError(name)


def exact_sources(case, prim):
    """Exact gravitational sources (8 components; only S_i and tau non-zero)
    and the exact K_ij of the stationary metric at the case's point."""
    coord, x0, psi, alpha, beta = metric_case(case)
    ref = ref_metric_sym(coord)
    gam = [psi ** 4 * r for r in ref]
    bl = [gam[i] * beta[i] for i in range(3)]
    g4 = sy.zeros(4, 4)
    g4[0, 0] = -alpha ** 2 + sum(bl[i] * beta[i] for i in range(3))
    for i in range(3):
        g4[0, 1 + i] = g4[1 + i, 0] = bl[i]
        g4[1 + i, 1 + i] = gam[i]
    subs = dict(zip(XS, x0))
    G = np.array(g4.subs(subs).evalf(30), dtype=float)
    dG = np.zeros((4, 4, 4))  # dG[l][mu][nu] = d_l g_mu_nu, d_0 = 0
    for l in range(3):
        dG[1 + l] = np.array(sy.diff(g4, XS[l]).subs(subs).evalf(30), dtype=float)
    Ginv = np.linalg.inv(G)
    # Gamma^0_{mu nu} of the 4-metric
    Chr0 = np.zeros((4, 4))
    for m in range(4):
        for n in range(4):
            Chr0[m, n] = 0.5 * sum(Ginv[0, l] * (dG[m, l, n] + dG[n, l, m] - dG[l, m, n]) for l in range(4))
    a0 = float(alpha.subs(subs))
    dal = np.array([0.0] + [float(sy.diff(alpha, XS[l]).subs(subs)) for l in range(3)])
    p0 = float(psi.subs(subs))
    b0 = np.array([float(b.subs(subs)) for b in beta])
    refv = np.array([float(r.subs(subs)) for r in ref])
    # T^{mu nu} from the primitives
    gd = p0 ** 4 * refv
    Wv = np.asarray(prim[1:4])
    W_ = math.sqrt(1.0 + (gd * Wv * Wv).sum())
    v = Wv / W_
    u = np.concatenate([[W_ / a0], W_ * (v - b0 / a0)])
    ud = G @ u
    B4 = np.concatenate([[0.0], prim[5:8]])
    b = (B4 + (ud @ B4) * u) / W_
    b2 = b @ G @ b
    rho, p = prim[0], prim[4]
    h = 1.0 + GAMMA / (GAMMA - 1.0) * p / rho
    T = (rho * h + b2) * np.outer(u, u) + (p + 0.5 * b2) * Ginv - np.outer(b, b)
    pre = a0 * p0 ** 6
    s = np.zeros(8)
    # flat-metric Christoffels at the point (reference metric diagonal)
    refd = [sy.diff(r, XS[l]) for r in ref for l in range(3)]  # noqa: F841
    Ch = np.zeros((3, 3, 3))  # Ch[l][i][j] = Gamma^l_ij of the reference metric
    for l in range(3):
        for i in range(3):
            for j in range(3):
                e = sy.Rational(1, 2) / ref[l] * (sy.diff(ref[l], XS[i]) * (1 if l == j else 0)
                                                   + sy.diff(ref[l], XS[j]) * (1 if l == i else 0)
                                                   - (sy.diff(ref[i], XS[l]) if i == j else 0))
                Ch[l, i, j] = float(e.subs(subs))
    Tmix = T @ G  # T^mu_nu
    for j in range(3):
        full = pre * 0.5 * np.einsum("mn,mn->", T, dG[1 + j])
        geo = sum(Ch[l, i, j] * pre * Tmix[1 + i, 1 + l] for l in range(3) for i in range(3))
        s[1 + j] = full - geo
    s[4] = pre * (T[1:, 0] @ dal[1:] - a0 * np.einsum("mn,mn->", T, Chr0))
    # K_ij = (D_i beta_j + D_j beta_i) / (2 alpha), D of gamma_ij = psi^4 ref
    g3 = sy.diag(*gam)
    g3i = g3.inv()
    C3 = [[[sum(g3i[k, m] * (sy.diff(g3[m, i], XS[j]) + sy.diff(g3[m, j], XS[i]) - sy.diff(g3[i, j], XS[m]))
                for m in range(3)) / 2 for j in range(3)] for i in range(3)] for k in range(3)]
    K = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            Dij = sy.diff(bl[j], XS[i]) - sum(C3[k][i][j] * bl[k] for k in range(3))
            Dji = sy.diff(bl[i], XS[j]) - sum(C3[k][j][i] * bl[k] for k in range(3))
            K[i, j] = float(((Dij + Dji) / (2 * alpha)).subs(subs).evalf(30))
    # scale: the magnitudes of the terms
    scale = pre * (np.abs(T).max() * (np.abs(dG).max() + np.abs(Chr0).max() + np.abs(Ch).max()))
    return s, K, scale


def grid_around(case, h):
    """A 3x3x3 grid whose cell (1,1,1) is centred on the case's point, the
    metric sampled at every cell centre (ghosts included) and a constant
    primitive state."""
    coord, x0, psi, alpha, beta = metric_case(case)
    p = W.grid(3, coord, [3, 3, 3], [x0[a] - 1.5 * h for a in range(3)], [x0[a] + 1.5 * h for a in range(3)],
               [[W.OUTFLOW, W.OUTFLOW]] * 3, gamma=GAMMA)
    c1, c2, c3 = W.centres(p)
    met = np.zeros((5,) + W.shape(p))
    fns = [sy.lambdify(XS, e, "numpy") for e in [psi, alpha] + list(beta)]
    for w, f in enumerate(fns):
        met[w] = np.broadcast_to(f(c1, c2, c3), met[w].shape)
    return p, met


def state(coord, x0):
    """Primitives (coordinate components) with v and B in every direction."""
    sc = [1.0, 1.0, 1.0]
    if coord == W.SPH:
        sc = [1.0, x0[0], x0[0] * math.sin(x0[1])]
    return np.array([0.9, 0.3 / sc[0], -0.25 / sc[1], 0.2 / sc[2], 0.45, 0.5 / sc[0], 0.35 / sc[1], -0.3 / sc[2]])


def oracle_grav(sources_fn, case, h, kij_exact):
    coord, x0, _, _, _ = metric_case(case)
    p, met = grid_around(case, h)
    prim = np.broadcast_to(state(coord, x0)[:, None, None, None], (8,) + W.shape(p)).copy()
    kij = None
    if kij_exact is not None:
        kij = np.zeros((6,) + W.shape(p))
        for m, (a, b) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
            kij[m] = kij_exact[a, b]
    return sources_fn(p, prim, met, 1, 1, 1, kij)[0]


def pin_error(sources_fn, case, supply_k):
    coord, x0, _, _, _ = metric_case(case)
    s_ex, K, scale = exact_sources(case, state(coord, x0))
    h = 2e-3
    s1 = oracle_grav(sources_fn, case, h, K if supply_k else None)
    s2 = oracle_grav(sources_fn, case, h / 2, K if supply_k else None)
    rich = (4.0 * s2 - s1) / 3.0
    err = np.abs(rich - s_ex)[[1, 2, 3, 4]].max() / scale
    return err, s_ex, rich


CASES = [("cart_general", True), ("sph_general", True), ("cart_rotating", False), ("sph_rotating", False)]


@pytest.mark.parametrize("case,supply_k", CASES)
def test_gravitational_sources_against_4metric(case, supply_k):
    err, s_ex, rich = pin_error(oracle.sources_cell, case, supply_k)
    print(f"  {case}: exact S,tau sources {s_ex[[1, 2, 3, 4]]}, oracle (Richardson) {rich[[1, 2, 3, 4]]}, "
          f"scaled error {err:.2e}")
    # the sources are not small next to their terms (the pin has teeth)
    assert np.abs(s_ex[[1, 2, 3, 4]]).max() > 1e-2 * 1.0
    assert err < 1e-9


def test_rotating_shift_k_equals_stationary_k():
    """For the rotating shifts, the CFC relation under maximal slicing that
    the oracle uses without a supplied K_ij gives the stationary K_ij:
    the rotating cases with and without the exact K agree."""
    for case in ("cart_rotating", "sph_rotating"):
        e1, _, r1 = pin_error(oracle.sources_cell, case, False)
        e2, _, r2 = pin_error(oracle.sources_cell, case, True)
        assert np.abs(r1 - r2).max() < 1e-9 * (np.abs(r1).max() + 1.0)


# ------------------------------------------------------------ planted mistakes

MUTANTS = {
    "k_beta_beta_sign": ("Kbb += TERM(K[a][b] * beta[a] * beta[b]);", "Kbb += TERM(-K[a][b] * beta[a] * beta[b]);"),
    "shift_derivative_index_order": ("for (int m = 0; m < 3; m++) v += TERM(T0d[m] * nb[a][m]);",
                                     "for (int m = 0; m < 3; m++) v += TERM(T0d[m] * nb[m][a]);"),
    "christoffel_index": ("for (int l = 0; l < 3; l++) v += G[m][a][l] * beta[l];",
                          "for (int l = 0; l < 3; l++) v += G[a][m][l] * beta[l];"),
    "dpsi_half": ("v += TERM(0.5 * Tjk * dg * ref[m]);", "v += TERM(Tjk * dg * ref[m]);"),
    "k_beta_factor_two": ("T0K += TERM(T[0][1 + a] * (2.0 * Kb - TERM(dalpha[a])));",
                          "T0K += TERM(T[0][1 + a] * (1.0 * Kb - TERM(dalpha[a])));"),
}


def _mutant_sources(tmp_path, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gmunu_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c), "-lm"])
    L = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    L.og_sources_cell.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]

    def fn(p, prim, met, i, j, k, kij=None):
        d = oracle.make_desc(p)
        prim, met = np.ascontiguousarray(prim), np.ascontiguousarray(met)
        kk = None if kij is None else np.ascontiguousarray(kij)
        g, e = np.zeros(8), np.zeros(8)
        L.og_sources_cell(ctypes.byref(d), prim.ctypes.data_as(P), met.ctypes.data_as(P),
                          None if kk is None else kk.ctypes.data_as(P), i, j, k, g.ctypes.data_as(P),
                          e.ctypes.data_as(P))
        return g, e

    return fn


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_fail_the_pin(tmp_path, name):
    fn = _mutant_sources(tmp_path, name)
    worst = max(pin_error(fn, case, supply_k)[0] for case, supply_k in CASES)
    print(f"  mutant {name}: worst scaled error {worst:.2e}")
    assert worst > 1e-4
