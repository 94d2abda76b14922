"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own construction route.

* Table 2 of the paper (dimensions of M0) -> tests/golden/table2_m0_dims.txt
* interpolation / differentiation exact on polynomials of degree <= p
* quadrature weights against closed-form simplex (Dirichlet) integrals
* the lift identity against closed-form volume and face integrals
* point-set symmetry, interiority, unisolvence
* Euler / viscous fluxes against closed forms, Rusanov consistency and
  antisymmetry
* RK45[2R+] against the Runge-Kutta order conditions
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import basis, elements, physics, rk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ORDERS = (1, 2, 3, 4)


def _table2():
    rows = []
    for line in open(os.path.join(GOLDEN, "table2_m0_dims.txt")):
        if line.strip() and not line.startswith("#"):
            t, p, nu, nf = line.split()
            rows.append((t, int(p), int(nu), int(nf)))
    return rows


@pytest.mark.parametrize("row", _table2())
def test_table2_operator_dims(row):
    name, p, nu, nf = row
    R = elements.get(name, p)
    assert R.M0.shape == (nf, nu)
    assert R.nupts == nu == elements.nupts(name, p)
    assert R.nfpts == nf == elements.nfpts(name, p)


def test_gauss_legendre_closed_form():
    x, w = basis.gauss_legendre(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    x, w = basis.gauss_legendre(3)
    assert np.allclose(x, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("p", ORDERS)
def test_point_sets_symmetric_interior_unisolvent(p):
    tri = basis.tri_barycentric(p)
    tet = basis.tet_barycentric(p)
    assert np.allclose(tri.sum(1), 1) and np.allclose(tet.sum(1), 1)
    assert tri.min() > 0.02 and tet.min() > 0.02
    for bary, n in ((tri, 3), (tet, 4)):
        key = {tuple(np.round(b, 12)) for b in bary}
        for perm in itertools.permutations(range(n)):
            assert {tuple(np.round(b[list(perm)], 12)) for b in bary} == key
    for name in ("tet", "pri", "hex"):
        R = elements.get(name, p)
        assert np.linalg.cond(R.V) < 50.0
    # hexahedron: Gauss-Legendre tensor set, invariant under the 48 symmetries
    # of the cube, strictly interior
    H = elements.get("hex", p).upts
    key = {tuple(np.round(x, 12)) for x in H}
    for perm in itertools.permutations(range(3)):
        for sg in itertools.product((-1, 1), repeat=3):
            assert {tuple(np.round(x[list(perm)] * sg, 12) + 0.0) for x in H} == key
    assert np.abs(H).max() < 1.0


def _monomials(name, p):
    """Exponents (a, b, c) of x^a y^b z^c spanning the element's space."""
    if name == "hex":
        return list(itertools.product(range(p + 1), repeat=3))
    out = []
    for a in range(p + 1):
        for b in range(p + 1 - a):
            if name == "tet":
                out += [(a, b, c) for c in range(p + 1 - a - b)]
            else:
                out += [(a, b, c) for c in range(p + 1)]
    return out


@pytest.mark.parametrize("name", ["tet", "pri", "hex"])
@pytest.mark.parametrize("p", ORDERS)
def test_interpolation_and_gradient_exact(name, p):
    R = elements.get(name, p)
    for (a, b, c) in _monomials(name, p):
        def f(x):
            return x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c

        def df(x, k):
            e = [a, b, c]
            if e[k] == 0:
                return np.zeros(len(x))
            e2 = list(e)
            e2[k] -= 1
            return e[k] * x[:, 0] ** e2[0] * x[:, 1] ** e2[1] * x[:, 2] ** e2[2]
        fu = f(R.upts)
        assert np.abs(R.M0 @ fu - f(R.fpts)).max() < 1e-13
        for k in range(3):
            assert np.abs(R.G[k] @ fu - df(R.upts, k)).max() < 5e-13


# --- closed-form integrals over the reference elements and faces ----------

def _dirichlet(exps, measure):
    """int over a simplex of prod lambda_i^e_i = measure * d! prod e_i! / (sum e + d)!"""
    d = len(exps) - 1
    num = math.factorial(d) * math.prod(math.factorial(e) for e in exps)
    return measure * num / math.factorial(sum(exps) + d)


def _zint(c):
    return (1.0 - (-1.0) ** (c + 1)) / (c + 1)


def _tet_lam(x):
    l1, l2, l3 = (1 + x[:, 0]) / 2, (1 + x[:, 1]) / 2, (1 + x[:, 2]) / 2
    return np.stack([1 - l1 - l2 - l3, l1, l2, l3], -1)


def _tet_vol_int(e):          # e = exponents of (l1, l2, l3)
    return _dirichlet((0,) + tuple(e), 4.0 / 3.0)


def _tet_face_int(f, e):
    """int over reference tet face f of l1^e1 l2^e2 l3^e3 (faces as in
    elements.TET_FACES: (0,1,2) l3=0, (0,1,3) l2=0, (0,2,3) l1=0, (1,2,3) l0=0)."""
    zero = {0: 3, 1: 2, 2: 1, 3: 0}[f]         # barycentric index vanishing on f
    full = (0,) + tuple(e)
    if zero > 0 and full[zero] > 0:
        return 0.0
    area = 2.0 * math.sqrt(3.0) if f == 3 else 2.0
    kept = [full[i] for i in range(4) if i != zero]
    return _dirichlet(tuple(kept), area)


def _pri_vol_int(e):          # exponents of (l1, l2, z)
    return _dirichlet((0, e[0], e[1]), 2.0) * _zint(e[2])


def _pri_face_int(f, e):
    a, b, c = e
    if f == 0:
        return _dirichlet((0, a, b), 2.0) * (-1.0) ** c
    if f == 1:
        return _dirichlet((0, a, b), 2.0)
    if f == 2:        # eta = -1: l2 = 0, xi in [-1,1] -> l1 in [0,1], d(xi) = 2 d(l1)
        return 0.0 if b else 2.0 / (a + 1) * _zint(c)
    if f == 3:        # xi + eta = 0: l1 + l2 = 1, edge length 2 sqrt 2
        return (2.0 * math.sqrt(2.0) * math.factorial(a) * math.factorial(b)
                / math.factorial(a + b + 1) * _zint(c))
    return 0.0 if a else 2.0 / (b + 1) * _zint(c)     # xi = -1


def _hex_vol_int(e):          # exponents of (x, y, z) on [-1, 1]^3
    return _zint(e[0]) * _zint(e[1]) * _zint(e[2])


def _hex_face_int(f, e):
    """Faces as in elements.HEX_FACES: t = -1, t = +1, s = -1, r = +1, s = +1, r = -1."""
    a, b, c = e
    axis, side = [(2, -1), (2, 1), (1, -1), (0, 1), (1, 1), (0, -1)][f]
    out = 1.0
    for k, ek in enumerate(e):
        out *= float(side) ** ek if k == axis else _zint(ek)
    return out


def _lam_monos(name, p):
    if name == "hex":
        return _monomials("hex", p)
    out = []
    for a in range(p + 1):
        for b in range(p + 1 - a):
            rng = range(p + 1 - a - b) if name == "tet" else range(p + 1)
            out += [(a, b, c) for c in rng]
    return out


def _lam_eval(name, x, e):
    if name == "hex":
        return x[:, 0] ** e[0] * x[:, 1] ** e[1] * x[:, 2] ** e[2]
    if name == "tet":
        lam = _tet_lam(x)
        return lam[:, 1] ** e[0] * lam[:, 2] ** e[1] * lam[:, 3] ** e[2]
    return ((1 + x[:, 0]) / 2) ** e[0] * ((1 + x[:, 1]) / 2) ** e[1] * x[:, 2] ** e[2]


_VOL = {"tet": _tet_vol_int, "pri": _pri_vol_int, "hex": _hex_vol_int}
_FACE = {"tet": _tet_face_int, "pri": _pri_face_int, "hex": _hex_face_int}


@pytest.mark.parametrize("name", ["tet", "pri", "hex"])
@pytest.mark.parametrize("p", ORDERS)
def test_quadrature_weights_closed_form(name, p):
    R = elements.get(name, p)
    vol = _VOL[name]
    assert abs(R.w.sum() - R.volume) < 1e-13
    for e in _lam_monos(name, p):
        assert abs(R.w @ _lam_eval(name, R.upts, e) - vol(e)) < 1e-13


@pytest.mark.parametrize("name", ["tet", "pri", "hex"])
@pytest.mark.parametrize("p", ORDERS)
def test_lift_identity_closed_form(name, p):
    """int phi (L g) = sum_f int_f phi g ds for phi in the solution space and
    g the face trace of a polynomial of the solution space."""
    R = elements.get(name, p)
    vol = _VOL[name]
    face = _FACE[name]
    monos = _lam_monos(name, p)
    Vm = np.stack([_lam_eval(name, R.upts, e) for e in monos], -1)    # [N_u][n_monos]
    rng = np.random.default_rng(3)
    for _ in range(6):
        ephi = monos[rng.integers(len(monos))]
        eh = monos[rng.integers(len(monos))]
        g = _lam_eval(name, R.fpts, eh)
        coef = np.linalg.solve(Vm, R.L @ g)                          # Lg in monomials
        lhs = sum(cm * vol(tuple(np.add(ephi, em))) for cm, em in zip(coef, monos))
        rhs = sum(face(f, tuple(np.add(ephi, eh))) for f in range(len(R.faces)))
        assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(rhs)), (ephi, eh, lhs, rhs)


# --- fluxes ---------------------------------------------------------------

G = 1.4


def test_inviscid_flux_closed_form():
    rho, u, v, w, p = 1.3, 0.4, -0.7, 0.2, 2.1
    E = p / (G - 1) + 0.5 * rho * (u * u + v * v + w * w)
    U = np.array([rho, rho * u, rho * v, rho * w, E])[:, None]
    F = physics.inviscid_flux(U, G)[..., 0]
    vel = [u, v, w]
    for j in range(3):
        want = [rho * vel[j]] + [rho * vel[i] * vel[j] + (p if i == j else 0) for i in range(3)] \
            + [(E + p) * vel[j]]
        assert np.allclose(F[j], want, rtol=1e-15, atol=1e-15)


def _rand_states(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2, n)
    vel = rng.uniform(-1, 1, (3, n))
    p = rng.uniform(0.5, 2, n)
    E = p / (G - 1) + 0.5 * rho * (vel ** 2).sum(0)
    return np.concatenate([rho[None], rho * vel, E[None]])


def test_rusanov_consistency_antisymmetry():
    UL, UR = _rand_states(50, 1), _rand_states(50, 2)
    n = np.random.default_rng(3).normal(size=(3, 50))
    n /= np.linalg.norm(n, axis=0)
    same = physics.rusanov(UL, UL, n, G)
    assert np.allclose(same, physics.normal_flux(physics.inviscid_flux(UL, G), n), atol=1e-14)
    assert np.allclose(physics.rusanov(UL, UR, n, G), -physics.rusanov(UR, UL, -n, G), atol=1e-14)
    # closed form: two states at rest, pressures 1 and 2, unit density
    UL1 = np.array([1.0, 0, 0, 0, 1.0 / (G - 1)])[:, None]
    UR1 = np.array([1.0, 0, 0, 0, 2.0 / (G - 1)])[:, None]
    nx = np.array([1.0, 0, 0])[:, None]
    lam = math.sqrt(G * 2.0)
    want = [0.0, 1.5, 0.0, 0.0, -0.5 * lam * (1.0 / (G - 1))]
    assert np.allclose(physics.rusanov(UL1, UR1, nx, G)[:, 0], want, atol=1e-15)


def test_viscous_flux_closed_form():
    """Linear velocity and temperature fields with a uniform density."""
    mu, pr = 0.03, 0.71
    rho, p = 1.1, 0.8
    A = np.array([[0.1, 0.3, -0.2], [0.05, -0.4, 0.7], [0.2, 0.1, 0.25]])   # dv_i/dx_j
    gT = np.array([0.3, -0.1, 0.2])                                          # d(p/rho)/dx_j
    v = np.array([0.4, -0.3, 0.2])
    E = p / (G - 1) + 0.5 * rho * v @ v
    U = np.array([rho, *(rho * v), E])[:, None]
    # conserved gradients with d(rho)/dx = 0: d(rho v_i) = rho A_ij;
    # dE/dx_j = rho d(p/rho)/dx_j / (G-1) + rho v_i A_ij
    Q = np.zeros((3, 5, 1))
    for j in range(3):
        Q[j, 1:4, 0] = rho * A[:, j]
        Q[j, 4, 0] = rho * gT[j] / (G - 1) + rho * v @ A[:, j]
    Fv = physics.viscous_flux(U, Q, G, mu, pr)[..., 0]
    tau = mu * (A + A.T - 2 / 3 * np.trace(A) * np.eye(3))
    kappa = mu * G / (pr * (G - 1))
    for j in range(3):
        assert np.allclose(Fv[j, 1:4], tau[:, j], atol=1e-15)
        assert abs(Fv[j, 4] - (v @ tau[:, j] + kappa * gT[j])) < 1e-14
        assert Fv[j, 0] == 0
    assert np.abs(physics.viscous_flux(U, np.zeros((3, 5, 1)), G, mu, pr)).max() == 0


# --- time stepping --------------------------------------------------------

def test_rk45_order_conditions():
    """The eight fourth-order conditions of RK45[2R+] and the four
    third-order conditions of its embedded solution."""
    A, b, bh, c = rk.rk45_butcher()
    assert np.allclose(A.sum(1), c)
    conds = [(b.sum(), 1), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ A @ c, 1 / 6),
             (b @ c ** 3, 1 / 4), (b @ (c * (A @ c)), 1 / 8), (b @ A @ c ** 2, 1 / 12),
             (b @ A @ A @ c, 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 1e-14
    for got, want in [(bh.sum(), 1), (bh @ c, 1 / 2), (bh @ c ** 2, 1 / 3), (bh @ A @ c, 1 / 6)]:
        assert abs(got - want) < 1e-14
    # it is genuinely an embedded pair, not a copy
    assert np.abs(b - bh).max() > 1e-3


def test_controller_factors_by_hand():
    """The PI step-size factors of the adaptive RK45[2R+] (k = 4, safety 0.9,
    factor clamped to [0.2, 5], at most 1 after a rejection), worked out by
    hand on error values whose powers are exact:
    * accepted, err = 1e-2, err_prev = 1e-1:
      0.9 (1e-2)^(-0.7/4) (1e-1)^(0.4/4) = 0.9 10^(0.35 - 0.1) = 0.9 10^0.25;
    * accepted, err = err_prev = 1: 0.9;
    * accepted, err = 1e-8, err_prev = 1e-4: 0.9 10^(1.4 - 0.4) = 9 -> 5;
    * accepted, err = 0: the maximum factor 5;
    * accepted, err = 1, err_prev = 1e-12 (below any floor): 0.9 10^-1.2 =
      0.0568 -> 0.2;
    * rejected, err = 16: 0.9 16^(-1/4) = 0.45;
    * rejected, err = 1e4: 0.9 10^-1 = 0.09 -> 0.2;
    * rejected, err = 1 + 1e-12: 0.9 (1 + 1e-12)^(-1/4) < 1, ~0.9."""
    cases = [((1e-2, 1e-1, True), 0.9 * 10 ** 0.25), ((1.0, 1.0, True), 0.9),
             ((1e-8, 1e-4, True), 5.0), ((0.0, 0.5, True), 5.0), ((1.0, 1e-12, True), 0.2),
             ((16.0, 1.0, False), 0.45), ((1e4, 1.0, False), 0.2), ((1.0 + 1e-12, 1.0, False), 0.9)]
    for (err, prev, acc), want in cases:
        got = rk.controller(err, prev, acc)
        assert abs(got - want) < 1e-12, (err, prev, acc, got, want)


def test_adaptive_err_prev_floor():
    """After an accepted step the controller's memory is max(err, 1e-4):
    y' = 0 has zero embedded error on every step, so each accepted step
    leaves err_prev = 1e-4 and grows dt by the maximum factor 5."""
    U = {"x": np.ones((2, 3, 5))}
    out = rk.rk45_adaptive(lambda V: {n: np.zeros_like(V[n]) for n in V}, U, 0.0, 10.0, 0.01, 1e-6, 1e-6)
    _, t, dt, err_prev, n_acc, n_rej, errs = out
    assert t == 10.0 and n_rej == 0 and err_prev == 1e-4 and max(errs) == 0.0
    # steps 0.01, 0.05, 0.25, 1.25, 6.25 (t = 7.81), then the last step is cut
    # to 10 - 7.81 and the next dt is five times that
    assert n_acc == 6 and abs(dt - 5.0 * (10.0 - (0.01 + 0.05 + 0.25 + 1.25 + 6.25))) < 1e-12


@pytest.mark.parametrize("stepper,order", [(rk.rk4_step, 4), (rk.rk45_step, 4),
                                           (rk.euler_step, 1)])
def test_rk_observed_order(stepper, order):
    lam = -1.3 + 0.7j

    def f(U):
        return {"y": lam * U["y"]}
    errs = []
    for n in (10, 20, 40):
        dt = 1.0 / n
        U = rk.run(stepper, f, {"y": np.array([1.0 + 0j])}, dt, n)
        errs.append(abs(U["y"][0] - np.exp(lam)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > order - 0.2).all(), rates


def test_rk45_two_register_matches_butcher():
    """The two-register form reproduces the full Butcher-tableau step."""
    A, b, _, _ = rk.rk45_butcher()
    M = np.array([[-0.3, 0.8], [-0.5, -0.2]])

    def f(U):
        return {"y": M @ U["y"]}
    y0 = np.array([1.0, -0.5])
    dt = 0.37
    k = []
    for i in range(5):
        Y = y0 + dt * sum(A[i, j] * k[j] for j in range(i)) if i else y0
        k.append(M @ Y)
    want = y0 + dt * sum(b[j] * k[j] for j in range(5))
    got = rk.rk45_step(f, {"y": y0}, dt)["y"]
    assert np.allclose(got, want, atol=1e-15)


# ---------------------------------------------------------------------------
# Adaptive RK45[2R+] (reading R10)
# ---------------------------------------------------------------------------

def test_embedded_error_is_difference_of_butcher_solutions():
    """The two-register error accumulation equals u(b) - u(bhat) of the
    Butcher tableau, on a nonlinear system."""
    from oracle import rk
    A, b, bhat, c = rk.rk45_butcher()
    f = lambda U: {"x": np.stack([U["x"][1], -np.sin(U["x"][0]) - 0.1 * U["x"][1]])}
    U = {"x": np.array([1.2, -0.4])}
    dt = 0.3
    k = []
    for i in range(5):
        Y = U["x"] + dt * sum(A[i, j] * k[j] for j in range(i))
        k.append(f({"x": Y})["x"])
    ub = U["x"] + dt * sum(b[i] * k[i] for i in range(5))
    uh = U["x"] + dt * sum(bhat[i] * k[i] for i in range(5))
    q, e = rk.rk45_step_with_error(f, U, dt)
    assert np.allclose(q["x"], ub, rtol=0, atol=1e-14)
    assert np.allclose(e["x"], ub - uh, rtol=0, atol=1e-14)


def test_embedded_error_is_third_order_local():
    """e = O(dt^4) on y' = y: halving dt divides it by ~16."""
    from oracle import rk
    f = lambda U: {"y": U["y"]}
    e1 = abs(rk.rk45_step_with_error(f, {"y": np.array([1.0])}, 0.2)[1]["y"][0])
    e2 = abs(rk.rk45_step_with_error(f, {"y": np.array([1.0])}, 0.1)[1]["y"][0])
    assert 13.0 < e1 / e2 < 19.0


def test_adaptive_error_tracks_tolerance():
    """On y' = -y + sin(3t) (exact solution known), the adaptive driver lands
    on t_end, rejects nothing once settled, and its global error falls with
    the tolerance and stays within a modest multiple of it."""
    from oracle import rk
    def exact(t):
        # y' = -y + sin 3t, y(0) = 1
        return (np.sin(3 * t) - 3 * np.cos(3 * t)) / 10 + 1.3 * np.exp(-t)
    state = {"t": 0.0}
    prev = None
    for tol in (1e-4, 1e-6, 1e-8):
        def f(U, _s=state):
            return {"y": -U["y"] + np.sin(3 * U["ty"]), "ty": np.ones(1)}
        U = {"y": np.array([1.0]), "ty": np.array([0.0])}
        U, t, dt, ep, na, nr, errs = rk.rk45_adaptive(f, U, 0.0, 5.0, 0.01, tol, tol)
        assert t == 5.0 and abs(U["ty"][0] - 5.0) < 1e-12
        g = abs(U["y"][0] - exact(5.0))
        assert g < 50 * tol
        if prev is not None:
            assert g < prev and na > prev_na
        prev, prev_na = g, na
