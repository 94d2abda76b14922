"""Pins of the closure reference (projection between orders, P1 moments,
the network's gradient) against closed forms and finite differences."""
import math

import numpy as np
import pytest

from oracle import closure, elements, mesh as omesh
from paper_1409_0405_amd import inputs

import test_oracle_pins as P


@pytest.mark.parametrize("name", ["tet", "pri"])
@pytest.mark.parametrize("p_src", [2, 4])
def test_projection_closed_form_orthogonality(name, p_src):
    """u - Pu is orthogonal to the order-1 space, with closed-form integrals
    of barycentric monomials; P reproduces order-1 data."""
    Pm = closure.projection_operator(name, p_src, 1)
    R1 = elements.get(name, 1)
    Rp = elements.get(name, p_src)
    vol = P._tet_vol_int if name == "tet" else P._pri_vol_int
    monos1 = P._lam_monos(name, 1)
    V1 = np.stack([P._lam_eval(name, R1.upts, e) for e in monos1], -1)
    for eu in P._lam_monos(name, p_src):
        u = P._lam_eval(name, Rp.upts, eu)
        coef = np.linalg.solve(V1, Pm @ u)                 # Pu in order-1 monomials
        for ephi in monos1:
            lhs = vol(tuple(np.add(eu, ephi)))
            rhs = sum(c * vol(tuple(np.add(em, ephi))) for c, em in zip(coef, monos1))
            assert abs(lhs - rhs) < 1e-12
        if eu in monos1:
            assert np.allclose(Pm @ u, P._lam_eval(name, R1.upts, eu), atol=1e-13)


@pytest.mark.parametrize("name", ["tet", "pri"])
def test_moments_reproduce_linear_functions(name):
    """sum_a m_a phi_a reproduces any linear function; the basis is
    orthonormal (closed-form monomial integrals)."""
    R = elements.get(name, 3)
    Mom = closure.moment_operator(name, 3)
    rng = np.random.default_rng(1)
    test_x = R.fpts
    for _ in range(5):
        c = rng.normal(size=4)
        u = c[0] + R.upts @ c[1:]
        m = Mom @ u
        rec = closure._linear_basis(name, test_x) @ m
        assert np.allclose(rec, c[0] + test_x @ c[1:], atol=1e-12)
    # orthonormality against closed forms: phi = L^-1 (1, xi, eta, zeta)
    vol = P._tet_vol_int if name == "tet" else P._pri_vol_int
    # monomials in barycentrics: 1, xi = 2 l1 - 1, eta = 2 l2 - 1, zeta
    if name == "tet":
        e = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
        to_mono = np.array([[1, 0, 0, 0], [-1, 2, 0, 0], [-1, 0, 2, 0], [-1, 0, 0, 2]], float)
    else:
        e = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
        to_mono = np.array([[1, 0, 0, 0], [-1, 2, 0, 0], [-1, 0, 2, 0], [0, 0, 0, 1]], float)
    Gl = np.array([[vol(tuple(np.add(a, b))) for b in e] for a in e])
    G = to_mono @ Gl @ to_mono.T                       # Gram of (1, xi, eta, zeta)
    Lc = np.linalg.cholesky(G)
    x = R.upts
    phi_closed = np.linalg.solve(Lc, np.stack([np.ones(len(x)), x[:, 0], x[:, 1], x[:, 2]]) ).T
    assert np.allclose(closure._linear_basis(name, x), phi_closed, atol=1e-13)


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(4)
    theta = closure.init_params(3) + 0.05 * rng.normal(size=closure.N_PARAM)
    x = rng.normal(size=(7, closure.N_IN))
    t = rng.normal(size=(7, closure.N_OUT))
    _, g = closure.mlp_loss_grad(theta, x, t)
    idx = rng.choice(closure.N_PARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (closure.mlp_loss_grad(tp, x, t)[0] - closure.mlp_loss_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_face_neighbours_symmetric():
    arrays = inputs.small_mixed_box(nxy=3, n_pri_layers=2, n_tet_layers=2, jitter=0.1)
    M = omesh.build_mesh(arrays, 1)
    nb = closure.face_neighbours(M)
    nt = M.types["tet"].nelem
    assert (nb[:nt, 4] == -1).all() and (nb[:nt, :4] >= 0).all() and (nb[nt:] >= 0).all()
    for e in range(len(nb)):
        for f in range(5):
            if nb[e, f] >= 0:
                assert e in nb[nb[e, f]]


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step moves every parameter by
    lr * g / (|g| + eps): a signed step of size lr where |g| >> eps."""
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = closure.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    bound = 1e-3 * 1e-8 / np.abs(g) + 1e-15           # lr eps / |g|
    assert (np.abs(new - (th - 1e-3 * np.sign(g))) <= bound).all()
    # a constant gradient keeps the step at lr (bias corrections cancel)
    for t in range(2, 6):
        new, m, v = closure.adam_step(new, g, m, v, t, 1e-3)
    assert (np.abs(new - (th - 5e-3 * np.sign(g))) <= 5 * bound + 1e-14).all()
