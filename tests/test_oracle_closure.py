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


# --- the network and the correction, against values worked out by hand ----

def _theta(**entries):
    """Parameter vector with the named entries set, every other zero.
    Keys: W1, b1, W2, b2, W3, b3; values: {index: value}."""
    parts = [np.zeros(s) for s in closure.SHAPES]
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    for k, vals in entries.items():
        for idx, v in vals.items():
            parts[names.index(k)][idx] = v
    return np.concatenate([q.ravel() for q in parts])


def test_mlp_forward_hand_computed():
    """y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 on one sample whose hidden
    values are exact: tanh(ln a) = (a^2 - 1) / (a^2 + 1).
    * h1[0] = tanh(W1[0,0] x0) = tanh(ln 2) = 3/5      (x0 = ln 2)
    * h1[1] = tanh(b1[1]) = tanh(ln 3) = 4/5           (bias inside tanh)
    * h1[2] = tanh(W1[2,5] x5) = tanh(ln 3) = 4/5      (x5 = ln 3; W1[5,2]
      stays zero, so a transposed W1 would move the value to h1[5])
    * h2[0] = tanh(W2[0,0] h1[0]) with W2[0,0] = (5/3) ln 2: tanh(ln 2) = 3/5
    * h2[3] = tanh(W2[3,1] h1[1] + W2[3,2] h1[2] + b2[3]) = tanh(ln 3) = 4/5
      with W2[3,1] = W2[3,2] = (5/8) ln 3, b2[3] = 0
    * y[4] = 2 h2[0] + b3[4] = 6/5 + 1/4 = 29/20; y[7] = -h2[3] = -4/5;
      y[9] = b3[9] = -1; every other output 0 (no activation on the output)."""
    ln2, ln3 = math.log(2.0), math.log(3.0)
    th = _theta(W1={(0, 0): 1.0, (2, 5): 1.0}, b1={1: ln3},
                W2={(0, 0): 5.0 / 3.0 * ln2, (3, 1): 0.625 * ln3, (3, 2): 0.625 * ln3},
                W3={(4, 0): 2.0, (7, 3): -1.0}, b3={4: 0.25, 9: -1.0})
    x = np.zeros((1, closure.N_IN))
    x[0, 0], x[0, 5] = ln2, ln3
    y, (_, h1, h2) = closure.mlp_forward(th, x)
    want_h1 = np.zeros(closure.N_H)
    want_h1[[0, 1, 2]] = [0.6, 0.8, 0.8]
    want_h2 = np.zeros(closure.N_H)
    want_h2[[0, 3]] = [0.6, 0.8]
    want_y = np.zeros(closure.N_OUT)
    want_y[[4, 7, 9]] = [29.0 / 20.0, -0.8, -1.0]
    assert np.abs(h1[0] - want_h1).max() < 1e-15
    assert np.abs(h2[0] - want_h2).max() < 1e-15
    assert np.abs(y[0] - want_y).max() < 1e-15


def _linear_basis_closed_form(name, x):
    """Gram-Schmidt of (1, xi, eta, zeta) on the reference element, worked
    out by hand from the simplex integrals int lambda^a = d! a! / (a + d)!:
    tet (volume 4/3, a = xi + 1/2, b = eta + 1/2, c = zeta + 1/2):
      sqrt(3)/2, sqrt(5) a, sqrt(45/8) (b + a/3), sqrt(15/2) (c + a/2 + b/2);
    prism (volume 4, a = xi + 1/3, b = eta + 1/3):
      1/2, 3 a / (2 sqrt 2), sqrt(3/2) (b + a/2), sqrt(3)/2 zeta."""
    xi, eta, zeta = x[:, 0], x[:, 1], x[:, 2]
    if name == "tet":
        a, b, c = xi + 0.5, eta + 0.5, zeta + 0.5
        return np.stack([np.full_like(xi, math.sqrt(3.0) / 2), math.sqrt(5.0) * a,
                         math.sqrt(45.0 / 8.0) * (b + a / 3), math.sqrt(7.5) * (c + a / 2 + b / 2)], -1)
    a, b = xi + 1.0 / 3.0, eta + 1.0 / 3.0
    return np.stack([np.full_like(xi, 0.5), 3 * a / (2 * math.sqrt(2.0)),
                     math.sqrt(1.5) * (b + a / 2), math.sqrt(3.0) / 2 * zeta], -1)


@pytest.mark.parametrize("p", [1, 3])
def test_correction_closed_form(p):
    """The nodal correction of each field is sum_a phi_a(xi_i) y_{v,a}, with
    y = (network output) * s_y + mu_y laid out [5 fields][4 moments]:
    * weights zero, output bias b3 and de-standardisation chosen per field:
      the correction is a known combination of the closed-form basis at the
      solution points, the same for every element of a type;
    * one path through the network: W1[0,0] = W2[0,0] = W3[0,0] = 1 on a
      uniform state of density 1, so the input is the density's first moment
      int phi_0 = sqrt(|ref|) (standardised with mean 0.25, scale 2) and
      y_0 = tanh(tanh((sqrt(|ref|) - 0.25) / 2))."""
    arrays = inputs.small_mixed_box(nxy=2, n_pri_layers=2, n_tet_layers=2, jitter=0.1, seed=4)
    M = omesh.build_mesh(arrays, p)
    U = {n: np.broadcast_to(np.array([1.0, 0.1, -0.2, 0.3, 3.0]), (tg.nelem, tg.ref.nupts, 5)).copy()
         for n, tg in M.types.items()}
    b3 = np.zeros(20)
    b3[0:4] = [2.0, 0.0, 0.0, 0.0]
    b3[4:8] = [0.0, 1.0, 0.0, 0.0]
    b3[8:12] = [0.0, 0.0, 1.0, 0.0]
    b3[12:16] = [0.0, 0.0, 0.0, 1.0]
    b3[16:20] = [1.0, -1.0, 0.5, 0.0]
    sy = np.linspace(0.5, 2.0, 20)
    my = np.linspace(-0.1, 0.1, 20)
    stats = (np.zeros(closure.N_IN), np.ones(closure.N_IN), my, sy)
    C = closure.correction(M, U, p, _theta(b3=dict(enumerate(b3))), stats)
    y = (b3 * sy + my).reshape(5, 4)
    for n, tg in M.types.items():
        phi = _linear_basis_closed_form(n, tg.ref.upts)            # [N_u][4]
        want = phi @ y.T                                             # [N_u][5]
        assert np.abs(C[n] - want[None]).max() < 1e-13, n
    # one path through the three layers
    mx = np.zeros(closure.N_IN)
    mx[0] = 0.25
    sx = np.full(closure.N_IN, 2.0)
    stats = (mx, sx, np.zeros(20), np.ones(20))
    C = closure.correction(M, U, p, _theta(W1={(0, 0): 1.0}, W2={(0, 0): 1.0}, W3={(0, 0): 1.0}), stats)
    for n, tg in M.types.items():
        vol = 4.0 / 3.0 if n == "tet" else 4.0
        y0 = math.tanh(math.tanh((math.sqrt(vol) - 0.25) / 2.0))
        phi = _linear_basis_closed_form(n, tg.ref.upts)
        want = np.zeros((tg.ref.nupts, 5))
        want[:, 0] = phi[:, 0] * y0
        assert np.abs(C[n] - want[None]).max() < 1e-13, n
