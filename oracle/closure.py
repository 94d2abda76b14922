"""Learned-closure reference: projection between orders, P1 moments, the
per-element MLP and its gradient, in FP64.

Test infrastructure (see ``oracle/__init__``).  Paper context: §3.4 runs the
cylinder case at orders p = 1..4 and initialises order p from order p-1
(p-sequencing); the learned closure uses the same kind of operator between
orders.  Everything below is a reading (R9): the closure is a per-element
network that predicts the P1 part of the difference between the filtered
high-order residual and the low-order residual of the filtered state,
Delta = Pi_1 R_4(U_4) - R_1(Pi_1 U_4).

Definitions:
* P1 moments of a field u on an element: m_a = int phi_a u over the
  reference element, phi_a (a = 0..3) the Gram-Schmidt orthonormalisation of
  (1, xi, eta, zeta), in that order, in the reference L2 inner product;
* projection from order p to order q: the L2 projection in the reference
  element, P = M_q^-1 C, M_q the order-q nodal mass matrix,
  C_ij = int l^q_i l^p_j (exact quadrature);
* features of element e (120): the 5 x 4 moments of e, then of its face
  neighbours in local face order (tets: four faces, a fifth block of zeros);
* network: y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3, 120 -> 64 -> 64 -> 20,
  on normalised inputs (x - mu_x) / s_x, outputs scaled back y * s_y + mu_y;
* the correction to the order-1 residual at the solution points is
  sum_a phi_a(x_i) y_{v,a} for field v.
"""
from __future__ import annotations

import numpy as np

from . import basis, elements

N_IN, N_H, N_OUT = 120, 64, 20
SHAPES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_OUT, N_H), (N_OUT,)]
N_PARAM = sum(int(np.prod(s)) for s in SHAPES)


def _closure_type(name):
    """The closure is defined on tets and prisms (the five-face neighbour
    stencil); other types are refused."""
    if name not in ("tet", "pri"):
        raise ValueError(f"closure not defined on '{name}' elements")
    return name


def _quad(name, deg):
    return basis.tet_quadrature(deg) if _closure_type(name) == "tet" else basis.prism_quadrature(deg)


def _linear_basis(name, x):
    """Orthonormal basis of the linear polynomials on the reference element:
    Gram-Schmidt of (1, xi, eta, zeta), in that order, under the reference
    L2 inner product (equivalently phi = L^-1 m with G = L L^T the Cholesky
    factor of the monomials' Gram matrix)."""
    def mono(y):
        return np.stack([np.ones(len(y)), y[:, 0], y[:, 1], y[:, 2]], axis=-1)
    qx, qw = _quad(name, 2)
    Mq = mono(qx)
    G = np.einsum("q,qa,qb->ab", qw, Mq, Mq)
    Lc = np.linalg.cholesky(G)
    return np.linalg.solve(Lc, mono(np.asarray(x, dtype=np.float64)).T).T


def _lagrange_at(name, p, x):
    """Nodal Lagrange basis of order p evaluated at points x: [n_x][N_u]."""
    ref = elements.get(name, p)
    bfn = basis.tet_basis if _closure_type(name) == "tet" else basis.prism_basis
    return bfn(p, x)[0] @ np.linalg.inv(ref.V)


def moment_operator(name, p):
    """[4][N_u]: P1 moments from nodal values of order p."""
    qx, qw = _quad(name, p + 2)
    phi = _linear_basis(name, qx)                       # [nq][4]
    L = _lagrange_at(name, p, qx)                       # [nq][N_u]
    return np.einsum("q,qa,qi->ai", qw, phi, L)


def lift_operator(name, p):
    """[N_u][4]: nodal values of order p of sum_a phi_a y_a."""
    return _linear_basis(name, elements.get(name, p).upts)


def projection_operator(name, p_src, p_dst):
    """[N_u(p_dst)][N_u(p_src)]: L2 projection in the reference element."""
    qx, qw = _quad(name, p_src + p_dst + 2)
    Ld = _lagrange_at(name, p_dst, qx)
    Ls = _lagrange_at(name, p_src, qx)
    M = np.einsum("q,qi,qj->ij", qw, Ld, Ld)
    C = np.einsum("q,qi,qj->ij", qw, Ld, Ls)
    return np.linalg.solve(M, C)


def project(U, p_src, p_dst):
    """Per-type states [E][N_u][5] from order p_src to order p_dst."""
    return {n: np.einsum("ij,ejv->eiv", projection_operator(n, p_src, p_dst), U[n]) for n in U}


def moments(U, p):
    """Per-type [E][5][4] moments of every field."""
    return {n: np.einsum("ai,eiv->eva", moment_operator(n, p), U[n]) for n in U}


def face_neighbours(mesh):
    """Global element id (type-major) of the neighbour across each local
    face [n_total][5], -1 where the element has no such face; built from the
    oracle's own flux-point pairing."""
    names = [_closure_type(n) for n in mesh.types]
    ntot = sum(mesh.types[n].nelem for n in names)
    base, g = {}, 0
    for n in names:
        base[n] = g
        g += mesh.types[n].nelem
    nb = -np.ones((ntot, 5), dtype=np.int64)

    def owner(gidx):
        for n in names:
            o = mesh.fpt_offset[n]
            tg = mesh.types[n]
            if o <= gidx < o + tg.nelem * tg.ref.nfpts:
                e, j = divmod(gidx - o, tg.ref.nfpts)
                return base[n] + e, int(tg.ref.fpt_face[j])
        raise ValueError(gidx)
    for a, b in zip(mesh.pair_L, mesh.pair_R):
        ea, fa = owner(a)
        eb, fb = owner(b)
        nb[ea, fa] = eb
        nb[eb, fb] = ea
    return nb


def features(mesh, U, p, nb=None):
    """[n_total][120] network inputs (type-major element order)."""
    mom = moments(U, p)
    own = np.concatenate([mom[n].reshape(-1, 20) for n in mesh.types])
    nb = face_neighbours(mesh) if nb is None else nb
    out = np.zeros((len(own), N_IN))
    out[:, :20] = own
    for f in range(5):
        ok = nb[:, f] >= 0
        out[ok, 20 * (f + 1):20 * (f + 2)] = own[nb[ok, f]]
    return out


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(1.0 / N_IN), (N_H, N_IN))
    W2 = rng.normal(0, np.sqrt(1.0 / N_H), (N_H, N_H))
    W3 = rng.normal(0, np.sqrt(1.0 / N_H), (N_OUT, N_H)) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(N_H), W2.ravel(), np.zeros(N_H), W3.ravel(),
                           np.zeros(N_OUT)])


def mlp_forward(theta, x):
    """x [n][120] (already normalised) -> y [n][20], with the activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = x @ W1.T + b1
    h1 = np.tanh(z1)
    z2 = h1 @ W2.T + b2
    h2 = np.tanh(z2)
    y = h2 @ W3.T + b3
    return y, (x, h1, h2)


def mlp_loss_grad(theta, x, target):
    """Mean squared error L = sum (y - t)^2 / n and dL/dtheta by hand-derived
    backpropagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (x, h1, h2) = mlp_forward(theta, x)
    n = len(x)
    dy = 2.0 * (y - target) / n                       # dL/dy
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ W3
    dz2 = dh2 * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (1.0 - h1 * h1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    loss = float(((y - target) ** 2).sum() / n)
    return loss, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def correction(mesh, U, p, theta, stats, nb=None):
    """Per-type nodal correction [E][N_u][5] of the order-p residual."""
    mx, sx, my, sy = stats
    x = (features(mesh, U, p, nb) - mx) / sx
    y, _ = mlp_forward(theta, x)
    y = y * sy + my                                   # [n_total][20] = [5 fields][4 moments]
    out, g = {}, 0
    for n, tg in mesh.types.items():
        E = tg.nelem
        Phi = lift_operator(n, p)                     # [N_u][4]
        out[n] = np.einsum("ia,eva->eiv", Phi, y[g:g + E].reshape(E, 5, 4))
        g += E
    return out


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns the
    new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
