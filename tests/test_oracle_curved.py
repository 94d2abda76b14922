"""Pins of the oracle's quadratically curved geometry (reading R12: the
quadratic Lagrange map of nodes on the element's order-2 lattice):

* the shape functions are nodal, sum to one and reproduce every quadratic
  polynomial and its gradient (closed forms) on all three types;
* a quadratic shear x' = x + c y (Ly - y) of a wall-bounded three-type box
  is represented exactly: J = 1 at every solution point and the volume is
  the box's;
* freestream on curved tets at p >= 2 (the adjugate of a quadratic map is
  quadratic, so it is interpolated exactly), and on curved hexahedra and
  prisms where it holds (p >= 2, p >= 3);
* discrete conservation on a curved periodic three-type box for any state;
* design-order convergence of the travelling density wave on curved tets.
"""
import math

import numpy as np
import pytest

from oracle import fr, mesh as omesh, reduce, rk
from paper_1409_0405_amd import inputs

L = (6.0, 7.0, 5.5)


@pytest.mark.parametrize("name", ["tet", "pri", "hex"])
def test_quadratic_shape_functions(name):
    q = omesh.quadratic_nodes(name)
    N, _ = omesh.quadratic_shape_functions(name, q)
    assert np.abs(N - np.eye(len(q))).max() < 1e-13
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.9, 0.1, (40, 3)) if name == "tet" else rng.uniform(-0.95, 0.95, (40, 3))
    if name == "pri":
        x[:, 1] = np.minimum(x[:, 1], -x[:, 0])          # inside the triangle
    N, dN = omesh.quadratic_shape_functions(name, x)
    assert np.abs(N.sum(axis=1) - 1).max() < 1e-13
    # a quadratic of the element's order-2 space and its gradient
    f = lambda y: 0.3 + y[:, 0] - 2 * y[:, 1] * y[:, 2] + 0.7 * y[:, 0] ** 2 + 0.4 * y[:, 2] ** 2
    g = lambda y: np.stack([1 + 1.4 * y[:, 0], -2 * y[:, 2], -2 * y[:, 1] + 0.8 * y[:, 2]], -1)
    assert np.abs(N @ f(q) - f(x)).max() < 1e-13
    assert np.abs(np.einsum("pnk,n->pk", dN, f(q)) - g(x)).max() < 1e-12


def _sheared_wall_box(c=0.05, seed=2):
    """Wall-bounded three-type box under x' = x + c y (Ly - y): quadratic
    in y, zero at the walls, periodic in x, volume preserving."""
    a = inputs.hybrid_box(4, 3, 4, 2, 2, L, jitter=0.1, seed=seed, y_bc="wall")
    Ly = L[1]
    phi = lambda X: np.concatenate([X[..., :1] + c * X[..., 1:2] * (Ly - X[..., 1:2]), X[..., 1:]], -1)
    out = dict(a, xyz=phi(a["xyz"]))
    for kind in ("tet", "pri", "hex"):
        X = a["xyz"][a[f"{kind}_v"]] + a[f"{kind}_img"].astype(np.float64) * a["period"]
        out[f"{kind}_q"] = phi(inputs._straight_points(kind, X, inputs._order2_lattice(kind)))
    return out


@pytest.mark.parametrize("p", (1, 3))
def test_exact_quadratic_shear(p):
    M = omesh.build_mesh(_sheared_wall_box(), p)
    vol = sum((tg.J_upts * tg.ref.w).sum() for tg in M.types.values())
    straight = omesh.build_mesh(inputs.hybrid_box(4, 3, 4, 2, 2, L, jitter=0.1, seed=2, y_bc="wall"), p)
    for n, tg in M.types.items():
        # the shear keeps each point's Jacobian determinant
        assert np.abs(tg.J_upts - straight.types[n].J_upts).max() < 1e-12 * np.abs(tg.J_upts).max()
    assert abs(vol - np.prod(L)) < 1e-11


@pytest.mark.parametrize("kind,p", [("tet", 2), ("tet", 3), ("tet", 4), ("hex", 2), ("hex", 4), ("pri", 3),
                                    ("pri", 4)])
def test_curved_freestream(kind, p):
    if kind == "tet":
        a = inputs.vortex_tet_cube(n=3, jitter=0.05)
    elif kind == "hex":
        a = inputs.hex_box(3, lengths=L, jitter=0.05)
    else:
        a = inputs.mixed_box(3, 3, 3, 0, L, jitter=0.05)
    M = omesh.build_mesh(inputs.curve(a, 0.03), p)
    for system in ("euler", "ns"):
        R = fr.rhs(M, fr.initial_state(M, inputs.uniform), fr.Params(system=system, mu=0.05))
        assert max(np.abs(R[n]).max() for n in R) < 1e-11


@pytest.mark.parametrize("p", (1, 2, 4))
def test_curved_conservation(p):
    M = omesh.build_mesh(inputs.curve(inputs.hybrid_box(4, 3, 4, 2, 2, L, jitter=0.1, seed=3), 0.03), p)
    U = fr.initial_state(M, inputs.taylor_green, mach=0.3)
    for n in U:
        U[n] = U[n] * inputs.random_perturbation(U[n].shape, 5, 0.05)
    R = fr.rhs(M, U, fr.Params(system="ns", mu=0.02))
    tot = reduce.integral(M, R)
    scale = reduce.integral(M, {n: np.abs(R[n]) for n in R})
    assert np.all(np.abs(tot) <= 1e-12 * scale), tot / scale


@pytest.mark.parametrize("p", (1, 2))
def test_curved_density_wave_convergence(p):
    kw = dict(direction=(1, 0, 0), vel=(1.0, 0.3, 0.2))
    errs = []
    t_end = 0.1
    for n in (3, 6):
        M = omesh.build_mesh(inputs.curve(inputs.vortex_tet_cube(n=n, jitter=0.05), 0.02), p)
        U = fr.initial_state(M, inputs.density_wave, **kw)
        prm = fr.Params(system="euler")
        nsteps = int(math.ceil(t_end / (0.3 / (n * (2 * p + 1) * 2.0))))
        U = rk.run(rk.rk4_step, lambda V: fr.rhs(M, V, prm), U, t_end / nsteps, nsteps)
        Ue = fr.initial_state(M, inputs.density_wave, t=t_end, **kw)
        errs.append(reduce.l2_norm(M, {k: U[k] - Ue[k] for k in U})[0])
    rate = math.log2(errs[0] / errs[1])
    assert rate >= p + 0.5, (errs, rate)
