"""Pins of the oracle's wall and far-field boundary conditions (reading R11:
weak imposition through a boundary state and a ghost state) on boxes bounded
in y and periodic in x and z:

* far-field freestream: a free stream crossing both boundaries (inflow at
  y = 0, outflow at y = Ly) leaves a zero residual, Euler and NS;
* wall at rest: fluid at rest at the wall temperature leaves a zero residual;
* discrete conservation with boundaries: the integral of the residual equals
  minus the boundary flux summed with the reference face weights
  (w^T L, the lift's integral of the face data); no mass crosses a wall;
* the wall's viscous terms against closed forms: a half-wave shear flow and
  a half-wave temperature profile vanishing at the walls give
  d(rho u)/dt = -mu A (pi/Ly)^2 sin(pi y/Ly) and
  dE/dt = -kappa a (pi/Ly)^2 sin(pi y/Ly) at t = 0, approached with p;
* the far-field state keeps the outgoing Riemann invariant of the interior,
  the incoming one of the free stream, and the entropy and tangential
  velocity of the upwind side.
"""
import math

import numpy as np
import pytest

from oracle import elements, fr, mesh as omesh, physics, reduce
from paper_1409_0405_amd import inputs

L = (6.0, 7.0, 5.5)
G = 1.4


def _box(p, bc, seed=5, jitter=0.12, n=(4, 3, 4)):
    a = inputs.hybrid_box(n[0], n[1], n[2], n[0] // 2, n[2] // 2, L, jitter=jitter, seed=seed, y_bc=bc)
    return omesh.build_mesh(a, p)


FREE = (1.2, 0.3, 0.4, -0.1, 0.9)      # rho, u, v, w, p: v > 0 enters at y = 0, leaves at y = Ly


@pytest.mark.parametrize("p", (1, 2, 3, 4))
@pytest.mark.parametrize("system", ["euler", "ns"])
def test_farfield_freestream(p, system):
    M = _box(p, "farfield")
    prm = fr.Params(system=system, mu=0.03, farfield=FREE)
    U = fr.initial_state(M, inputs.uniform, rho=FREE[0], u=FREE[1], v=FREE[2], w=FREE[3], p=FREE[4])
    R = fr.rhs(M, U, prm)
    assert max(np.abs(R[n]).max() for n in R) < 1e-12


@pytest.mark.parametrize("p", (1, 3))
@pytest.mark.parametrize("system", ["euler", "ns"])
def test_wall_at_rest(p, system):
    M = _box(p, "wall")
    prm = fr.Params(system=system, mu=0.03, t_wall=0.75)
    U = fr.initial_state(M, inputs.uniform, rho=1.2, u=0.0, v=0.0, w=0.0, p=0.9)   # p / rho = 0.75
    R = fr.rhs(M, U, prm)
    assert max(np.abs(R[n]).max() for n in R) < 1e-12


def _face_weights(M):
    """Reference face weight of every flux point, global flux order."""
    out = np.zeros(M.nfpts_total)
    for n, tg in M.types.items():
        om = tg.ref.w @ tg.ref.L
        o = M.fpt_offset[n]
        out[o:o + tg.nelem * tg.ref.nfpts] = np.tile(om, tg.nelem)
    return out


@pytest.mark.parametrize("bc", ["wall", "farfield"])
@pytest.mark.parametrize("p", (1, 2, 4))
def test_conservation_equals_boundary_flux(bc, p):
    M = _box(p, bc, seed=7)
    prm = fr.Params(system="ns", mu=0.02, t_wall=1.0, farfield=FREE)
    U = fr.initial_state(M, inputs.taylor_green, mach=0.3)
    for n in U:
        U[n] = U[n] * inputs.random_perturbation(U[n].shape, 11, 0.05)
    want = {}
    R = fr.rhs(M, U, prm, want=want)
    tot = reduce.integral(M, R)
    Fn = np.concatenate([want["Fn"][n].reshape(-1, 5) for n in M.types])
    bflux = (_face_weights(M)[M.bnd_idx, None] * Fn[M.bnd_idx]).sum(axis=0)
    scale = reduce.integral(M, {n: np.abs(R[n]) for n in R})
    assert np.all(np.abs(tot + bflux) <= 1e-12 * scale), (tot, bflux)
    if bc == "wall":
        assert abs(tot[0]) <= 1e-12 * scale[0]          # no mass through a wall
        assert np.abs(bflux[1:]).max() > 1e-6 * scale[1:].max()   # but momentum and energy do cross


def _wall_decay_errors(kind, mu=0.5, pr=0.71):
    errs = []
    Ly = L[1]
    kappa = mu * G / (pr * (G - 1.0))
    for p in (2, 3, 4):
        M = _box(p, "wall", jitter=0.05, n=(4, 4, 4))
        if kind == "shear":
            A, pres = 1e-2, 1.0
            U = fr.initial_state(M, inputs.shear_wave, amp=A, Ly=2 * Ly, p=pres)
            prm = fr.Params(system="ns", mu=mu, prandtl=pr, t_wall=pres)
            field, coef = 1, -mu * A
        else:
            a = 1e-2
            U = fr.initial_state(M, inputs.thermal_wave, amp=a, Ly=2 * Ly)
            prm = fr.Params(system="ns", mu=mu, prandtl=pr, t_wall=1.0)
            field, coef = 4, -kappa * a
        R = fr.rhs(M, U, prm)
        want = {n: coef * (math.pi / Ly) ** 2 * np.sin(math.pi * M.types[n].x_upts[..., 1] / Ly)
                for n in M.types}
        err = reduce.l2_norm(M, {n: R[n][..., field] - want[n] for n in R})
        errs.append(err / reduce.l2_norm(M, want))
    return errs


@pytest.mark.parametrize("kind", ["shear", "thermal"])
def test_wall_viscous_closed_forms(kind):
    errs = _wall_decay_errors(kind)
    assert errs[-1] < 0.05 and errs[0] > errs[1] > errs[2], errs


def test_farfield_state_riemann_invariants():
    rng = np.random.default_rng(2)
    n = rng.normal(size=(3, 400))
    n /= np.linalg.norm(n, axis=0)
    rho = rng.uniform(0.8, 1.2, 400)
    v = rng.uniform(-0.3, 0.3, (3, 400))
    p = rng.uniform(0.6, 0.9, 400)
    UL = np.concatenate([rho[None], rho * v, (p / (G - 1) + 0.5 * rho * (v * v).sum(0))[None]])
    Ub = physics.farfield_state(UL, n, G, FREE)
    rb, vb, pb = physics.primitives(Ub, G)
    cb, cL = np.sqrt(G * pb / rb), np.sqrt(G * p / rho)
    vf = np.array(FREE[1:4])[:, None]
    cf = math.sqrt(G * FREE[4] / FREE[0])
    vnb, vnL, vnf = (vb * n).sum(0), (v * n).sum(0), (vf * n).sum(0)
    assert np.allclose(vnb + 2 * cb / (G - 1), vnL + 2 * cL / (G - 1), atol=1e-13)
    assert np.allclose(vnb - 2 * cb / (G - 1), vnf - 2 * cf / (G - 1), atol=1e-13)
    out = vnb > 0
    assert 50 < out.sum() < 350
    ent_b = pb / rb ** G
    assert np.allclose(ent_b[out], (p / rho ** G)[out], rtol=1e-13)
    assert np.allclose(ent_b[~out], FREE[4] / FREE[0] ** G, rtol=1e-13)
    vt = vb - vnb * n
    assert np.allclose(vt[:, out], (v - vnL * n)[:, out], atol=1e-13)
    assert np.allclose(vt[:, ~out], (vf - vnf * n)[:, ~out], atol=1e-13)


def test_unlisted_boundary_face_is_an_error():
    a = inputs.hybrid_box(4, 3, 4, 2, 2, L, jitter=0.1, seed=1, y_bc="wall")
    a["bfaces"] = a["bfaces"][1:]
    with pytest.raises(ValueError):
        omesh.build_mesh(a, 1)
