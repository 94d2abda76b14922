"""Point-wise physics: Euler and Navier-Stokes fluxes, Rusanov and LDG.

Test infrastructure (see ``oracle/__init__``).

Paper, Section 3.4: compressible Navier-Stokes with constant viscosity,
a Rusanov Riemann solver for the inviscid interface flux.  Readings (R5,
R6): ideal gas, Stokes hypothesis, heat flux from a constant
Prandtl number; local Lax-Friedrichs wave speed max(|v.n|+c) over both
sides; the viscous interface flux is local DG (LDG) with switch beta and
penalty tau.

State arrays have the five conserved fields (rho, rho u, rho v, rho w, E) on
the first axis; gradients have shape [3][5][...] (direction first).
"""
from __future__ import annotations

import numpy as np


def primitives(U, gamma):
    rho = U[0]
    v = U[1:4] / rho
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * (v * v).sum(axis=0))
    return rho, v, p


def inviscid_flux(U, gamma):
    """F[j][field] for direction j: rho v_j, rho v_i v_j + p delta_ij,
    (E + p) v_j."""
    rho, v, p = primitives(U, gamma)
    F = np.empty((3,) + U.shape)
    for j in range(3):
        F[j, 0] = U[1 + j]
        for i in range(3):
            F[j, 1 + i] = U[1 + i] * v[j] + (p if i == j else 0.0)
        F[j, 4] = (U[4] + p) * v[j]
    return F


def viscous_flux(U, Q, gamma, mu, prandtl):
    """Viscous flux Fv[j][field] from the state and the physical gradient
    Q[j][field] = d(field)/dx_j:
      stress tau = mu (grad v + grad v^T - 2/3 div v I),
      heat flux q = -mu gamma / (Pr (gamma-1)) grad(p / rho),
      Fv_j = (0, tau_xj, tau_yj, tau_zj, v_i tau_ij - q_j)."""
    rho, v, p = primitives(U, gamma)
    E = U[4]
    # velocity gradients dv_i/dx_j = (d(rho v_i)/dx_j - v_i drho/dx_j) / rho
    dv = np.empty((3, 3) + rho.shape)          # [i][j]
    for i in range(3):
        for j in range(3):
            dv[i, j] = (Q[j, 1 + i] - v[i] * Q[j, 0]) / rho
    # grad(p/rho) = (gamma-1) [ (grad E - (E/rho) grad rho)/rho - v_i grad v_i ]
    dT = np.empty((3,) + rho.shape)
    for j in range(3):
        dT[j] = (gamma - 1.0) * ((Q[j, 4] - E / rho * Q[j, 0]) / rho
                                 - sum(v[i] * dv[i, j] for i in range(3)))
    div = dv[0, 0] + dv[1, 1] + dv[2, 2]
    tau = np.empty((3, 3) + rho.shape)
    for i in range(3):
        for j in range(3):
            tau[i, j] = mu * (dv[i, j] + dv[j, i] - (2.0 / 3.0 * div if i == j else 0.0))
    kappa = mu * gamma / (prandtl * (gamma - 1.0))
    Fv = np.zeros((3,) + U.shape)
    for j in range(3):
        for i in range(3):
            Fv[j, 1 + i] = tau[i, j]
        Fv[j, 4] = sum(v[i] * tau[i, j] for i in range(3)) + kappa * dT[j]
    return Fv


def normal_flux(F, n):
    """F [3][5][...] dotted with n [3][...] -> [5][...]."""
    return np.einsum("j...,jv...->v...", n, F)


def rusanov(UL, UR, n, gamma):
    """Rusanov flux through unit normal n (pointing from L to R):
    F* = (F(UL) + F(UR)).n / 2 - lam (UR - UL) / 2,
    lam = max(|vL.n| + cL, |vR.n| + cR)."""
    rl, vl, pl = primitives(UL, gamma)
    rr, vr, pr = primitives(UR, gamma)
    cl = np.sqrt(gamma * pl / rl)
    cr = np.sqrt(gamma * pr / rr)
    lam = np.maximum(np.abs((vl * n).sum(axis=0)) + cl, np.abs((vr * n).sum(axis=0)) + cr)
    fl = normal_flux(inviscid_flux(UL, gamma), n)
    fr = normal_flux(inviscid_flux(UR, gamma), n)
    return 0.5 * (fl + fr) - 0.5 * lam * (UR - UL)


def ldg_common_solution(UL, UR, beta):
    """C = (1/2 - beta) UL + (1/2 + beta) UR."""
    return (0.5 - beta) * UL + (0.5 + beta) * UR


def ldg_common_viscous(FvL, FvR, UL, UR, n, beta, tau):
    """Common viscous normal flux, in the sign of the total flux
    F_inv - F_vis:  -[(1/2 + beta) FvL + (1/2 - beta) FvR].n + tau (UL - UR)."""
    fv = (0.5 + beta) * FvL + (0.5 - beta) * FvR
    return -normal_flux(fv, n) + tau * (UL - UR)


# ---------------------------------------------------------------------------
# Boundary conditions (reading R11).  Section 3.2 applies a no-slip
# isothermal wall at the body and Riemann-invariant conditions at the far
# field without defining them; both are imposed weakly through a boundary state Ub (used
# for the LDG common solution and the viscous flux) and a ghost state (the
# right state of the Rusanov flux).  Temperature is p / rho throughout.
# ---------------------------------------------------------------------------

def wall_states(UL, gamma, t_wall):
    """No-slip isothermal wall: Ub = (rho_L, 0, 0, 0, rho_L t_wall/(gamma-1));
    ghost = (rho_L, -rho_L v_L, rho_L t_wall/(gamma-1) + rho_L |v_L|^2/2),
    the interior velocity mirrored (average zero) at the wall temperature."""
    rho, v, _ = primitives(UL, gamma)
    eint = rho * t_wall / (gamma - 1.0)
    Ub = np.zeros_like(UL)
    Ub[0] = rho
    Ub[4] = eint
    G = np.empty_like(UL)
    G[0] = rho
    G[1:4] = -UL[1:4]
    G[4] = eint + 0.5 * rho * (v * v).sum(axis=0)
    return Ub, G


def farfield_state(UL, n, gamma, free):
    """Riemann-invariant far field for the free stream free = (rho, u, v, w, p)
    and the outward unit normal n: the outgoing invariant v.n + 2c/(gamma-1)
    from the interior, the incoming v.n - 2c/(gamma-1) from the free stream;
    entropy p/rho^gamma and tangential velocity from the interior where the
    boundary normal velocity points out of the domain (outflow), else from
    the free stream.  Returns the boundary state (also the ghost state)."""
    rho, v, p = primitives(UL, gamma)
    rf = free[0]
    vf = np.asarray(free[1:4], dtype=np.float64).reshape((3,) + (1,) * (UL.ndim - 1))
    pf = free[4]
    vnL = (v * n).sum(axis=0)
    vnf = (vf * n).sum(axis=0)
    cL = np.sqrt(gamma * p / rho)
    cf = np.sqrt(gamma * pf / rf)
    rp = vnL + 2.0 * cL / (gamma - 1.0)
    rm = vnf - 2.0 * cf / (gamma - 1.0)
    vnb = 0.5 * (rp + rm)
    cb = 0.25 * (gamma - 1.0) * (rp - rm)
    out = vnb > 0
    ent = np.where(out, p / rho ** gamma, pf / rf ** gamma)
    vt = np.where(out, v - vnL * n, vf - vnf * n)
    rhob = (cb * cb / (gamma * ent)) ** (1.0 / (gamma - 1.0))
    pb = rhob * cb * cb / gamma
    vb = vt + vnb * n
    Ub = np.empty_like(UL)
    Ub[0] = rhob
    Ub[1:4] = rhob * vb
    Ub[4] = pb / (gamma - 1.0) + 0.5 * rhob * (vb * vb).sum(axis=0)
    return Ub


BC_WALL, BC_FARFIELD = 1, 2


def boundary_states(UL, n, kind, gamma, t_wall, free):
    """(Ub, ghost) per boundary point; kind 1 wall, 2 far field."""
    Ub = np.empty_like(UL)
    G = np.empty_like(UL)
    w = kind == BC_WALL
    if w.any():
        Ub[:, w], G[:, w] = wall_states(UL[:, w], gamma, t_wall)
    f = kind == BC_FARFIELD
    if f.any():
        Ub[:, f] = farfield_state(UL[:, f], n[:, f], gamma, free)
        G[:, f] = Ub[:, f]
    return Ub, G


def boundary_flux(UL, QL, n, kind, gamma, t_wall, free, ns, mu=0.0, prandtl=0.71, tau=0.1):
    """Common normal flux out of the domain at boundary points, in the sign
    of the total flux F_inv - F_vis: Rusanov(UL, ghost; n), and for
    Navier-Stokes - F_vis(Ub, Q_L).n + tau (U_L - Ub)."""
    Ub, G = boundary_states(UL, n, kind, gamma, t_wall, free)
    fn = rusanov(UL, G, n, gamma)
    if ns:
        fn = fn - normal_flux(viscous_flux(Ub, QL, gamma, mu, prandtl), n) + tau * (UL - Ub)
    return fn
