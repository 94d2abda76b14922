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
