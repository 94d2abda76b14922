"""The FR right-hand side, step by step, in FP64.

Test infrastructure (see ``oracle/__init__``).

Paper: Section 2.1 (operator products and point-wise operations), Table 2
(the interpolation operator M0), Section 3.4 (DG-type scheme, Rusanov
interface flux, Euler / Navier-Stokes with constant viscosity).

With the transformed flux F~_k = sum_j adj[k][j] F_j (adj = J dxi/dx) the
scheme evaluated here is (readings R2, R3, R5, R6):

  a1  U_f = M0 U                                   state at flux points
  a2  C = (1/2-beta) U_L + (1/2+beta) U_R          common solution (NS)
  a3  Q~_k = G_k U + L (n_k (C - U_f))             corrected gradient (NS)
      Q_j = sum_k adj[k][j] Q~_k / J               physical gradient
  a4  Q_f = M0 Q                                   gradient at flux points (NS)
  a5  F~ = adj (F_inv(U) - F_vis(U, Q))            transformed flux
  a6  Fn* = s [Rusanov(U_L, U_R; n) + LDG viscous] common normal flux,
      side L stores +, side R stores - (each with its own s = |adj^T n_ref|);
      at boundary points (wall, far field) the boundary and ghost states of
      reading R11 stand in for side R
  a7  R~ = sum_k G_k F~_k + L (Fn* - n_ref . M0 F~)
  a8  R = -R~ / J

n_k in a3 and n_ref in a7 are the reference-face outward unit normals; L
lifts with the reference face measure.

State layout at this module's interface: per type, arrays [E][N_u][5].
``to_lib`` / ``from_lib`` convert from/to the library's [N_u][5][ld]
layout.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import physics
from .mesh import Mesh


@dataclass
class Params:
    system: str = "euler"        # 'euler' or 'ns'
    gamma: float = 1.4
    mu: float = 0.0
    prandtl: float = 0.71
    beta: float = 0.5
    tau: float = 0.1
    t_wall: float = 1.0                                  # wall temperature p / rho
    farfield: tuple = (1.0, 0.0, 0.0, 0.0, 1.0 / 1.4)    # free stream (rho, u, v, w, p)


def to_lib(U, ld=None):
    """[E][N][5] -> [N][5][ld] (zero padded)."""
    E, N, V = U.shape
    ld = ld or E
    out = np.zeros((N, V, ld))
    out[:, :, :E] = np.transpose(U, (1, 2, 0))
    return out


def from_lib(A, E):
    """[N][5][ld] -> [E][N][5]."""
    return np.ascontiguousarray(np.transpose(A[:, :, :E], (2, 0, 1)))


def _gather(mesh: Mesh, per_type):
    """Concatenate per-type flux-point arrays [E][N_f][...] into the global
    flux array [n_fpts_total][...]."""
    return np.concatenate([per_type[n].reshape((-1,) + per_type[n].shape[2:])
                           for n in mesh.types])


def _scatter(mesh: Mesh, glob):
    out = {}
    for n, tg in mesh.types.items():
        o = mesh.fpt_offset[n]
        m = tg.nelem * tg.ref.nfpts
        out[n] = glob[o:o + m].reshape((tg.nelem, tg.ref.nfpts) + glob.shape[1:])
    return out


def rhs(mesh: Mesh, U: dict, prm: Params, want=None):
    """Right-hand side R = dU/dt for the per-type states U[name] [E][N_u][5].

    Returns R (dict of [E][N_u][5]); if ``want`` is a dict, intermediates
    are stored in it: 'Uf', 'C', 'Q', 'Qf', 'Ft', 'Fn' (per type, flux point
    arrays [E][N_f][...], solution point arrays [E][N_u][...])."""
    ns = prm.system == "ns"
    T = mesh.types

    # a1: interpolate to flux points
    Uf = {n: np.einsum("fi,eiv->efv", T[n].ref.M0, U[n]) for n in T}
    Ufg = _gather(mesh, Uf)
    UL = Ufg[mesh.pair_L].T            # [5][n_pairs]
    UR = Ufg[mesh.pair_R].T
    nh = mesh.pair_nhat.T              # [3][n_pairs]

    Q = Qf = C = None
    if ns:
        # a2: common solution, stored at both sides' flux points
        Cp = physics.ldg_common_solution(UL, UR, prm.beta).T
        Cg = np.zeros_like(Ufg)
        Cg[mesh.pair_L] = Cp
        Cg[mesh.pair_R] = Cp
        if len(mesh.bnd_idx):
            # boundary points: the common solution is the boundary state
            Ub, _ = physics.boundary_states(Ufg[mesh.bnd_idx].T, mesh.bnd_nhat.T, mesh.bnd_kind,
                                            prm.gamma, prm.t_wall, prm.farfield)
            Cg[mesh.bnd_idx] = Ub.T
        C = _scatter(mesh, Cg)
        # a3: corrected reference gradient, then physical gradient
        Q = {}
        for n, tg in T.items():
            ref = tg.ref
            dU = C[n] - Uf[n]                                            # [E][N_f][5]
            Qt = np.stack([np.einsum("ij,ejv->eiv", ref.G[k], U[n])
                           + np.einsum("if,efv->eiv", ref.L, ref.norm_ref[None, :, k, None] * dU)
                           for k in range(3)], axis=2)                   # [E][N_u][k][5]
            Q[n] = np.einsum("eikj,eikv->eijv", tg.adj_upts, Qt) / tg.J_upts[:, :, None, None]
        # a4: gradient at flux points
        Qf = {n: np.einsum("fi,eijv->efjv", T[n].ref.M0, Q[n]) for n in T}

    # a5: transformed flux at solution points
    Ft = {}
    for n, tg in T.items():
        Ue = np.moveaxis(U[n], 2, 0)                                     # [5][E][N_u]
        F = physics.inviscid_flux(Ue, prm.gamma)                         # [3][5][E][N_u]
        if ns:
            Qe = np.moveaxis(Q[n], (2, 3), (0, 1))                       # [3][5][E][N_u]
            F = F - physics.viscous_flux(Ue, Qe, prm.gamma, prm.mu, prm.prandtl)
        Ft[n] = np.einsum("eikj,jvei->eikv", tg.adj_upts, F)             # [E][N_u][k][5]

    # a6: common normal flux at interfaces
    fn = physics.rusanov(UL, UR, nh, prm.gamma)
    if ns:
        Qfg = _gather(mesh, Qf)                                          # [n][3][5]
        QL = np.moveaxis(Qfg[mesh.pair_L], 0, -1)                        # [3][5][n_pairs]
        QR = np.moveaxis(Qfg[mesh.pair_R], 0, -1)
        FvL = physics.viscous_flux(UL, QL, prm.gamma, prm.mu, prm.prandtl)
        FvR = physics.viscous_flux(UR, QR, prm.gamma, prm.mu, prm.prandtl)
        fn = fn + physics.ldg_common_viscous(FvL, FvR, UL, UR, nh, prm.beta, prm.tau)
    Fng = np.zeros_like(Ufg)
    Fng[mesh.pair_L] = (mesh.pair_sL * fn).T
    Fng[mesh.pair_R] = -(mesh.pair_sR * fn).T
    if len(mesh.bnd_idx):
        QB = np.moveaxis(_gather(mesh, Qf)[mesh.bnd_idx], 0, -1) if ns else None
        fb = physics.boundary_flux(Ufg[mesh.bnd_idx].T, QB, mesh.bnd_nhat.T, mesh.bnd_kind, prm.gamma,
                                   prm.t_wall, prm.farfield, ns, prm.mu, prm.prandtl, prm.tau)
        Fng[mesh.bnd_idx] = (mesh.bnd_s * fb).T
    Fn = _scatter(mesh, Fng)

    # a7, a8: divergence plus correction, then -1/J
    R = {}
    for n, tg in T.items():
        ref = tg.ref
        div = sum(np.einsum("ij,ejv->eiv", ref.G[k], Ft[n][:, :, k]) for k in range(3))
        Ftf = np.einsum("fi,eikv->efkv", ref.M0, Ft[n])                  # [E][N_f][k][5]
        fn_int = np.einsum("fk,efkv->efv", ref.norm_ref, Ftf)
        corr = np.einsum("if,efv->eiv", ref.L, Fn[n] - fn_int)
        R[n] = -(div + corr) / tg.J_upts[:, :, None]

    if want is not None:
        want.update(Uf=Uf, C=C, Q=Q, Qf=Qf, Ft=Ft, Fn=Fn)
    return R


def points_per_type(mesh: Mesh):
    """Physical solution-point positions [E][N_u][3] per type."""
    return {n: tg.x_upts for n, tg in mesh.types.items()}


def initial_state(mesh: Mesh, fn, **kw):
    """Evaluate a field function fn(x, y, z) -> [5][...] at the solution
    points: returns per type [E][N_u][5]."""
    out = {}
    for n, tg in mesh.types.items():
        x = tg.x_upts
        out[n] = np.moveaxis(fn(x[..., 0], x[..., 1], x[..., 2], **kw), 0, -1)
    return out
