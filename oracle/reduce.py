"""Global FP64 sums over the mesh.

Test infrastructure (see ``oracle/__init__``).

Integrals use the element quadrature built from the solution points:
int_e f dx = sum_i w_i J_ei f_ei, with w_i = int l_i over the reference
element (reading R3).  Paper context: Section 3.4 names the conserved
system; these sums are its conservation and kinetic-energy diagnostics.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh


def integral(mesh: Mesh, F: dict):
    """sum over types, elements and points of w_i J_ei F_ei[...]."""
    tot = 0.0
    for n, tg in mesh.types.items():
        wJ = tg.ref.w[None, :] * tg.J_upts
        tot = tot + np.einsum("ei,ei...->...", wJ, F[n])
    return tot


def volume(mesh: Mesh):
    return float(sum((tg.ref.w[None, :] * tg.J_upts).sum() for tg in mesh.types.values()))


def kinetic_energy(mesh: Mesh, U: dict):
    """Mean kinetic energy |Omega|^-1 int rho |v|^2 / 2."""
    ke = {n: 0.5 * (U[n][..., 1] ** 2 + U[n][..., 2] ** 2 + U[n][..., 3] ** 2) / U[n][..., 0]
          for n in U}
    return integral(mesh, ke) / volume(mesh)


def kinetic_energy_rate(mesh: Mesh, U: dict, R: dict):
    """d/dt of the mean kinetic energy given R = dU/dt:
    |Omega|^-1 int (v . R_mom - |v|^2 R_rho / 2)."""
    out = {}
    for n in U:
        rho = U[n][..., 0]
        v = U[n][..., 1:4] / rho[..., None]
        out[n] = (v * R[n][..., 1:4]).sum(-1) - 0.5 * (v * v).sum(-1) * R[n][..., 0]
    return integral(mesh, out) / volume(mesh)


def l2_norm(mesh: Mesh, F: dict):
    """Per-field sqrt(int F^2)."""
    return np.sqrt(integral(mesh, {n: F[n] ** 2 for n in F}))
