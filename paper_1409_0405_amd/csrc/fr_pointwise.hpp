// Point-wise arithmetic of the FR right-hand side shared by the kernels
// that evaluate it (the solution-point kernel, the fused gradient kernel and
// the interface kernels), so that every path computes the same bits.
// Internal header (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace frd {
namespace {

// ---------------------------------------------------------------------------
// Geometry at a solution point from the Jacobian coefficients.
// Tet: constant columns c0..c2.  Prism: dx/dxi = A1 + C1 z,
// dx/deta = B1 + C2 z, dx/dzeta = C0 + C1 x + C2 y.  Hexahedron (trilinear
// map, coefficients c1..c7): dx/dr = c1 + c4 s + c5 t + c7 st,
// dx/ds = c2 + c4 r + c6 t + c7 rt, dx/dt = c3 + c5 r + c6 s + c7 rs.
// adj[k][j] = J dxi_k/dx_j (rows are cross products of the columns).
// ---------------------------------------------------------------------------
template <typename T, int ET>
__device__ __forceinline__ T metric(const T *__restrict__ g, int64_t ld, int64_t e,
                                    const T *__restrict__ xi, T adj[3][3]) {
    T c[3][3];
    if (ET == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) c[k][d] = g[(3 * k + d) * ld + e];
    } else if (ET == 2) {
        const T r = xi[0], sv = xi[1], t = xi[2];
        const T st = sv * t, rt = r * t, rs = r * sv;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T c1 = g[d * ld + e], c2 = g[(3 + d) * ld + e], c3 = g[(6 + d) * ld + e];
            const T c4 = g[(9 + d) * ld + e], c5 = g[(12 + d) * ld + e], c6 = g[(15 + d) * ld + e];
            const T c7 = g[(18 + d) * ld + e];
            c[0][d] = c1 + c4 * sv + c5 * t + c7 * st;
            c[1][d] = c2 + c4 * r + c6 * t + c7 * rt;
            c[2][d] = c3 + c5 * r + c6 * sv + c7 * rs;
        }
    } else {
        const T x = xi[0], y = xi[1], z = xi[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T A1 = g[d * ld + e], B1 = g[(3 + d) * ld + e], C0 = g[(6 + d) * ld + e];
            const T C1 = g[(9 + d) * ld + e], C2 = g[(12 + d) * ld + e];
            c[0][d] = A1 + C1 * z;
            c[1][d] = B1 + C2 * z;
            c[2][d] = C0 + C1 * x + C2 * y;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        adj[k][0] = c[k1][1] * c[k2][2] - c[k1][2] * c[k2][1];
        adj[k][1] = c[k1][2] * c[k2][0] - c[k1][0] * c[k2][2];
        adj[k][2] = c[k1][0] * c[k2][1] - c[k1][1] * c[k2][0];
    }
    return c[0][0] * adj[0][0] + c[0][1] * adj[0][1] + c[0][2] * adj[0][2];
}

// Inviscid flux F[j][v] of the conserved state u, with the constant
// reference pressure pref taken out of the momentum flux's pressure term
// (pref = 0: the plain flux; p returns the full pressure).  A constant flux
// has zero discrete divergence on a mesh that preserves a uniform state, so
// every residual is unchanged in exact arithmetic when the volume and the
// interface fluxes both leave pref out, while single precision no longer
// rounds the large constant part of the pressure at low Mach number.
template <typename T>
__device__ __forceinline__ void euler_flux(const T u[5], T gamma, T pref, T F[3][5], T &p) {
    const T rinv = T(1) / u[0];
    const T v[3] = {u[1] * rinv, u[2] * rinv, u[3] * rinv};
    p = (gamma - T(1)) * (u[4] - T(0.5) * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
    const T pm = p - pref;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[j][0] = u[1 + j];
        F[j][1] = u[1] * v[j];
        F[j][2] = u[2] * v[j];
        F[j][3] = u[3] * v[j];
        F[j][1 + j] += pm;
        F[j][4] = (u[4] + p) * v[j];
    }
}

// Viscous flux Fv[j][v] from the state u and the physical gradient q[j][v]:
// tau = mu (grad v + grad v^T - 2/3 div v I), heat flux from grad(p/rho) with
// conductivity mu gamma / (Pr (gamma - 1)).
template <typename T>
__device__ __forceinline__ void viscous_flux(const T u[5], const T q[3][5], T gamma, T mu,
                                             T prandtl, T Fv[3][5]) {
    const T rinv = T(1) / u[0];
    const T v[3] = {u[1] * rinv, u[2] * rinv, u[3] * rinv};
    const T e = u[4] * rinv;
    T dv[3][3], dT[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int i = 0; i < 3; ++i) dv[i][j] = (q[j][1 + i] - v[i] * q[j][0]) * rinv;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
        dT[j] = (gamma - T(1)) * ((q[j][4] - e * q[j][0]) * rinv -
                                  (v[0] * dv[0][j] + v[1] * dv[1][j] + v[2] * dv[2][j]));
    const T div = dv[0][0] + dv[1][1] + dv[2][2];
    const T kappa = mu * gamma / (prandtl * (gamma - T(1)));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Fv[j][0] = 0;
        T work = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T tau = mu * (dv[i][j] + dv[j][i]);
            if (i == j) tau -= mu * T(2.0 / 3.0) * div;
            Fv[j][1 + i] = tau;
            work += v[i] * tau;
        }
        Fv[j][4] = work + kappa * dT[j];
    }
}

// Work at one solution point: the physical gradient q = adj^T qt / J (NS)
// and the transformed flux Ft = adj (F_inv(u) - F_vis(u, q)).  Section 3.4:
// compressible Navier-Stokes with constant viscosity; Section 2.1: the
// point-wise step between the operator products.
template <typename T, bool NS>
__device__ __forceinline__ void upts_point(const T u[5], const T qt[3][5], const T adj[3][3], T Jinv, T gamma,
                                           T mu, T prandtl, T pref, T q[3][5], T Ft[3][5]) {
    T F[3][5], p;
    euler_flux(u, gamma, pref, F, p);
    if (NS) {
        T Fv[3][5];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v)
                q[j][v] = (adj[0][j] * qt[0][v] + adj[1][j] * qt[1][v] + adj[2][j] * qt[2][v]) * Jinv;
        viscous_flux(u, q, gamma, mu, prandtl, Fv);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) F[j][v] -= Fv[j][v];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v) Ft[k][v] = adj[k][0] * F[0][v] + adj[k][1] * F[1][v] + adj[k][2] * F[2][v];
}

}  // namespace
}  // namespace frd
