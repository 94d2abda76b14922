"""Polynomials, point sets and quadrature for the reference elements.

Test infrastructure (see ``oracle/__init__``).  Paper context: the operator
dimensions of Table 2 follow from the solution-point counts
N_u = (p+1)(p+2)(p+3)/6 (tet) and (p+1)^2(p+2)/2 (prism) and the flux-point
counts on the faces; the paper defers the point sets themselves to the PyFR
method paper, so the sets below are a reading (R1: closed-form symmetric
interior sets built from 1-D Gauss-Legendre nodes).

Reference triangle: (-1,-1), (1,-1), (-1,1).
Reference tet:      (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).
Reference prism:    reference triangle x [-1, 1].
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre
from scipy import special

TRI_VERTS = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
TET_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0],
                      [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])


# ---------------------------------------------------------------------------
# Orthonormal Jacobi polynomials (weight (1-x)^a (1+x)^b on [-1, 1])
# ---------------------------------------------------------------------------

def _jacobi_norm2(n, a, b):
    return (2.0 ** (a + b + 1) / (2 * n + a + b + 1)
            * math.gamma(n + a + 1) * math.gamma(n + b + 1)
            / (math.gamma(n + a + b + 1) * math.factorial(n)))


def jacobi(n, a, b, x):
    """Orthonormal Jacobi polynomial of degree n at x."""
    return special.eval_jacobi(n, a, b, x) / math.sqrt(_jacobi_norm2(n, a, b))


def djacobi(n, a, b, x):
    """Derivative of ``jacobi(n, a, b, x)``, from
    d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1)."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return (0.5 * (n + a + b + 1) * special.eval_jacobi(n - 1, a + 1, b + 1, x)
            / math.sqrt(_jacobi_norm2(n, a, b)))


# ---------------------------------------------------------------------------
# Orthonormal modal bases and their reference-space gradients
# ---------------------------------------------------------------------------

def line_basis(p, x):
    """Orthonormal Legendre basis on [-1,1]: values [n_pts][p+1] and
    derivatives [n_pts][p+1]."""
    x = np.asarray(x, dtype=np.float64)
    v = np.stack([jacobi(n, 0, 0, x) for n in range(p + 1)], axis=-1)
    d = np.stack([djacobi(n, 0, 0, x) for n in range(p + 1)], axis=-1)
    return v, d


def tri_basis(p, rs):
    """Orthonormal (Dubiner/Koornwinder) basis on the reference triangle.

    Collapsed coordinates a = 2(1+r)/(1-s) - 1, b = s;
    psi_ij = sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i, i + j <= p.
    Returns values [n_pts][n_modes] and gradients [n_pts][n_modes][2].
    Points must avoid the collapsed vertex s = 1."""
    rs = np.asarray(rs, dtype=np.float64)
    r, s = rs[:, 0], rs[:, 1]
    a = 2.0 * (1.0 + r) / (1.0 - s) - 1.0
    b = s
    da_dr = 2.0 / (1.0 - s)
    da_ds = 2.0 * (1.0 + r) / (1.0 - s) ** 2
    vals, grads = [], []
    for i in range(p + 1):
        for j in range(p + 1 - i):
            f, df = jacobi(i, 0, 0, a), djacobi(i, 0, 0, a)
            g, dg = jacobi(j, 2 * i + 1, 0, b), djacobi(j, 2 * i + 1, 0, b)
            w = (1.0 - b) ** i
            dw = -i * (1.0 - b) ** (i - 1) if i > 0 else np.zeros_like(b)
            psi = math.sqrt(2.0) * f * g * w
            dpsi_da = math.sqrt(2.0) * df * g * w
            dpsi_db = math.sqrt(2.0) * f * (dg * w + g * dw)
            vals.append(psi)
            grads.append(np.stack([dpsi_da * da_dr,
                                   dpsi_da * da_ds + dpsi_db], axis=-1))
    return np.stack(vals, axis=-1), np.stack(grads, axis=1)


def tet_basis(p, rst):
    """Orthonormal basis on the reference tet.

    Collapsed coordinates a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t;
    psi_ijk = 2 sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i
              P_k^(2i+2j+2,0)(c) (1-c)^(i+j),  i + j + k <= p.
    Returns values [n_pts][n_modes] and gradients [n_pts][n_modes][3]."""
    rst = np.asarray(rst, dtype=np.float64)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    a = 2.0 * (1.0 + r) / (-s - t) - 1.0
    b = 2.0 * (1.0 + s) / (1.0 - t) - 1.0
    c = t
    # chain rule: d(a,b,c)/d(r,s,t)
    da = np.stack([2.0 / (-s - t), 2.0 * (1.0 + r) / (s + t) ** 2,
                   2.0 * (1.0 + r) / (s + t) ** 2], axis=-1)
    db = np.stack([np.zeros_like(r), 2.0 / (1.0 - t),
                   2.0 * (1.0 + s) / (1.0 - t) ** 2], axis=-1)
    dc = np.stack([np.zeros_like(r), np.zeros_like(r), np.ones_like(r)], axis=-1)
    C = 2.0 * math.sqrt(2.0)
    vals, grads = [], []
    for i in range(p + 1):
        for j in range(p + 1 - i):
            for k in range(p + 1 - i - j):
                f, df = jacobi(i, 0, 0, a), djacobi(i, 0, 0, a)
                g, dg = jacobi(j, 2 * i + 1, 0, b), djacobi(j, 2 * i + 1, 0, b)
                h = jacobi(k, 2 * i + 2 * j + 2, 0, c)
                dh = djacobi(k, 2 * i + 2 * j + 2, 0, c)
                wb = (1.0 - b) ** i
                dwb = -i * (1.0 - b) ** (i - 1) if i > 0 else np.zeros_like(b)
                wc = (1.0 - c) ** (i + j)
                dwc = (-(i + j) * (1.0 - c) ** (i + j - 1) if i + j > 0
                       else np.zeros_like(c))
                psi = C * f * g * wb * h * wc
                dpa = C * df * g * wb * h * wc
                dpb = C * f * (dg * wb + g * dwb) * h * wc
                dpc = C * f * g * wb * (dh * wc + h * dwc)
                vals.append(psi)
                grads.append(dpa[:, None] * da + dpb[:, None] * db + dpc[:, None] * dc)
    return np.stack(vals, axis=-1), np.stack(grads, axis=1)


def prism_basis(p, rst):
    """Tensor basis psi_ij(r,s) * L_k(t) on the reference prism, spanning
    P_p(triangle) (x) P_p(line).  Values [n_pts][n_modes], gradients
    [n_pts][n_modes][3]."""
    rst = np.asarray(rst, dtype=np.float64)
    tv, tg = tri_basis(p, rst[:, :2])
    lv, ld = line_basis(p, rst[:, 2])
    vals = np.einsum("pa,pk->pak", tv, lv).reshape(len(rst), -1)
    gr = np.einsum("pa,pk->pak", tg[:, :, 0], lv).reshape(len(rst), -1)
    gs = np.einsum("pa,pk->pak", tg[:, :, 1], lv).reshape(len(rst), -1)
    gt = np.einsum("pa,pk->pak", tv, ld).reshape(len(rst), -1)
    return vals, np.stack([gr, gs, gt], axis=-1)


def hex_basis(p, rst):
    """Tensor Legendre basis L_i(r) L_j(s) L_k(t) on [-1, 1]^3 spanning
    Q_p (degree <= p in each variable).  Values [n_pts][n_modes], gradients
    [n_pts][n_modes][3]."""
    rst = np.asarray(rst, dtype=np.float64)
    vr, dr = line_basis(p, rst[:, 0])
    vs, ds = line_basis(p, rst[:, 1])
    vt, dt = line_basis(p, rst[:, 2])
    n = len(rst)
    vals = np.einsum("pi,pj,pk->pkji", vr, vs, vt).reshape(n, -1)
    gr = np.einsum("pi,pj,pk->pkji", dr, vs, vt).reshape(n, -1)
    gs = np.einsum("pi,pj,pk->pkji", vr, ds, vt).reshape(n, -1)
    gt = np.einsum("pi,pj,pk->pkji", vr, vs, dt).reshape(n, -1)
    return vals, np.stack([gr, gs, gt], axis=-1)


# ---------------------------------------------------------------------------
# Point sets (reading R1): symmetric interior sets built from 1-D
# Gauss-Legendre nodes, solution points and face flux points alike.
# ---------------------------------------------------------------------------

def gauss_legendre(n):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x, w = legendre.leggauss(n)
    return x, w


def tri_barycentric(p):
    """Barycentric coordinates [n][3] of the triangle set of order p.

    With v_0 < ... < v_p the Gauss-Legendre nodes mapped to (0, 1) and
    i_0 + i_1 + i_2 = p, lambda_a = (1 + 2 v_{i_a} - v_{i_b} - v_{i_c}) / 3.
    Order: i_2 outer, i_1 inner, i_0 = p - i_1 - i_2."""
    v = 0.5 * (1.0 + gauss_legendre(p + 1)[0])
    out = []
    for i2 in range(p + 1):
        for i1 in range(p + 1 - i2):
            i0 = p - i1 - i2
            ii = (i0, i1, i2)
            lam = [(1.0 + 2.0 * v[ii[a]] - v[ii[(a + 1) % 3]] - v[ii[(a + 2) % 3]]) / 3.0
                   for a in range(3)]
            out.append(lam)
    return np.array(out)


def tet_barycentric(p):
    """Barycentric coordinates [n][4] of the tet set of order p:
    lambda_a = (1 + 3 v_{i_a} - sum_{b != a} v_{i_b}) / 4, sum i = p.
    Order: i_3 outer, then i_2, then i_1, i_0 = p - i_1 - i_2 - i_3."""
    v = 0.5 * (1.0 + gauss_legendre(p + 1)[0])
    out = []
    for i3 in range(p + 1):
        for i2 in range(p + 1 - i3):
            for i1 in range(p + 1 - i3 - i2):
                i0 = p - i1 - i2 - i3
                ii = (i0, i1, i2, i3)
                tot = sum(v[k] for k in ii)
                out.append([(1.0 + 4.0 * v[ii[a]] - tot) / 4.0 for a in range(4)])
    return np.array(out)


def tri_points(p):
    """Triangle set in reference (r, s) coordinates [n][2]."""
    return tri_barycentric(p) @ TRI_VERTS


def tet_points(p):
    return tet_barycentric(p) @ TET_VERTS


def prism_points(p):
    """Triangle set x Gauss-Legendre in t; index = k * n_tri + (tri index)."""
    tri = tri_points(p)
    z = gauss_legendre(p + 1)[0]
    return np.array([[r, s, zk] for zk in z for (r, s) in tri])


def hex_points(p):
    """Gauss-Legendre product set; index = (k (p+1) + j) (p+1) + i (r fastest)."""
    x = gauss_legendre(p + 1)[0]
    return np.array([[x[i], x[j], x[k]] for k in range(p + 1) for j in range(p + 1) for i in range(p + 1)])


# ---------------------------------------------------------------------------
# Quadrature (collapsed Gauss-Jacobi products)
# ---------------------------------------------------------------------------

def tri_quadrature(deg):
    """Rule on the reference triangle exact for degree <= deg."""
    n = deg // 2 + 2
    a, wa = gauss_legendre(n)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    r = 0.5 * (1.0 + A) * (1.0 - B) - 1.0
    s = B
    return np.stack([r.ravel(), s.ravel()], axis=-1), W.ravel()


def tet_quadrature(deg):
    """Rule on the reference tet exact for degree <= deg."""
    n = deg // 2 + 2
    a, wa = gauss_legendre(n)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    c, wc = special.roots_jacobi(n, 2.0, 0.0)
    A, B, Cc = np.meshgrid(a, b, c, indexing="ij")
    W = np.einsum("i,j,k->ijk", wa, wb, wc) * 0.125
    r = 0.25 * (1.0 + A) * (1.0 - B) * (1.0 - Cc) - 1.0
    s = 0.5 * (1.0 + B) * (1.0 - Cc) - 1.0
    t = Cc
    return np.stack([r.ravel(), s.ravel(), t.ravel()], axis=-1), W.ravel()


def prism_quadrature(deg):
    tq, tw = tri_quadrature(deg)
    z, wz = gauss_legendre(deg // 2 + 2)
    pts = np.array([[r, s, zk] for zk in z for (r, s) in tq])
    w = np.array([wk * wt for wk in wz for wt in tw])
    return pts, w


def hex_quadrature(deg):
    """Gauss-Legendre product rule on [-1, 1]^3 exact for degree <= deg in
    each variable."""
    x, w = gauss_legendre(deg // 2 + 2)
    pts = np.array([[xi, xj, xk] for xk in x for xj in x for xi in x])
    wt = np.array([wi * wj * wk for wk in w for wj in w for wi in w])
    return pts, wt
