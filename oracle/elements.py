"""Reference elements and their constant operator matrices.

Test infrastructure (see ``oracle/__init__``).

Paper, Section 2.1: most of an FR step is a product of a constant operator
matrix with a state matrix; Table 2 gives the dimensions of the
volume-to-surface interpolation operator M0 for tets and prisms.  The other
operators (gradient, divergence, correction lift) follow from the DG-type FR
scheme of Section 3.4 (R2: the correction is the DG lift built in the
reference element with the point-wise 1/J of FR; R3: operators by exact
modal projection, integrals with the reference face measure).

Construction route (modal, orthonormal):
  V   = psi(solution points)                 (N_u x N_u)
  M0  = psi(flux points) V^-1                (N_f x N_u)
  G_k = dpsi/dxi_k(solution points) V^-1     (N_u x N_u), k = 0, 1, 2
  L   = V H,  H[a, (f,j)] = int_f psi_a l^f_j ds   (N_u x N_f)
        which equals M^-1 E with the nodal mass matrix M = (V V^T)^-1 and
        E[i, (f,j)] = int_f l_i l^f_j ds, because psi_a = sum_i V[i,a] l_i.
  w   = V^-T int psi                         (volume quadrature weights)
Face integrals use the reference face's own surface measure.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import basis

# Reference element vertices
PRI_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0],
                      [-1.0, -1.0, 1.0], [1.0, -1.0, 1.0], [-1.0, 1.0, 1.0]])

# Faces as local vertex tuples.  Triangles (a, b, c): flux points are the
# triangle set with barycentrics (l0, l1, l2) placed at l0 a + l1 b + l2 c.
# Quads (a, b, c, d): a-b is the first edge, d lies across from a and c from
# b; the point for Gauss-Legendre nodes (s_i, t_j) is a + (1+s_i)/2 (b-a) +
# (1+t_j)/2 (d-a), index j * (p+1) + i.
TET_FACES = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
PRI_FACES = [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)]
# Hexahedron [-1, 1]^3: vertices 0-3 counter-clockwise at t = -1, 4-7 above them
HEX_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [1.0, 1.0, -1.0], [-1.0, 1.0, -1.0],
                      [-1.0, -1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, 1.0], [-1.0, 1.0, 1.0]])
HEX_FACES = [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]

TET_VOLUME = 4.0 / 3.0
PRI_VOLUME = 4.0
HEX_VOLUME = 8.0


def _outward_normal(verts, face, centroid):
    P = verts[list(face)]
    n = np.cross(P[1] - P[0], P[-1] - P[0])
    n = n / np.linalg.norm(n)
    if np.dot(n, P[0] - centroid) < 0:
        n = -n
    return n


def _face_area(verts, face):
    P = verts[list(face)]
    if len(face) == 3:
        return 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    return np.linalg.norm(np.cross(P[1] - P[0], P[3] - P[0]))


def face_points_param(p, nverts):
    """Face point set in the face's own parameter space: triangle (r, s) on
    the reference triangle, quad (s, t) on [-1, 1]^2."""
    if nverts == 3:
        return basis.tri_points(p)
    x = basis.gauss_legendre(p + 1)[0]
    return np.array([[si, tj] for tj in x for si in x])


def face_map(verts, face, uv):
    """Reference-space position of face parameter points uv."""
    P = verts[list(face)]
    if len(face) == 3:
        l0 = -0.5 * (uv[:, 0] + uv[:, 1])
        l1 = 0.5 * (1.0 + uv[:, 0])
        l2 = 0.5 * (1.0 + uv[:, 1])
        return l0[:, None] * P[0] + l1[:, None] * P[1] + l2[:, None] * P[2]
    s = 0.5 * (1.0 + uv[:, 0])
    t = 0.5 * (1.0 + uv[:, 1])
    return P[0] + s[:, None] * (P[1] - P[0]) + t[:, None] * (P[3] - P[0])


def face_lagrange(p, nverts, uv):
    """Face Lagrange basis on the face point set, evaluated at uv [n][2]:
    returns [n_uv][n_face_pts]."""
    fp = face_points_param(p, nverts)
    if nverts == 3:
        Vf = basis.tri_basis(p, fp)[0]
        Vq = basis.tri_basis(p, uv)[0]
        return Vq @ np.linalg.inv(Vf)
    x = basis.gauss_legendre(p + 1)[0]
    V1 = basis.line_basis(p, x)[0]
    inv1 = np.linalg.inv(V1)
    ls = basis.line_basis(p, uv[:, 0])[0] @ inv1      # [n][p+1]
    lt = basis.line_basis(p, uv[:, 1])[0] @ inv1
    return np.einsum("ni,nj->nji", ls, lt).reshape(len(uv), -1)


def face_quadrature_param(p, nverts):
    """Face rule in parameter space, exact for degree 2p+2 (quad: per
    direction), with weights summing to the parameter-space area."""
    if nverts == 3:
        return basis.tri_quadrature(2 * p + 2)
    x, w = basis.gauss_legendre(p + 2)
    return (np.array([[si, tj] for tj in x for si in x]),
            np.array([wj * wi for wj in w for wi in w]))


@dataclass
class RefElement:
    """Operators of one element type at order p (all float64)."""
    name: str
    p: int
    verts: np.ndarray
    faces: list
    upts: np.ndarray            # [N_u][3]
    fpts: np.ndarray            # [N_f][3]
    fpt_face: np.ndarray        # [N_f] local face id
    face_offsets: list          # first flux point of each face
    norm_ref: np.ndarray        # [N_f][3] outward unit normal of the reference face
    M0: np.ndarray = field(repr=False, default=None)     # [N_f][N_u]
    G: np.ndarray = field(repr=False, default=None)      # [3][N_u][N_u]
    L: np.ndarray = field(repr=False, default=None)      # [N_u][N_f]
    w: np.ndarray = field(repr=False, default=None)      # [N_u]
    V: np.ndarray = field(repr=False, default=None)
    volume: float = 0.0

    @property
    def nupts(self):
        return len(self.upts)

    @property
    def nfpts(self):
        return len(self.fpts)


def _basis_fn(name):
    return {"tet": basis.tet_basis, "pri": basis.prism_basis, "hex": basis.hex_basis}[name]


def _quad_fn(name):
    return {"tet": basis.tet_quadrature, "pri": basis.prism_quadrature, "hex": basis.hex_quadrature}[name]


def build(name, p):
    """Build the reference element 'tet', 'pri' or 'hex' at order p."""
    if name == "tet":
        verts, faces, upts, vol = basis.TET_VERTS, TET_FACES, basis.tet_points(p), TET_VOLUME
    elif name == "pri":
        verts, faces, upts, vol = PRI_VERTS, PRI_FACES, basis.prism_points(p), PRI_VOLUME
    elif name == "hex":
        verts, faces, upts, vol = HEX_VERTS, HEX_FACES, basis.hex_points(p), HEX_VOLUME
    else:
        raise ValueError(name)
    centroid = verts.mean(axis=0)

    fpts, fpt_face, norm_ref, offs = [], [], [], []
    for fi, face in enumerate(faces):
        offs.append(sum(len(x) for x in fpts))
        uv = face_points_param(p, len(face))
        pts = face_map(verts, face, uv)
        fpts.append(pts)
        fpt_face += [fi] * len(pts)
        norm_ref.append(np.repeat(_outward_normal(verts, face, centroid)[None], len(pts), 0))
    fpts = np.concatenate(fpts)
    norm_ref = np.concatenate(norm_ref)

    bfn = _basis_fn(name)
    V, _ = bfn(p, upts)
    Vinv = np.linalg.inv(V)
    Vf, _ = bfn(p, fpts)
    _, dV = bfn(p, upts)
    M0 = Vf @ Vinv
    G = np.stack([dV[:, :, k] @ Vinv for k in range(3)])

    # Lift: L = V H, H[a,(f,j)] = int_f psi_a l^f_j ds (reference face measure)
    H = np.zeros((len(upts), len(fpts)))
    for fi, face in enumerate(faces):
        nv = len(face)
        q_uv, q_w = face_quadrature_param(p, nv)
        param_area = 2.0 if nv == 3 else 4.0
        scale = _face_area(verts, face) / param_area
        q_x = face_map(verts, face, q_uv)
        psi_q, _ = bfn(p, q_x)                    # [nq][N_u modes]
        lf_q = face_lagrange(p, nv, q_uv)         # [nq][n_face_pts]
        n0 = offs[fi]
        H[:, n0:n0 + lf_q.shape[1]] = scale * np.einsum("q,qa,qj->aj", q_w, psi_q, lf_q)
    L = V @ H

    # Volume weights w_i = int l_i
    qx, qw = _quad_fn(name)(2 * p + 2)
    psi_q, _ = bfn(p, qx)
    w = Vinv.T @ (psi_q.T @ qw)

    return RefElement(name=name, p=p, verts=verts, faces=faces, upts=upts, fpts=fpts,
                      fpt_face=np.array(fpt_face), face_offsets=offs, norm_ref=norm_ref,
                      M0=M0, G=G, L=L, w=w, V=V, volume=vol)


_CACHE = {}


def get(name, p):
    key = (name, p)
    if key not in _CACHE:
        _CACHE[key] = build(name, p)
    return _CACHE[key]


def nupts(name, p):
    if name == "tet":
        return (p + 1) * (p + 2) * (p + 3) // 6
    if name == "hex":
        return (p + 1) ** 3
    return (p + 1) ** 2 * (p + 2) // 2


def nfpts(name, p):
    tri = (p + 1) * (p + 2) // 2
    if name == "tet":
        return 4 * tri
    if name == "hex":
        return 6 * (p + 1) ** 2
    return 2 * tri + 3 * (p + 1) ** 2
