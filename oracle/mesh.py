"""Element geometry, face matching and flux-point pairing.

Test infrastructure (see ``oracle/__init__``).

Paper, Section 2.1 and Section 3.3: elements of several types on one mixed
unstructured grid; interfaces couple neighbouring elements only through
data at their shared faces.  Geometry (reading R4): straight-sided
elements, the tet affine, the prism mapped by its six-node shape
functions (linear on the triangle times linear in t) and the hexahedron
by its eight-node trilinear ones; the metric terms are evaluated exactly
at every point from the mapping's derivatives.  Curved elements (Section
3.3, reading R12) replace the straight map by the quadratic Lagrange map of
nodes on the element's order-2 lattice.

Conventions used here and documented for the library alike:
* global element id is type-major: tets 0..n_tet-1, then prisms, then hexahedra;
* a face pair's side L is the (global id, local face) that sorts first;
* flux points pair by physical position (after periodic unwrapping);
* faces listed as boundary faces (wall or far field, reading R11) pair with
  nothing: their flux points form the boundary point list.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import elements

TYPES = ("tet", "pri", "hex")


def quadratic_nodes(name):
    """Reference coordinates of the quadratic geometry nodes (reading R12):
    the order-2 lattice of the element, tet (a, b, c) with a + b + c <= 2,
    prism (a, b) with a + b <= 2 times k <= 2, hexahedron (i, j, k) <= 2,
    at -1 + index on each axis; enumerated with the last axis outermost and
    the first innermost."""
    out = []
    for c in range(3):
        for b in range(3 if name != "tet" else 3 - c):
            for a in range(3 - b - (c if name == "tet" else 0) if name != "hex" else 3):
                out.append((-1.0 + a, -1.0 + b, -1.0 + c))
    return np.array(out)


def _quadratic_monomials(name):
    if name == "hex":
        return [(a, b, c) for a in range(3) for b in range(3) for c in range(3)]
    if name == "pri":
        return [(a, b, c) for a in range(3) for b in range(3 - a) for c in range(3)]
    return [(a, b, c) for a in range(3) for b in range(3 - a) for c in range(3 - a - b)]


def _mono_eval(monos, x):
    V = np.stack([x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for a, b, c in monos], -1)
    dV = np.zeros(V.shape + (3,))
    for m, e in enumerate(monos):
        for k in range(3):
            if e[k]:
                ee = list(e)
                ee[k] -= 1
                dV[:, m, k] = e[k] * x[:, 0] ** ee[0] * x[:, 1] ** ee[1] * x[:, 2] ** ee[2]
    return V, dV


def quadratic_shape_functions(name, x):
    """Lagrange shape functions of the quadratic geometry nodes (values
    [n_pts][n_nodes], reference derivatives [n_pts][n_nodes][3]): the
    element's order-2 space (P2, P2 x P2 in zeta, Q2) interpolating at
    quadratic_nodes."""
    monos = _quadratic_monomials(name)
    Vn, _ = _mono_eval(monos, quadratic_nodes(name))
    Vinv = np.linalg.inv(Vn)
    V, dV = _mono_eval(monos, np.asarray(x, dtype=np.float64))
    return V @ Vinv, np.einsum("pmk,mn->pnk", dV, Vinv)


def shape_functions(name, x):
    """Shape functions N [n_pts][n_verts] and their reference derivatives
    dN [n_pts][n_verts][3] of the straight-sided element map."""
    r, s, t = x[:, 0], x[:, 1], x[:, 2]
    one = np.ones_like(r)
    zero = np.zeros_like(r)
    if name == "tet":
        N = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], -1)
        dN = np.array([[-0.5, -0.5, -0.5], [0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
        dN = np.broadcast_to(dN, (len(x), 4, 3)).copy()
        return N, dN
    if name == "hex":
        # trilinear: N_a = (1 + r r_a)(1 + s s_a)(1 + t t_a) / 8
        V = elements.HEX_VERTS
        fr = 1 + r[:, None] * V[:, 0]
        fs = 1 + s[:, None] * V[:, 1]
        ft = 1 + t[:, None] * V[:, 2]
        N = fr * fs * ft / 8
        dN = np.stack([V[:, 0] * fs * ft, fr * V[:, 1] * ft, fr * fs * V[:, 2]], -1) / 8
        return N, dN
    l = [-(r + s) / 2, (1 + r) / 2, (1 + s) / 2]
    dl = [(-0.5 * one, -0.5 * one), (0.5 * one, zero), (zero, 0.5 * one)]
    lo, hi = (1 - t) / 2, (1 + t) / 2
    N = np.stack([l[0] * lo, l[1] * lo, l[2] * lo, l[0] * hi, l[1] * hi, l[2] * hi], -1)
    dN = []
    for half, dh in ((lo, -0.5), (hi, 0.5)):
        for a in range(3):
            dN.append(np.stack([dl[a][0] * half, dl[a][1] * half, l[a] * dh], -1))
    return N, np.stack(dN, axis=1)


@dataclass
class TypeGeom:
    name: str
    ref: elements.RefElement
    nelem: int
    verts: np.ndarray      # [E][nv] global vertex ids
    X: np.ndarray          # [E][nv][3] unwrapped vertex coordinates
    x_upts: np.ndarray     # [E][N_u][3] physical solution point positions
    x_fpts: np.ndarray     # [E][N_f][3]
    J_upts: np.ndarray     # [E][N_u]
    adj_upts: np.ndarray   # [E][N_u][3][3]  adj[k][j] = J dxi_k/dx_j
    n_fpts: np.ndarray     # [E][N_f][3]  adj^T n_ref (physical normal scaled)


def geometry(name, ref, X, curved=False):
    """Physical positions, Jacobian determinant and adjugate at the points;
    X are the element's vertices, or with curved=True its quadratic nodes."""
    def at(pts):
        N, dN = quadratic_shape_functions(name, pts) if curved else shape_functions(name, pts)
        x = np.einsum("pa,eai->epi", N, X)
        Jm = np.einsum("pak,eai->epik", dN, X)          # dx_i / dxi_k
        J = np.linalg.det(Jm)
        adj = J[..., None, None] * np.linalg.inv(Jm)    # [k][j] = J dxi_k/dx_j
        return x, J, adj
    xu, Ju, adju = at(ref.upts)
    xf, _, adjf = at(ref.fpts)
    nf = np.einsum("epkj,pk->epj", adjf, ref.norm_ref)
    return xu, xf, Ju, adju, nf


@dataclass
class Mesh:
    p: int
    types: dict            # name -> TypeGeom (only types with elements)
    fpt_offset: dict       # name -> offset of the type's flux points in the global flux array
    nfpts_total: int
    pair_L: np.ndarray     # [n_pairs] global flux index of side L
    pair_R: np.ndarray     # [n_pairs] global flux index of side R
    pair_nhat: np.ndarray  # [n_pairs][3] unit normal pointing out of side L
    pair_sL: np.ndarray    # [n_pairs] |adj^T n_ref| on side L
    pair_sR: np.ndarray    # [n_pairs]
    bnd_idx: np.ndarray = None    # [n_bnd] global flux index of boundary points
    bnd_nhat: np.ndarray = None   # [n_bnd][3] outward unit normal
    bnd_s: np.ndarray = None      # [n_bnd] |adj^T n_ref|
    bnd_kind: np.ndarray = None   # [n_bnd] 1 wall, 2 far field


def build_mesh(mesh_arrays, p, tol=1e-9):
    """Build geometry and the interface pairing from the generator's arrays.

    Raises ValueError on a non-positive Jacobian, an unmatched face, or a
    face whose flux points do not coincide."""
    types = {}
    gid0 = 0
    gid_base = {}
    for name in TYPES:
        v = mesh_arrays.get(f"{name}_v", np.zeros((0, 0), np.int64))
        if len(v) == 0:
            continue
        ref = elements.get(name, p)
        X = mesh_arrays["xyz"][v] + mesh_arrays[f"{name}_img"].astype(np.float64) * mesh_arrays["period"]
        Xq = mesh_arrays.get(f"{name}_q")
        if Xq is not None and len(Xq):
            # quadratically curved elements (reading R12): unwrapped node positions
            xu, xf, Ju, adju, nf = geometry(name, ref, np.asarray(Xq, dtype=np.float64), curved=True)
        else:
            xu, xf, Ju, adju, nf = geometry(name, ref, X)
        if (Ju <= 0).any():
            bad = int(np.argwhere((Ju <= 0).any(axis=1))[0, 0])
            raise ValueError(f"non-positive Jacobian in {name} element {bad}")
        types[name] = TypeGeom(name, ref, len(v), v, X, xu, xf, Ju, adju, nf)
        gid_base[name] = gid0
        gid0 += len(v)

    fpt_offset, off = {}, 0
    for name, tg in types.items():
        fpt_offset[name] = off
        off += tg.nelem * tg.ref.nfpts

    # Boundary faces (reading R11): [n][4] = (type index, element, local face,
    # kind); they take part in no pairing
    bnd = set()
    bfaces = np.asarray(mesh_arrays.get("bfaces", np.zeros((0, 4), np.int64)), dtype=np.int64).reshape(-1, 4)
    for ti, e, fi, kind in bfaces:
        name = TYPES[ti]
        if name not in types or not (0 <= e < types[name].nelem) or not (0 <= fi < len(types[name].ref.faces)):
            raise ValueError(f"boundary face ({ti}, {e}, {fi}) does not exist")
        if kind not in (1, 2) or (name, e, fi) in bnd:
            raise ValueError(f"bad or repeated boundary face ({ti}, {e}, {fi})")
        bnd.add((name, int(e), int(fi)))

    # Face matching by sorted global vertex ids
    faces = {}
    for name, tg in types.items():
        for fi, face in enumerate(tg.ref.faces):
            keys = np.sort(tg.verts[:, list(face)], axis=1)
            for e in range(tg.nelem):
                if (name, e, fi) in bnd:
                    continue
                faces.setdefault(tuple(keys[e]), []).append((gid_base[name] + e, fi, name, e))
    pL, pR, nh, sL, sR = [], [], [], [], []
    scale = max(np.ptp(mesh_arrays["xyz"], axis=0).max(), 1.0)
    period = np.asarray(mesh_arrays["period"], dtype=np.float64)

    def centroid(rec):
        _, fi, name, e = rec
        return types[name].X[e, list(types[name].ref.faces[fi])].mean(axis=0)

    def same_face(r1, r2):
        """Same vertex ids and centroids equal modulo the period: the two
        sides of one face.  (On periodic meshes two cells wide, distinct faces
        can share all vertex ids.)"""
        d = centroid(r1) - centroid(r2)
        with np.errstate(invalid="ignore", divide="ignore"):
            d = np.where(period > 0, d - period * np.round(d / np.where(period > 0, period, 1.0)), d)
        return np.abs(d).max() <= tol * scale

    pairs = []
    for key, lst in faces.items():
        lst.sort()
        left = list(lst)
        while left:
            r1 = left.pop(0)
            match = [r2 for r2 in left if same_face(r1, r2)]
            if len(match) != 1:
                raise ValueError(f"face {key} of element {r1[0]} matches {len(match)} faces")
            left.remove(match[0])
            pairs.append((r1, match[0]))
    for (_, fa, na, ea), (_, fb, nb, eb) in pairs:
        A, B = types[na], types[nb]
        ja = np.arange(A.ref.face_offsets[fa], A.ref.face_offsets[fa] + _nface(A.ref, fa))
        jb = np.arange(B.ref.face_offsets[fb], B.ref.face_offsets[fb] + _nface(B.ref, fb))
        # periodic shift between the two unwrapped copies of the shared face
        va = A.verts[ea, list(A.ref.faces[fa])[0]]
        ia = list(A.verts[ea]).index(va)
        ib = list(B.verts[eb]).index(va)
        shift = A.X[ea, ia] - B.X[eb, ib]
        xa = A.x_fpts[ea, ja]
        xb = B.x_fpts[eb, jb] + shift
        d = np.linalg.norm(xa[:, None, :] - xb[None, :, :], axis=-1)
        match = d.argmin(axis=1)
        if (d[np.arange(len(ja)), match] > tol * scale).any() or len(set(match)) != len(ja):
            raise ValueError(f"flux points of face {key} do not coincide")
        for k, j in enumerate(ja):
            jj = jb[match[k]]
            pL.append(fpt_offset[na] + ea * A.ref.nfpts + j)
            pR.append(fpt_offset[nb] + eb * B.ref.nfpts + jj)
            n = A.n_fpts[ea, j]
            s = np.linalg.norm(n)
            nh.append(n / s)
            sL.append(s)
            sR.append(np.linalg.norm(B.n_fpts[eb, jj]))
    bi, bn, bs, bk = [], [], [], []
    for ti, e, fi, kind in sorted(map(tuple, bfaces)):
        name = TYPES[ti]
        tg = types[name]
        for j in range(tg.ref.face_offsets[fi], tg.ref.face_offsets[fi] + _nface(tg.ref, fi)):
            n = tg.n_fpts[e, j]
            bi.append(fpt_offset[name] + e * tg.ref.nfpts + j)
            bs.append(np.linalg.norm(n))
            bn.append(n / bs[-1])
            bk.append(kind)
    return Mesh(p, types, fpt_offset, off, np.array(pL), np.array(pR), np.array(nh),
                np.array(sL), np.array(sR), np.array(bi, dtype=np.int64),
                np.array(bn).reshape(-1, 3), np.array(bs), np.array(bk, dtype=np.int64))


def _nface(ref, f):
    return int((ref.fpt_face == f).sum())
