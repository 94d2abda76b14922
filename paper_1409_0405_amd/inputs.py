"""Seeded synthetic inputs: periodic tet/prism/hex meshes and initial fields.

This module holds input generation only (vertex lattices, jitter, element
connectivity, closed-form initial conditions evaluated at given physical
points).  It holds none of the flux reconstruction arithmetic, so both the
library side and the FP64 oracle may consume what it produces.

Mesh arrays (all numpy, host memory):

* ``xyz``      float64 [n_vertices][3]  unique (periodic) vertex coordinates
* ``tet_v``    int64   [n_tets][4]      vertex ids, positively oriented
* ``tet_img``  int8    [n_tets][4][3]   periodic image shift per element vertex;
                                        the unwrapped vertex is xyz[v] + img*period
* ``pri_v``    int64   [n_prisms][6]    0-2 bottom triangle (counter-clockwise
                                        seen from above), 3-5 top, k+3 above k
* ``pri_img``  int8    [n_prisms][6][3]
* ``hex_v``    int64   [n_hex][8]       0-3 bottom quad (counter-clockwise seen
                                        from above), 4-7 top, k+4 above k
                                        (optional: absent means no hexahedra)
* ``hex_img``  int8    [n_hex][8][3]
* ``period``   float64 [3]                 0 for a direction that is not periodic
* ``bfaces``   int64   [n][4]          optional boundary faces: (type 0 tet / 1
                                        prism / 2 hex, element, local face,
                                        kind 1 wall / 2 far field)

Element order is chosen for locality of interface gathers: tets are numbered
shape-major (the six Kuhn shapes of a cube are six blocks, cubes run fastest
inside a block); prisms are numbered triangle-major (the two triangles of an
x-y quad are two blocks, then layer, then quad).  With that order the
neighbour across a given local face of consecutive elements is, away from
the periodic seams, at a constant index offset.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GAMMA = 1.4


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def _kuhn_shapes():
    """The six tetrahedra of the Kuhn (Freudenthal) split of the unit cube
    along the (0,0,0)->(1,1,1) diagonal, as corner offsets, each ordered so
    that det(v1-v0, v2-v0, v3-v0) > 0."""
    shapes = []
    for perm in itertools.permutations(range(3)):
        v0 = np.zeros(3, dtype=int)
        v1 = v0.copy(); v1[perm[0]] = 1
        v2 = v1.copy(); v2[perm[1]] = 1
        v3 = np.ones(3, dtype=int)
        if _perm_sign(perm) > 0:
            shapes.append((v0, v1, v2, v3))
        else:
            shapes.append((v0, v2, v1, v3))
    return shapes


# Two triangles of the x-y quad, split along (i,j)->(i+1,j+1), both
# counter-clockwise; the diagonal matches the Kuhn split's z-faces.
_QUAD_TRIS = (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1)))


def mixed_box(nx, ny, n_pri_layers, n_tet_layers, lengths, z_split=None,
              jitter=0.0, seed=0):
    """Periodic box [0,Lx)x[0,Ly)x[0,Lz): prisms (extruded x-y triangles) on
    z in [0, z_split), Kuhn-split tets on z in [z_split, Lz).

    ``n_pri_layers`` prism layers, ``n_tet_layers`` cube layers; either may
    be zero.  Every vertex coordinate is jittered by U(-a, a) times the local
    spacing on that axis (a = ``jitter``); on z levels between two spacings
    the smaller is used.  Draw order: vertex id order, x then y then z.
    """
    Lx, Ly, Lz = (float(v) for v in lengths)
    if z_split is None:
        z_split = 0.0 if n_pri_layers == 0 else (Lz if n_tet_layers == 0 else 0.5 * Lz)
    zl = []
    for k in range(n_pri_layers):
        zl.append(k * z_split / n_pri_layers)
    for k in range(n_tet_layers):
        zl.append(z_split + k * (Lz - z_split) / n_tet_layers)
    zl = np.asarray(zl, dtype=np.float64)
    nz = len(zl)
    if nz == 0:
        raise ValueError("empty mesh")
    dz = np.diff(np.append(zl, Lz))                # spacing above each level
    dz_below = np.roll(dz, 1)
    hz = np.minimum(dz, dz_below)

    hx, hy = Lx / nx, Ly / ny
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    xyz = np.stack([ix * hx, iy * hy, zl[iz]], axis=-1).reshape(-1, 3)
    if jitter:
        rng = np.random.default_rng(seed)
        r = rng.uniform(-1.0, 1.0, size=xyz.shape)
        scale = np.stack([np.full(nz * ny * nx, hx), np.full(nz * ny * nx, hy),
                          hz[iz.reshape(-1)]], axis=-1)
        xyz = xyz + jitter * r * scale

    def vid(kx, ky, kz):
        return (np.mod(kz, nz) * ny + np.mod(ky, ny)) * nx + np.mod(kx, nx)

    def img(kx, ky, kz):
        return np.stack([kx >= nx, ky >= ny, kz >= nz], axis=-1).astype(np.int8)

    # tets: shape-major, then cube (layer, y, x)
    tet_v, tet_img = [], []
    if n_tet_layers:
        cz, cy, cx = np.meshgrid(np.arange(n_pri_layers, nz), np.arange(ny),
                                 np.arange(nx), indexing="ij")
        cz, cy, cx = cz.reshape(-1), cy.reshape(-1), cx.reshape(-1)
        for shape in _kuhn_shapes():
            vs, ims = [], []
            for off in shape:
                kx, ky, kz = cx + off[0], cy + off[1], cz + off[2]
                vs.append(vid(kx, ky, kz))
                ims.append(img(kx, ky, kz))
            tet_v.append(np.stack(vs, axis=-1))
            tet_img.append(np.stack(ims, axis=1))
    tet_v = np.concatenate(tet_v) if tet_v else np.zeros((0, 4), np.int64)
    tet_img = np.concatenate(tet_img) if tet_img else np.zeros((0, 4, 3), np.int8)

    # prisms: triangle-major, then layer, then quad (y, x)
    pri_v, pri_img = [], []
    if n_pri_layers:
        cz, cy, cx = np.meshgrid(np.arange(0, n_pri_layers), np.arange(ny),
                                 np.arange(nx), indexing="ij")
        cz, cy, cx = cz.reshape(-1), cy.reshape(-1), cx.reshape(-1)
        for tri in _QUAD_TRIS:
            vs, ims = [], []
            for dk in (0, 1):
                for (di, dj) in tri:
                    kx, ky, kz = cx + di, cy + dj, cz + dk
                    vs.append(vid(kx, ky, kz))
                    ims.append(img(kx, ky, kz))
            pri_v.append(np.stack(vs, axis=-1))
            pri_img.append(np.stack(ims, axis=1))
    pri_v = np.concatenate(pri_v) if pri_v else np.zeros((0, 6), np.int64)
    pri_img = np.concatenate(pri_img) if pri_img else np.zeros((0, 6, 3), np.int8)

    return {
        "xyz": np.ascontiguousarray(xyz, dtype=np.float64),
        "tet_v": np.ascontiguousarray(tet_v, dtype=np.int64),
        "tet_img": np.ascontiguousarray(tet_img, dtype=np.int8),
        "pri_v": np.ascontiguousarray(pri_v, dtype=np.int64),
        "pri_img": np.ascontiguousarray(pri_img, dtype=np.int8),
        "period": np.array([Lx, Ly, Lz], dtype=np.float64),
    }


# Local faces of each element type (vertex positions within the element), in
# the order the mesh format numbers them; used only to name boundary faces.
LOCAL_FACES = {
    "tet": [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)],
    "pri": [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
    "hex": [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)],
}
BC_WALL, BC_FARFIELD = 1, 2


def hybrid_box(nx, ny, nz, x_split, z_split, lengths, jitter=0.0, seed=0, y_bc=None):
    """Periodic box of nx x ny x nz cells holding all three element types
    with conforming interfaces:

    * cells ix <  x_split, iz <  z_split: hexahedra;
    * cells ix >= x_split, iz <  z_split: prisms extruded along z (the x-y
      quad split along (i,j)->(i+1,j+1)), meeting the hexahedra through
      x-faces;
    * cells ix <  x_split, iz >= z_split: prisms extruded along x (the y-z
      quad split along (j,k)->(j+1,k+1)), meeting the hexahedra through
      z-faces;
    * cells ix >= x_split, iz >= z_split: Kuhn-split tets, meeting both
      prism kinds through triangles whose diagonals match the Kuhn split.

    ``x_split = nx, z_split = nz`` gives a pure hexahedral box,
    ``x_split = 0`` the prism/tet layers of ``mixed_box``.  Vertices are
    jittered by U(-a, a) times the cell size on each axis, drawn in vertex
    id order (x fastest, then y, then z; per vertex x, y, z).

    ``y_bc`` = "wall" or "farfield" makes y bounded instead of periodic: the
    planes y = 0 and y = Ly are boundaries of that kind (their vertices keep
    y exact), listed in ``bfaces`` [n][4] = (type 0 tet / 1 prism / 2 hex,
    element, local face, kind 1 wall / 2 far field), and period[1] is 0.

    Element order: hexahedra (z, y, x) with x fastest; z-prisms triangle
    major, then (z, y, x); x-prisms triangle-major, then (z, y, x); tets
    shape-major, then (z, y, x).
    """
    Lx, Ly, Lz = (float(v) for v in lengths)
    if not (0 <= x_split <= nx and 0 <= z_split <= nz) or min(nx, ny, nz) < 1:
        raise ValueError("bad hybrid box split")
    if y_bc not in (None, "wall", "farfield"):
        raise ValueError("y_bc must be None, 'wall' or 'farfield'")
    h = np.array([Lx / nx, Ly / ny, Lz / nz])
    nyv = ny + 1 if y_bc else ny                   # vertex rows in y
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(nyv), np.arange(nx), indexing="ij")
    xyz = np.stack([ix, iy, iz], axis=-1).reshape(-1, 3) * h
    if jitter:
        rng = np.random.default_rng(seed)
        r = jitter * rng.uniform(-1.0, 1.0, size=xyz.shape) * h
        if y_bc:
            on_bnd = (iy.reshape(-1) == 0) | (iy.reshape(-1) == ny)
            r[on_bnd, 1] = 0.0
        xyz = xyz + r
    n = np.array([nx, ny if not y_bc else 1 << 30, nz])

    def corner(c, off):
        k = c + np.asarray(off)[None, :]
        ky = k[:, 1] if y_bc else np.mod(k[:, 1], ny)
        vid = (np.mod(k[:, 2], nz) * nyv + ky) * nx + np.mod(k[:, 0], nx)
        return vid, (k >= n[None, :]).astype(np.int8)

    def cells(x0, x1, z0, z1):
        cz, cy, cx = np.meshgrid(np.arange(z0, z1), np.arange(ny), np.arange(x0, x1), indexing="ij")
        return np.stack([cx.reshape(-1), cy.reshape(-1), cz.reshape(-1)], axis=-1)

    def build(cl, shapes, nv):
        vs, ims = [], []
        for shape in shapes:
            sv, si = zip(*(corner(cl, off) for off in shape))
            vs.append(np.stack(sv, axis=-1))
            ims.append(np.stack(si, axis=1))
        if not vs or len(cl) == 0:
            return np.zeros((0, nv), np.int64), np.zeros((0, nv, 3), np.int8)
        return np.concatenate(vs), np.concatenate(ims)

    hex_shape = [[(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                  (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]]
    zpri = [[(a, b, dk) for dk in (0, 1) for (a, b) in tri] for tri in _QUAD_TRIS]
    xpri = [[(di, a, b) for di in (0, 1) for (a, b) in tri] for tri in _QUAD_TRIS]
    tets = [[tuple(o) for o in shape] for shape in _kuhn_shapes()]
    hex_v, hex_img = build(cells(0, x_split, 0, z_split), hex_shape, 8)
    pz_v, pz_img = build(cells(x_split, nx, 0, z_split), zpri, 6)
    px_v, px_img = build(cells(0, x_split, z_split, nz), xpri, 6)
    tet_v, tet_img = build(cells(x_split, nx, z_split, nz), tets, 4)
    c = np.ascontiguousarray
    out = {
        "xyz": c(xyz, dtype=np.float64),
        "tet_v": c(tet_v, dtype=np.int64), "tet_img": c(tet_img, dtype=np.int8),
        "pri_v": c(np.concatenate([pz_v, px_v]), dtype=np.int64),
        "pri_img": c(np.concatenate([pz_img, px_img]), dtype=np.int8),
        "hex_v": c(hex_v, dtype=np.int64), "hex_img": c(hex_img, dtype=np.int8),
        "period": np.array([Lx, 0.0 if y_bc else Ly, Lz], dtype=np.float64),
    }
    if y_bc:
        kind = BC_WALL if y_bc == "wall" else BC_FARFIELD
        rows = []
        for ti, name in enumerate(("tet", "pri", "hex")):
            ky = (out[f"{name}_v"] // nx) % nyv                  # vertex row of each element vertex
            for fi, face in enumerate(LOCAL_FACES[name]):
                fk = ky[:, list(face)]
                hit = np.flatnonzero((fk == 0).all(axis=1) | (fk == ny).all(axis=1))
                rows += [(ti, int(e), fi, kind) for e in hit]
        out["bfaces"] = np.array(rows, dtype=np.int64).reshape(-1, 4)
    return out


def hex_box(n, lengths=(2.0 * math.pi,) * 3, jitter=0.0, seed=0, y_bc=None):
    """Box of n^3 hexahedra (``hybrid_box`` with no other type), periodic
    unless ``y_bc`` bounds it in y."""
    return hybrid_box(n, n, n, n, n, lengths, jitter=jitter, seed=seed, y_bc=y_bc)


def _order2_lattice(kind):
    """Reference coordinates of an element's order-2 node lattice, the node
    order of the mesh format's quadratic geometry: tet (a, b, c) with
    a + b + c <= 2, prism (a, b) with a + b <= 2 times c <= 2, hexahedron
    (a, b, c) <= 2; coordinates -1 + index; c outermost, a innermost."""
    pts = []
    for c in range(3):
        nb = 3 - c if kind == "tet" else 3
        for b in range(nb):
            na = 3 if kind == "hex" else (3 - b - c if kind == "tet" else 3 - b)
            for a in range(na):
                pts.append((a - 1.0, b - 1.0, c - 1.0))
    return np.array(pts)


def _straight_points(kind, X, r):
    """Positions of reference points r [n][3] under the straight-sided map of
    elements with unwrapped vertices X [E][nv][3] -> [E][n][3]."""
    x, y, z = r[:, 0], r[:, 1], r[:, 2]
    if kind == "tet":
        W = np.stack([-(1 + x + y + z) / 2, (1 + x) / 2, (1 + y) / 2, (1 + z) / 2], -1)
    elif kind == "pri":
        tri = [-(x + y) / 2, (1 + x) / 2, (1 + y) / 2]
        W = np.stack([t * (1 - z) / 2 for t in tri] + [t * (1 + z) / 2 for t in tri], -1)
    else:
        sg = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                       [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
        W = np.prod(1 + r[:, None, :] * sg[None], axis=-1) / 8
    return np.einsum("na,eai->eni", W, X)


def curve(mesh, amp=0.02):
    """Quadratically curved version of a straight mesh: every element gets
    the nodes of its order-2 lattice (``tet_q`` [E][10][3], ``pri_q``
    [E][18][3], ``hex_q`` [E][27][3], unwrapped), placed by the straight map
    and then moved by the smooth deformation x_i += amp L_i prod_{j != i}
    sin(2 pi x_j / L_j), periodic in the periodic directions (a bounded
    direction i instead gets a factor sin(pi x_i / L_i) so its boundary
    planes stay flat).  Vertices move with the same deformation, so shared
    nodes coincide and faces stay conforming."""
    per = np.asarray(mesh["period"], dtype=np.float64)
    ext = np.where(per > 0, per, mesh["xyz"].max(axis=0) - mesh["xyz"].min(axis=0))

    def phi(x):
        s = np.sin(2 * np.pi * x / ext)
        out = x.copy()
        for i in range(3):
            j, k = [d for d in range(3) if d != i]
            d = amp * ext[i] * s[..., j] * s[..., k]
            if per[i] == 0:
                d = d * np.sin(np.pi * x[..., i] / ext[i])
            out[..., i] = x[..., i] + d
        return out

    out = dict(mesh)
    out["xyz"] = phi(np.asarray(mesh["xyz"], dtype=np.float64))
    for kind in ("tet", "pri", "hex"):
        v = mesh.get(f"{kind}_v")
        if v is None or not len(v):
            continue
        X = mesh["xyz"][v] + mesh[f"{kind}_img"].astype(np.float64) * per
        out[f"{kind}_q"] = np.ascontiguousarray(phi(_straight_points(kind, X, _order2_lattice(kind))))
    return out


def unwrapped(mesh, kind):
    """Unwrapped vertex coordinates [n_elem][n_vert][3] of 'tet', 'pri' or 'hex'."""
    v = mesh[f"{kind}_v"]
    im = mesh[f"{kind}_img"].astype(np.float64)
    return mesh["xyz"][v] + im * mesh["period"]


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def vortex_tet_cube(n=6, jitter=0.05, seed=0):
    """Periodic unit cube, n^3 cubes x 6 Kuhn tets, jittered (the small FP64
    Euler workload: n=6 gives 1,296 tets)."""
    return mixed_box(n, n, 0, n, (1.0, 1.0, 1.0), jitter=jitter, seed=seed)


def tgv_mixed_box(nxy=32, n_pri_layers=54, n_tet_layers=32, jitter=0.10, seed=0):
    """Periodic [0,2pi)^3: prisms on z in [0,pi), Kuhn tets on z in [pi,2pi).
    Defaults give 110,592 prisms and 196,608 tets with conforming triangular
    interfaces at z=pi and z=0=2pi."""
    L = 2.0 * math.pi
    return mixed_box(nxy, nxy, n_pri_layers, n_tet_layers, (L, L, L),
                     z_split=math.pi, jitter=jitter, seed=seed)


def small_mixed_box(nxy=3, n_pri_layers=2, n_tet_layers=2, jitter=0.10, seed=0,
                    L=2.0 * math.pi):
    """A few-dozen-element version of the mixed box for oracle-sized tests."""
    return mixed_box(nxy, nxy, n_pri_layers, n_tet_layers, (L, L, L),
                     z_split=0.5 * L, jitter=jitter, seed=seed)


# ----------------------------------------------------------------------------
# Initial conditions: conserved variables (rho, rho u, rho v, rho w, E) at
# physical points x, y, z (arrays of any common shape).  Output [5, ...].
# ----------------------------------------------------------------------------

def _conserved(rho, u, v, w, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def isentropic_vortex(x, y, z, eps=5.0, mach=0.5, radius=0.1, centre=(0.5, 0.5),
                      period=(1.0, 1.0), gamma=GAMMA):
    """2-D isentropic vortex in x-y (extruded in z) on a freestream with
    rho = p = 1 moving along +x at the given Mach number.  The vortex is
    placed at the periodic image of ``centre`` nearest to each point."""
    u_inf = mach * math.sqrt(gamma)
    dx = x - centre[0]
    dy = y - centre[1]
    dx = dx - period[0] * np.round(dx / period[0])
    dy = dy - period[1] * np.round(dy / period[1])
    r2 = (dx * dx + dy * dy) / (radius * radius)
    f = np.exp(0.5 * (1.0 - r2))
    du = -eps / (2.0 * math.pi) * f * dy / radius
    dv = eps / (2.0 * math.pi) * f * dx / radius
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return _conserved(rho, u_inf + du, dv, np.zeros_like(x) + 0.0 * z, p, gamma)


def taylor_green(x, y, z, mach=0.1, gamma=GAMMA, rho0=1.0, v0=1.0):
    """Taylor-Green vortex on [0,2pi)^3 at constant temperature."""
    p0 = rho0 * v0 * v0 / (gamma * mach * mach)
    u = v0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -v0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = p0 + rho0 * v0 * v0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = rho0 * p / p0
    return _conserved(rho, u, v, w, p, gamma)


def density_wave(x, y, z, amp=0.2, vel=(1.0, 1.0, 1.0), p=1.0, k=2.0 * math.pi,
                 t=0.0, direction=(1.0, 1.0, 1.0), gamma=GAMMA):
    """Exact periodic Euler solution: rho = 1 + amp sin(k d.(x - vel t)),
    constant velocity and pressure (d has integer components so that the
    wave is periodic on the unit cube)."""
    ph = k * (direction[0] * (x - vel[0] * t) + direction[1] * (y - vel[1] * t)
              + direction[2] * (z - vel[2] * t))
    rho = 1.0 + amp * np.sin(ph)
    one = np.ones_like(rho)
    return _conserved(rho, vel[0] * one, vel[1] * one, vel[2] * one, p * one, gamma)


def shear_wave(x, y, z, amp=1e-3, Ly=2.0 * math.pi, rho=1.0, p=1.0 / (GAMMA * 0.01),
               gamma=GAMMA):
    """u = amp sin(2 pi y / Ly), v = w = 0, constant rho and p."""
    u = amp * np.sin(2.0 * math.pi * y / Ly)
    one = np.ones_like(u)
    return _conserved(rho * one, u, 0 * one, 0 * one, p * one, gamma)


def thermal_wave(x, y, z, amp=1e-2, Ly=2.0 * math.pi, p=1.0, gamma=GAMMA):
    """Fluid at rest, uniform pressure, p/rho = 1 + amp sin(2 pi y / Ly)."""
    T = 1.0 + amp * np.sin(2.0 * math.pi * y / Ly)
    rho = p / T
    zero = np.zeros_like(T)
    return _conserved(rho, zero, zero, zero, p + zero, gamma)


def uniform(x, y, z, rho=1.2, u=0.3, v=-0.2, w=0.1, p=0.9, gamma=GAMMA):
    one = np.ones_like(np.asarray(x, dtype=np.float64))
    return _conserved(rho * one, u * one, v * one, w * one, p * one, gamma)


def random_perturbation(shape, seed, amp=1e-2):
    """Seeded multiplicative noise for parity inputs (values in [1-amp, 1+amp])."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, size=shape)


# ----------------------------------------------------------------------------
# Batched workload: many independent periodic Euler problems
# ----------------------------------------------------------------------------

def batch_problems(n=512, seed=0, e_min=100, e_max=20000):
    """n independent problems on the unit box, each half prisms (z < 1/2) and
    half tets (z > 1/2) by volume on an m x m x 2m grid (8 m^3 elements):
    target element counts log-uniform in [e_min, e_max], m = max(2,
    round((E/8)^(1/3))), orders uniform in {1, 2, 3, 4}, vertex jitter 5 %.
    Returns a list of dicts: mesh arrays, order p, vortex centre (random
    phase) and the problem's seed."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        e = float(np.exp(rng.uniform(np.log(e_min), np.log(e_max))))
        p = int(rng.integers(1, 5))
        centre = (float(rng.uniform()), float(rng.uniform()))
        m = max(2, int(round((e / 8.0) ** (1.0 / 3.0))))
        arrays = mixed_box(m, m, m, m, (1.0, 1.0, 1.0), z_split=0.5, jitter=0.05,
                           seed=seed * 100003 + b)
        out.append({"mesh": arrays, "p": p, "centre": centre, "m": m, "seed": seed * 100003 + b})
    return out
