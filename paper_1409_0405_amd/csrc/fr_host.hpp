// Host-side core of the FR library: reference operators, geometry, pairing.
// Internal header (not part of the C ABI).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace frh {

constexpr int NVAR = 5;
constexpr int NTYPE = 3;          // 0 tet, 1 prism, 2 hexahedron
constexpr int ELEM_BITS = 22;     // side word: elem | fpt << 22 | type << 30
constexpr int64_t MAX_ELEM = int64_t(1) << ELEM_BITS;

inline const char *type_name(int t) { return t == 0 ? "tet" : (t == 1 ? "prism" : "hex"); }

// Reference element of one type at one order, built in extended precision and
// stored as double.  Point / face conventions:
//  * triangle point set (order p): barycentrics with i0+i1+i2 = p,
//    lambda_a = (1 + 2 v_{i_a} - v_{i_b} - v_{i_c}) / 3 from the Gauss-Legendre
//    nodes v mapped to (0,1); enumeration i2 outer, i1 inner;
//  * tet point set: lambda_a = (1 + 3 v_{i_a} - sum_{b!=a} v_{i_b}) / 4,
//    enumeration i3, i2, i1 (outer to inner);
//  * prism solution points: Gauss-Legendre layer in zeta (outer) x triangle
//    set (inner);
//  * hexahedron [-1,1]^3 (vertices 0-3 counter-clockwise at zeta = -1, k+4
//    above k): Gauss-Legendre tensor points, index (k(p+1) + j)(p+1) + i
//    with xi fastest;
//  * faces: tet (0,1,2) (0,1,3) (0,2,3) (1,2,3); prism (0,1,2) (3,4,5)
//    (0,1,4,3) (1,2,5,4) (2,0,3,5); hexahedron (0,1,2,3) (4,5,6,7) (0,1,5,4)
//    (1,2,6,5) (2,3,7,6) (3,0,4,7); triangle-face points l0 a + l1 b + l2 c;
//    quad-face points a + (1+s_i)/2 (b-a) + (1+t_j)/2 (d-a), index j(p+1)+i.
struct RefOps {
    int etype = 0, p = 0, nu = 0, nf = 0;
    std::vector<double> upts;   // [nu][3]
    std::vector<double> fpts;   // [nf][3]
    std::vector<int> fface;     // [nf] local face of each flux point
    std::vector<int> face_off;  // [nfaces + 1]
    std::vector<double> nref;   // [nf][3] outward unit reference normals
    std::vector<double> M0;     // [nf][nu]
    std::vector<double> G;      // [3][nu][nu]
    std::vector<double> L;      // [nu][nf]
    std::vector<double> w;      // [nu]
    double volume = 0;
};

RefOps build_ref(int etype, int p);
// build_ref memoised per (type, order); thread safe.
const RefOps &ref_cached(int etype, int p);

int n_upts(int etype, int p);
int n_fpts(int etype, int p);

// Learned-closure operators (reference element).  phi_a (a = 0..3) is the
// Gram-Schmidt orthonormalisation of (1, xi, eta, zeta), in that order,
// under the reference L2 inner product.
//   moments    [4][nu(p)]   m_a = int phi_a u from nodal values of order p
//   lift       [nu(p)][4]   nodal values of sum_a phi_a y_a
//   projection [nu(q)][nu(p)]  L2 projection from order p to order q
std::vector<double> build_moments(int etype, int p);
std::vector<double> build_lift(int etype, int p);
std::vector<double> build_projection(int etype, int p, int q);

// Reference vertices and faces
const std::vector<std::vector<int>> &faces_of(int etype);
int n_verts(int etype);
void ref_vertex(int etype, int v, double out[3]);

// Jacobian coefficient vectors of one element from its (unwrapped) vertices:
// tet  -> 9 values: columns dx/dxi, dx/deta, dx/dzeta (constant);
// prism-> 15 values: A1, B1, C0, C1, C2 with dx/dxi = A1 + C1 z,
//         dx/deta = B1 + C2 z, dx/dzeta = C0 + C1 x + C2 y;
// hex  -> 21 values: c1..c7 of the trilinear map x = c0 + c1 r + c2 s + c3 t
//         + c4 rs + c5 rt + c6 st + c7 rst, so dx/dr = c1 + c4 s + c5 t + c7 st,
//         dx/ds = c2 + c4 r + c6 t + c7 rt, dx/dt = c3 + c5 r + c6 s + c7 rs.
int n_geom(int etype);
void geom_coeffs(int etype, const double *X, double *c);
// Jacobian matrix columns at a reference point from the coefficients.
void jac_at(int etype, const double *c, const double *xi, double col[3][3]);
// Physical position of a reference point.
void map_point(int etype, const double *X, const double *xi, double out[3]);

// Quadratically curved geometry: nodes on the element's order-2 lattice
// (tet (a,b,c) a+b+c <= 2, prism (a,b) a+b <= 2 times c <= 2, hexahedron
// (a,b,c) <= 2; reference coordinates -1 + index; c outermost, a innermost)
// and their Lagrange shape functions N [nq], reference derivatives dN [nq][3].
int n_qnodes(int etype);
void quad_shape(int etype, const double *xi, double *N, double *dN);

struct PairTable {
    // one entry per paired flux point, sorted by (type L, fpt L, elem L)
    std::vector<uint32_t> sideL, sideR;   // elem | fpt << 22 | type << 30
    std::vector<double> nhat;             // [n][3] unit normal out of side L
    std::vector<double> sL, sR;           // |adj^T n_ref| on each side
};

// Boundary flux points (faces listed as wall or far field), sorted like the
// pairs by (type, flux point, element).
struct BndTable {
    std::vector<uint32_t> side;           // elem | fpt << 22 | type << 30
    std::vector<double> nhat;             // [n][3] outward unit normal
    std::vector<double> s;                // |adj^T n_ref|
    std::vector<int8_t> kind;             // 1 wall, 2 far field
};

struct TypeHost {
    int64_t nelem = 0, ld = 0;
    RefOps ops;
    std::vector<double> X;       // [nelem][nverts][3] unwrapped vertices
    std::vector<double> Xq;      // [nelem][nq][3] quadratic nodes (curved types), else empty
    // curved types: shape functions and reference derivatives of the nodes at
    // the solution points [nu][nq], [nu][nq][3] and flux points [nf][nq], [nf][nq][3]
    std::vector<double> qN_u, qdN_u, qN_f, qdN_f;
    std::vector<double> geom;    // [n_geom][nelem]
    std::vector<double> jdet;    // [nelem][nu] Jacobian determinant at upts
};

struct MeshHost {
    int p = 0;
    TypeHost t[NTYPE];
    PairTable pairs;
    BndTable bnd;
    double volume = 0;
};

// Neighbour across each local face, global type-major element id
// [n_tet + n_pri][5], -1 where the element has no such face (tets and prisms
// only: the caller refuses meshes with hexahedra).
std::vector<int32_t> face_neighbours(const MeshHost &m);

// Builds geometry and pairing; returns false with a message on a bad mesh.
// Jacobian columns and physical position of element e of type t at a
// reference point (straight or curved geometry).
void elem_jac(const TypeHost &T, int t, int64_t e, const double *xi, double col[3][3]);
void elem_point(const TypeHost &T, int t, int64_t e, const double *xi, double out[3]);
// The same at solution point i (flux = false) or flux point i (flux = true),
// from tabulated shape functions for curved types.
void elem_jac_at(const TypeHost &T, int t, int64_t e, bool flux, int i, double col[3][3]);
void elem_point_at(const TypeHost &T, int t, int64_t e, bool flux, int i, double out[3]);
// Fill the tables above (curved types).
void tabulate_quad(TypeHost &T, int t);

// Per type t: nelem[t] elements, connectivity conn[t] [nelem][n_verts(t)],
// periodic images img[t] (may be null), quadratic nodes quad[t] [nelem][nq][3]
// (null: straight-sided).  Boundary faces bfaces [nbf][4] = (type, element,
// local face, kind 1 wall / 2 far field) pair with nothing.
bool build_mesh_host(int p, int64_t nv, const double *xyz, const int64_t nelem[NTYPE],
                     const int64_t *const conn[NTYPE], const int8_t *const img[NTYPE],
                     const double *const quad[NTYPE], const double period[3], int64_t nbf,
                     const int64_t *bfaces, MeshHost &m, std::string &err);

// Merge independent meshes of one order into one element array per type.
// Element indices of each part are offset by the elements of the parts
// before it (elem_off[part][type]); the pairing stays within each part.
bool merge_meshes(const std::vector<MeshHost> &parts, MeshHost &out,
                  std::vector<std::array<int64_t, NTYPE>> &elem_off, std::string &err);

inline uint32_t pack_side(int64_t e, int f, int t) {
    return uint32_t(e) | (uint32_t(f) << ELEM_BITS) | (uint32_t(t) << 30);
}
inline int64_t side_elem(uint32_t s) { return int64_t(s & ((1u << ELEM_BITS) - 1)); }
inline int side_fpt(uint32_t s) { return int((s >> ELEM_BITS) & 0xffu); }
inline int side_type(uint32_t s) { return int(s >> 30); }

}  // namespace frh
