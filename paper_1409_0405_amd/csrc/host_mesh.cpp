// Element geometry, face matching and flux-point pairing (host).
//
// Paper, Sections 2.1 and 3.3: a mixed unstructured grid of tets, prisms and
// hexahedra; elements interact only through their shared faces.
// Straight-sided elements: the tet map is affine, the prism map is linear on
// the triangle times linear in zeta, the hexahedron map trilinear, and the
// metric terms are evaluated exactly from the map's derivatives.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "fr_host.hpp"

namespace frh {

int n_geom(int etype) { return etype == 0 ? 9 : (etype == 1 ? 15 : 21); }

// Reference vertex signs of the hexahedron (vertices 0-3 at zeta = -1
// counter-clockwise, k+4 above k).
static const int HEX_SIGN[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                   {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

void geom_coeffs(int etype, const double *X, double *c) {
    auto V = [&](int v, int d) { return X[3 * v + d]; };
    if (etype == 2) {
        // c_k = sum_a m_k(r_a, s_a, t_a) X_a / 8 for the monomials
        // m = r, s, t, rs, rt, st, rst
        for (int d = 0; d < 3; ++d)
            for (int k = 0; k < 7; ++k) {
                double acc = 0;
                for (int a = 0; a < 8; ++a) {
                    const int r = HEX_SIGN[a][0], sg = HEX_SIGN[a][1], t = HEX_SIGN[a][2];
                    const int m[7] = {r, sg, t, r * sg, r * t, sg * t, r * sg * t};
                    acc += m[k] * V(a, d);
                }
                c[3 * k + d] = acc / 8;
            }
        return;
    }
    if (etype == 0) {
        for (int d = 0; d < 3; ++d) {
            c[d] = 0.5 * (V(1, d) - V(0, d));
            c[3 + d] = 0.5 * (V(2, d) - V(0, d));
            c[6 + d] = 0.5 * (V(3, d) - V(0, d));
        }
        return;
    }
    for (int d = 0; d < 3; ++d) {
        double A1 = 0.25 * (V(1, d) - V(0, d) + V(4, d) - V(3, d));
        double B1 = 0.25 * (V(2, d) - V(0, d) + V(5, d) - V(3, d));
        double D0 = 0.5 * (V(3, d) - V(0, d));
        double D1 = 0.5 * (V(4, d) - V(1, d));
        double D2 = 0.5 * (V(5, d) - V(2, d));
        double C1 = 0.5 * (D1 - D0), C2 = 0.5 * (D2 - D0);
        c[d] = A1;
        c[3 + d] = B1;
        c[6 + d] = D0 + C1 + C2;
        c[9 + d] = C1;
        c[12 + d] = C2;
    }
}

void jac_at(int etype, const double *c, const double *xi, double col[3][3]) {
    const double r = xi[0], sg = xi[1], t = xi[2];
    for (int d = 0; d < 3; ++d) {
        if (etype == 2) {
            auto C = [&](int k) { return c[3 * (k - 1) + d]; };
            col[0][d] = C(1) + C(4) * sg + C(5) * t + C(7) * sg * t;
            col[1][d] = C(2) + C(4) * r + C(6) * t + C(7) * r * t;
            col[2][d] = C(3) + C(5) * r + C(6) * sg + C(7) * r * sg;
        } else if (etype == 0) {
            col[0][d] = c[d];
            col[1][d] = c[3 + d];
            col[2][d] = c[6 + d];
        } else {
            col[0][d] = c[d] + c[9 + d] * xi[2];
            col[1][d] = c[3 + d] + c[12 + d] * xi[2];
            col[2][d] = c[6 + d] + c[9 + d] * xi[0] + c[12 + d] * xi[1];
        }
    }
}

void map_point(int etype, const double *X, const double *xi, double out[3]) {
    double N[8];
    int nv = n_verts(etype);
    if (etype == 2) {
        for (int a = 0; a < 8; ++a)
            N[a] = (1 + HEX_SIGN[a][0] * xi[0]) * (1 + HEX_SIGN[a][1] * xi[1]) * (1 + HEX_SIGN[a][2] * xi[2]) / 8;
    } else if (etype == 0) {
        N[0] = -(1 + xi[0] + xi[1] + xi[2]) / 2;
        N[1] = (1 + xi[0]) / 2;
        N[2] = (1 + xi[1]) / 2;
        N[3] = (1 + xi[2]) / 2;
    } else {
        double l[3] = {-(xi[0] + xi[1]) / 2, (1 + xi[0]) / 2, (1 + xi[1]) / 2};
        for (int a = 0; a < 3; ++a) {
            N[a] = l[a] * (1 - xi[2]) / 2;
            N[a + 3] = l[a] * (1 + xi[2]) / 2;
        }
    }
    for (int d = 0; d < 3; ++d) {
        out[d] = 0;
        for (int a = 0; a < nv; ++a) out[d] += N[a] * X[3 * a + d];
    }
}

void elem_jac(const TypeHost &T, int t, int64_t e, const double *xi, double col[3][3]) {
    if (!T.Xq.empty()) {
        const int nq = n_qnodes(t);
        double N[27], dN[81];
        quad_shape(t, xi, N, dN);
        const double *Xq = &T.Xq[size_t(e) * nq * 3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) {
                double s = 0;
                for (int a = 0; a < nq; ++a) s += dN[3 * a + k] * Xq[3 * a + d];
                col[k][d] = s;
            }
        return;
    }
    double c[21];
    for (int k = 0; k < n_geom(t); ++k) c[k] = T.geom[size_t(k) * T.nelem + e];
    jac_at(t, c, xi, col);
}

void elem_point(const TypeHost &T, int t, int64_t e, const double *xi, double out[3]) {
    if (!T.Xq.empty()) {
        const int nq = n_qnodes(t);
        double N[27];
        quad_shape(t, xi, N, nullptr);
        const double *Xq = &T.Xq[size_t(e) * nq * 3];
        for (int d = 0; d < 3; ++d) {
            out[d] = 0;
            for (int a = 0; a < nq; ++a) out[d] += N[a] * Xq[3 * a + d];
        }
        return;
    }
    map_point(t, &T.X[size_t(e) * n_verts(t) * 3], xi, out);
}

void tabulate_quad(TypeHost &T, int t) {
    const int nq = n_qnodes(t), nu = T.ops.nu, nf = T.ops.nf;
    T.qN_u.assign(size_t(nu) * nq, 0);
    T.qdN_u.assign(size_t(nu) * nq * 3, 0);
    T.qN_f.assign(size_t(nf) * nq, 0);
    T.qdN_f.assign(size_t(nf) * nq * 3, 0);
    for (int i = 0; i < nu; ++i) quad_shape(t, &T.ops.upts[3 * i], &T.qN_u[size_t(i) * nq], &T.qdN_u[size_t(i) * nq * 3]);
    for (int i = 0; i < nf; ++i) quad_shape(t, &T.ops.fpts[3 * i], &T.qN_f[size_t(i) * nq], &T.qdN_f[size_t(i) * nq * 3]);
}

void elem_jac_at(const TypeHost &T, int t, int64_t e, bool flux, int i, double col[3][3]) {
    if (T.Xq.empty()) {
        elem_jac(T, t, e, flux ? &T.ops.fpts[3 * i] : &T.ops.upts[3 * i], col);
        return;
    }
    const int nq = n_qnodes(t);
    const double *dN = (flux ? T.qdN_f.data() : T.qdN_u.data()) + size_t(i) * nq * 3;
    const double *Xq = &T.Xq[size_t(e) * nq * 3];
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) {
            double s = 0;
            for (int a = 0; a < nq; ++a) s += dN[3 * a + k] * Xq[3 * a + d];
            col[k][d] = s;
        }
}

void elem_point_at(const TypeHost &T, int t, int64_t e, bool flux, int i, double out[3]) {
    if (T.Xq.empty()) {
        elem_point(T, t, e, flux ? &T.ops.fpts[3 * i] : &T.ops.upts[3 * i], out);
        return;
    }
    const int nq = n_qnodes(t);
    const double *N = (flux ? T.qN_f.data() : T.qN_u.data()) + size_t(i) * nq;
    const double *Xq = &T.Xq[size_t(e) * nq * 3];
    for (int d = 0; d < 3; ++d) {
        out[d] = 0;
        for (int a = 0; a < nq; ++a) out[d] += N[a] * Xq[3 * a + d];
    }
}

namespace {

void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// adj[k][j] = J dxi_k/dx_j; its rows are cross products of Jacobian columns.
double adjugate(const double col[3][3], double adj[3][3]) {
    cross3(col[1], col[2], adj[0]);
    cross3(col[2], col[0], adj[1]);
    cross3(col[0], col[1], adj[2]);
    return col[0][0] * adj[0][0] + col[0][1] * adj[0][1] + col[0][2] * adj[0][2];
}

struct FaceRec {
    std::array<int64_t, 4> key;   // sorted vertex ids (4th = -1 for triangles)
    int64_t gid;
    int face, type;
    int64_t elem;
};

}  // namespace

bool build_mesh_host(int p, int64_t nv, const double *xyz, const int64_t nelem[NTYPE],
                     const int64_t *const conn[NTYPE], const int8_t *const img[NTYPE],
                     const double *const quad[NTYPE], const double period[3], int64_t nbf,
                     const int64_t *bfaces, MeshHost &m, std::string &err) {
    m.p = p;
    m.volume = 0;
    for (int t = 0; t < NTYPE; ++t) {
        TypeHost &T = m.t[t];
        T.nelem = nelem[t];
        T.ld = (T.nelem + 63) / 64 * 64;
        if (T.nelem == 0) continue;
        if (T.nelem >= MAX_ELEM) {
            err = "too many elements of one type (limit 2^22)";
            return false;
        }
        T.ops = ref_cached(t, p);
        const int nvt = n_verts(t), ng = n_geom(t), nu = T.ops.nu, nf = T.ops.nf;
        T.X.resize(size_t(T.nelem) * nvt * 3);
        if (quad && quad[t]) {
            T.Xq.assign(quad[t], quad[t] + size_t(T.nelem) * n_qnodes(t) * 3);
            tabulate_quad(T, t);
        }
        T.geom.assign(size_t(ng) * T.nelem, 0);
        T.jdet.resize(size_t(T.nelem) * nu);
        for (int64_t e = 0; e < T.nelem; ++e) {
            double *X = &T.X[size_t(e) * nvt * 3];
            for (int a = 0; a < nvt; ++a) {
                int64_t v = conn[t][e * nvt + a];
                if (v < 0 || v >= nv) {
                    err = "vertex id out of range in " + std::string(type_name(t)) + " " +
                          std::to_string(e);
                    return false;
                }
                for (int d = 0; d < 3; ++d) {
                    double sh = img[t] ? img[t][(e * nvt + a) * 3 + d] * period[d] : 0.0;
                    X[3 * a + d] = xyz[3 * v + d] + sh;
                }
            }
            double c[21];
            geom_coeffs(t, X, c);
            for (int k = 0; k < ng; ++k) T.geom[size_t(k) * T.nelem + e] = c[k];
            // J > 0 at every solution and flux point
            for (int i = 0; i < nu + nf; ++i) {
                double col[3][3], adj[3][3];
                elem_jac_at(T, t, e, i >= nu, i < nu ? i : i - nu, col);
                double J = adjugate(col, adj);
                if (!(J > 0)) {
                    err = std::string("non-positive Jacobian in ") + type_name(t) + " " +
                          std::to_string(e);
                    return false;
                }
                if (i < nu) {
                    T.jdet[size_t(e) * nu + i] = J;
                    m.volume += T.ops.w[i] * J;
                }
            }
        }
    }

    // boundary faces: validated, then left out of the matching
    std::vector<std::array<int64_t, 4>> bl;
    if (nbf < 0 || (nbf && !bfaces)) {
        err = "bad boundary face list";
        return false;
    }
    for (int64_t i = 0; i < nbf; ++i) {
        const int64_t *b = bfaces + 4 * i;
        if (b[0] < 0 || b[0] >= NTYPE || b[1] < 0 || b[1] >= m.t[b[0]].nelem || b[2] < 0 ||
            b[2] >= int64_t(faces_of(int(b[0])).size()) || (b[3] != 1 && b[3] != 2)) {
            err = "boundary face " + std::to_string(i) + " names no face of the mesh or an unknown kind";
            return false;
        }
        bl.push_back({b[0], b[1], b[2], b[3]});
    }
    std::sort(bl.begin(), bl.end());
    for (size_t i = 1; i < bl.size(); ++i)
        if (bl[i][0] == bl[i - 1][0] && bl[i][1] == bl[i - 1][1] && bl[i][2] == bl[i - 1][2]) {
            err = "boundary face listed twice: " + std::string(type_name(int(bl[i][0]))) + " " +
                  std::to_string(bl[i][1]) + " face " + std::to_string(bl[i][2]);
            return false;
        }
    auto is_bnd = [&](int t, int64_t e, int f) {
        const std::array<int64_t, 4> key{t, e, f, 0};
        auto it = std::lower_bound(bl.begin(), bl.end(), key);
        return it != bl.end() && (*it)[0] == t && (*it)[1] == e && (*it)[2] == f;
    };

    // faces keyed by their sorted vertex ids
    std::vector<FaceRec> recs;
    int64_t gbase[NTYPE] = {0, nelem[0], nelem[0] + nelem[1]};
    for (int t = 0; t < NTYPE; ++t) {
        const TypeHost &T = m.t[t];
        if (!T.nelem) continue;
        const auto &faces = faces_of(t);
        const int nvt = n_verts(t);
        for (int64_t e = 0; e < T.nelem; ++e)
            for (size_t f = 0; f < faces.size(); ++f) {
                if (!bl.empty() && is_bnd(t, e, int(f))) continue;
                FaceRec r;
                r.key = {-1, -1, -1, -1};
                for (size_t a = 0; a < faces[f].size(); ++a) r.key[a] = conn[t][e * nvt + faces[f][a]];
                std::sort(r.key.begin(), r.key.begin() + faces[f].size());
                r.gid = gbase[t] + e;
                r.face = int(f);
                r.type = t;
                r.elem = e;
                recs.push_back(r);
            }
    }
    std::sort(recs.begin(), recs.end(), [](const FaceRec &a, const FaceRec &b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.gid != b.gid) return a.gid < b.gid;
        return a.face < b.face;
    });

    struct PP {
        uint32_t L, R;
        double n[3], sL, sR;
    };
    std::vector<PP> pp;
    double scale = 1.0;
    for (int64_t v = 0; v < nv; ++v)
        for (int d = 0; d < 3; ++d) scale = std::max(scale, std::fabs(xyz[3 * v + d]));
    const double tol = 1e-9 * scale;

    // Faces with the same vertex set are the same physical face seen from two
    // elements, except on periodic meshes only two cells wide, where distinct
    // faces can share all vertex ids: those are told apart by their centroids,
    // which coincide modulo the period for the two sides of one face.
    auto centroid = [&](const FaceRec &r, double c[3]) {
        const int nvt = n_verts(r.type);
        const double *X = &m.t[r.type].X[size_t(r.elem) * nvt * 3];
        const auto &F = faces_of(r.type)[r.face];
        c[0] = c[1] = c[2] = 0;
        for (int a : F)
            for (int d = 0; d < 3; ++d) c[d] += X[3 * a + d] / double(F.size());
    };
    auto same_face = [&](const FaceRec &x, const FaceRec &y) {
        double cx[3], cy[3];
        centroid(x, cx);
        centroid(y, cy);
        for (int d = 0; d < 3; ++d) {
            double dd = cx[d] - cy[d];
            if (period[d] > 0) dd -= period[d] * std::round(dd / period[d]);
            if (std::fabs(dd) > tol) return false;
        }
        return true;
    };
    auto pair_faces = [&](const FaceRec &A, const FaceRec &B) -> bool {   // A sorts first: side L
        const TypeHost &TA = m.t[A.type], &TB = m.t[B.type];
        const int nvA = n_verts(A.type), nvB = n_verts(B.type);
        const double *XA = &TA.X[size_t(A.elem) * nvA * 3];
        const double *XB = &TB.X[size_t(B.elem) * nvB * 3];
        // periodic shift between the two unwrapped copies: via a shared vertex
        int64_t v0 = A.key[0];
        int ia = -1, ib = -1;
        for (int a = 0; a < nvA; ++a)
            if (conn[A.type][A.elem * nvA + a] == v0) ia = a;
        for (int a = 0; a < nvB; ++a)
            if (conn[B.type][B.elem * nvB + a] == v0) ib = a;
        double shift[3];
        for (int d = 0; d < 3; ++d) shift[d] = XA[3 * ia + d] - XB[3 * ib + d];
        const int fa0 = TA.ops.face_off[A.face], fa1 = TA.ops.face_off[A.face + 1];
        const int fb0 = TB.ops.face_off[B.face], fb1 = TB.ops.face_off[B.face + 1];
        if (fa1 - fa0 != fb1 - fb0) {
            err = "non-conforming face between " + std::string(type_name(A.type)) + " " +
                  std::to_string(A.elem) + " and " + type_name(B.type) + " " + std::to_string(B.elem);
            return false;
        }
        std::vector<char> used(fb1 - fb0, 0);
        double xbs[25][3];
        for (int jb = fb0; jb < fb1; ++jb) {
            elem_point_at(TB, B.type, B.elem, true, jb, xbs[jb - fb0]);
            for (int d = 0; d < 3; ++d) xbs[jb - fb0][d] += shift[d];
        }
        for (int ja = fa0; ja < fa1; ++ja) {
            double xa[3];
            elem_point_at(TA, A.type, A.elem, true, ja, xa);
            int best = -1;
            double bd = 1e300;
            for (int jb = fb0; jb < fb1; ++jb) {
                const double *xb = xbs[jb - fb0];
                double d2 = 0;
                for (int d = 0; d < 3; ++d) d2 += (xa[d] - xb[d]) * (xa[d] - xb[d]);
                if (d2 < bd) { bd = d2; best = jb; }
            }
            if (std::sqrt(bd) > tol || used[best - fb0]) {
                err = "flux points do not coincide on the face between " +
                      std::string(type_name(A.type)) + " " + std::to_string(A.elem) + " and " +
                      type_name(B.type) + " " + std::to_string(B.elem);
                return false;
            }
            used[best - fb0] = 1;
            PP q;
            q.L = pack_side(A.elem, ja, A.type);
            q.R = pack_side(B.elem, best, B.type);
            double col[3][3], adj[3][3], nA[3], nB[3];
            elem_jac_at(TA, A.type, A.elem, true, ja, col);
            adjugate(col, adj);
            for (int jd = 0; jd < 3; ++jd) {
                nA[jd] = 0;
                for (int k = 0; k < 3; ++k) nA[jd] += adj[k][jd] * TA.ops.nref[3 * ja + k];
            }
            elem_jac_at(TB, B.type, B.elem, true, best, col);
            adjugate(col, adj);
            for (int jd = 0; jd < 3; ++jd) {
                nB[jd] = 0;
                for (int k = 0; k < 3; ++k) nB[jd] += adj[k][jd] * TB.ops.nref[3 * best + k];
            }
            q.sL = std::sqrt(nA[0] * nA[0] + nA[1] * nA[1] + nA[2] * nA[2]);
            q.sR = std::sqrt(nB[0] * nB[0] + nB[1] * nB[1] + nB[2] * nB[2]);
            for (int d = 0; d < 3; ++d) q.n[d] = nA[d] / q.sL;
            pp.push_back(q);
        }
        return true;
    };
    for (size_t i = 0; i < recs.size();) {
        size_t j = i;
        while (j < recs.size() && recs[j].key == recs[i].key) ++j;
        std::vector<char> done(j - i, 0);
        for (size_t x = i; x < j; ++x) {
            if (done[x - i]) continue;
            size_t y = x + 1;
            while (y < j && (done[y - i] || !same_face(recs[x], recs[y]))) ++y;
            if (y == j) {
                err = "unmatched face: " + std::string(type_name(recs[x].type)) + " " +
                      std::to_string(recs[x].elem) + " face " + std::to_string(recs[x].face);
                return false;
            }
            done[x - i] = done[y - i] = 1;
            if (!pair_faces(recs[x], recs[y])) return false;
        }
        i = j;
    }

    // order by (type L, flux point L, element L) for coalesced side-L access
    auto keyL = [](uint32_t s) {
        return (uint64_t(side_type(s)) << 40) | (uint64_t(side_fpt(s)) << 32) | uint64_t(side_elem(s));
    };
    std::sort(pp.begin(), pp.end(), [&](const PP &a, const PP &b) { return keyL(a.L) < keyL(b.L); });

    // boundary points: outward normal adj^T n_ref at each flux point of the face
    {
        struct BP {
            uint32_t side;
            double n[3], s;
            int8_t kind;
        };
        std::vector<BP> bp;
        for (const auto &b : bl) {
            const int t = int(b[0]);
            const TypeHost &T = m.t[t];
            for (int j = T.ops.face_off[b[2]]; j < T.ops.face_off[b[2] + 1]; ++j) {
                double col[3][3], adj[3][3], nn[3];
                elem_jac_at(T, t, b[1], true, j, col);
                adjugate(col, adj);
                for (int jd = 0; jd < 3; ++jd) {
                    nn[jd] = 0;
                    for (int k = 0; k < 3; ++k) nn[jd] += adj[k][jd] * T.ops.nref[3 * j + k];
                }
                BP q;
                q.side = pack_side(b[1], j, t);
                q.s = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
                for (int d = 0; d < 3; ++d) q.n[d] = nn[d] / q.s;
                q.kind = int8_t(b[3]);
                bp.push_back(q);
            }
        }
        std::sort(bp.begin(), bp.end(), [&](const BP &a, const BP &b) { return keyL(a.side) < keyL(b.side); });
        BndTable &B = m.bnd;
        B = BndTable();
        for (const BP &q : bp) {
            B.side.push_back(q.side);
            for (int d = 0; d < 3; ++d) B.nhat.push_back(q.n[d]);
            B.s.push_back(q.s);
            B.kind.push_back(q.kind);
        }
    }
    PairTable &P = m.pairs;
    const size_t n = pp.size();
    P.sideL.resize(n);
    P.sideR.resize(n);
    P.nhat.resize(3 * n);
    P.sL.resize(n);
    P.sR.resize(n);
    for (size_t i = 0; i < n; ++i) {
        P.sideL[i] = pp[i].L;
        P.sideR[i] = pp[i].R;
        for (int d = 0; d < 3; ++d) P.nhat[3 * i + d] = pp[i].n[d];
        P.sL[i] = pp[i].sL;
        P.sR[i] = pp[i].sR;
    }
    return true;
}

std::vector<int32_t> face_neighbours(const MeshHost &m) {
    const int64_t nt = m.t[0].nelem, ntot = nt + m.t[1].nelem;
    std::vector<int32_t> nb(size_t(ntot) * 5, -1);
    auto info = [&](uint32_t s, int64_t &g, int &f) {
        const int t = side_type(s);
        g = (t ? nt : 0) + side_elem(s);
        f = m.t[t].ops.fface[side_fpt(s)];
    };
    for (size_t j = 0; j < m.pairs.sideL.size(); ++j) {
        int64_t gl, gr;
        int fl, fr;
        info(m.pairs.sideL[j], gl, fl);
        info(m.pairs.sideR[j], gr, fr);
        nb[size_t(gl) * 5 + fl] = int32_t(gr);
        nb[size_t(gr) * 5 + fr] = int32_t(gl);
    }
    return nb;
}

bool merge_meshes(const std::vector<MeshHost> &parts, MeshHost &out,
                  std::vector<std::array<int64_t, NTYPE>> &elem_off, std::string &err) {
    if (parts.empty()) {
        err = "no meshes to merge";
        return false;
    }
    out = MeshHost();
    out.p = parts[0].p;
    elem_off.assign(parts.size(), std::array<int64_t, NTYPE>{});
    for (int t = 0; t < NTYPE; ++t) {
        int64_t n = 0;
        for (size_t i = 0; i < parts.size(); ++i) {
            if (parts[i].p != out.p) {
                err = "merged meshes must share one order";
                return false;
            }
            elem_off[i][t] = n;
            n += parts[i].t[t].nelem;
            if (parts[i].t[t].nelem && !out.t[t].ops.nu) out.t[t].ops = parts[i].t[t].ops;
        }
        if (n >= MAX_ELEM) {
            err = "too many elements of one type in a merged batch (limit 2^22)";
            return false;
        }
        TypeHost &T = out.t[t];
        T.nelem = n;
        T.ld = (n + 63) / 64 * 64;
        if (!n) continue;
        int ncurved = 0, nparts = 0;
        for (const auto &P : parts)
            if (P.t[t].nelem) {
                ++nparts;
                ncurved += !P.t[t].Xq.empty();
            }
        if (ncurved && ncurved != nparts) {
            err = "merged meshes of one order must be all curved or all straight for each type";
            return false;
        }
        const int ng = n_geom(t);
        T.geom.assign(size_t(ng) * n, 0.0);
        for (size_t i = 0; i < parts.size(); ++i) {
            const TypeHost &P = parts[i].t[t];
            if (!P.nelem) continue;
            T.X.insert(T.X.end(), P.X.begin(), P.X.end());
            T.Xq.insert(T.Xq.end(), P.Xq.begin(), P.Xq.end());
            if (!P.Xq.empty() && T.qN_u.empty()) {
                T.qN_u = P.qN_u;
                T.qdN_u = P.qdN_u;
                T.qN_f = P.qN_f;
                T.qdN_f = P.qdN_f;
            }
            T.jdet.insert(T.jdet.end(), P.jdet.begin(), P.jdet.end());
            for (int k = 0; k < ng; ++k)
                std::copy(P.geom.begin() + size_t(k) * P.nelem, P.geom.begin() + size_t(k + 1) * P.nelem,
                          T.geom.begin() + size_t(k) * n + elem_off[i][t]);
        }
    }
    struct PP {
        uint32_t L, R;
        double n[3], sL, sR;
    };
    std::vector<PP> pp;
    auto shift = [&](uint32_t side, size_t i) {
        const int t = side_type(side);
        return pack_side(side_elem(side) + elem_off[i][t], side_fpt(side), t);
    };
    struct BP {
        uint32_t side;
        double n[3], s;
        int8_t kind;
    };
    std::vector<BP> bp;
    for (size_t i = 0; i < parts.size(); ++i) {
        const PairTable &P = parts[i].pairs;
        for (size_t j = 0; j < P.sideL.size(); ++j)
            pp.push_back({shift(P.sideL[j], i), shift(P.sideR[j], i),
                          {P.nhat[3 * j], P.nhat[3 * j + 1], P.nhat[3 * j + 2]}, P.sL[j], P.sR[j]});
        const BndTable &B = parts[i].bnd;
        for (size_t j = 0; j < B.side.size(); ++j)
            bp.push_back({shift(B.side[j], i), {B.nhat[3 * j], B.nhat[3 * j + 1], B.nhat[3 * j + 2]}, B.s[j],
                          B.kind[j]});
        out.volume += parts[i].volume;
    }
    auto keyL = [](uint32_t s) {
        return (uint64_t(side_type(s)) << 40) | (uint64_t(side_fpt(s)) << 32) | uint64_t(side_elem(s));
    };
    std::stable_sort(pp.begin(), pp.end(), [&](const PP &a, const PP &b) { return keyL(a.L) < keyL(b.L); });
    std::stable_sort(bp.begin(), bp.end(), [&](const BP &a, const BP &b) { return keyL(a.side) < keyL(b.side); });
    for (const BP &q : bp) {
        out.bnd.side.push_back(q.side);
        for (int d = 0; d < 3; ++d) out.bnd.nhat.push_back(q.n[d]);
        out.bnd.s.push_back(q.s);
        out.bnd.kind.push_back(q.kind);
    }
    PairTable &T = out.pairs;
    T.sideL.resize(pp.size());
    T.sideR.resize(pp.size());
    T.nhat.resize(3 * pp.size());
    T.sL.resize(pp.size());
    T.sR.resize(pp.size());
    for (size_t j = 0; j < pp.size(); ++j) {
        T.sideL[j] = pp[j].L;
        T.sideR[j] = pp[j].R;
        for (int d = 0; d < 3; ++d) T.nhat[3 * j + d] = pp[j].n[d];
        T.sL[j] = pp[j].sL;
        T.sR[j] = pp[j].sR;
    }
    return true;
}

}  // namespace frh
