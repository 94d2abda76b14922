// Reference operators of the FR scheme, built on the host.
//
// Paper, Section 2.1: an FR step is mostly products of constant operator
// matrices with state matrices; Table 2 gives the dimensions of the
// volume-to-surface interpolation operator M0 for tets, prisms and hexahedra.  The correction is the DG lift
// (Section 3.4: "a DG scheme"), built in the reference element.
//
// Construction route: a monomial basis phi_a, its Vandermonde matrix at the
// solution points inverted by Gauss-Jordan elimination in long double, and
// Duffy-collapsed Gauss-Legendre quadrature for the nodal mass matrix and the
// face integrals:
//   M0  = Phi(fpts) V^-1,       G_k = dPhi/dxi_k(upts) V^-1,
//   L   = M^-1 E,  M_ij = int l_i l_j,  E_i(f,j) = int_f l_i l^f_j ds,
//   w   = V^-T int phi,
// with the Lagrange functions l_i = sum_a phi_a Vinv[a][i] evaluated at the
// quadrature points.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>

#include "fr_host.hpp"

namespace frh {

using ld = long double;

namespace {

// Gauss-Legendre nodes (ascending) and weights on [-1,1] by Newton's method on
// the three-term Legendre recurrence.
void gauss_legendre(int n, std::vector<ld> &x, std::vector<ld> &w) {
    x.assign(n, 0);
    w.assign(n, 0);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        ld dp = 0;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            dp = n * (z * p1 - p0) / (z * z - 1);
            ld dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-19L) break;
        }
        ld p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2 / ((1 - z * z) * dp * dp);
    }
}

// Gauss-Jordan inverse with partial pivoting, in place, row-major n x n.
void invert(std::vector<ld> &A, int n) {
    std::vector<ld> I(size_t(n) * n, 0);
    for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[size_t(r) * n + c]) > std::fabs(A[size_t(piv) * n + c])) piv = r;
        if (A[size_t(piv) * n + c] == 0) throw std::runtime_error("singular matrix");
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[size_t(piv) * n + k], A[size_t(c) * n + k]);
                std::swap(I[size_t(piv) * n + k], I[size_t(c) * n + k]);
            }
        ld d = A[size_t(c) * n + c];
        for (int k = 0; k < n; ++k) {
            A[size_t(c) * n + k] /= d;
            I[size_t(c) * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            ld f = A[size_t(r) * n + c];
            if (f == 0) continue;
            for (int k = 0; k < n; ++k) {
                A[size_t(r) * n + k] -= f * A[size_t(c) * n + k];
                I[size_t(r) * n + k] -= f * I[size_t(c) * n + k];
            }
        }
    }
    A.swap(I);
}

// C = A (m x k) * B (k x n)
std::vector<ld> matmul(const std::vector<ld> &A, const std::vector<ld> &B, int m, int k, int n) {
    std::vector<ld> C(size_t(m) * n, 0);
    for (int i = 0; i < m; ++i)
        for (int l = 0; l < k; ++l) {
            ld a = A[size_t(i) * k + l];
            if (a == 0) continue;
            for (int j = 0; j < n; ++j) C[size_t(i) * n + j] += a * B[size_t(l) * n + j];
        }
    return C;
}

ld ipow(ld x, int e) {
    ld r = 1;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// Monomial basis of the element space: tet X^a Y^b Z^c (a+b+c <= p), prism
// X^a Y^b t^c (a+b <= p, c <= p), with X = (1+xi)/2, Y = (1+eta)/2,
// Z = (1+zeta)/2 and t = zeta; hexahedron xi^a eta^b zeta^c (a, b, c <= p),
// centred monomials (the tensor Vandermonde's condition number is the
// product of the 1-D ones, small on [-1, 1]).
struct Monos {
    int etype, p;
    std::vector<int> e;   // [n][3]
    Monos(int et, int pp) : etype(et), p(pp) {
        for (int a = 0; a <= p; ++a)
            for (int b = 0; b <= (etype == 2 ? p : p - a); ++b)
                for (int c = 0; c <= (etype == 0 ? p - a - b : p); ++c) {
                    e.push_back(a);
                    e.push_back(b);
                    e.push_back(c);
                }
    }
    int n() const { return int(e.size() / 3); }
    // values [n] and gradient [3][n] at reference point x
    void eval(const ld *x, ld *val, ld *grad) const {
        const bool hex = etype == 2;
        ld X = hex ? x[0] : (1 + x[0]) / 2, Y = hex ? x[1] : (1 + x[1]) / 2;
        ld Z = etype == 0 ? (1 + x[2]) / 2 : x[2];
        ld dXY = hex ? ld(1) : ld(0.5), dZ = etype == 0 ? ld(0.5) : ld(1);
        for (int m = 0; m < n(); ++m) {
            int a = e[3 * m], b = e[3 * m + 1], c = e[3 * m + 2];
            ld va = ipow(X, a), vb = ipow(Y, b), vc = ipow(Z, c);
            val[m] = va * vb * vc;
            if (grad) {
                grad[m] = (a ? a * ipow(X, a - 1) * dXY : 0) * vb * vc;
                grad[n() + m] = va * (b ? b * ipow(Y, b - 1) * dXY : 0) * vc;
                grad[2 * n() + m] = va * vb * (c ? c * ipow(Z, c - 1) * dZ : 0);
            }
        }
    }
};

const ld TET_V[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
const ld PRI_V[6][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1},
                        {-1, -1, 1},  {1, -1, 1},  {-1, 1, 1}};

const ld HEX_V[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                        {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

const ld *vert(int etype, int v) { return etype == 0 ? TET_V[v] : (etype == 1 ? PRI_V[v] : HEX_V[v]); }

// Triangle barycentrics of the order-p set.
std::vector<ld> tri_bary(int p) {
    std::vector<ld> x, w;
    gauss_legendre(p + 1, x, w);
    std::vector<ld> v(p + 1), out;
    for (int i = 0; i <= p; ++i) v[i] = (1 + x[i]) / 2;
    for (int i2 = 0; i2 <= p; ++i2)
        for (int i1 = 0; i1 + i2 <= p; ++i1) {
            int ii[3] = {p - i1 - i2, i1, i2};
            for (int a = 0; a < 3; ++a)
                out.push_back((1 + 2 * v[ii[a]] - v[ii[(a + 1) % 3]] - v[ii[(a + 2) % 3]]) / 3);
        }
    return out;
}

std::vector<ld> tet_bary(int p) {
    std::vector<ld> x, w;
    gauss_legendre(p + 1, x, w);
    std::vector<ld> v(p + 1), out;
    for (int i = 0; i <= p; ++i) v[i] = (1 + x[i]) / 2;
    for (int i3 = 0; i3 <= p; ++i3)
        for (int i2 = 0; i2 + i3 <= p; ++i2)
            for (int i1 = 0; i1 + i2 + i3 <= p; ++i1) {
                int ii[4] = {p - i1 - i2 - i3, i1, i2, i3};
                ld tot = v[ii[0]] + v[ii[1]] + v[ii[2]] + v[ii[3]];
                for (int a = 0; a < 4; ++a) out.push_back((1 + 4 * v[ii[a]] - tot) / 4);
            }
    return out;
}

// Quadrature on the reference element by Duffy collapse of Gauss-Legendre.
void volume_rule(int etype, int n, std::vector<ld> &pts, std::vector<ld> &wts) {
    std::vector<ld> x, w;
    gauss_legendre(n, x, w);
    pts.clear();
    wts.clear();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                ld a = x[i], b = x[j], c = x[k];
                if (etype == 2) {
                    pts.push_back(a);
                    pts.push_back(b);
                    pts.push_back(c);
                    wts.push_back(w[i] * w[j] * w[k]);
                } else if (etype == 0) {
                    pts.push_back((1 + a) * (1 - b) * (1 - c) / 4 - 1);
                    pts.push_back((1 + b) * (1 - c) / 2 - 1);
                    pts.push_back(c);
                    wts.push_back(w[i] * w[j] * w[k] * (1 - b) * (1 - c) * (1 - c) / 8);
                } else {
                    pts.push_back((1 + a) * (1 - b) / 2 - 1);
                    pts.push_back(b);
                    pts.push_back(c);
                    wts.push_back(w[i] * w[j] * w[k] * (1 - b) / 2);
                }
            }
}

// Face parameter rule: triangle (u,v) on the reference triangle, quad (s,t)
// on [-1,1]^2.
void face_rule(int nv, int n, std::vector<ld> &uv, std::vector<ld> &wts) {
    std::vector<ld> x, w;
    gauss_legendre(n, x, w);
    uv.clear();
    wts.clear();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (nv == 3) {
                uv.push_back((1 + x[i]) * (1 - x[j]) / 2 - 1);
                uv.push_back(x[j]);
                wts.push_back(w[i] * w[j] * (1 - x[j]) / 2);
            } else {
                uv.push_back(x[i]);
                uv.push_back(x[j]);
                wts.push_back(w[i] * w[j]);
            }
        }
}

// Face parameter coordinates of the face point set.
std::vector<ld> face_param_points(int nv, int p) {
    std::vector<ld> out;
    if (nv == 3) {
        auto b = tri_bary(p);
        for (size_t i = 0; i < b.size() / 3; ++i) {
            out.push_back(-1 + 2 * b[3 * i + 1]);
            out.push_back(-1 + 2 * b[3 * i + 2]);
        }
    } else {
        std::vector<ld> x, w;
        gauss_legendre(p + 1, x, w);
        for (int j = 0; j <= p; ++j)
            for (int i = 0; i <= p; ++i) {
                out.push_back(x[i]);
                out.push_back(x[j]);
            }
    }
    return out;
}

void face_map(int etype, const std::vector<int> &f, const ld *uv, ld *out) {
    const ld *A = vert(etype, f[0]), *B = vert(etype, f[1]);
    if (f.size() == 3) {
        const ld *C = vert(etype, f[2]);
        ld l0 = -(uv[0] + uv[1]) / 2, l1 = (1 + uv[0]) / 2, l2 = (1 + uv[1]) / 2;
        for (int d = 0; d < 3; ++d) out[d] = l0 * A[d] + l1 * B[d] + l2 * C[d];
    } else {
        const ld *D = vert(etype, f[3]);
        ld s = (1 + uv[0]) / 2, t = (1 + uv[1]) / 2;
        for (int d = 0; d < 3; ++d) out[d] = A[d] + s * (B[d] - A[d]) + t * (D[d] - A[d]);
    }
}

void cross(const ld *a, const ld *b, ld *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Face Lagrange basis of the face point set, evaluated at parameter uv.
struct FaceLagrange {
    int nv, p, n;
    std::vector<ld> vinv;      // triangle: inverse face Vandermonde (monomials)
    std::vector<ld> nodes;     // quad: 1-D Gauss-Legendre nodes
    FaceLagrange(int nv_, int p_) : nv(nv_), p(p_) {
        if (nv == 3) {
            n = (p + 1) * (p + 2) / 2;
            auto pts = face_param_points(3, p);
            vinv.resize(size_t(n) * n);
            for (int i = 0; i < n; ++i) mono(&pts[2 * i], &vinv[size_t(i) * n]);
            invert(vinv, n);
        } else {
            n = (p + 1) * (p + 1);
            std::vector<ld> w;
            gauss_legendre(p + 1, nodes, w);
        }
    }
    void mono(const ld *uv, ld *v) const {   // (1+u)/2^a (1+v)/2^b, a+b <= p
        int m = 0;
        for (int a = 0; a <= p; ++a)
            for (int b = 0; a + b <= p; ++b)
                v[m++] = ipow((1 + uv[0]) / 2, a) * ipow((1 + uv[1]) / 2, b);
    }
    ld lag1(int i, ld s) const {
        ld r = 1;
        for (int m = 0; m <= p; ++m)
            if (m != i) r *= (s - nodes[m]) / (nodes[i] - nodes[m]);
        return r;
    }
    void eval(const ld *uv, ld *out) const {
        if (nv == 3) {
            std::vector<ld> v(n);
            mono(uv, v.data());
            for (int j = 0; j < n; ++j) {
                ld s = 0;
                for (int a = 0; a < n; ++a) s += v[a] * vinv[size_t(a) * n + j];
                out[j] = s;
            }
        } else {
            for (int jt = 0; jt <= p; ++jt)
                for (int is = 0; is <= p; ++is) out[jt * (p + 1) + is] = lag1(is, uv[0]) * lag1(jt, uv[1]);
        }
    }
};

}  // namespace

int n_upts(int etype, int p) {
    if (etype == 2) return (p + 1) * (p + 1) * (p + 1);
    return etype == 0 ? (p + 1) * (p + 2) * (p + 3) / 6 : (p + 1) * (p + 1) * (p + 2) / 2;
}

int n_fpts(int etype, int p) {
    int tri = (p + 1) * (p + 2) / 2;
    if (etype == 2) return 6 * (p + 1) * (p + 1);
    return etype == 0 ? 4 * tri : 2 * tri + 3 * (p + 1) * (p + 1);
}

const std::vector<std::vector<int>> &faces_of(int etype) {
    static const std::vector<std::vector<int>> tet = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    static const std::vector<std::vector<int>> pri = {
        {0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
    static const std::vector<std::vector<int>> hex = {
        {0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
    return etype == 0 ? tet : (etype == 1 ? pri : hex);
}

int n_verts(int etype) { return etype == 0 ? 4 : (etype == 1 ? 6 : 8); }

void ref_vertex(int etype, int v, double out[3]) {
    for (int d = 0; d < 3; ++d) out[d] = double(vert(etype, v)[d]);
}

RefOps build_ref(int etype, int p) {
    RefOps R;
    R.etype = etype;
    R.p = p;
    R.nu = n_upts(etype, p);
    R.nf = n_fpts(etype, p);
    const int nu = R.nu, nf = R.nf;

    // solution points
    std::vector<ld> up;
    if (etype == 0) {
        auto b = tet_bary(p);
        for (int i = 0; i < nu; ++i)
            for (int d = 0; d < 3; ++d) {
                ld s = 0;
                for (int a = 0; a < 4; ++a) s += b[4 * i + a] * TET_V[a][d];
                up.push_back(s);
            }
    } else if (etype == 2) {
        std::vector<ld> x, w;
        gauss_legendre(p + 1, x, w);
        for (int k = 0; k <= p; ++k)
            for (int j = 0; j <= p; ++j)
                for (int i = 0; i <= p; ++i) {
                    up.push_back(x[i]);
                    up.push_back(x[j]);
                    up.push_back(x[k]);
                }
    } else {
        auto b = tri_bary(p);
        std::vector<ld> z, w;
        gauss_legendre(p + 1, z, w);
        int nt = int(b.size() / 3);
        for (int k = 0; k <= p; ++k)
            for (int i = 0; i < nt; ++i) {
                up.push_back(b[3 * i] * -1 + b[3 * i + 1] * 1 + b[3 * i + 2] * -1);
                up.push_back(b[3 * i] * -1 + b[3 * i + 1] * -1 + b[3 * i + 2] * 1);
                up.push_back(z[k]);
            }
    }

    // flux points and reference normals
    const auto &faces = faces_of(etype);
    std::vector<ld> fp;
    ld cen[3] = {0, 0, 0};
    int nvt = n_verts(etype);
    for (int v = 0; v < nvt; ++v)
        for (int d = 0; d < 3; ++d) cen[d] += vert(etype, v)[d] / nvt;
    std::vector<ld> area(faces.size());
    R.face_off.push_back(0);
    for (size_t f = 0; f < faces.size(); ++f) {
        const auto &F = faces[f];
        auto uv = face_param_points(int(F.size()), p);
        int n = int(uv.size() / 2);
        const ld *A = vert(etype, F[0]), *B = vert(etype, F[1]), *Lst = vert(etype, F.back());
        ld e1[3], e2[3], nn[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = B[d] - A[d];
            e2[d] = Lst[d] - A[d];
        }
        cross(e1, e2, nn);
        ld len = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        area[f] = F.size() == 3 ? len / 2 : len;
        ld dotc = 0;
        for (int d = 0; d < 3; ++d) dotc += nn[d] / len * (A[d] - cen[d]);
        ld sgn = dotc < 0 ? -1 : 1;
        for (int i = 0; i < n; ++i) {
            ld x[3];
            face_map(etype, F, &uv[2 * i], x);
            for (int d = 0; d < 3; ++d) fp.push_back(x[d]);
            for (int d = 0; d < 3; ++d) R.nref.push_back(double(sgn * nn[d] / len));
            R.fface.push_back(int(f));
        }
        R.face_off.push_back(R.face_off.back() + n);
    }
    if (int(fp.size() / 3) != nf) throw std::runtime_error("flux point count");

    // Vandermonde and its inverse
    Monos B(etype, p);
    if (B.n() != nu) throw std::runtime_error("basis size");
    std::vector<ld> V(size_t(nu) * nu), Vk(3 * size_t(nu) * nu), val(nu), grad(3 * nu);
    for (int i = 0; i < nu; ++i) {
        B.eval(&up[3 * i], val.data(), grad.data());
        for (int a = 0; a < nu; ++a) {
            V[size_t(i) * nu + a] = val[a];
            for (int k = 0; k < 3; ++k) Vk[(size_t(k) * nu + i) * nu + a] = grad[k * nu + a];
        }
    }
    std::vector<ld> Vinv = V;
    invert(Vinv, nu);

    std::vector<ld> Vf(size_t(nf) * nu);
    for (int j = 0; j < nf; ++j) {
        B.eval(&fp[3 * j], val.data(), nullptr);
        for (int a = 0; a < nu; ++a) Vf[size_t(j) * nu + a] = val[a];
    }
    auto M0 = matmul(Vf, Vinv, nf, nu, nu);
    std::vector<ld> G(3 * size_t(nu) * nu);
    for (int k = 0; k < 3; ++k) {
        std::vector<ld> Vkk(Vk.begin() + size_t(k) * nu * nu, Vk.begin() + size_t(k + 1) * nu * nu);
        auto Gk = matmul(Vkk, Vinv, nu, nu, nu);
        std::copy(Gk.begin(), Gk.end(), G.begin() + size_t(k) * nu * nu);
    }

    // Nodal mass matrix M_ij = int l_i l_j from the Lagrange values
    // l_i(q) = sum_a phi_a(q) Vinv[a][i] at the quadrature points, and the
    // integrals of the monomials.
    std::vector<ld> qp, qw;
    volume_rule(etype, p + 3, qp, qw);
    std::vector<ld> Mass(size_t(nu) * nu, 0), ints(nu, 0), lq(nu);
    for (size_t q = 0; q < qw.size(); ++q) {
        B.eval(&qp[3 * q], val.data(), nullptr);
        for (int a = 0; a < nu; ++a) ints[a] += qw[q] * val[a];
        for (int i = 0; i < nu; ++i) {
            ld s = 0;
            for (int a = 0; a < nu; ++a) s += val[a] * Vinv[size_t(a) * nu + i];
            lq[i] = s;
        }
        for (int i = 0; i < nu; ++i)
            for (int j = 0; j < nu; ++j) Mass[size_t(i) * nu + j] += qw[q] * lq[i] * lq[j];
    }
    ld vol = 0;
    for (auto x : qw) vol += x;
    R.volume = double(vol);

    // Face matrix E_i(f,j) = int_f l_i l^f_j ds
    std::vector<ld> E(size_t(nu) * nf, 0);
    for (size_t f = 0; f < faces.size(); ++f) {
        const auto &F = faces[f];
        int nvf = int(F.size());
        FaceLagrange FL(nvf, p);
        std::vector<ld> fuv, fw;
        face_rule(nvf, p + 2, fuv, fw);
        ld scale = area[f] / (nvf == 3 ? 2 : 4);
        std::vector<ld> lf(FL.n);
        for (size_t q = 0; q < fw.size(); ++q) {
            ld x[3];
            face_map(etype, F, &fuv[2 * q], x);
            B.eval(x, val.data(), nullptr);
            for (int i = 0; i < nu; ++i) {
                ld s = 0;
                for (int a = 0; a < nu; ++a) s += val[a] * Vinv[size_t(a) * nu + i];
                lq[i] = s;
            }
            FL.eval(&fuv[2 * q], lf.data());
            for (int i = 0; i < nu; ++i)
                for (int j = 0; j < FL.n; ++j)
                    E[size_t(i) * nf + R.face_off[f] + j] += scale * fw[q] * lq[i] * lf[j];
        }
    }
    invert(Mass, nu);
    auto L = matmul(Mass, E, nu, nu, nf);

    // weights w_i = sum_a Vinv[a][i] int phi_a
    R.w.assign(nu, 0);
    for (int i = 0; i < nu; ++i) {
        ld s = 0;
        for (int a = 0; a < nu; ++a) s += Vinv[size_t(a) * nu + i] * ints[a];
        R.w[i] = double(s);
    }

    auto todbl = [](const std::vector<ld> &v) { return std::vector<double>(v.begin(), v.end()); };
    // Entries that vanish analytically (the tensor structure of prisms and
    // hexahedra, symmetries of the point sets) come out of the Vandermonde
    // route as rounding residue below 1e-12 of the operator's largest entry,
    // while every genuine entry is above 1e-4 of it: set the residue to zero
    // so that the structural zeros are exact.
    auto chop = [](std::vector<ld> &v, size_t begin, size_t end) {
        ld mx = 0;
        for (size_t i = begin; i < end; ++i) mx = std::max(mx, std::fabs(v[i]));
        for (size_t i = begin; i < end; ++i)
            if (std::fabs(v[i]) <= ld(1e-10) * mx) v[i] = 0;
    };
    chop(M0, 0, M0.size());
    for (int k = 0; k < 3; ++k) chop(G, size_t(k) * nu * nu, size_t(k + 1) * nu * nu);
    chop(L, 0, L.size());
    R.upts = todbl(up);
    R.fpts = todbl(fp);
    R.M0 = todbl(M0);
    R.G = todbl(G);
    R.L = todbl(L);
    return R;
}

namespace {

// Nodal Lagrange values of order p at reference point x (monomial route).
struct Lagrange {
    Monos B;
    std::vector<ld> Vinv;
    int n;
    Lagrange(int etype, int p) : B(etype, p) {
        const RefOps &R = ref_cached(etype, p);
        n = R.nu;
        Vinv.assign(size_t(n) * n, 0);
        std::vector<ld> val(n);
        for (int i = 0; i < n; ++i) {
            ld x[3] = {R.upts[3 * i], R.upts[3 * i + 1], R.upts[3 * i + 2]};
            B.eval(x, val.data(), nullptr);
            for (int a = 0; a < n; ++a) Vinv[size_t(i) * n + a] = val[a];
        }
        invert(Vinv, n);
    }
    void eval(const ld *x, ld *out) const {
        std::vector<ld> val(n);
        B.eval(x, val.data(), nullptr);
        for (int i = 0; i < n; ++i) {
            ld s = 0;
            for (int a = 0; a < n; ++a) s += val[a] * Vinv[size_t(a) * n + i];
            out[i] = s;
        }
    }
};

// phi = Linv (1, xi, eta, zeta) with G = L L^T over the reference element.
void p1_basis(int etype, ld Linv[4][4]) {
    std::vector<ld> qp, qw;
    volume_rule(etype, 3, qp, qw);
    ld G[4][4] = {};
    for (size_t q = 0; q < qw.size(); ++q) {
        ld m[4] = {1, qp[3 * q], qp[3 * q + 1], qp[3 * q + 2]};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) G[a][b] += qw[q] * m[a] * m[b];
    }
    ld L[4][4] = {};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j <= i; ++j) {
            ld s = G[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = (i == j) ? std::sqrt(s) : s / L[j][j];
        }
    for (int c = 0; c < 4; ++c)           // Linv columns by forward substitution
        for (int i = 0; i < 4; ++i) {
            ld s = (i == c) ? 1 : 0;
            for (int k = 0; k < i; ++k) s -= L[i][k] * Linv[k][c];
            Linv[i][c] = s / L[i][i];
        }
}

void p1_eval(const ld Linv[4][4], const ld *x, ld phi[4]) {
    const ld m[4] = {1, x[0], x[1], x[2]};
    for (int a = 0; a < 4; ++a) {
        phi[a] = 0;
        for (int b = 0; b <= a; ++b) phi[a] += Linv[a][b] * m[b];
    }
}

}  // namespace

std::vector<double> build_moments(int etype, int p) {
    Lagrange Lg(etype, p);
    ld Linv[4][4];
    p1_basis(etype, Linv);
    std::vector<ld> qp, qw;
    volume_rule(etype, p + 3, qp, qw);
    std::vector<ld> acc(size_t(4) * Lg.n, 0), l(Lg.n);
    for (size_t q = 0; q < qw.size(); ++q) {
        ld phi[4];
        p1_eval(Linv, &qp[3 * q], phi);
        Lg.eval(&qp[3 * q], l.data());
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < Lg.n; ++i) acc[size_t(a) * Lg.n + i] += qw[q] * phi[a] * l[i];
    }
    return std::vector<double>(acc.begin(), acc.end());
}

std::vector<double> build_lift(int etype, int p) {
    const RefOps &R = ref_cached(etype, p);
    ld Linv[4][4];
    p1_basis(etype, Linv);
    std::vector<double> out(size_t(R.nu) * 4);
    for (int i = 0; i < R.nu; ++i) {
        ld x[3] = {R.upts[3 * i], R.upts[3 * i + 1], R.upts[3 * i + 2]}, phi[4];
        p1_eval(Linv, x, phi);
        for (int a = 0; a < 4; ++a) out[size_t(i) * 4 + a] = double(phi[a]);
    }
    return out;
}

std::vector<double> build_projection(int etype, int p, int q) {
    Lagrange Ls(etype, p), Ld(etype, q);
    std::vector<ld> qp, qw;
    volume_rule(etype, (p + q) / 2 + 3, qp, qw);
    const int ns = Ls.n, nd = Ld.n;
    std::vector<ld> M(size_t(nd) * nd, 0), C(size_t(nd) * ns, 0), ls(ns), lq(nd);
    for (size_t k = 0; k < qw.size(); ++k) {
        Ls.eval(&qp[3 * k], ls.data());
        Ld.eval(&qp[3 * k], lq.data());
        for (int i = 0; i < nd; ++i) {
            for (int j = 0; j < nd; ++j) M[size_t(i) * nd + j] += qw[k] * lq[i] * lq[j];
            for (int j = 0; j < ns; ++j) C[size_t(i) * ns + j] += qw[k] * lq[i] * ls[j];
        }
    }
    invert(M, nd);
    auto P = matmul(M, C, nd, nd, ns);
    return std::vector<double>(P.begin(), P.end());
}

int n_qnodes(int etype) { return etype == 0 ? 10 : (etype == 1 ? 18 : 27); }

namespace {
// Order-2 geometry basis of one type: monomials xi^a eta^b zeta^c of the
// element's order-2 space and the inverse of their Vandermonde matrix at the
// lattice nodes.
struct QuadBasis {
    int nq = 0;
    std::vector<int> e;       // [nq][3] monomial exponents
    std::vector<ld> Vinv;     // [nq][nq]
};

QuadBasis make_quad_basis(int etype) {
    QuadBasis B;
    for (int a = 0; a <= 2; ++a)
        for (int b = 0; b <= (etype == 2 ? 2 : 2 - a); ++b)
            for (int c = 0; c <= (etype == 0 ? 2 - a - b : 2); ++c) {
                B.e.push_back(a);
                B.e.push_back(b);
                B.e.push_back(c);
            }
    B.nq = int(B.e.size() / 3);
    std::vector<ld> nodes;
    for (int c = 0; c <= 2; ++c)
        for (int b = 0; b <= (etype == 0 ? 2 - c : 2); ++b)
            for (int a = 0; a <= (etype == 2 ? 2 : (etype == 0 ? 2 - b - c : 2 - b)); ++a) {
                nodes.push_back(a - 1);
                nodes.push_back(b - 1);
                nodes.push_back(c - 1);
            }
    if (int(nodes.size() / 3) != B.nq) throw std::runtime_error("quadratic lattice size");
    B.Vinv.assign(size_t(B.nq) * B.nq, 0);
    for (int i = 0; i < B.nq; ++i)
        for (int m = 0; m < B.nq; ++m)
            B.Vinv[size_t(i) * B.nq + m] =
                ipow(nodes[3 * i], B.e[3 * m]) * ipow(nodes[3 * i + 1], B.e[3 * m + 1]) * ipow(nodes[3 * i + 2], B.e[3 * m + 2]);
    invert(B.Vinv, B.nq);
    return B;
}

const QuadBasis &quad_basis(int etype) {
    static const QuadBasis b[3] = {make_quad_basis(0), make_quad_basis(1), make_quad_basis(2)};
    return b[etype];
}
}  // namespace

void quad_shape(int etype, const double *xi, double *N, double *dN) {
    const QuadBasis &B = quad_basis(etype);
    const int nq = B.nq;
    ld v[27], d[3][27];
    for (int m = 0; m < nq; ++m) {
        const int a = B.e[3 * m], b = B.e[3 * m + 1], c = B.e[3 * m + 2];
        const ld x = xi[0], y = xi[1], z = xi[2];
        v[m] = ipow(x, a) * ipow(y, b) * ipow(z, c);
        d[0][m] = a ? a * ipow(x, a - 1) * ipow(y, b) * ipow(z, c) : 0;
        d[1][m] = b ? b * ipow(x, a) * ipow(y, b - 1) * ipow(z, c) : 0;
        d[2][m] = c ? c * ipow(x, a) * ipow(y, b) * ipow(z, c - 1) : 0;
    }
    for (int n = 0; n < nq; ++n) {
        ld s = 0, g[3] = {0, 0, 0};
        for (int m = 0; m < nq; ++m) {
            const ld w = B.Vinv[size_t(m) * nq + n];
            s += v[m] * w;
            for (int k = 0; k < 3; ++k) g[k] += d[k][m] * w;
        }
        if (N) N[n] = double(s);
        if (dN)
            for (int k = 0; k < 3; ++k) dN[3 * n + k] = double(g[k]);
    }
}

const RefOps &ref_cached(int etype, int p) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, RefOps> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(etype, p);
    auto it = cache.find(key);
    if (it == cache.end()) it = cache.emplace(key, build_ref(etype, p)).first;
    return it->second;
}

}  // namespace frh
