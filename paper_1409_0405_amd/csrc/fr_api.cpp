// C ABI of the FR library (declared in include/fr.h): mesh setup, the
// right-hand-side pipeline, Runge-Kutta stepping and FP64 reductions.
//
// Right-hand side per element type (paper Section 2.1: operator products with
// constant operators plus point-wise kernels; Section 3.4: DG-type scheme):
//   1  U_f  = M0 U                                   operator product
//   2  D    = C - U_f, the jump to the common LDG solution C at each
//             paired flux point                                 (NS)
//   3  Q~   = [G_k | L_k] [U; D], L_k = L diag(n_ref,k)  operator product (NS)
//   4  Q    = adj^T Q~ / J;  F~ = adj (F_inv - F_vis)  point-wise
//   5  Q_f  = M0 Q                                   operator product (NS)
//   6  Fn*  = common transformed normal flux at paired flux points
//   7  R~   = [G'_0 G'_1 G'_2 | L] [F~; Fn*],
//             G'_k = G_k - L_k M0                    operator product
//   8  R    = -R~ / J, fused with the Runge-Kutta register update
// Step 7 folds the correction L (Fn* - n_ref . M0 F~) into the divergence
// operator, so F~ is read once.  Step 3 takes the jump D, which the interface
// kernel forms directly (no cancellation between L C and L M0 U); a side whose
// LDG weight is zero (beta = +-1/2) has D = 0 and is never written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fr.h"
#include "fr_device.hpp"
#include "fr_host.hpp"

namespace {

thread_local std::string g_create_error;

struct DevBase {
    virtual ~DevBase() = default;
};

template <typename T>
struct DevType {
    int nu = 0, nf = 0;
    int64_t nelem = 0, ld = 0;
    frd::Op<T> Aint, Agint, Agrad, Adiv;          // Agint: M0 for the gradients
    frd::Op<T> Fgrad, Fgint;                      // fused gradient stage (step lists, one row block per group)
    // fused gradient stage: bit f of qmask[e] is set when an interface or
    // boundary kernel reads the gradient on face f of element e (the other
    // flux points are not written); fbit[s] = 1 << face of the flux point in
    // row slot s of Fgint (0 for padding slots)
    uint8_t *qmask = nullptr, *fbit = nullptr;
    // gradient stage form: 0 three kernels, 1 fused per tile, 2 fused and
    // streaming (FP32); set from the operator's size at setup, the autotuner
    // keeps the fastest
    int grad_form = 1;
    frd::OpSplit Sint, Sgint, Sgrad, Sdiv;        // split-precision forms only
    T *geom = nullptr, *xi = nullptr;
    T *jinv = nullptr;        // [nu][ld] 1 / J at the solution points (host FP64, rounded)
    T *padj = nullptr;        // [9][nu][ld] adjugate at the solution points (curved types only)
    T *Uf = nullptr, *Cf = nullptr, *Qt = nullptr, *Q = nullptr, *Qf = nullptr;
    T *Ft = nullptr, *Fn = nullptr, *Rt = nullptr, *R = nullptr;
    T *reg[3] = {nullptr, nullptr, nullptr};
    T *ereg = nullptr;        // embedded error of the adaptive RK45 (allocated on first use)
    T *dte = nullptr;         // per-element step size (batched problems)
    double *wJ = nullptr;
};

template <typename T>
struct Dev : DevBase {
    DevType<T> t[frh::NTYPE];
    uint32_t *sideL = nullptr, *sideR = nullptr;
    T *pgeo = nullptr;
    int64_t npairs = 0;
    uint32_t *bside = nullptr;      // boundary points
    T *bgeo = nullptr;              // [4][nb]
    int8_t *bkind = nullptr;
    int64_t nb = 0;
    double *partial = nullptr, *red_out = nullptr;
    std::vector<void *> allocs;
    ~Dev() override {
        for (void *p : allocs) (void)hipFree(p);
    }
};

}  // namespace

// Per-kernel HIP event timing (fr_profile / fr_profile_read).
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> recs;   // (kernel class, start event index)
    ~Profiler() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Learned closure attached to a mesh (fr_closure_attach).
struct Closure {
    const float *params = nullptr;
    const uint16_t *params_bf16 = nullptr;
    const float *stats = nullptr;
    bool bf16 = true;
    int32_t *nb = nullptr;                    // [ntot][5]
    float *mom = nullptr, *feat = nullptr, *y = nullptr;
    float *Mom[2] = {nullptr, nullptr};       // [4][nu] per type
    float *lift[2] = {nullptr, nullptr};      // [nu][4] per type
    std::vector<void *> allocs;
    ~Closure() {
        for (void *p : allocs) (void)hipFree(p);
    }
};

struct fr_mesh_s {
    int order = 0, system = 0, precision = 0;
    uint32_t flags = 0;
    double gamma = 1.4, mu = 0, prandtl = 0.72, beta = 0.5, tau = 0.1;
    double t_wall = 1.0, farfield[5] = {1.0, 0.0, 0.0, 0.0, 1.0 / 1.4};
    double pref = 0;          // reference pressure left out of the momentum flux
    frh::MeshHost host;
    hipStream_t create_stream = nullptr;
    bool device = false;
    std::unique_ptr<DevBase> dev;
    Profiler prof;
    std::unique_ptr<Closure> closure;
    // projection operators to other orders, key 16 * type + target order
    // (fragments live in the device allocations of this mesh)
    std::map<int, frd::Op<float>> proj_f;
    std::map<int, frd::Op<double>> proj_d;
    std::string err;
};

namespace {

fr_status fail(fr_mesh m, fr_status st, const std::string &msg) {
    if (m)
        m->err = msg;
    else
        g_create_error = msg;
    return st;
}

#define FR_HIP(m, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(m, e_ == hipErrorOutOfMemory ? FR_ERR_OUT_OF_MEMORY : FR_ERR_DEVICE, \
                        std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

// Kernel classes of the profiler: 0..7 operator products (4 * type + op) of
// tets and prisms, 8/9 solution-point kernel (tet/prism), 10 common solution,
// 11 common flux, 12/13 negdivconf (tet/prism), 14/15 closure, 16..19
// hexahedron products (16 + op), 20 hexahedron solution-point kernel, 21
// hexahedron negdivconf, 22 / 23 boundary states / boundary flux, 24 / 25
// fused gradient stage (tet / prism).
constexpr int PROF_NCLASS = FR_PROF_NCLASS;
constexpr int prof_op(int t, int op) { return t < 2 ? 4 * t + op : 16 + op; }
constexpr int prof_upts(int t) { return t < 2 ? 8 + t : 20; }
constexpr int prof_neg(int t) { return t < 2 ? 12 + t : 21; }
constexpr int prof_gradflux(int t) { return 24 + t; }
constexpr size_t PROF_NONE = size_t(-1);

size_t prof_begin(fr_mesh m, hipStream_t s) {
    Profiler &P = m->prof;
    if (!P.on) return PROF_NONE;
    while (P.pool.size() < P.used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return PROF_NONE;
        P.pool.push_back(e);
    }
    size_t i = P.used;
    P.used += 2;
    (void)hipEventRecord(P.pool[i], s);
    return i;
}

void prof_end(fr_mesh m, size_t i, int cls, hipStream_t s) {
    if (i == PROF_NONE) return;
    (void)hipEventRecord(m->prof.pool[i + 1], s);
    m->prof.recs.push_back({cls, i});
}

// Launch wrapped in profiler events.
#define FR_LAUNCH(m, cls, s, call)            \
    do {                                       \
        size_t pi_ = prof_begin(m, s);         \
        FR_HIP(m, call);                       \
        prof_end(m, pi_, cls, s);              \
    } while (0)

// Fragment order for the MFMA product kernel (see frd::Op).  Stage 5 also
// fills idx = [koff (nmg + 1) | klist] and compacts f per row group.
// Row order for the step-list product: groups of `gsize` rows filled
// greedily, each next row the one adding the fewest K steps (of 4 columns)
// to the group's union (ties: lowest row), so that rows touching the same
// columns (one layer of a prism, one line of a hexahedron) share a group.
std::vector<int> cluster_rows(const std::vector<double> &A, int M, int K, int gsize) {
    const int Kb = (K + 3) / 4;
    std::vector<std::vector<char>> mask(M, std::vector<char>(Kb, 0));
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < K; ++c)
            if (A[size_t(r) * K + c] != 0.0) mask[r][c / 4] = 1;
    std::vector<char> used(M, 0);
    std::vector<int> order;
    while (int(order.size()) < M) {
        std::vector<char> uni(Kb, 0);
        for (int n = 0; n < gsize && int(order.size()) < M; ++n) {
            int best = -1, best_add = 1 << 30;
            for (int r = 0; r < M; ++r) {
                if (used[r]) continue;
                int add = 0;
                for (int kb = 0; kb < Kb; ++kb) add += mask[r][kb] && !uni[kb];
                if (add < best_add) {
                    best_add = add;
                    best = r;
                }
            }
            used[best] = 1;
            order.push_back(best);
            for (int kb = 0; kb < Kb; ++kb) uni[kb] |= mask[best][kb];
        }
    }
    return order;
}

template <typename T>
frd::Op<T> fragment(const std::vector<double> &A_in, int M, int K, std::vector<T> &f, int cap = 0,
                    int stage = 0, std::vector<int32_t> *idx = nullptr, bool cluster = true) {
    frd::Op<T> op;
    op.M = M;
    op.stage = stage;
    // stages 5 and 6 (step lists): rows permuted into clustered groups
    // (perm[r'] = source row), unless the caller has ordered them
    const bool steps = stage == 5 || stage == 6;
    std::vector<int> perm;
    std::vector<double> Aperm;
    const std::vector<double> &A = steps ? Aperm : A_in;
    // an even number of K steps; a multiple of the chunk (4 or 8 steps) when
    // the B panel is staged through LDS
    const int kmul = (stage == 2 || stage == 4) ? 8 : (stage == 1 || stage == 3) ? 4 : 2;
    op.Kb = ((K + 3) / 4 + kmul - 1) / kmul * kmul;
    frd::row_groups(M, cap ? cap : (sizeof(T) == 4 ? 8 : 4), op.nmg, op.mbw);
    const int Mb = op.nmg * op.mbw;
    if (steps) {
        if (cluster) {
            perm = cluster_rows(A_in, M, K, 16 * op.mbw);
        } else {
            perm.resize(M);
            for (int r = 0; r < M; ++r) perm[r] = r;
        }
        Aperm.resize(size_t(M) * K);
        for (int r = 0; r < M; ++r)
            std::copy(A_in.begin() + size_t(perm[r]) * K, A_in.begin() + size_t(perm[r] + 1) * K,
                      Aperm.begin() + size_t(r) * K);
    }
    f.assign(size_t(Mb) * op.Kb * 64, T(0));
    // stage 4 groups four K steps per lane: [mb][Kb / 4][lane][4]
    for (int mb = 0; mb < Mb; ++mb)
        for (int kb = 0; kb < op.Kb; ++kb)
            for (int l = 0; l < 64; ++l) {
                int r = 16 * mb + (l % 16), c = 4 * kb + l / 16;
                const size_t at = stage == 4 ? ((size_t(mb) * (op.Kb / 4) + kb / 4) * 64 + l) * 4 + kb % 4
                                             : (size_t(mb) * op.Kb + kb) * 64 + l;
                if (r < M && c < K) f[at] = T(A[size_t(r) * K + c]);
            }
    if (steps) {
        // each list padded with zero fragments to a multiple of the steps the
        // kernel keeps in flight (2 for stage 5, 4 for stage 6)
        const size_t mult = stage == 6 ? 4 : 2;
        std::vector<T> dense;
        dense.swap(f);
        std::vector<int32_t> koff(op.nmg + 1), klist;
        for (int g = 0; g < op.nmg; ++g) {
            koff[g] = int32_t(klist.size());
            std::vector<int> ks;
            for (int kb = 0; kb < op.Kb; ++kb) {
                bool nz = false;
                for (int m = 0; m < op.mbw && !nz; ++m)
                    for (int l = 0; l < 64 && !nz; ++l)
                        nz = dense[(size_t(g * op.mbw + m) * op.Kb + kb) * 64 + l] != T(0);
                if (nz) ks.push_back(kb);
            }
            const size_t nreal = ks.size();
            if (ks.empty()) ks.push_back(0);
            while (ks.size() % mult) ks.push_back(ks.back());
            for (size_t j = 0; j < ks.size(); ++j) {
                klist.push_back(ks[j]);
                for (int m = 0; m < op.mbw; ++m)
                    for (int l = 0; l < 64; ++l)
                        f.push_back(j < nreal ? dense[(size_t(g * op.mbw + m) * op.Kb + ks[j]) * 64 + l] : T(0));
            }
        }
        koff[op.nmg] = int32_t(klist.size());
        if (idx) {
            idx->assign(koff.begin(), koff.end());
            idx->insert(idx->end(), klist.begin(), klist.end());
            for (int r = 0; r < Mb * 16; ++r) idx->push_back(r < M ? perm[r] : -1);
        }
    }
    return op;
}

// Device copy of a fragment array (and, stages 5 and 6, its step lists); the
// allocations are appended to `allocs`.
template <typename T>
hipError_t upload_op(frd::Op<T> &op, const std::vector<T> &f, const std::vector<int32_t> &idx,
                     std::vector<void *> &allocs) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(f.size(), 1) * sizeof(T));
    if (e != hipSuccess) return e;
    allocs.push_back(p);
    if ((e = hipMemcpy(p, f.data(), f.size() * sizeof(T), hipMemcpyHostToDevice)) != hipSuccess) return e;
    op.frag = static_cast<T *>(p);
    if (op.stage == 5 || op.stage == 6) {
        if ((e = hipMalloc(&p, idx.size() * sizeof(int32_t))) != hipSuccess) return e;
        allocs.push_back(p);
        if ((e = hipMemcpy(p, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        op.koff = static_cast<int32_t *>(p);
        op.klist = op.koff + op.nmg + 1;
        op.rowmap = op.klist + idx[op.nmg];
    }
    return hipSuccess;
}

// 16-bit parts of an operator for the split-precision product kernel (see
// frd::OpSplit), each rounded to nearest even: BF16 (format 1) h, m, l with
// A = h + m + l to ~24 bits; FP16 (format 2) h = round(A),
// l = round((A - h) 2^11).
uint16_t to_bf16(double x) {
    float f = float(x);
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7fffu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}
double from_bf16(uint16_t h) {
    uint32_t b = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}
uint16_t to_f16(double x) {
    _Float16 h = _Float16(float(x));
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}
double from_f16(uint16_t u) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return double(float(h));
}

frd::OpSplit fragment_split(const std::vector<double> &A, int M, int K, int format,
                            std::vector<uint16_t> parts[3], int cap = 0) {
    frd::OpSplit op;
    op.M = M;
    op.format = format;
    op.Kb = ((K + 31) / 32 + 1) / 2 * 2;
    frd::row_groups(M, cap ? cap : (format == 2 ? 2 : 4), op.nmg, op.mbw);
    const int np = format == 2 ? 2 : 3;
    const double scale = format == 2 ? 2048.0 : 1.0;
    op.inv_scale = float(1.0 / scale);
    const int Mb = op.nmg * op.mbw;
    for (int q = 0; q < 3; ++q) parts[q].assign(q < np ? size_t(Mb) * op.Kb * 64 * 8 : 0, 0);
    for (int mb = 0; mb < Mb; ++mb)
        for (int kb = 0; kb < op.Kb; ++kb)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j) {
                    const int r = 16 * mb + l % 16, c = 32 * kb + 8 * (l / 16) + j;
                    if (r >= M || c >= K) continue;
                    double rem = A[size_t(r) * K + c];
                    const size_t o = ((size_t(mb) * op.Kb + kb) * 64 + l) * 8 + j;
                    if (format == 2) {
                        parts[0][o] = to_f16(rem);
                        parts[1][o] = to_f16((rem - from_f16(parts[0][o])) * scale);
                    } else {
                        for (int q = 0; q < 3; ++q) {
                            parts[q][o] = to_bf16(rem);
                            rem -= from_bf16(parts[q][o]);
                        }
                    }
                }
    return op;
}

// Operators of one reference element for the products of steps 3 and 7:
//   grad: rows (k, i): [G_k | L_k]                        (3 nu) x (nu + nf)
//   div:  row i: [G_0 - L_0 M0, G_1 - L_1 M0, G_2 - L_2 M0 | L]  nu x (3 nu + nf)
void folded_ops(const frh::RefOps &R, std::vector<double> &grad, std::vector<double> &div) {
    const int nu = R.nu, nf = R.nf;
    std::vector<double> Gp(3 * size_t(nu) * nu);
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < nu; ++i)
            for (int j = 0; j < nu; ++j) {
                double s = R.G[(size_t(k) * nu + i) * nu + j];
                for (int f = 0; f < nf; ++f)
                    s -= R.L[size_t(i) * nf + f] * R.nref[3 * f + k] * R.M0[size_t(f) * nu + j];
                Gp[(size_t(k) * nu + i) * nu + j] = s;
            }
    const int Kg = nu + nf;
    grad.assign(3 * size_t(nu) * Kg, 0);
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < nu; ++i) {
            double *row = &grad[(size_t(k) * nu + i) * Kg];
            for (int j = 0; j < nu; ++j) row[j] = R.G[(size_t(k) * nu + i) * nu + j];
            for (int f = 0; f < nf; ++f) row[nu + f] = R.L[size_t(i) * nf + f] * R.nref[3 * f + k];
        }
    const int Kd = 3 * nu + nf;
    div.assign(size_t(nu) * Kd, 0);
    for (int i = 0; i < nu; ++i) {
        double *row = &div[size_t(i) * Kd];
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < nu; ++j) row[k * nu + j] = Gp[(size_t(k) * nu + i) * nu + j];
        for (int f = 0; f < nf; ++f) row[3 * nu + f] = R.L[size_t(i) * nf + f];
    }
}

template <typename T>
fr_status dev_alloc(fr_mesh m, Dev<T> &d, T *&p, size_t n) {
    void *q = nullptr;
    FR_HIP(m, hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
    d.allocs.push_back(q);
    p = static_cast<T *>(q);
    return FR_OK;
}

template <typename T>
fr_status dev_upload(fr_mesh m, Dev<T> &d, T *&p, const std::vector<T> &h, hipStream_t s) {
    fr_status st = dev_alloc(m, d, p, h.size());
    if (st) return st;
    (void)s;
    if (!h.empty()) FR_HIP(m, hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return FR_OK;
}

template <typename T>
std::vector<T> cast(const std::vector<double> &v) {
    return std::vector<T>(v.begin(), v.end());
}

template <typename T>
fr_status setup_device(fr_mesh m, hipStream_t s) {
    auto dp = std::make_unique<Dev<T>>();
    Dev<T> &d = *dp;
    const bool ns = m->system == FR_NAVIER_STOKES;
    fr_status st;
#define FR_TRY(x)                 \
    do {                          \
        if ((st = (x))) return st; \
    } while (0)
    std::vector<int32_t> gint_rows[frh::NTYPE];   // row slot -> flux point of Fgint (-1: padding)
    for (int t = 0; t < frh::NTYPE; ++t) {
        const frh::TypeHost &H = m->host.t[t];
        DevType<T> &D = d.t[t];
        D.nelem = H.nelem;
        D.ld = H.ld;
        if (!H.nelem) continue;
        const frh::RefOps &R = H.ops;
        D.nu = R.nu;
        D.nf = R.nf;
        const int nu = R.nu, nf = R.nf;
        const size_t ld = size_t(H.ld);
        std::vector<double> grad, div;
        folded_ops(R, grad, div);
        T *p;
        std::vector<T> f;
        D.Aint = fragment<T>(R.M0, nf, nu, f);
        FR_TRY(dev_upload(m, d, p, f, s));
        D.Aint.frag = p;
        D.Agrad = fragment<T>(grad, 3 * nu, nu + nf, f);
        FR_TRY(dev_upload(m, d, p, f, s));
        D.Agrad.frag = p;
        D.Adiv = fragment<T>(div, nu, 3 * nu + nf, f);
        FR_TRY(dev_upload(m, d, p, f, s));
        D.Adiv.frag = p;
        D.Agint = D.Aint;
        if (ns && (m->precision == FR_FP32 || m->precision == FR_FP64)) {
            // the fused gradient stage walks the step lists of one row block
            std::vector<int32_t> idx;
            D.Fgrad = fragment<T>(grad, 3 * nu, nu + nf, f, 1, 6, &idx);
            FR_HIP(m, upload_op(D.Fgrad, f, idx, d.allocs));
            D.Fgint = fragment<T>(R.M0, nf, nu, f, 1, 6, &idx);
            FR_HIP(m, upload_op(D.Fgint, f, idx, d.allocs));
            gint_rows[t].assign(idx.end() - 16 * D.Fgint.nmg, idx.end());
            // before autotuning: the fused stage where its gradient product
            // has work for at least half of the workgroup's wavefronts
            // (measured on the mixed Taylor-Green mesh: it loses for tets at
            // p <= 2 and prisms at p = 1, wins above)
            D.grad_form = D.Fgrad.nmg >= 4 ? 1 : 0;
        }
        if (m->precision == FR_SPLIT_BF16 || m->precision == FR_SPLIT_FP16) {
            const int fmt = m->precision == FR_SPLIT_FP16 ? 2 : 1;
            std::vector<uint16_t> parts[3];
            auto up = [&](frd::OpSplit op, frd::OpSplit &dst) -> fr_status {
                for (int q = 0; q < 3; ++q) {
                    if (parts[q].empty()) continue;
                    void *ptr;
                    FR_HIP(m, hipMalloc(&ptr, parts[q].size() * 2));
                    d.allocs.push_back(ptr);
                    FR_HIP(m, hipMemcpy(ptr, parts[q].data(), parts[q].size() * 2, hipMemcpyHostToDevice));
                    op.part[q] = static_cast<uint16_t *>(ptr);
                }
                dst = op;
                return FR_OK;
            };
            FR_TRY(up(fragment_split(R.M0, nf, nu, fmt, parts), D.Sint));
            FR_TRY(up(fragment_split(grad, 3 * nu, nu + nf, fmt, parts), D.Sgrad));
            FR_TRY(up(fragment_split(div, nu, 3 * nu + nf, fmt, parts), D.Sdiv));
            D.Sgint = D.Sint;
        }

        const int ng = frh::n_geom(t);
        std::vector<double> g(size_t(ng) * ld, 0.0);
        for (int k = 0; k < ng; ++k)
            for (int64_t e = 0; e < H.nelem; ++e) g[k * ld + e] = H.geom[size_t(k) * H.nelem + e];
        // padding columns: copy element 0 so that padded lanes see a valid metric
        for (int k = 0; k < ng; ++k)
            for (size_t e = size_t(H.nelem); e < ld; ++e) g[k * ld + e] = H.geom[size_t(k) * H.nelem];
        FR_TRY(dev_upload(m, d, D.geom, cast<T>(g), s));
        FR_TRY(dev_upload(m, d, D.xi, cast<T>(R.upts), s));
        std::vector<double> wJ(size_t(nu) * ld, 0.0), jinv(size_t(nu) * ld, 1.0);
        for (int i = 0; i < nu; ++i)
            for (int64_t e = 0; e < H.nelem; ++e) {
                wJ[i * ld + e] = R.w[i] * H.jdet[size_t(e) * nu + i];
                jinv[i * ld + e] = 1.0 / H.jdet[size_t(e) * nu + i];
            }
        FR_TRY(dev_upload(m, d, D.jinv, cast<T>(jinv), s));
        if (!H.Xq.empty()) {
            // curved: adj[k][j] = (col[k1] x col[k2])_j per solution point
            std::vector<double> pa(9 * size_t(nu) * ld, 0.0);
            for (int i = 0; i < nu; ++i)
                for (size_t e = 0; e < ld; ++e) {
                    double col[3][3];
                    frh::elem_jac_at(H, t, int64_t(e < size_t(H.nelem) ? e : 0), false, i, col);
                    for (int k = 0; k < 3; ++k) {
                        const double *a1 = col[(k + 1) % 3], *a2 = col[(k + 2) % 3];
                        const double c3[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                                              a1[0] * a2[1] - a1[1] * a2[0]};
                        for (int j = 0; j < 3; ++j) pa[(size_t(3 * k + j) * nu + i) * ld + e] = c3[j];
                    }
                }
            FR_TRY(dev_upload(m, d, D.padj, cast<T>(pa), s));
        }
        {
            void *q;
            FR_HIP(m, hipMalloc(&q, wJ.size() * sizeof(double)));
            d.allocs.push_back(q);
            D.wJ = static_cast<double *>(q);
            FR_HIP(m, hipMemcpy(D.wJ, wJ.data(), wJ.size() * sizeof(double), hipMemcpyHostToDevice));
        }
        const size_t su = size_t(nu) * 5 * ld, sf = size_t(nf) * 5 * ld;
        FR_TRY(dev_alloc(m, d, D.Uf, sf));
        FR_TRY(dev_alloc(m, d, D.Fn, sf));
        FR_TRY(dev_alloc(m, d, D.Ft, 3 * su));
        FR_TRY(dev_alloc(m, d, D.Rt, su));
        FR_TRY(dev_alloc(m, d, D.R, su));
        if (ns) {
            FR_TRY(dev_alloc(m, d, D.Cf, sf));
            FR_TRY(dev_alloc(m, d, D.Qt, 3 * su));
            FR_TRY(dev_alloc(m, d, D.Q, 3 * su));
            FR_TRY(dev_alloc(m, d, D.Qf, 3 * sf));
        }
        for (int r = 0; r < 3; ++r) {
            FR_TRY(dev_alloc(m, d, D.reg[r], su));
            FR_HIP(m, hipMemsetAsync(D.reg[r], 0, su * sizeof(T), s));
        }
        FR_HIP(m, hipMemsetAsync(D.Uf, 0, sf * sizeof(T), s));
        FR_HIP(m, hipMemsetAsync(D.Ft, 0, 3 * su * sizeof(T), s));
        FR_HIP(m, hipMemsetAsync(D.Fn, 0, sf * sizeof(T), s));
        if (ns) {
            FR_HIP(m, hipMemsetAsync(D.Cf, 0, sf * sizeof(T), s));
            FR_HIP(m, hipMemsetAsync(D.Qf, 0, 3 * sf * sizeof(T), s));
            FR_HIP(m, hipMemsetAsync(D.Qt, 0, 3 * su * sizeof(T), s));
            FR_HIP(m, hipMemsetAsync(D.Q, 0, 3 * su * sizeof(T), s));
        }
    }
    const frh::PairTable &P = m->host.pairs;
    d.npairs = int64_t(P.sideL.size());
    {
        void *q;
        FR_HIP(m, hipMalloc(&q, std::max<size_t>(P.sideL.size(), 1) * 4));
        d.allocs.push_back(q);
        d.sideL = static_cast<uint32_t *>(q);
        FR_HIP(m, hipMalloc(&q, std::max<size_t>(P.sideR.size(), 1) * 4));
        d.allocs.push_back(q);
        d.sideR = static_cast<uint32_t *>(q);
        if (d.npairs) {
            FR_HIP(m, hipMemcpy(d.sideL, P.sideL.data(), P.sideL.size() * 4, hipMemcpyHostToDevice));
            FR_HIP(m, hipMemcpy(d.sideR, P.sideR.data(), P.sideR.size() * 4, hipMemcpyHostToDevice));
        }
    }
    std::vector<T> pg(5 * size_t(d.npairs));
    for (int64_t i = 0; i < d.npairs; ++i) {
        for (int k = 0; k < 3; ++k) pg[size_t(k) * d.npairs + i] = T(P.nhat[3 * i + k]);
        pg[3 * size_t(d.npairs) + i] = T(P.sL[i]);
        pg[4 * size_t(d.npairs) + i] = T(P.sR[i]);
    }
    FR_TRY(dev_upload(m, d, d.pgeo, pg, s));
    {
        const frh::BndTable &B = m->host.bnd;
        d.nb = int64_t(B.side.size());
        void *q;
        FR_HIP(m, hipMalloc(&q, std::max<size_t>(B.side.size(), 1) * 4));
        d.allocs.push_back(q);
        d.bside = static_cast<uint32_t *>(q);
        FR_HIP(m, hipMalloc(&q, std::max<size_t>(B.kind.size(), 1)));
        d.allocs.push_back(q);
        d.bkind = static_cast<int8_t *>(q);
        if (d.nb) {
            FR_HIP(m, hipMemcpy(d.bside, B.side.data(), B.side.size() * 4, hipMemcpyHostToDevice));
            FR_HIP(m, hipMemcpy(d.bkind, B.kind.data(), B.kind.size(), hipMemcpyHostToDevice));
        }
        std::vector<T> bg(4 * size_t(d.nb));
        for (int64_t i = 0; i < d.nb; ++i) {
            for (int k = 0; k < 3; ++k) bg[size_t(k) * d.nb + i] = T(B.nhat[3 * i + k]);
            bg[3 * size_t(d.nb) + i] = T(B.s[i]);
        }
        FR_TRY(dev_upload(m, d, d.bgeo, bg, s));
    }
    if (ns) {
        // faces whose flux-point gradient the common flux reads: a side with
        // a nonzero LDG weight (computed as the interface kernel does, in T),
        // and every boundary face
        const bool readL = T(0.5) + T(m->beta) != T(0), readR = T(0.5) - T(m->beta) != T(0);
        std::vector<uint8_t> qm[frh::NTYPE];
        for (int t = 0; t < frh::NTYPE; ++t)
            if (d.t[t].Fgrad.frag) qm[t].assign(size_t(d.t[t].ld), 0);
        auto mark = [&](uint32_t side) {
            const int t = frh::side_type(side);
            if (qm[t].empty()) return;
            const int face = m->host.t[t].ops.fface[frh::side_fpt(side)];
            qm[t][size_t(frh::side_elem(side))] |= uint8_t(1u << face);
        };
        for (size_t i = 0; i < P.sideL.size(); ++i) {
            if (readL) mark(P.sideL[i]);
            if (readR) mark(P.sideR[i]);
        }
        for (uint32_t side : m->host.bnd.side) mark(side);
        for (int t = 0; t < frh::NTYPE; ++t) {
            if (qm[t].empty()) continue;
            DevType<T> &D = d.t[t];
            const std::vector<int> &ff = m->host.t[t].ops.fface;
            std::vector<uint8_t> fb(gint_rows[t].size(), 0);
            for (size_t j = 0; j < fb.size(); ++j)
                if (gint_rows[t][j] >= 0) fb[j] = uint8_t(1u << ff[size_t(gint_rows[t][j])]);
            void *q;
            FR_HIP(m, hipMalloc(&q, qm[t].size()));
            d.allocs.push_back(q);
            D.qmask = static_cast<uint8_t *>(q);
            FR_HIP(m, hipMemcpy(D.qmask, qm[t].data(), qm[t].size(), hipMemcpyHostToDevice));
            FR_HIP(m, hipMalloc(&q, fb.size()));
            d.allocs.push_back(q);
            D.fbit = static_cast<uint8_t *>(q);
            FR_HIP(m, hipMemcpy(D.fbit, fb.data(), fb.size(), hipMemcpyHostToDevice));
        }
    }
    {
        void *q;
        FR_HIP(m, hipMalloc(&q, size_t(frh::NTYPE) * frd::RED_BLOCKS * 8 * sizeof(double)));
        d.allocs.push_back(q);
        d.partial = static_cast<double *>(q);
        FR_HIP(m, hipMalloc(&q, size_t(frh::NTYPE) * 8 * sizeof(double)));
        d.allocs.push_back(q);
        d.red_out = static_cast<double *>(q);
    }
    FR_HIP(m, hipStreamSynchronize(s));
#undef FR_TRY
    m->dev = std::move(dp);
    return FR_OK;
}

template <typename T>
Dev<T> &dev_of(fr_mesh m) {
    return *static_cast<Dev<T> *>(m->dev.get());
}

// Output handling of the last pipeline step (see frd::NegArgs).
template <typename T>
struct StageOut {
    T *out = nullptr, *acc = nullptr;
    const T *base = nullptr;
    T a = 0, b = 1;
    bool per_elem_dt = false;   // scale the stage by the per-element step size
    T *err = nullptr;           // error register: err = (err_set ? 0 : err) + c k
    T c = 0;
    bool err_set = false;
};

// Operator product through the kernel of the mesh's precision.
// With ep the product's output goes through the last pipeline step instead
// of into C.
template <typename T>
hipError_t opmul(fr_mesh m, int tag, const frd::Op<T> &A, const frd::OpSplit &S, const T *B1,
                 int64_t ldb1, int K1, const T *B2, int64_t ldb2, int K2, T *C, int64_t ldc,
                 int64_t ncols, hipStream_t s, const frd::NegArgs<T> *ep = nullptr) {
    if constexpr (std::is_same<T, float>::value) {
        if (m->precision == FR_SPLIT_BF16 || m->precision == FR_SPLIT_FP16)
            return frd::launch_opmul_split(tag, S, B1, ldb1, K1, B2, ldb2, K2, C, ldc, ncols, s, ep);
    }
    return frd::launch_opmul<T>(tag, A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, ncols, s, ep);
}

// Arguments of the fused gradient stage of one element type on state U.
template <typename T>
frd::GradFluxArgs<T> gradflux_args(fr_mesh m, const DevType<T> &D, const T *U) {
    frd::GradFluxArgs<T> ga;
    ga.U = U;
    ga.Cf = D.Cf;
    ga.Ft = D.Ft;
    ga.Qf = D.Qf;
    ga.geom = D.geom;
    ga.xi = D.xi;
    ga.padj = D.padj;
    ga.pjinv = D.padj ? D.jinv : nullptr;
    ga.ld = D.ld;
    ga.nelem = D.nelem;
    ga.nu = D.nu;
    ga.nf = D.nf;
    ga.gamma = T(m->gamma);
    ga.mu = T(m->mu);
    ga.prandtl = T(m->prandtl);
    ga.pref = T(m->pref);
    ga.G = D.Fgrad;
    ga.M = D.Fgint;
    ga.qmask = D.qmask;
    ga.fbit = D.fbit;
    return ga;
}

// Solution-point kernel arguments of one element type on state U.
template <typename T>
frd::UptsArgs<T> upts_args(fr_mesh m, const DevType<T> &D, const T *U) {
    frd::UptsArgs<T> ua{U, D.Qt, D.Q, D.Ft, D.geom, D.xi, D.ld, D.nelem, D.nu,
                        T(m->gamma), T(m->mu), T(m->prandtl)};
    ua.padj = D.padj;
    ua.pjinv = D.jinv;
    ua.pref = T(m->pref);
    return ua;
}

template <typename T>
fr_status rhs_pipeline(fr_mesh m, const T *const U[frh::NTYPE], const StageOut<T> so[frh::NTYPE],
                       hipStream_t s) {
    Dev<T> &d = dev_of<T>(m);
    const bool ns = m->system == FR_NAVIER_STOKES;
    const T gamma = T(m->gamma), mu = T(m->mu), pr = T(m->prandtl);
    for (int t = 0; t < frh::NTYPE; ++t) {
        DevType<T> &D = d.t[t];
        if (!D.nelem) continue;
        const int64_t w5 = 5 * D.ld;
        FR_LAUNCH(m, prof_op(t, frd::OP_INTERP), s,
                  opmul<T>(m, 4 * t + frd::OP_INTERP, D.Aint, D.Sint, U[t], w5, D.nu, nullptr, 0, 0, D.Uf, w5, w5, s));
    }
    frd::PairArgs<T> pa{};
    pa.sideL = d.sideL;
    pa.sideR = d.sideR;
    pa.geo = d.pgeo;
    pa.npairs = d.npairs;
    for (int t = 0; t < frh::NTYPE; ++t) {
        pa.Uf[t] = d.t[t].Uf;
        pa.Qf[t] = d.t[t].Qf;
        pa.Cf[t] = d.t[t].Cf;
        pa.Fn[t] = d.t[t].Fn;
        pa.ld[t] = d.t[t].ld;
    }
    pa.gamma = gamma;
    pa.mu = mu;
    pa.prandtl = pr;
    pa.beta = T(m->beta);
    pa.tau = T(m->tau);
    pa.pref = T(m->pref);
    frd::BndArgs<T> ba{};
    ba.side = d.bside;
    ba.geo = d.bgeo;
    ba.kind = d.bkind;
    ba.nb = d.nb;
    for (int t = 0; t < frh::NTYPE; ++t) {
        ba.Uf[t] = d.t[t].Uf;
        ba.Qf[t] = d.t[t].Qf;
        ba.Cf[t] = d.t[t].Cf;
        ba.Fn[t] = d.t[t].Fn;
        ba.ld[t] = d.t[t].ld;
    }
    ba.gamma = gamma;
    ba.mu = mu;
    ba.prandtl = pr;
    ba.tau = T(m->tau);
    ba.t_wall = T(m->t_wall);
    for (int k = 0; k < 5; ++k) ba.free[k] = T(m->farfield[k]);
    ba.pref = T(m->pref);
    // Navier-Stokes tets and prisms: corrected gradient, point-wise work and
    // gradient interpolation in one kernel (FR_SEPARATE_GRADIENT: three)
    bool fused[frh::NTYPE] = {false, false, false};
    for (int t = 0; t < frh::NTYPE; ++t)
        fused[t] = ns && d.t[t].nelem && d.t[t].Fgrad.frag && d.t[t].grad_form > 0 &&
                   !(m->flags & FR_SEPARATE_GRADIENT);
    if (ns) {
        FR_LAUNCH(m, 10, s, frd::launch_common_solution<T>(pa, s));
        if (d.nb) FR_LAUNCH(m, 22, s, frd::launch_boundary_solution<T>(ba, s));
        for (int t = 0; t < frh::NTYPE; ++t) {
            DevType<T> &D = d.t[t];
            if (!D.nelem) continue;
            if (fused[t]) {
                const frd::GradFluxArgs<T> ga = gradflux_args<T>(m, D, U[t]);
                FR_LAUNCH(m, prof_gradflux(t), s, frd::launch_gradflux<T>(t, ga, s, D.grad_form == 2));
                continue;
            }
            const int64_t w5 = 5 * D.ld;
            FR_LAUNCH(m, prof_op(t, frd::OP_GRAD), s,
                      opmul<T>(m, 4 * t + frd::OP_GRAD, D.Agrad, D.Sgrad, U[t], w5, D.nu, D.Cf, w5, D.nf, D.Qt, w5, w5, s));
        }
    }
    for (int t = 0; t < frh::NTYPE; ++t) {
        DevType<T> &D = d.t[t];
        if (!D.nelem) continue;
        if (fused[t]) continue;
        const frd::UptsArgs<T> ua = upts_args<T>(m, D, U[t]);
        FR_LAUNCH(m, prof_upts(t), s, frd::launch_upts<T>(t, ns, ua, s));
        if (ns) {
            const int64_t w15 = 15 * D.ld;
            FR_LAUNCH(m, prof_op(t, frd::OP_GRADINTERP), s,
                      opmul<T>(m, 4 * t + frd::OP_GRADINTERP, D.Agint, D.Sgint, D.Q, w15, D.nu, nullptr, 0, 0, D.Qf, w15, w15, s));
        }
    }
    FR_LAUNCH(m, 11, s, frd::launch_common_flux<T>(ns, pa, s));
    if (d.nb) FR_LAUNCH(m, 23, s, frd::launch_boundary_flux<T>(ns, ba, s));
    const Closure *cl = (m->closure && m->closure->params) ? m->closure.get() : nullptr;
    if (cl) {
        const int64_t ntot = d.t[0].nelem + d.t[1].nelem;
        for (int t = 0; t < 2; ++t) {   // the closure covers tets and prisms only
            DevType<T> &D = d.t[t];
            if (!D.nelem) continue;
            // feature-major moments, inputs and outputs: every access coalesced
            FR_LAUNCH(m, 14, s, frd::launch_moments<T>(U[t], nullptr, D.ld, D.nelem, D.nu, cl->Mom[t], cl->mom,
                                                       t ? d.t[0].nelem : 0, 1, ntot, nullptr, s));
        }
        FR_LAUNCH(m, 14, s, frd::launch_features(cl->mom, 1, ntot, cl->nb, ntot, cl->stats, cl->feat, 1, ntot, s));
        FR_LAUNCH(m, 15, s, frd::launch_mlp_forward(cl->params, cl->params_bf16, cl->bf16, cl->feat, 1, ntot, ntot,
                                                    cl->stats, false, cl->y, 1, ntot, s));
    }
    for (int t = 0; t < frh::NTYPE; ++t) {
        DevType<T> &D = d.t[t];
        if (!D.nelem) continue;
        const int64_t w5 = 5 * D.ld;
        frd::NegArgs<T> na{D.Rt, so[t].out, so[t].acc, so[t].base, so[t].a, so[t].b,
                           D.jinv, D.ld, D.nelem, D.nu,
                           so[t].per_elem_dt ? D.dte : nullptr};
        na.err = so[t].err;
        na.c = so[t].c;
        na.err_set = so[t].err_set;
        if (cl && t < 2) {
            na.cy = cl->y;
            na.cys = d.t[0].nelem + d.t[1].nelem;
            na.clift = cl->lift[t];
            na.goff = t ? d.t[0].nelem : 0;
        }
        // -R~/J and the register update ride in the divergence product's
        // store (R~ never reaches memory) unless the closure or
        // FR_SEPARATE_UPDATE asks for the separate kernel
        if (!na.cy && !(m->flags & FR_SEPARATE_UPDATE)) {
            na.fuse = true;
            FR_LAUNCH(m, prof_op(t, frd::OP_DIV), s,
                      opmul<T>(m, 4 * t + frd::OP_DIV, D.Adiv, D.Sdiv, D.Ft, w5, 3 * D.nu, D.Fn, w5, D.nf, D.Rt, w5,
                               w5, s, &na));
            continue;
        }
        FR_LAUNCH(m, prof_op(t, frd::OP_DIV), s,
                  opmul<T>(m, 4 * t + frd::OP_DIV, D.Adiv, D.Sdiv, D.Ft, w5, 3 * D.nu, D.Fn, w5, D.nf, D.Rt, w5, w5, s));
        FR_LAUNCH(m, prof_neg(t), s, frd::launch_negdivconf<T>(t, na, s));
    }
    return FR_OK;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

template <typename T>
fr_status rhs_entry(fr_mesh m, const void *const u[FR_NTYPES], void *const r[FR_NTYPES], hipStream_t s) {
    const T *U[frh::NTYPE] = {nullptr, nullptr, nullptr};
    StageOut<T> so[frh::NTYPE];
    for (int t = 0; t < frh::NTYPE; ++t) {
        if (!m->host.t[t].nelem) continue;
        if (!u || !r || !u[t] || !r[t]) return fail(m, FR_ERR_INVALID_ARG, "null state pointer");
        if (!aligned(u[t], 4 * sizeof(T)) || !aligned(r[t], 4 * sizeof(T)))
            return fail(m, FR_ERR_INVALID_ARG, "state pointers must be 4-element aligned");
        if (u[t] == r[t]) return fail(m, FR_ERR_INVALID_ARG, "r_dev aliases u_dev");
        U[t] = static_cast<const T *>(u[t]);
        so[t].out = static_cast<T *>(r[t]);
    }
    return rhs_pipeline<T>(m, U, so, s);
}

// partial / red_out: device memory for the per-block partial sums
// [NTYPE][RED_BLOCKS][8] and the [NTYPE][8] results (the mesh's own buffers
// when null).  Every type's sums go to their own slots, so one copy and one
// synchronisation bring them all back; the host adds them type by type.
template <typename T>
fr_status reduce_impl(fr_mesh m, int what, double *out, hipStream_t s, double *partial = nullptr,
                      double *red_out = nullptr) {
    Dev<T> &d = dev_of<T>(m);
    if (!partial) partial = d.partial;
    if (!red_out) red_out = d.red_out;
    int nq = (what == 4) ? 2 : (what == 5 ? 1 : 5);
    std::vector<double> tot(8, 0.0);
    const bool needR = what == 2 || what == 3 || what == 4;
    if (needR) {
        const T *U[frh::NTYPE] = {d.t[0].reg[0], d.t[1].reg[0], d.t[2].reg[0]};
        StageOut<T> so[frh::NTYPE];
        for (int t = 0; t < frh::NTYPE; ++t) so[t].out = d.t[t].R;
        fr_status st = rhs_pipeline<T>(m, U, so, s);
        if (st) return st;
    }
    for (int t = 0; t < frh::NTYPE; ++t) {
        DevType<T> &D = d.t[t];
        if (!D.nelem) continue;
        double *pt = partial + size_t(t) * frd::RED_BLOCKS * 8;
        frd::RedArgs<T> ra{D.reg[0], needR ? D.R : nullptr, D.wJ, D.ld, D.nelem, D.nu, what, pt};
        FR_HIP(m, frd::launch_reduce<T>(ra, s));
        FR_HIP(m, frd::launch_reduce_final(pt, frd::RED_BLOCKS, red_out + 8 * t, s));
    }
    double h[frh::NTYPE * 8];
    FR_HIP(m, hipMemcpyAsync(h, red_out, sizeof(h), hipMemcpyDeviceToHost, s));
    FR_HIP(m, hipStreamSynchronize(s));
    for (int t = 0; t < frh::NTYPE; ++t)
        if (d.t[t].nelem)
            for (int q = 0; q < 8; ++q) tot[q] += h[8 * t + q];
    if (what == 4) {
        tot[0] /= m->host.volume;
        tot[1] /= m->host.volume;
    }
    for (int q = 0; q < nq; ++q) out[q] = tot[q];
    return FR_OK;
}

// RK45[2R+] (Kennedy, Carpenter & Lewis 2000, RK4(3)5[2R+]C): sub-diagonal
// a[i+1][i], weights b and the embedded third-order weights bhat.
const double RK45_A[4] = {970286171893.0 / 4311952581923.0, 6584761158862.0 / 12103376702013.0,
                          2251764453980.0 / 15575788980749.0, 26877169314380.0 / 34165994151039.0};
const double RK45_B[5] = {1153189308089.0 / 22510343858157.0, 1772645290293.0 / 4653164025191.0,
                          -1672844663538.0 / 4480602732383.0, 2114624349019.0 / 3568978502595.0,
                          5198255086312.0 / 14908931495163.0};
const double RK45_BHAT[5] = {1016888040809.0 / 7410784769900.0, 11231460423587.0 / 58533540763752.0,
                             -1563879915014.0 / 6823010717585.0, 606302364029.0 / 971179775848.0,
                             1097981568119.0 / 3980877426909.0};

template <typename T>
fr_status rk_impl(fr_mesh m, int scheme, double dt, int nsteps, hipStream_t s,
                  bool per_elem_dt = false, bool allow_check = true) {
    Dev<T> &d = dev_of<T>(m);
    static const double rk4_a[4] = {0.5, 0.5, 1.0, 0.0};
    static const double rk4_b[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    // RK45[2R+]: a[i][j] = b[j] for j < i-1, so two registers suffice
    const double *rk45_a = RK45_A, *rk45_b = RK45_B;
    for (int step = 0; step < nsteps; ++step) {
        if (scheme == FR_FWD_EULER) {
            const T *U[frh::NTYPE] = {d.t[0].reg[0], d.t[1].reg[0], d.t[2].reg[0]};
            StageOut<T> so[frh::NTYPE];
            for (int t = 0; t < frh::NTYPE; ++t) {
                so[t].acc = d.t[t].reg[0];
                so[t].a = T(dt);
                so[t].per_elem_dt = per_elem_dt;
            }
            fr_status st = rhs_pipeline<T>(m, U, so, s);
            if (st) return st;
        } else if (scheme == FR_RK4) {
            for (int t = 0; t < frh::NTYPE; ++t)
                if (d.t[t].nelem)
                    FR_HIP(m, frd::launch_copy<T>(d.t[t].reg[2], d.t[t].reg[0],
                                                  int64_t(d.t[t].nu) * 5 * d.t[t].ld, s));
            for (int st_i = 0; st_i < 4; ++st_i) {
                const T *U[frh::NTYPE];
                StageOut<T> so[frh::NTYPE];
                for (int t = 0; t < frh::NTYPE; ++t) {
                    U[t] = st_i == 0 ? d.t[t].reg[0] : d.t[t].reg[1];
                    so[t].acc = d.t[t].reg[2];
                    so[t].a = T(rk4_b[st_i] * dt);
                    so[t].out = st_i < 3 ? d.t[t].reg[1] : nullptr;
                    so[t].base = d.t[t].reg[0];
                    so[t].b = T(rk4_a[st_i] * dt);
                    so[t].per_elem_dt = per_elem_dt;
                }
                fr_status st = rhs_pipeline<T>(m, U, so, s);
                if (st) return st;
            }
            for (int t = 0; t < frh::NTYPE; ++t) std::swap(d.t[t].reg[0], d.t[t].reg[2]);
        } else if (scheme == FR_RK45_2RP) {
            for (int st_i = 0; st_i < 5; ++st_i) {
                const T *U[frh::NTYPE];
                StageOut<T> so[frh::NTYPE];
                for (int t = 0; t < frh::NTYPE; ++t) {
                    U[t] = st_i == 0 ? d.t[t].reg[0] : d.t[t].reg[1];
                    so[t].acc = d.t[t].reg[0];
                    so[t].a = T(rk45_b[st_i] * dt);
                    so[t].out = st_i < 4 ? d.t[t].reg[1] : nullptr;
                    so[t].b = st_i < 4 ? T((rk45_a[st_i] - rk45_b[st_i]) * dt) : T(0);
                    so[t].per_elem_dt = per_elem_dt;
                }
                fr_status st = rhs_pipeline<T>(m, U, so, s);
                if (st) return st;
            }
        } else {
            return fail(m, FR_ERR_INVALID_ARG, "unknown scheme");
        }
    }
    if (allow_check && (m->flags & FR_CHECK_FINITE)) {
        double bad = 0;
        fr_status st = reduce_impl<T>(m, 5, &bad, s);
        if (st) return st;
        if (bad > 0) return fail(m, FR_ERR_NONFINITE, "non-finite value in the solution");
    }
    return FR_OK;
}

// Adaptive RK45[2R+] (see fr_rk45_adaptive): registers reg[0] = solution q,
// reg[1] = stage input r, reg[2] = the solution at the start of the step,
// ereg = embedded error.
template <typename T>
fr_status rk_adaptive_impl(fr_mesh m, double t_end, double state[3], double atol, double rtol,
                           int max_attempts, int32_t counts[2], hipStream_t s) {
    Dev<T> &d = dev_of<T>(m);
    int64_t ndof = 0;
    for (int t = 0; t < frh::NTYPE; ++t) {
        DevType<T> &D = d.t[t];
        if (!D.nelem) continue;
        if (!D.ereg)
            if (fr_status st = dev_alloc(m, d, D.ereg, size_t(D.nu) * 5 * D.ld)) return st;
        ndof += int64_t(D.nu) * 5 * D.nelem;
    }
    constexpr double K = 4.0, SAFETY = 0.9, FAC_MIN = 0.2, FAC_MAX = 5.0, ERR_FLOOR = 1e-4;
    double t = state[0], dt = state[1], err_prev = state[2];
    counts[0] = counts[1] = 0;
    while (t < t_end && counts[0] + counts[1] < max_attempts) {
        const bool last = t + dt >= t_end;
        const double h = last ? t_end - t : dt;
        for (int ty = 0; ty < frh::NTYPE; ++ty)
            if (d.t[ty].nelem)
                FR_HIP(m, frd::launch_copy<T>(d.t[ty].reg[2], d.t[ty].reg[0], int64_t(d.t[ty].nu) * 5 * d.t[ty].ld, s));
        for (int st_i = 0; st_i < 5; ++st_i) {
            const T *U[frh::NTYPE];
            StageOut<T> so[frh::NTYPE];
            for (int ty = 0; ty < frh::NTYPE; ++ty) {
                U[ty] = st_i == 0 ? d.t[ty].reg[0] : d.t[ty].reg[1];
                so[ty].acc = d.t[ty].reg[0];
                so[ty].a = T(RK45_B[st_i] * h);
                so[ty].out = st_i < 4 ? d.t[ty].reg[1] : nullptr;
                so[ty].b = st_i < 4 ? T((RK45_A[st_i] - RK45_B[st_i]) * h) : T(0);
                so[ty].err = d.t[ty].ereg;
                so[ty].c = T((RK45_B[st_i] - RK45_BHAT[st_i]) * h);
                so[ty].err_set = st_i == 0;
            }
            fr_status st = rhs_pipeline<T>(m, U, so, s);
            if (st) return st;
        }
        // fused error norm: sum (e / (atol + rtol max(|u_old|, |u_new|)))^2 in FP64
        double sum = 0;
        for (int ty = 0; ty < frh::NTYPE; ++ty) {
            DevType<T> &D = d.t[ty];
            if (!D.nelem) continue;
            double *pt = d.partial + size_t(ty) * frd::RED_BLOCKS * 8;
            frd::RedArgs<T> ra{D.reg[0], D.ereg, D.wJ, D.ld, D.nelem, D.nu, 6, pt};
            ra.U0 = D.reg[2];
            ra.atol = atol;
            ra.rtol = rtol;
            FR_HIP(m, frd::launch_reduce<T>(ra, s));
            FR_HIP(m, frd::launch_reduce_final(pt, frd::RED_BLOCKS, d.red_out + 8 * ty, s));
        }
        double hsum[frh::NTYPE * 8];
        FR_HIP(m, hipMemcpyAsync(hsum, d.red_out, sizeof(hsum), hipMemcpyDeviceToHost, s));
        FR_HIP(m, hipStreamSynchronize(s));
        for (int ty = 0; ty < frh::NTYPE; ++ty)
            if (d.t[ty].nelem) sum += hsum[8 * ty];
        const double err = std::sqrt(sum / double(ndof));
        if (!std::isfinite(err)) {
            for (int ty = 0; ty < frh::NTYPE; ++ty)
                if (d.t[ty].nelem)
                    FR_HIP(m, frd::launch_copy<T>(d.t[ty].reg[0], d.t[ty].reg[2], int64_t(d.t[ty].nu) * 5 * d.t[ty].ld, s));
            state[0] = t;
            state[1] = dt;
            state[2] = err_prev;
            return fail(m, FR_ERR_NONFINITE, "non-finite error estimate; the step was undone");
        }
        if (err <= 1.0) {
            double fac = err == 0.0 ? FAC_MAX : SAFETY * std::pow(err, -0.7 / K) * std::pow(err_prev, 0.4 / K);
            fac = std::min(FAC_MAX, std::max(FAC_MIN, fac));
            t = last ? t_end : t + h;
            err_prev = std::max(err, ERR_FLOOR);
            dt = h * fac;
            counts[0] += 1;
        } else {
            for (int ty = 0; ty < frh::NTYPE; ++ty)
                if (d.t[ty].nelem)
                    FR_HIP(m, frd::launch_copy<T>(d.t[ty].reg[0], d.t[ty].reg[2], int64_t(d.t[ty].nu) * 5 * d.t[ty].ld, s));
            dt = h * std::min(1.0, std::max(FAC_MIN, SAFETY * std::pow(err, -1.0 / K)));
            counts[1] += 1;
        }
    }
    state[0] = t;
    state[1] = dt;
    state[2] = err_prev;
    return FR_OK;
}

fr_status check_mesh(fr_mesh m, int etype, bool need_device) {
    if (!m) return FR_ERR_INVALID_ARG;
    if (etype < 0 || etype >= frh::NTYPE) return fail(m, FR_ERR_INVALID_ARG, "unknown element type");
    if (need_device && !m->device) return fail(m, FR_ERR_INVALID_ARG, "mesh was created validate-only");
    return FR_OK;
}

template <typename T>
fr_status copy_state(fr_mesh m, int etype, void *dst, const void *src, bool to_reg,
                            hipStream_t s) {
    Dev<T> &d = dev_of<T>(m);
    DevType<T> &D = d.t[etype];
    if (!D.nelem) return FR_OK;
    const size_t n = size_t(D.nu) * 5 * D.ld * sizeof(T);
    if (to_reg)
        FR_HIP(m, hipMemcpyAsync(D.reg[0], src, n, hipMemcpyDeviceToDevice, s));
    else
        FR_HIP(m, hipMemcpyAsync(dst, D.reg[0], n, hipMemcpyDeviceToDevice, s));
    return FR_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for every operator product of every element type, time each
// row-blocking candidate (row blocks of 16 per wavefront) on the mesh's own
// buffers and keep the fastest.  The blocking does not change any output's
// accumulation order, so results are bitwise unchanged.
// ---------------------------------------------------------------------------
template <typename T>
fr_status autotune_impl(fr_mesh m, hipStream_t s, std::string &report) {
    Dev<T> &d = dev_of<T>(m);
    const bool split = m->precision == FR_SPLIT_BF16 || m->precision == FR_SPLIT_FP16;
    const int fmt = m->precision == FR_SPLIT_FP16 ? 2 : 1;
    const bool ns = m->system == FR_NAVIER_STOKES;
    hipEvent_t e0, e1;
    FR_HIP(m, hipEventCreate(&e0));
    FR_HIP(m, hipEventCreate(&e1));
    std::vector<int> caps;
    if (split) caps = fmt == 2 ? std::vector<int>{1, 2} : std::vector<int>{1, 2, 4};
    else caps = sizeof(T) == 4 ? std::vector<int>{1, 2, 4, 8} : std::vector<int>{1, 2, 4};
    fr_status st = FR_OK;
    for (int t = 0; t < frh::NTYPE && !st; ++t) {
        DevType<T> &D = d.t[t];
        if (!D.nelem) continue;
        const frh::RefOps &R = m->host.t[t].ops;
        std::vector<double> grad, div;
        folded_ops(R, grad, div);
        const int nu = D.nu, nf = D.nf;
        const int64_t w5 = 5 * D.ld, w15 = 15 * D.ld;
        struct Case {
            int op;
            const std::vector<double> *A;
            int M, K;
            const T *B1;
            int64_t l1;
            int K1;
            const T *B2;
            int64_t l2;
            int K2;
            T *C;
            int64_t lc, ncols;
            frd::Op<T> *dst;
            frd::OpSplit *sdst;
        };
        std::vector<Case> cases = {
            {frd::OP_INTERP, &R.M0, nf, nu, D.reg[0], w5, nu, nullptr, 0, 0, D.Uf, w5, w5, &D.Aint, &D.Sint},
            {frd::OP_DIV, &div, nu, 3 * nu + nf, D.Ft, w5, 3 * nu, D.Fn, w5, nf, D.Rt, w5, w5, &D.Adiv, &D.Sdiv}};
        if (ns) {
            cases.push_back({frd::OP_GRAD, &grad, 3 * nu, nu + nf, D.reg[0], w5, nu, D.Cf, w5, nf, D.Qt, w5, w5,
                             &D.Agrad, &D.Sgrad});
            cases.push_back({frd::OP_GRADINTERP, &R.M0, nf, nu, D.Q, w15, nu, nullptr, 0, 0, D.Qf, w15, w15,
                             &D.Agint, &D.Sgint});
        }
        for (const Case &c : cases) {
            float best = 1e30f;
            int best_cap = -1, best_stage = 0;
            std::vector<void *> bufs;
            frd::Op<T> best_op;
            frd::OpSplit best_sop;
            std::vector<std::pair<int, int>> cands;
            for (int cap : caps)
                for (int stage = 0; stage < (split ? 2 : 7); ++stage) {
                    if (sizeof(T) != 4 && (stage == 1 || stage == 2 || stage == 4)) continue;
                    int nmg, mbw;
                    frd::row_groups(c.M, cap, nmg, mbw);
                    if ((stage == 5 || stage == 6) && mbw > 4) continue;
                    if (split) {
                        if (stage == 1 && (nmg > 8 || nmg * (fmt == 2 ? 2 : 3) * 4096 > 65536)) continue;
                        cands.push_back({cap, stage});
                        continue;
                    }
                    if ((stage == 1 || stage == 2) && nmg > 8) continue;
                    if (stage == 4 && size_t(mbw) * ((((c.K + 3) / 4) + 7) / 8 * 8) * 256 > 65536) continue;
                    cands.push_back({cap, stage});
                }
            for (auto [cap, stage] : cands) {
                frd::Op<T> op;
                frd::OpSplit sop;
                std::vector<void *> mine;
                if (split) {
                    std::vector<uint16_t> parts[3];
                    sop = fragment_split(*c.A, c.M, c.K, fmt, parts, cap);
                    sop.stage = stage;
                    for (int q = 0; q < 3; ++q) {
                        if (parts[q].empty()) continue;
                        void *p;
                        FR_HIP(m, hipMalloc(&p, parts[q].size() * 2));
                        FR_HIP(m, hipMemcpy(p, parts[q].data(), parts[q].size() * 2, hipMemcpyHostToDevice));
                        sop.part[q] = static_cast<uint16_t *>(p);
                        mine.push_back(p);
                    }
                } else {
                    std::vector<T> f;
                    std::vector<int32_t> idx;
                    op = fragment<T>(*c.A, c.M, c.K, f, cap, stage, &idx);
                    FR_HIP(m, upload_op(op, f, idx, mine));
                }
                // the divergence is timed with the fused store the RK stages
                // use: read, update and write an accumulator and write the
                // output (both the R~ buffer here, unused when fused)
                frd::NegArgs<T> na{};
                na.out = D.Rt;
                na.acc = D.Rt;
                na.a = T(0);
                na.b = T(1);
                na.jinv = D.jinv;
                na.ld = D.ld;
                na.nelem = D.nelem;
                na.nu = D.nu;
                na.fuse = true;
                const frd::NegArgs<T> *ep =
                    c.op == frd::OP_DIV && !(m->flags & FR_SEPARATE_UPDATE) ? &na : nullptr;
                auto run = [&]() -> hipError_t {
                    if constexpr (std::is_same<T, float>::value) {
                        if (split)
                            return frd::launch_opmul_split(4 * t + c.op, sop, c.B1, c.l1, c.K1, c.B2, c.l2,
                                                           c.K2, c.C, c.lc, c.ncols, s, ep);
                    }
                    return frd::launch_opmul<T>(4 * t + c.op, op, c.B1, c.l1, c.K1, c.B2, c.l2, c.K2,
                                                c.C, c.lc, c.ncols, s, ep);
                };
                FR_HIP(m, run());
                FR_HIP(m, hipEventRecord(e0, s));
                for (int r = 0; r < 3; ++r) FR_HIP(m, run());
                FR_HIP(m, hipEventRecord(e1, s));
                FR_HIP(m, hipEventSynchronize(e1));
                float ms = 0;
                FR_HIP(m, hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    for (void *p : bufs) (void)hipFree(p);
                    bufs = mine;
                    best = ms;
                    best_cap = cap;
                    best_stage = stage;
                    best_op = op;
                    best_sop = sop;
                } else {
                    for (void *p : mine) (void)hipFree(p);
                }
            }
            for (void *p : bufs) d.allocs.push_back(p);
            if (split)
                *c.sdst = best_sop;
            else
                *c.dst = best_op;
            static const char *const short_name[frh::NTYPE] = {"tet", "pri", "hex"};
            report += short_name[t] + std::string(" op") + std::to_string(c.op) + " cap " +
                      std::to_string(best_cap) + " stage " + std::to_string(best_stage) + " " +
                      std::to_string(best / 3 * 1e3) + " us; ";
        }
        // the gradient stage (Navier-Stokes): the fused kernel
        // against the three separate kernels with the variants just chosen
        if (ns && D.Fgrad.frag && !(m->flags & FR_SEPARATE_GRADIENT)) {
            const T *U = D.reg[0];
            auto run = [&](int form) -> hipError_t {
                if (form > 0) return frd::launch_gradflux<T>(t, gradflux_args<T>(m, D, U), s, form == 2);
                hipError_t e = opmul<T>(m, 4 * t + frd::OP_GRAD, D.Agrad, D.Sgrad, U, w5, nu, D.Cf, w5, nf, D.Qt,
                                        w5, w5, s);
                if (e == hipSuccess) e = frd::launch_upts<T>(t, true, upts_args<T>(m, D, U), s);
                if (e == hipSuccess)
                    e = opmul<T>(m, 4 * t + frd::OP_GRADINTERP, D.Agint, D.Sgint, D.Q, w15, nu, nullptr, 0, 0,
                                 D.Qf, w15, w15, s);
                return e;
            };
            const int nform = sizeof(T) == 4 && t < 2 ? 3 : 2;   // streaming: FP32 tets and prisms
            float ms[3] = {0, 0, 0};
            for (int form = 0; form < nform; ++form) {
                FR_HIP(m, run(form));
                FR_HIP(m, hipEventRecord(e0, s));
                for (int r = 0; r < 3; ++r) FR_HIP(m, run(form));
                FR_HIP(m, hipEventRecord(e1, s));
                FR_HIP(m, hipEventSynchronize(e1));
                FR_HIP(m, hipEventElapsedTime(&ms[form], e0, e1));
            }
            int best = 0;
            for (int form = 1; form < nform; ++form)
                if (ms[form] < ms[best]) best = form;
            D.grad_form = best;
            static const char *const sn[frh::NTYPE] = {"tet", "pri", "hex"};
            report += sn[t] + std::string(" gradient stage: separate ") + std::to_string(ms[0] / 3 * 1e3) +
                      " us, fused " + std::to_string(ms[1] / 3 * 1e3) + " us" +
                      (nform > 2 ? ", streaming " + std::to_string(ms[2] / 3 * 1e3) + " us" : std::string()) +
                      ", form " + std::to_string(best) + "; ";
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches of independent problems
// ---------------------------------------------------------------------------
struct fr_batch_s {
    int n = 0, system = 0, precision = 0;
    std::unique_ptr<fr_mesh_s> group[4];     // one merged mesh per order p = 1..4
    struct Prob {
        int g = 0;
        int64_t off[frh::NTYPE] = {}, ne[frh::NTYPE] = {}, ld[frh::NTYPE] = {};
        int nu[frh::NTYPE] = {};
    };
    std::vector<Prob> prob;
    hipStream_t stream = nullptr;             // stream the step graph replays on
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // register pointers (group, type, register) the graph was captured with:
    // an RK4 step swaps registers, after which the graph would advance a
    // stale buffer, so a mismatch re-captures it
    std::vector<const void *> graph_regs;
    bool use_graph = true;
    std::string err;
    ~fr_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

fr_status bfail(fr_batch b, fr_status st, const std::string &msg) {
    if (b)
        b->err = msg;
    else
        g_create_error = msg;
    return st;
}

#define FR_BHIP(b, call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return bfail(b, e_ == hipErrorOutOfMemory ? FR_ERR_OUT_OF_MEMORY : FR_ERR_DEVICE, \
                         std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

template <typename T>
fr_status batch_alloc_dt(fr_mesh m) {
    Dev<T> &d = dev_of<T>(m);
    for (int t = 0; t < frh::NTYPE; ++t) {
        if (!d.t[t].nelem) continue;
        FR_HIP(m, hipMalloc(reinterpret_cast<void **>(&d.t[t].dte), size_t(d.t[t].ld) * sizeof(T)));
        d.allocs.push_back(d.t[t].dte);
        FR_HIP(m, hipMemset(d.t[t].dte, 0, size_t(d.t[t].ld) * sizeof(T)));
    }
    return FR_OK;
}

template <typename T>
void *group_reg(fr_mesh m, int t) {
    return dev_of<T>(m).t[t].reg[0];
}

template <typename T>
T *group_dte(fr_mesh m, int t) {
    return dev_of<T>(m).t[t].dte;
}

// Host tables of one mesh description.
bool build_host(const fr_mesh_desc &d, frh::MeshHost &h, std::string &err) {
    const int64_t ne[frh::NTYPE] = {d.n_tets, d.n_prisms, d.n_hex};
    const int64_t *const conn[frh::NTYPE] = {d.tet_v, d.pri_v, d.hex_v};
    const int8_t *const img[frh::NTYPE] = {d.tet_img, d.pri_img, d.hex_img};
    const double *const quad[frh::NTYPE] = {d.tet_q, d.pri_q, d.hex_q};
    return frh::build_mesh_host(d.order, d.n_vertices, d.xyz, ne, conn, img, quad, d.period, d.n_bfaces,
                                d.bfaces, h, err);
}

}  // namespace

extern "C" {

fr_status fr_mesh_create(const fr_mesh_desc *desc, void *stream, fr_mesh *out) {
    g_create_error.clear();
    if (!desc || !out) return fail(nullptr, FR_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (desc->order < 1 || desc->order > 4)
        return fail(nullptr, FR_ERR_UNSUPPORTED, "order must be 1..4");
    if (desc->system != FR_EULER && desc->system != FR_NAVIER_STOKES)
        return fail(nullptr, FR_ERR_INVALID_ARG, "unknown system");
    if (desc->precision < FR_FP32 || desc->precision > FR_SPLIT_FP16)
        return fail(nullptr, FR_ERR_UNSUPPORTED, "unsupported precision");
    if (desc->n_vertices <= 0 || !desc->xyz || desc->n_tets < 0 || desc->n_prisms < 0 || desc->n_hex < 0 ||
        (desc->n_tets && !desc->tet_v) || (desc->n_prisms && !desc->pri_v) || (desc->n_hex && !desc->hex_v) ||
        desc->n_tets + desc->n_prisms + desc->n_hex == 0)
        return fail(nullptr, FR_ERR_INVALID_ARG, "empty or inconsistent mesh arrays");
    if (!(desc->gamma > 1) || desc->mu < 0 ||
        (desc->system == FR_NAVIER_STOKES && !(desc->prandtl > 0)) || !std::isfinite(desc->p_ref))
        return fail(nullptr, FR_ERR_INVALID_ARG, "invalid physical constants");
    if (desc->n_bfaces < 0 || (desc->n_bfaces && !desc->bfaces))
        return fail(nullptr, FR_ERR_INVALID_ARG, "inconsistent boundary face list");
    for (int64_t i = 0; i < desc->n_bfaces; ++i) {
        const int64_t kind = desc->bfaces[4 * i + 3];
        if (kind == FR_BC_WALL && !(desc->t_wall > 0))
            return fail(nullptr, FR_ERR_INVALID_ARG, "wall faces need a positive wall temperature");
        if (kind == FR_BC_FARFIELD && !(desc->farfield[0] > 0 && desc->farfield[4] > 0))
            return fail(nullptr, FR_ERR_INVALID_ARG, "far-field faces need a positive free-stream density and pressure");
    }
    auto m = std::make_unique<fr_mesh_s>();
    m->order = desc->order;
    m->system = desc->system;
    m->precision = desc->precision;
    m->flags = desc->flags;
    m->gamma = desc->gamma;
    m->mu = desc->mu;
    m->prandtl = desc->prandtl;
    m->beta = desc->ldg_beta;
    m->tau = desc->ldg_tau;
    m->t_wall = desc->t_wall;
    for (int k = 0; k < 5; ++k) m->farfield[k] = desc->farfield[k];
    m->pref = desc->p_ref;
    std::string err;
    try {
        if (!build_host(*desc, m->host, err)) return fail(nullptr, FR_ERR_BAD_MESH, err);
    } catch (const std::exception &ex) {
        return fail(nullptr, FR_ERR_BAD_MESH, ex.what());
    }
    if (!(desc->flags & FR_VALIDATE_ONLY)) {
        hipStream_t s = static_cast<hipStream_t>(stream);
        m->create_stream = s;
        fr_status st = m->precision != FR_FP64 ? setup_device<float>(m.get(), s)
                                               : setup_device<double>(m.get(), s);
        if (st) {
            g_create_error = m->err;
            return st;
        }
        m->device = true;
    }
    *out = m.release();
    return FR_OK;
}

fr_status fr_mesh_destroy(fr_mesh mesh) {
    if (!mesh) return FR_OK;
    if (mesh->device) (void)hipStreamSynchronize(mesh->create_stream);
    delete mesh;
    return FR_OK;
}

fr_status fr_mesh_query(fr_mesh m, int32_t etype, int64_t *n_elem, int32_t *n_upts,
                        int32_t *n_fpts, int64_t *ld) {
    if (fr_status st = check_mesh(m, etype, false)) return st;
    const frh::TypeHost &H = m->host.t[etype];
    if (n_elem) *n_elem = H.nelem;
    if (n_upts) *n_upts = frh::n_upts(etype, m->order);
    if (n_fpts) *n_fpts = frh::n_fpts(etype, m->order);
    if (ld) *ld = H.ld;
    return FR_OK;
}

fr_status fr_upts_coords(fr_mesh m, int32_t etype, double *xyz) {
    if (fr_status st = check_mesh(m, etype, false)) return st;
    if (!xyz) return fail(m, FR_ERR_INVALID_ARG, "null output");
    const frh::TypeHost &H = m->host.t[etype];
    if (!H.nelem) return FR_OK;
    const int nu = H.ops.nu;
    for (int i = 0; i < nu; ++i)
        for (int64_t e = 0; e < H.nelem; ++e) {
            double x[3];
            frh::elem_point_at(H, etype, e, false, i, x);
            for (int d = 0; d < 3; ++d) xyz[(size_t(i) * 3 + d) * H.nelem + e] = x[d];
        }
    return FR_OK;
}

fr_status fr_operator(fr_mesh m, int32_t etype, int32_t which, double *out, int32_t *rows,
                      int32_t *cols) {
    if (fr_status st = check_mesh(m, etype, false)) return st;
    const frh::TypeHost &H = m->host.t[etype];
    if (!H.nelem) return fail(m, FR_ERR_INVALID_ARG, "mesh has no elements of that type");
    const frh::RefOps &R = H.ops;
    const double *src;
    int r, c;
    switch (which) {
        case 0: src = R.M0.data(); r = R.nf; c = R.nu; break;
        case 1: case 2: case 3: src = R.G.data() + size_t(which - 1) * R.nu * R.nu; r = R.nu; c = R.nu; break;
        case 4: src = R.L.data(); r = R.nu; c = R.nf; break;
        case 5: src = R.w.data(); r = 1; c = R.nu; break;
        case 6: src = R.nref.data(); r = R.nf; c = 3; break;
        default: return fail(m, FR_ERR_INVALID_ARG, "unknown operator");
    }
    if (rows) *rows = r;
    if (cols) *cols = c;
    if (out) std::memcpy(out, src, size_t(r) * c * sizeof(double));
    return FR_OK;
}

fr_status fr_set_solution(fr_mesh m, int32_t etype, const void *u, void *stream) {
    if (fr_status st = check_mesh(m, etype, true)) return st;
    if (!u && m->host.t[etype].nelem) return fail(m, FR_ERR_INVALID_ARG, "null state");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? copy_state<float>(m, etype, nullptr, u, true, s)
                                   : copy_state<double>(m, etype, nullptr, u, true, s);
}

fr_status fr_get_solution(fr_mesh m, int32_t etype, void *u, void *stream) {
    if (fr_status st = check_mesh(m, etype, true)) return st;
    if (!u && m->host.t[etype].nelem) return fail(m, FR_ERR_INVALID_ARG, "null state");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? copy_state<float>(m, etype, u, nullptr, false, s)
                                   : copy_state<double>(m, etype, u, nullptr, false, s);
}

fr_status fr_rhs(fr_mesh m, const void *const u[FR_NTYPES], void *const r[FR_NTYPES], void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? rhs_entry<float>(m, u, r, s) : rhs_entry<double>(m, u, r, s);
}

fr_status fr_rk_step(fr_mesh m, int32_t scheme, double dt, int32_t n_steps, void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (n_steps < 0 || !std::isfinite(dt)) return fail(m, FR_ERR_INVALID_ARG, "bad step count or dt");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? rk_impl<float>(m, scheme, dt, n_steps, s)
                                   : rk_impl<double>(m, scheme, dt, n_steps, s);
}

fr_status fr_rk45_adaptive(fr_mesh m, double t_end, double state[3], double atol, double rtol,
                           int32_t max_attempts, int32_t counts[2], void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!state || !counts) return fail(m, FR_ERR_INVALID_ARG, "null state or counts");
    if (!(state[1] > 0) || !(state[2] > 0) || !(atol >= 0) || !(rtol >= 0) || !(atol + rtol > 0) ||
        max_attempts < 0 || !std::isfinite(t_end) || !std::isfinite(state[0]))
        return fail(m, FR_ERR_INVALID_ARG, "dt and err_prev must be positive, tolerances non-negative");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? rk_adaptive_impl<float>(m, t_end, state, atol, rtol, max_attempts, counts, s)
                                   : rk_adaptive_impl<double>(m, t_end, state, atol, rtol, max_attempts, counts, s);
}

}  // extern "C"

namespace {

// Device memory of fr_reduce_noalloc: the per-block partial sums of the
// reduction ([NTYPE][RED_BLOCKS][8] doubles) and its [NTYPE][8] results.  The
// reduction's grid is fixed (RED_BLOCKS blocks striding over each type's
// elements), so this array is large enough for every mesh.  Each GPU the library runs on holds its own
// copy until the process ends; in host code the name stands for no device
// address, so the address is looked up once per device (hipGetSymbolAddress)
// and only that pointer is passed to kernels and copies.
constexpr size_t NOALLOC_DOUBLES = size_t(frh::NTYPE) * (size_t(frd::RED_BLOCKS) * 8 + 8);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// This device's copy of `scratch` (looked up on its first use, with the
// device current); null with the HIP error in *err on failure.
double *scratch_of_current_device(hipError_t *err) {
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

fr_status fr_reduce_noalloc(fr_mesh m, int32_t what, double *out, void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!out || what < 1 || what > 4) return fail(m, FR_ERR_INVALID_ARG, "bad reduction request");
    hipError_t e = hipSuccess;
    double *ptr = scratch_of_current_device(&e);
    if (!ptr) return fail(m, FR_ERR_DEVICE, std::string("device scratch of fr_reduce_noalloc: ") + hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *partial = ptr, *res = ptr + size_t(frh::NTYPE) * frd::RED_BLOCKS * 8;
    return m->precision != FR_FP64 ? reduce_impl<float>(m, what, out, s, partial, res)
                                   : reduce_impl<double>(m, what, out, s, partial, res);
}

fr_status fr_reduce(fr_mesh m, int32_t what, double *out, void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!out || what < 1 || what > 4) return fail(m, FR_ERR_INVALID_ARG, "bad reduction request");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? reduce_impl<float>(m, what, out, s)
                                   : reduce_impl<double>(m, what, out, s);
}

fr_status fr_intermediate(fr_mesh m, int32_t etype, int32_t which, void *dst, void *stream) {
    if (fr_status st = check_mesh(m, etype, true)) return st;
    if (!dst) return fail(m, FR_ERR_INVALID_ARG, "null destination");
    if (which == 2 && m->system != FR_NAVIER_STOKES)
        return fail(m, FR_ERR_INVALID_ARG, "gradients exist for Navier-Stokes only");
    if (which < 0 || which > 2) return fail(m, FR_ERR_INVALID_ARG, "unknown intermediate");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const frh::TypeHost &H = m->host.t[etype];
    if (!H.nelem) return FR_OK;
    const size_t esz = m->precision != FR_FP64 ? 4 : 8;
    const size_t n = size_t(H.ops.nf) * (which == 2 ? 15 : 5) * H.ld * esz;
    const void *src;
    if (m->precision != FR_FP64) {
        auto &D = dev_of<float>(m).t[etype];
        src = which == 0 ? (void *)D.Uf : which == 1 ? (void *)D.Fn : (void *)D.Qf;
    } else {
        auto &D = dev_of<double>(m).t[etype];
        src = which == 0 ? (void *)D.Uf : which == 1 ? (void *)D.Fn : (void *)D.Qf;
    }
    FR_HIP(m, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, s));
    return FR_OK;
}

fr_status fr_profile(fr_mesh m, int32_t enable) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    m->prof.on = enable != 0;
    m->prof.recs.clear();
    m->prof.used = 0;
    return FR_OK;
}

fr_status fr_profile_read(fr_mesh m, double *total_ms, int64_t *count) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!total_ms || !count) return fail(m, FR_ERR_INVALID_ARG, "null output");
    for (int c = 0; c < PROF_NCLASS; ++c) {
        total_ms[c] = 0;
        count[c] = 0;
    }
    Profiler &P = m->prof;
    for (auto &r : P.recs) {
        FR_HIP(m, hipEventSynchronize(P.pool[r.second + 1]));
        float ms = 0;
        FR_HIP(m, hipEventElapsedTime(&ms, P.pool[r.second], P.pool[r.second + 1]));
        total_ms[r.first] += ms;
        count[r.first] += 1;
    }
    P.recs.clear();
    P.used = 0;
    return FR_OK;
}

}  // extern "C"

namespace {
template <typename T>
fr_status set_blocking_impl(fr_mesh m, int t, int op, int cap, int stage) {
    Dev<T> &d = dev_of<T>(m);
    DevType<T> &D = d.t[t];
    const frh::RefOps &R = m->host.t[t].ops;
    std::vector<double> grad, div;
    folded_ops(R, grad, div);
    const int nu = D.nu, nf = D.nf;
    const std::vector<double> *A = op == frd::OP_GRAD ? &grad : op == frd::OP_DIV ? &div : &R.M0;
    const int M = op == frd::OP_GRAD ? 3 * nu : op == frd::OP_DIV ? nu : nf;
    const int K = op == frd::OP_GRAD ? nu + nf : op == frd::OP_DIV ? 3 * nu + nf : nu;
    const bool split = m->precision == FR_SPLIT_BF16 || m->precision == FR_SPLIT_FP16;
    if (split) {
        if (stage > 1) return fail(m, FR_ERR_UNSUPPORTED, "the split forms have stages 0 and 1");
        const int fmt = m->precision == FR_SPLIT_FP16 ? 2 : 1;
        if (cap > (fmt == 2 ? 2 : 4)) return fail(m, FR_ERR_UNSUPPORTED, "row-block cap too large for this form");
        std::vector<uint16_t> parts[3];
        frd::OpSplit so = fragment_split(*A, M, K, fmt, parts, cap);
        so.stage = stage;
        if (stage == 1 && (so.nmg > 8 || so.nmg * (fmt == 2 ? 2 : 3) * 4096 > 65536))
            return fail(m, FR_ERR_UNSUPPORTED, "too many row groups to share the split operand");
        for (int q = 0; q < 3; ++q) {
            if (parts[q].empty()) continue;
            void *p;
            FR_HIP(m, hipMalloc(&p, parts[q].size() * 2));
            d.allocs.push_back(p);
            FR_HIP(m, hipMemcpy(p, parts[q].data(), parts[q].size() * 2, hipMemcpyHostToDevice));
            so.part[q] = static_cast<uint16_t *>(p);
        }
        frd::OpSplit *dst[4] = {&D.Sint, &D.Sgrad, &D.Sgint, &D.Sdiv};
        *dst[op] = so;
        return FR_OK;
    }
    if (cap > (sizeof(T) == 4 ? 8 : 4)) return fail(m, FR_ERR_UNSUPPORTED, "row-block cap too large for this precision");
    const bool lds = stage == 1 || stage == 2 || stage == 4;
    if (lds && sizeof(T) != 4) return fail(m, FR_ERR_UNSUPPORTED, "LDS staging is for the FP32 product only");
    std::vector<T> f;
    std::vector<int32_t> idx;
    frd::Op<T> o = fragment<T>(*A, M, K, f, cap, stage, &idx);
    if ((stage == 1 || stage == 2) && o.nmg > 8)
        return fail(m, FR_ERR_UNSUPPORTED, "LDS staging needs at most 8 row groups");
    if (stage == 4 && size_t(o.mbw) * o.Kb * 256 > 65536)
        return fail(m, FR_ERR_UNSUPPORTED, "operator slice too large for LDS");
    if ((stage == 5 || stage == 6) && o.mbw > 4)
        return fail(m, FR_ERR_UNSUPPORTED, "the step-list product takes at most 4 row blocks per wavefront");
    FR_HIP(m, upload_op(o, f, idx, d.allocs));
    frd::Op<T> *dst[4] = {&D.Aint, &D.Agrad, &D.Agint, &D.Adiv};
    *dst[op] = o;
    return FR_OK;
}
}  // namespace

extern "C" {

fr_status fr_set_blocking(fr_mesh m, int32_t etype, int32_t op, int32_t cap, int32_t stage) {
    if (fr_status st = check_mesh(m, etype, true)) return st;
    if (op == 4) {
        // the gradient stage's form (stage 0 separate, 1 fused, 2 streaming)
        if (stage < 0 || stage > 2) return fail(m, FR_ERR_INVALID_ARG, "gradient stage form 0..2");
        if (!m->host.t[etype].nelem) return FR_OK;
        const bool have = m->precision == FR_FP64 ? dev_of<double>(m).t[etype].Fgrad.frag != nullptr
                                                  : dev_of<float>(m).t[etype].Fgrad.frag != nullptr;
        if (stage > 0 && !have) return fail(m, FR_ERR_UNSUPPORTED, "no fused gradient stage for this type or form");
        if (stage == 2 && (m->precision != FR_FP32 || etype == 2))
            return fail(m, FR_ERR_UNSUPPORTED, "the streaming gradient stage is FP32 tets and prisms only");
        if (m->precision == FR_FP64)
            dev_of<double>(m).t[etype].grad_form = stage;
        else
            dev_of<float>(m).t[etype].grad_form = stage;
        return FR_OK;
    }
    if (op < 0 || op > 3 || cap < 1 || stage < 0 || stage > 6)
        return fail(m, FR_ERR_INVALID_ARG, "operator 0..4, cap >= 1, stage 0..6");
    if (!m->host.t[etype].nelem) return FR_OK;
    return m->precision != FR_FP64 ? set_blocking_impl<float>(m, etype, op, cap, stage)
                                   : set_blocking_impl<double>(m, etype, op, cap, stage);
}

fr_status fr_autotune(fr_mesh m, void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string rep;
    fr_status st = m->precision != FR_FP64 ? autotune_impl<float>(m, s, rep) : autotune_impl<double>(m, s, rep);
    if (!st) m->err = rep;
    return st;
}

fr_status fr_batch_create(int32_t n, const fr_mesh_desc *descs, void *stream, fr_batch *out) {
    g_create_error.clear();
    if (n <= 0 || !descs || !out) return bfail(nullptr, FR_ERR_INVALID_ARG, "null argument or empty batch");
    *out = nullptr;
    const fr_mesh_desc &d0 = descs[0];
    for (int i = 0; i < n; ++i) {
        const fr_mesh_desc &d = descs[i];
        bool same_bc = d.t_wall == d0.t_wall;
        for (int k = 0; k < 5; ++k) same_bc = same_bc && d.farfield[k] == d0.farfield[k];
        if (d.system != d0.system || d.precision != d0.precision || d.gamma != d0.gamma ||
            d.mu != d0.mu || d.prandtl != d0.prandtl || d.ldg_beta != d0.ldg_beta ||
            d.ldg_tau != d0.ldg_tau || d.p_ref != d0.p_ref || !std::isfinite(d.p_ref) || !same_bc)
            return bfail(nullptr, FR_ERR_INVALID_ARG,
                         "problem " + std::to_string(i) + ": system, precision and constants must match");
        if (d.order < 1 || d.order > 4)
            return bfail(nullptr, FR_ERR_UNSUPPORTED, "problem " + std::to_string(i) + ": order must be 1..4");
        if (d.flags & FR_VALIDATE_ONLY)
            return bfail(nullptr, FR_ERR_INVALID_ARG, "batches are built on the device");
    }
    if (d0.precision < FR_FP32 || d0.precision > FR_SPLIT_FP16)
        return bfail(nullptr, FR_ERR_UNSUPPORTED, "unsupported precision");
    auto b = std::make_unique<fr_batch_s>();
    b->n = n;
    b->system = d0.system;
    b->precision = d0.precision;
    b->prob.resize(n);
    std::vector<frh::MeshHost> parts[4];
    std::vector<int> members[4];
    for (int i = 0; i < n; ++i) {
        const fr_mesh_desc &d = descs[i];
        frh::MeshHost h;
        std::string err;
        try {
            if (!build_host(d, h, err))
                return bfail(nullptr, FR_ERR_BAD_MESH, "problem " + std::to_string(i) + ": " + err);
        } catch (const std::exception &ex) {
            return bfail(nullptr, FR_ERR_BAD_MESH, ex.what());
        }
        b->prob[i].g = d.order - 1;
        for (int t = 0; t < frh::NTYPE; ++t) {
            b->prob[i].ne[t] = h.t[t].nelem;
            b->prob[i].ld[t] = h.t[t].ld;
            b->prob[i].nu[t] = frh::n_upts(t, d.order);
        }
        parts[d.order - 1].push_back(std::move(h));
        members[d.order - 1].push_back(i);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int g = 0; g < 4; ++g) {
        if (parts[g].empty()) continue;
        auto m = std::make_unique<fr_mesh_s>();
        m->order = g + 1;
        m->system = d0.system;
        m->precision = d0.precision;
        m->flags = d0.flags & ~uint32_t(FR_CHECK_FINITE);
        m->gamma = d0.gamma;
        m->mu = d0.mu;
        m->prandtl = d0.prandtl;
        m->beta = d0.ldg_beta;
        m->tau = d0.ldg_tau;
        m->t_wall = d0.t_wall;
        for (int k = 0; k < 5; ++k) m->farfield[k] = d0.farfield[k];
        m->pref = d0.p_ref;
        std::vector<std::array<int64_t, frh::NTYPE>> off;
        std::string err;
        if (!frh::merge_meshes(parts[g], m->host, off, err)) return bfail(nullptr, FR_ERR_BAD_MESH, err);
        parts[g].clear();
        for (size_t j = 0; j < members[g].size(); ++j)
            for (int t = 0; t < frh::NTYPE; ++t) b->prob[members[g][j]].off[t] = off[j][t];
        m->create_stream = s;
        fr_status st = m->precision != FR_FP64 ? setup_device<float>(m.get(), s) : setup_device<double>(m.get(), s);
        if (!st) st = m->precision != FR_FP64 ? batch_alloc_dt<float>(m.get()) : batch_alloc_dt<double>(m.get());
        if (st) return bfail(nullptr, st, m->err);
        m->device = true;
        std::string rep;
        st = m->precision != FR_FP64 ? autotune_impl<float>(m.get(), s, rep) : autotune_impl<double>(m.get(), s, rep);
        if (st) return bfail(nullptr, st, m->err);
        b->group[g] = std::move(m);
    }
    FR_BHIP(nullptr, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    FR_BHIP(nullptr, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    FR_BHIP(nullptr, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    *out = b.release();
    return FR_OK;
}

fr_status fr_batch_destroy(fr_batch b) {
    if (!b) return FR_OK;
    for (auto &g : b->group)
        if (g) (void)hipStreamSynchronize(g->create_stream);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
    return FR_OK;
}

fr_status fr_batch_query(fr_batch b, int32_t problem, int32_t etype, int64_t *n_elem, int32_t *n_upts,
                         int64_t *ld) {
    if (!b) return FR_ERR_INVALID_ARG;
    if (problem < 0 || problem >= b->n || etype < 0 || etype >= frh::NTYPE)
        return bfail(b, FR_ERR_INVALID_ARG, "problem or element type out of range");
    const auto &P = b->prob[problem];
    if (n_elem) *n_elem = P.ne[etype];
    if (n_upts) *n_upts = P.nu[etype];
    if (ld) *ld = P.ld[etype];
    return FR_OK;
}

static fr_status batch_copy(fr_batch b, int problem, int etype, void *dst, const void *src, bool to_reg,
                            hipStream_t s) {
    if (!b) return FR_ERR_INVALID_ARG;
    if (problem < 0 || problem >= b->n || etype < 0 || etype >= frh::NTYPE)
        return bfail(b, FR_ERR_INVALID_ARG, "problem or element type out of range");
    const auto &P = b->prob[problem];
    if (!P.ne[etype]) return FR_OK;
    if (!(to_reg ? src : dst)) return bfail(b, FR_ERR_INVALID_ARG, "null state");
    fr_mesh m = b->group[P.g].get();
    const size_t esz = m->precision != FR_FP64 ? 4 : 8;
    char *reg = static_cast<char *>(m->precision != FR_FP64 ? group_reg<float>(m, etype) : group_reg<double>(m, etype));
    const size_t gpitch = size_t(m->host.t[etype].ld) * esz, ppitch = size_t(P.ld[etype]) * esz;
    char *greg = reg + size_t(P.off[etype]) * esz;
    const size_t rows = size_t(P.nu[etype]) * 5, width = size_t(P.ne[etype]) * esz;
    if (to_reg)
        FR_BHIP(b, hipMemcpy2DAsync(greg, gpitch, src, ppitch, width, rows, hipMemcpyDeviceToDevice, s));
    else
        FR_BHIP(b, hipMemcpy2DAsync(dst, ppitch, greg, gpitch, width, rows, hipMemcpyDeviceToDevice, s));
    return FR_OK;
}

fr_status fr_batch_upts_coords(fr_batch b, int32_t problem, int32_t etype, double *xyz) {
    if (!b || !xyz) return FR_ERR_INVALID_ARG;
    if (problem < 0 || problem >= b->n || etype < 0 || etype >= frh::NTYPE)
        return bfail(b, FR_ERR_INVALID_ARG, "problem or element type out of range");
    const auto &P = b->prob[problem];
    if (!P.ne[etype]) return FR_OK;
    const frh::TypeHost &H = b->group[P.g]->host.t[etype];
    const int nu = H.ops.nu;
    for (int i = 0; i < nu; ++i)
        for (int64_t e = 0; e < P.ne[etype]; ++e) {
            double x[3];
            frh::elem_point_at(H, etype, P.off[etype] + e, false, i, x);
            for (int d = 0; d < 3; ++d) xyz[(size_t(i) * 3 + d) * P.ne[etype] + e] = x[d];
        }
    return FR_OK;
}

fr_status fr_batch_set_solution(fr_batch b, int32_t problem, int32_t etype, const void *u_dev, void *stream) {
    return batch_copy(b, problem, etype, nullptr, u_dev, true, static_cast<hipStream_t>(stream));
}

fr_status fr_batch_get_solution(fr_batch b, int32_t problem, int32_t etype, void *u_dev, void *stream) {
    return batch_copy(b, problem, etype, u_dev, nullptr, false, static_cast<hipStream_t>(stream));
}

fr_status fr_batch_set_dt(fr_batch b, const double *dt_host, void *stream) {
    if (!b || !dt_host) return FR_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int g = 0; g < 4; ++g) {
        fr_mesh m = b->group[g].get();
        if (!m) continue;
        for (int t = 0; t < frh::NTYPE; ++t) {
            const int64_t ld = m->host.t[t].ld;
            if (!ld) continue;
            std::vector<double> h(size_t(ld), 0.0);
            for (int i = 0; i < b->n; ++i) {
                const auto &P = b->prob[i];
                if (P.g != g) continue;
                if (!(dt_host[i] >= 0) || !std::isfinite(dt_host[i]))
                    return bfail(b, FR_ERR_INVALID_ARG, "dt of problem " + std::to_string(i));
                for (int64_t e = 0; e < P.ne[t]; ++e) h[size_t(P.off[t] + e)] = dt_host[i];
            }
            if (m->precision != FR_FP64) {
                std::vector<float> f(h.begin(), h.end());
                FR_BHIP(b, hipMemcpyAsync(group_dte<float>(m, t), f.data(), f.size() * 4, hipMemcpyHostToDevice, s));
                FR_BHIP(b, hipStreamSynchronize(s));
            } else {
                FR_BHIP(b, hipMemcpyAsync(group_dte<double>(m, t), h.data(), h.size() * 8, hipMemcpyHostToDevice, s));
                FR_BHIP(b, hipStreamSynchronize(s));
            }
        }
    }
    return FR_OK;
}

fr_status fr_batch_set_graph(fr_batch b, int32_t enable) {
    if (!b) return FR_ERR_INVALID_ARG;
    b->use_graph = enable != 0;
    return FR_OK;
}

fr_status fr_batch_rk_step(fr_batch b, int32_t scheme, int32_t n_steps, void *stream) {
    if (!b) return FR_ERR_INVALID_ARG;
    if (n_steps < 0) return bfail(b, FR_ERR_INVALID_ARG, "negative step count");
    if (scheme != FR_RK4 && scheme != FR_RK45_2RP && scheme != FR_FWD_EULER)
        return bfail(b, FR_ERR_INVALID_ARG, "unknown scheme");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto step_all = [&](hipStream_t st, int steps) -> fr_status {
        for (int g = 0; g < 4; ++g) {
            fr_mesh m = b->group[g].get();
            if (!m) continue;
            fr_status r = m->precision != FR_FP64 ? rk_impl<float>(m, scheme, 1.0, steps, st, true, false)
                                                  : rk_impl<double>(m, scheme, 1.0, steps, st, true, false);
            if (r) return bfail(b, r, m->err);
        }
        return FR_OK;
    };
    // RK4 swaps its registers every step and cannot be replayed as one graph
    if (!b->use_graph || scheme != FR_RK45_2RP) return step_all(s, n_steps);
    std::vector<const void *> regs;
    for (int g = 0; g < 4; ++g) {
        fr_mesh m = b->group[g].get();
        if (!m) continue;
        for (int t = 0; t < frh::NTYPE; ++t)
            for (int r = 0; r < 3; ++r)
                regs.push_back(m->precision != FR_FP64 ? static_cast<const void *>(dev_of<float>(m).t[t].reg[r])
                                                       : static_cast<const void *>(dev_of<double>(m).t[t].reg[r]));
    }
    if (b->exec && regs != b->graph_regs) {
        // the captured launches still use the previous register order: wait
        // for its replays on the batch stream, then capture again
        FR_BHIP(b, hipStreamSynchronize(b->stream));
        FR_BHIP(b, hipGraphExecDestroy(b->exec));
        FR_BHIP(b, hipGraphDestroy(b->graph));
        b->exec = nullptr;
        b->graph = nullptr;
    }
    if (!b->exec) {
        FR_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        fr_status r = step_all(b->stream, 1);
        hipGraph_t gph = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &gph);
        if (r) {
            if (gph) (void)hipGraphDestroy(gph);
            return r;
        }
        if (e != hipSuccess) return bfail(b, FR_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        b->graph = gph;
        FR_BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_regs = regs;
    }
    FR_BHIP(b, hipEventRecord(b->ev_in, s));
    FR_BHIP(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
    for (int i = 0; i < n_steps; ++i) FR_BHIP(b, hipGraphLaunch(b->exec, b->stream));
    FR_BHIP(b, hipEventRecord(b->ev_out, b->stream));
    FR_BHIP(b, hipStreamWaitEvent(s, b->ev_out, 0));
    return FR_OK;
}

const char *fr_batch_last_error(fr_batch b) { return b ? b->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

struct fr_mlp_s {
    float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *partial = nullptr;
    uint16_t *params_bf16 = nullptr;
    int step = 0;
    std::string err;
    std::vector<void *> allocs;
    ~fr_mlp_s() {
        for (void *p : allocs) (void)hipFree(p);
    }
};

namespace {
fr_status mfail(fr_mlp n, fr_status st, const std::string &msg) {
    if (n)
        n->err = msg;
    else
        g_create_error = msg;
    return st;
}
#define FR_MHIP(n, call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return mfail(n, e_ == hipErrorOutOfMemory ? FR_ERR_OUT_OF_MEMORY : FR_ERR_DEVICE, \
                         std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

// Host-side FP32 upload into a fresh device allocation owned by `allocs`.
template <typename V>
hipError_t upload_vec(std::vector<void *> &allocs, const std::vector<V> &h, V *&dst) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(h.size(), 1) * sizeof(V));
    if (e != hipSuccess) return e;
    allocs.push_back(p);
    dst = static_cast<V *>(p);
    return h.empty() ? hipSuccess : hipMemcpy(p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice);
}
}  // namespace

extern "C" {

fr_status fr_mlp_create(uint64_t seed, fr_mlp *out) {
    if (!out) return FR_ERR_INVALID_ARG;
    *out = nullptr;
    auto n = std::make_unique<fr_mlp_s>();
    const int np = frd::MLP_NPARAM;
    // Glorot-style init from a 64-bit LCG + Box-Muller (seeded, portable)
    std::vector<float> p(np, 0.0f);
    uint64_t st = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto unif = [&]() {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        return (double((st >> 11) & ((1ULL << 53) - 1)) + 0.5) / double(1ULL << 53);
    };
    auto normal = [&]() { return std::sqrt(-2.0 * std::log(unif())) * std::cos(6.283185307179586 * unif()); };
    const int H = frd::MLP_H, I = frd::MLP_IN, O = frd::MLP_OUT;
    int o = 0;
    for (int i = 0; i < H * I; ++i) p[o++] = float(normal() * std::sqrt(1.0 / I));
    o += H;
    for (int i = 0; i < H * H; ++i) p[o++] = float(normal() * std::sqrt(1.0 / H));
    o += H;
    for (int i = 0; i < O * H; ++i) p[o++] = float(0.1 * normal() * std::sqrt(1.0 / H));
    std::vector<float> z(np + 1, 0.0f);
    FR_MHIP(nullptr, upload_vec(n->allocs, p, n->params));
    FR_MHIP(nullptr, upload_vec(n->allocs, z, n->grad));
    FR_MHIP(nullptr, upload_vec(n->allocs, z, n->m));
    FR_MHIP(nullptr, upload_vec(n->allocs, z, n->v));
    std::vector<uint16_t> zb(np, 0);
    FR_MHIP(nullptr, upload_vec(n->allocs, zb, n->params_bf16));
    std::vector<float> part(size_t(frd::MLP_GRAD_BLOCKS) * (np + 1), 0.0f);
    FR_MHIP(nullptr, upload_vec(n->allocs, part, n->partial));
    FR_MHIP(nullptr, frd::launch_to_bf16(n->params, n->params_bf16, nullptr));
    FR_MHIP(nullptr, hipDeviceSynchronize());
    *out = n.release();
    return FR_OK;
}

fr_status fr_mlp_destroy(fr_mlp n) {
    if (n) (void)hipDeviceSynchronize();
    delete n;
    return FR_OK;
}

fr_status fr_mlp_set_params(fr_mlp n, const float *host) {
    if (!n || !host) return FR_ERR_INVALID_ARG;
    FR_MHIP(n, hipMemcpy(n->params, host, frd::MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
    FR_MHIP(n, frd::launch_to_bf16(n->params, n->params_bf16, nullptr));
    FR_MHIP(n, hipDeviceSynchronize());
    n->step = 0;
    return FR_OK;
}

fr_status fr_mlp_get_params(fr_mlp n, float *host) {
    if (!n || !host) return FR_ERR_INVALID_ARG;
    FR_MHIP(n, hipMemcpy(host, n->params, frd::MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    return FR_OK;
}

fr_status fr_mlp_forward(fr_mlp n, const float *x, int64_t count, const float *stats, float *y,
                         int32_t bf16_weights, void *stream) {
    if (!n || !x || !y || count < 0) return FR_ERR_INVALID_ARG;
    FR_MHIP(n, frd::launch_mlp_forward(n->params, n->params_bf16, bf16_weights != 0, x, frd::MLP_IN, 1, count,
                                       stats, true, y, frd::MLP_OUT, 1,
                                       static_cast<hipStream_t>(stream)));
    return FR_OK;
}

fr_status fr_mlp_grad(fr_mlp n, const float *x, const float *target, const int32_t *idx, int64_t count,
                      const float *stats, double *loss_host, void *stream) {
    if (!n || !x || !target || count <= 0) return FR_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FR_MHIP(n, frd::launch_mlp_grad(n->params, x, target, idx, count, stats, n->partial, frd::MLP_GRAD_BLOCKS,
                                    n->grad, s));
    if (loss_host) {
        float l = 0;
        FR_MHIP(n, hipMemcpyAsync(&l, n->grad + frd::MLP_NPARAM, sizeof(float), hipMemcpyDeviceToHost, s));
        FR_MHIP(n, hipStreamSynchronize(s));
        *loss_host = l;
    }
    return FR_OK;
}

fr_status fr_mlp_get_grad(fr_mlp n, float *host, void *stream) {
    if (!n || !host) return FR_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FR_MHIP(n, hipMemcpyAsync(host, n->grad, frd::MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    FR_MHIP(n, hipStreamSynchronize(s));
    return FR_OK;
}

fr_status fr_mlp_adam(fr_mlp n, float lr, void *stream) {
    if (!n || !(lr >= 0)) return FR_ERR_INVALID_ARG;
    n->step += 1;
    FR_MHIP(n, frd::launch_adam(n->params, n->grad, n->m, n->v, lr, 0.9f, 0.999f, 1e-8f, n->step,
                                n->params_bf16, static_cast<hipStream_t>(stream)));
    return FR_OK;
}

const char *fr_mlp_last_error(fr_mlp n) { return n ? n->err.c_str() : g_create_error.c_str(); }

fr_status fr_project(fr_mesh src, const void *const u_src[FR_NTYPES], fr_mesh dst, void *const u_dst[FR_NTYPES],
                     void *stream) {
    if (fr_status st = check_mesh(src, 0, true)) return st;
    if (fr_status st = check_mesh(dst, 0, true)) return st;
    if ((src->precision == FR_FP64) != (dst->precision == FR_FP64))
        return fail(src, FR_ERR_INVALID_ARG, "projection between meshes of different scalar types");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int t = 0; t < frh::NTYPE; ++t) {
        const int64_t ne = src->host.t[t].nelem;
        if (ne != dst->host.t[t].nelem) return fail(src, FR_ERR_INVALID_ARG, "meshes differ in element counts");
        if (!ne) continue;
        if (!u_src || !u_dst || !u_src[t] || !u_dst[t]) return fail(src, FR_ERR_INVALID_ARG, "null state");
        const int M = frh::n_upts(t, dst->order), K = frh::n_upts(t, src->order);
        const int64_t w5 = 5 * src->host.t[t].ld;
        const int key = 16 * t + dst->order;
        if (src->precision != FR_FP64) {
            auto it = src->proj_f.find(key);
            if (it == src->proj_f.end()) {
                std::vector<float> f;
                frd::Op<float> op = fragment<float>(frh::build_projection(t, src->order, dst->order), M, K, f);
                float *p;
                FR_HIP(src, upload_vec(dev_of<float>(src).allocs, f, p));
                op.frag = p;
                it = src->proj_f.emplace(key, op).first;
            }
            FR_HIP(src, frd::launch_opmul<float>(4 * t, it->second, static_cast<const float *>(u_src[t]), w5, K,
                                                 nullptr, 0, 0, static_cast<float *>(u_dst[t]), w5, w5, s));
        } else {
            auto it = src->proj_d.find(key);
            if (it == src->proj_d.end()) {
                std::vector<double> f;
                frd::Op<double> op = fragment<double>(frh::build_projection(t, src->order, dst->order), M, K, f);
                double *p;
                FR_HIP(src, upload_vec(dev_of<double>(src).allocs, f, p));
                op.frag = p;
                it = src->proj_d.emplace(key, op).first;
            }
            FR_HIP(src, frd::launch_opmul<double>(4 * t, it->second, static_cast<const double *>(u_src[t]), w5, K,
                                                  nullptr, 0, 0, static_cast<double *>(u_dst[t]), w5, w5, s));
        }
    }
    return FR_OK;
}

}  // extern "C"

namespace {
fr_status closure_tables(fr_mesh m) {
    if (m->host.t[2].nelem)
        return fail(m, FR_ERR_UNSUPPORTED, "the closure is defined on tet and prism meshes only");
    if (m->closure) return FR_OK;
    auto c = std::make_unique<Closure>();
    const int64_t ntot = m->host.t[0].nelem + m->host.t[1].nelem;
    std::vector<int32_t> nb = frh::face_neighbours(m->host);
    FR_HIP(m, upload_vec(c->allocs, nb, c->nb));
    std::vector<float> z(size_t(ntot) * 20, 0.0f), zf(size_t(ntot) * frd::MLP_IN, 0.0f);
    FR_HIP(m, upload_vec(c->allocs, z, c->mom));
    FR_HIP(m, upload_vec(c->allocs, z, c->y));
    FR_HIP(m, upload_vec(c->allocs, zf, c->feat));
    for (int t = 0; t < 2; ++t) {   // tets and prisms (hexahedra refused above)
        if (!m->host.t[t].nelem) continue;
        const std::vector<double> Mo = frh::build_moments(t, m->order), Li = frh::build_lift(t, m->order);
        FR_HIP(m, upload_vec(c->allocs, std::vector<float>(Mo.begin(), Mo.end()), c->Mom[t]));
        FR_HIP(m, upload_vec(c->allocs, std::vector<float>(Li.begin(), Li.end()), c->lift[t]));
    }
    c->params = nullptr;
    m->closure = std::move(c);
    return FR_OK;
}

template <typename T>
fr_status closure_moments_impl(fr_mesh m, const void *const u[FR_NTYPES], const void *const b[FR_NTYPES], float *mom,
                               int64_t rs, int64_t cs, const float *ystats, hipStream_t s) {
    Dev<T> &d = dev_of<T>(m);
    for (int t = 0; t < 2; ++t) {   // tets and prisms (hexahedra refused by closure_tables)
        if (!d.t[t].nelem) continue;
        if (!u || !u[t] || (b && !b[t])) return fail(m, FR_ERR_INVALID_ARG, "null state");
        FR_HIP(m, frd::launch_moments<T>(static_cast<const T *>(u[t]), b ? static_cast<const T *>(b[t]) : nullptr,
                                         d.t[t].ld, d.t[t].nelem, d.t[t].nu, m->closure->Mom[t], mom,
                                         t ? d.t[0].nelem : 0, rs, cs, ystats, s));
    }
    return FR_OK;
}

}  // namespace

extern "C" {

fr_status fr_closure_moments(fr_mesh m, const void *const u[FR_NTYPES], float *mom, void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!mom) return fail(m, FR_ERR_INVALID_ARG, "null output");
    if (fr_status st = closure_tables(m)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->precision != FR_FP64 ? closure_moments_impl<float>(m, u, nullptr, mom, 20, 1, nullptr, s)
                                   : closure_moments_impl<double>(m, u, nullptr, mom, 20, 1, nullptr, s);
}

fr_status fr_closure_targets(fr_mesh m, const void *const a[FR_NTYPES], const void *const b[FR_NTYPES],
                             const float *stats,
                             float *out, void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!out || !b) return fail(m, FR_ERR_INVALID_ARG, "null argument");
    if (fr_status st = closure_tables(m)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float *ys = stats ? stats + 2 * frd::MLP_IN : nullptr;
    return m->precision != FR_FP64 ? closure_moments_impl<float>(m, a, b, out, 20, 1, ys, s)
                                   : closure_moments_impl<double>(m, a, b, out, 20, 1, ys, s);
}

fr_status fr_closure_features(fr_mesh m, const void *const u[FR_NTYPES], const float *stats, float *feat,
                              void *stream) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!feat) return fail(m, FR_ERR_INVALID_ARG, "null output");
    if (fr_status st = closure_tables(m)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t ntot = m->host.t[0].nelem + m->host.t[1].nelem;
    fr_status st = m->precision != FR_FP64
                       ? closure_moments_impl<float>(m, u, nullptr, m->closure->mom, 1, ntot, nullptr, s)
                       : closure_moments_impl<double>(m, u, nullptr, m->closure->mom, 1, ntot, nullptr, s);
    if (st) return st;
    FR_HIP(m, frd::launch_features(m->closure->mom, 1, ntot, m->closure->nb, ntot, stats, feat, frd::MLP_IN, 1, s));
    return FR_OK;
}

fr_status fr_closure_attach(fr_mesh m, fr_mlp net, const float *stats, int32_t bf16_weights) {
    if (fr_status st = check_mesh(m, 0, true)) return st;
    if (!net) {
        if (m->closure) m->closure->params = nullptr;
        m->closure.reset();
        return FR_OK;
    }
    if (!stats) return fail(m, FR_ERR_INVALID_ARG, "normalisation statistics are required");
    if (fr_status st = closure_tables(m)) return st;
    m->closure->params = net->params;
    m->closure->params_bf16 = net->params_bf16;
    m->closure->stats = stats;
    m->closure->bf16 = bf16_weights != 0;
    return FR_OK;
}

const char *fr_last_error(fr_mesh m) {
    return m ? m->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
