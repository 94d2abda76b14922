// Device kernels of the FR library: argument blocks and launchers.
// Internal header (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace frd {

constexpr int NVAR = 5;
constexpr int NTYPE = 3;   // 0 tet, 1 prism, 2 hexahedron

// Fragment-ordered operator for the MFMA product kernel: element
// [mb][kb][lane] holds A[16 mb + lane % 16][4 kb + lane / 16], zero padded to
// nmg * mbw row blocks of 16 (nmg row groups of mbw blocks, one wavefront per
// row group and column panel) and to Kb * 4 columns, Kb even.
template <typename T>
struct Op {
    const T *frag = nullptr;
    int M = 0, Kb = 0, nmg = 0, mbw = 0;
    // 0 / 3 = every wavefront streams its B panel itself with 2 / 4 K steps
    // of loads in flight; 1 / 2 (FP32 only) = the row groups of a panel share
    // B staged through LDS in chunks of 4 / 8 K steps (nmg <= 8); 4 (FP32
    // only) = the row group's A slice sits in LDS, shared by four panels
    // (fragments grouped by four K steps, mbw * Kb * 256 bytes <= 64 KiB).
    // Kb is a multiple of 2, 4, 8, 4, 8 respectively.  5 = like 0, but each
    // row group walks only the K steps where one of its fragments is nonzero:
    // klist[koff[g] .. koff[g+1]) lists them (padded to an even count with
    // zero fragments), and frag holds the group's fragments compacted in that
    // order, [step][mbw][lane] (mbw <= 4).  6 = 5 with 4 steps of loads in
    // flight instead of 2 (lists padded to a multiple of 4).  The rows are
    // permuted so that
    // rows touching the same columns share a group: fragment row r' is
    // operator row rowmap[r'] (-1 for padding).  All variants give identical
    // bits for finite B (skipped products are exact zeros).
    int stage = 0;
    const int32_t *klist = nullptr, *koff = nullptr, *rowmap = nullptr;
};

// Row grouping of an M-row operator: at most `cap` blocks of 16 rows per
// wavefront, as few groups as possible, blocks spread evenly.
inline void row_groups(int M, int cap, int &nmg, int &mbw) {
    const int Mb = (M + 15) / 16;
    nmg = (Mb + cap - 1) / cap;
    mbw = (Mb + nmg - 1) / nmg;
}

// C[M][ncols] = A[M][K1 + K2] . [B1 (K1 rows); B2 (K2 rows)], row strides
// ldb1, ldb2, ldc (elements); ncols a multiple of 64.  tag = 4 * element type +
// operator (0 interpolation, 1 gradient, 2 gradient interpolation, 3
// divergence), 0..11, names the kernel instantiation.
// With ep (fuse set; divergence only) the product's output goes through the
// last pipeline step (negdivconf_kernel's update) instead of into C.
enum { OP_INTERP = 0, OP_GRAD = 1, OP_GRADINTERP = 2, OP_DIV = 3 };
template <typename T>
struct NegArgs;
template <typename T>
hipError_t launch_opmul(int tag, const Op<T> &A, const T *B1, int64_t ldb1, int K1, const T *B2,
                        int64_t ldb2, int K2, T *C, int64_t ldc, int64_t ncols, hipStream_t s,
                        const NegArgs<T> *ep = nullptr);

// Split-precision operator for the 16-bit MFMA product kernel.  BF16
// (format 1): A = h + m + l, three parts; FP16 (format 2): A = h + l / 2^11,
// two parts.  Fragment element [mb][kb][lane][j] of each part =
// part[16 mb + lane % 16][32 kb + 8 (lane / 16) + j], zero padded to
// nmg * mbw row blocks and Kb (even) steps of 32 columns.
struct OpSplit {
    const uint16_t *part[3] = {nullptr, nullptr, nullptr};
    int M = 0, Kb = 0, nmg = 0, mbw = 0, format = 1;
    float inv_scale = 1.0f;
    // 0 = every wavefront splits its B panel itself; 1 = the row groups of a
    // panel (nmg <= 8, nmg * parts * 4 KiB <= 64 KiB) share the split B
    // through LDS.  Both give identical bits.
    int stage = 0;
};
// C = A [B1; B2] with the FP32 state B split on the fly into 16-bit parts
// like A, products of the leading part pairs on the matrix cores, FP32
// accumulation (six products for BF16, three for FP16).
hipError_t launch_opmul_split(int tag, const OpSplit &A, const float *B1, int64_t ldb1, int K1,
                              const float *B2, int64_t ldb2, int K2, float *C, int64_t ldc,
                              int64_t ncols, hipStream_t s, const NegArgs<float> *ep = nullptr);

// Point-wise work at the solution points of one element type (ETYPE 0 tet,
// 1 prism, 2 hexahedron): physical gradient Q from the reference gradient Qt
// (NS) and the transformed flux Ft = adj (F_inv - F_vis).
template <typename T>
struct UptsArgs {
    const T *U;        // [nu][5][ld]
    const T *Qt;       // [3 nu][5][ld] reference gradient (NS)
    T *Q;              // [nu][15][ld] physical gradient, index j*5+v (NS)
    T *Ft;             // [3 nu][5][ld] transformed flux, row k*nu+i
    const T *geom;     // [ng][ld] Jacobian coefficients
    const T *xi;       // [nu][3] reference coordinates of the solution points
    int64_t ld, nelem;
    int nu;
    T gamma, mu, prandtl;
    // curved elements: adjugate [9][nu][ld] (entry 3k + j = J dxi_k/dx_j)
    // and 1 / J [nu][ld] per point, used instead of geom when padj is set
    const T *padj = nullptr, *pjinv = nullptr;
    T pref = 0;        // reference pressure left out of the momentum flux
};
template <typename T>
hipError_t launch_upts(int etype, bool ns, const UptsArgs<T> &a, hipStream_t s);

// Fused gradient stage of one element type (Navier-Stokes; tets and prisms):
// per tile of elements (all five fields), the corrected gradient product
// Qt = [G_k | L_k] [U; Cf], the point-wise work (Q = adj^T Qt / J, Ft) and the
// gradient interpolation Qf = M0 Q, with Qt and Q held in LDS.  Gives the
// bits of the separate kernels (same operator fragments, same K order, same
// point-wise arithmetic).
template <typename T>
struct GradFluxArgs {
    const T *U;          // [nu][5][ld]
    const T *Cf;         // [nf][5][ld] jump to the common solution
    T *Ft;               // [3 nu][5][ld] transformed flux, row k nu + i
    T *Qf;               // [nf][15][ld] physical gradient at the flux points
    const T *geom;       // [ng][ld] Jacobian coefficients (straight elements)
    const T *xi;         // [nu][3]
    const T *padj = nullptr, *pjinv = nullptr;   // curved: [9][nu][ld], [nu][ld]
    int64_t ld = 0, nelem = 0;
    int nu = 0, nf = 0;
    T gamma = 0, mu = 0, prandtl = 0, pref = 0;
    Op<T> G;             // [G_k | L_k], 3 nu x (nu + nf): step lists, one row block per group (stage 6)
    Op<T> M;             // M0, nf x nu: step lists, one row block per group (stage 6)
    // Qf is written at the flux point of row slot s of M for element e only
    // where qmask[e] & fbit[s] (the faces whose gradient an interface or
    // boundary kernel reads); every point when qmask is null
    const uint8_t *qmask = nullptr;   // [ld]
    const uint8_t *fbit = nullptr;    // [16 M.nmg] 1 << local face of the row's flux point
};
// LDS bytes of one workgroup of the fused kernel (0: shape not supported).
template <typename T>
size_t gradflux_lds(int etype, const GradFluxArgs<T> &a);
// stream: the streaming form (FP32 only), a workgroup per run of tiles with
// the next tile's input loaded straight into LDS while one is computed.
template <typename T>
hipError_t launch_gradflux(int etype, const GradFluxArgs<T> &a, hipStream_t s, bool stream = false);

// Interface work on the paired flux points.
template <typename T>
struct PairArgs {
    const uint32_t *sideL, *sideR;   // elem | fpt << 22 | type << 30
    const T *geo;                    // [5][npairs]: nx, ny, nz, sL, sR
    int64_t npairs;
    const T *Uf[NTYPE];              // [nf][5][ld]
    const T *Qf[NTYPE];              // [nf][15][ld]
    T *Cf[NTYPE];                    // [nf][5][ld]
    T *Fn[NTYPE];                    // [nf][5][ld]
    int64_t ld[NTYPE];
    T gamma, mu, prandtl, beta, tau;
    T pref = 0;                      // reference pressure left out of the momentum flux
};
template <typename T>
hipError_t launch_common_solution(const PairArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_common_flux(bool ns, const PairArgs<T> &a, hipStream_t s);

// Boundary flux points (no-slip isothermal wall, kind 1; Riemann-invariant
// far field, kind 2), imposed weakly: a boundary state Ub (the LDG common
// solution and the state of the viscous flux) and a ghost state (the right
// state of the Rusanov flux) from the interior trace.
template <typename T>
struct BndArgs {
    const uint32_t *side;            // elem | fpt << 22 | type << 30
    const T *geo;                    // [4][nb]: nx, ny, nz (outward unit normal), s
    const int8_t *kind;              // [nb]
    int64_t nb;
    const T *Uf[NTYPE];
    const T *Qf[NTYPE];
    T *Cf[NTYPE];
    T *Fn[NTYPE];
    int64_t ld[NTYPE];
    T gamma, mu, prandtl, tau;
    T t_wall;                        // wall temperature p / rho
    T free[5];                       // free stream rho, u, v, w, p
    T pref = 0;                      // reference pressure left out of the momentum flux
};
// Cf = Ub - U_f at each boundary point (NS).
template <typename T>
hipError_t launch_boundary_solution(const BndArgs<T> &a, hipStream_t s);
// Fn = s [Rusanov(U_f, ghost; n) (- Fv(Ub, Q_f).n + tau (U_f - Ub))].
template <typename T>
hipError_t launch_boundary_flux(bool ns, const BndArgs<T> &a, hipStream_t s);

// k = -Rt / J at each solution point (times dte[e] if given), then
//   acc += a k (if acc), out = (base ? base : (acc ? acc : 0)) + b k (if out).
template <typename T>
struct NegArgs {
    const T *Rt;
    T *out;
    T *acc;
    const T *base;
    T a, b;
    const T *jinv;     // [nu][ld] 1 / J
    int64_t ld, nelem;
    int nu;
    const T *dte;      // per-element step size, or null
    // learned closure: k += sum_a lift[i][a] y[(v * 4 + a) * cys + goff + e]
    const float *cy = nullptr;
    int64_t cys = 0;
    // embedded error register of the adaptive RK45[2R+]: err = (stage 0 ? 0 : err) + c k
    T *err = nullptr;
    T c = 0;
    bool err_set = false;
    const float *clift = nullptr;   // [nu][4]
    int64_t goff = 0;
    // set: applied in the divergence product's store (Rt unused)
    bool fuse = false;
};
template <typename T>
hipError_t launch_negdivconf(int etype, const NegArgs<T> &a, hipStream_t s);

// FP64 reductions: per-block partial sums of nq quantities over one type,
// written to partial[block][nq]; a second pass sums the blocks in order.
template <typename T>
struct RedArgs {
    const T *U;          // [nu][5][ld]
    const T *R;          // [nu][5][ld] or null
    const double *wJ;    // [nu][ld]
    int64_t ld, nelem;
    int nu, what;
    double *partial;     // [nblocks][8]
    // what 6 (error norm): sum (R / (atol + rtol max(|U0|, |U|)))^2
    const T *U0 = nullptr;
    double atol = 0, rtol = 0;
};
constexpr int RED_BLOCKS = 512;
template <typename T>
hipError_t launch_reduce(const RedArgs<T> &a, hipStream_t s);
hipError_t launch_reduce_final(const double *partial, int nblocks, double *out, hipStream_t s);

// Learned closure (fr_closure.hip).
constexpr int MLP_IN = 120, MLP_H = 64, MLP_OUT = 20;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;
constexpr int MLP_NSTATS = 2 * MLP_IN + 2 * MLP_OUT;   // mu_x, s_x, mu_y, s_y
constexpr int MLP_GRAD_BLOCKS = 256;
template <typename T>
hipError_t launch_moments(const T *U, const T *B, int64_t ld, int64_t nelem, int nu, const float *Mom,
                          float *mom, int64_t goff, int64_t rs, int64_t cs, const float *ystats,
                          hipStream_t s);
hipError_t launch_features(const float *mom, int64_t rs, int64_t cs, const int32_t *nb, int64_t ntot,
                           const float *stats, float *feat, int64_t frs, int64_t fcs, hipStream_t s);
hipError_t launch_mlp_forward(const float *P, const uint16_t *Pb, bool bf16, const float *X, int64_t xrs,
                              int64_t xcs, int64_t n, const float *stats, bool norm_in, float *Y, int64_t yrs,
                              int64_t ycs, hipStream_t s);
hipError_t launch_mlp_grad(const float *P, const float *X, const float *Tg, const int32_t *idx, int64_t n,
                           const float *stats, float *partial, int nblk, float *grad, hipStream_t s);
hipError_t launch_adam(float *P, const float *G, float *M, float *V, float lr, float b1, float b2, float eps,
                       int t, uint16_t *Pb, hipStream_t s);
hipError_t launch_to_bf16(const float *P, uint16_t *Pb, hipStream_t s);

template <typename T>
hipError_t launch_copy(T *dst, const T *src, int64_t n, hipStream_t s);

}  // namespace frd
