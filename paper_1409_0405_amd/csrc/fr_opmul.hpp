// Operator-product kernels of the FR right-hand side (gfx950 matrix cores)
// and their per-instantiation launchers.  Included by the translation units
// that instantiate them (one per element type and precision, so that they
// compile in parallel) and by fr_kernels.hip, which dispatches on the tag.
//
// Paper, Section 2.1: the products C <- A B of a small constant operator A
// with very wide row-major state matrices B.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "fr_device.hpp"

namespace frd {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = floatx4;
};
template <>
struct Vec4<double> {
    using type = doublex4;
};

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16 x 16 result held in accumulator element r of lane group g
// (lanes 16 g .. 16 g + 15 hold columns 0..15).  Both instructions take A as
// A[lane % 16][lane / 16] and B as B[lane / 16][lane % 16]; the FP32 result
// holds four consecutive rows per lane group, the FP64 result rows strided
// by four.
template <typename T>
__device__ __forceinline__ int acc_row(int g, int r);
template <>
__device__ __forceinline__ int acc_row<float>(int g, int r) { return 4 * g + r; }
template <>
__device__ __forceinline__ int acc_row<double>(int g, int r) { return g + 4 * r; }

// Returns x unchanged, but opaque to the optimiser: used on the values that
// enter a software-pipelined loop, so that the loop-carried registers are not
// all plain loads (otherwise the loads of the next K step get merged into
// one load at the loop head, right before their use, and every step waits
// for memory).
template <typename V>
__device__ __forceinline__ V opaque(V x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  The
// operator products renumber them so that every XCD runs one contiguous range
// of logical workgroups (the grid is a multiple of 8): the row groups of a
// 64-column panel, split over neighbouring workgroups, then read the panel of
// B through the same L2 instead of fetching it from HBM once per XCD.
__device__ __forceinline__ unsigned xcd_block() {
    return (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
}
inline unsigned xcd_grid(int64_t nblocks) { return unsigned((nblocks + 7) / 8 * 8); }

// The last pipeline step at one (solution point i, field v, element e), with
// o = (5 i + v) ld + e: k = -r / J (plus the learned closure's lifted
// correction), times the element's step size, into the error, accumulator
// and output registers (frd::NegArgs).  negdivconf_kernel and the fused
// store of the divergence products both call it, so the two give the same
// bits.
template <typename T>
__device__ __forceinline__ void neg_update(const NegArgs<T> &a, int i, int v, int64_t e, int64_t o,
                                           T r) {
    const T Jinv = a.jinv[int64_t(i) * a.ld + e];
    const T sc = a.dte ? a.dte[e] : T(1);
    T k = -r * Jinv;
    if (a.cy) {
        const float *y = a.cy + (a.goff + e) + int64_t(v) * 4 * a.cys;
        const float *l = a.clift + i * 4;
        k += T(l[0] * y[0] + l[1] * y[a.cys] + l[2] * y[2 * a.cys] + l[3] * y[3 * a.cys]);
    }
    k *= sc;
    if (a.err) a.err[o] = (a.err_set ? T(0) : a.err[o]) + a.c * k;
    T accv = 0;
    if (a.acc) {
        accv = a.acc[o] + a.a * k;
        a.acc[o] = accv;
    }
    if (a.out) a.out[o] = (a.base ? a.base[o] : accv) + a.b * k;
}

// Store of four consecutive columns of one output row.  For a divergence
// product with ep.fuse set the row is solution point i and the columns are
// (field v, elements e .. e + 3) of the [point][field][ld] layout (ldc = 5
// ld, checked at launch): the values go through neg_update's arithmetic
// instead of being stored, and the padding elements past nelem are skipped.
// The register pointers are 4-element aligned (checked at entry).
template <int TAG, typename T, typename V4>
__device__ __forceinline__ void store_c(T *C, int64_t ldc, int row, int64_t col, const V4 &val,
                                        const NegArgs<T> &ep) {
    if constexpr (TAG % 4 == 3) {
        if (ep.fuse) {
            const int v = int(col / ep.ld);
            const int64_t e0 = col - int64_t(v) * ep.ld;
            const int64_t o0 = int64_t(row) * ldc + col;
            if (e0 + 3 < ep.nelem && !ep.cy) {
                // four whole elements: the same arithmetic as neg_update on
                // 16-byte (FP32) / 32-byte (FP64) loads and stores
                const V4 J = *reinterpret_cast<const V4 *>(ep.jinv + int64_t(row) * ep.ld + e0);
                const V4 S = ep.dte ? *reinterpret_cast<const V4 *>(ep.dte + e0) : V4{1, 1, 1, 1};
                V4 k;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    k[j] = -T(val[j]) * J[j];
                    k[j] *= S[j];
                }
                if (ep.err) {
                    V4 er = ep.err_set ? V4{0, 0, 0, 0} : *reinterpret_cast<const V4 *>(ep.err + o0);
#pragma unroll
                    for (int j = 0; j < 4; ++j) er[j] = er[j] + ep.c * k[j];
                    *reinterpret_cast<V4 *>(ep.err + o0) = er;
                }
                V4 accv = V4{0, 0, 0, 0};
                if (ep.acc) {
                    accv = *reinterpret_cast<const V4 *>(ep.acc + o0);
#pragma unroll
                    for (int j = 0; j < 4; ++j) accv[j] = accv[j] + ep.a * k[j];
                    *reinterpret_cast<V4 *>(ep.acc + o0) = accv;
                }
                if (ep.out) {
                    V4 o = ep.base ? *reinterpret_cast<const V4 *>(ep.base + o0) : accv;
#pragma unroll
                    for (int j = 0; j < 4; ++j) o[j] = o[j] + ep.b * k[j];
                    *reinterpret_cast<V4 *>(ep.out + o0) = o;
                }
                return;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (e0 + j < ep.nelem) neg_update(ep, row, v, e0 + j, o0 + j, T(val[j]));
            return;
        }
    }
    *reinterpret_cast<V4 *>(C + int64_t(row) * ldc + col) = val;
}

// ---------------------------------------------------------------------------
// Operator product C = A [B1; B2] on the matrix cores.  TAG (4 * element type
// + operator id) only names the instantiation, so that a profiler reports each
// operator separately.
//
// One wavefront owns a 64-column panel of C and MBW row blocks of 16.  The 64
// columns are split into four interleaved MFMA column blocks: block n holds
// columns 4 j + n (j = 0..15), so lane l reads the four consecutive columns
// 4 (l % 16) .. +3 of one B row with a single vector load and writes four
// consecutive columns of one C row with a single vector store.  A is read in
// fragment order (one coalesced load per MFMA) from L2-resident memory and is
// zero padded to whole row groups and to an even number of K steps, so the K
// loop is branch free: rows of B past K are clamped to a real row (finite
// values times zero columns of A).
// ---------------------------------------------------------------------------
template <typename T, int MBW, int TAG, int D>
__global__ __launch_bounds__(256) void opmul_kernel(Op<T> A, const T *__restrict__ B1,
                                                    int64_t ldb1, int K1,
                                                    const T *__restrict__ B2, int64_t ldb2,
                                                    int K2, T *__restrict__ C, int64_t ldc,
                                                    int64_t npanels, int nmg, NegArgs<T> ep) {
    using v4 = typename Vec4<T>::type;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t(xcd_block()) * blockDim.x + threadIdx.x) >> 6;
    const int64_t panel = wid / nmg;
    const int mg = int(wid - panel * nmg);
    if (panel >= npanels) return;
    const int mb0 = mg * MBW;
    const int64_t col = panel * 64 + 4 * (lane & 15);
    const int krow = lane >> 4;
    const int K = K1 + K2;
    const int Kb = A.Kb;

    auto bptr = [&](int kb) -> const v4 * {
        const int k = min(4 * kb + krow, K - 1);
        const T *p = k < K1 ? B1 + int64_t(k) * ldb1 : B2 + int64_t(k - K1) * ldb2;
        return reinterpret_cast<const v4 *>(p + col);
    };

    v4 acc[MBW][4];
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = v4{0, 0, 0, 0};

    // D register sets, one per K step in flight (Kb is a multiple of D): set
    // d is refilled with step kb + d + D right after its matrix instructions
    // issue, so D steps of loads are outstanding while the others multiply.
    const T *Af = A.frag + size_t(mb0) * Kb * 64 + lane;
    T a[D][MBW];
    v4 b[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        b[d] = opaque(*bptr(d));
#pragma unroll
        for (int m = 0; m < MBW; ++m) a[d][m] = opaque(Af[(size_t(m) * Kb + d) * 64]);
    }
    for (int kb = 0; kb < Kb; kb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
                acc[m][0] = mfma16(a[d][m], b[d][0], acc[m][0]);
                acc[m][1] = mfma16(a[d][m], b[d][1], acc[m][1]);
                acc[m][2] = mfma16(a[d][m], b[d][2], acc[m][2]);
                acc[m][3] = mfma16(a[d][m], b[d][3], acc[m][3]);
            }
            const int kn = min(kb + d + D, Kb - 1);
            b[d] = *bptr(kn);
#pragma unroll
            for (int m = 0; m < MBW; ++m) a[d][m] = Af[(size_t(m) * Kb + kn) * 64];
        }
    }
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (mb0 + m) + acc_row<T>(krow, r);
            if (row < A.M)
                store_c<TAG>(C, ldc, row, col, v4{acc[m][0][r], acc[m][1][r], acc[m][2][r], acc[m][3][r]}, ep);
        }
    }
}

// ---------------------------------------------------------------------------
// Operator product over the nonzero K steps of each row group only.  The
// operators of tensor-product elements are mostly structural zeros (a row of
// a hexahedron's derivative touches one line of points, a prism's in-layer
// derivative one triangle layer), so a row group of MBW x 16 rows needs only
// a fraction of the K steps: the group's step list (shared by the wavefront,
// read through scalar loads) drives the same pipelined loop as opmul_kernel
// with D = 2 or 4 steps in flight (the list is padded with zero fragments to a
// multiple of D), over fragments stored compacted per group.
// Rows are grouped by the columns they touch and written back through a row
// map.  The products left out are exact zeros, so every output keeps the bits
// of the dense kernels.
// ---------------------------------------------------------------------------
template <typename T, int MBW, int TAG, int D>
__global__ __launch_bounds__(256) void opmul_sparse_kernel(Op<T> A, const T *__restrict__ B1,
                                                           int64_t ldb1, int K1,
                                                           const T *__restrict__ B2, int64_t ldb2,
                                                           int K2, T *__restrict__ C, int64_t ldc,
                                                           int64_t npanels, int nmg, NegArgs<T> ep) {
    using v4 = typename Vec4<T>::type;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t(xcd_block()) * blockDim.x + threadIdx.x) >> 6;
    const int64_t panel = wid / nmg;
    const int mg = int(wid - panel * nmg);
    if (panel >= npanels) return;
    const int mb0 = mg * MBW;
    const int64_t col = panel * 64 + 4 * (lane & 15);
    const int krow = lane >> 4;
    const int K = K1 + K2;
    const int s0 = A.koff[mg];
    const int ns = A.koff[mg + 1] - s0;       // a multiple of D, >= D
    const int32_t *__restrict__ kl = A.klist + s0;

    auto bptr = [&](int kb) -> const v4 * {
        const int k = min(4 * kb + krow, K - 1);
        const T *p = k < K1 ? B1 + int64_t(k) * ldb1 : B2 + int64_t(k - K1) * ldb2;
        return reinterpret_cast<const v4 *>(p + col);
    };

    v4 acc[MBW][4];
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = v4{0, 0, 0, 0};

    const T *Af = A.frag + size_t(s0) * MBW * 64 + lane;
    T a[D][MBW];
    v4 b[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        b[d] = opaque(*bptr(kl[d]));
#pragma unroll
        for (int m = 0; m < MBW; ++m) a[d][m] = opaque(Af[(size_t(d) * MBW + m) * 64]);
    }
    for (int st = 0; st < ns; st += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
                acc[m][0] = mfma16(a[d][m], b[d][0], acc[m][0]);
                acc[m][1] = mfma16(a[d][m], b[d][1], acc[m][1]);
                acc[m][2] = mfma16(a[d][m], b[d][2], acc[m][2]);
                acc[m][3] = mfma16(a[d][m], b[d][3], acc[m][3]);
            }
            const int sn = min(st + d + D, ns - 1);
            b[d] = *bptr(kl[sn]);
#pragma unroll
            for (int m = 0; m < MBW; ++m) a[d][m] = Af[(size_t(sn) * MBW + m) * 64];
        }
    }
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = A.rowmap[16 * (mb0 + m) + acc_row<T>(krow, r)];
            if (row >= 0)
                store_c<TAG>(C, ldc, row, col, v4{acc[m][0][r], acc[m][1][r], acc[m][2][r], acc[m][3][r]}, ep);
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 operator product with the B panel staged through LDS.  One workgroup
// per 64-column panel and one wavefront per row group (nmg waves): the group
// loads B cooperatively in chunks of KS K steps (4 KS rows x 64 columns,
// one 16-byte load per thread and row quarter), double buffered, so each B
// element is read from memory once per panel instead of once per row group,
// and the next chunk's loads (and A fragments) are in flight while the
// current chunk is multiplied.  Every output sums the same products in the
// same order as opmul_kernel, so both kernels give identical bits.
// ---------------------------------------------------------------------------
template <int MBW, int TAG, int KS>
__global__ __launch_bounds__(512) void opmul_lds_kernel(Op<float> A, const float *__restrict__ B1,
                                                        int64_t ldb1, int K1,
                                                        const float *__restrict__ B2,
                                                        int64_t ldb2, int K2,
                                                        float *__restrict__ C, int64_t ldc,
                                                        int64_t npanels, NegArgs<float> ep) {
    constexpr int NV = 64 * KS;                 // 16-byte vectors per chunk
    const unsigned blk = xcd_block();
    if (blk >= npanels) return;                 // whole workgroup: padding of the grid
    __shared__ floatx4 Bs[2][NV];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, mg = tid >> 6;
    const int krow = lane >> 4;
    const int64_t col0 = int64_t(blk) * 64;
    const int K = K1 + K2, Kb = A.Kb;
    const int nchunk = Kb / KS;

    floatx4 rv[KS];                             // nthr >= 64: at most KS vectors per thread
    auto gload = [&](int c) {
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int i = tid + j * nthr;
            if (i < NV) {
                const int k = min(4 * KS * c + (i >> 4), K - 1);
                const float *p = k < K1 ? B1 + int64_t(k) * ldb1 : B2 + int64_t(k - K1) * ldb2;
                rv[j] = *reinterpret_cast<const floatx4 *>(p + col0 + 4 * (i & 15));
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int i = tid + j * nthr;
            if (i < NV) Bs[buf][i] = rv[j];
        }
    };
    const float *Af = A.frag + size_t(mg) * MBW * Kb * 64 + lane;
    float ac[MBW][KS], an[MBW][KS];
    auto aload = [&](int c, float (&a)[MBW][KS]) {
#pragma unroll
        for (int m = 0; m < MBW; ++m)
#pragma unroll
            for (int q = 0; q < KS; ++q) a[m][q] = Af[(size_t(m) * Kb + min(KS * c + q, Kb - 1)) * 64];
    };

    floatx4 acc[MBW][4];
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = floatx4{0, 0, 0, 0};

    gload(0);
    aload(0, ac);
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int q = 0; q < KS; ++q) ac[m][q] = opaque(ac[m][q]);
    sstore(0);
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const bool more = c + 1 < nchunk;
        if (more) {
            __builtin_amdgcn_s_setprio(2);
            gload(c + 1);
            aload(c + 1, an);
            __builtin_amdgcn_s_setprio(1);
        }
        const floatx4 *Bc = Bs[c & 1];
        // Kb is a multiple of KS (the fragment is zero padded): no tail test.
        // Issue priority: highest while a wave sends out the next chunk's
        // loads, raised over its matrix instructions, normal otherwise, so
        // the loads leave early and the SIMD keeps feeding the matrix core
        // (measured: 4 % on this kernel; the same in the direct and
        // step-list kernels slows them)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const floatx4 b = Bc[(4 * q + krow) * 16 + (lane & 15)];
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
                acc[m][0] = mfma16(ac[m][q], b[0], acc[m][0]);
                acc[m][1] = mfma16(ac[m][q], b[1], acc[m][1]);
                acc[m][2] = mfma16(ac[m][q], b[2], acc[m][2]);
                acc[m][3] = mfma16(ac[m][q], b[3], acc[m][3]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        if (more) {
            sstore((c + 1) & 1);
#pragma unroll
            for (int m = 0; m < MBW; ++m)
#pragma unroll
                for (int q = 0; q < KS; ++q) ac[m][q] = an[m][q];
        }
        __syncthreads();
    }
    const int64_t col = col0 + 4 * (lane & 15);
    const int mb0 = mg * MBW;
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (mb0 + m) + acc_row<float>(krow, r);
            if (row < A.M)
                store_c<TAG>(C, ldc, row, col, floatx4{acc[m][0][r], acc[m][1][r], acc[m][2][r], acc[m][3][r]}, ep);
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 operator product with the operator slice in LDS.  A workgroup of four
// wavefronts takes four consecutive 64-column panels and one row group; the
// group's A fragments (MBW row blocks x Kb steps) are copied to LDS once and
// read from there by all four (16 bytes per lane and row block for four K
// steps), so the matrix instructions no longer wait on L2 latency for A.  B
// streams from memory as in opmul_kernel, two groups of four K steps in
// flight (Kb is a multiple of 8).  Fragment layout for this variant:
// [mb][Kb / 4][lane][4], element j of lane l = A[16 mb + l % 16][4 (4 q + j) + l / 16].
// Every output sums the same products in the same order as opmul_kernel.
// ---------------------------------------------------------------------------
template <int MBW, int TAG>
__global__ __launch_bounds__(256) void opmul_ldsa_kernel(Op<float> A, const float *__restrict__ B1,
                                                         int64_t ldb1, int K1,
                                                         const float *__restrict__ B2, int64_t ldb2,
                                                         int K2, float *__restrict__ C, int64_t ldc,
                                                         int64_t npanels, int nmg, NegArgs<float> ep) {
    extern __shared__ floatx4 As[];             // [MBW][Kb / 4][64]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int Kb = A.Kb, Kq = Kb / 4;
    const unsigned blk = xcd_block();
    const int mg = int(blk % unsigned(nmg));
    const int64_t panel = int64_t(blk / unsigned(nmg)) * 4 + w;
    const int mb0 = mg * MBW;
    const floatx4 *Ag = reinterpret_cast<const floatx4 *>(A.frag) + size_t(mb0) * Kq * 64;
    for (int i = threadIdx.x; i < MBW * Kq * 64; i += 256) As[i] = Ag[i];
    __syncthreads();
    if (panel >= npanels) return;
    const int64_t col = panel * 64 + 4 * (lane & 15);
    const int krow = lane >> 4;
    const int K = K1 + K2;
    auto bptr = [&](int kb) -> const floatx4 * {
        const int k = min(4 * kb + krow, K - 1);
        const float *p = k < K1 ? B1 + int64_t(k) * ldb1 : B2 + int64_t(k - K1) * ldb2;
        return reinterpret_cast<const floatx4 *>(p + col);
    };
    floatx4 acc[MBW][4];
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = floatx4{0, 0, 0, 0};
    floatx4 b[2][4];
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int q = 0; q < 4; ++q) b[d][q] = opaque(*bptr(4 * d + q));
    for (int g = 0; g < Kq; g += 2) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            floatx4 a[MBW];
#pragma unroll
            for (int m = 0; m < MBW; ++m) a[m] = As[(m * Kq + g + d) * 64 + lane];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int m = 0; m < MBW; ++m) {
                    acc[m][0] = mfma16(a[m][q], b[d][q][0], acc[m][0]);
                    acc[m][1] = mfma16(a[m][q], b[d][q][1], acc[m][1]);
                    acc[m][2] = mfma16(a[m][q], b[d][q][2], acc[m][2]);
                    acc[m][3] = mfma16(a[m][q], b[d][q][3], acc[m][3]);
                }
            const int gn = min(g + d + 2, Kq - 1);
#pragma unroll
            for (int q = 0; q < 4; ++q) b[d][q] = *bptr(4 * gn + q);
        }
    }
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (mb0 + m) + acc_row<float>(krow, r);
            if (row < A.M)
                store_c<TAG>(C, ldc, row, col, floatx4{acc[m][0][r], acc[m][1][r], acc[m][2][r], acc[m][3][r]}, ep);
        }
    }
}

// ---------------------------------------------------------------------------
// Split-precision operator product (16-bit matrix cores, FP32 accumulate).
//
// Same panel / row-group decomposition as opmul_kernel, with the 16x16x32
// BF16 or FP16 instruction: lane l holds row l % 16 of A and column l % 16 of
// a B block with the eight K values 8 (l / 16) .. +7.  Each lane loads eight
// consecutive B rows of its four interleaved columns (eight 16-byte loads)
// and splits every value on the fly:
//  * BF16, three parts (x = h + m + l, each a truncation of the remainder,
//    exact up to the last bits of FP32): six products h.h + h.m + m.h +
//    h.l + m.m + l.h, one accumulator (BF16 has the FP32 exponent range);
//  * FP16, two parts (h = x rounded toward zero, l = (x - h) 2^11): three
//    products h.h + (h.l + l.h) / 2^11, the scaled terms in a second
//    accumulator against FP16 underflow.
// A is split on the host the same way (rounded to nearest).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

template <bool F16>
__device__ __forceinline__ floatx4 mfma16x32(uintx4 a, uintx4 b, floatx4 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                       __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                        __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ unsigned hi16x2(float x0, float x1) {
    return (__builtin_bit_cast(unsigned, x0) >> 16) |
           (__builtin_bit_cast(unsigned, x1) & 0xffff0000u);
}
__device__ __forceinline__ float trunc16(float x) {
    return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, x) & 0xffff0000u);
}

// Parts of two values, packed two per 32-bit word: p[0] = h, p[1] = m or l, p[2] = l.
template <bool F16>
__device__ __forceinline__ void split2(float x0, float x1, unsigned p[F16 ? 2 : 3]) {
    if constexpr (F16) {
        typedef __fp16 half2v __attribute__((ext_vector_type(2)));
        const half2v h = __builtin_amdgcn_cvt_pkrtz(x0, x1);
        const float l0 = (x0 - float(h[0])) * 2048.0f, l1 = (x1 - float(h[1])) * 2048.0f;
        p[0] = __builtin_bit_cast(unsigned, h);
        p[1] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(l0, l1));
    } else {
        const float r0 = x0 - trunc16(x0), r1 = x1 - trunc16(x1);
        const float q0 = r0 - trunc16(r0), q1 = r1 - trunc16(r1);
        p[0] = hi16x2(x0, x1);
        p[1] = hi16x2(r0, r1);
        p[2] = hi16x2(q0, q1);
    }
}

template <int MBW, bool F16, int TAG>
__global__ __launch_bounds__(256) void opmul_split_kernel(OpSplit A, const float *__restrict__ B1,
                                                          int64_t ldb1, int K1,
                                                          const float *__restrict__ B2,
                                                          int64_t ldb2, int K2,
                                                          float *__restrict__ C, int64_t ldc,
                                                          int64_t npanels, int nmg, NegArgs<float> ep) {
    constexpr int NP = F16 ? 2 : 3;       // parts per operand
    constexpr int NACC = F16 ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t(xcd_block()) * blockDim.x + threadIdx.x) >> 6;
    const int64_t panel = wid / nmg;
    const int mg = int(wid - panel * nmg);
    if (panel >= npanels) return;
    const int mb0 = mg * MBW;
    const int64_t col = panel * 64 + 4 * (lane & 15);
    const int g = lane >> 4;
    const int K = K1 + K2;
    const int Kb = A.Kb;

    auto row = [&](int k) -> floatx4 {
        k = min(k, K - 1);
        const float *p = k < K1 ? B1 + int64_t(k) * ldb1 : B2 + int64_t(k - K1) * ldb2;
        return *reinterpret_cast<const floatx4 *>(p + col);
    };

    floatx4 acc[NACC][MBW][4];
#pragma unroll
    for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int m = 0; m < MBW; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[c][m][n] = floatx4{0, 0, 0, 0};

    const uintx4 *Ap[3];
#pragma unroll
    for (int q = 0; q < NP; ++q)
        Ap[q] = reinterpret_cast<const uintx4 *>(A.part[q]) + size_t(mb0) * Kb * 64 + lane;

    // One register set of B rows: it is split into 16-bit parts, then
    // refilled with the next K step while the matrix instructions run.
    floatx4 x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = row(8 * g + j);
    for (int kb = 0; kb < Kb; ++kb) {
        uintx4 b[NP][4];
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned pp[NP];
                split2<F16>(x[2 * q][n], x[2 * q + 1][n], pp);
#pragma unroll
                for (int t = 0; t < NP; ++t) b[t][n][q] = pp[t];
            }
        const int kn = 32 * min(kb + 1, Kb - 1) + 8 * g;
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = row(kn + j);
#pragma unroll
        for (int m = 0; m < MBW; ++m) {
            uintx4 a[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) a[q] = Ap[q][(size_t(m) * Kb + kb) * 64];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                if constexpr (F16) {
                    acc[0][m][n] = mfma16x32<F16>(a[0], b[0][n], acc[0][m][n]);
                    acc[1][m][n] = mfma16x32<F16>(a[0], b[1][n], acc[1][m][n]);
                    acc[1][m][n] = mfma16x32<F16>(a[1], b[0][n], acc[1][m][n]);
                } else {
                    // smallest terms first
                    floatx4 t = mfma16x32<F16>(a[0], b[2][n], acc[0][m][n]);
                    t = mfma16x32<F16>(a[1], b[1][n], t);
                    t = mfma16x32<F16>(a[2], b[0][n], t);
                    t = mfma16x32<F16>(a[0], b[1][n], t);
                    t = mfma16x32<F16>(a[1], b[0][n], t);
                    acc[0][m][n] = mfma16x32<F16>(a[0], b[0][n], t);
                }
            }
        }
    }
    const float is = A.inv_scale;
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rw = 16 * (mb0 + m) + 4 * g + r;
            if (rw < A.M) {
                floatx4 out;
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    out[n] = NACC == 2 ? acc[0][m][n][r] + acc[NACC - 1][m][n][r] * is : acc[0][m][n][r];
                store_c<TAG>(C, ldc, rw, col, out, ep);
            }
        }
    }
}

// Split-precision product with the split B shared through LDS.  One
// workgroup per 64-column panel and one wavefront per row group (nmg waves).
// K steps of 32 are taken in groups of nmg: in each group, wavefront w loads
// and splits step (group * nmg + w) for the whole panel (the same per-lane
// work as opmul_split_kernel does for every step) and leaves the parts in
// LDS in matrix-operand order; then every wavefront multiplies all nmg steps
// of the group from LDS.  The split work per wavefront drops by nmg, the next
// group's rows are loaded while the current group is multiplied, and every
// output sums the same products in the same order as opmul_split_kernel.
template <int MBW, bool F16, int TAG>
__global__ __launch_bounds__(512) void opmul_split_lds_kernel(OpSplit A, const float *__restrict__ B1,
                                                              int64_t ldb1, int K1,
                                                              const float *__restrict__ B2,
                                                              int64_t ldb2, int K2,
                                                              float *__restrict__ C, int64_t ldc,
                                                              int64_t npanels, NegArgs<float> ep) {
    constexpr int NP = F16 ? 2 : 3;
    constexpr int NACC = F16 ? 2 : 1;
    extern __shared__ uintx4 Bs[];              // [nmg][NP][4][64]
    const unsigned blk = xcd_block();
    if (blk >= npanels) return;                 // whole workgroup: padding of the grid
    const int nmg = int(blockDim.x >> 6);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t col = int64_t(blk) * 64 + 4 * (lane & 15);
    const int g = lane >> 4;
    const int K = K1 + K2;
    const int Kb = A.Kb;
    const int mb0 = w * MBW;

    auto row = [&](int k) -> floatx4 {
        k = min(k, K - 1);
        const float *p = k < K1 ? B1 + int64_t(k) * ldb1 : B2 + int64_t(k - K1) * ldb2;
        return *reinterpret_cast<const floatx4 *>(p + col);
    };

    floatx4 acc[NACC][MBW][4];
#pragma unroll
    for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int m = 0; m < MBW; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[c][m][n] = floatx4{0, 0, 0, 0};

    const uintx4 *Ap[3];
#pragma unroll
    for (int q = 0; q < NP; ++q)
        Ap[q] = reinterpret_cast<const uintx4 *>(A.part[q]) + size_t(mb0) * Kb * 64 + lane;

    const int ngroups = (Kb + nmg - 1) / nmg;
    floatx4 x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = row(32 * w + 8 * g + j);
    uintx4 *mine = Bs + size_t(w) * NP * 4 * 64 + lane;
    for (int gr = 0; gr < ngroups; ++gr) {
        if (gr * nmg + w < Kb) {
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                uintx4 b[NP];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    unsigned pp[NP];
                    split2<F16>(x[2 * q][n], x[2 * q + 1][n], pp);
#pragma unroll
                    for (int t = 0; t < NP; ++t) b[t][q] = pp[t];
                }
#pragma unroll
                for (int t = 0; t < NP; ++t) mine[(t * 4 + n) * 64] = b[t];
            }
        }
        const int kn = 32 * ((gr + 1) * nmg + w) + 8 * g;     // next group's rows (clamped)
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = row(kn + j);
        __syncthreads();
        const int nc = min(nmg, Kb - gr * nmg);
        // A fragments one K step ahead (the first of the group loaded here)
        uintx4 an[MBW][NP];
#pragma unroll
        for (int m = 0; m < MBW; ++m)
#pragma unroll
            for (int q = 0; q < NP; ++q) an[m][q] = opaque(Ap[q][(size_t(m) * Kb + gr * nmg) * 64]);
        for (int c = 0; c < nc; ++c) {
            const int kb = gr * nmg + c;
            uintx4 ac[MBW][NP];
#pragma unroll
            for (int m = 0; m < MBW; ++m)
#pragma unroll
                for (int q = 0; q < NP; ++q) ac[m][q] = an[m][q];
            const int kq = min(kb + 1, Kb - 1);
#pragma unroll
            for (int m = 0; m < MBW; ++m)
#pragma unroll
                for (int q = 0; q < NP; ++q) an[m][q] = Ap[q][(size_t(m) * Kb + kq) * 64];
            const uintx4 *src = Bs + size_t(c) * NP * 4 * 64 + lane;
            uintx4 b[NP][4];
#pragma unroll
            for (int t = 0; t < NP; ++t)
#pragma unroll
                for (int n = 0; n < 4; ++n) b[t][n] = src[(t * 4 + n) * 64];
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
                const uintx4 *a = ac[m];
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    if constexpr (F16) {
                        acc[0][m][n] = mfma16x32<F16>(a[0], b[0][n], acc[0][m][n]);
                        acc[1][m][n] = mfma16x32<F16>(a[0], b[1][n], acc[1][m][n]);
                        acc[1][m][n] = mfma16x32<F16>(a[1], b[0][n], acc[1][m][n]);
                    } else {
                        floatx4 tt = mfma16x32<F16>(a[0], b[2][n], acc[0][m][n]);
                        tt = mfma16x32<F16>(a[1], b[1][n], tt);
                        tt = mfma16x32<F16>(a[2], b[0][n], tt);
                        tt = mfma16x32<F16>(a[0], b[1][n], tt);
                        tt = mfma16x32<F16>(a[1], b[0][n], tt);
                        acc[0][m][n] = mfma16x32<F16>(a[0], b[0][n], tt);
                    }
                }
            }
        }
        __syncthreads();
    }
    const float is = A.inv_scale;
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rw = 16 * (mb0 + m) + 4 * g + r;
            if (rw < A.M) {
                floatx4 out;
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    out[n] = NACC == 2 ? acc[0][m][n][r] + acc[NACC - 1][m][n][r] * is : acc[0][m][n][r];
                store_c<TAG>(C, ldc, rw, col, out, ep);
            }
        }
    }
}


}  // namespace

template <typename T, int TAG>
hipError_t launch_opmul_tag(const Op<T> &A, const T *B1, int64_t ldb1, int K1, const T *B2,
                            int64_t ldb2, int K2, T *C, int64_t ldc, int64_t npanels,
                            hipStream_t s, const NegArgs<T> &E) {
    const int nmg = A.nmg, mbw = A.mbw;
    if (A.Kb % ((A.stage == 2 || A.stage == 4) ? 8 : (A.stage == 1 || A.stage == 3) ? 4 : 2))
        return hipErrorInvalidValue;
    if (A.stage == 4 && sizeof(T) != 4) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
        if (A.stage == 4) {
            const size_t lds = size_t(mbw) * A.Kb * 64 * sizeof(float);
            if (lds > 65536) return hipErrorInvalidValue;
            const dim3 g{xcd_grid((npanels + 3) / 4 * nmg)}, b{256u};
#define FR_LDSA(w)                                                                                   \
    case w:                                                                                          \
        opmul_ldsa_kernel<w, TAG><<<g, b, lds, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, nmg, E); \
        break;
            switch (mbw) {
                FR_LDSA(1) FR_LDSA(2) FR_LDSA(3) FR_LDSA(4) FR_LDSA(5) FR_LDSA(6) FR_LDSA(7) FR_LDSA(8)
                default: return hipErrorInvalidValue;
            }
#undef FR_LDSA
            return hipGetLastError();
        }
        if (A.stage == 1 || A.stage == 2) {
            if (nmg > 8) return hipErrorInvalidValue;
            const dim3 g{xcd_grid(npanels)}, b{unsigned(64 * nmg)};
#define FR_LDS(w)                                                                                  \
    case w:                                                                                        \
        if (A.stage == 2)                                                                          \
            opmul_lds_kernel<w, TAG, 8><<<g, b, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, E); \
        else                                                                                       \
            opmul_lds_kernel<w, TAG, 4><<<g, b, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, E); \
        break;
            switch (mbw) {
                FR_LDS(1) FR_LDS(2) FR_LDS(3) FR_LDS(4) FR_LDS(5) FR_LDS(6) FR_LDS(7) FR_LDS(8)
                default: return hipErrorInvalidValue;
            }
#undef FR_LDS
            return hipGetLastError();
        }
    }
    const int64_t nwaves = npanels * nmg;
    const dim3 grid(xcd_grid((nwaves + 3) / 4)), block(256);
    if (A.stage == 5 || A.stage == 6) {
        if (!A.klist || !A.koff || !A.rowmap) return hipErrorInvalidValue;
#define FR_SPARSE(w)                                                                                       \
    case w:                                                                                                \
        if (A.stage == 6)                                                                                  \
            opmul_sparse_kernel<T, w, TAG, 4><<<grid, block, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, nmg, E); \
        else                                                                                               \
            opmul_sparse_kernel<T, w, TAG, 2><<<grid, block, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, nmg, E); \
        break;
        switch (mbw) {
            FR_SPARSE(1) FR_SPARSE(2) FR_SPARSE(3) FR_SPARSE(4)
            default: return hipErrorInvalidValue;
        }
#undef FR_SPARSE
        return hipGetLastError();
    }
#define FR_MBW(w)                                                                                \
    case w:                                                                                      \
        if (A.stage == 3)                                                                        \
            opmul_kernel<T, w, TAG, 4><<<grid, block, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, \
                                                              npanels, nmg, E);                  \
        else                                                                                     \
            opmul_kernel<T, w, TAG, 2><<<grid, block, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, \
                                                              npanels, nmg, E);                  \
        break;
    if (sizeof(T) == 4) {
        switch (mbw) {
            FR_MBW(1) FR_MBW(2) FR_MBW(3) FR_MBW(4) FR_MBW(5) FR_MBW(6) FR_MBW(7) FR_MBW(8)
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (mbw) {
            FR_MBW(1) FR_MBW(2) FR_MBW(3) FR_MBW(4)
            default: return hipErrorInvalidValue;
        }
    }
#undef FR_MBW
    return hipGetLastError();
}

template <bool F16, int TAG>
hipError_t launch_split_tag(const OpSplit &A, const float *B1, int64_t ldb1, int K1,
                            const float *B2, int64_t ldb2, int K2, float *C, int64_t ldc,
                            int64_t npanels, hipStream_t s, const NegArgs<float> &E) {
    if (A.stage == 1) {
        const size_t lds = size_t(A.nmg) * (F16 ? 2 : 3) * 4 * 64 * 16;
        if (A.nmg > 8 || lds > 65536) return hipErrorInvalidValue;
        const dim3 g{xcd_grid(npanels)}, b{unsigned(64 * A.nmg)};
#define FR_SLDS(w)                                                                                       \
    case w:                                                                                              \
        opmul_split_lds_kernel<w, F16, TAG><<<g, b, lds, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, E); \
        break;
        switch (A.mbw) {
            FR_SLDS(1) FR_SLDS(2) FR_SLDS(3) FR_SLDS(4)
            default: return hipErrorInvalidValue;
        }
#undef FR_SLDS
        return hipGetLastError();
    }
    const int64_t nwaves = npanels * A.nmg;
    const dim3 grid(xcd_grid((nwaves + 3) / 4)), block(256);
#define FR_MBW(w)                                                                           \
    case w:                                                                                 \
        opmul_split_kernel<w, F16, TAG><<<grid, block, 0, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, \
                                                               C, ldc, npanels, A.nmg, E);   \
        break;
    switch (A.mbw) {
        FR_MBW(1) FR_MBW(2) FR_MBW(3) FR_MBW(4)
        default: return hipErrorInvalidValue;
    }
#undef FR_MBW
    return hipGetLastError();
}

// Explicit instantiation (definition / declaration) of the launchers of one
// tag: the FP32 and FP64 products, and the two split forms.
#define FR_OPMUL_INSTANCE(T, t) template hipError_t launch_opmul_tag<T, t>(const Op<T> &, const T *, int64_t, int, const T *, int64_t, int, T *, int64_t, int64_t, hipStream_t, const NegArgs<T> &);
#define FR_OPMUL_EXTERN(T, t) extern template hipError_t launch_opmul_tag<T, t>(const Op<T> &, const T *, int64_t, int, const T *, int64_t, int, T *, int64_t, int64_t, hipStream_t, const NegArgs<T> &);
#define FR_SPLIT_INSTANCE(f, t) template hipError_t launch_split_tag<f, t>(const OpSplit &, const float *, int64_t, int, const float *, int64_t, int, float *, int64_t, int64_t, hipStream_t, const NegArgs<float> &);
#define FR_SPLIT_EXTERN(f, t) extern template hipError_t launch_split_tag<f, t>(const OpSplit &, const float *, int64_t, int, const float *, int64_t, int, float *, int64_t, int64_t, hipStream_t, const NegArgs<float> &);

}  // namespace frd
