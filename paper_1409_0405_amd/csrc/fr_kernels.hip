// HIP kernels of the FR right-hand side for gfx950 (CDNA4).
//
// Paper, Section 2.1: an FR step is mostly products C <- A B of a small
// constant operator A with very wide row-major state matrices B (block-by-
// panel shape), plus point-wise operations at solution and flux points.
// Section 3.4: DG-type scheme, Rusanov interface flux, compressible
// Navier-Stokes with constant viscosity.
//
// State layout per element type: [point][field][ld], element index fastest,
// so every point-wise access of a wavefront is one contiguous segment and the
// operator products see B as K rows of (fields x ld) contiguous columns.
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
            gload(c + 1);
            aload(c + 1, an);
        }
        const floatx4 *Bc = Bs[c & 1];
        // Kb is a multiple of KS (the fragment is zero padded): no tail test
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
                                                          int64_t npanels, int nmg) {
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
                *reinterpret_cast<floatx4 *>(C + int64_t(rw) * ldc + col) = out;
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
                                                              int64_t npanels) {
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
                *reinterpret_cast<floatx4 *>(C + int64_t(rw) * ldc + col) = out;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Geometry at a solution point from the Jacobian coefficients.
// Tet: constant columns c0..c2.  Prism: dx/dxi = A1 + C1 z,
// dx/deta = B1 + C2 z, dx/dzeta = C0 + C1 x + C2 y.  Hexahedron (trilinear
// map, coefficients c1..c7): dx/dr = c1 + c4 s + c5 t + c7 st,
// dx/ds = c2 + c4 r + c6 t + c7 rt, dx/dt = c3 + c5 r + c6 s + c7 rs.
// adj[k][j] = J dxi_k/dx_j (rows are cross products of the columns).
// ---------------------------------------------------------------------------
template <typename T, int ET>
__device__ __forceinline__ T metric(const T *__restrict__ g, int64_t ld, int64_t e,
                                    const T *__restrict__ xi, T adj[3][3]) {
    T c[3][3];
    if (ET == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) c[k][d] = g[(3 * k + d) * ld + e];
    } else if (ET == 2) {
        const T r = xi[0], sv = xi[1], t = xi[2];
        const T st = sv * t, rt = r * t, rs = r * sv;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T c1 = g[d * ld + e], c2 = g[(3 + d) * ld + e], c3 = g[(6 + d) * ld + e];
            const T c4 = g[(9 + d) * ld + e], c5 = g[(12 + d) * ld + e], c6 = g[(15 + d) * ld + e];
            const T c7 = g[(18 + d) * ld + e];
            c[0][d] = c1 + c4 * sv + c5 * t + c7 * st;
            c[1][d] = c2 + c4 * r + c6 * t + c7 * rt;
            c[2][d] = c3 + c5 * r + c6 * sv + c7 * rs;
        }
    } else {
        const T x = xi[0], y = xi[1], z = xi[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T A1 = g[d * ld + e], B1 = g[(3 + d) * ld + e], C0 = g[(6 + d) * ld + e];
            const T C1 = g[(9 + d) * ld + e], C2 = g[(12 + d) * ld + e];
            c[0][d] = A1 + C1 * z;
            c[1][d] = B1 + C2 * z;
            c[2][d] = C0 + C1 * x + C2 * y;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        adj[k][0] = c[k1][1] * c[k2][2] - c[k1][2] * c[k2][1];
        adj[k][1] = c[k1][2] * c[k2][0] - c[k1][0] * c[k2][2];
        adj[k][2] = c[k1][0] * c[k2][1] - c[k1][1] * c[k2][0];
    }
    return c[0][0] * adj[0][0] + c[0][1] * adj[0][1] + c[0][2] * adj[0][2];
}

// Inviscid flux F[j][v] of the conserved state u.
template <typename T>
__device__ __forceinline__ void euler_flux(const T u[5], T gamma, T F[3][5], T &p) {
    const T rinv = T(1) / u[0];
    const T v[3] = {u[1] * rinv, u[2] * rinv, u[3] * rinv};
    p = (gamma - T(1)) * (u[4] - T(0.5) * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[j][0] = u[1 + j];
        F[j][1] = u[1] * v[j];
        F[j][2] = u[2] * v[j];
        F[j][3] = u[3] * v[j];
        F[j][1 + j] += p;
        F[j][4] = (u[4] + p) * v[j];
    }
}

// Viscous flux Fv[j][v] from the state u and the physical gradient q[j][v]:
// tau = mu (grad v + grad v^T - 2/3 div v I), heat flux from grad(p/rho) with
// conductivity mu gamma / (Pr (gamma - 1)).
template <typename T>
__device__ __forceinline__ void viscous_flux(const T u[5], const T q[3][5], T gamma, T mu,
                                             T prandtl, T Fv[3][5]) {
    const T rinv = T(1) / u[0];
    const T v[3] = {u[1] * rinv, u[2] * rinv, u[3] * rinv};
    const T e = u[4] * rinv;
    T dv[3][3], dT[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int i = 0; i < 3; ++i) dv[i][j] = (q[j][1 + i] - v[i] * q[j][0]) * rinv;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
        dT[j] = (gamma - T(1)) * ((q[j][4] - e * q[j][0]) * rinv -
                                  (v[0] * dv[0][j] + v[1] * dv[1][j] + v[2] * dv[2][j]));
    const T div = dv[0][0] + dv[1][1] + dv[2][2];
    const T kappa = mu * gamma / (prandtl * (gamma - T(1)));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Fv[j][0] = 0;
        T work = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T tau = mu * (dv[i][j] + dv[j][i]);
            if (i == j) tau -= mu * T(2.0 / 3.0) * div;
            Fv[j][1 + i] = tau;
            work += v[i] * tau;
        }
        Fv[j][4] = work + kappa * dT[j];
    }
}

// ---------------------------------------------------------------------------
// Point-wise solution-point kernel: physical gradient and transformed flux.
// One thread per (element, solution point); blockIdx.y is the point.
// ---------------------------------------------------------------------------
template <typename T, int ET, bool NS>
__global__ __launch_bounds__(256) void upts_kernel(UptsArgs<T> a) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (e >= a.nelem) return;
    const int64_t ld = a.ld;
    T adj[3][3], Jinv;
    if (a.padj) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) adj[k][j] = a.padj[(int64_t(3 * k + j) * a.nu + i) * ld + e];
        Jinv = a.pjinv[int64_t(i) * ld + e];
    } else {
        Jinv = T(1) / metric<T, ET>(a.geom, ld, e, a.xi + 3 * i, adj);
    }
    T u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = a.U[(int64_t(i) * 5 + v) * ld + e];
    T F[3][5], p;
    euler_flux(u, a.gamma, F, p);
    if (NS) {
        T qt[3][5], q[3][5], Fv[3][5];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v)
                qt[k][v] = a.Qt[((int64_t(k) * a.nu + i) * 5 + v) * ld + e];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                q[j][v] = (adj[0][j] * qt[0][v] + adj[1][j] * qt[1][v] + adj[2][j] * qt[2][v]) * Jinv;
                a.Q[(int64_t(i) * 15 + j * 5 + v) * ld + e] = q[j][v];
            }
        viscous_flux(u, q, a.gamma, a.mu, a.prandtl, Fv);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) F[j][v] -= Fv[j][v];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v)
            a.Ft[((int64_t(k) * a.nu + i) * 5 + v) * ld + e] =
                adj[k][0] * F[0][v] + adj[k][1] * F[1][v] + adj[k][2] * F[2][v];
}

// Per-type kernel argument of an element type t in {0, 1, 2}, selected
// without indexing the argument block (which would be a memory load per
// thread).
template <typename P>
__device__ __forceinline__ P pick(const P (&v)[NTYPE], int t) {
    return t == 0 ? v[0] : (t == 1 ? v[1] : v[2]);
}

// Side word: element (22 bits) | flux point << 22 (8 bits) | type << 30.
__device__ __forceinline__ void unpack(uint32_t s, int64_t &e, int &f, int &t) {
    e = s & 0x3fffffu;
    f = (s >> 22) & 0xff;
    t = s >> 30;
}

// Jump to the common solution of the LDG scheme at each paired flux point,
// C = (1/2 - beta) U_L + (1/2 + beta) U_R, stored per side as D = C - U_f:
//   D_L = (1/2 + beta) (U_R - U_L),   D_R = (1/2 - beta) (U_L - U_R).
// A side whose weight is zero keeps the zeros the buffer was created with.
template <typename T>
__global__ __launch_bounds__(256) void common_solution_kernel(PairArgs<T> a) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.npairs) return;
    int64_t eL, eR;
    int fL, fR, tL, tR;
    unpack(a.sideL[p], eL, fL, tL);
    unpack(a.sideR[p], eR, fR, tR);
    const int64_t ldL = pick(a.ld, tL), ldR = pick(a.ld, tR);
    const T wL = T(0.5) + a.beta, wR = T(0.5) - a.beta;
    const T *__restrict__ uL = pick(a.Uf, tL) + int64_t(fL) * 5 * ldL + eL;
    const T *__restrict__ uR = pick(a.Uf, tR) + int64_t(fR) * 5 * ldR + eR;
    T jump[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) jump[v] = uR[v * ldR] - uL[v * ldL];     // all loads first
    if (wL != T(0)) {
        T *dL = pick(a.Cf, tL) + int64_t(fL) * 5 * ldL + eL;
#pragma unroll
        for (int v = 0; v < 5; ++v) dL[v * ldL] = wL * jump[v];
    }
    if (wR != T(0)) {
        T *dR = pick(a.Cf, tR) + int64_t(fR) * 5 * ldR + eR;
#pragma unroll
        for (int v = 0; v < 5; ++v) dR[v * ldR] = -wR * jump[v];
    }
}

// Common transformed normal flux at each paired flux point:
//   f = Rusanov(U_L, U_R; n) [- ((1/2+beta) Fv_L + (1/2-beta) Fv_R).n
//       + tau (U_L - U_R)]   (NS terms in brackets)
// side L stores sL f, side R stores -sR f.
template <typename T, bool NS>
__global__ __launch_bounds__(256) void common_flux_kernel(PairArgs<T> a) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.npairs) return;
    int64_t eL, eR;
    int fL, fR, tL, tR;
    unpack(a.sideL[p], eL, fL, tL);
    unpack(a.sideR[p], eR, fR, tR);
    const int64_t ldL = pick(a.ld, tL), ldR = pick(a.ld, tR);
    const int64_t P = a.npairs;
    const T n[3] = {a.geo[p], a.geo[P + p], a.geo[2 * P + p]};
    const T sL = a.geo[3 * P + p], sR = a.geo[4 * P + p];
    T uL[5], uR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        uL[v] = pick(a.Uf, tL)[(int64_t(fL) * 5 + v) * ldL + eL];
        uR[v] = pick(a.Uf, tR)[(int64_t(fR) * 5 + v) * ldR + eR];
    }
    // gradients of the sides whose LDG weight is not zero, loaded together
    // with the states (beta = +-1/2, the usual choice, needs one side only:
    // the other term would be an exact zero)
    const T wl = T(0.5) + a.beta, wr = T(0.5) - a.beta;
    T qL[3][5], qR[3][5];
    if (NS && wl != T(0)) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) qL[j][v] = pick(a.Qf, tL)[(int64_t(fL) * 15 + j * 5 + v) * ldL + eL];
    }
    if (NS && wr != T(0)) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) qR[j][v] = pick(a.Qf, tR)[(int64_t(fR) * 15 + j * 5 + v) * ldR + eR];
    }
    T FL[3][5], FR[3][5], pL, pR;
    euler_flux(uL, a.gamma, FL, pL);
    euler_flux(uR, a.gamma, FR, pR);
    const T vnL = (uL[1] * n[0] + uL[2] * n[1] + uL[3] * n[2]) / uL[0];
    const T vnR = (uR[1] * n[0] + uR[2] * n[1] + uR[3] * n[2]) / uR[0];
    const T cL = sqrt(a.gamma * pL / uL[0]), cR = sqrt(a.gamma * pR / uR[0]);
    const T lam = fmax(fabs(vnL) + cL, fabs(vnR) + cR);
    T f[5];
#pragma unroll
    for (int v = 0; v < 5; ++v)
        f[v] = T(0.5) * (n[0] * (FL[0][v] + FR[0][v]) + n[1] * (FL[1][v] + FR[1][v]) +
                         n[2] * (FL[2][v] + FR[2][v])) -
               T(0.5) * lam * (uR[v] - uL[v]);
    if (NS) {
        T FvL[3][5], FvR[3][5];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) FvL[j][v] = FvR[j][v] = T(0);
        if (wl != T(0)) viscous_flux(uL, qL, a.gamma, a.mu, a.prandtl, FvL);
        if (wr != T(0)) viscous_flux(uR, qR, a.gamma, a.mu, a.prandtl, FvR);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            T fv = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) fv += n[j] * (wl * FvL[j][v] + wr * FvR[j][v]);
            f[v] += -fv + a.tau * (uL[v] - uR[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        pick(a.Fn, tL)[(int64_t(fL) * 5 + v) * ldL + eL] = sL * f[v];
        pick(a.Fn, tR)[(int64_t(fR) * 5 + v) * ldR + eR] = -sR * f[v];
    }
}

// ---------------------------------------------------------------------------
// Boundary points.  Wall (kind 1): Ub = (rho, 0, 0, 0, rho T_w / (gamma - 1)),
// ghost = (rho, -rho v, rho T_w / (gamma - 1) + rho |v|^2 / 2), the interior
// velocity mirrored at the wall temperature.  Far field (kind 2): the
// outgoing invariant v.n + 2c/(gamma-1) of the interior and the incoming
// v.n - 2c/(gamma-1) of the free stream fix v.n and c; entropy p/rho^gamma
// and tangential velocity come from the interior where the flow leaves the
// domain, else from the free stream; the ghost is Ub.  Temperature is p/rho.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void boundary_states(const T u[5], const T n[3], int kind, const BndArgs<T> &a,
                                                T ub[5], T gh[5]) {
    const T g1 = a.gamma - T(1);
    const T rinv = T(1) / u[0];
    if (kind == 1) {
        const T eint = u[0] * a.t_wall / g1;
        const T ke = T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * rinv;
        ub[0] = u[0];
        ub[1] = ub[2] = ub[3] = T(0);
        ub[4] = eint;
        gh[0] = u[0];
        gh[1] = -u[1];
        gh[2] = -u[2];
        gh[3] = -u[3];
        gh[4] = eint + ke;
        return;
    }
    const T v[3] = {u[1] * rinv, u[2] * rinv, u[3] * rinv};
    const T p = g1 * (u[4] - T(0.5) * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
    const T vnL = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    const T vnf = a.free[1] * n[0] + a.free[2] * n[1] + a.free[3] * n[2];
    const T cL = sqrt(a.gamma * p * rinv), cf = sqrt(a.gamma * a.free[4] / a.free[0]);
    const T rp = vnL + T(2) * cL / g1, rm = vnf - T(2) * cf / g1;
    const T vnb = T(0.5) * (rp + rm), cb = T(0.25) * g1 * (rp - rm);
    const bool out = vnb > T(0);
    const T ent = out ? p / pow(u[0], a.gamma) : a.free[4] / pow(a.free[0], a.gamma);
    T vb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vb[d] = (out ? v[d] - vnL * n[d] : a.free[1 + d] - vnf * n[d]) + vnb * n[d];
    const T rhob = pow(cb * cb / (a.gamma * ent), T(1) / g1);
    const T pb = rhob * cb * cb / a.gamma;
    ub[0] = rhob;
    ub[1] = rhob * vb[0];
    ub[2] = rhob * vb[1];
    ub[3] = rhob * vb[2];
    ub[4] = pb / g1 + T(0.5) * rhob * (vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2]);
#pragma unroll
    for (int k = 0; k < 5; ++k) gh[k] = ub[k];
}

template <typename T>
__global__ __launch_bounds__(256) void boundary_solution_kernel(BndArgs<T> a) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.nb) return;
    int64_t e;
    int f, t;
    unpack(a.side[p], e, f, t);
    const int64_t ld = pick(a.ld, t);
    const T n[3] = {a.geo[p], a.geo[a.nb + p], a.geo[2 * a.nb + p]};
    T u[5], ub[5], gh[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = pick(a.Uf, t)[(int64_t(f) * 5 + v) * ld + e];
    boundary_states(u, n, int(a.kind[p]), a, ub, gh);
#pragma unroll
    for (int v = 0; v < 5; ++v) pick(a.Cf, t)[(int64_t(f) * 5 + v) * ld + e] = ub[v] - u[v];
}

template <typename T, bool NS>
__global__ __launch_bounds__(256) void boundary_flux_kernel(BndArgs<T> a) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.nb) return;
    int64_t e;
    int f, t;
    unpack(a.side[p], e, f, t);
    const int64_t ld = pick(a.ld, t);
    const int64_t nb = a.nb;
    const T n[3] = {a.geo[p], a.geo[nb + p], a.geo[2 * nb + p]};
    const T sc = a.geo[3 * nb + p];
    T u[5], ub[5], gh[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = pick(a.Uf, t)[(int64_t(f) * 5 + v) * ld + e];
    T q[3][5];
    if (NS) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int v = 0; v < 5; ++v) q[j][v] = pick(a.Qf, t)[(int64_t(f) * 15 + j * 5 + v) * ld + e];
    }
    boundary_states(u, n, int(a.kind[p]), a, ub, gh);
    T FL[3][5], FR[3][5], pL, pR;
    euler_flux(u, a.gamma, FL, pL);
    euler_flux(gh, a.gamma, FR, pR);
    const T vnL = (u[1] * n[0] + u[2] * n[1] + u[3] * n[2]) / u[0];
    const T vnR = (gh[1] * n[0] + gh[2] * n[1] + gh[3] * n[2]) / gh[0];
    const T lam = fmax(fabs(vnL) + sqrt(a.gamma * pL / u[0]), fabs(vnR) + sqrt(a.gamma * pR / gh[0]));
    T fl[5];
#pragma unroll
    for (int v = 0; v < 5; ++v)
        fl[v] = T(0.5) * (n[0] * (FL[0][v] + FR[0][v]) + n[1] * (FL[1][v] + FR[1][v]) +
                          n[2] * (FL[2][v] + FR[2][v])) -
                T(0.5) * lam * (gh[v] - u[v]);
    if (NS) {
        T Fv[3][5];
        viscous_flux(ub, q, a.gamma, a.mu, a.prandtl, Fv);
#pragma unroll
        for (int v = 0; v < 5; ++v)
            fl[v] += -(n[0] * Fv[0][v] + n[1] * Fv[1][v] + n[2] * Fv[2][v]) + a.tau * (u[v] - ub[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) pick(a.Fn, t)[(int64_t(f) * 5 + v) * ld + e] = sc * fl[v];
}

// R = -Rt / J at each solution point, fused with a Runge-Kutta register update.
template <typename T, int ET>
__global__ __launch_bounds__(256) void negdivconf_kernel(NegArgs<T> a) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (e >= a.nelem) return;
    const int64_t ld = a.ld;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const int64_t o = (int64_t(i) * 5 + v) * ld + e;
        neg_update(a, i, v, e, o, a.Rt[o]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(RedArgs<T> a) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t n = int64_t(a.nu) * a.nelem;
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n;
         idx += int64_t(gridDim.x) * blockDim.x) {
        const int i = int(idx / a.nelem);
        const int64_t e = idx - int64_t(i) * a.nelem;
        const double wJ = a.wJ[int64_t(i) * a.ld + e];
        double u[5], r[5] = {0, 0, 0, 0, 0};
        for (int v = 0; v < 5; ++v) {
            u[v] = double(a.U[(int64_t(i) * 5 + v) * a.ld + e]);
            if (a.R) r[v] = double(a.R[(int64_t(i) * 5 + v) * a.ld + e]);
        }
        if (a.what == 1) {
            for (int v = 0; v < 5; ++v) s[v] += wJ * u[v];
        } else if (a.what == 2) {
            for (int v = 0; v < 5; ++v) s[v] += wJ * r[v];
        } else if (a.what == 3) {
            for (int v = 0; v < 5; ++v) s[v] += wJ * r[v] * r[v];
        } else if (a.what == 4) {
            const double vx = u[1] / u[0], vy = u[2] / u[0], vz = u[3] / u[0];
            const double v2 = vx * vx + vy * vy + vz * vz;
            s[0] += wJ * 0.5 * u[0] * v2;
            s[1] += wJ * (vx * r[1] + vy * r[2] + vz * r[3] - 0.5 * v2 * r[0]);
        } else if (a.what == 5) {
            for (int v = 0; v < 5; ++v) s[0] += isfinite(u[v]) ? 0.0 : 1.0;
        } else if (a.what == 6) {
            for (int v = 0; v < 5; ++v) {
                const double u0 = double(a.U0[(int64_t(i) * 5 + v) * a.ld + e]);
                const double q = r[v] / (a.atol + a.rtol * fmax(fabs(u0), fabs(u[v])));
                s[0] += q * q;
            }
        }
    }
    __shared__ double sh[8][256];
    for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w)
            for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 8) a.partial[int64_t(blockIdx.x) * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

// out[q] = sum_b partial[b][q]: block q, fixed summation tree (deterministic)
__global__ __launch_bounds__(256) void reduce_final_kernel(const double *partial, int nblocks, double *out) {
    const int q = blockIdx.x;
    double s = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[int64_t(b) * 8 + q];
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0];
}

template <typename T>
__global__ void copy_kernel(T *dst, const T *src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
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

template <typename T>
hipError_t launch_opmul(int tag, const Op<T> &A, const T *B1, int64_t ldb1, int K1, const T *B2,
                        int64_t ldb2, int K2, T *C, int64_t ldc, int64_t ncols, hipStream_t s,
                        const NegArgs<T> *ep) {
    if (ncols % 64 || K1 + K2 <= 0 || A.nmg * A.mbw * 16 < A.M) return hipErrorInvalidValue;
    const NegArgs<T> E = ep ? *ep : NegArgs<T>{};
    // the fused store addresses the divergence output layout [nu][5][ld]
    if (E.fuse && (tag % 4 != 3 || E.ld % 64 || ldc != 5 * E.ld || ncols != ldc || A.M != E.nu ||
                   E.nelem > E.ld || !E.jinv))
        return hipErrorInvalidValue;
    const int64_t npanels = ncols / 64;
#define FR_TAG(t) \
    case t: return launch_opmul_tag<T, t>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels, s, E);
    switch (tag) {
        FR_TAG(0) FR_TAG(1) FR_TAG(2) FR_TAG(3) FR_TAG(4) FR_TAG(5) FR_TAG(6) FR_TAG(7)
        FR_TAG(8) FR_TAG(9) FR_TAG(10) FR_TAG(11)
        default: return hipErrorInvalidValue;
    }
#undef FR_TAG
}

template <bool F16, int TAG>
hipError_t launch_split_tag(const OpSplit &A, const float *B1, int64_t ldb1, int K1,
                            const float *B2, int64_t ldb2, int K2, float *C, int64_t ldc,
                            int64_t npanels, hipStream_t s) {
    if (A.stage == 1) {
        const size_t lds = size_t(A.nmg) * (F16 ? 2 : 3) * 4 * 64 * 16;
        if (A.nmg > 8 || lds > 65536) return hipErrorInvalidValue;
        const dim3 g{xcd_grid(npanels)}, b{unsigned(64 * A.nmg)};
#define FR_SLDS(w)                                                                                       \
    case w:                                                                                              \
        opmul_split_lds_kernel<w, F16, TAG><<<g, b, lds, s>>>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, npanels); \
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
                                                               C, ldc, npanels, A.nmg);      \
        break;
    switch (A.mbw) {
        FR_MBW(1) FR_MBW(2) FR_MBW(3) FR_MBW(4)
        default: return hipErrorInvalidValue;
    }
#undef FR_MBW
    return hipGetLastError();
}

hipError_t launch_opmul_split(int tag, const OpSplit &A, const float *B1, int64_t ldb1, int K1,
                              const float *B2, int64_t ldb2, int K2, float *C, int64_t ldc,
                              int64_t ncols, hipStream_t s) {
    if (ncols % 64 || K1 + K2 <= 0 || A.nmg * A.mbw * 16 < A.M || (A.Kb & 1))
        return hipErrorInvalidValue;
    const int64_t np = ncols / 64;
#define FR_TAG(t)                                                                            \
    case t:                                                                                  \
        return A.format == 2 ? launch_split_tag<true, t>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, np, s) \
                             : launch_split_tag<false, t>(A, B1, ldb1, K1, B2, ldb2, K2, C, ldc, np, s);
    switch (tag) {
        FR_TAG(0) FR_TAG(1) FR_TAG(2) FR_TAG(3) FR_TAG(4) FR_TAG(5) FR_TAG(6) FR_TAG(7)
        FR_TAG(8) FR_TAG(9) FR_TAG(10) FR_TAG(11)
        default: return hipErrorInvalidValue;
    }
#undef FR_TAG
}

template <typename T>
hipError_t launch_upts(int etype, bool ns, const UptsArgs<T> &a, hipStream_t s) {
    const dim3 grid(unsigned((a.nelem + 255) / 256), unsigned(a.nu)), block(256);
    if (etype == 0) {
        if (ns) upts_kernel<T, 0, true><<<grid, block, 0, s>>>(a);
        else upts_kernel<T, 0, false><<<grid, block, 0, s>>>(a);
    } else if (etype == 1) {
        if (ns) upts_kernel<T, 1, true><<<grid, block, 0, s>>>(a);
        else upts_kernel<T, 1, false><<<grid, block, 0, s>>>(a);
    } else {
        if (ns) upts_kernel<T, 2, true><<<grid, block, 0, s>>>(a);
        else upts_kernel<T, 2, false><<<grid, block, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_common_solution(const PairArgs<T> &a, hipStream_t s) {
    if (!a.npairs) return hipSuccess;
    common_solution_kernel<T><<<unsigned((a.npairs + 255) / 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_common_flux(bool ns, const PairArgs<T> &a, hipStream_t s) {
    if (!a.npairs) return hipSuccess;
    const unsigned g = unsigned((a.npairs + 255) / 256);
    if (ns) common_flux_kernel<T, true><<<g, 256, 0, s>>>(a);
    else common_flux_kernel<T, false><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_boundary_solution(const BndArgs<T> &a, hipStream_t s) {
    if (!a.nb) return hipSuccess;
    boundary_solution_kernel<T><<<unsigned((a.nb + 255) / 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_boundary_flux(bool ns, const BndArgs<T> &a, hipStream_t s) {
    if (!a.nb) return hipSuccess;
    const unsigned g = unsigned((a.nb + 255) / 256);
    if (ns) boundary_flux_kernel<T, true><<<g, 256, 0, s>>>(a);
    else boundary_flux_kernel<T, false><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_negdivconf(int etype, const NegArgs<T> &a, hipStream_t s) {
    const dim3 grid(unsigned((a.nelem + 255) / 256), unsigned(a.nu)), block(256);
    if (etype == 0) negdivconf_kernel<T, 0><<<grid, block, 0, s>>>(a);
    else if (etype == 1) negdivconf_kernel<T, 1><<<grid, block, 0, s>>>(a);
    else negdivconf_kernel<T, 2><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const RedArgs<T> &a, hipStream_t s) {
    reduce_kernel<T><<<RED_BLOCKS, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_reduce_final(const double *partial, int nblocks, double *out, hipStream_t s) {
    reduce_final_kernel<<<8, 256, 0, s>>>(partial, nblocks, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    copy_kernel<T><<<1024, 256, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

#define FR_INSTANTIATE(T)                                                                     \
    template hipError_t launch_opmul<T>(int, const Op<T> &, const T *, int64_t, int,          \
                                        const T *, int64_t, int, T *, int64_t, int64_t,       \
                                        hipStream_t, const NegArgs<T> *);                     \
    template hipError_t launch_upts<T>(int, bool, const UptsArgs<T> &, hipStream_t);          \
    template hipError_t launch_common_solution<T>(const PairArgs<T> &, hipStream_t);          \
    template hipError_t launch_common_flux<T>(bool, const PairArgs<T> &, hipStream_t);        \
    template hipError_t launch_boundary_solution<T>(const BndArgs<T> &, hipStream_t);         \
    template hipError_t launch_boundary_flux<T>(bool, const BndArgs<T> &, hipStream_t);       \
    template hipError_t launch_negdivconf<T>(int, const NegArgs<T> &, hipStream_t);           \
    template hipError_t launch_reduce<T>(const RedArgs<T> &, hipStream_t);                    \
    template hipError_t launch_copy<T>(T *, const T *, int64_t, hipStream_t);

FR_INSTANTIATE(float)
FR_INSTANTIATE(double)

}  // namespace frd
