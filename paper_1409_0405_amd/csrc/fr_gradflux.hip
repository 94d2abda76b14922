// Fused gradient stage of the Navier-Stokes right-hand side (gfx950).
//
// Paper, Section 2.1: an FR step is operator products C <- A B with the
// element state as B, separated by point-wise work.  Between the common
// solution and the common flux the separate kernels pass three arrays
// through memory: the reference gradient Qt (corrected gradient product),
// the physical gradient Q and the transformed flux Ft (point-wise kernel),
// and Q again (gradient interpolation).  Here one workgroup takes a tile of
// NE elements with all five fields and keeps Qt and Q in LDS:
//   1. B = [U; Cf] of the tile -> LDS;
//   2. Qt = [G_k | L_k] B on the matrix cores -> LDS;
//   3. per (solution point, element): Q = adj^T Qt / J (in place), and
//      Ft = adj (F_inv(U) - F_vis(U, Q)) -> memory;
//   4. Qf = M0 Q on the matrix cores -> memory.
// Only U and Cf are read and only Ft and Qf are written, Qf only on the
// faces whose gradient the interface and boundary kernels read (with the
// usual LDG weights one side of each interface).  The operator
// fragments are those of the step-list products (one row block per group),
// walked in the same K order, and the point-wise arithmetic is the shared
// upts_point, so every value has the bits of the separate kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fr_device.hpp"
#include "fr_opmul.hpp"
#include "fr_pointwise.hpp"

namespace frd {
namespace {

template <int ET>
constexpr int n_geom_coeffs() { return ET == 0 ? 9 : ET == 1 ? 15 : 21; }

// Entry i of a step list through the scalar data cache: the lists are
// read-only and the index is uniform in the wavefront, and a constant-space
// load lets the compiler use a scalar load, which the vector-memory counter
// (the operator fragments in flight) does not wait for.
__device__ __forceinline__ int sload(const int32_t *p, int i) {
    return ((const __attribute__((address_space(4))) int32_t *)p)[i];
}

// 16 (4) bytes from memory straight into LDS (global_load_lds): lane l of
// the wavefront writes dst + 16 l (dst + 4 l), dst uniform in the wavefront.
__device__ __forceinline__ void load_lds16(const void *src, void *dst) {
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}
__device__ __forceinline__ void load_lds4(const void *src, void *dst) {
    __builtin_amdgcn_global_load_lds(src, dst, 4, 0, 0);
}

// acc[n] += A_g B[:, 16 n .. 16 n + 15] for row block g of a step-list
// operator (one row block per group), B in LDS: brow(kb) points at row
// 4 kb + krow, column lane % 16 of B.  The list is walked in chunks of CH
// steps (lists are padded to a multiple of four; CH is 4 or 2): while the
// CH NB matrix instructions of one chunk issue, the operator fragments
// (memory) and the B values (LDS) of the next chunk are already on their
// way, so a wave waits for neither.  The K order is the list order, as in
// the step-list product kernel.
template <typename T, int NB, int CH = 4, typename V4, typename RowFn>
__device__ __forceinline__ void step_products(const Op<T> &A, int g, int lane, RowFn brow, V4 (&acc)[NB]) {
    static_assert(CH == 2 || CH == 4, "chunks of 2 or 4 steps");
    const int s0 = sload(A.koff, g), ns = sload(A.koff, g + 1) - s0;   // a multiple of 4, >= 4
    const int32_t *kl = A.klist + s0;
    const T *Af = A.frag + size_t(s0) * 64 + lane;
    T a0[CH], b0[CH][NB];
#pragma unroll
    for (int d = 0; d < CH; ++d) {
        a0[d] = Af[size_t(d) * 64];
        const T *br = brow(sload(kl, d));
#pragma unroll
        for (int n = 0; n < NB; ++n) b0[d][n] = br[16 * n];
    }
    for (int st = 0; st < ns; st += CH) {
        // the next chunk (the last chunk loads itself again: in bounds, unused)
        const int nx = min(st + CH, ns - CH);
        T a1[CH], b1[CH][NB];
#pragma unroll
        for (int d = 0; d < CH; ++d) {
            a1[d] = Af[size_t(nx + d) * 64];
            const T *br = brow(sload(kl, nx + d));
#pragma unroll
            for (int n = 0; n < NB; ++n) b1[d][n] = br[16 * n];
        }
        // keep the scheduler from sinking the loads above next to their use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < CH; ++d)
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[n] = mfma16(a0[d], b0[d][n], acc[n]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < CH; ++d) {
            a0[d] = a1[d];
#pragma unroll
            for (int n = 0; n < NB; ++n) b0[d][n] = b1[d][n];
        }
    }
}

// Steps of a list that carry operator entries: the list is padded to a
// multiple of 4 by repeating its last step with zero fragments (a real
// step names each K step once, so a repeat can only be padding).  The deep
// walkers below stop there; an accumulator that starts at +0 is never -0
// (a sum of opposite zeros rounds to +0), so the products they leave out
// (exact zeros) would not have changed any bit of it.
__device__ __forceinline__ int real_steps(const int32_t *kl, int ns) {
    int n = ns;
    while (n > 1 && sload(kl, n - 1) == sload(kl, n - 2)) --n;
    return n;
}

// acc[n] += A_g B[:, 16 n .. 16 n + 15] like step_products, with the
// operator fragments (memory) 4 steps ahead of their use and the B values
// (LDS) one step ahead.
template <typename T, int NB, typename V4, typename RowFn>
__device__ __forceinline__ void step_products_deep(const Op<T> &A, int g, int lane, RowFn brow, V4 (&acc)[NB]) {
    const int s0 = sload(A.koff, g), ns = sload(A.koff, g + 1) - s0;   // a multiple of 4, >= 4
    const int32_t *kl = A.klist + s0;
    const T *Af = A.frag + size_t(s0) * 64 + lane;
    T a[4], b0[NB], b1[NB];
#pragma unroll
    for (int d = 0; d < 4; ++d) a[d] = Af[size_t(d) * 64];
    {
        const T *br = brow(sload(kl, 0));
#pragma unroll
        for (int n = 0; n < NB; ++n) b0[n] = br[16 * n];
    }
    const int nr = real_steps(kl, ns);
    for (int st = 0; st < nr; st += 4) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (st + d >= nr) break;
            const T *br = brow(sload(kl, min(st + d + 1, ns - 1)));
#pragma unroll
            for (int n = 0; n < NB; ++n) b1[n] = br[16 * n];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[n] = mfma16(a[d], b0[n], acc[n]);
            __builtin_amdgcn_sched_barrier(0);
            a[d] = Af[size_t(min(st + d + 4, ns - 1)) * 64];
#pragma unroll
            for (int n = 0; n < NB; ++n) b0[n] = b1[n];
        }
    }
}

// acc[j][i] += A_g Q_j[:, column block NH i + h] for row block g of a
// step-list operator and all three gradient directions j: one operator
// fragment feeds 3 NBI matrix instructions.  q points at row 0, column
// 16 h + lane % 16 of Q_0 in LDS, Q_j is jstride values further on; rows
// past the last solution point are clamped to it (times zero columns of A).
// The fragments (memory) travel 4 steps ahead of their use, the Q values
// (LDS) one step; the K order is the list order, as in step_products.
template <typename T, int NBI, int NH, int W5, typename V4>
__device__ __forceinline__ void interp3_products(const Op<T> &A, int g, int lane, int krow, const T *q,
                                                 int jstride, int nu, V4 (&acc)[3][NBI]) {
    const int s0 = sload(A.koff, g), ns = sload(A.koff, g + 1) - s0;   // a multiple of 4, >= 4
    const int32_t *kl = A.klist + s0;
    const T *Af = A.frag + size_t(s0) * 64 + lane;
    auto qload = [&](int s, T (&b)[3][NBI]) {
        const T *br = q + min(4 * sload(kl, s) + krow, nu - 1) * W5;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < NBI; ++i) b[j][i] = br[j * jstride + 16 * NH * i];
    };
    T a[4], b0[3][NBI], b1[3][NBI];
#pragma unroll
    for (int d = 0; d < 4; ++d) a[d] = Af[size_t(d) * 64];
    qload(0, b0);
    const int nr = real_steps(kl, ns);
    for (int st = 0; st < nr; st += 4) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (st + d >= nr) break;
            qload(min(st + d + 1, ns - 1), b1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int i = 0; i < NBI; ++i) acc[j][i] = mfma16(a[d], b0[j][i], acc[j][i]);
            __builtin_amdgcn_sched_barrier(0);
            a[d] = Af[size_t(min(st + d + 4, ns - 1)) * 64];
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int i = 0; i < NBI; ++i) b0[j][i] = b1[j][i];
        }
    }
}

// Tile of NE elements with all five fields: row r of a tile in LDS holds W5
// columns, (field v, element e) at v NE + e and zeros up to W5; column block
// n of the matrix instructions is columns 16 n .. 16 n + 15.
template <int NE>
struct TileShape {
    static constexpr int W5 = (5 * NE + 15) / 16 * 16;
    static constexpr int NB = W5 / 16;
};

// Elements per tile.  The wider the tile, the more matrix instructions each
// operator fragment feeds (NE / 16 x 5 in FP32), which the measurements
// favour over more workgroups per CU: FP32 tets and prisms take 32 (at
// p = 4: 69 KB of LDS, two workgroups per CU for tets; 147 KB, one
// workgroup of 16 wavefronts for prisms), hexahedra 16 (123 KB; 32 would not
// fit, 8 was 24 % slower), FP64 4 (its LDS footprint per value is twice as
// large).
template <typename T, int ET>
constexpr int tile_elems() { return sizeof(T) == 4 ? (ET == 2 ? 16 : 32) : 4; }

// One workgroup of NW wavefronts per tile.  MG: row blocks of the gradient
// operator per wavefront (>= nmg / NW); their accumulators stay in registers
// until every wavefront has finished reading B, so that Qt takes B's place in
// LDS and a tile needs max(B, Qt) of it.
template <typename T, int ET, int NE, int NW, int MG>
__global__ __launch_bounds__(64 * NW) void gradflux_kernel(GradFluxArgs<T> a) {
    using v4 = typename Vec4<T>::type;
    constexpr int W5 = TileShape<NE>::W5, NB = TileShape<NE>::NB;
    constexpr int NG = n_geom_coeffs<ET>();
    constexpr int VPR = NE * int(sizeof(T)) / 16;       // 16-byte vectors per (row, field)
    constexpr int CH = NB > 5 ? 2 : 4;                   // step-list chunk: B values in flight fit registers
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int Kp = 4 * a.G.Kb;
    const int nu = a.nu;
    // one region: B = [U; Cf] ([Kp][W5]) for the gradient product, then Qt
    // and, in place, Q ([3 nu][W5], row k nu + i)
    T *Bs = reinterpret_cast<T *>(lds_raw);
    T *QT = Bs;
    T *Gs = Bs + size_t(max(Kp, 3 * nu)) * W5;           // [NG][NE] Jacobian coefficients
    T *Xs = Gs + NG * NE;                                // [nu][3] reference coordinates

    const int64_t e0 = int64_t(xcd_block()) * NE;
    if (e0 >= a.nelem) return;                           // whole workgroup: padding of the grid
    // the wavefront index is uniform in the wavefront: say so, so that the
    // step lists are read through scalar loads and the loops branch on
    // scalars
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int krow = lane >> 4, c16 = lane & 15;
    const int64_t ld = a.ld;

    // 1. B rows: U (k < nu), Cf (nu <= k < nu + nf), zero up to Kp
    if constexpr (sizeof(T) == 4 && W5 == 5 * NE) {
        // straight from memory into LDS (global_load_lds: no registers, and
        // every load of the tile in flight before the one wait): chunk c
        // (16 bytes) of B is row k, field v, elements 4 q .. 4 q + 3 with
        // c = VPR (5 k + v) + q, and lane l of a wavefront instruction
        // writes chunk base + l; the coefficients likewise, the reference
        // coordinates value by value
        const int nchunk = (nu + a.nf) * 5 * VPR;
        for (int base = w * 64; base < nchunk; base += NW * 64) {
            const int c = base + lane;
            if (c < nchunk) {
                const int q = c % VPR, kv = c / VPR, v = kv % 5, k = kv / 5;
                const T *src = k < nu ? a.U + (int64_t(k) * 5 + v) * ld + e0 + 4 * q
                                      : a.Cf + (int64_t(k - nu) * 5 + v) * ld + e0 + 4 * q;
                load_lds16(src, Bs + size_t(base) * 4);
            }
        }
        if (!a.padj)
            for (int base = w * 64; base < NG * VPR; base += NW * 64) {
                const int c = base + lane;
                if (c < NG * VPR)
                    load_lds16(a.geom + int64_t(c / VPR) * ld + e0 + 4 * (c % VPR), Gs + size_t(base) * 4);
            }
        for (int base = w * 64; base < 3 * nu; base += NW * 64) {
            const int c = base + lane;
            if (c < 3 * nu) load_lds4(a.xi + c, Xs + base);
        }
        for (int idx = (nu + a.nf) * W5 + tid; idx < Kp * W5; idx += 64 * NW) Bs[idx] = T(0);
        __builtin_amdgcn_s_waitcnt(0);                   // this wavefront's direct loads are in LDS
    } else {
        for (int idx = tid; idx < 3 * nu; idx += 64 * NW) Xs[idx] = a.xi[idx];
        const int nvec = Kp * 5 * VPR;
        for (int idx = tid; idx < nvec; idx += 64 * NW) {
            const int q = idx % VPR, kv = idx / VPR;
            const int v = kv % 5, k = kv / 5;
            floatx4 val = {0, 0, 0, 0};
            if (k < nu)
                val = *reinterpret_cast<const floatx4 *>(a.U + (int64_t(k) * 5 + v) * ld + e0 +
                                                         q * (16 / sizeof(T)));
            else if (k < nu + a.nf)
                val = *reinterpret_cast<const floatx4 *>(a.Cf + (int64_t(k - nu) * 5 + v) * ld + e0 +
                                                         q * (16 / sizeof(T)));
            *reinterpret_cast<floatx4 *>(Bs + k * W5 + v * NE + q * (16 / sizeof(T))) = val;
        }
        if constexpr (W5 > 5 * NE) {
            constexpr int PADC = W5 - 5 * NE;
            for (int idx = tid; idx < Kp * PADC; idx += 64 * NW)
                Bs[(idx / PADC) * W5 + 5 * NE + idx % PADC] = T(0);
        }
        if (!a.padj)
            for (int idx = tid; idx < NG * NE; idx += 64 * NW)
                Gs[idx] = a.geom[int64_t(idx / NE) * ld + e0 + idx % NE];
    }
    __syncthreads();

    // 2. Qt = [G_k | L_k] B: wavefront w takes row blocks w, w + NW, ..., each
    // against every column block
    // (the Qt row of each accumulator is loaded before the products, so
    // that its latency hides behind them)
    v4 acc[MG][NB];
    int qrow[MG][4];
#pragma unroll
    for (int m = 0; m < MG; ++m) {
        const int g = w + m * NW;
#pragma unroll
        for (int r = 0; r < 4; ++r) qrow[m][r] = g < a.G.nmg ? a.G.rowmap[16 * g + acc_row<T>(krow, r)] : -1;
    }
#pragma unroll
    for (int m = 0; m < MG; ++m) {
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[m][n] = v4{0, 0, 0, 0};
        const int g = w + m * NW;
        if (g < a.G.nmg) {
            auto brow = [&](int kb) { return Bs + (4 * kb + krow) * W5 + c16; };
            if constexpr (sizeof(T) == 4)
                step_products_deep<T, NB>(a.G, g, lane, brow, acc[m]);
            else
                step_products<T, NB, CH>(a.G, g, lane, brow, acc[m]);
        }
    }
    // the states of this thread's first PI points of the point-wise phase,
    // from B while it is still in LDS (at p = 4 three cover every point of
    // an FP32 tet or prism tile)
    constexpr int PI = sizeof(T) == 4 && ET < 2 ? 3 : 2;
    T u0[PI][5];
#pragma unroll
    for (int q = 0; q < PI; ++q) {
        const int it = q * 64 * NW + tid;
        const int i = it / NE, e = it - i * NE;
        if (it < nu * NE) {
#pragma unroll
            for (int v = 0; v < 5; ++v) u0[q][v] = Bs[i * W5 + v * NE + e];
        }
    }
    __syncthreads();                                     // every wavefront is done with B
#pragma unroll
    for (int m = 0; m < MG; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = qrow[m][r];
            if (row >= 0) {
#pragma unroll
                for (int n = 0; n < NB; ++n) QT[row * W5 + 16 * n + c16] = acc[m][n][r];
            }
        }
    }
    __syncthreads();

    // 3. point-wise: one (solution point, element) per thread; Q replaces Qt
    // in place, Ft goes to memory.  A thread's first PI states came from B
    // above; further ones (B's place in LDS holds Qt now) come again from
    // memory, where L2 serves them, and a thread loads those of its next PI
    // points first, so that no load queues behind the Ft stores of the
    // points before it (memory operations of a wavefront retire in order).
    for (int base = 0; base < nu * NE; base += PI * 64 * NW) {
        T uu[PI][5];
#pragma unroll
        for (int q = 0; q < PI; ++q) {
            const int it = base + q * 64 * NW + tid;
            const int i = it / NE, e = it - i * NE;
            if (base == 0) {
#pragma unroll
                for (int v = 0; v < 5; ++v) uu[q][v] = u0[q][v];
            } else if (it < nu * NE && e0 + e < a.nelem) {
#pragma unroll
                for (int v = 0; v < 5; ++v) uu[q][v] = a.U[(int64_t(i) * 5 + v) * ld + e0 + e];
            }
        }
#pragma unroll
        for (int q = 0; q < PI; ++q) {
            const int it = base + q * 64 * NW + tid;
            const int i = it / NE, e = it - i * NE;
            const int64_t eg = e0 + e;
            if (it >= nu * NE || eg >= a.nelem) continue;
            T adj[3][3], Jinv;
            if (a.padj) {
                // (the metric is waited for inside this branch: left in
                // flight, it would make the straight elements wait at the
                // join, and with it for the previous point's Ft stores)
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < 3; ++j) adj[k][j] = a.padj[(int64_t(3 * k + j) * nu + i) * ld + eg];
                Jinv = a.pjinv[int64_t(i) * ld + eg];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < 3; ++j) adj[k][j] = opaque(adj[k][j]);
                Jinv = opaque(Jinv);
            } else {
                Jinv = T(1) / metric<T, ET>(Gs, NE, e, Xs + 3 * i, adj);
            }
            T qt[3][5], q3[3][5], Ft[3][5];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) qt[k][v] = QT[(k * nu + i) * W5 + v * NE + e];
            upts_point<T, true>(uu[q], qt, adj, Jinv, a.gamma, a.mu, a.prandtl, a.pref, q3, Ft);
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int v = 0; v < 5; ++v) QT[(j * nu + i) * W5 + v * NE + e] = q3[j][v];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) a.Ft[((int64_t(k) * nu + i) * 5 + v) * ld + eg] = Ft[k][v];
        }
    }
    __syncthreads();

    // 4. Qf = M0 Q for each gradient direction j: work items (row block, j).
    // Column block n of lane l is element (16 n + l) % NE of the tile, stored
    // only on the faces of it whose gradient is read (qm); the flux point
    // and face of each accumulator row are loaded before the products,
    // behind which their latency hides.
    // (column blocks n and n + NE / 16 hold the same element)
    constexpr int NQ = NE >= 16 ? NE / 16 : 1;
    unsigned qm[NQ];
#pragma unroll
    for (int n = 0; n < NQ; ++n) qm[n] = a.qmask ? unsigned(a.qmask[e0 + (16 * n + c16) % NE]) : 0xffu;
    if constexpr (sizeof(T) == 4 && NB == 10) {
        // tiles of 32 (tets, prisms): work items (row block, column half)
        // with the three directions together, so each operator fragment is
        // loaded once for 15 matrix instructions and every wavefront takes
        // at most one item at p = 4.  (Hexahedra, tiles of 16, keep the
        // items per direction below: with one item per row block, 10 items
        // would leave 6 of the 16 wavefronts idle.)
        constexpr int NH = 2, NBI = 5;
        for (int it = w; it < a.M.nmg * NH; it += NW) {
            const int g = it / NH, h = it - NH * g;
            int frow[4];
            unsigned fb[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int slot = 16 * g + acc_row<T>(krow, r);
                frow[r] = a.M.rowmap[slot];
                fb[r] = a.qmask ? unsigned(a.fbit[slot]) : 1u;
            }
            v4 acc3[3][NBI];
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int i = 0; i < NBI; ++i) acc3[j][i] = v4{0, 0, 0, 0};
            interp3_products<T, NBI, NH, W5>(a.M, g, lane, krow, QT + 16 * h + c16, nu * W5, nu, acc3);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = frow[r];
                if (f < 0) continue;
#pragma unroll
                for (int i = 0; i < NBI; ++i) {
                    const int n = NH * i + h;
                    const int flat = 16 * n + c16, v = flat / NE, e = flat - v * NE;
                    if (v < 5 && e0 + e < a.nelem && (qm[n % NQ] & fb[r])) {
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            a.Qf[(int64_t(f) * 15 + j * 5 + v) * ld + e0 + e] = acc3[j][i][r];
                    }
                }
            }
        }
        return;
    }
    for (int it = w; it < a.M.nmg * 3; it += NW) {
        const int g = it / 3, j = it - 3 * g;
        int frow[4];
        unsigned fb[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int slot = 16 * g + acc_row<T>(krow, r);
            frow[r] = a.M.rowmap[slot];
            fb[r] = a.qmask ? unsigned(a.fbit[slot]) : 1u;
        }
        const T *Qj = QT + size_t(j) * nu * W5 + c16;
        v4 acc2[NB];
#pragma unroll
        for (int n = 0; n < NB; ++n) acc2[n] = v4{0, 0, 0, 0};
        // rows of B past K are clamped to a real row (times zero columns of A)
        auto qrowp = [&](int kb) { return Qj + min(4 * kb + krow, nu - 1) * W5; };
        if constexpr (sizeof(T) == 4)
            step_products_deep<T, NB>(a.M, g, lane, qrowp, acc2);
        else
            step_products<T, NB, CH>(a.M, g, lane, qrowp, acc2);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = frow[r];
            if (f < 0) continue;
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int flat = 16 * n + c16, v = flat / NE, e = flat - v * NE;
                if (v < 5 && e0 + e < a.nelem && (qm[n % NQ] & fb[r]))
                    a.Qf[(int64_t(f) * 15 + j * 5 + v) * ld + e0 + e] = acc2[n][r];
            }
        }
    }
}

constexpr size_t GRADFLUX_LDS_MAX = 160 * 1024;

// Streaming form (FP32): a workgroup takes a contiguous run of tiles and,
// while it works on one, the next tile's B = [U; Cf] and Jacobian
// coefficients travel straight from memory into a second LDS buffer
// (global_load_lds: no registers, no wait until the tile starts), so the
// matrix cores do not sit idle on the loads.  LDS: Qt / Q [3 nu][80], B
// [Kp][80], two geometry buffers, reference coordinates.  Same arithmetic,
// same bits as gradflux_kernel.
template <int ET, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(ET == 0 ? 4 : 2))) void gradflux_stream_kernel(GradFluxArgs<float> a, int tiles_per_wg) {
    using v4 = floatx4;
    constexpr int NE = 16, W5 = 80, NB = 5;
    constexpr int NG = n_geom_coeffs<ET>();
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int Kp = 4 * a.G.Kb;
    const int nu = a.nu, nf = a.nf;
    float *QT = reinterpret_cast<float *>(lds_raw);      // [3 nu][W5]
    float *Bs = QT + size_t(3 * nu) * W5;                // [Kp][W5]
    float *Gs = Bs + size_t(Kp) * W5;                    // [2][NG][NE]
    float *Xs = Gs + 2 * NG * NE;                        // [nu][3]

    const int64_t ntiles = (a.nelem + NE - 1) / NE;
    const int64_t t_begin = int64_t(xcd_block()) * tiles_per_wg;
    const int64_t t_end = min(t_begin + tiles_per_wg, ntiles);
    if (t_begin >= t_end) return;                        // whole workgroup
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int krow = lane >> 4, c16 = lane & 15;
    const int64_t ld = a.ld;

    // rows of B past K stay zero (the direct loads skip them)
    for (int idx = tid; idx < (Kp - nu - nf) * W5; idx += 64 * NW) Bs[(nu + nf) * W5 + idx] = 0.0f;
    for (int idx = tid; idx < 3 * nu; idx += 64 * NW) Xs[idx] = a.xi[idx];

    // B and the coefficients of tile `tile` into LDS: chunk c (16 bytes) of
    // B is row k, field v, elements 4 q .. 4 q + 3 with c = 4 (5 k + v) + q;
    // lane l of a wavefront instruction writes chunk base + l
    auto issue = [&](int64_t tile, float *gdst) {
        const int64_t e0 = tile * NE;
        const int nchunk = (nu + nf) * 5 * 4;
        for (int base = w * 64; base < nchunk; base += NW * 64) {
            const int c = base + lane, q = c & 3, kv = c >> 2, v = kv % 5, k = kv / 5;
            if (c < nchunk) {
                const float *src = k < nu ? a.U + (int64_t(k) * 5 + v) * ld + e0 + 4 * q
                                          : a.Cf + (int64_t(k - nu) * 5 + v) * ld + e0 + 4 * q;
                __builtin_amdgcn_global_load_lds(src, Bs + size_t(base) * 4, 16, 0, 0);
            }
        }
        if (!a.padj && w == NW - 1) {
            // NG rows of 16 coefficients: 4 NG chunks, one instruction
            const int c = lane, g = c >> 2, q = c & 3;
            if (c < 4 * NG) __builtin_amdgcn_global_load_lds(a.geom + int64_t(g) * ld + e0 + 4 * q, gdst, 16, 0, 0);
        }
    };
    issue(t_begin, Gs);
    int buf = 0;
    for (int64_t tile = t_begin; tile < t_end; ++tile, buf ^= 1) {
        const int64_t e0 = tile * NE;
        float *G = Gs + buf * NG * NE;
        __builtin_amdgcn_s_waitcnt(0);                   // this wavefront's direct loads (and stores) are done
        __syncthreads();                                 // everyone's: B and G of this tile are in LDS

        // 1. Qt = [G_k | L_k] B -> LDS
        for (int g = w; g < a.G.nmg; g += NW) {
            v4 acc[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[n] = v4{0, 0, 0, 0};
            step_products<float, NB>(a.G, g, lane, [&](int kb) { return Bs + (4 * kb + krow) * W5 + c16; }, acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = a.G.rowmap[16 * g + acc_row<float>(krow, r)];
                if (row >= 0) {
#pragma unroll
                    for (int n = 0; n < NB; ++n) QT[row * W5 + 16 * n + c16] = acc[n][r];
                }
            }
        }
        __syncthreads();                                 // B is free, Qt complete
        if (tile + 1 < t_end) issue(tile + 1, Gs + (buf ^ 1) * NG * NE);

        // 2. point-wise: Q replaces Qt in place, Ft to memory
        for (int it = tid; it < nu * NE; it += 64 * NW) {
            const int i = it / NE, e = it - i * NE;
            const int64_t eg = e0 + e;
            if (eg >= a.nelem) continue;
            float adj[3][3], Jinv;
            if (a.padj) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < 3; ++j) adj[k][j] = a.padj[(int64_t(3 * k + j) * nu + i) * ld + eg];
                Jinv = a.pjinv[int64_t(i) * ld + eg];
            } else {
                Jinv = 1.0f / metric<float, ET>(G, NE, e, Xs + 3 * i, adj);
            }
            float u[5], qt[3][5], q[3][5], Ft[3][5];
#pragma unroll
            for (int v = 0; v < 5; ++v) u[v] = a.U[(int64_t(i) * 5 + v) * ld + eg];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) qt[k][v] = QT[(k * nu + i) * W5 + v * NE + e];
            upts_point<float, true>(u, qt, adj, Jinv, a.gamma, a.mu, a.prandtl, a.pref, q, Ft);
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int v = 0; v < 5; ++v) QT[(j * nu + i) * W5 + v * NE + e] = q[j][v];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) a.Ft[((int64_t(k) * nu + i) * 5 + v) * ld + eg] = Ft[k][v];
        }
        __syncthreads();

        // 3. Qf = M0 Q (the faces whose gradient is read, as above)
        const unsigned qm = a.qmask ? unsigned(a.qmask[e0 + c16]) : 0xffu;
        for (int it = w; it < a.M.nmg * 3; it += NW) {
            const int g = it / 3, j = it - 3 * g;
            const float *Qj = QT + size_t(j) * nu * W5 + c16;
            v4 acc2[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n) acc2[n] = v4{0, 0, 0, 0};
            step_products<float, NB>(a.M, g, lane, [&](int kb) { return Qj + min(4 * kb + krow, nu - 1) * W5; },
                                     acc2);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int slot = 16 * g + acc_row<float>(krow, r), f = a.M.rowmap[slot];
                if (f < 0 || e0 + c16 >= a.nelem || (a.qmask && !(qm & a.fbit[slot]))) continue;
#pragma unroll
                for (int n = 0; n < NB; ++n) a.Qf[(int64_t(f) * 15 + j * 5 + n) * ld + e0 + c16] = acc2[n][r];
            }
        }
        // the next iteration's barrier keeps Qt of the next tile from
        // overwriting Q while it is read here
    }
}


template <typename T, int ET, int NE, int NW, int MG>
hipError_t launch_gf_mg(const GradFluxArgs<T> &a, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(gradflux_kernel<T, ET, NE, NW, MG>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(GRADFLUX_LDS_MAX));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t ntiles = (a.nelem + NE - 1) / NE;
    gradflux_kernel<T, ET, NE, NW, MG><<<xcd_grid(ntiles), 64 * NW, lds, s>>>(a);
    return hipGetLastError();
}

template <typename T, int ET, int NE, int NW>
hipError_t launch_gf(const GradFluxArgs<T> &a, size_t lds, hipStream_t s) {
    const int mg = (a.G.nmg + NW - 1) / NW;
    if (mg <= 1) return launch_gf_mg<T, ET, NE, NW, 1>(a, lds, s);
    if (mg <= 2) return launch_gf_mg<T, ET, NE, NW, 2>(a, lds, s);
    if (mg <= 4) return launch_gf_mg<T, ET, NE, NW, 4>(a, lds, s);
    return hipErrorInvalidValue;
}

size_t gradflux_stream_lds_bytes(int etype, const GradFluxArgs<float> &a) {
    const int ng = etype == 0 ? 9 : 15;
    return (size_t(3 * a.nu) * 80 + size_t(4 * a.G.Kb) * 80 + 2 * size_t(ng) * 16 + size_t(3 * a.nu)) * 4;
}

template <int ET, int NW>
hipError_t launch_gf_stream(const GradFluxArgs<float> &a, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    static int ncu = 0;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(gradflux_stream_kernel<ET, NW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(GRADFLUX_LDS_MAX));
        if (e != hipSuccess) return e;
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        attr_set = true;
    }
    // as many workgroups as fit at once (LDS-bound), each a contiguous run of tiles
    const int per_cu = std::max(1, int(GRADFLUX_LDS_MAX / lds));
    const int64_t ntiles = (a.nelem + 15) / 16;
    int64_t nwg = std::min<int64_t>(ntiles, int64_t(ncu) * per_cu);
    const int tiles_per_wg = int((ntiles + nwg - 1) / nwg);
    nwg = (ntiles + tiles_per_wg - 1) / tiles_per_wg;
    gradflux_stream_kernel<ET, NW><<<xcd_grid(nwg), 64 * NW, lds, s>>>(a, tiles_per_wg);
    return hipGetLastError();
}

}  // namespace

namespace {
template <typename T, int ET>
size_t gradflux_lds_t(const GradFluxArgs<T> &a) {
    constexpr int NE = tile_elems<T, ET>();
    constexpr int W5 = TileShape<NE>::W5;
    const size_t n = size_t(std::max(4 * a.G.Kb, 3 * a.nu)) * W5 + size_t(n_geom_coeffs<ET>()) * NE +
                     size_t(3 * a.nu);
    const size_t bytes = n * sizeof(T);
    return bytes <= GRADFLUX_LDS_MAX ? bytes : 0;
}
}  // namespace

template <typename T>
size_t gradflux_lds(int etype, const GradFluxArgs<T> &a) {
    return etype == 0 ? gradflux_lds_t<T, 0>(a) : etype == 1 ? gradflux_lds_t<T, 1>(a)
                                                : etype == 2 ? gradflux_lds_t<T, 2>(a) : 0;
}

template <typename T>
hipError_t launch_gradflux(int etype, const GradFluxArgs<T> &a, hipStream_t s, bool stream) {
    size_t lds = gradflux_lds<T>(etype, a);
    if constexpr (std::is_same<T, float>::value) {
        if (stream) {
            if (etype > 1) return hipErrorInvalidValue;   // the streaming form covers tets and prisms
            lds = gradflux_stream_lds_bytes(etype, a);
            if (lds > GRADFLUX_LDS_MAX) return hipErrorInvalidValue;
        }
    } else {
        if (stream) return hipErrorInvalidValue;
    }
    // operator layout: step lists (4 steps in flight), one row block per group
    if (!lds || a.G.stage != 6 || a.M.stage != 6 || a.G.mbw != 1 || a.M.mbw != 1 || !a.G.klist ||
        !a.G.koff || !a.G.rowmap || !a.M.klist || !a.M.koff || !a.M.rowmap || a.G.M != 3 * a.nu ||
        a.M.M != a.nf || 4 * a.G.Kb < a.nu + a.nf || 4 * a.M.Kb < a.nu || a.ld % 64 || a.nelem > a.ld ||
        (reinterpret_cast<uintptr_t>(a.U) | reinterpret_cast<uintptr_t>(a.Cf) |
         reinterpret_cast<uintptr_t>(a.geom)) % 16 ||
        reinterpret_cast<uintptr_t>(a.xi) % 4)   // 16- and 4-byte direct loads into LDS
        return hipErrorInvalidValue;
    if (!a.nelem) return hipSuccess;
    if constexpr (std::is_same<T, float>::value) {
        if (stream) return etype == 0 ? launch_gf_stream<0, 8>(a, lds, s) : launch_gf_stream<1, 8>(a, lds, s);
    }
    // wavefronts per workgroup: tets 8 in FP32 (7 row blocks of the
    // gradient operator at p = 4), prisms 16 (15 row blocks), hexahedra 16
    // (24: two per wavefront); FP64 4, 4 and 8
    if (etype == 0) return launch_gf<T, 0, tile_elems<T, 0>(), sizeof(T) == 4 ? 8 : 4>(a, lds, s);
    if (etype == 1) return launch_gf<T, 1, tile_elems<T, 1>(), sizeof(T) == 4 ? 16 : 4>(a, lds, s);
    return launch_gf<T, 2, tile_elems<T, 2>(), sizeof(T) == 4 ? 16 : 8>(a, lds, s);
}

template size_t gradflux_lds<float>(int, const GradFluxArgs<float> &);
template size_t gradflux_lds<double>(int, const GradFluxArgs<double> &);
template hipError_t launch_gradflux<float>(int, const GradFluxArgs<float> &, hipStream_t, bool);
template hipError_t launch_gradflux<double>(int, const GradFluxArgs<double> &, hipStream_t, bool);

}  // namespace frd
