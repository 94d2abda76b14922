/*
 * fr.h - C ABI of the MI355X flux reconstruction (FR) right-hand-side library.
 *
 * The library evaluates the FR right-hand side of the compressible Euler and
 * Navier-Stokes equations (constant viscosity) on mixed tetrahedral / prismatic
 * / hexahedral periodic grids, and advances it with explicit Runge-Kutta schemes.  The
 * operations follow the paper "Heterogeneous Computing on Mixed Unstructured
 * Grids with PyFR" (Witherden, Vermeire, Vincent):
 *   - Section 2.1: an FR step is mostly products C <- c1 A B + c2 C of a
 *     constant operator matrix A with row-major state matrices B, C, plus
 *     point-wise operations at solution and flux points; Table 2 gives the
 *     dimensions of the volume-to-surface interpolation operator M0;
 *   - Section 3.4: DG-type spatial scheme, Rusanov interface flux, RK45[2R+];
 *   - Table 1: element types, arbitrary order, Euler / RK4 / RK45 steppers,
 *     single and double precision, Euler and Navier-Stokes systems.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Element types: FR_TET = 0, FR_PRI = 1, FR_HEX = 2.  Global element ids are
 * type-major (tets, then prisms, then hexahedra).  Solution state per type is a device array laid out
 * [n_upts][5][ld] of the mesh's scalar type (double for FR_FP64, float for
 * every other precision): point-major, then the conserved field (rho, rho u, rho v, rho w,
 * E), then the element index, fastest; ld >= n_elem is a multiple of 64 and
 * is reported by fr_mesh_query.  Columns n_elem..ld-1 are padding: they are
 * read and written but never mix with real elements.
 *
 * Ownership: fr_mesh_create allocates every device buffer the mesh needs
 * (operators, geometry, interface tables, intermediates, Runge-Kutta
 * registers); fr_rhs and fr_rk_step allocate nothing.  Pointers passed in are
 * borrowed for the duration of the call (host arrays) or of the enqueued work
 * (device arrays).
 *
 * Streams: every entry point that takes a `stream` (a hipStream_t, NULL for the
 * default stream) enqueues its work there and returns without waiting, except
 * fr_reduce and fr_mesh_destroy, which synchronise the stream.
 *
 * Errors: every call returns an fr_status; no exception crosses the ABI.
 * fr_last_error(mesh) returns a message for the last failure on that mesh
 * (fr_last_error(NULL): the last failure of fr_mesh_create on this thread).
 * An asynchronous device fault surfaces as FR_ERR_DEVICE on a later call.
 */
#ifndef FR_H
#define FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FR_OK = 0,
    FR_ERR_INVALID_ARG = 1,   /* NULL pointer, unknown enum, wrong sizes */
    FR_ERR_BAD_MESH = 2,      /* J <= 0, unmatched or non-conforming face */
    FR_ERR_UNSUPPORTED = 3,   /* order outside 1..4, precision not built */
    FR_ERR_OUT_OF_MEMORY = 4, /* device allocation failed */
    FR_ERR_DEVICE = 5,        /* HIP runtime error */
    FR_ERR_NONFINITE = 6      /* FR_CHECK_FINITE found a NaN / Inf */
} fr_status;

typedef enum { FR_TET = 0, FR_PRI = 1, FR_HEX = 2 } fr_etype;
/* Number of element types: arrays indexed by element type have this length. */
#define FR_NTYPES 3
typedef enum { FR_EULER = 0, FR_NAVIER_STOKES = 1 } fr_system;
/* FR_SPLIT_BF16 / FR_SPLIT_FP16: FP32 state and point-wise arithmetic; the
 * operator products run on the 16-bit matrix cores with both operands split
 * into 16-bit parts and FP32 accumulation: BF16 three parts (six products,
 * ~24-bit operands), FP16 two parts (three products, ~22-bit operands; the
 * state must stay below 65504 in magnitude). */
typedef enum { FR_FP32 = 0, FR_FP64 = 1, FR_SPLIT_BF16 = 2, FR_SPLIT_FP16 = 3 } fr_precision;
typedef enum { FR_RK4 = 0, FR_RK45_2RP = 1, FR_FWD_EULER = 2 } fr_scheme;

/* fr_mesh_desc.bfaces kinds */
#define FR_BC_WALL 1
#define FR_BC_FARFIELD 2

/* fr_mesh_desc.flags */
#define FR_VALIDATE_ONLY 0x1u  /* build host-side tables only; no device work */
#define FR_CHECK_FINITE 0x2u   /* fr_rk_step ends with a finiteness check */
/* Run -R~/J and the RK register update as a kernel of their own after the
 * divergence product.  By default (every precision, no closure) they are
 * applied in the divergence product's store, so R~ is never written; both
 * orders of work give the same bits.  The autotuner times the divergence
 * products the way the right-hand side runs them. */
#define FR_SEPARATE_UPDATE 0x4u
/* Navier-Stokes in FP32 / FP64: run the corrected gradient
 * product, the solution-point work (physical gradient, transformed flux) and
 * the gradient interpolation as three kernels that pass the reference and
 * physical gradients through memory.  By default one kernel does all three
 * per tile of elements with those gradients in LDS wherever the gradient
 * operator has at least four 16-row blocks (tets from p = 3, prisms and
 * hexahedra from p = 2), the three kernels below that; fr_autotune then
 * keeps whichever form is fastest per element type.  All give the same
 * bits. */
#define FR_SEPARATE_GRADIENT 0x8u

typedef struct fr_mesh_s *fr_mesh;   /* opaque, library-owned */

/*
 * Mesh and physics description (host memory, read during fr_mesh_create).
 *
 * order      polynomial order p of the solution, 1..4 on the GPU (Table 2).
 * system     FR_EULER or FR_NAVIER_STOKES (Section 3.4, Table 1).
 * precision  scalar type of the state and of the device arithmetic (the split
 *            forms keep an FP32 state).
 * gamma      ratio of specific heats; mu dynamic viscosity (ignored for
 *            Euler); prandtl Prandtl number; ldg_beta, ldg_tau the LDG switch
 *            and penalty of the viscous interface flux.
 * xyz        [n_vertices][3] vertex coordinates.
 * tet_v      [n_tets][4] vertex ids; prism vertex ids pri_v [n_prisms][6] list
 *            the bottom triangle 0-2 (counter-clockwise seen from above) and
 *            then the top 3-5, vertex k+3 above vertex k; hexahedron vertex
 *            ids hex_v [n_hex][8] list the bottom quad 0-3 (counter-clockwise
 *            seen from above) and then the top 4-7, vertex k+4 above vertex k
 *            (trilinear map; Table 2 gives its operator sizes).
 * tet_img, pri_img, hex_img  periodic image shift per element vertex
 *            [..][n][3] (int8, unwrapped vertex = xyz[v] + img * period), or
 *            NULL for none.
 *            At most 2^22 - 1 elements of each type; faces between elements
 *            must be conforming (a hexahedron meets prisms through their
 *            quadrilateral faces).
 * period     box lengths of the periodic directions (used with the images);
 *            0 for a direction that is not periodic.
 * bfaces     [n_bfaces][4] boundary faces: (element type, element index,
 *            local face, kind FR_BC_WALL / FR_BC_FARFIELD), or NULL.  Local
 *            faces by vertex positions: tet (0,1,2) (0,1,3) (0,2,3) (1,2,3);
 *            prism (0,1,2) (3,4,5) (0,1,4,3) (1,2,5,4) (2,0,3,5); hexahedron
 *            (0,1,2,3) (4,5,6,7) (0,1,5,4) (1,2,6,5) (2,3,7,6) (3,0,4,7).
 *            Every face that meets no other element must be listed.
 *            Section 3.2 names the two kinds (no-slip isothermal wall at the
 *            body, Riemann invariants at the far field); both are imposed
 *            weakly through a boundary state Ub (the LDG common solution and
 *            the state of the viscous flux, with the interior gradient) and a
 *            ghost state (the right state of the Rusanov flux), temperature
 *            meaning p / rho:
 *              wall: Ub = (rho, 0, 0, 0, rho t_wall / (gamma - 1)), ghost =
 *                the interior velocity mirrored at the wall temperature;
 *              far field: v.n and the sound speed from the outgoing invariant
 *                of the interior and the incoming one of the free stream,
 *                entropy and tangential velocity from the upwind side;
 *                ghost = Ub.
 *            The common flux adds, for Navier-Stokes, -Fv(Ub, Q).n +
 *            ldg_tau (U - Ub).
 * t_wall     wall temperature p / rho (> 0 when there are wall faces).
 * farfield   free stream (rho, u, v, w, p) of the far-field faces.
 * tet_q, pri_q, hex_q  quadratically curved elements of that type (Section
 *            3.3): [n][nq][3] unwrapped positions of the nodes of each
 *            element's order-2 lattice, or NULL for straight-sided elements.
 *            nq = 10 tet, lattice (a, b, c) with a + b + c <= 2; 18 prism,
 *            (a, b) with a + b <= 2 times c <= 2; 27 hexahedron, (a, b, c)
 *            <= 2; node at reference point (-1 + a, -1 + b, -1 + c), c
 *            outermost and a innermost.  The geometry is the quadratic
 *            Lagrange interpolant of the nodes; the vertex nodes must agree
 *            with xyz (and the images), neighbours must share face nodes.
 *            The metric terms are then stored per solution point (9 + 1
 *            values).
 * p_ref      reference pressure taken out of the pressure term of the
 *            momentum flux, in the volume flux and in the interface and
 *            boundary fluxes alike (0: the plain flux).  The flux of a
 *            uniform state has zero discrete divergence on a mesh that
 *            preserves such a state (every straight-sided mesh; curved ones
 *            at the orders where the metric terms are interpolated exactly),
 *            so the residual is unchanged in exact arithmetic, while single
 *            precision no longer rounds the large constant part of the
 *            pressure gradient at low Mach number.  A batch takes it from its
 *            first description (all must agree).
 */
typedef struct {
    int32_t order;
    int32_t system;
    int32_t precision;
    uint32_t flags;
    double gamma, mu, prandtl, ldg_beta, ldg_tau;
    int64_t n_vertices;
    const double *xyz;
    int64_t n_tets;
    const int64_t *tet_v;
    const int8_t *tet_img;
    int64_t n_prisms;
    const int64_t *pri_v;
    const int8_t *pri_img;
    double period[3];
    int64_t n_hex;
    const int64_t *hex_v;
    const int8_t *hex_img;
    int64_t n_bfaces;
    const int64_t *bfaces;
    double t_wall;
    double farfield[5];
    const double *tet_q, *pri_q, *hex_q;
    double p_ref;
} fr_mesh_desc;

/* Build operators (FP64 on the host), geometry and the interface pairing,
 * allocate and upload every device buffer.  Errors: FR_ERR_INVALID_ARG,
 * FR_ERR_BAD_MESH (message names the element / face), FR_ERR_UNSUPPORTED,
 * FR_ERR_OUT_OF_MEMORY, FR_ERR_DEVICE.  With FR_VALIDATE_ONLY no HIP call is
 * made; only fr_mesh_query, fr_upts_coords, fr_operator and fr_mesh_destroy
 * may then be used. */
fr_status fr_mesh_create(const fr_mesh_desc *desc, void *stream, fr_mesh *out);

/* Free the mesh and its device buffers (synchronises the stream it was
 * created on).  NULL is accepted. */
fr_status fr_mesh_destroy(fr_mesh mesh);

/* Element count, solution points per element and leading dimension ld of
 * one element type (n_elem = 0 when the mesh has none). */
fr_status fr_mesh_query(fr_mesh mesh, int32_t etype, int64_t *n_elem,
                        int32_t *n_upts, int32_t *n_fpts, int64_t *ld);

/* Physical solution-point positions, host array [n_upts][3][n_elem]. */
fr_status fr_upts_coords(fr_mesh mesh, int32_t etype, double *xyz_host);

/* Copy a host-built FP64 operator of one element type to a host array of
 * rows*cols doubles, row-major.  which: 0 = M0 (n_fpts x n_upts), 1..3 =
 * gradient d/dxi_k (n_upts x n_upts), 4 = correction lift L (n_upts x n_fpts),
 * 5 = quadrature weights (1 x n_upts), 6 = outward unit normals of the
 * reference faces at the flux points (n_fpts x 3).  out may be NULL to query
 * the shape. */
fr_status fr_operator(fr_mesh mesh, int32_t etype, int32_t which, double *out,
                      int32_t *rows, int32_t *cols);

/* Copy a caller device state of one type into / out of the mesh's solution
 * register (the state fr_rk_step advances).  u_dev is [n_upts][5][ld]. */
fr_status fr_set_solution(fr_mesh mesh, int32_t etype, const void *u_dev, void *stream);
fr_status fr_get_solution(fr_mesh mesh, int32_t etype, void *u_dev, void *stream);

/* One right-hand-side evaluation R = dU/dt (Section 2.1 operator products and
 * point-wise kernels, Section 3.4 scheme).  u_dev[t] / r_dev[t] are the
 * caller's device states of type t ([n_upts][5][ld]); entries of types the
 * mesh does not have are ignored and may be NULL.  r_dev must not alias u_dev. */
fr_status fr_rhs(fr_mesh mesh, const void *const u_dev[FR_NTYPES], void *const r_dev[FR_NTYPES],
                 void *stream);

/* Advance the mesh's solution register n_steps steps of size dt with the
 * given scheme (Table 1; FR_RK45_2RP is the two-register RK45[2R+] of Section
 * 3.4, fixed step).  With FR_CHECK_FINITE set at create, ends with a device
 * reduction and returns FR_ERR_NONFINITE if any value is NaN / Inf (this
 * synchronises the stream). */
fr_status fr_rk_step(fr_mesh mesh, int32_t scheme, double dt, int32_t n_steps,
                     void *stream);

/* Adaptive RK45[2R+]: advance the solution register from state[0] (time) to
 * t_end with error control by the scheme's embedded third-order solution
 * (Section 3.4 names the scheme; the controller is this library's reading).
 * Per attempt: e = dt sum_i (b_i - bhat_i) k_i accumulated in a third
 * register; err = RMS over all values of e / (atol + rtol max(|u_old|,
 * |u_new|)), summed in FP64 on the device; accepted if err <= 1.  Step size:
 * accepted dt * clamp(0.9 err^(-0.7/4) err_prev^(0.4/4), 0.2, 5), err_prev =
 * max(err, 1e-4); rejected (the step is undone) dt * clamp(0.9 err^(-1/4),
 * 0.2, 1); the last step is cut to land on t_end exactly.
 * state: in/out {t, dt (next proposed step), err_prev (1 to start)}.
 * counts: out {accepted, rejected}.  Stops at t_end or after max_attempts
 * attempts.  Synchronises the stream once per attempt.  Allocates the error
 * register on first use.  FR_ERR_NONFINITE (step undone) if the error
 * estimate is not finite. */
fr_status fr_rk45_adaptive(fr_mesh mesh, double t_end, double state[3], double atol, double rtol,
                           int32_t max_attempts, int32_t counts[2], void *stream);

/* Global FP64 reductions over the mesh's solution register U (and, for the
 * residual items, over R(U), evaluated here).  Integrals use the element
 * quadrature: int f = sum_e sum_i w_i J_ei f_ei.  `what` selects one item:
 *   FR_RED_INT_U      5 doubles: integral of each conserved field
 *   FR_RED_INT_R      5 doubles: integral of each field of R(U) (zero on a
 *                     periodic mesh up to rounding: discrete conservation)
 *   FR_RED_NORM2_R    5 doubles: integral of R(U)^2 per field
 *   FR_RED_KE         2 doubles: mean kinetic energy and its rate d/dt
 *                     (from R(U)), both divided by the mesh volume
 * Synchronises the stream. */
#define FR_RED_INT_U 1
#define FR_RED_INT_R 2
#define FR_RED_NORM2_R 3
#define FR_RED_KE 4
fr_status fr_reduce(fr_mesh mesh, int32_t what, double *out_host, void *stream);

/* fr_reduce for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same items, arguments, kernels and results (bitwise), but the partial
 * sums and the results live in a device array of the library's own, one per
 * GPU, held until the process ends: 3 x (512 x 8 + 8) doubles (98.5 KB),
 * enough for any mesh (the reduction's grid is fixed per element type).  The call allocates nothing.  The
 * array's address on the current device is looked up on its first use there.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (other threads, other streams) race; calls on different GPUs do not.
 * Synchronises the stream.  Errors: as fr_reduce, FR_ERR_DEVICE if the
 * array's address cannot be found. */
fr_status fr_reduce_noalloc(fr_mesh mesh, int32_t what, double *out_host, void *stream);

/* Copy an interface intermediate of the last fr_rhs into a caller device
 * array of the mesh's scalar type, layout [n_fpts][nvar][ld]:
 *   which 0: state at flux points U_f (nvar 5)
 *         1: common normal flux, transformed (nvar 5)
 *         2: physical gradient at flux points (NS only; nvar 15, direction
 *            major: index j*5 + field).  The fused gradient stage (FP32
 *            and FP64, where it runs) writes
 *            it only on the faces whose gradient the common flux reads:
 *            boundary faces, and the sides of an interface whose LDG weight
 *            1/2 +- beta is not zero (with beta = 1/2 side L only); the
 *            other points keep what they held before. */
fr_status fr_intermediate(fr_mesh mesh, int32_t etype, int32_t which, void *dst_dev,
                          void *stream);

/* Per-kernel timing with HIP events (measurement support).  While enabled,
 * every kernel the library launches is bracketed by two HIP events recorded
 * on its stream.  fr_profile(mesh, 1) enables and clears, 0 disables.
 * fr_profile_read waits for the recorded events, writes per kernel class the
 * summed duration in milliseconds and the launch count (arrays of
 * FR_PROF_NCLASS), and clears the records.  Classes: 4 * etype + op for the
 * operator products of tets and prisms (op 0 interpolation to flux points, 1
 * corrected gradient, 2 gradient interpolation, 3 divergence plus
 * correction), 8 + etype the solution-point flux kernel, 10 common solution,
 * 11 common interface flux, 12 + etype negdivconf with the Runge-Kutta
 * update, 14 closure inputs (moments and neighbour gathering), 15 closure
 * network forward; hexahedra: 16 + op the products, 20 the solution-point
 * kernel, 21 negdivconf; 22 boundary states, 23 boundary flux; 24 + etype
 * the fused gradient stage of tets, prisms and hexahedra (corrected
 * gradient, point-wise work and gradient interpolation in one kernel). */
#define FR_PROF_NCLASS 27
fr_status fr_profile(fr_mesh mesh, int32_t enable);
fr_status fr_profile_read(fr_mesh mesh, double *total_ms, int64_t *count);

/* Operator-product autotuner: for every operator of every element type,
 * time the row-blocking candidates (16-row blocks per wavefront) on this
 * mesh's buffers and keep the fastest.  Results are bitwise unchanged (the
 * blocking does not change any output's accumulation order).  Synchronises
 * the stream; the choice is reported by fr_last_error(mesh) on success. */
fr_status fr_autotune(fr_mesh mesh, void *stream);

/* Force the operator-product variant of one operator of one element type:
 * op 0 interpolation, 1 corrected gradient, 2 gradient interpolation,
 * 3 divergence; cap = most 16-row blocks per wavefront (1..8 FP32, 1..4
 * FP64 and split BF16, 1..2 split FP16); stage 0 / 3 = direct B loads with
 * 2 / 4 K steps in flight, 1 / 2 = B staged through LDS in chunks of 4 / 8 K
 * steps (FP32 only, at most 8 row groups), 4 = the operator's row-group slice
 * held in LDS for four panels (FP32 only, at most 64 KiB of it), 5 = direct
 * loads over only the K steps where the row group's operator fragments are
 * nonzero (the structural zeros of prisms and hexahedra; at most 4 row
 * blocks per wavefront), 6 = the same with 4 instead of 2 K steps of loads
 * in flight.  The split forms have stage 0 (each wavefront splits
 * its B panel) and 1 (the panel's row groups, at most 8 and 64 KiB of parts,
 * share the split B in LDS).  op 4 selects the form of the Navier-Stokes
 * gradient stage (FP32 and FP64; cap ignored): stage 0 the three separate
 * kernels, 1 one fused kernel per tile of elements, 2 (FP32 tets and
 * prisms) the fused kernel streaming runs of tiles with the next tile's
 * input loaded into LDS during the current one.  Results are bitwise the same for every
 * variant (for finite states).  Synchronous
 * (uploads the operator); FR_ERR_UNSUPPORTED for a combination the form
 * does not have. */
fr_status fr_set_blocking(fr_mesh mesh, int32_t etype, int32_t op, int32_t cap, int32_t stage);

/* ------------------------------------------------------------------------
 * Batches of independent problems (many small meshes, mixed orders).
 *
 * fr_batch_create builds each problem's operators, geometry and pairing,
 * then merges the problems of one order into one element array per type
 * (elements are independent and interfaces pair only within a problem, so
 * the merged right-hand side equals the per-problem ones).  All problems
 * must share system, precision and physical constants; orders 1..4 may mix.
 * Every merged group is autotuned at creation.  The batch owns all buffers.
 *
 * Per-problem states use the same layout as a single mesh of that problem:
 * [n_upts][5][ld] with ld from fr_batch_query.  fr_batch_set_dt sets one step
 * size per problem (host array of n doubles).  fr_batch_rk_step advances every
 * problem n_steps steps on `stream`; with graphs enabled (the default) an
 * RK45[2R+] step of all groups is captured once as a HIP graph and replayed
 * (one graph launch per step).  Errors as for meshes; messages from
 * fr_batch_last_error. */
typedef struct fr_batch_s *fr_batch;
fr_status fr_batch_create(int32_t n, const fr_mesh_desc *descs, void *stream, fr_batch *out);
fr_status fr_batch_destroy(fr_batch batch);
fr_status fr_batch_query(fr_batch batch, int32_t problem, int32_t etype, int64_t *n_elem,
                         int32_t *n_upts, int64_t *ld);
/* Physical solution-point positions of one problem, host [n_upts][3][n_elem]. */
fr_status fr_batch_upts_coords(fr_batch batch, int32_t problem, int32_t etype, double *xyz_host);
fr_status fr_batch_set_solution(fr_batch batch, int32_t problem, int32_t etype,
                                const void *u_dev, void *stream);
fr_status fr_batch_get_solution(fr_batch batch, int32_t problem, int32_t etype, void *u_dev,
                                void *stream);
fr_status fr_batch_set_dt(fr_batch batch, const double *dt_host, void *stream);
fr_status fr_batch_set_graph(fr_batch batch, int32_t enable);
fr_status fr_batch_rk_step(fr_batch batch, int32_t scheme, int32_t n_steps, void *stream);
const char *fr_batch_last_error(fr_batch batch);

/* ------------------------------------------------------------------------
 * Learned closure (low-order meshes) and its network.
 *
 * The closure adds to the residual of a mesh the P1 part of a correction
 * predicted per element by a fully connected network, 120 -> 64 -> 64 -> 20
 * with tanh, from the P1 moments of the element and of its face neighbours.
 * P1 moments of a field: m_a = integral over the reference element of
 * phi_a u, phi_a the Gram-Schmidt orthonormalisation of (1, xi, eta, zeta) in
 * that order.  Network inputs, element g (type-major), 120 floats: the 5 x 4
 * moments of g (field-major), then those of the neighbours across local
 * faces 0..4 (zeros where a tet has no fifth face).  Outputs: 5 x 4 moments
 * of the residual correction, lifted to the solution points as
 * sum_a phi_a(x_i) y_a.  Parameters (FP32, FR_MLP_NPARAM floats): W1 [64][120],
 * b1 [64], W2 [64][64], b2 [64], W3 [20][64], b3 [20].  Statistics
 * (FR_MLP_NSTATS floats): mu_x [120], s_x [120], mu_y [20], s_y [20]; inputs
 * are normalised as (x - mu_x) / s_x and outputs scaled back as y s_y + mu_y.
 */
#define FR_MLP_NPARAM 13204
#define FR_MLP_NSTATS 280
typedef struct fr_mlp_s *fr_mlp;
/* Network with seeded initial weights, Adam state and gradient workspace. */
fr_status fr_mlp_create(uint64_t seed, fr_mlp *out);
fr_status fr_mlp_destroy(fr_mlp net);
fr_status fr_mlp_set_params(fr_mlp net, const float *params_host);
fr_status fr_mlp_get_params(fr_mlp net, float *params_host);
/* y[n][20] = network(x[n][120]) on the device.  With stats_dev, x is
 * standardised (x - mu_x) / s_x as it is read and y scaled back y s_y + mu_y
 * (the same convention as fr_mlp_grad); NULL: raw in and out.
 * bf16_weights: use the weights rounded to BF16 (FP32 accumulation). */
fr_status fr_mlp_forward(fr_mlp net, const float *x_dev, int64_t n, const float *stats_dev,
                         float *y_dev, int32_t bf16_weights, void *stream);
/* Gradient of L = sum_s |y_s - t_s|^2 / n (FP32 weights) over the rows
 * idx_dev[0..n) of x_dev / t_dev (idx_dev NULL: rows 0..n).  With stats_dev,
 * rows are standardised as they are read: x by (mu_x, s_x), t by (mu_y, s_y)
 * (the loss is then that of the normalised targets).  The loss is written to
 * *loss_host if not NULL (this synchronises the stream).  The gradient stays
 * in the network's workspace for fr_mlp_get_grad / fr_mlp_adam. */
fr_status fr_mlp_grad(fr_mlp net, const float *x_dev, const float *t_dev, const int32_t *idx_dev,
                      int64_t n, const float *stats_dev, double *loss_host, void *stream);
fr_status fr_mlp_get_grad(fr_mlp net, float *grad_host, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the last gradient. */
fr_status fr_mlp_adam(fr_mlp net, float lr, void *stream);
const char *fr_mlp_last_error(fr_mlp net);

/* L2 projection (reference element) of a state of mesh src, order p, to the
 * order q of mesh dst; both meshes have the same elements and scalar type.
 * States [n_upts][5][ld] of each mesh.  Allocates its operators on first use. */
fr_status fr_project(fr_mesh src, const void *const u_src[FR_NTYPES], fr_mesh dst,
                     void *const u_dst[FR_NTYPES], void *stream);
/* P1 moments [n_tet + n_pri][20] of a state, and the network inputs
 * [n_tet + n_pri][120] (normalised with stats_dev unless NULL).  The closure
 * is defined on tet and prism meshes: a mesh with hexahedra gives
 * FR_ERR_UNSUPPORTED here and in fr_closure_targets / fr_closure_attach
 * (entry FR_HEX of the state arrays is ignored). */
fr_status fr_closure_moments(fr_mesh mesh, const void *const u_dev[FR_NTYPES], float *mom_dev, void *stream);
fr_status fr_closure_features(fr_mesh mesh, const void *const u_dev[FR_NTYPES], const float *stats_dev,
                              float *feat_dev, void *stream);
/* Network targets [n_tet + n_pri][20]: P1 moments of a_dev - b_dev,
 * normalised as (m - mu_y) / s_y with stats_dev unless NULL. */
fr_status fr_closure_targets(fr_mesh mesh, const void *const a_dev[FR_NTYPES], const void *const b_dev[FR_NTYPES],
                             const float *stats_dev, float *out_dev, void *stream);
/* Attach (net != NULL) or detach (net == NULL) the closure: every later
 * fr_rhs / fr_rk_step of this mesh adds the lifted network correction to the
 * residual.  net and stats_dev stay owned by the caller and must outlive the
 * attachment. */
fr_status fr_closure_attach(fr_mesh mesh, fr_mlp net, const float *stats_dev, int32_t bf16_weights);

/* Message of the last failure on mesh (NULL: of fr_mesh_create on this
 * thread).  Never NULL; valid until the next call on the same mesh. */
const char *fr_last_error(fr_mesh mesh);

#ifdef __cplusplus
}
#endif
#endif /* FR_H */
