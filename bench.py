#!/usr/bin/env python3
"""Throughput of the FR right-hand side on one MI355X.

Workload: compressible Navier-Stokes (Re 1600, Ma 0.1, Pr 0.71), Taylor-Green
initial state, order p = 4, FP32, on the periodic [0, 2 pi)^3 box with
110,592 prisms (z < pi) and 196,608 tets (z > pi), vertices jittered by 10 %
(seed 0); Rusanov + LDG interface fluxes.

One step = one RK45[2R+] step (five right-hand-side evaluations with the
fused register updates) plus the FP64 conservation integral of the solution.
The reported value is GDOF/s per right-hand-side evaluation:
5 * n_dof * steps / wall time, n_dof = solution points x 5 fields.

Also reported: the roofline of the dominant kernel (per-kernel HIP event
timing on the library's stream, in a separate instrumented pass over the same
steps), the FP64 oracle's throughput on a bounded sample of the same
workload on the host CPU, and the split-precision forms (16-bit matrix-core
operator products) with their speedup over FP32 and the relative L2 error of
their right-hand side against the FP64 build of the same kernels.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import re
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s per RHS eval, mixed prism/tet p=4, plain FP32 vs split-BF16; HBM %"
PEAK_HBM = 8.0e12          # B/s
PEAK_FP32_MFMA = 157.3e12  # FLOP/s, dense
RIDGE = PEAK_FP32_MFMA / PEAK_HBM

# HBM bytes per launch measured with rocprofv3 --pmc on this workload
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, the factors read off the state
# copies of known size), keyed (kernel class, 16-row blocks per wavefront,
# stage) for the products and (class, 0, 0) for the point-wise kernels and the
# fused gradient stage; the file below holds the commands and counts.  A
# variant not listed reports traffic null.
TRAFFIC_SOURCE = "profiles/rhs_ns_p4_tgv_mixed_hbm_counters.md"
MEASURED_TRAFFIC = {
    ('gradflux_tet', 0, 0): 1164.4e6,
    ('gradflux_pri', 0, 0): 1257.8e6,
    ('interp_tet', 2, 1): 373.8e6,
    ('interp_pri', 2, 1): 398.8e6,
    ('interp_pri', 1, 1): 398.5e6,
    ('interp_tet', 4, 0): 373.8e6,
    ('interp_tet', 2, 0): 373.7e6,
    ('div_tet', 1, 3): 995.2e6,
    ('div_tet', 1, 1): 1037.2e6,
    ('div_pri', 1, 6): 1208.7e6,
    ('common_flux', 0, 0): 1966.5e6,
    ('common_solution', 0, 0): 795.9e6,
    ('div_pri', 5, 0): 1067.5e6,
    ('div_tet', 3, 0): 926.3e6,
    ('grad_pri', 1, 0): 897.2e6,
    ('grad_pri', 1, 3): 897.3e6,
    ('grad_pri', 1, 4): 897.6e6,
    ('grad_pri', 1, 5): 903.0e6,
    ('grad_pri', 1, 6): 906.4e6,
    ('grad_pri', 2, 0): 897.4e6,
    ('grad_pri', 2, 1): 903.8e6,
    ('grad_pri', 2, 2): 901.8e6,
    ('grad_pri', 2, 3): 897.6e6,
    ('grad_pri', 2, 4): 898.3e6,
    ('grad_pri', 2, 5): 913.5e6,
    ('grad_pri', 2, 6): 900.4e6,
    ('grad_pri', 3, 0): 898.6e6,
    ('grad_pri', 3, 1): 899.4e6,
    ('grad_pri', 3, 2): 901.3e6,
    ('grad_pri', 3, 3): 903.3e6,
    ('grad_pri', 3, 4): 901.0e6,
    ('grad_pri', 3, 5): 938.0e6,
    ('grad_pri', 3, 6): 913.1e6,
    ('grad_pri', 4, 0): 898.8e6,
    ('grad_pri', 4, 1): 903.7e6,
    ('grad_pri', 4, 2): 906.4e6,
    ('grad_pri', 4, 3): 898.2e6,
    ('grad_pri', 4, 4): 906.2e6,
    ('grad_pri', 4, 5): 903.6e6,
    ('grad_pri', 4, 6): 910.0e6,
    ('grad_pri', 5, 0): 903.8e6,
    ('grad_pri', 5, 1): 900.0e6,
    ('grad_pri', 5, 2): 908.6e6,
    ('grad_pri', 5, 3): 909.1e6,
    ('grad_pri', 5, 4): 908.2e6,
    ('grad_pri', 8, 0): 907.6e6,
    ('grad_pri', 8, 1): 903.4e6,
    ('grad_pri', 8, 2): 2097.9e6,
    ('grad_pri', 8, 3): 903.0e6,
    ('grad_tet', 7, 0): 788.0e6,
    ('gradinterp_pri', 1, 0): 1194.7e6,
    ('gradinterp_pri', 1, 1): 1194.7e6,
    ('gradinterp_pri', 1, 2): 1194.7e6,
    ('gradinterp_pri', 1, 3): 1194.8e6,
    ('gradinterp_pri', 1, 4): 1194.8e6,
    ('gradinterp_pri', 1, 5): 1200.9e6,
    ('gradinterp_pri', 1, 6): 1196.3e6,
    ('gradinterp_pri', 2, 0): 1194.7e6,
    ('gradinterp_pri', 2, 1): 1195.0e6,
    ('gradinterp_pri', 2, 2): 1195.0e6,
    ('gradinterp_pri', 2, 3): 1194.8e6,
    ('gradinterp_pri', 2, 4): 1194.9e6,
    ('gradinterp_pri', 2, 5): 1206.9e6,
    ('gradinterp_pri', 2, 6): 1201.0e6,
    ('gradinterp_pri', 3, 0): 1194.9e6,
    ('gradinterp_pri', 3, 1): 1195.1e6,
    ('gradinterp_pri', 3, 2): 1195.1e6,
    ('gradinterp_pri', 3, 3): 1195.0e6,
    ('gradinterp_pri', 3, 4): 1195.6e6,
    ('gradinterp_pri', 3, 5): 1199.4e6,
    ('gradinterp_pri', 3, 6): 1197.4e6,
    ('gradinterp_pri', 4, 0): 1194.9e6,
    ('gradinterp_pri', 4, 1): 1195.2e6,
    ('gradinterp_pri', 4, 2): 1195.1e6,
    ('gradinterp_pri', 4, 3): 1194.9e6,
    ('gradinterp_pri', 4, 4): 1195.4e6,
    ('gradinterp_pri', 4, 5): 1198.0e6,
    ('gradinterp_pri', 4, 6): 1198.3e6,
    ('gradinterp_pri', 7, 0): 1195.5e6,
    ('gradinterp_pri', 7, 1): 1195.5e6,
    ('gradinterp_pri', 7, 2): 1996.6e6,
    ('gradinterp_pri', 7, 3): 1197.1e6,
    ('gradinterp_pri', 7, 4): 1196.7e6,
    ('gradinterp_tet', 4, 0): 1120.8e6,
    ('interp_pri', 7, 0): 399.1e6,
    ('interp_tet', 4, 0): 373.8e6,
    ('upts_pri', 0, 0): 1811.1e6,
    ('upts_tet', 0, 0): 1570.8e6,
}


PRODUCT_OPS = {"interp": 0, "grad": 1, "gradinterp": 2, "div": 3}
ACC_STEPS = 100            # RK45[2R+] steps of the precision forms' accuracy table
TYPE_SHORT = ("tet", "pri", "hex")


def product_row_blocks(mesh, k):
    """16-row blocks of the operator of product kernel class k ('grad_pri',
    ...), and its (element type, operator) indices; None for other kernels."""
    op, _, name = k.partition("_")
    if op not in PRODUCT_OPS or name not in TYPE_SHORT:
        return None
    t = TYPE_SHORT.index(name)
    q = mesh.query(t)
    M = {"interp": q["nfpts"], "gradinterp": q["nfpts"], "grad": 3 * q["nupts"], "div": q["nupts"]}[op]
    return -(-M // 16), t, PRODUCT_OPS[op]


def variant_of(mesh, k, report):
    """(rows blocks per wavefront, stage) the autotuner chose for product k."""
    rb = product_row_blocks(mesh, k)
    if rb is None:
        return None
    Mb, t, op = rb
    m_ = re.search(rf"{TYPE_SHORT[t]} op{op} cap (\d+) stage (\d+)", report or "")
    if not m_:
        return None
    nmg = -(-Mb // int(m_.group(1)))
    return -(-Mb // nmg), int(m_.group(2))


def operator_nnz(mesh, t):
    """Structural nonzeros of the four products' operators of type t (the
    library's FP64 reference operators, whose analytic zeros are exact):
    interpolation M0, corrected gradient [G_k | L n_k], divergence
    [G_k - L n_k M0 | L]."""
    import numpy as np
    M0 = mesh.operator(t, 0)
    G = [mesh.operator(t, 1 + k) for k in range(3)]
    L = mesh.operator(t, 4)
    nref = mesh.operator(t, 6)                       # [nf][3]
    grad = np.concatenate([np.concatenate([G[k], L * nref[:, k][None, :]], axis=1) for k in range(3)])
    div = np.concatenate([G[k] - (L * nref[:, k][None, :]) @ M0 for k in range(3)] + [L], axis=1)
    nz = lambda A: int(np.count_nonzero(np.abs(A) > 1e-10 * np.abs(A).max()))
    return {"interp": nz(M0), "gradinterp": nz(M0), "grad": nz(grad), "div": nz(div)}


def kernel_model(mesh, system):
    """Algorithmic FLOPs and bytes per launch of each kernel class (FP32).

    Operator products C = A B: the paper's dense-operator count 2 M K n flops
    ("flops") and 4 (K + M) n bytes over the n = fields x elements real
    columns; the structural nonzeros' 2 nnz(A) n is kept beside it
    ("nnz_flops").  The divergence product also carries the last step's
    bytes (its store applies -R~/J and the register update).  Point-wise
    kernels: the values they must read and write once (states, gradients,
    fluxes, geometry)."""
    ns = system == "ns"
    out = {}
    s = 4
    npairs = 0
    for t, name in ((0, "tet"), (1, "pri"), (2, "hex")):
        q = mesh.query(t)
        E, nu, nf = q["nelem"], q["nupts"], q["nfpts"]
        if not E:
            continue
        npairs += E * nf
        cols5 = 5 * E
        nnz = operator_nnz(mesh, t)
        ops = {"interp": (nf, nu, cols5), "div": (nu, 3 * nu + nf, cols5)}
        if ns:
            ops["grad"] = (3 * nu, nu + nf, cols5)
            ops["gradinterp"] = (nf, nu, 3 * cols5)
        for op, (M, K, n) in ops.items():
            out[f"{op}_{name}"] = {"flops": 2.0 * M * K * n, "nnz_flops": 2.0 * nnz[op] * n,
                                   "bytes": s * (K + M) * n}
        ng = (9, 15, 21)[t]
        if ns:
            # fused gradient stage: reads U and the jump Cf, writes Ft and Qf
            g, gi = ops["grad"], ops["gradinterp"]
            out[f"gradflux_{name}"] = {
                "flops": 2.0 * (g[0] * g[1] * g[2] + gi[0] * gi[1] * gi[2]),
                "nnz_flops": 2.0 * (nnz["grad"] * g[2] + nnz["gradinterp"] * gi[2]),
                "bytes": float(s * (5 * nu + 5 * nf + 15 * nu + 15 * nf) * E + s * ng * E)}
        pt = (5 + (15 + 15 if ns else 0) + 15) * nu * E * s + ng * E * s
        out[f"upts_{name}"] = {"flops": 0.0, "bytes": float(pt)}
        neg = (5 + 5 + 5) * nu * E * s + ng * E * s
        out[f"negdivconf_{name}"] = {"flops": 0.0, "bytes": float(neg)}
        # the divergence product applies -R~/J and the register update in
        # its store: R~ is neither written nor read back
        out[f"div_{name}"]["bytes"] += neg - 2 * 5 * nu * E * s
    npairs //= 2
    # with the LDG beta = 1/2 (the default) only side L's gradient enters the
    # common viscous flux
    per_pair = (2 * 5 + (15 if ns else 0) + 2 * 5 + 5) * s + 8
    out["common_flux"] = {"flops": 0.0, "bytes": float(per_pair * npairs)}
    if ns:
        # beta = 1/2: the jump to the common solution is written on side L only
        out["common_solution"] = {"flops": 0.0, "bytes": float((2 * 5 + 5) * s * npairs + 8 * npairs)}
    return out


def boundary_points(arrays, p):
    """Flux points on the listed boundary faces (order p): (p+1)(p+2)/2 per
    triangle, (p+1)^2 per quadrilateral."""
    from paper_1409_0405_amd import inputs
    bf = arrays.get("bfaces")
    if bf is None:
        return 0
    n = 0
    for t, _, f, _ in bf:
        nv = len(inputs.LOCAL_FACES[("tet", "pri", "hex")[t]][f])
        n += (p + 1) * (p + 2) // 2 if nv == 3 else (p + 1) ** 2
    return n


def _oracle_sample():
    """The bounded sample of the headline workload the oracle evaluates: the
    same mesh structure, order, physics and state on fewer elements."""
    from oracle import fr, mesh as om
    from paper_1409_0405_amd import inputs
    arrays = inputs.tgv_mixed_box(nxy=6, n_pri_layers=10, n_tet_layers=6, jitter=0.10, seed=0)
    O = om.build_mesh(arrays, 4)
    U = fr.initial_state(O, inputs.taylor_green, mach=0.1)
    prm = fr.Params(system="ns", mu=1.0 / 1600.0, prandtl=0.71)
    return O, U, prm


def _oracle_worker(args):
    """One host core: oracle right-hand sides on the sample for about
    `seconds` (NumPy thread pools limited to one thread); returns (count,
    seconds, DOF per RHS)."""
    seconds, start_at = args
    from threadpoolctl import threadpool_limits
    from oracle import fr
    O, U, prm = _oracle_sample()
    dof = sum(tg.nelem * tg.ref.nupts * 5 for tg in O.types.values())
    with threadpool_limits(limits=1):
        fr.rhs(O, U, prm)                                # first call outside the timing
        while time.time() < start_at:                    # every worker starts together
            time.sleep(0.01)
        n, t0 = 0, time.perf_counter()
        while True:
            fr.rhs(O, U, prm)
            n += 1
            el = time.perf_counter() - t0
            if el > seconds:
                break
    return n, el, dof


def host_cores():
    """Host cores this process may use: the affinity set, capped by the
    thread count the environment grants (OMP_NUM_THREADS) when it is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(n, int(env))) if env and env.isdigit() else n


def cpu_baseline(target_seconds):
    """The FP64 oracle on a bounded sample of the same workload (same mesh
    structure, order and physics, fewer elements): on one core, and on every
    host core at once, one worker process per core evaluating the sample's
    right-hand side, which splits the work over the cores by elements as the
    paper's OpenMP backend splits the columns of B (the sample's periodic
    RHS is not cut into slices: each core evaluates a whole sample, and the
    throughput is the sum).  nproc and the BLAS thread count are reported."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_info
    n1, el1, dof = _oracle_worker((target_seconds, 0.0))
    cores = host_cores()
    ctx = mp.get_context("spawn")                       # the parent holds a GPU context: no fork
    start_at = time.time() + 5.0 + 0.02 * cores
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(target_seconds, start_at)] * cores)
    rate_all = sum(n * d / el for n, el, d in res)
    blas = [{"api": x.get("internal_api"), "threads": x.get("num_threads")} for x in threadpool_info()]
    from oracle import mesh as om  # noqa: F401  (the workers imported it too)
    return {"value": rate_all / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "one_core": {"value": dof * n1 / el1 / 1e9, "unit": "GDOF/s", "cores": 1},
            "nproc": os.cpu_count(), "blas_threads_per_worker": 1, "blas_pools_parent": blas,
            "sample": f"NS p=4 RHS evaluations of the FP64 NumPy oracle on a 720-prism / 1,296-tet periodic TGV "
                      f"box of the headline's structure ({dof} DOF), about {target_seconds:.0f} s per worker: "
                      f"{n1} on one core; {sum(r[0] for r in res)} over {cores} worker processes at once "
                      f"(NumPy pools limited to one thread each)"}


def measured_peaks():
    """Reference peaks measured on this device, as the paper measures its
    platforms: a 1 GiB to 1 GiB device copy, and the best rate of the vendor
    GEMM (torch.matmul, i.e. hipBLASLt / rocBLAS) in FP32 and BF16 over a few
    large square sizes."""
    import torch
    out = {}
    n = 1 << 28                                        # 2^28 floats = 1 GiB
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    out["copy_GBps"] = 10 * 2 * 4 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    for name, dt in (("sgemm_TFLOPs", torch.float32), ("bf16_gemm_TFLOPs", torch.bfloat16)):
        best = 0.0
        for m in (4096, 8192, 16384):
            x = torch.randn(m, m, device="cuda", dtype=dt)
            y = torch.randn(m, m, device="cuda", dtype=dt)
            torch.matmul(x, y)
            reps = 3 if m == 16384 else 5
            e0.record()
            for _ in range(reps):
                torch.matmul(x, y)
            e1.record()
            e1.synchronize()
            best = max(best, reps * 2.0 * m ** 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12)
            del x, y
        out[name] = best
    # the vendor FP32 GEMM on the shape of the dominant product (prism
    # corrected gradient: 225 x 180 operator, 552,960 columns), for comparison
    A = torch.randn(225, 180, device="cuda")
    B = torch.randn(180, 552960, device="cuda")
    for _ in range(3):
        torch.matmul(A, B)
    e0.record()
    for _ in range(10):
        torch.matmul(A, B)
    e1.record()
    e1.synchronize()
    out["vendor_sgemm_grad_pri_shape_us"] = e0.elapsed_time(e1) / 10 * 1e3
    del A, B
    torch.cuda.empty_cache()
    return out


def closure_at_size(stream, t_end=8.0, n_int=20, epochs=30, cfl=0.3, log=None):
    """The learned closure judged a-posteriori at the headline's full size
    (110,592 prisms + 196,608 tets, Taylor-Green, Re 1600, Ma 0.1): order 4
    and order 1 advanced side by side to t_end from the Taylor-Green state
    and its L2 projection, training pairs taken along the order-1 trajectory
    at n_int + 1 snapshots (inputs from U_1(t), targets from the filtered
    order-4 residual), the network trained on all of them, then order 1 run
    again from the projection with and without the closure (BF16 weights).
    Reported: the relative L2 over the snapshots of each run's kinetic-energy
    dissipation rate against order 4's."""
    import numpy as np
    import torch
    from paper_1409_0405_amd import closure as cl, frlib, inputs
    t_start = time.time()
    arrays = inputs.tgv_mixed_box()
    kw = dict(system="ns", precision="fp32", mu=1.0 / 1600.0, prandtl=0.71, stream=stream, check_finite=True)
    hi = frlib.Mesh(arrays, 4, **kw)
    lo = frlib.Mesh(arrays, 1, **kw)
    hi.autotune(stream)
    lo.autotune(stream)
    nel = {"tet": hi.query(0)["nelem"], "pri": hi.query(1)["nelem"]}
    h_ref = math.pi / 54                           # the prism layers' spacing
    dt4, dt1 = cl.dt_for(4, h_ref, cfl=cfl), cl.dt_for(1, h_ref, cfl=cfl)
    sb4, sb1 = max(1, round(t_end / n_int / dt4)), max(1, round(t_end / n_int / dt1))
    dt4, dt1 = t_end / n_int / sb4, t_end / n_int / sb1
    if log:
        log(f"closure at size: order 4 dt {dt4:.3e} x {sb4}, order 1 dt {dt1:.3e} x {sb1} per interval")
    cl.load_tgv(hi, stream=stream)
    cl.load_filtered(hi, lo, stream=stream)
    X, Y, times, rates4, _ = cl.generate_along_trajectory(hi, lo, dt4, sb4, dt1, sb1, n_int + 1, stream, log=log)
    nsamp = len(X)
    stats = cl.stats_of(X, Y)
    net, hist = cl.train(X, Y, stats, epochs=epochs, batch=8192, lr=2e-3, log=log)
    del X, Y
    torch.cuda.empty_cache()

    def run(with_net):
        cl.load_tgv(hi, stream=stream)
        cl.load_filtered(hi, lo, stream=stream)
        if with_net:
            lo.closure_attach(net, stats.data_ptr(), bf16_weights=True)
        try:
            return cl.dissipation_history(lo, dt1, n_int + 1, sb1, stream, log=log)
        except frlib.FrError as err:            # FR_CHECK_FINITE: the run went non-finite
            if log:
                log(f"order-1 run stopped: {err}")
            return None
        finally:
            lo.closure_attach(None)
    plain, corr = run(False), run(True)
    e = lambda r: None if r is None else float(np.sqrt(np.mean((r - rates4) ** 2) / np.mean(rates4 ** 2)))
    out = {"experiment": "closure_at_size", "elements": nel, "t_end": t_end, "snapshots": n_int + 1,
           "samples": int(nsamp), "epochs": epochs, "cfl": cfl,
           "train_loss_first_last": [float(hist[0]), float(hist[-1])],
           "times": [float(x) for x in times],
           "order4_rates": [float(x) for x in rates4],
           "order1_rates": None if plain is None else [float(x) for x in plain],
           "closure_rates": None if corr is None else [float(x) for x in corr],
           "aposteriori_rel_err_vs_order4": {"plain_order1": e(plain), "closure_bf16": e(corr)},
           "finite": {"plain_order1": plain is not None, "closure_bf16": corr is not None},
           "seconds": time.time() - t_start}
    hi.close()
    lo.close()
    return out


def closure_form(steps, warmup, arrays, mach, mu, pr, stream):
    """Cost of the learned closure in the order-1 residual on the full mixed
    mesh: RK45[2R+] steps of the order-1 NS solve without and with the network
    attached (BF16 and FP32 weights; seeded weights, unit statistics: the
    timing does not depend on the trained values)."""
    import numpy as np
    import torch
    from paper_1409_0405_amd import frlib, inputs
    m = frlib.Mesh(arrays, 1, system="ns", precision="fp32", mu=mu, prandtl=pr, stream=stream)
    dof = 0
    for t in (0, 1):
        q = m.query(t)
        x = m.upts_coords(t)
        U = inputs.taylor_green(x[:, 0], x[:, 1], x[:, 2], mach=mach)
        u = frlib.to_device_state(m, t, np.transpose(U, (1, 0, 2)).astype(np.float32))
        m.set_solution(t, u.data_ptr(), stream)
        torch.cuda.synchronize()
        dof += q["nupts"] * q["nelem"] * 5
    net = frlib.MLP(0)
    stats = torch.cat([torch.zeros(120), torch.ones(120), torch.zeros(20),
                       torch.full((20,), 1e-6)]).float().cuda()
    dt = 1e-4
    out = {"order": 1, "n_dof": dof}
    for label, attach in (("plain", None), ("closure_bf16", True), ("closure_fp32", False)):
        if attach is None:
            m.closure_attach(None)
        else:
            m.closure_attach(net, stats.data_ptr(), bf16_weights=attach)
        m.rk_step(frlib.FR_RK45_2RP, dt, max(warmup, 1), stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.rk_step(frlib.FR_RK45_2RP, dt, steps, stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[label] = {"ms_per_step": 1e3 * el / steps, "value": 5.0 * dof * steps / el / 1e9}
    m.closure_attach(net, stats.data_ptr(), bf16_weights=True)
    m.profile(True)
    m.rk_step(frlib.FR_RK45_2RP, dt, 2, stream)
    prof = m.profile_read()
    m.profile(False)
    m.closure_attach(None)
    for k in ("closure_inputs", "closure_forward"):
        ms, cnt = prof[k]
        out[k + "_us_per_rhs"] = 1e3 * ms / 10 if cnt else None       # 2 steps x 5 stages
    out["overhead_bf16"] = out["closure_bf16"]["ms_per_step"] / out["plain"]["ms_per_step"] - 1.0
    out["unit"] = "GDOF/s per RHS"
    m.close()
    return out


def batch_form(steps, warmup, cfl=0.2):
    """512 independent periodic Euler problems (vortex at a random centre,
    element counts log-uniform in [100, 20000], orders uniform in 1..4, half
    prisms and half tets by volume), FP32, advanced together: one HIP-graph
    launch per RK45[2R+] step, operator products autotuned per order."""
    import numpy as np
    import torch
    from paper_1409_0405_amd import frlib, inputs
    probs = inputs.batch_problems(n=512, seed=0)
    t0 = time.perf_counter()
    B = frlib.Batch([(b["mesh"], b["p"]) for b in probs], system="euler", precision="fp32")
    t_create = time.perf_counter() - t0
    lam = 0.5 * math.sqrt(1.4) + math.sqrt(1.4)
    dts, dof, nelem = [], 0, 0
    for i, b in enumerate(probs):
        for t in (0, 1):
            q = B.query(i, t)
            if not q["nelem"]:
                continue
            x = B.upts_coords(i, t)
            U = inputs.isentropic_vortex(x[:, 0], x[:, 1], x[:, 2], centre=b["centre"], radius=0.15)
            dev = torch.zeros((q["nupts"], 5, max(q["ld"], 64)), dtype=torch.float32, device="cuda")
            dev[:, :, :q["nelem"]] = torch.as_tensor(np.transpose(U, (1, 0, 2)), dtype=torch.float32)
            B.set_solution(i, t, dev.data_ptr())
            torch.cuda.synchronize()
            dof += q["nupts"] * q["nelem"] * 5
            nelem += q["nelem"]
        dts.append(cfl * (0.5 / b["m"]) / (lam * (2 * b["p"] + 1)))
    B.set_dt(dts)
    out = {"problems": len(probs), "elements": nelem, "n_dof": dof, "create_s": t_create}
    for graph in (True, False):
        B.set_graph(graph)
        B.rk_step(frlib.FR_RK45_2RP, max(warmup, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.rk_step(frlib.FR_RK45_2RP, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        key = "graph" if graph else "eager"
        out[key] = {"ms_per_step": 1e3 * el / steps, "value": 5.0 * dof * steps / el / 1e9}
    # the state must stay finite
    x = B.state_tensor(0, 0 if B.query(0, 0)["nelem"] else 1)
    B.get_solution(0, 0 if B.query(0, 0)["nelem"] else 1, x.data_ptr())
    torch.cuda.synchronize()
    out["finite"] = bool(torch.isfinite(x).all().item())
    out["unit"] = "GDOF/s per RHS"
    B.close()
    return out


def graph_form(arrays, p, steps, warmup, mach, mu, pr, dt):
    """The headline mesh as a one-problem batch (autotuned at creation), whose
    RK45[2R+] step the library captures once as a HIP graph: the per-step
    and per-stage time of graph replay against the same steps launched
    eagerly."""
    import numpy as np
    import torch
    from paper_1409_0405_amd import frlib, inputs
    B = frlib.Batch([(arrays, p)], system="ns", precision="fp32", mu=mu, prandtl=pr)
    dof = 0
    for t in (0, 1):
        q = B.query(0, t)
        x = B.upts_coords(0, t)
        U = inputs.taylor_green(x[:, 0], x[:, 1], x[:, 2], mach=mach)
        dev = B.state_tensor(0, t)
        dev[:, :, :q["nelem"]] = torch.as_tensor(np.transpose(U, (1, 0, 2)), dtype=torch.float32)
        dev[:, :, q["nelem"]:] = dev[:, :, :1]
        B.set_solution(0, t, dev.data_ptr())
        torch.cuda.synchronize()
        dof += q["nupts"] * q["nelem"] * 5
    B.set_dt([dt])
    out = {"n_dof": dof}
    for graph in (True, False):
        B.set_graph(graph)
        B.rk_step(frlib.FR_RK45_2RP, max(warmup, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.rk_step(frlib.FR_RK45_2RP, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["graph" if graph else "eager"] = {"ms_per_step": 1e3 * el / steps, "ms_per_stage": 1e3 * el / steps / 5,
                                              "value": 5.0 * dof * steps / el / 1e9}
    x = B.state_tensor(0, 1)
    B.get_solution(0, 1, x.data_ptr())
    torch.cuda.synchronize()
    out["finite"] = bool(torch.isfinite(x).all().item())
    out["unit"] = "GDOF/s per RHS"
    B.close()
    return out


def roofline_of(model, avg_s, k, key="flops"):
    """Roofline entry of kernel class k from its algorithmic model (flops of
    the given key: the paper's dense count, or the structural nonzeros) and
    its average launch duration."""
    mdl = model[k]
    if mdl.get(key) and mdl[key] / mdl["bytes"] > RIDGE:
        roof = {"bound": "mfma", "achieved": mdl[key] / avg_s / 1e12, "peak": 157.3, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": mdl["bytes"] / avg_s / 1e9, "peak": 8000.0, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    return roof


def structural(model, avg_s, k):
    """The same kernel against the roof of its structural-nonzero work."""
    if "nnz_flops" not in model.get(k, {}):
        return None
    r = roofline_of(model, avg_s, k, "nnz_flops")
    return {x: r[x] for x in ("bound", "achieved", "unit", "frac")}


def walks_nonzeros(k, variant):
    """Whether kernel class k walks only its operators' structural nonzeros
    (step-list products, stages 5 and 6, and the fused gradient stage): such
    a kernel is priced on its structural work, since the paper's dense count
    would credit it with work it skips (a fraction above 1 of the roof)."""
    return k.startswith("gradflux_") or bool(variant and variant[1] in (5, 6))


def workload_form(name, arrays, h_ref, steps, warmup, mach, mu, pr, stream, cfl=0.3, p=4, **mesh_kw):
    """Another mesh of the same physics (NS Taylor-Green, p = 4, FP32,
    autotuned): RK45[2R+] steps timed like the main workload, then a
    per-kernel profile and the dominant kernel's roofline.  mesh_kw: boundary
    data (t_wall, farfield) of bounded meshes."""
    mesh_kw.setdefault("p_ref", 1.0 / (1.4 * mach * mach))
    import numpy as np
    import torch
    from paper_1409_0405_amd import frlib, inputs
    m = frlib.Mesh(arrays, p, system="ns", precision="fp32", mu=mu, prandtl=pr, stream=stream, **mesh_kw)
    report = m.autotune(stream)
    print(f"autotune {name}: {report}", file=sys.stderr, flush=True)
    types, dof, counts = [], 0, {}
    for t in range(3):
        q = m.query(t)
        if not q["nelem"]:
            continue
        x = m.upts_coords(t)
        U = np.transpose(inputs.taylor_green(x[:, 0], x[:, 1], x[:, 2], mach=mach), (1, 0, 2)).astype(np.float32)
        u = frlib.to_device_state(m, t, U)
        m.set_solution(t, u.data_ptr(), stream)
        torch.cuda.synchronize()
        del u
        types.append(t)
        dof += 5 * q["nupts"] * q["nelem"]
        counts[frlib.TYPE_NAMES[t]] = q["nelem"]
    dt = cfl * h_ref / ((1.0 + 1.0 / mach) * (2 * p + 1))

    def step():
        m.rk_step(frlib.FR_RK45_2RP, dt, 1, stream)
        return m.reduce(frlib.FR_RED_INT_U, stream)
    i0 = step()
    for _ in range(max(warmup - 1, 0)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        i1 = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"elements": counts, "n_dof": dof, "ms_per_step": 1e3 * el / steps,
           "value": 5.0 * dof * steps / el / 1e9, "unit": "GDOF/s per RHS",
           "finite": bool(np.all(np.isfinite(i1))),
           "mass_energy_drift": float(np.max(np.abs(i1 - i0)[[0, 4]] / np.abs(i0)[[0, 4]]))}
    nprof = max(3, min(steps, 10))
    m.profile(True)
    for _ in range(nprof):
        m.rk_step(frlib.FR_RK45_2RP, dt, 1, stream)
    prof = m.profile_read()
    m.profile(False)
    model = kernel_model(m, "ns")
    nbp = boundary_points(arrays, p)
    if nbp:
        # boundary points: state and gradient traces in, the jump and the flux out
        model["boundary_solution"] = {"flops": 0.0, "bytes": float(4 * (5 + 5) * nbp + 17 * nbp)}
        model["boundary_flux"] = {"flops": 0.0, "bytes": float(4 * (5 + 15 + 5) * nbp + 17 * nbp)}
    rows = sorted(((ms, k, cnt) for k, (ms, cnt) in prof.items() if cnt), reverse=True)
    tot = sum(r[0] for r in rows)
    kern = {}
    for ms, k, cnt in rows:
        avg = ms / cnt * 1e-3
        kern[k] = {"share": ms / tot, "avg_us": avg * 1e6}
        if k in model:
            key = "nnz_flops" if walks_nonzeros(k, variant_of(m, k, report)) else "flops"
            kern[k].update(roofline_of(model, avg, k, key), priced_on="structural" if key == "nnz_flops" else "dense")
            if "nnz_flops" in model[k]:
                kern[k]["dense_frac"] = roofline_of(model, avg, k)["frac"]
                kern[k]["structural_frac"] = structural(model, avg, k)["frac"]
    ms, k, cnt = rows[0]
    key = "nnz_flops" if walks_nonzeros(k, variant_of(m, k, report)) else "flops"
    out["roofline"] = dict(roofline_of(model, ms / cnt * 1e-3, k, key), kernel=k, avg_launch_us=1e3 * ms / cnt,
                           share_of_step=ms / tot, priced_on="structural" if key == "nnz_flops" else "dense",
                           structural=structural(model, ms / cnt * 1e-3, k))
    out["kernels"] = kern
    m.close()
    del m
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cfl", type=float, default=0.3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--no-hex", action="store_true", help="skip the hexahedral and three-type workloads")
    ap.add_argument("--workload", choices=("mixed", "hex", "hybrid", "curved_wall"), default="mixed",
                    help="hex / hybrid / curved_wall: run only that workload's form (for profiling) and print it")
    ap.add_argument("--closure-at-size", action="store_true",
                    help="train and judge the learned closure on the full headline mesh (about 15 minutes)")
    ap.add_argument("--variants", action="store_true",
                    help="time every variant of the prism corrected-gradient and gradient-"
                         "interpolation products on this workload (one JSON line) instead of the bench")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the right-hand side runs on a single "
              "MI355X here (sharding by mesh partition is not built); run with --gpus 1",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1409_0405_amd import frlib, inputs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    mu, mach, pr, p = 1.0 / 1600.0, 0.1, 0.71, 4
    L = 2 * math.pi
    # reference pressure left out of the momentum flux: the Taylor-Green p0
    p_ref = 1.0 / (1.4 * mach * mach)

    def hex_form():
        hx = workload_form("hex", inputs.hex_box(50, jitter=0.10, seed=0), L / 50, args.steps, args.warmup,
                           mach, mu, pr, stream)
        hx["workload"] = "periodic [0,2pi)^3, 50^3 hexahedra (jitter 10 %), NS TGV Re1600 Ma0.1, p=4, FP32"
        return hx

    def hybrid_form():
        hy = workload_form("hybrid", inputs.hybrid_box(48, 48, 48, 24, 24, (L, L, L), jitter=0.10, seed=0),
                           L / 48, args.steps, args.warmup, mach, mu, pr, stream)
        hy["workload"] = ("periodic [0,2pi)^3, 48^3 cells: hexahedra | z-prisms below, x-prisms | Kuhn tets "
                          "above (jitter 10 %), NS TGV Re1600 Ma0.1, p=4, FP32")
        return hy

    def curved_wall_form():
        # walls at the Taylor-Green temperature p0 / rho0 = 1 / (gamma Ma^2)
        cw = workload_form("curved_wall", inputs.curve(inputs.hybrid_box(48, 48, 48, 24, 24, (L, L, L), jitter=0.05,
                                                                        seed=0, y_bc="wall"), 0.02),
                           L / 48, args.steps, args.warmup, mach, mu, pr, stream, t_wall=1.0 / (1.4 * mach * mach))
        cw["workload"] = ("the 48^3-cell three-type box bounded by no-slip isothermal walls at y = 0, 2pi and "
                          "quadratically curved (deformation amplitude 2 %, jitter 5 %), NS TGV Re1600 Ma0.1, p=4, FP32")
        return cw

    if args.workload != "mixed":
        form = {"hex": hex_form, "hybrid": hybrid_form, "curved_wall": curved_wall_form}[args.workload]
        print(json.dumps({"form": args.workload, **form()}), flush=True)
        return
    if args.closure_at_size:
        print(json.dumps(closure_at_size(stream, log=lambda msg: print(msg, file=sys.stderr, flush=True))),
              flush=True)
        return
    arrays = inputs.tgv_mixed_box()

    tuned = {}

    def make_mesh(precision):
        m = frlib.Mesh(arrays, p, system="ns", precision=precision, mu=mu, prandtl=pr,
                       stream=stream, p_ref=p_ref)
        if not args.no_autotune and precision != "fp64":
            tuned[precision] = m.autotune(stream)
            print(f"autotune {precision}: {tuned[precision]}", file=sys.stderr, flush=True)
        return m

    t_setup = time.perf_counter()
    mesh = make_mesh("fp32")
    qs = [mesh.query(t) for t in (0, 1)]
    host_state, dof = [], 0
    for t in (0, 1):
        q = mesh.query(t)
        x = mesh.upts_coords(t)                                        # [nu][3][E]
        U = inputs.taylor_green(x[:, 0], x[:, 1], x[:, 2], mach=mach)  # [5][nu][E]
        host_state.append(np.transpose(U, (1, 0, 2)).astype(np.float32))
        dof += q["nupts"] * q["nelem"] * 5
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"setup {t_setup:.1f} s, {dof} DOF", file=sys.stderr, flush=True)

    h_ref = math.pi / 54                  # smallest unjittered spacing (prism layers)
    lam = 1.0 + 1.0 / mach                # V0 + c0
    dt = args.cfl * h_ref / (lam * (2 * p + 1))

    def load(m):
        for t in (0, 1):
            u = frlib.to_device_state(m, t, host_state[t])
            m.set_solution(t, u.data_ptr(), stream)
            torch.cuda.synchronize()
            del u

    def timed(m, steps, warmup):
        """RK45[2R+] steps plus the FP64 conservation integral, timed."""
        load(m)

        def step():
            m.rk_step(frlib.FR_RK45_2RP, dt, 1, stream)
            return m.reduce(frlib.FR_RED_INT_U, stream)   # FP64, synchronising
        i0 = step()
        for _ in range(max(warmup - 1, 0)):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            i1 = step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        drift = float(np.max(np.abs(i1 - i0)[[0, 4]] / np.abs(i0)[[0, 4]]))
        return 1e3 * el / steps, 5.0 * dof * steps / el / 1e9, drift, bool(np.all(np.isfinite(i1)))

    def state_of(m):
        out = []
        for t in (0, 1):
            x = frlib.state_tensor(m, t)
            m.get_solution(t, x.data_ptr(), stream)
            torch.cuda.synchronize()
            out.append(x.double())
        return out

    nel = [qs[t]["nelem"] for t in (0, 1)]

    def rel_err_pair(A, B):
        """Relative L2 of A against B over both types: per field, and for
        density, momentum (as a vector field) and energy."""
        num = np.zeros(5)
        den = np.zeros(5)
        for t in (0, 1):
            ne = nel[t]
            d = A[t][:, :, :ne] - B[t][:, :, :ne]
            num += (d ** 2).sum(dim=(0, 2)).cpu().numpy()
            den += (B[t][:, :, :ne] ** 2).sum(dim=(0, 2)).cpu().numpy()
        vec = [num[0] / den[0], num[1:4].sum() / den[1:4].sum(), num[4] / den[4]]
        return {"per_field": [float(x) for x in np.sqrt(num / den)],
                "rho_momentum_energy": [float(np.sqrt(x)) for x in vec]}

    def rhs_of(m):
        u = [frlib.to_device_state(m, t, host_state[t]) for t in (0, 1)]
        r = [frlib.state_tensor(m, t) for t in (0, 1)]
        m.rhs([x.data_ptr() for x in u], [x.data_ptr() for x in r], stream)
        torch.cuda.synchronize()
        out = [x.double() for x in r]
        del u, r
        return out

    if args.variants:
        # every (row blocks per wavefront, staging) variant of the two largest
        # prism products, six RHS evaluations each; used with rocprofv3 --pmc
        # to measure each variant's HBM traffic
        u = [frlib.to_device_state(mesh, t, host_state[t]) for t in (0, 1)]
        r = [frlib.state_tensor(mesh, t) for t in (0, 1)]
        out_v = {}
        for k in ("grad_pri", "gradinterp_pri"):
            Mb, t, op = product_row_blocks(mesh, k)
            rows = []
            for stage in (0, 1, 2, 3, 4, 5, 6):
                print(f"variants {k} stage {stage}", file=sys.stderr, flush=True)
                for cap in (1, 2, 3, 4, 5, 6, 8):
                    try:
                        mesh.set_blocking(t, op, cap, stage)
                    except frlib.FrError:
                        continue
                    mesh.profile(True)
                    for _ in range(6):
                        mesh.rhs([x.data_ptr() for x in u], [x.data_ptr() for x in r], stream)
                    ms, cnt = mesh.profile_read()[k]
                    mesh.profile(False)
                    nmg = -(-Mb // cap)
                    rows.append({"cap": cap, "rows_blocks_per_wave": -(-Mb // nmg), "stage": stage,
                                 "avg_us": 1e3 * ms / cnt})
            out_v[k] = rows
        print(json.dumps({"variants": out_v}), flush=True)
        return

    ms_per_step, value, drift, finite = timed(mesh, args.steps, args.warmup)
    print(f"fp32: {ms_per_step:.3f} ms/step, {value:.2f} GDOF/s per RHS, mass/energy drift {drift:.2e}",
          file=sys.stderr, flush=True)
    # one RHS: HIP events around each of 20 back-to-back fr_rhs calls after 5
    # warm-ups, on the library's stream; the median
    u_r = [frlib.to_device_state(mesh, t, host_state[t]) for t in (0, 1)]
    r_r = [frlib.state_tensor(mesh, t) for t in (0, 1)]
    cur = torch.cuda.current_stream()
    for _ in range(5):
        mesh.rhs([x.data_ptr() for x in u_r], [x.data_ptr() for x in r_r], stream)
    times_r = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        mesh.rhs([x.data_ptr() for x in u_r], [x.data_ptr() for x in r_r], stream)
        e1.record(cur)
        e1.synchronize()
        times_r.append(e0.elapsed_time(e1))
    rhs_med = float(np.median(times_r))
    del u_r, r_r
    # the operator products once each (the fused gradient stage's entry
    # repeats the corrected-gradient and gradient-interpolation products)
    prods = {k: v for k, v in kernel_model(mesh, "ns").items() if not k.startswith("gradflux_")}
    f_alg = sum(v["flops"] for v in prods.values())
    f_nnz = sum(v.get("nnz_flops", 0.0) for v in prods.values())
    print(f"fr_rhs median {rhs_med:.3f} ms", file=sys.stderr, flush=True)
    roof = None
    rhs_traffic = None
    if not args.no_profile:
        nprof = max(3, min(args.steps, 10))
        load(mesh)
        mesh.profile(True)
        for _ in range(nprof):
            mesh.rk_step(frlib.FR_RK45_2RP, dt, 1, stream)
        prof = mesh.profile_read()
        mesh.profile(False)
        model = kernel_model(mesh, "ns")
        rows = sorted(((ms, k, cnt) for k, (ms, cnt) in prof.items() if cnt), reverse=True)
        tot = sum(r[0] for r in rows)
        for ms, k, cnt in rows:
            avg = ms / cnt * 1e-3
            mdl = model.get(k, {"flops": 0, "bytes": 0})
            print(f"  {k:16s} {ms / nprof:8.3f} ms/step {100 * ms / tot:5.1f}%  avg {avg * 1e6:8.1f} us"
                  f"  {mdl['flops'] / avg / 1e12:7.1f} TFLOP/s dense  {mdl.get('nnz_flops', 0) / avg / 1e12:6.1f}"
                  f" structural  {mdl['bytes'] / avg / 1e9:7.0f} GB/s", file=sys.stderr, flush=True)
        # the HBM bytes one RHS moves, from the measured per-launch traffic of
        # each kernel variant the timed steps ran (null if one is not in the
        # table)
        per_rhs = [MEASURED_TRAFFIC.get((kk,) + (variant_of(mesh, kk, tuned.get("fp32", "")) or (0, 0)))
                   for _, kk, cc in rows]
        rhs_traffic = float(sum(per_rhs)) if all(x is not None for x in per_rhs) else None
        ms, k, cnt = rows[0]
        avg = ms / cnt * 1e-3
        vt = variant_of(mesh, k, tuned.get("fp32", ""))
        key = "nnz_flops" if walks_nonzeros(k, vt) else "flops"
        # the dominant kernel on the work it does: the dense-operator count
        # for dense products, the structural nonzeros for kernels that skip
        # the zero fragments (both kept in the record)
        roof = roofline_of(model, avg, k, key)
        roof["priced_on"] = "structural" if key == "nnz_flops" else "dense"
        roof["dense"] = {x: roofline_of(model, avg, k)[x] for x in ("bound", "achieved", "unit", "frac")}
        roof["structural"] = structural(model, avg, k)
        roof["hbm"] = {"achieved": model[k]["bytes"] / avg / 1e9, "unit": "GB/s",
                       "frac": model[k]["bytes"] / avg / PEAK_HBM, "algorithmic_bytes": model[k]["bytes"]}
        if vt:
            roof["variant"] = {"rows_blocks_per_wave": vt[0], "stage": vt[1]}
        roof["traffic"] = MEASURED_TRAFFIC.get((k,) + (vt or (0, 0)))
        roof["traffic_source"] = (f"{TRAFFIC_SOURCE}: {k}" + (f" (row blocks {vt[0]}, stage {vt[1]})" if vt else "")
                                  if roof["traffic"] else None)
        roof["kernel"] = k
        roof["avg_launch_us"] = avg * 1e6
        roof["share_of_step"] = ms / tot

    forms = None
    if not args.no_forms:
        # accuracy of each precision on this workload against the FP64 build
        # of the same kernels (itself held to the oracle within 1e-11 on
        # sampled elements of this mesh, tests/test_gpu_fullsize.py): the RHS
        # of the same FP32 input, and the state after 100 RK45[2R+] steps
        nsteps_total = ACC_STEPS
        ref64 = make_mesh("fp64")
        R64 = rhs_of(ref64)
        load(ref64)
        ref64.rk_step(frlib.FR_RK45_2RP, dt, nsteps_total, stream)
        U64 = state_of(ref64)
        ref64.close()
        del ref64
        torch.cuda.empty_cache()
        load(mesh)                     # the FP32 mesh, the same number of steps
        mesh.rk_step(frlib.FR_RK45_2RP, dt, nsteps_total, stream)
        fp32_state = state_of(mesh)
        forms = {"accuracy_steps": ACC_STEPS, "accuracy_reference": "FP64 build of the same kernels",
                 "fp32": {"value": value, "ms_per_step": ms_per_step,
                          "rhs_rel_l2_vs_fp64": rel_err_pair(rhs_of(mesh), R64),
                          "state_rel_l2_vs_fp64": rel_err_pair(fp32_state, U64)}}
        del fp32_state
        for prec in ("split_bf16", "split_fp16"):
            m2 = make_mesh(prec)
            ms2, v2, d2, f2 = timed(m2, args.steps, args.warmup)
            load(m2)
            m2.rk_step(frlib.FR_RK45_2RP, dt, nsteps_total, stream)
            st = rel_err_pair(state_of(m2), U64)
            forms[prec] = {"value": v2, "ms_per_step": ms2, "speedup_vs_fp32": v2 / value,
                           "rhs_rel_l2_vs_fp64": rel_err_pair(rhs_of(m2), R64),
                           "state_rel_l2_vs_fp64": st, "finite": f2,
                           "mass_energy_drift": d2}
            print(f"{prec}: {ms2:.3f} ms/step, {v2:.2f} GDOF/s per RHS "
                  f"(x{v2 / value:.2f}), rhs error {forms[prec]['rhs_rel_l2_vs_fp64']}, state error {st}",
                  file=sys.stderr, flush=True)
            m2.close()
            del m2
            torch.cuda.empty_cache()
        print(f"fp32 rhs error {forms['fp32']['rhs_rel_l2_vs_fp64']}, state error "
              f"{forms['fp32']['state_rel_l2_vs_fp64']}", file=sys.stderr, flush=True)

    if not args.no_forms:
        mesh.close()
        torch.cuda.empty_cache()
        cf = closure_form(args.steps, args.warmup, arrays, mach, mu, pr, stream)
        forms["closure_p1"] = cf
        print(f"closure: {cf}", file=sys.stderr, flush=True)

    if not args.no_batch:
        mesh.close()
        torch.cuda.empty_cache()
        bf = batch_form(args.steps, args.warmup)
        forms = forms or {}
        forms["batch_512_euler"] = bf
        print(f"batch: {bf}", file=sys.stderr, flush=True)
        gf = graph_form(arrays, p, args.steps, args.warmup, mach, mu, pr, dt)
        forms["rk_graph_headline"] = gf
        print(f"rk graph: {gf}", file=sys.stderr, flush=True)

    if not args.no_hex:
        mesh.close()
        torch.cuda.empty_cache()
        forms = forms or {}
        hx = hex_form()
        forms["hex_p4"] = hx
        print(f"hex: {hx}", file=sys.stderr, flush=True)
        hy = hybrid_form()
        forms["hybrid_p4"] = hy
        print(f"hybrid: {hy}", file=sys.stderr, flush=True)
        cw = curved_wall_form()
        forms["curved_wall_p4"] = cw
        print(f"curved wall: {cw}", file=sys.stderr, flush=True)

    peaks = None
    if not args.no_peaks:
        peaks = measured_peaks()
        print(f"peaks: {peaks}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)

    # whole right-hand side against the HBM roof of its algorithmic bytes:
    # 4 B x 5 fields x (2 N_u + 8 N_f) per element (state in and out, traces
    # and gradient traces written and read once) plus geometry
    b_alg = 0
    for t in (0, 1):
        q = qs[t]
        b_alg += 4 * 5 * (2 * q["nupts"] + 8 * q["nfpts"]) * q["nelem"] + 4 * (9 if t == 0 else 15) * q["nelem"]
    t_rhs = ms_per_step / 5 * 1e-3
    hbm = {"algorithmic_bytes_per_rhs": b_alg, "achieved_GBps": b_alg / t_rhs / 1e9,
           "frac_of_8TBps": b_alg / t_rhs / PEAK_HBM}
    if rhs_traffic:
        # the bytes the kernels actually move (rocprofv3 counters, per launch)
        hbm["measured_traffic_per_rhs"] = rhs_traffic
        hbm["measured_traffic_GBps"] = rhs_traffic / t_rhs / 1e9
        hbm["measured_traffic_frac_of_8TBps"] = rhs_traffic / t_rhs / PEAK_HBM
        hbm["traffic_source"] = TRAFFIC_SOURCE
    # whole right-hand side against both roofs: T_roof = max(B_alg / 8 TB/s,
    # F_alg / 157.3 TFLOP/s) with F_alg the dense operator products, over the
    # measured time of one RHS (RK45 step / 5, and the back-to-back fr_rhs median)
    t_roof = max(b_alg / PEAK_HBM, f_alg / (PEAK_FP32_MFMA))
    whole = {"algorithmic_flops_per_rhs": f_alg, "algorithmic_bytes_per_rhs": b_alg,
             "binding_roof": "mfma" if f_alg / PEAK_FP32_MFMA > b_alg / PEAK_HBM else "hbm",
             "roof_ms": 1e3 * t_roof, "rhs_ms_from_steps": 1e3 * t_rhs, "frac_from_steps": t_roof / t_rhs}
    if rhs_med is not None:
        whole["rhs_ms_median"] = rhs_med
        whole["frac"] = t_roof / (rhs_med * 1e-3)
        # against the structural-nonzero work of the products instead
        t_nnz = max(b_alg / PEAK_HBM, f_nnz / PEAK_FP32_MFMA)
        whole["structural"] = {"flops_per_rhs": f_nnz,
                               "binding_roof": "mfma" if f_nnz / PEAK_FP32_MFMA > b_alg / PEAK_HBM else "hbm",
                               "roof_ms": 1e3 * t_nnz, "frac": t_nnz / (rhs_med * 1e-3)}

    out = {
        "metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Navier-Stokes Taylor-Green Re1600 Ma0.1, p=4, FP32, "
                               "110592 prisms + 196608 tets, RK45[2R+] steps",
                   "n_dof": dof, "rhs_per_step": 5, "dt": dt, "parallelism": "single GPU",
                   "finite": finite, "mass_energy_drift": drift,
                   "autotuned": not args.no_autotune},
        "roofline": roof, "cpu_baseline": cpu, "forms": forms, "rhs_hbm": hbm, "rhs_roofline": whole,
        "peaks_measured": peaks,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
