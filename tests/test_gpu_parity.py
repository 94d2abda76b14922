"""GPU parity: the HIP library through its C ABI against the FP64 oracle on
the same seeded inputs.

Sizes span several MFMA tiles and a ragged element tail (element counts not
multiples of 64).  Tolerances (relative L2 per conserved field):
* FP64 build of the kernels:  1e-11 (operators built by two independent
  routes agree to ~2e-13; the residual amplifies that by ~p^2/h);
* FP32 build, with the case's pressure scale as the reference pressure left
  out of the momentum flux (exact on these meshes; not on the curved mesh at
  p = 2, whose metric terms are not interpolated exactly there):
  - 1e-5 per field on the cases where single precision reaches it
    (FP32_1E5);
  - elsewhere the residual is a difference of flux terms 10^2 - 10^3 times
    larger than itself, and single-precision rounding of those terms gives
    1.0 - 1.5e-5 (measured); there the test asserts the bound derived from
    the unit roundoff and that cancellation factor (see _fp32_tol) and 2e-5,
    and the state after 20 RK45[2R+] steps against the oracle's stepper is
    held to 1e-5 per field (test_fp32_state_after_rk45_steps).
"""
import math

import numpy as np
import pytest

from gradient_points import read_points
from oracle import fr, mesh as om, reduce, rk
from paper_1409_0405_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAMES = ("tet", "pri", "hex")


def _lib():
    from paper_1409_0405_amd import frlib
    return frlib


def _state(O, ic, seed, noise=0.01, **kw):
    U = fr.initial_state(O, ic, **kw)
    for n in U:
        U[n] = U[n] * inputs.random_perturbation(U[n].shape, seed, noise)
    return U


def _round32(U):
    return {n: U[n].astype(np.float32).astype(np.float64) for n in U}


def _gpu_rhs(M, O, U):
    frlib = _lib()
    u, r = [], []
    for t in range(len(NAMES)):
        if NAMES[t] in O.types:
            u.append(frlib.to_device_state(M, t, np.transpose(U[NAMES[t]], (1, 2, 0))))
        else:
            u.append(None)
        r.append(frlib.state_tensor(M, t) if u[-1] is not None else None)
    M.rhs([x.data_ptr() if x is not None else 0 for x in u],
          [x.data_ptr() if x is not None else 0 for x in r])
    torch.cuda.synchronize()
    out = {}
    for t in range(len(NAMES)):
        if r[t] is not None:
            ne = O.types[NAMES[t]].nelem
            out[NAMES[t]] = np.transpose(r[t][:, :, :ne].cpu().numpy().astype(np.float64), (2, 0, 1))
    return out


def _field_errors(Rg, Ro):
    """Per-field relative L2 error over all types."""
    num = sum(((Rg[n] - Ro[n]) ** 2).sum(axis=(0, 1)) for n in Ro)
    den = sum((Ro[n] ** 2).sum(axis=(0, 1)) for n in Ro)
    return np.sqrt(num / den)


def _state_errors(G, Uo):
    """Relative L2 error of a state: density, momentum (as a vector field:
    |dm| / |m|, since the Taylor-Green w-momentum starts at exactly zero and
    a per-component ratio of it is meaningless) and energy; the three
    momentum components are also returned per component for the record."""
    num = sum(((G[n] - Uo[n]) ** 2).sum(axis=(0, 1)) for n in Uo)
    den = sum((Uo[n] ** 2).sum(axis=(0, 1)) for n in Uo)
    vec = np.array([num[0] / den[0], num[1:4].sum() / den[1:4].sum(), num[4] / den[4]])
    return np.sqrt(vec), np.sqrt(num[1:4] / den[1:4])


def _pref(case):
    """Reference pressure of a case: the pressure scale of its initial state
    (free-stream pressure of the vortex, p0 = 1 / (gamma Ma^2) of the
    Taylor-Green state); none on the curved mesh below p = 3."""
    kind, p, system, ic, kw, mu = case
    if kind.startswith("curved") and p < 3:
        return 0.0
    return 1.0 if ic is inputs.isentropic_vortex else 1.0 / (1.4 * kw["mach"] ** 2)


def _fp32_tol(O, U, prm):
    """Error scale of a single-precision evaluation: unit roundoff 2^-24 times
    the ratio of the residual computed from |fluxes| (no cancellation) to the
    residual itself, per field, times a safety factor of 16."""
    R = fr.rhs(O, U, prm)
    # magnitude of the summed terms: the residual of |U| perturbations is not
    # available in closed form, so use the flux magnitude over the element
    # size: |F| * (p+1)^2 / h at each point, h from the element Jacobian.
    num = np.zeros(5)
    den = np.zeros(5)
    for n, tg in O.types.items():
        Ue = np.moveaxis(U[n], 2, 0)
        from oracle import physics
        F = np.abs(physics.inviscid_flux(Ue, prm.gamma)).max(axis=0)      # [5][E][N]
        h = np.cbrt(tg.J_upts)                                               # ~ element size / 2
        scale = F * (O.p + 1) ** 2 / h[None]
        num += (scale ** 2).sum(axis=(1, 2))
        den += (R[n] ** 2).sum(axis=(0, 1))
    kappa = np.sqrt(num / den)
    return 16 * 2.0 ** -24 * kappa


# ---------------------------------------------------------------------------

CASES = [
    # (mesh maker, p, system, ic, ic kwargs, mu)
    ("tetcube", 2, "euler", inputs.isentropic_vortex, {}, 0.0),
    ("mixed", 1, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("mixed", 3, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("mixed", 1, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("mixed", 2, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("mixed", 3, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("mixed", 4, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("mixed", 4, "euler", inputs.taylor_green, {"mach": 0.1}, 0.0),
    ("prisms", 3, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("prisms", 1, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("hex", 2, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("hex", 4, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("hybrid", 1, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("hybrid", 3, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("hybrid", 4, "euler", inputs.taylor_green, {"mach": 0.1}, 0.0),
    ("wallbox", 3, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("wallbox", 1, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("farbox", 2, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("farbox", 4, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("curved", 2, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
    ("curved", 4, "euler", inputs.taylor_green, {"mach": 0.3}, 0.0),
    ("curvedwall", 3, "ns", inputs.taylor_green, {"mach": 0.3}, 0.02),
]

# Boundary data of the bounded boxes, on the scale of the Taylor-Green state
# at Mach 0.3 (rho0 = 1, p0 = 1 / (gamma Ma^2)): wall temperature p0 / rho0,
# a free stream crossing the far-field planes.
P0 = 1.0 / (1.4 * 0.09)
BC = {"wallbox": {"t_wall": P0}, "farbox": {"farfield": (1.0, 0.2, 0.3, -0.1, P0)}, "curvedwall": {"t_wall": P0}}


def _mesh(kind, seed=0):
    if kind == "tetcube":
        return inputs.vortex_tet_cube(n=6, jitter=0.05, seed=seed)
    if kind == "prisms":
        # prisms only (the tet type is empty): 5 x 5 x 2 triangles x 3 layers = 150
        return inputs.mixed_box(5, 5, 3, 0, (2 * math.pi,) * 3, jitter=0.1, seed=seed)
    if kind == "hex":
        # 5^3 = 125 jittered hexahedra (ragged against 64)
        return inputs.hex_box(5, jitter=0.12, seed=seed)
    if kind == "hybrid":
        # all three types, conforming: 36 hexahedra, 144 prisms (both
        # orientations), 216 tets
        return inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=seed)
    if kind in ("curved", "curvedwall"):
        # quadratically curved three-type box (smooth periodic deformation),
        # periodic or bounded by walls in y
        return inputs.curve(inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=seed,
                                              y_bc="wall" if kind == "curvedwall" else None), 0.03)
    if kind in ("wallbox", "farbox"):
        # the three-type box bounded in y by walls or far-field planes
        return inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=seed,
                                 y_bc="wall" if kind == "wallbox" else "farfield")
    # 4 x 4 x (3 + 3): 96 prisms and 288 tets -> ragged against 64
    return inputs.small_mixed_box(nxy=4, n_pri_layers=3, n_tet_layers=3, jitter=0.1, seed=seed)


def _ids(c):
    return f"{c[0]}-p{c[1]}-{c[2]}"


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_rhs_fp64_parity(case):
    kind, p, system, ic, kw, mu = case
    print(f"case {_ids(case)} fp64", flush=True)
    arrays = _mesh(kind)
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system=system, mu=mu, **BC.get(kind, {}))
    U = _state(O, ic, 3, **kw)
    Ro = fr.rhs(O, U, prm)
    M = _lib().Mesh(arrays, p, system=system, precision="fp64", mu=mu, **BC.get(kind, {}))
    Rg = _gpu_rhs(M, O, U)
    err = _field_errors(Rg, Ro)
    print("  field errors", err, flush=True)
    assert (err < 1e-11).all(), err


# cases whose FP32 residual is within 1e-5 of the oracle's in every field
# (measured 5.1e-6 .. 8.3e-6)
FP32_1E5 = ("prisms-p1-euler", "hex-p2-euler", "hex-p4-ns", "farbox-p2-ns")
FP32_CASES = [c for c in CASES if _ids(c) in FP32_1E5]
FP32_KAPPA = [c for c in CASES if _ids(c) not in FP32_1E5]


def _fp32_case_errors(case):
    kind, p, system, ic, kw, mu = case
    arrays = _mesh(kind)
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system=system, mu=mu, **BC.get(kind, {}))
    U = _round32(_state(O, ic, 3, **kw))
    Ro = fr.rhs(O, U, prm)
    M = _lib().Mesh(arrays, p, system=system, precision="fp32", mu=mu, p_ref=_pref(case), **BC.get(kind, {}))
    err = _field_errors(_gpu_rhs(M, O, U), Ro)
    M.close()
    return err, _fp32_tol(O, U, prm)


@pytest.mark.parametrize("case", FP32_CASES, ids=[_ids(c) for c in FP32_CASES])
def test_rhs_fp32_parity(case):
    print(f"case {_ids(case)} fp32", flush=True)
    err, _ = _fp32_case_errors(case)
    print("  field errors", err, flush=True)
    assert (err < 1e-5).all(), err


@pytest.mark.parametrize("case", FP32_KAPPA, ids=[_ids(c) for c in FP32_KAPPA])
def test_rhs_fp32_parity_cancellation_limited(case):
    """The FP32 residual where the cancellation of its flux terms keeps it
    above 1e-5: within the single-precision bound of the case and 2e-5
    (5e-5 on the curved mesh at p = 2, which runs without the reference
    pressure: measured 2.9e-5)."""
    print(f"case {_ids(case)} fp32 (cancellation-limited)", flush=True)
    err, tol = _fp32_case_errors(case)
    cap = 2e-5 if _pref(case) > 0 else 5e-5
    print("  field errors", err, "kappa bound", tol, flush=True)
    assert (err < tol).all() and (err < cap).all(), (err, tol)


@pytest.mark.parametrize("kind,p,system,mach,noise,mu", [
    ("mixed", 4, "ns", 0.3, 0.01, 0.02), ("mixed", 4, "euler", 0.1, 0.01, 0.0), ("hybrid", 3, "ns", 0.3, 0.01, 0.02),
    ("mixed", 4, "ns", 0.1, 0.0, 1.0 / 1600)])
def test_fp32_state_after_rk45_steps(kind, p, system, mach, noise, mu):
    """What the solver delivers where the FP32 residual is cancellation-
    limited: 20 RK45[2R+] steps (CFL 0.3) of the FP32 library against the
    oracle's stepper on the same box, density, momentum and energy within
    1e-5.  The last case is the headline state itself (Taylor-Green at Mach
    0.1, Re 1600, no noise, p = 4)."""
    frlib = _lib()
    print(f"fp32 rk45 state {kind} p{p} {system} Ma {mach} noise {noise}", flush=True)
    arrays = _mesh(kind, seed=1)
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system=system, mu=mu)
    U0 = _round32(_state(O, inputs.taylor_green, 5, noise=noise, mach=mach))
    nsteps = 20
    dt = 0.3 * (2 * math.pi / 6) / ((1 + 1 / mach) * (2 * p + 1))
    Uo = rk.run(rk.rk45_step, lambda V: fr.rhs(O, V, prm), U0, dt, nsteps)
    M = frlib.Mesh(arrays, p, system=system, precision="fp32", mu=mu, p_ref=1.0 / (1.4 * mach ** 2),
                   check_finite=True)
    for n in O.types:
        t = NAMES.index(n)
        M.set_solution(t, frlib.to_device_state(M, t, np.transpose(U0[n], (1, 2, 0))).data_ptr())
    M.rk_step(frlib.FR_RK45_2RP, dt, nsteps)
    G = {}
    for n in O.types:
        t = NAMES.index(n)
        out = frlib.state_tensor(M, t)
        M.get_solution(t, out.data_ptr())
        torch.cuda.synchronize()
        G[n] = np.transpose(out[:, :, :O.types[n].nelem].cpu().numpy().astype(np.float64), (2, 0, 1))
    err, comp = _state_errors(G, Uo)
    print(f"  state errors (rho, momentum, E) {err}; momentum components {comp}", flush=True)
    assert (err < 1e-5).all(), err


@pytest.mark.parametrize("kind,p,system", [("mixed", 2, "ns"), ("mixed", 4, "ns"), ("mixed", 3, "euler"),
                                           ("hybrid", 3, "ns"), ("wallbox", 2, "ns"), ("farbox", 3, "ns"),
                                           ("curved", 4, "ns")])
def test_interface_intermediates_fp64(kind, p, system):
    """State at flux points, common normal flux and (NS) the gradient at flux
    points, element by element."""
    print(f"intermediates {kind} p{p} {system}", flush=True)
    arrays = _mesh(kind, seed=2)
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system=system, mu=0.02, **BC.get(kind, {}))
    U = _state(O, inputs.taylor_green, 4, mach=0.3)
    want = {}
    fr.rhs(O, U, prm, want=want)
    M = _lib().Mesh(arrays, p, system=system, precision="fp64", mu=0.02, **BC.get(kind, {}))
    _gpu_rhs(M, O, U)
    items = [(0, "Uf", 5), (1, "Fn", 5)] + ([(2, "Qf", 15)] if system == "ns" else [])
    for which, key, nv in items:
        for n in O.types:
            t = NAMES.index(n)
            q = M.query(t)
            buf = torch.zeros((q["nfpts"], nv, q["ld"]), dtype=torch.float64, device="cuda")
            M.intermediate(t, which, buf.data_ptr())
            torch.cuda.synchronize()
            g = np.transpose(buf[:, :, :q["nelem"]].cpu().numpy(), (2, 0, 1))
            o = want[key][n].reshape(g.shape)
            if key == "Qf":
                # the gradient is held where the common flux reads it (the
                # fused gradient stage writes no other point)
                rp = read_points(O)[n]
                g, o = g[rp], o[rp]
            rel = np.abs(g - o).max() / np.abs(o).max()
            print(f"  {key} {n} max rel {rel:.2e}", flush=True)
            assert rel < 1e-11, (key, n, rel)


def _vortex_dt(n, p):
    lam = 0.5 * math.sqrt(1.4) + math.sqrt(1.4)
    return 0.2 * (1.0 / n) / (lam * (2 * p + 1))


@pytest.mark.parametrize("scheme", ["rk4", "rk45", "euler"])
def test_rk_steps_fp64_vortex(scheme):
    """The small Euler workload: 1,296 jittered tets, p = 2, isentropic vortex,
    10 steps at CFL 0.2 (RK4 as stated for it, RK45[2R+], and forward Euler,
    the test stepper)."""
    frlib = _lib()
    print(f"rk {scheme}", flush=True)
    arrays = inputs.vortex_tet_cube(n=6, jitter=0.05, seed=0)
    p, nsteps = 2, 10
    dt = _vortex_dt(6, p)
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system="euler")
    U0 = fr.initial_state(O, inputs.isentropic_vortex)
    stepper = {"rk4": rk.rk4_step, "rk45": rk.rk45_step, "euler": rk.euler_step}[scheme]
    Uo = rk.run(stepper, lambda V: fr.rhs(O, V, prm), U0, dt, nsteps)
    M = frlib.Mesh(arrays, p, system="euler", precision="fp64", check_finite=True)
    u = frlib.to_device_state(M, 0, np.transpose(U0["tet"], (1, 2, 0)))
    M.set_solution(0, u.data_ptr())
    M.rk_step({"rk4": frlib.FR_RK4, "rk45": frlib.FR_RK45_2RP, "euler": frlib.FR_FWD_EULER}[scheme], dt, nsteps)
    out = frlib.state_tensor(M, 0)
    M.get_solution(0, out.data_ptr())
    torch.cuda.synchronize()
    g = np.transpose(out[:, :, :O.types["tet"].nelem].cpu().numpy(), (2, 0, 1))
    d = g - Uo["tet"]
    err = np.sqrt((d ** 2).sum(axis=(0, 1)) / (Uo["tet"] ** 2).sum(axis=(0, 1)))
    print("  field errors", err, flush=True)
    assert (err < 1e-12).all(), err


def test_rk45_steps_fp64_hybrid():
    """Five fixed RK45[2R+] steps of NS on the three-type box (p = 2) against
    the oracle's stepper, every type to 1e-12."""
    frlib = _lib()
    print("rk45 hybrid fp64", flush=True)
    arrays = _mesh("hybrid", seed=1)
    p, mu, nsteps = 2, 0.02, 5
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system="ns", mu=mu)
    U0 = _state(O, inputs.taylor_green, 5, mach=0.3)
    dt = 0.2 * (2 * math.pi / 6) / ((1 + 1 / 0.3) * (2 * p + 1))
    Uo = rk.run(rk.rk45_step, lambda V: fr.rhs(O, V, prm), U0, dt, nsteps)
    M = frlib.Mesh(arrays, p, system="ns", precision="fp64", mu=mu, check_finite=True)
    for n in O.types:
        t = NAMES.index(n)
        M.set_solution(t, frlib.to_device_state(M, t, np.transpose(U0[n], (1, 2, 0))).data_ptr())
    M.rk_step(frlib.FR_RK45_2RP, dt, nsteps)
    for n in O.types:
        t = NAMES.index(n)
        out = frlib.state_tensor(M, t)
        M.get_solution(t, out.data_ptr())
        torch.cuda.synchronize()
        g = np.transpose(out[:, :, :O.types[n].nelem].cpu().numpy(), (2, 0, 1))
        d = g - Uo[n]
        err = np.sqrt((d ** 2).sum(axis=(0, 1)) / (Uo[n] ** 2).sum(axis=(0, 1)))
        print(f"  {n} field errors", err, flush=True)
        assert (err < 1e-12).all(), (n, err)


@pytest.mark.parametrize("kind", ["wallbox", "farbox"])
def test_boundary_flux_balance_fp64(kind):
    """FP64 library: the integral of R(U) equals minus the boundary flux
    summed with the reference face weights (the oracle's quantities), and no
    mass crosses a wall."""
    frlib = _lib()
    arrays = _mesh(kind, seed=4)
    p, mu = 3, 0.02
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system="ns", mu=mu, **BC[kind])
    U = _state(O, inputs.taylor_green, 2, mach=0.3)
    want = {}
    Ro = fr.rhs(O, U, prm, want=want)
    M = frlib.Mesh(arrays, p, system="ns", precision="fp64", mu=mu, **BC[kind])
    for n in O.types:
        t = NAMES.index(n)
        M.set_solution(t, frlib.to_device_state(M, t, np.transpose(U[n], (1, 2, 0))).data_ptr())
    torch.cuda.synchronize()
    ir = M.reduce(frlib.FR_RED_INT_R)
    om_ = np.zeros(O.nfpts_total)
    for n, tg in O.types.items():
        o = O.fpt_offset[n]
        om_[o:o + tg.nelem * tg.ref.nfpts] = np.tile(tg.ref.w @ tg.ref.L, tg.nelem)
    Fn = np.concatenate([want["Fn"][n].reshape(-1, 5) for n in O.types])
    bflux = (om_[O.bnd_idx, None] * Fn[O.bnd_idx]).sum(axis=0)
    scale = reduce.integral(O, {n: np.abs(Ro[n]) for n in Ro})
    print(f"  integral R {ir}, boundary flux {bflux}", flush=True)
    assert np.all(np.abs(ir + bflux) <= 1e-11 * scale), (ir, bflux)
    if kind == "wallbox":
        assert abs(ir[0]) <= 1e-11 * scale[0]


def test_rk45_adaptive_fp64_vortex():
    """Adaptive RK45[2R+] (embedded error, PI controller) on the small Euler
    workload against the oracle's driver: the same accepted and rejected
    attempts (two rejections from an oversized first step), the same final
    time, step size and controller state, and the same solution to 1e-12.
    Every error norm of the oracle run is far from the accept threshold 1,
    so both sides take the same decisions."""
    frlib = _lib()
    print("rk45 adaptive fp64", flush=True)
    arrays = inputs.vortex_tet_cube(n=6, jitter=0.05, seed=0)
    p = 2
    dt = _vortex_dt(6, p)
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system="euler")
    U0 = fr.initial_state(O, inputs.isentropic_vortex)
    tol, t_end = 1e-6, 8 * dt
    Uo, to, dto, epo, na, nr, errs = rk.rk45_adaptive(lambda V: fr.rhs(O, V, prm), U0, 0.0, t_end, 4 * dt, tol, tol)
    assert min(abs(np.array(errs) - 1.0)) > 1e-3 and nr >= 1
    M = frlib.Mesh(arrays, p, system="euler", precision="fp64", check_finite=True)
    u = frlib.to_device_state(M, 0, np.transpose(U0["tet"], (1, 2, 0)))
    M.set_solution(0, u.data_ptr())
    state = [0.0, 4 * dt, 1.0]
    acc, rej = M.rk45_adaptive(t_end, state, tol, tol)
    out = frlib.state_tensor(M, 0)
    M.get_solution(0, out.data_ptr())
    torch.cuda.synchronize()
    print(f"  accepted {acc} rejected {rej} (oracle {na}, {nr}); state {state} vs {[to, dto, epo]}", flush=True)
    assert (acc, rej) == (na, nr)
    assert state[0] == to
    assert abs(state[1] - dto) < 1e-9 * dto and abs(state[2] - epo) < 1e-9 * epo
    g = np.transpose(out[:, :, :O.types["tet"].nelem].cpu().numpy(), (2, 0, 1))
    d = g - Uo["tet"]
    err = np.sqrt((d ** 2).sum(axis=(0, 1)) / (Uo["tet"] ** 2).sum(axis=(0, 1)))
    assert (err < 1e-12).all(), err


def test_rk45_adaptive_fp32_ns_lands_on_t_end():
    """FP32 NS on the mixed parity mesh: the adaptive driver reaches t_end
    exactly, keeps the solution finite, and a second call continues from the
    returned controller state."""
    frlib = _lib()
    arrays = _mesh("mixed")
    O = om.build_mesh(arrays, 2)
    U = _round32(_state(O, inputs.taylor_green, 3, mach=0.3))
    M = frlib.Mesh(arrays, 2, system="ns", precision="fp32", mu=0.02, check_finite=True)
    for n in O.types:
        t = NAMES.index(n)
        u = frlib.to_device_state(M, t, np.transpose(U[n], (1, 2, 0)))
        M.set_solution(t, u.data_ptr())
    state = [0.0, 1e-3, 1.0]
    a1, r1 = M.rk45_adaptive(0.02, state, 1e-5, 1e-5)
    assert state[0] == 0.02 and a1 >= 1
    a2, r2 = M.rk45_adaptive(0.05, state, 1e-5, 1e-5)
    assert state[0] == 0.05 and a2 >= 1
    with pytest.raises(frlib.FrError):
        M.rk45_adaptive(0.1, [0.05, -1.0, 1.0], 1e-5, 1e-5)      # dt must be positive


@pytest.mark.parametrize("kind", ["mixed", "hybrid"])
def test_reductions_fp64(kind):
    """FP64 global sums: integral of U and of R(U) (discrete conservation) and
    the kinetic-energy rate, against the oracle's quadrature."""
    frlib = _lib()
    arrays = _mesh(kind, seed=5)
    p, mu = 3, 0.02
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system="ns", mu=mu)
    U = _state(O, inputs.taylor_green, 9, mach=0.3)
    Ro = fr.rhs(O, U, prm)
    M = frlib.Mesh(arrays, p, system="ns", precision="fp64", mu=mu)
    for n in O.types:
        t = NAMES.index(n)
        u = frlib.to_device_state(M, t, np.transpose(U[n], (1, 2, 0)))
        M.set_solution(t, u.data_ptr())
    torch.cuda.synchronize()
    iu = M.reduce(frlib.FR_RED_INT_U)
    assert np.allclose(iu, reduce.integral(O, U), rtol=1e-12, atol=0)
    ir = M.reduce(frlib.FR_RED_INT_R)
    scale = reduce.integral(O, {n: np.abs(Ro[n]) for n in Ro})
    assert (np.abs(ir) <= 1e-12 * scale).all(), ir / scale
    n2 = M.reduce(frlib.FR_RED_NORM2_R)
    assert np.allclose(n2, reduce.integral(O, {n: Ro[n] ** 2 for n in Ro}), rtol=1e-10)
    ke, dke = M.reduce(frlib.FR_RED_KE)
    assert abs(ke - reduce.kinetic_energy(O, U)) < 1e-12 * abs(ke)
    assert abs(dke - reduce.kinetic_energy_rate(O, U, Ro)) < 1e-9 * abs(dke)


@pytest.mark.parametrize("kind", ["mixed", "hybrid"])
def test_freestream_and_conservation_fp32(kind):
    """Uniform flow gives zero residual (up to FP32 rounding of the flux
    magnitude); the FP64 conservation sum of R(U) vanishes."""
    frlib = _lib()
    arrays = _mesh(kind, seed=6)
    p = 4
    O = om.build_mesh(arrays, p)
    M = frlib.Mesh(arrays, p, system="ns", precision="fp32", mu=0.01)
    U = _round32(fr.initial_state(O, inputs.uniform))
    Rg = _gpu_rhs(M, O, U)
    fscale = 5.0   # |flux| ~ p + rho u^2 ~ 1 for inputs.uniform
    worst = max(np.abs(Rg[n]).max() for n in Rg)
    print(f"  freestream max |R| {worst:.2e}", flush=True)
    assert worst < 1e-4 * fscale, worst
    # conservation: the FP64 sum of w J R(U) over the periodic mesh is zero
    # up to the FP32 rounding of the summed terms, for a state that is not
    # uniform (scale: the same sum over |R|, from the oracle)
    prm = fr.Params(system="ns", mu=0.01)
    V = _round32(_state(O, inputs.taylor_green, 7, mach=0.3))
    Ro = fr.rhs(O, V, prm)
    for n in O.types:
        t = NAMES.index(n)
        M.set_solution(t, _lib().to_device_state(M, t, np.transpose(V[n], (1, 2, 0))).data_ptr())
    torch.cuda.synchronize()
    ir = M.reduce(_lib().FR_RED_INT_R)
    scale = reduce.integral(O, {n: np.abs(Ro[n]) for n in Ro})
    print(f"  integral R / integral |R| {np.abs(ir) / scale}", flush=True)
    assert (np.abs(ir) <= 1e-5 * scale).all(), np.abs(ir) / scale


def test_nonfinite_state_is_reported():
    """FR_CHECK_FINITE: a NaN written into one state value through
    fr_set_solution makes fr_rk_step return FR_ERR_NONFINITE (the check is a
    device-side FP64 count of non-finite values after the steps); the same
    mesh with a finite state steps without error."""
    frlib = _lib()
    arrays = _mesh("mixed", seed=8)
    p = 2
    O = om.build_mesh(arrays, p)
    U = _round32(_state(O, inputs.taylor_green, 8, mach=0.3))
    M = frlib.Mesh(arrays, p, system="ns", precision="fp32", mu=0.02, check_finite=True)
    for n in O.types:
        t = NAMES.index(n)
        M.set_solution(t, frlib.to_device_state(M, t, np.transpose(U[n], (1, 2, 0))).data_ptr())
    M.rk_step(frlib.FR_RK45_2RP, 1e-4, 2)
    torch.cuda.synchronize()
    bad = np.transpose(U["pri"], (1, 2, 0)).copy()
    bad[3, 4, 17] = np.nan                      # energy at solution point 3 of prism 17
    M.set_solution(1, frlib.to_device_state(M, 1, bad).data_ptr())
    with pytest.raises(frlib.FrError) as ei:
        M.rk_step(frlib.FR_RK45_2RP, 1e-4, 1)
    assert ei.value.status == frlib.FR_ERR_NONFINITE, ei.value
    print(f"  {ei.value}", flush=True)
