"""The gradient stage of the Navier-Stokes residual (corrected gradient
product, solution-point work, gradient interpolation) runs for tets, prisms
and hexahedra as one kernel per tile of elements with the reference and physical
gradients in LDS.  With FR_SEPARATE_GRADIENT it runs as three kernels that
pass those gradients through memory.  Both walk the same operator fragments
in the same order and share the point-wise arithmetic, so every result is
bitwise the same: the residual, the interface intermediates (state and
common flux at the flux points, the gradient where the common flux reads it)
and RK45[2R+] steps, in FP32 and FP64, on straight, curved and wall-bounded
meshes.  The fused kernel writes the flux-point gradient only on the faces
whose gradient is read; the others keep their initial zero.

The reference pressure p_ref left out of the momentum flux changes no
residual beyond rounding (the discrete divergence of a uniform flux vanishes
on these meshes): FP64 against the oracle to 1e-11 with and without it."""
import math

import numpy as np
import pytest

from gradient_points import read_points
from oracle import fr, mesh as om
from paper_1409_0405_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAMES = ("tet", "pri", "hex")
P0 = 1.0 / (1.4 * 0.09)      # Taylor-Green reference pressure at Mach 0.3


def _arrays(kind):
    if kind == "hybrid":
        return inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=2)
    if kind == "curvedwall":
        return inputs.curve(inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=2,
                                              y_bc="wall"), 0.03)
    if kind == "wallbox":
        return inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=2, y_bc="wall")
    if kind == "tiny":
        # 2 x 2 x (1 + 1): 8 prisms and 24 tets, fewer than one tile of each
        return inputs.small_mixed_box(nxy=2, n_pri_layers=1, n_tet_layers=1, jitter=0.1, seed=2)
    if kind == "hexbox":
        # 5 x 5 x 5 jittered hexahedra
        return inputs.hex_box(5, jitter=0.1, seed=2)
    if kind == "big":
        # 8 x 8 x (4 + 4): 512 prisms and 1,536 tets, many tiles of both types
        return inputs.small_mixed_box(nxy=8, n_pri_layers=4, n_tet_layers=4, jitter=0.1, seed=2)
    # 4 x 4 x (3 + 3): 96 prisms and 288 tets, ragged against the tiles
    return inputs.small_mixed_box(nxy=4, n_pri_layers=3, n_tet_layers=3, jitter=0.1, seed=2)


def _state(O, seed, mach=0.3):
    U = fr.initial_state(O, inputs.taylor_green, mach=mach)
    for n in U:
        U[n] = U[n] * inputs.random_perturbation(U[n].shape, seed, 0.01)
    return U


def _run(M, O, U, dt):
    """fr_rhs of U with its interface intermediates, then 3 RK45[2R+] steps
    from U; every result as a device tensor."""
    from paper_1409_0405_amd import frlib
    ts = [NAMES.index(n) for n in O.types]
    ptr = lambda d: [d[t].data_ptr() if t in d else 0 for t in range(3)]
    u = {t: frlib.to_device_state(M, t, np.transpose(U[NAMES[t]], (1, 2, 0))) for t in ts}
    r = {t: frlib.state_tensor(M, t) for t in ts}
    M.profile(True)
    M.rhs(ptr(u), ptr(r))
    prof = M.profile_read()
    M.profile(False)
    inter = {}
    for t in ts:
        q = M.query(t)
        for which, nv in ((0, 5), (1, 5), (2, 15)):
            buf = torch.zeros((q["nfpts"], nv, q["ld"]), dtype=r[t].dtype, device="cuda")
            M.intermediate(t, which, buf.data_ptr())
            inter[(t, which)] = buf
    for t in ts:
        M.set_solution(t, u[t].data_ptr())
    M.rk_step(frlib.FR_RK45_2RP, dt, 3)
    s = {t: frlib.state_tensor(M, t) for t in ts}
    for t in ts:
        M.get_solution(t, s[t].data_ptr())
    torch.cuda.synchronize()
    return r, inter, s, prof


def same_bits(a, b):
    """Bit-for-bit equality of two float tensors (torch.equal compares values,
    so +0 and -0 would pass it)."""
    it = torch.int32 if a.dtype == torch.float32 else torch.int64
    return a.shape == b.shape and a.dtype == b.dtype and torch.equal(a.view(it), b.view(it))


CASES = [("mixed", 1, "fp32"), ("mixed", 2, "fp32"), ("mixed", 3, "fp32"), ("mixed", 4, "fp32"),
         ("mixed", 2, "fp64"), ("mixed", 4, "fp64"), ("big", 4, "fp32"), ("hybrid", 3, "fp32"),
         ("hybrid", 3, "fp64"), ("hybrid", 4, "fp32"), ("curvedwall", 3, "fp32"), ("wallbox", 2, "fp64"),
         ("hexbox", 4, "fp32"), ("hexbox", 2, "fp64"), ("hexbox", 1, "fp32"), ("tiny", 4, "fp32"),
         ("tiny", 3, "fp64")]


@pytest.mark.parametrize("kind,p,prec", CASES, ids=[f"{k}-p{p}-{q}" for k, p, q in CASES])
def test_fused_gradient_stage_gives_the_bits_of_the_separate_kernels(kind, p, prec):
    from paper_1409_0405_amd import frlib
    arrays = _arrays(kind)
    O = om.build_mesh(arrays, p)
    U = _state(O, 4)
    kw = {"t_wall": P0} if kind in ("curvedwall", "wallbox") else {}
    out = []
    for separate in (False, True):
        print(f"{kind} p{p} {prec} separate_gradient={separate}", flush=True)
        M = frlib.Mesh(arrays, p, system="ns", precision=prec, mu=0.02, separate_gradient=separate, **kw)
        if not separate:
            # the fused form, also where the default (chosen by the operator's
            # size before autotuning) would be the separate kernels
            for n in O.types:
                M.set_gradient_form(NAMES.index(n), 1)
        out.append(_run(M, O, U, 2e-3))
        M.close()
    (r0, i0, s0, p0), (r1, i1, s1, p1) = out
    ts = sorted(r0)
    rp = read_points(O)
    # the fused kernel ran for the types present, and only there
    for t in range(3):
        n, g = "gradflux_" + NAMES[t], "grad_" + NAMES[t]
        assert p0[n][1] == (1 if t in ts else 0) and p1[n][1] == 0, (n, p0[n], p1[n])
        assert p0[g][1] == 0 and p1[g][1] == (1 if t in ts else 0), (g, p0[g], p1[g])
    for t in ts:
        assert same_bits(r0[t], r1[t]), ("rhs", NAMES[t])
        ne = O.types[NAMES[t]].nelem
        for which in (0, 1):
            assert same_bits(i0[(t, which)][:, :, :ne], i1[(t, which)][:, :, :ne]), ("intermediate", which, NAMES[t])
        # the gradient at flux points: the same bits where the common flux
        # reads it; the fused kernel (of a fresh mesh) leaves the other
        # points at their initial zero, the separate kernels write them
        mask = torch.from_numpy(np.ascontiguousarray(rp[NAMES[t]].T)).to("cuda")[:, None, :]
        q0, q1 = i0[(t, 2)][:, :, :ne], i1[(t, 2)][:, :, :ne]
        assert same_bits(torch.where(mask, q0, 0), torch.where(mask, q1, 0)), ("Qf read", NAMES[t])
        assert not torch.where(mask, 0, q0).any(), ("Qf written off the read faces", NAMES[t])
        assert torch.where(mask, 0, q1).any()
        print(f"  {NAMES[t]}: gradient written at {float(mask.float().mean()):.3f} of the flux points", flush=True)
        assert same_bits(s0[t], s1[t]), ("rk45 steps", NAMES[t])
    assert max(float(r0[t].abs().max()) for t in ts) > 1e-3


@pytest.mark.parametrize("kind,p", [("mixed", 4), ("big", 4), ("mixed", 2), ("curvedwall", 3), ("hybrid", 1),
                                    ("hexbox", 3)])
def test_every_gradient_stage_form_gives_the_same_bits(kind, p):
    """FP32: the autotuner's forms of the gradient stage (separate kernels,
    fused per tile, fused and streaming for tets and prisms) give the same
    residual and flux-point gradient, whichever it picks; forced through
    fr_set_blocking's gradient-stage switch."""
    from paper_1409_0405_amd import frlib
    arrays = _arrays(kind)
    O = om.build_mesh(arrays, p)
    U = _state(O, 9)
    kw = {"t_wall": P0} if kind == "curvedwall" else {}
    ts = [NAMES.index(n) for n in O.types]
    rp = read_points(O)
    outs = []
    for form in (0, 1, 2):
        M = frlib.Mesh(arrays, p, system="ns", precision="fp32", mu=0.02, **kw)
        for t in ts:
            # the streaming form covers tets and prisms; hexahedra take the
            # fused one there
            M.set_gradient_form(t, min(form, 1) if t == 2 else form)
        r, inter, s, prof = _run(M, O, U, 2e-3)
        M.close()
        n_fused = sum(prof[k][1] for k in ("gradflux_tet", "gradflux_pri", "gradflux_hex"))
        assert (n_fused > 0) == (form > 0), (form, prof)
        outs.append((r, inter, s))
    for form in (1, 2):
        for t in ts:
            assert same_bits(outs[0][0][t], outs[form][0][t]), ("rhs", form, NAMES[t])
            ne = O.types[NAMES[t]].nelem
            mask = torch.from_numpy(np.ascontiguousarray(rp[NAMES[t]].T)).to("cuda")[:, None, :]
            assert same_bits(torch.where(mask, outs[0][1][(t, 2)][:, :, :ne], 0),
                             torch.where(mask, outs[form][1][(t, 2)][:, :, :ne], 0)), ("Qf", form)
            assert same_bits(outs[0][2][t], outs[form][2][t]), ("rk45", form, NAMES[t])


@pytest.mark.parametrize("kind,system", [("mixed", "ns"), ("hybrid", "ns"), ("mixed", "euler"),
                                         ("wallbox", "ns")])
def test_reference_pressure_keeps_the_residual_fp64(kind, system):
    """p_ref = the Taylor-Green reference pressure: FP64 residual against the
    oracle's plain residual to 1e-11 per field, as without it."""
    from paper_1409_0405_amd import frlib
    p = 3
    arrays = _arrays(kind)
    O = om.build_mesh(arrays, p)
    kw = {"t_wall": P0} if kind == "wallbox" else {}
    prm = fr.Params(system=system, mu=0.02, **kw)
    U = _state(O, 6)
    Ro = fr.rhs(O, U, prm)
    ts = [NAMES.index(n) for n in O.types]
    for pref in (0.0, P0):
        M = frlib.Mesh(arrays, p, system=system, precision="fp64", mu=0.02, p_ref=pref, **kw)
        u = {t: frlib.to_device_state(M, t, np.transpose(U[NAMES[t]], (1, 2, 0))) for t in ts}
        r = {t: frlib.state_tensor(M, t) for t in ts}
        M.rhs([u[t].data_ptr() if t in u else 0 for t in range(3)], [r[t].data_ptr() if t in r else 0 for t in range(3)])
        torch.cuda.synchronize()
        num = np.zeros(5)
        den = np.zeros(5)
        for t in ts:
            n = NAMES[t]
            g = np.transpose(r[t][:, :, :O.types[n].nelem].cpu().numpy(), (2, 0, 1))
            num += ((g - Ro[n]) ** 2).sum(axis=(0, 1))
            den += (Ro[n] ** 2).sum(axis=(0, 1))
        err = np.sqrt(num / den)
        print(f"  {kind} {system} p_ref={pref:.3f}: field errors {err}", flush=True)
        assert (err < 1e-11).all(), (pref, err)
        M.close()
