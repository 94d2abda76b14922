"""Thin ctypes binding of libfr.so (C ABI in include/fr.h).

Argument marshalling only: every step of the right-hand side runs in the HIP
library.  Device arrays are passed as raw pointers (``torch.Tensor.data_ptr()``)
together with a HIP stream handle (``torch.cuda.current_stream().cuda_stream``);
torch is used for device memory and streams only.

Loading fails loudly if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfr.so")

FR_OK, FR_ERR_INVALID_ARG, FR_ERR_BAD_MESH, FR_ERR_UNSUPPORTED = 0, 1, 2, 3
FR_ERR_OUT_OF_MEMORY, FR_ERR_DEVICE, FR_ERR_NONFINITE = 4, 5, 6
FR_TET, FR_PRI, FR_HEX = 0, 1, 2
NTYPES = 3
TYPE_NAMES = ("tet", "pri", "hex")
FR_EULER, FR_NAVIER_STOKES = 0, 1
FR_FP32, FR_FP64, FR_SPLIT_BF16, FR_SPLIT_FP16 = 0, 1, 2, 3
PRECISIONS = {"fp32": FR_FP32, "fp64": FR_FP64, "split_bf16": FR_SPLIT_BF16,
              "split_fp16": FR_SPLIT_FP16}
FR_RK4, FR_RK45_2RP, FR_FWD_EULER = 0, 1, 2
FR_VALIDATE_ONLY, FR_CHECK_FINITE, FR_SEPARATE_UPDATE, FR_SEPARATE_GRADIENT = 0x1, 0x2, 0x4, 0x8
FR_BC_WALL, FR_BC_FARFIELD = 1, 2
FR_RED_INT_U, FR_RED_INT_R, FR_RED_NORM2_R, FR_RED_KE = 1, 2, 3, 4

EXPORTED = ("fr_mesh_create", "fr_mesh_destroy", "fr_mesh_query", "fr_upts_coords",
            "fr_operator", "fr_set_solution", "fr_get_solution", "fr_rhs", "fr_rk_step",
            "fr_reduce", "fr_intermediate", "fr_profile", "fr_profile_read", "fr_autotune",
            "fr_batch_create", "fr_batch_destroy", "fr_batch_query", "fr_batch_upts_coords",
            "fr_batch_set_solution",
            "fr_batch_get_solution", "fr_batch_set_dt", "fr_batch_set_graph", "fr_batch_rk_step",
            "fr_batch_last_error", "fr_mlp_create", "fr_mlp_destroy", "fr_mlp_set_params",
            "fr_mlp_get_params", "fr_mlp_forward", "fr_mlp_grad", "fr_mlp_get_grad", "fr_mlp_adam",
            "fr_mlp_last_error", "fr_project", "fr_closure_moments", "fr_closure_features",
            "fr_closure_targets", "fr_set_blocking", "fr_rk45_adaptive",
            "fr_closure_attach", "fr_reduce_noalloc", "fr_last_error")
MLP_NPARAM, MLP_NSTATS = 13204, 280

PROF_CLASSES = ("interp_tet", "grad_tet", "gradinterp_tet", "div_tet",
                "interp_pri", "grad_pri", "gradinterp_pri", "div_pri",
                "upts_tet", "upts_pri", "common_solution", "common_flux",
                "negdivconf_tet", "negdivconf_pri", "closure_inputs", "closure_forward",
                "interp_hex", "grad_hex", "gradinterp_hex", "div_hex", "upts_hex", "negdivconf_hex",
                "boundary_solution", "boundary_flux", "gradflux_tet", "gradflux_pri", "gradflux_hex")


class FrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fr status {status}: {msg}")
        self.status = status


class fr_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32), ("system", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("ldg_beta", ctypes.c_double), ("ldg_tau", ctypes.c_double),
        ("n_vertices", ctypes.c_int64), ("xyz", ctypes.POINTER(ctypes.c_double)),
        ("n_tets", ctypes.c_int64), ("tet_v", ctypes.POINTER(ctypes.c_int64)),
        ("tet_img", ctypes.POINTER(ctypes.c_int8)),
        ("n_prisms", ctypes.c_int64), ("pri_v", ctypes.POINTER(ctypes.c_int64)),
        ("pri_img", ctypes.POINTER(ctypes.c_int8)),
        ("period", ctypes.c_double * 3),
        ("n_hex", ctypes.c_int64), ("hex_v", ctypes.POINTER(ctypes.c_int64)),
        ("hex_img", ctypes.POINTER(ctypes.c_int8)),
        ("n_bfaces", ctypes.c_int64), ("bfaces", ctypes.POINTER(ctypes.c_int64)),
        ("t_wall", ctypes.c_double), ("farfield", ctypes.c_double * 5),
        ("tet_q", ctypes.POINTER(ctypes.c_double)), ("pri_q", ctypes.POINTER(ctypes.c_double)),
        ("hex_q", ctypes.POINTER(ctypes.c_double)),
        ("p_ref", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libfr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise FrError(-1, f"{_LIB_PATH} is not built; run python -m paper_1409_0405_amd.build")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.fr_mesh_create.argtypes = [ctypes.POINTER(fr_mesh_desc), vp, ctypes.POINTER(vp)]
        L.fr_mesh_destroy.argtypes = [vp]
        L.fr_mesh_query.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.fr_upts_coords.argtypes = [vp, i32, ctypes.POINTER(dbl)]
        L.fr_operator.argtypes = [vp, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)]
        L.fr_set_solution.argtypes = [vp, i32, vp, vp]
        L.fr_get_solution.argtypes = [vp, i32, vp, vp]
        L.fr_rhs.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.fr_rk_step.argtypes = [vp, i32, dbl, i32, vp]
        L.fr_reduce.argtypes = [vp, i32, ctypes.POINTER(dbl), vp]
        L.fr_reduce_noalloc.argtypes = [vp, i32, ctypes.POINTER(dbl), vp]
        L.fr_intermediate.argtypes = [vp, i32, i32, vp, vp]
        L.fr_profile.argtypes = [vp, i32]
        L.fr_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.fr_autotune.argtypes = [vp, vp]
        L.fr_batch_create.argtypes = [i32, ctypes.POINTER(fr_mesh_desc), vp, ctypes.POINTER(vp)]
        L.fr_batch_destroy.argtypes = [vp]
        L.fr_batch_query.argtypes = [vp, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                     ctypes.POINTER(i64)]
        L.fr_batch_upts_coords.argtypes = [vp, i32, i32, ctypes.POINTER(dbl)]
        L.fr_batch_set_solution.argtypes = [vp, i32, i32, vp, vp]
        L.fr_batch_get_solution.argtypes = [vp, i32, i32, vp, vp]
        L.fr_batch_set_dt.argtypes = [vp, ctypes.POINTER(dbl), vp]
        L.fr_batch_set_graph.argtypes = [vp, i32]
        L.fr_batch_rk_step.argtypes = [vp, i32, i32, vp]
        L.fr_batch_last_error.argtypes = [vp]
        L.fr_batch_last_error.restype = ctypes.c_char_p
        fp, ip = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)
        L.fr_mlp_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
        L.fr_mlp_destroy.argtypes = [vp]
        L.fr_mlp_set_params.argtypes = [vp, fp]
        L.fr_mlp_get_params.argtypes = [vp, fp]
        L.fr_mlp_forward.argtypes = [vp, vp, i64, vp, vp, i32, vp]
        L.fr_mlp_grad.argtypes = [vp, vp, vp, vp, i64, vp, ctypes.POINTER(dbl), vp]
        L.fr_mlp_get_grad.argtypes = [vp, fp, vp]
        L.fr_mlp_adam.argtypes = [vp, ctypes.c_float, vp]
        L.fr_mlp_last_error.argtypes = [vp]
        L.fr_mlp_last_error.restype = ctypes.c_char_p
        L.fr_project.argtypes = [vp, ctypes.POINTER(vp), vp, ctypes.POINTER(vp), vp]
        L.fr_closure_moments.argtypes = [vp, ctypes.POINTER(vp), vp, vp]
        L.fr_closure_features.argtypes = [vp, ctypes.POINTER(vp), vp, vp, vp]
        L.fr_set_blocking.argtypes = [vp, i32, i32, i32, i32]
        L.fr_rk45_adaptive.argtypes = [vp, dbl, ctypes.POINTER(dbl), dbl, dbl, i32, ctypes.POINTER(i32), vp]
        L.fr_closure_targets.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, vp]
        L.fr_closure_attach.argtypes = [vp, vp, vp, i32]
        L.fr_last_error.argtypes = [vp]
        L.fr_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("fr_last_error", "fr_batch_last_error", "fr_mlp_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st, mesh_ptr=None):
    if st != FR_OK:
        msg = lib().fr_last_error(mesh_ptr).decode()
        raise FrError(st, msg)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _type_ptrs(ptrs):
    """Per-type device pointers (tet, prism, hexahedron) as the C array the
    ABI takes; missing trailing entries are NULL."""
    ptrs = list(ptrs or [])
    if len(ptrs) > NTYPES:
        raise ValueError("more pointers than element types")
    ptrs += [0] * (NTYPES - len(ptrs))
    return (ctypes.c_void_p * NTYPES)(*[ctypes.c_void_p(p or 0) for p in ptrs])


def make_desc(keep, mesh_arrays, order, system="euler", precision="fp32", gamma=1.4, mu=0.0,
              prandtl=0.71, ldg_beta=0.5, ldg_tau=0.1, validate_only=False, check_finite=False,
              t_wall=1.0, farfield=(1.0, 0.0, 0.0, 0.0, 1.0 / 1.4), separate_update=False,
              separate_gradient=False, p_ref=0.0):
    """fr_mesh_desc for the generator's mesh arrays; the numpy arrays it points
    into are appended to ``keep`` (they must outlive the create call).
    separate_update: FR_SEPARATE_UPDATE (-R~/J and the RK update as a kernel
    of their own instead of in the divergence product's store);
    separate_gradient: FR_SEPARATE_GRADIENT (the gradient stage as three
    kernels); p_ref: reference pressure left out of the momentum flux."""
    d = fr_mesh_desc()
    d.order = order
    d.system = {"euler": FR_EULER, "ns": FR_NAVIER_STOKES}[system]
    d.precision = PRECISIONS[precision]
    d.flags = ((FR_VALIDATE_ONLY if validate_only else 0) | (FR_CHECK_FINITE if check_finite else 0)
               | (FR_SEPARATE_UPDATE if separate_update else 0)
               | (FR_SEPARATE_GRADIENT if separate_gradient else 0))
    d.p_ref = float(p_ref)
    d.gamma, d.mu, d.prandtl, d.ldg_beta, d.ldg_tau = gamma, mu, prandtl, ldg_beta, ldg_tau
    xyz = np.ascontiguousarray(mesh_arrays["xyz"], dtype=np.float64)
    tv = np.ascontiguousarray(mesh_arrays["tet_v"], dtype=np.int64)
    ti = np.ascontiguousarray(mesh_arrays["tet_img"], dtype=np.int8)
    pv = np.ascontiguousarray(mesh_arrays["pri_v"], dtype=np.int64)
    pi = np.ascontiguousarray(mesh_arrays["pri_img"], dtype=np.int8)
    hv = np.ascontiguousarray(mesh_arrays.get("hex_v", np.zeros((0, 8))), dtype=np.int64)
    hi = np.ascontiguousarray(mesh_arrays.get("hex_img", np.zeros((0, 8, 3))), dtype=np.int8)
    keep += [xyz, tv, ti, pv, pi, hv, hi]
    d.n_vertices = len(xyz)
    d.xyz = _ptr(xyz, ctypes.c_double)
    d.n_tets = len(tv)
    d.tet_v = _ptr(tv, ctypes.c_int64) if len(tv) else None
    d.tet_img = _ptr(ti, ctypes.c_int8) if len(tv) else None
    d.n_prisms = len(pv)
    d.pri_v = _ptr(pv, ctypes.c_int64) if len(pv) else None
    d.pri_img = _ptr(pi, ctypes.c_int8) if len(pv) else None
    d.n_hex = len(hv)
    d.hex_v = _ptr(hv, ctypes.c_int64) if len(hv) else None
    d.hex_img = _ptr(hi, ctypes.c_int8) if len(hv) else None
    bf = np.ascontiguousarray(mesh_arrays.get("bfaces", np.zeros((0, 4))), dtype=np.int64).reshape(-1, 4)
    keep.append(bf)
    d.n_bfaces = len(bf)
    d.bfaces = _ptr(bf, ctypes.c_int64) if len(bf) else None
    for kind, nq in (("tet", 10), ("pri", 18), ("hex", 27)):
        q = mesh_arrays.get(f"{kind}_q")
        if q is not None and len(q):
            q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, nq, 3)
            keep.append(q)
            setattr(d, f"{kind}_q", _ptr(q, ctypes.c_double))
    d.t_wall = float(t_wall)
    for k in range(5):
        d.farfield[k] = float(farfield[k])
    for k in range(3):
        d.period[k] = float(mesh_arrays["period"][k])
    return d


class Mesh:
    """A mesh handle owning its library-side buffers (fr_mesh)."""

    def __init__(self, mesh_arrays, order, system="euler", precision="fp32", gamma=1.4,
                 mu=0.0, prandtl=0.71, ldg_beta=0.5, ldg_tau=0.1, validate_only=False,
                 check_finite=False, stream=0, t_wall=1.0, farfield=(1.0, 0.0, 0.0, 0.0, 1.0 / 1.4),
                 separate_update=False, separate_gradient=False, p_ref=0.0):
        self._keep = []
        d = make_desc(self._keep, mesh_arrays, order, system, precision, gamma, mu, prandtl,
                      ldg_beta, ldg_tau, validate_only, check_finite, t_wall, farfield, separate_update,
                      separate_gradient, p_ref)
        h = ctypes.c_void_p()
        _check(lib().fr_mesh_create(ctypes.byref(d), ctypes.c_void_p(stream), ctypes.byref(h)))
        self.h = h
        self.order, self.system, self.precision = order, system, precision
        self.dtype = np.float64 if precision == "fp64" else np.float32

    def autotune(self, stream=0):
        """Pick the fastest row blocking of every operator product; returns the
        library's report."""
        _check(lib().fr_autotune(self.h, ctypes.c_void_p(stream)), self.h)
        return lib().fr_last_error(self.h).decode()

    def close(self):
        if getattr(self, "h", None):
            lib().fr_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, etype):
        ne, ld = ctypes.c_int64(), ctypes.c_int64()
        nu, nf = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fr_mesh_query(self.h, etype, ctypes.byref(ne), ctypes.byref(nu),
                                   ctypes.byref(nf), ctypes.byref(ld)), self.h)
        return {"nelem": ne.value, "nupts": nu.value, "nfpts": nf.value, "ld": ld.value}

    def upts_coords(self, etype):
        q = self.query(etype)
        out = np.zeros((q["nupts"], 3, q["nelem"]))
        if q["nelem"]:
            _check(lib().fr_upts_coords(self.h, etype, _ptr(out, ctypes.c_double)), self.h)
        return out

    def operator(self, etype, which):
        r, c = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fr_operator(self.h, etype, which, None, ctypes.byref(r), ctypes.byref(c)), self.h)
        out = np.zeros((r.value, c.value))
        _check(lib().fr_operator(self.h, etype, which, _ptr(out, ctypes.c_double), None, None), self.h)
        return out

    def set_solution(self, etype, u_ptr, stream=0):
        _check(lib().fr_set_solution(self.h, etype, ctypes.c_void_p(u_ptr), ctypes.c_void_p(stream)), self.h)

    def get_solution(self, etype, u_ptr, stream=0):
        _check(lib().fr_get_solution(self.h, etype, ctypes.c_void_p(u_ptr), ctypes.c_void_p(stream)), self.h)

    def rhs(self, u_ptrs, r_ptrs, stream=0):
        U = _type_ptrs(u_ptrs)
        R = _type_ptrs(r_ptrs)
        _check(lib().fr_rhs(self.h, U, R, ctypes.c_void_p(stream)), self.h)

    def rk_step(self, scheme, dt, n_steps, stream=0):
        _check(lib().fr_rk_step(self.h, scheme, float(dt), int(n_steps), ctypes.c_void_p(stream)), self.h)

    def rk45_adaptive(self, t_end, state, atol, rtol, max_attempts=1000000, stream=0):
        """Adaptive RK45[2R+] to t_end; state = [t, dt, err_prev] (updated in
        place); returns (accepted, rejected)."""
        st = (ctypes.c_double * 3)(*[float(x) for x in state])
        cnt = (ctypes.c_int32 * 2)()
        _check(lib().fr_rk45_adaptive(self.h, float(t_end), st, float(atol), float(rtol), int(max_attempts), cnt,
                                      ctypes.c_void_p(stream)), self.h)
        state[:] = [st[0], st[1], st[2]]
        return int(cnt[0]), int(cnt[1])

    def reduce(self, what, stream=0):
        out = np.zeros(8)
        _check(lib().fr_reduce(self.h, what, _ptr(out, ctypes.c_double), ctypes.c_void_p(stream)), self.h)
        return out[:2] if what == FR_RED_KE else out[:5]


    def reduce_noalloc(self, what, stream=0):
        """fr_reduce through fr_reduce_noalloc (device scratch of the
        library's own; allocates nothing)."""
        out = np.zeros(8)
        _check(lib().fr_reduce_noalloc(self.h, int(what), _ptr(out, ctypes.c_double), ctypes.c_void_p(stream)), self.h)
        return out[:2] if what == FR_RED_KE else out[:5]
    def profile(self, enable):
        _check(lib().fr_profile(self.h, 1 if enable else 0), self.h)

    def profile_read(self):
        """{class name: (total ms, launches)} of the kernels recorded since
        profiling was enabled or last read."""
        ms = np.zeros(len(PROF_CLASSES))
        cnt = np.zeros(len(PROF_CLASSES), dtype=np.int64)
        _check(lib().fr_profile_read(self.h, _ptr(ms, ctypes.c_double), _ptr(cnt, ctypes.c_int64)), self.h)
        return {n: (float(ms[i]), int(cnt[i])) for i, n in enumerate(PROF_CLASSES)}

    def project_to(self, dst, u_ptrs, v_ptrs, stream=0):
        """L2-project a state of this mesh onto mesh dst (same elements)."""
        U = _type_ptrs(u_ptrs)
        V = _type_ptrs(v_ptrs)
        _check(lib().fr_project(self.h, U, dst.h, V, ctypes.c_void_p(stream)), self.h)

    def closure_moments(self, u_ptrs, mom_ptr, stream=0):
        U = _type_ptrs(u_ptrs)
        _check(lib().fr_closure_moments(self.h, U, ctypes.c_void_p(mom_ptr), ctypes.c_void_p(stream)), self.h)

    def closure_features(self, u_ptrs, stats_ptr, feat_ptr, stream=0):
        U = _type_ptrs(u_ptrs)
        _check(lib().fr_closure_features(self.h, U, ctypes.c_void_p(stats_ptr or 0), ctypes.c_void_p(feat_ptr),
                                         ctypes.c_void_p(stream)), self.h)

    def set_blocking(self, etype, op, cap, stage=0):
        _check(lib().fr_set_blocking(self.h, int(etype), int(op), int(cap), int(stage)), self.h)

    def set_gradient_form(self, etype, form):
        """Navier-Stokes gradient stage of an element type: 0 separate
        kernels, 1 fused per tile, 2 fused and streaming (FP32 tets and
        prisms)."""
        _check(lib().fr_set_blocking(self.h, int(etype), 4, 1, int(form)), self.h)

    def closure_targets(self, a_ptrs, b_ptrs, stats_ptr, out_ptr, stream=0):
        A = _type_ptrs(a_ptrs)
        B = _type_ptrs(b_ptrs)
        _check(lib().fr_closure_targets(self.h, A, B, ctypes.c_void_p(stats_ptr or 0), ctypes.c_void_p(out_ptr),
                                        ctypes.c_void_p(stream)), self.h)

    def closure_attach(self, net, stats_ptr=0, bf16_weights=True):
        _check(lib().fr_closure_attach(self.h, net.h if net is not None else None,
                                       ctypes.c_void_p(stats_ptr or 0), 1 if bf16_weights else 0), self.h)

    def intermediate(self, etype, which, dst_ptr, stream=0):
        _check(lib().fr_intermediate(self.h, etype, which, ctypes.c_void_p(dst_ptr),
                                     ctypes.c_void_p(stream)), self.h)


class Batch:
    """Many independent problems advanced together (fr_batch)."""

    def __init__(self, problems, system="euler", precision="fp32", stream=0, **kw):
        """problems: list of (mesh arrays, order)."""
        self._keep = []
        descs = (fr_mesh_desc * len(problems))()
        for i, (arrays, p) in enumerate(problems):
            descs[i] = make_desc(self._keep, arrays, p, system, precision, **kw)
        h = ctypes.c_void_p()
        st = lib().fr_batch_create(len(problems), descs, ctypes.c_void_p(stream), ctypes.byref(h))
        if st != FR_OK:
            raise FrError(st, lib().fr_batch_last_error(None).decode())
        self.h = h
        self.n = len(problems)
        self.precision = precision
        self.orders = [p for _, p in problems]

    def _check(self, st):
        if st != FR_OK:
            raise FrError(st, lib().fr_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().fr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, problem, etype):
        ne, ld = ctypes.c_int64(), ctypes.c_int64()
        nu = ctypes.c_int32()
        self._check(lib().fr_batch_query(self.h, problem, etype, ctypes.byref(ne), ctypes.byref(nu),
                                         ctypes.byref(ld)))
        return {"nelem": ne.value, "nupts": nu.value, "ld": ld.value}

    def upts_coords(self, problem, etype):
        q = self.query(problem, etype)
        out = np.zeros((q["nupts"], 3, q["nelem"]))
        if q["nelem"]:
            self._check(lib().fr_batch_upts_coords(self.h, problem, etype, _ptr(out, ctypes.c_double)))
        return out

    def set_solution(self, problem, etype, u_ptr, stream=0):
        self._check(lib().fr_batch_set_solution(self.h, problem, etype, ctypes.c_void_p(u_ptr),
                                                ctypes.c_void_p(stream)))

    def get_solution(self, problem, etype, u_ptr, stream=0):
        self._check(lib().fr_batch_get_solution(self.h, problem, etype, ctypes.c_void_p(u_ptr),
                                                ctypes.c_void_p(stream)))

    def set_dt(self, dts, stream=0):
        a = np.ascontiguousarray(dts, dtype=np.float64)
        self._check(lib().fr_batch_set_dt(self.h, _ptr(a, ctypes.c_double), ctypes.c_void_p(stream)))

    def set_graph(self, enable):
        self._check(lib().fr_batch_set_graph(self.h, 1 if enable else 0))

    def rk_step(self, scheme, n_steps, stream=0):
        self._check(lib().fr_batch_rk_step(self.h, scheme, int(n_steps), ctypes.c_void_p(stream)))

    def state_tensor(self, problem, etype, device="cuda"):
        import torch
        q = self.query(problem, etype)
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        return torch.zeros((q["nupts"], 5, max(q["ld"], 64)), dtype=dt, device=device)


class MLP:
    """The closure network (fr_mlp): weights, Adam state, gradient workspace."""

    def __init__(self, seed=0):
        h = ctypes.c_void_p()
        st = lib().fr_mlp_create(int(seed), ctypes.byref(h))
        if st != FR_OK:
            raise FrError(st, lib().fr_mlp_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != FR_OK:
            raise FrError(st, lib().fr_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().fr_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == MLP_NPARAM
        self._check(lib().fr_mlp_set_params(self.h, _ptr(a, ctypes.c_float)))

    def get_params(self):
        a = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(lib().fr_mlp_get_params(self.h, _ptr(a, ctypes.c_float)))
        return a

    def forward(self, x_ptr, n, y_ptr, stats_ptr=0, bf16_weights=False, stream=0):
        self._check(lib().fr_mlp_forward(self.h, ctypes.c_void_p(x_ptr), int(n), ctypes.c_void_p(stats_ptr or 0),
                                         ctypes.c_void_p(y_ptr), 1 if bf16_weights else 0,
                                         ctypes.c_void_p(stream)))

    def grad(self, x_ptr, t_ptr, n, idx_ptr=0, stats_ptr=0, want_loss=True, stream=0):
        loss = ctypes.c_double()
        self._check(lib().fr_mlp_grad(self.h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(t_ptr),
                                      ctypes.c_void_p(idx_ptr or 0), int(n), ctypes.c_void_p(stats_ptr or 0),
                                      ctypes.byref(loss) if want_loss else None, ctypes.c_void_p(stream)))
        return loss.value if want_loss else None

    def get_grad(self, stream=0):
        a = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(lib().fr_mlp_get_grad(self.h, _ptr(a, ctypes.c_float), ctypes.c_void_p(stream)))
        return a

    def adam(self, lr, stream=0):
        self._check(lib().fr_mlp_adam(self.h, float(lr), ctypes.c_void_p(stream)))


# ---------------------------------------------------------------------------
# torch helpers (device memory and streams only)
# ---------------------------------------------------------------------------

def state_tensor(mesh: Mesh, etype, device="cuda"):
    """Zeroed device state [n_upts][5][ld] of the mesh's dtype."""
    import torch
    q = mesh.query(etype)
    dt = torch.float64 if mesh.precision == "fp64" else torch.float32
    return torch.zeros((q["nupts"], 5, max(q["ld"], 64)), dtype=dt, device=device)


def to_device_state(mesh: Mesh, etype, U_host, device="cuda"):
    """Host array [n_upts][5][n_elem] -> padded device state."""
    import torch
    t = state_tensor(mesh, etype, device)
    ne = U_host.shape[2]
    t[:, :, :ne] = torch.as_tensor(np.ascontiguousarray(U_host), dtype=t.dtype).to(device)
    if ne < t.shape[2] and ne > 0:     # padding columns: copy a real element
        t[:, :, ne:] = t[:, :, :1]
    return t


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream
