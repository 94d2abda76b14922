"""The last pipeline step, -R~/J followed by the RK register update (FR's
pointwise 1/J and the 2-register RK45[2R+] / RK4 updates), runs in the
divergence products' store by default.  With FR_SEPARATE_UPDATE it runs as
a kernel of its own after the product, which first writes R~ to memory.
Both orders of work do the same arithmetic on the same values, so every
result is bitwise the same:

* fr_rhs, fixed RK45[2R+] and RK4 steps, and the adaptive RK45[2R+] with
  its error register;
* a batch of problems with per-problem step sizes;
* FP32, FP64 and the split BF16 / FP16 forms, on the mixed tet/prism box and
  the three-type box (element counts ragged against the 64-column panels).
"""
import math

import numpy as np
import pytest

from oracle import fr, mesh as om
from paper_1409_0405_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAMES = ("tet", "pri", "hex")


def _arrays(kind):
    if kind == "hybrid":
        return inputs.hybrid_box(6, 4, 6, 3, 3, (2 * math.pi,) * 3, jitter=0.1, seed=2)
    return inputs.small_mixed_box(nxy=4, n_pri_layers=3, n_tet_layers=3, jitter=0.1, seed=2)


def _run(M, U, ts, dt):
    """fr_rhs of U, then 3 RK45[2R+] and 2 RK4 steps from U, then the
    adaptive RK45[2R+] to a short end time; returns every result."""
    from paper_1409_0405_amd import frlib
    ptr = lambda d: [d[t].data_ptr() if t in d else 0 for t in range(3)]
    u = {t: frlib.to_device_state(M, t, np.transpose(U[NAMES[t]], (1, 2, 0))) for t in ts}
    r = {t: frlib.state_tensor(M, t) for t in ts}
    M.rhs(ptr(u), ptr(r))
    for t in ts:
        M.set_solution(t, u[t].data_ptr())
    M.rk_step(frlib.FR_RK45_2RP, dt, 3)
    M.rk_step(frlib.FR_RK4, dt, 2)
    s = {t: frlib.state_tensor(M, t) for t in ts}
    for t in ts:
        M.get_solution(t, s[t].data_ptr())
    state = [0.0, dt, 1.0]
    counts = M.rk45_adaptive(8 * dt, state, 1e-5, 1e-5)
    a = {t: frlib.state_tensor(M, t) for t in ts}
    for t in ts:
        M.get_solution(t, a[t].data_ptr())
    torch.cuda.synchronize()
    return r, s, a, counts, state


@pytest.mark.parametrize("kind,prec", [("mixed", "fp32"), ("mixed", "fp64"), ("hybrid", "fp32"),
                                       ("hybrid", "fp64"), ("mixed", "split_bf16"), ("hybrid", "split_fp16")])
def test_fused_update_gives_the_bits_of_the_separate_kernel(kind, prec):
    from paper_1409_0405_amd import frlib
    p = 3
    arrays = _arrays(kind)
    O = om.build_mesh(arrays, p)
    U = fr.initial_state(O, inputs.taylor_green, mach=0.3)
    ts = [NAMES.index(n) for n in O.types]
    dt = 2e-3
    out = []
    for separate in (False, True):
        print(f"{kind} {prec} separate_update={separate}", flush=True)
        M = frlib.Mesh(arrays, p, system="ns", precision=prec, mu=0.02, separate_update=separate)
        out.append(_run(M, U, ts, dt))
        M.close()
    (r0, s0, a0, c0, st0), (r1, s1, a1, c1, st1) = out
    for t in ts:
        assert torch.equal(r0[t], r1[t]), ("rhs", NAMES[t])
        assert torch.equal(s0[t], s1[t]), ("rk steps", NAMES[t])
        assert torch.equal(a0[t], a1[t]), ("adaptive", NAMES[t])
    assert c0 == c1 and st0 == st1
    assert c0[0] >= 2
    # the residual is not trivially zero
    assert max(float(r0[t].abs().max()) for t in ts) > 1e-3


def test_fused_update_batch_with_per_problem_steps_fp32():
    from paper_1409_0405_amd import frlib
    probs = inputs.batch_problems(n=4, seed=3, e_min=64, e_max=500)
    res = []
    for separate in (False, True):
        print(f"batch separate_update={separate}", flush=True)
        B = frlib.Batch([(b["mesh"], b["p"]) for b in probs], system="euler", precision="fp32",
                        separate_update=separate)
        for i, b in enumerate(probs):
            O = om.build_mesh(b["mesh"], b["p"])
            U = fr.initial_state(O, inputs.isentropic_vortex, centre=b["centre"], radius=0.15)
            for t, n in enumerate(NAMES[:2]):
                q = B.query(i, t)
                if q["nelem"]:
                    x = B.state_tensor(i, t)
                    x[:, :, :q["nelem"]] = torch.as_tensor(np.transpose(U[n], (1, 2, 0)), dtype=x.dtype)
                    x[:, :, q["nelem"]:] = x[:, :, :1]
                    B.set_solution(i, t, x.data_ptr())
        torch.cuda.synchronize()
        lam = 1.5 * math.sqrt(1.4)
        B.set_dt([0.2 * (0.5 / b["m"]) / (lam * (2 * b["p"] + 1)) for b in probs])
        B.rk_step(frlib.FR_RK45_2RP, 3)
        got = []
        for i in range(len(probs)):
            for t in range(2):
                x = B.state_tensor(i, t)
                B.get_solution(i, t, x.data_ptr())
                got.append(x)
        torch.cuda.synchronize()
        res.append(got)
        B.close()
    for x, y in zip(*res):
        assert torch.equal(x, y)
