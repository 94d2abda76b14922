"""fr_reduce_noalloc: the reductions of fr_reduce with the partial sums and
results in the library's own per-GPU device array instead of the mesh's
buffers.  Through the C-ABI on two meshes in a row, the second smaller than
the first (and in the other precision), every item must give the bits of
fr_reduce on the same mesh and state; the array keeps the first call's
contents, so a stale value would show in the second."""
import math

import numpy as np
import pytest

from oracle import fr, mesh as om
from paper_1409_0405_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAMES = ("tet", "pri", "hex")


def _mesh_and_state(arrays, p, system, prec, seed):
    from paper_1409_0405_amd import frlib
    O = om.build_mesh(arrays, p)
    U = fr.initial_state(O, inputs.taylor_green, mach=0.3)
    for n in U:
        U[n] = U[n] * inputs.random_perturbation(U[n].shape, seed, 0.01)
    M = frlib.Mesh(arrays, p, system=system, precision=prec, mu=0.02)
    keep = []
    for n in O.types:
        t = NAMES.index(n)
        u = frlib.to_device_state(M, t, np.transpose(U[n], (1, 2, 0)))
        M.set_solution(t, u.data_ptr())
        keep.append(u)
    torch.cuda.synchronize()
    return M


def test_noalloc_reduce_gives_the_bits_of_fr_reduce_on_two_meshes_in_a_row():
    from paper_1409_0405_amd import frlib
    big = inputs.small_mixed_box(nxy=8, n_pri_layers=4, n_tet_layers=4, jitter=0.1, seed=2)
    small = inputs.hybrid_box(3, 2, 3, 1, 1, (2 * math.pi,) * 3, jitter=0.1, seed=5)
    items = (frlib.FR_RED_INT_U, frlib.FR_RED_INT_R, frlib.FR_RED_NORM2_R, frlib.FR_RED_KE)
    for label, arrays, p, system, prec in (("big p3 ns fp64", big, 3, "ns", "fp64"),
                                           ("small p2 euler fp32", small, 2, "euler", "fp32")):
        print(f"fr_reduce_noalloc on {label}", flush=True)
        M = _mesh_and_state(arrays, p, system, prec, seed=7)
        for what in items:
            a = M.reduce_noalloc(what)
            b = M.reduce(what)
            assert np.isfinite(a).all() and np.abs(a).max() > 0, (label, what, a)
            assert np.array_equal(a, b), (label, what, a, b)
        # rejected item numbers leave the call without touching the device
        with pytest.raises(frlib.FrError):
            M.reduce_noalloc(5)
        M.close()
