"""CPU check of the full-size GPU test's premise: the oracle's Navier-Stokes
residual of an element, evaluated on the patch of its two neighbour layers
(outer faces as boundaries, elements in the full mesh's order), equals the
residual evaluated on the whole periodic mesh."""
import numpy as np
import pytest

from oracle import fr, mesh as om
from paper_1409_0405_amd import inputs

import test_gpu_fullsize as F


@pytest.mark.parametrize("which", ["mixed", "hybrid"])
def test_patch_residual_equals_full_mesh_residual(which):
    if which == "mixed":
        arrays = inputs.tgv_mixed_box(nxy=8, n_pri_layers=8, n_tet_layers=8, jitter=0.1, seed=2)
    else:
        arrays = inputs.hybrid_box(8, 8, 8, 4, 4, (2 * np.pi,) * 3, jitter=0.1, seed=2)
    p = 2
    O = om.build_mesh(arrays, p)
    prm = fr.Params(system="ns", mu=0.02)
    Uo = fr.initial_state(O, inputs.taylor_green, mach=0.3)
    for n in Uo:
        Uo[n] = Uo[n] * inputs.random_perturbation(Uo[n].shape, 4, 0.02)
    R = fr.rhs(O, Uo, prm)
    nb, _ = F._neighbours(arrays)
    counts = [len(arrays.get(f"{n}_v", [])) for n in F.NAMES]
    starts = np.cumsum([0] + counts)
    U = {t: np.transpose(Uo[n], (1, 2, 0)) for t, n in enumerate(F.NAMES) if n in Uo}
    sample = F._interior_sample(arrays, nb, 3, 1, [t for t in range(3) if counts[t]])
    assert len(sample) >= 6
    for g in sample:
        t = int(np.searchsorted(starts, g, side="right") - 1)
        pa, (tc, ic) = F._patch(arrays, g, nb)
        P = om.build_mesh(pa, p)
        Rp = fr.rhs(P, F._patch_state(U, g, nb, starts, P), prm)
        want = R[F.NAMES[t]][g - starts[t]]
        got = Rp[F.NAMES[tc]][ic]
        assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max(), (g, np.abs(got - want).max())
