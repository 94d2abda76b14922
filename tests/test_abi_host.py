"""CPU tests of the C ABI: the library loads, exports every entry point that
include/fr.h declares, and its host-side logic (validate-only meshes, no GPU)
matches the oracle: operators built by an independent route, solution-point
coordinates, and the error codes of bad inputs."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import elements, mesh as om
from paper_1409_0405_amd import frlib, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fr.h")).read()
    return sorted(set(re.findall(r"^(?:fr_status|const char \*)\s*(fr_\w+)\(", src, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(frlib.EXPORTED)


def test_header_constants_match_binding():
    """Every #define FR_* and enum constant of the header has the binding's
    value (flags, element types, boundary kinds, precisions, schemes)."""
    src = open(os.path.join(ROOT, "include", "fr.h")).read()
    consts = {k: int(v, 0) for k, v in re.findall(r"^#define\s+(FR_\w+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", src, re.M)}
    consts.update({k: int(v) for k, v in re.findall(r"\b(FR_[A-Z0-9_]+)\s*=\s*(\d+)", src)})
    assert consts["FR_SEPARATE_UPDATE"] == 0x4
    checked = 0
    for k, v in consts.items():
        if hasattr(frlib, k):
            assert getattr(frlib, k) == v, k
            checked += 1
    assert checked >= 12
    assert consts["FR_NTYPES"] == frlib.NTYPES == len(frlib.TYPE_NAMES)
    assert consts["FR_PROF_NCLASS"] == len(frlib.PROF_CLASSES)
    assert (consts["FR_MLP_NPARAM"], consts["FR_MLP_NSTATS"]) == (frlib.MLP_NPARAM, frlib.MLP_NSTATS)


def test_library_exports_declared_symbols():
    L = frlib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    # and the shared object really carries them as dynamic symbols
    so = ctypes.CDLL(frlib._LIB_PATH)
    for name in _declared():
        assert ctypes.cast(getattr(so, name), ctypes.c_void_p).value


def _hybrid(seed=2):
    return inputs.hybrid_box(4, 3, 4, 2, 2, (6.0, 7.0, 5.5), jitter=0.12, seed=seed)


@pytest.mark.parametrize("p", (1, 2, 3, 4))
def test_operators_match_oracle(p):
    M = frlib.Mesh(_hybrid(), p, system="ns", validate_only=True)
    for t, name in enumerate(frlib.TYPE_NAMES):
        R = elements.get(name, p)
        assert np.abs(M.operator(t, 0) - R.M0).max() < 1e-13
        for k in range(3):
            assert np.abs(M.operator(t, 1 + k) - R.G[k]).max() < 5e-13
        assert np.abs(M.operator(t, 4) - R.L).max() < 1e-12
        assert np.abs(M.operator(t, 5)[0] - R.w).max() < 1e-13
        assert np.abs(M.operator(t, 6) - R.norm_ref).max() < 1e-15


@pytest.mark.parametrize("which", ["mixed", "hybrid"])
def test_upts_coords_match_oracle(which):
    arrays = (inputs.small_mixed_box(nxy=3, n_pri_layers=2, n_tet_layers=2, jitter=0.1, seed=3)
              if which == "mixed" else _hybrid(3))
    M = frlib.Mesh(arrays, 3, validate_only=True)
    O = om.build_mesh(arrays, 3)
    for t, name in enumerate(frlib.TYPE_NAMES):
        if name not in O.types:
            assert M.query(t)["nelem"] == 0
            continue
        x = M.upts_coords(t)
        assert np.abs(x - np.transpose(O.types[name].x_upts, (1, 2, 0))).max() < 1e-13
        q = M.query(t)
        assert q["nelem"] == O.types[name].nelem and q["ld"] % 64 == 0 and q["ld"] >= q["nelem"]


def test_full_size_mesh_validates():
    """The 110,592-prism / 196,608-tet periodic box builds and pairs."""
    M = frlib.Mesh(inputs.tgv_mixed_box(), 4, system="ns", validate_only=True)
    assert M.query(0)["nelem"] == 196608 and M.query(1)["nelem"] == 110592
    assert M.query(1)["nupts"] == 75 and M.query(1)["nfpts"] == 105


@pytest.mark.parametrize("p", (1, 4))
def test_curved_coordinates_and_operators_match_oracle(p):
    """Quadratically curved three-type box: solution-point positions from the
    library's quadratic map equal the oracle's."""
    arrays = inputs.curve(_hybrid(4), 0.03)
    M = frlib.Mesh(arrays, p, system="ns", validate_only=True)
    O = om.build_mesh(arrays, p)
    for t, name in enumerate(frlib.TYPE_NAMES):
        assert np.abs(M.upts_coords(t) - np.transpose(O.types[name].x_upts, (1, 2, 0))).max() < 1e-12


def test_hex_box_sizes_validate():
    """Table 2 sizes of the hexahedron at p = 4 and the element count of a
    periodic hexahedral box."""
    M = frlib.Mesh(inputs.hex_box(12, jitter=0.1), 4, system="ns", validate_only=True)
    q = M.query(frlib.FR_HEX)
    assert (q["nelem"], q["nupts"], q["nfpts"]) == (1728, 125, 150)
    assert M.query(frlib.FR_TET)["nelem"] == 0 and M.query(frlib.FR_PRI)["nelem"] == 0


def _expect(status, fn):
    with pytest.raises(frlib.FrError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)
    return str(ei.value)


def test_error_codes():
    good = inputs.small_mixed_box(nxy=3, n_pri_layers=2, n_tet_layers=2, jitter=0.1)
    _expect(frlib.FR_ERR_UNSUPPORTED, lambda: frlib.Mesh(good, 5, validate_only=True))
    _expect(frlib.FR_ERR_UNSUPPORTED, lambda: frlib.Mesh(good, 0, validate_only=True))
    # inverted tet: swap two vertices
    bad = {k: v.copy() for k, v in good.items()}
    bad["tet_v"][7, [1, 2]] = bad["tet_v"][7, [2, 1]]
    bad["tet_img"][7, [1, 2]] = bad["tet_img"][7, [2, 1]]
    msg = _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(bad, 2, validate_only=True))
    assert "tet 7" in msg
    # unmatched face: drop an element
    bad = {k: v.copy() for k, v in good.items()}
    bad["pri_v"] = bad["pri_v"][1:]
    bad["pri_img"] = bad["pri_img"][1:]
    _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(bad, 2, validate_only=True))
    # non-coincident flux points: break a periodic image
    bad = {k: v.copy() for k, v in good.items()}
    bad["tet_img"][0, 3, 0] += 1
    _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(bad, 2, validate_only=True))
    # unknown system / bad constants
    _expect(frlib.FR_ERR_INVALID_ARG, lambda: frlib.Mesh(good, 2, validate_only=True, gamma=0.5))
    # inverted hexahedron: swap bottom and top
    bad = {k: v.copy() for k, v in _hybrid().items()}
    bad["hex_v"][5] = bad["hex_v"][5][[4, 5, 6, 7, 0, 1, 2, 3]]
    bad["hex_img"][5] = bad["hex_img"][5][[4, 5, 6, 7, 0, 1, 2, 3]]
    msg = _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(bad, 2, validate_only=True))
    assert "hex 5" in msg
    # a hexahedron face meeting two triangles is non-conforming: drop the
    # prism layer between hexahedra and tets
    hyb = _hybrid()
    nz_pri = len(hyb["pri_v"]) // 2                      # z-prisms come first
    bad = dict(hyb, pri_v=hyb["pri_v"][:nz_pri], pri_img=hyb["pri_img"][:nz_pri])
    _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(bad, 2, validate_only=True))
    # bounded box: a boundary face left unlisted, listed twice, or naming no face
    wall = inputs.hybrid_box(4, 3, 4, 2, 2, (6.0, 7.0, 5.5), jitter=0.1, seed=1, y_bc="wall")
    frlib.Mesh(wall, 2, validate_only=True)
    for bf in (wall["bfaces"][1:], np.concatenate([wall["bfaces"], wall["bfaces"][:1]]),
               np.concatenate([wall["bfaces"][1:], [[2, 10 ** 6, 0, 1]]])):
        _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(dict(wall, bfaces=bf), 2, validate_only=True))
    _expect(frlib.FR_ERR_INVALID_ARG, lambda: frlib.Mesh(wall, 2, validate_only=True, t_wall=-1.0))
    far = inputs.hybrid_box(4, 3, 4, 2, 2, (6.0, 7.0, 5.5), jitter=0.1, seed=1, y_bc="farfield")
    _expect(frlib.FR_ERR_INVALID_ARG,
            lambda: frlib.Mesh(far, 2, validate_only=True, farfield=(0.0, 0.0, 0.0, 0.0, 1.0)))
    # validate-only meshes refuse device work
    M = frlib.Mesh(good, 2, validate_only=True)
    _expect(frlib.FR_ERR_INVALID_ARG, lambda: M.rk_step(frlib.FR_RK4, 1e-3, 1))


def test_two_cell_periodic_mesh_validates():
    """Distinct faces sharing all vertex ids (periodic, two cells wide) are
    told apart; solution points match the oracle's."""
    arrays = inputs.mixed_box(2, 2, 2, 2, (1.0, 1.0, 1.0), z_split=0.5, jitter=0.05, seed=9)
    M = frlib.Mesh(arrays, 2, validate_only=True)
    O = om.build_mesh(arrays, 2)
    for t, name in enumerate(("tet", "pri")):
        assert np.abs(M.upts_coords(t) - np.transpose(O.types[name].x_upts, (1, 2, 0))).max() < 1e-13


def test_size_limits_and_degenerate_meshes():
    """The per-type element limit of the side word (2^22 - 1), an empty mesh,
    and a periodic direction one cell wide (a face would pair with itself):
    all refused with an error, never built."""
    base = inputs.hex_box(2)
    empty = dict(base, hex_v=np.zeros((0, 8), np.int64), hex_img=np.zeros((0, 8, 3), np.int8))
    _expect(frlib.FR_ERR_INVALID_ARG, lambda: frlib.Mesh(empty, 2, validate_only=True))
    n = 1 << 22
    big = dict(base, hex_v=np.zeros((n, 8), np.int64), hex_img=np.zeros((n, 8, 3), np.int8))
    msg = _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(big, 1, validate_only=True))
    assert "too many elements" in msg
    del big
    _expect(frlib.FR_ERR_BAD_MESH, lambda: frlib.Mesh(inputs.hex_box(1), 2, validate_only=True))
    with pytest.raises(ValueError):
        om.build_mesh(inputs.hex_box(1), 2)
