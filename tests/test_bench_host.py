"""Host logic of the benchmark's measurement (no GPU): roofline pricing,
the autotuner report's variant parsing, and the measured-traffic table."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Mesh:
    """Stand-in for frlib.Mesh.query at p = 4."""
    SIZES = {0: (35, 60), 1: (75, 105), 2: (125, 150)}

    def query(self, t):
        nu, nf = self.SIZES[t]
        return {"nelem": 1000, "nupts": nu, "nfpts": nf, "ld": 1024}


def test_roofline_prices_above_and_below_the_ridge(bench):
    ridge = bench.PEAK_FP32_MFMA / bench.PEAK_HBM
    model = {"a": {"flops": 2 * ridge * 1e9, "bytes": 1e9}, "b": {"flops": 0.5 * ridge * 1e9, "bytes": 1e9}}
    ra = bench.roofline_of(model, 1e-3, "a")
    rb = bench.roofline_of(model, 1e-3, "b")
    assert ra["bound"] == "mfma" and ra["unit"] == "TFLOP/s"
    assert ra["achieved"] == pytest.approx(2 * ridge * 1e9 / 1e-3 / 1e12)
    assert rb["bound"] == "hbm" and rb["achieved"] == pytest.approx(1e9 / 1e-3 / 1e9)
    for r in (ra, rb):
        assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])


def test_step_list_kernels_are_priced_on_structural_work(bench):
    assert bench.walks_nonzeros("gradflux_pri", None)
    assert bench.walks_nonzeros("div_pri", (1, 6)) and bench.walks_nonzeros("grad_hex", (2, 5))
    assert not bench.walks_nonzeros("div_tet", (1, 1)) and not bench.walks_nonzeros("interp_tet", None)


def test_variant_of_reads_the_autotuner_report(bench):
    report = ("tet op0 cap 2 stage 0 80.1 us; tet op3 cap 1 stage 1 202.0 us; "
              "pri op0 cap 2 stage 1 128.5 us; pri op3 cap 1 stage 6 335.7 us; hex op2 cap 1 stage 5 158.7 us; ")
    m = _Mesh()
    # tets: 60 flux points = 4 row blocks, at most 2 per wavefront
    assert bench.variant_of(m, "interp_tet", report) == (2, 0)
    # tets: 35 solution points = 3 row blocks, one per wavefront
    assert bench.variant_of(m, "div_tet", report) == (1, 1)
    # prisms: 105 flux points = 7 row blocks over 4 wavefronts, 2 each at most
    assert bench.variant_of(m, "interp_pri", report) == (2, 1)
    assert bench.variant_of(m, "div_pri", report) == (1, 6)
    assert bench.variant_of(m, "gradinterp_hex", report) == (1, 5)
    assert bench.variant_of(m, "grad_pri", report) is None           # not in the report
    assert bench.variant_of(m, "common_flux", report) is None        # not a product


def test_measured_traffic_table_names_known_kernels(bench):
    from paper_1409_0405_amd import frlib
    assert os.path.exists(os.path.join(ROOT, bench.TRAFFIC_SOURCE))
    for (k, rb, stage), v in bench.MEASURED_TRAFFIC.items():
        assert k in frlib.PROF_CLASSES, k
        assert 0 <= stage <= 6 and rb >= 0 and v > 0
    # every kernel class of a headline right-hand side has a measured variant
    for k in ("gradflux_tet", "gradflux_pri", "interp_tet", "interp_pri", "div_tet", "div_pri",
              "common_flux", "common_solution"):
        assert any(key[0] == k for key in bench.MEASURED_TRAFFIC), k


def test_host_cores_honours_the_thread_limit(bench, monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.host_cores() == min(3, len(os.sched_getaffinity(0)))
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.host_cores() == len(os.sched_getaffinity(0))
