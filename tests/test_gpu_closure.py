"""GPU parity of the learned-closure path through the C ABI against the FP64
oracle (oracle/closure.py) on seeded inputs: projection between orders, P1
moments, network inputs and targets, the network's forward pass (FP32 and
BF16 weights), its gradient, the Adam update, and the order-1 residual with
the closure attached.

Tolerances: the projection runs in the mesh's scalar type (FP64: 1e-12
relative, operators built by two independent routes); moments, inputs and
the network run in FP32 (relative 1e-5 of the compared quantity's scale:
sums of at most ~130 products, unit roundoff 6e-8)."""
import numpy as np
import pytest

from oracle import closure as oc, fr, mesh as om
from paper_1409_0405_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAMES = ("tet", "pri")


def _lib():
    from paper_1409_0405_amd import frlib
    return frlib


def _arrays(seed=0):
    # 4 x 4 x (3 + 3): 96 prisms and 288 tets (ragged against 64)
    return inputs.small_mixed_box(nxy=4, n_pri_layers=3, n_tet_layers=3, jitter=0.1, seed=seed)


def _oracle_state(O, seed):
    U = fr.initial_state(O, inputs.taylor_green, mach=0.3)
    return {n: U[n] * inputs.random_perturbation(U[n].shape, seed, 0.05) for n in U}


def _to_dev(M, U):
    frlib = _lib()
    return [frlib.to_device_state(M, t, np.transpose(U[NAMES[t]], (1, 2, 0))) for t in (0, 1)]


def _from_dev(ts, O):
    out = {}
    for t in (0, 1):
        ne = O.types[NAMES[t]].nelem
        out[NAMES[t]] = np.transpose(ts[t][:, :, :ne].cpu().numpy().astype(np.float64), (2, 0, 1))
    return out


def _ptrs(ts):
    return [t.data_ptr() for t in ts]


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _bf16(theta):
    """Round-to-nearest-even of float32 values to bfloat16 (returned as float64)."""
    b = np.ascontiguousarray(theta, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _random_stats(rng):
    return (rng.normal(0, 1, oc.N_IN), rng.uniform(0.5, 2.0, oc.N_IN),
            rng.normal(0, 0.1, oc.N_OUT), rng.uniform(0.05, 0.2, oc.N_OUT))


def _stats_dev(st):
    return torch.as_tensor(np.concatenate(st).astype(np.float32), device="cuda")


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = oc.init_params(seed)
    th += rng.normal(0, 0.05, th.shape)          # non-zero biases too
    return th.astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,p_src,p_dst,tol", [
    ("fp64", 4, 1, 1e-12), ("fp64", 1, 3, 1e-12), ("fp64", 3, 2, 1e-12), ("fp32", 4, 1, 2e-6)])
def test_projection_parity(precision, p_src, p_dst, tol):
    print(f"projection {precision} {p_src}->{p_dst}", flush=True)
    frlib = _lib()
    arrays = _arrays()
    O = om.build_mesh(arrays, p_src)
    U = _oracle_state(O, 1)
    src = frlib.Mesh(arrays, p_src, system="euler", precision=precision)
    dst = frlib.Mesh(arrays, p_dst, system="euler", precision=precision)
    u = _to_dev(src, U)
    v = [frlib.state_tensor(dst, t) for t in (0, 1)]
    src.project_to(dst, _ptrs(u), _ptrs(v))
    src.project_to(dst, _ptrs(u), _ptrs(v))       # second call reuses the cached operator
    torch.cuda.synchronize()
    got = _from_dev(v, O)
    want = oc.project(U, p_src, p_dst)
    for n in NAMES:
        assert _rel(got[n], want[n]) < tol, n


@pytest.mark.parametrize("precision", ("fp64", "fp32"))
def test_moments_features_targets_parity(precision):
    print(f"moments/features {precision}", flush=True)
    frlib = _lib()
    p = 2
    arrays = _arrays(seed=2)
    O = om.build_mesh(arrays, p)
    U = _oracle_state(O, 3)
    B = _oracle_state(O, 4)
    if precision == "fp32":
        U = {n: U[n].astype(np.float32).astype(np.float64) for n in U}
        B = {n: B[n].astype(np.float32).astype(np.float64) for n in B}
    M = frlib.Mesh(arrays, p, system="euler", precision=precision)
    u, b = _to_dev(M, U), _to_dev(M, B)
    ntot = sum(O.types[n].nelem for n in NAMES)
    mom = torch.zeros((ntot, 20), dtype=torch.float32, device="cuda")
    M.closure_moments(_ptrs(u), mom.data_ptr())
    feat = torch.zeros((ntot, oc.N_IN), dtype=torch.float32, device="cuda")
    M.closure_features(_ptrs(u), 0, feat.data_ptr())
    rng = np.random.default_rng(5)
    st = _random_stats(rng)
    sd = _stats_dev(st)
    featn = torch.zeros_like(feat)
    M.closure_features(_ptrs(u), sd.data_ptr(), featn.data_ptr())
    tg = torch.zeros_like(mom)
    M.closure_targets(_ptrs(u), _ptrs(b), 0, tg.data_ptr())
    tgn = torch.zeros_like(mom)
    M.closure_targets(_ptrs(u), _ptrs(b), sd.data_ptr(), tgn.data_ptr())
    torch.cuda.synchronize()

    om_ = oc.moments(U, p)
    want_mom = np.concatenate([om_[n].reshape(-1, 20) for n in NAMES])
    got = mom.cpu().numpy()
    # per column: relative to the column's scale
    scale = np.abs(want_mom).max(axis=0) + 1e-30
    assert (np.abs(got - want_mom) / scale).max() < 1e-5

    want_feat = oc.features(O, U, p)
    sc = np.abs(want_feat).max(axis=0) + 1e-30
    assert (np.abs(feat.cpu().numpy() - want_feat) / sc).max() < 1e-5
    # neighbour structure is exact: zero blocks where (and only where) the oracle has them
    assert ((feat.cpu().numpy() == 0) == (want_feat == 0)).all()
    mx, sx, my, sy = st
    wantn = (want_feat - mx) / sx
    assert np.abs(featn.cpu().numpy() - wantn).max() < 1e-5 * (np.abs(want_feat).max() / sx.min() + 1)

    ob = oc.moments(B, p)
    want_t = want_mom - np.concatenate([ob[n].reshape(-1, 20) for n in NAMES])
    sct = np.abs(want_t).max(axis=0) + 1e-30
    assert (np.abs(tg.cpu().numpy() - want_t) / sct).max() < 1e-5
    wtn = (want_t - my) / sy
    assert (np.abs(tgn.cpu().numpy() - wtn) / (np.abs(wtn).max(axis=0) + 1)).max() < 1e-5


@pytest.mark.parametrize("bf16", (False, True))
def test_mlp_forward_parity(bf16):
    print(f"mlp forward bf16={bf16}", flush=True)
    frlib = _lib()
    rng = np.random.default_rng(11)
    n = 1000                                       # ragged against the 64-sample block
    x = rng.normal(0, 1.5, (n, oc.N_IN))
    th = _theta(3)
    st = _random_stats(rng)
    net = frlib.MLP(0)
    net.set_params(th)
    xd = torch.as_tensor(x.astype(np.float32), device="cuda")
    yd = torch.zeros((n, oc.N_OUT), dtype=torch.float32, device="cuda")
    sd = _stats_dev(st)
    net.forward(xd.data_ptr(), n, yd.data_ptr(), sd.data_ptr(), bf16_weights=bf16)
    yr = torch.zeros_like(yd)
    net.forward(xd.data_ptr(), n, yr.data_ptr(), 0, bf16_weights=bf16)
    torch.cuda.synchronize()
    mx, sx, my, sy = st
    xs = x.astype(np.float32).astype(np.float64)
    thw = _bf16(th) if bf16 else th
    y, _ = oc.mlp_forward(thw, (xs - mx) / sx)
    want = y * sy + my
    assert _rel(yd.cpu().numpy(), want) < 1e-5
    yraw, _ = oc.mlp_forward(thw, xs)
    assert _rel(yr.cpu().numpy(), yraw) < 1e-5
    if bf16:    # the rounding really is in effect
        y32, _ = oc.mlp_forward(th, xs)
        assert _rel(yr.cpu().numpy(), y32) > 1e-4


@pytest.mark.parametrize("n", (1, 777, 20000))
def test_mlp_grad_and_adam_parity(n):
    print(f"mlp grad n={n}", flush=True)
    frlib = _lib()
    rng = np.random.default_rng(n)
    rows = n + 321
    x = rng.normal(0, 1.5, (rows, oc.N_IN)).astype(np.float32)
    t = rng.normal(0, 0.1, (rows, oc.N_OUT)).astype(np.float32)
    idx = rng.permutation(rows)[:n].astype(np.int32)
    st = _random_stats(rng)
    th = _theta(7)
    net = frlib.MLP(0)
    net.set_params(th)
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    idd = torch.as_tensor(idx, device="cuda")
    sd = _stats_dev(st)
    loss = net.grad(xd.data_ptr(), td.data_ptr(), n, idx_ptr=idd.data_ptr(), stats_ptr=sd.data_ptr())
    g = net.get_grad().astype(np.float64)
    mx, sx, my, sy = st
    xn = (x[idx].astype(np.float64) - mx) / sx
    tn = (t[idx].astype(np.float64) - my) / sy
    want_loss, want_g = oc.mlp_loss_grad(th, xn, tn)
    assert abs(loss - want_loss) < 1e-5 * want_loss
    assert _rel(g, want_g) < 1e-4
    # without stats and index: rows 0..n of already-normalised data
    xnd = torch.as_tensor(xn.astype(np.float32), device="cuda")
    tnd = torch.as_tensor(tn.astype(np.float32), device="cuda")
    loss2 = net.grad(xnd.data_ptr(), tnd.data_ptr(), n)
    assert abs(loss2 - want_loss) < 1e-5 * want_loss
    # Adam: three steps from zero moments against the oracle update fed the
    # same (device) gradients
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    ref = th.copy()
    for step in range(1, 4):
        net.grad(xd.data_ptr(), td.data_ptr(), n, idx_ptr=idd.data_ptr(), stats_ptr=sd.data_ptr(),
                 want_loss=False)
        gs = net.get_grad().astype(np.float64)
        net.adam(1e-3)
        ref, m, v = oc.adam_step(ref, gs, m, v, step, 1e-3)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - ref).max() < 1e-6 * max(1.0, np.abs(ref).max()), step


@pytest.mark.parametrize("bf16", (False, True))
def test_rhs_with_closure_parity(bf16):
    """Order-1 residual with the closure attached: the oracle's residual plus
    its lifted network correction.  The mesh runs in FP64, the correction in
    FP32: the bound is 1e-11 of the residual plus 3e-5 of the correction
    (the input normalisation amplifies relative input rounding ~15x here)."""
    print(f"rhs + closure bf16={bf16}", flush=True)
    frlib = _lib()
    p = 1
    arrays = _arrays(seed=4)
    O = om.build_mesh(arrays, p)
    prm = fr.Params("ns", 1.4, 0.02)
    U = _oracle_state(O, 6)
    M = frlib.Mesh(arrays, p, system="ns", precision="fp64", mu=0.02)
    u = _to_dev(M, U)
    r = [frlib.state_tensor(M, t) for t in (0, 1)]
    rng = np.random.default_rng(8)
    # statistics that put the inputs near unit scale
    want_feat = oc.features(O, U, p)
    st = (want_feat.mean(0), want_feat.std(0) + 1e-3, rng.normal(0, 0.1, oc.N_OUT),
          rng.uniform(0.5, 1.0, oc.N_OUT))
    th = _theta(9)
    net = frlib.MLP(0)
    net.set_params(th)
    sd = _stats_dev(st)
    M.closure_attach(net, sd.data_ptr(), bf16_weights=bf16)
    M.rhs(_ptrs(u), _ptrs(r))
    torch.cuda.synchronize()
    got = _from_dev(r, O)
    R = fr.rhs(O, U, prm)
    st32 = tuple(np.asarray(a, dtype=np.float32).astype(np.float64) for a in st)
    C = oc.correction(O, U, p, _bf16(th) if bf16 else th, st32)
    for n in NAMES:
        err = np.linalg.norm(got[n] - (R[n] + C[n]))
        assert err < 1e-11 * np.linalg.norm(R[n]) + 3e-5 * np.linalg.norm(C[n]), n
        assert np.linalg.norm(C[n]) > 1e-3 * np.linalg.norm(R[n])       # the correction is not negligible
    # detaching restores the plain residual
    M.closure_attach(None)
    M.rhs(_ptrs(u), _ptrs(r))
    torch.cuda.synchronize()
    got = _from_dev(r, O)
    for n in NAMES:
        assert _rel(got[n], R[n]) < 1e-11


def test_trained_closure_reduces_apriori_dissipation_error():
    """The network trained by the library's own kernels on filtered order-4
    runs (reduced Taylor-Green box, 1,792 prisms + 3,072 tets, Re 1600, Ma
    0.1) brings the kinetic-energy dissipation rate of the order-1 residual
    at the filtered states of held-out snapshots much closer to the order-4
    rate than the order-1 residual without it; BF16 weights at inference
    keep that gain.  Measured against the plain order-4 solve."""
    import math
    from paper_1409_0405_amd import closure as cl, frlib
    print("closure vs order 4: generate", flush=True)
    arrays = inputs.tgv_mixed_box(nxy=8, n_pri_layers=14, n_tet_layers=8, jitter=0.1, seed=0)
    hi, lo = cl.tgv_meshes(arrays)
    n_snap, T_end = 21, 8.0
    h_ref = min(math.pi / 14, math.pi / 16)
    dt = cl.dt_for(4, h_ref, cfl=0.25)
    sb = max(1, round(T_end / (n_snap - 1) / dt))
    dt = T_end / (n_snap - 1) / sb
    cl.load_tgv(hi)
    X, Y, times, rates4, states = cl.generate(hi, lo, dt, n_snap, sb)
    ntot = X.shape[0] // n_snap
    test_s = np.arange(2, n_snap, 5)
    train_s = np.setdiff1d(np.arange(n_snap), test_s)
    rows = lambda ss: torch.as_tensor(np.concatenate([np.arange(s * ntot, (s + 1) * ntot) for s in ss]),
                                      device="cuda")
    Xtr, Ytr = X[rows(train_s)].contiguous(), Y[rows(train_s)].contiguous()
    Xte, Yte = X[rows(test_s)].contiguous(), Y[rows(test_s)].contiguous()
    stats = cl.stats_of(Xtr, Ytr)
    print("closure vs order 4: train", flush=True)
    net, hist = cl.train(Xtr, Ytr, stats, epochs=40, batch=4096, lr=2e-3)
    assert hist[-1] < 0.6 * hist[0]
    # held-out targets: the network explains a good part of their variance
    yp = torch.zeros_like(Yte)
    net.forward(Xte.data_ptr(), len(Xte), yp.data_ptr(), stats.data_ptr())
    torch.cuda.synchronize()
    frac = (((yp - Yte) ** 2).sum(0) / ((Yte - Yte.mean(0)) ** 2).sum(0)).cpu().numpy()
    print("held-out unexplained variance per output", np.round(frac, 3), flush=True)
    assert frac.mean() < 0.7
    plain = cl.apriori_rates(lo, [states[s] for s in test_s])
    corr = cl.apriori_rates(lo, [states[s] for s in test_s], net, stats)
    corr16 = cl.apriori_rates(lo, [states[s] for s in test_s], net, stats, bf16_weights=True)
    ref = rates4[test_s]
    e = lambda r: float(np.sqrt(np.mean((r - ref) ** 2) / np.mean(ref ** 2)))
    print(f"a-priori dissipation-rate error vs order 4: plain {e(plain):.3e}, closure {e(corr):.3e}, "
          f"closure BF16 {e(corr16):.3e}", flush=True)
    assert e(corr) < 0.33 * e(plain)
    assert e(corr16) < 0.33 * e(plain)


def test_closure_trained_along_trajectory_runs_stably():
    """Trained on the order-1 run itself (inputs and order-1 residuals from
    U_1(t), targets against the filtered order-4 residual), the closure keeps
    the order-1 Taylor-Green run finite over t in [0, 8], and on this machine
    (8 x 8 x 22 cells) its kinetic-energy dissipation rate is closer to the
    plain order-4 run's than the plain order-1 run's is (relative L2 over the
    21 snapshots).  The gain is mesh dependent: on the 16 x 16 x 43 box the
    same recipe ends slightly worse than plain order 1."""
    import math
    from paper_1409_0405_amd import closure as cl, frlib
    print("closure along the trajectory: generate", flush=True)
    arrays = inputs.tgv_mixed_box(nxy=8, n_pri_layers=14, n_tet_layers=8, jitter=0.1, seed=0)
    hi = frlib.Mesh(arrays, 4, system="ns", precision="fp32", mu=1.0 / 1600.0, check_finite=True)
    lo = frlib.Mesh(arrays, 1, system="ns", precision="fp32", mu=1.0 / 1600.0, check_finite=True)
    n_int, T_end = 20, 8.0
    h_ref = min(math.pi / 14, math.pi / 16)
    dt4, dt1 = cl.dt_for(4, h_ref, cfl=0.25), cl.dt_for(1, h_ref, cfl=0.25)
    sb4, sb1 = max(1, round(T_end / n_int / dt4)), max(1, round(T_end / n_int / dt1))
    dt4, dt1 = T_end / n_int / sb4, T_end / n_int / sb1
    cl.load_tgv(hi)
    cl.load_filtered(hi, lo)
    X, Y, times, rates4, _ = cl.generate_along_trajectory(hi, lo, dt4, sb4, dt1, sb1, n_int + 1)
    stats = cl.stats_of(X, Y)
    print("closure along the trajectory: train", flush=True)
    net, hist = cl.train(X, Y, stats, epochs=30, batch=4096, lr=2e-3)
    assert hist[-1] < hist[0]

    def run(with_net):
        cl.load_tgv(hi)
        cl.load_filtered(hi, lo)
        if with_net:
            lo.closure_attach(net, stats.data_ptr(), bf16_weights=True)
        try:
            return cl.dissipation_history(lo, dt1, n_int + 1, sb1)
        finally:
            lo.closure_attach(None)
    plain, corr = run(False), run(True)
    assert np.isfinite(corr).all()
    e = lambda r: float(np.sqrt(np.mean((r - rates4) ** 2) / np.mean(rates4 ** 2)))
    print(f"a-posteriori dissipation-rate error vs order 4: plain {e(plain):.3f}, closure {e(corr):.3f}",
          flush=True)
    assert e(corr) < e(plain), (e(corr), e(plain))


def test_closure_refuses_hexahedra():
    """The closure's neighbour stencil covers tets and prisms: on a mesh with
    hexahedra the closure entry points report FR_ERR_UNSUPPORTED."""
    frlib = _lib()
    arrays = inputs.hybrid_box(4, 3, 4, 2, 2, (2 * np.pi,) * 3, jitter=0.1, seed=1)
    M = frlib.Mesh(arrays, 1, system="ns", precision="fp32", mu=0.02)
    net = frlib.MLP(seed=0)
    stats = torch.ones(frlib.MLP_NSTATS, dtype=torch.float32, device="cuda")
    ntot = sum(M.query(t)["nelem"] for t in range(3))
    mom = torch.zeros((ntot, 20), dtype=torch.float32, device="cuda")
    for call in (lambda: M.closure_attach(net, stats.data_ptr(), bf16_weights=True),
                 lambda: M.closure_moments([0, 0, 0], mom.data_ptr())):
        with pytest.raises(frlib.FrError) as ei:
            call()
        assert ei.value.status == frlib.FR_ERR_UNSUPPORTED
