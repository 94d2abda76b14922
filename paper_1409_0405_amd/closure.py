"""Learned subgrid closure: training data from the solver's own high-order
runs, training with the library's network kernels, and its a-posteriori
assessment on the kinetic-energy dissipation rate.

Pipeline (every numerical step runs in libfr; torch only holds device
memory; host numpy only draws the shuffles and forms the normalisation
statistics):

1. run order q (4) from the Taylor-Green state, and at snapshot times take
   U_q, its residual R_q(U_q), the projections Pi_1 U_q and Pi_1 R_q(U_q),
   and the order-1 residual R_1(Pi_1 U_q);
2. inputs  = P1 moments of Pi_1 U_q on each element and its face neighbours;
   targets = P1 moments of Pi_1 R_q(U_q) - R_1(Pi_1 U_q);
3. train the 120-64-64-20 network (Adam, mean squared error on normalised
   data);
4. run order 1 with and without the attached closure from Pi_1 U_q(0) and
   compare the kinetic-energy dissipation rate -dE_k/dt with order q's.

generate_along_trajectory() is the variant whose inputs and order-1
residuals come from the order-1 run itself (advanced beside order q), so the
network is trained on the states it is later applied to.
"""
from __future__ import annotations

import math

import numpy as np

from . import frlib, inputs


def _states(mesh):
    return [frlib.state_tensor(mesh, t) for t in (0, 1)]


def _ptrs(ts):
    return [t.data_ptr() for t in ts]


def tgv_meshes(arrays, q=4, mu=1.0 / 1600.0, prandtl=0.71, stream=0):
    hi = frlib.Mesh(arrays, q, system="ns", precision="fp32", mu=mu, prandtl=prandtl, stream=stream)
    lo = frlib.Mesh(arrays, 1, system="ns", precision="fp32", mu=mu, prandtl=prandtl, stream=stream)
    return hi, lo


def load_tgv(mesh, mach=0.1, stream=0):
    import torch
    for t in (0, 1):
        q = mesh.query(t)
        if not q["nelem"]:
            continue
        x = mesh.upts_coords(t)
        U = inputs.taylor_green(x[:, 0], x[:, 1], x[:, 2], mach=mach)
        u = frlib.to_device_state(mesh, t, np.transpose(U, (1, 0, 2)))
        mesh.set_solution(t, u.data_ptr(), stream)
        torch.cuda.synchronize()


def dt_for(order, h_min, mach=0.1, cfl=0.3):
    return cfl * h_min / ((1.0 + 1.0 / mach) * (2 * order + 1))


def generate(hi, lo, dt, n_snap, steps_between, stream=0):
    """Inputs [N][120] and targets [N][20] (device float32) from snapshots of
    the order-q run of mesh hi (whose solution register holds the state),
    plus the times, the order-q dissipation rates at the snapshots and the
    projected order-1 states (device tensors per element type)."""
    import torch
    ntot = sum(hi.query(t)["nelem"] for t in (0, 1))
    X = torch.zeros((n_snap, ntot, 120), dtype=torch.float32, device="cuda")
    Y = torch.zeros((n_snap, ntot, 20), dtype=torch.float32, device="cuda")
    uq, rq = _states(hi), _states(hi)
    u1, r1, pr = _states(lo), _states(lo), _states(lo)
    times, rates, states = [], [], []
    t_now = 0.0
    for k in range(n_snap):
        if k:
            hi.rk_step(frlib.FR_RK45_2RP, dt, steps_between, stream)
            t_now += dt * steps_between
        for t in (0, 1):
            hi.get_solution(t, uq[t].data_ptr(), stream)
        hi.rhs(_ptrs(uq), _ptrs(rq), stream)
        hi.project_to(lo, _ptrs(uq), _ptrs(u1), stream)
        hi.project_to(lo, _ptrs(rq), _ptrs(pr), stream)
        lo.rhs(_ptrs(u1), _ptrs(r1), stream)
        lo.closure_targets(_ptrs(pr), _ptrs(r1), 0, Y[k].data_ptr(), stream)
        lo.closure_features(_ptrs(u1), 0, X[k].data_ptr(), stream)
        torch.cuda.synchronize()
        times.append(t_now)
        rates.append(-hi.reduce(frlib.FR_RED_KE, stream)[1])
        states.append([x.clone() for x in u1])
    return X.reshape(-1, 120), Y.reshape(-1, 20), np.array(times), np.array(rates), states


def generate_along_trajectory(hi, lo, dt_hi, steps_hi, dt_lo, steps_lo, n_snap, stream=0, log=None):
    """Like generate(), but the inputs and the order-1 residual come from the
    order-1 solution itself, advanced beside the order-q run from the
    filtered initial state (both meshes hold their initial states): targets
    = P1 moments of Pi_1 R_q(U_q(t)) - R_1(U_1(t)).  The network then sees
    the states it will be applied to."""
    import torch
    ntot = sum(hi.query(t)["nelem"] for t in (0, 1))
    X = torch.zeros((n_snap, ntot, 120), dtype=torch.float32, device="cuda")
    Y = torch.zeros((n_snap, ntot, 20), dtype=torch.float32, device="cuda")
    uq, rq = _states(hi), _states(hi)
    u1, r1, pr = _states(lo), _states(lo), _states(lo)
    times, rates, states = [], [], []
    t_now = 0.0
    for k in range(n_snap):
        if k:
            hi.rk_step(frlib.FR_RK45_2RP, dt_hi, steps_hi, stream)
            lo.rk_step(frlib.FR_RK45_2RP, dt_lo, steps_lo, stream)
            t_now += dt_hi * steps_hi
        for t in (0, 1):
            hi.get_solution(t, uq[t].data_ptr(), stream)
            lo.get_solution(t, u1[t].data_ptr(), stream)
        hi.rhs(_ptrs(uq), _ptrs(rq), stream)
        hi.project_to(lo, _ptrs(rq), _ptrs(pr), stream)
        lo.rhs(_ptrs(u1), _ptrs(r1), stream)
        lo.closure_targets(_ptrs(pr), _ptrs(r1), 0, Y[k].data_ptr(), stream)
        lo.closure_features(_ptrs(u1), 0, X[k].data_ptr(), stream)
        torch.cuda.synchronize()
        times.append(t_now)
        rates.append(-hi.reduce(frlib.FR_RED_KE, stream)[1])
        states.append([x.clone() for x in u1])
        if log:
            log(f"snapshot {k + 1}/{n_snap}: t = {t_now:.3f}, order-{hi.order} dissipation rate {rates[-1]:.4e}")
    return X.reshape(-1, 120), Y.reshape(-1, 20), np.array(times), np.array(rates), states


def load_filtered(hi, lo, stream=0):
    """Order-1 solution of lo = L2 projection of the order-q solution of hi."""
    import torch
    uq, u1 = _states(hi), _states(lo)
    for t in (0, 1):
        hi.get_solution(t, uq[t].data_ptr(), stream)
    hi.project_to(lo, _ptrs(uq), _ptrs(u1), stream)
    for t in (0, 1):
        lo.set_solution(t, u1[t].data_ptr(), stream)
    torch.cuda.synchronize()


def stats_of(X, Y):
    """mu_x, s_x, mu_y, s_y (float32, FR_MLP_NSTATS values) from a sample."""
    import torch
    idx = np.random.default_rng(0).choice(len(X), min(len(X), 200000), replace=False)
    xs = X[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    ys = Y[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    sx = xs.std(0)
    sy = ys.std(0)
    sx[sx < 1e-12] = 1.0
    sy[sy < 1e-12] = 1.0
    st = np.concatenate([xs.mean(0), sx, ys.mean(0), sy]).astype(np.float32)
    return torch.as_tensor(st, device="cuda")


def train(X, Y, stats, epochs=20, batch=8192, lr=2e-3, seed=0, log=None):
    """Adam on the raw data, standardised by the gradient kernel with stats
    (cosine learning-rate decay, reshuffled every epoch); returns the network
    and the per-epoch loss on the normalised targets."""
    import torch
    net = frlib.MLP(seed)
    n = len(X)
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device="cuda")
        tot, cnt = 0.0, 0
        for b0 in range(0, n, batch):
            nb = min(batch, n - b0)
            loss = net.grad(X.data_ptr(), Y.data_ptr(), nb, idx_ptr=perm[b0:b0 + nb].data_ptr(),
                            stats_ptr=stats.data_ptr())
            step += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * min(1.0, step / max(1, epochs * math.ceil(n / batch)))))
            net.adam(lr_t)
            tot += loss * nb
            cnt += nb
        hist.append(tot / cnt)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return net, hist


def dissipation_history(mesh, dt, n_snap, steps_between, stream=0, log=None):
    """-dE_k/dt of the mesh's current solution at n_snap times."""
    out = []
    for k in range(n_snap):
        if k:
            mesh.rk_step(frlib.FR_RK45_2RP, dt, steps_between, stream)
        out.append(-mesh.reduce(frlib.FR_RED_KE, stream)[1])
        if log:
            log(f"snapshot {k + 1}/{n_snap}: dissipation rate {out[-1]:.4e}")
    return np.array(out)


def apriori_rates(lo, states, net=None, stats=None, bf16_weights=False, stream=0):
    """-dE_k/dt of the order-1 residual at each projected state, with the
    closure attached when net is given (a-priori: no time integration)."""
    import torch
    if net is not None:
        lo.closure_attach(net, stats.data_ptr(), bf16_weights=bf16_weights)
    out = []
    try:
        for st in states:
            for t in (0, 1):
                lo.set_solution(t, st[t].data_ptr(), stream)
            torch.cuda.synchronize()
            out.append(-lo.reduce(frlib.FR_RED_KE, stream)[1])
    finally:
        if net is not None:
            lo.closure_attach(None)
    return np.array(out)
