"""Explicit Runge-Kutta steppers.

Test infrastructure (see ``oracle/__init__``).

Paper, Table 1 (time steppers Euler, RK4, RK45) and Section 3.4 (the
RK45[2R+] scheme of Kennedy, Carpenter and Lewis).  Reading R7: fixed step
size, no error controller.

RK45[2R+] is the five-stage, fourth-order "RK4(3)5[2R+]C" scheme of
Kennedy, Carpenter & Lewis (2000), with an embedded third-order solution.
Its Butcher matrix has a[i][j] = b[j] for j < i-1, so only the
sub-diagonal a[i+1][i] and the weights b are free; two registers suffice:

    for each stage i:  k = f(r);  q = q + b_i dt k;  r = q + (a_{i+1,i} - b_i) dt k
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

# Sub-diagonal a[i+1][i], i = 0..3
RK45_A = [Fraction(970286171893, 4311952581923),
          Fraction(6584761158862, 12103376702013),
          Fraction(2251764453980, 15575788980749),
          Fraction(26877169314380, 34165994151039)]
RK45_B = [Fraction(1153189308089, 22510343858157),
          Fraction(1772645290293, 4653164025191),
          Fraction(-1672844663538, 4480602732383),
          Fraction(2114624349019, 3568978502595),
          Fraction(5198255086312, 14908931495163)]
RK45_BHAT = [Fraction(1016888040809, 7410784769900),
             Fraction(11231460423587, 58533540763752),
             Fraction(-1563879915014, 6823010717585),
             Fraction(606302364029, 971179775848),
             Fraction(1097981568119, 3980877426909)]


def rk45_butcher():
    """Full Butcher tableau (A, b, bhat, c) of RK45[2R+] as floats."""
    s = 5
    A = np.zeros((s, s))
    b = np.array([float(x) for x in RK45_B])
    for i in range(1, s):
        for j in range(i):
            A[i, j] = float(RK45_A[i - 1]) if j == i - 1 else b[j]
    c = A.sum(axis=1)
    return A, b, np.array([float(x) for x in RK45_BHAT]), c


RK4_A = np.array([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]])
RK4_B = np.array([1 / 6, 1 / 3, 1 / 3, 1 / 6])


def _axpy(a, x, y):
    return {n: a * x[n] + y[n] for n in x}


def euler_step(f, U, dt):
    R = f(U)
    return {n: U[n] + dt * R[n] for n in U}


def rk4_step(f, U, dt):
    """Classical four-stage RK4, written as stages of its Butcher tableau."""
    k = []
    for i in range(4):
        Y = dict(U)
        for j in range(i):
            if RK4_A[i, j]:
                Y = _axpy(dt * RK4_A[i, j], k[j], Y)
        k.append(f(Y))
    out = dict(U)
    for j in range(4):
        out = _axpy(dt * RK4_B[j], k[j], out)
    return out


def rk45_step(f, U, dt):
    """RK45[2R+] in its two-register form."""
    q = dict(U)
    r = dict(U)
    for i in range(5):
        k = f(r)
        bi = float(RK45_B[i])
        q = _axpy(dt * bi, k, q)
        if i < 4:
            r = _axpy(dt * (float(RK45_A[i]) - bi), k, q)
    return q


def run(stepper, f, U, dt, n):
    for _ in range(n):
        U = stepper(f, U, dt)
    return U


# ---------------------------------------------------------------------------
# Adaptive RK45[2R+] (reading R10: the embedded third-order solution of the
# scheme as error estimate, a PI step-size controller).
#
#   e = dt sum_i (b_i - bhat_i) k_i                    (u_4th - u_3rd)
#   err = sqrt( mean over all values of (e / (atol + rtol max(|u_old|, |u_new|)))^2 )
#   accept if err <= 1;  k = 4 (e = O(dt^4))
#   accepted: fac = SAFETY err^(-0.7/k) err_prev^(0.4/k), err_prev = max(err, 1e-4)
#   rejected: fac = SAFETY err^(-1/k), at most 1
#   dt <- dt * min(FAC_MAX, max(FAC_MIN, fac)); the last step is cut to land on t_end.
# ---------------------------------------------------------------------------
ADAPT_K = 4.0
ADAPT_SAFETY, ADAPT_FAC_MIN, ADAPT_FAC_MAX, ADAPT_ERR_FLOOR = 0.9, 0.2, 5.0, 1e-4


def rk45_step_with_error(f, U, dt):
    """One RK45[2R+] step in two-register form, plus the embedded error
    e = u_4th - u_3rd accumulated stage by stage."""
    q = dict(U)
    r = dict(U)
    e = {n: np.zeros_like(U[n]) for n in U}
    for i in range(5):
        k = f(r)
        bi = float(RK45_B[i])
        q = _axpy(dt * bi, k, q)
        e = _axpy(dt * (bi - float(RK45_BHAT[i])), k, e)
        if i < 4:
            r = _axpy(dt * (float(RK45_A[i]) - bi), k, q)
    return q, e


def error_norm(e, u_old, u_new, atol, rtol):
    num = 0.0
    cnt = 0
    for n in e:
        sc = atol + rtol * np.maximum(np.abs(u_old[n]), np.abs(u_new[n]))
        num += float(((e[n] / sc) ** 2).sum())
        cnt += e[n].size
    return np.sqrt(num / cnt)


def controller(err, err_prev, accepted):
    """Step-size factor of the PI controller (reading R10)."""
    if accepted:
        fac = ADAPT_FAC_MAX if err == 0.0 else \
            ADAPT_SAFETY * err ** (-0.7 / ADAPT_K) * err_prev ** (0.4 / ADAPT_K)
        return min(ADAPT_FAC_MAX, max(ADAPT_FAC_MIN, fac))
    return min(1.0, max(ADAPT_FAC_MIN, ADAPT_SAFETY * err ** (-1.0 / ADAPT_K)))


def rk45_adaptive(f, U, t, t_end, dt, atol, rtol, err_prev=1.0, max_attempts=100000):
    """Advance from t to t_end; returns (U, t, dt, err_prev, n_accepted,
    n_rejected, errors) with errors the error norm of every attempt."""
    n_acc = n_rej = 0
    errors = []
    while t < t_end and n_acc + n_rej < max_attempts:
        last = t + dt >= t_end
        h = t_end - t if last else dt
        V, e = rk45_step_with_error(f, U, h)
        err = error_norm(e, U, V, atol, rtol)
        errors.append(err)
        if err <= 1.0:
            fac = controller(err, err_prev, True)
            U, t = V, (t_end if last else t + h)
            err_prev = max(err, ADAPT_ERR_FLOOR)
            dt = h * fac
            n_acc += 1
        else:
            dt = h * controller(err, err_prev, False)
            n_rej += 1
    return U, t, dt, err_prev, n_acc, n_rej, errors
