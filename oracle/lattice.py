"""Quasi-periodic image sums (oracle; test infrastructure only).

The exterior operators of eq. (8) use the quasi-periodic kernel
    sum_m alpha^m Phi(x, y + m h),   h = (0, H),  alpha = exp(i beta),
    beta = k H sin(theta)                               (Sec. 2, eqs. 3, 7)
whose plain truncation converges only like O(1/sqrt(q)) (remark after eq. 8).
Sec. 3.3 splits the sum into a direct part |m| <= q and two tails m > q,
m < -q, each written as a Fourier integral (eq. 17) taken on the contour
t = +-sqrt(u^2 - 2iku) (eq. 18).  The printed forms are garbled; this module
uses the forms re-derived from the Sommerfeld integral
    H0(k sqrt(X^2 + Y^2)) = (1/(i pi)) int e^{iXt - mu|Y|} / mu dt,
    mu = sqrt(t^2 - k^2), Re mu >= 0,
which give (reading of eq. 17: prefactor 1/(i pi), geometric series summed)
    T+ = (1/(i pi)) int e^{iXt + mu Y} e^{(q+1)(i beta - mu H)} / (1 - e^{i beta - mu H}) dt / mu
    T- = (1/(i pi)) int e^{iXt - mu Y} e^{-(q+1)(i beta + mu H)} / (1 - e^{-i beta - mu H}) dt / mu
for (X, Y) = x - y.  On the contour, u = s^2 gives mu = s^2 - ik, t = +-s sqrt(s^2 - 2ik)
and dt/mu = 2 ds / sqrt(s^2 - 2ik) (reading of eq. 18: the Jacobian is
restored and the end-point singularity removed).  Derivatives act on the
integrand as d/dX -> i t and d/dY -> +mu (T+) or -mu (T-), and the order-n
Hankel functions follow from the identities after eq. (17):
    H_n(k|x|) e^{i n th} = (-1/k)^n (d1 + i d2)^n H0,
    H_-n(k|x|) e^{-i n th} = k^-n (d1 - i d2)^n H0.
The s-integral is taken by adaptive Gauss-Kronrod quadrature (scipy
quad_vec), an independent rule from the fixed rule of the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad_vec
from scipy.special import hankel1

from .kernels import kernels_sdkt


def choose_q(k: float, H: float, x_max: float, y_max: float, q_min: int = 2) -> int:
    """Direct-sum cut-off.  Besides (q+1)H > |Y|, the contour factor
    |e^{iXt}| <= exp(sqrt(k) |X| s) is kept tame against the Gaussian
    exp(-((q+1)H - |Y|) s^2): its peak exp(k X^2 / (4((q+1)H - |Y|))) is held
    below e^2, so that no cancellation is forced on the quadrature."""
    q = q_min
    while True:
        gap = (q + 1) * H - y_max
        if gap > 0.5 * H and k * x_max ** 2 / (4.0 * gap) <= 2.0:
            return q
        q += 1


def _s_max(k, H, q, x_max, y_max, order_growth=0.0):
    gap = (q + 1) * H - y_max
    # exp(-gap s^2 + k x_max + order_growth*log(1+s^2)) below 1e-22
    s = 1.0
    while -gap * s * s + k * x_max + order_growth * math.log(1.0 + s * s * (1.0 + 2.0 / max(k, 1e-3))) > -52.0:
        s *= 1.25
    return s


def _contour(s, k):
    root = np.sqrt(s * s - 2j * k)
    return s * root, s * s - 1j * k, 2.0 / root       # t_plus, mu, dt/mu per ds


def tails(k, H, beta, X, Y, q, factor_fn, x_max=None, y_max=None, order_growth=0.0,
          epsrel=1e-13):
    """Sum over |m| >= q+1 of alpha^m [P(d/dX, d/dY) H0](k |(X, Y - mH)|).

    factor_fn(it, muY) returns P(it, muY) as an array broadcasting with X;
    muY is +mu for the upper tail and -mu for the lower one."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if x_max is None:
        x_max = float(np.max(np.abs(X))) if X.size else 0.0
    if y_max is None:
        y_max = float(np.max(np.abs(Y))) if Y.size else 0.0
    e_up = np.exp(1j * beta)
    e_dn = np.exp(-1j * beta)

    def integrand(s):
        tp, mu, jac = _contour(s, k)
        out = 0.0
        for t in (tp, -tp):
            ex_up = 1j * X * t + mu * Y + (q + 1) * (1j * beta - mu * H)
            ex_dn = 1j * X * t - mu * Y - (q + 1) * (1j * beta + mu * H)
            den_up = 1.0 - e_up * np.exp(-mu * H)
            den_dn = 1.0 - e_dn * np.exp(-mu * H)
            out = out + np.exp(ex_up) / den_up * factor_fn(1j * t, mu) \
                      + np.exp(ex_dn) / den_dn * factor_fn(1j * t, -mu)
        return out * jac

    smax = _s_max(k, H, q, x_max, y_max, order_growth)
    # break points grade the rule towards s = 0, where a near-Wood pole sits
    pts = [smax * f for f in (1e-3, 1e-2, 0.05, 0.15, 0.3, 0.5)]
    val, _ = quad_vec(integrand, 0.0, smax, epsabs=1e-300, epsrel=epsrel, points=pts,
                      norm="max", limit=20000)
    return val / (1j * math.pi)


def tail_rule(k, H, beta, q, x_max, y_max, n_gl=20, epsrel=1e-14):
    """Fixed quadrature rule in s for the tails, built from the intervals that the
    adaptive rule selects on probe separations spanning |X| <= x_max, |Y| <= y_max,
    with n_gl Gauss-Legendre nodes per interval (the rule of eq. 19 is not
    printed; this is the reading)."""
    px = np.linspace(-x_max, x_max, 7)
    py = np.linspace(-y_max, y_max, 7)
    PX, PY = np.meshgrid(px, py)
    PX, PY = PX.ravel(), PY.ravel()
    e_up = np.exp(1j * beta)
    e_dn = np.exp(-1j * beta)

    def integrand(s):
        tp, mu, jac = _contour(s, k)
        out = 0.0
        for t in (tp, -tp):
            g2 = np.stack([np.ones_like(PX), 1j * t * np.ones_like(PX), mu * np.ones_like(PX),
                           (1j * t) ** 2 + mu * mu + 0 * PX])
            out = out + g2 * (np.exp(1j * PX * t + mu * PY + (q + 1) * (1j * beta - mu * H))
                              / (1.0 - e_up * np.exp(-mu * H))
                              + np.exp(1j * PX * t - mu * PY - (q + 1) * (1j * beta + mu * H))
                              / (1.0 - e_dn * np.exp(-mu * H)))
        return out * jac

    smax = _s_max(k, H, q, x_max, y_max, 2.0)
    pts = [smax * f for f in (1e-3, 1e-2, 0.05, 0.15, 0.3, 0.5)]
    _, _, info = quad_vec(integrand, 0.0, smax, epsabs=1e-300, epsrel=epsrel, points=pts,
                          norm="max", limit=20000, full_output=True)
    iv = np.array(sorted(map(tuple, info.intervals)))
    xi, wi = np.polynomial.legendre.leggauss(n_gl)
    a, b = iv[:, 0:1], iv[:, 1:2]
    s = (0.5 * (a + b) + 0.5 * (b - a) * xi[None, :]).ravel()
    w = (0.5 * (b - a) * wi[None, :]).ravel()
    return s, w


def tails_separable(k, H, beta, q, xt, nut, ys, nys, rule):
    """Tails (|m| >= q+1) of the image sums of H0, -n.grad H0, nu.grad H0 and
    -(nu.grad)(n.grad) H0 for every (target, source) pair.

    The integrand factors exactly into a target part exp(i x1 t +- mu x2) and a
    source part exp(-i y1 t -+ mu y2), so with a fixed rule in s each tail is a
    matrix product over the nodes.  xt, nut: [T, 2]; ys, nys: [S, 2].
    Returns an array [4, T, S] (S, D, K, T order, without the factor i/4)."""
    s, w = rule
    root = np.sqrt(s * s - 2j * k)
    mu = s * s - 1j * k
    jac = 2.0 / root
    out = np.zeros((4, xt.shape[0], ys.shape[0]), dtype=np.complex128)
    for sg in (1.0, -1.0):
        t = sg * s * root
        gx = 1j * t
        for up in (True, False):
            sY = 1.0 if up else -1.0
            gy = sY * mu
            if up:
                den = 1.0 - np.exp(1j * beta - mu * H)
                A = np.exp(1j * xt[:, 0:1] * t + mu * (xt[:, 1:2] - (q + 1) * H) + (q + 1) * 1j * beta)
                B = np.exp(-1j * ys[:, 0:1] * t - mu * ys[:, 1:2])
            else:
                den = 1.0 - np.exp(-1j * beta - mu * H)
                A = np.exp(1j * xt[:, 0:1] * t - mu * (xt[:, 1:2] + (q + 1) * H) - (q + 1) * 1j * beta)
                B = np.exp(-1j * ys[:, 0:1] * t + mu * ys[:, 1:2])
            A = A * (w * jac / den)[None, :]
            fK = nut[:, 0:1] * gx + nut[:, 1:2] * gy            # nu_x . grad_d   [T, Q]
            fN = nys[:, 0:1] * gx + nys[:, 1:2] * gy            # n_y . grad_d    [S, Q]
            Bt = B.T
            out[0] += A @ Bt
            out[1] += A @ (-(fN * B)).T
            out[2] += (A * fK) @ Bt
            out[3] += -((A * fK) @ (fN * B).T)
    return out / (1j * math.pi)


def periodic_offzero_kernels(k, H, theta, xt, nut, ys, nys, q=None, x_max=None, y_max=None):
    """Sum over m != 0 of alpha^m (S, D, K, T)(x, y + m h) for every target x
    (normal nu) and source point y (normal n).

    xt, nut: [T, 2]; ys, nys: [S, 2].  Direct part 1 <= |m| <= q with the
    free-space kernels, plus both tails.  Returns four arrays [T, S]."""
    beta = k * H * math.sin(theta)
    dx = xt[:, None, 0] - ys[None, :, 0]
    dy = xt[:, None, 1] - ys[None, :, 1]
    if x_max is None:
        x_max = float(np.max(np.abs(dx))) if dx.size else 0.0
    if y_max is None:
        y_max = float(np.max(np.abs(dy))) if dy.size else 0.0
    if q is None:
        q = choose_q(k, H, x_max, y_max)
    S = np.zeros(dx.shape, dtype=np.complex128)
    D = np.zeros_like(S)
    K = np.zeros_like(S)
    T = np.zeros_like(S)
    for m in range(-q, q + 1):
        if m == 0:
            continue
        am = np.exp(1j * m * beta)
        s_, d_, k_, t_ = kernels_sdkt(k, dx, dy - m * H, nut[:, None, 0], nut[:, None, 1],
                                      nys[None, :, 0], nys[None, :, 1])
        S += am * s_
        D += am * d_
        K += am * k_
        T += am * t_
    rule = tail_rule(k, H, beta, q, x_max, y_max)
    tl = tails_separable(k, H, beta, q, xt, nut, ys, nys, rule)
    S += 0.25j * tl[0]
    D += 0.25j * tl[1]
    K += 0.25j * tl[2]
    T += 0.25j * tl[3]
    return S, D, K, T


def lattice_sum_orders(k, H, theta, ox, oy, nu_max, exclude=(), q=None):
    """S_nu(o) = sum over m not in `exclude` of alpha^m H_nu(k|o - m h|) e^{i nu arg(o - m h)},
    nu = -nu_max..nu_max (the lattice sum folded into the top-level M2L, eq. 13 and Sec. 3.3).
    Returns an array [2 nu_max + 1] ordered nu = -nu_max..nu_max."""
    beta = k * H * math.sin(theta)
    if q is None:
        q = choose_q(k, H, abs(ox), abs(oy))
    q = max(q, max([abs(m) for m in exclude], default=0))
    nus = np.arange(-nu_max, nu_max + 1)
    out = np.zeros(nus.size, dtype=np.complex128)
    excl = set(int(m) for m in exclude)
    for m in range(-q, q + 1):
        if m in excl:
            continue
        vx, vy = ox, oy - m * H
        r = math.hypot(vx, vy)
        th = math.atan2(vy, vx)
        out += np.exp(1j * m * beta) * hankel1(nus, k * r) * np.exp(1j * nus * th)

    X = np.array([ox], dtype=np.float64)
    Y = np.array([oy], dtype=np.float64)

    def fac(it, muY):
        # (d1 + i d2) -> it + i muY ; (d1 - i d2) -> it - i muY
        plus = (it + 1j * muY) * (-1.0 / k)
        minus = (it - 1j * muY) * (1.0 / k)
        res = []
        for nu in nus:
            res.append((plus ** nu if nu >= 0 else minus ** (-nu)) * np.ones_like(X))
        return np.stack(res)

    tl = tails(k, H, beta, X, Y, q, fac, abs(ox), abs(oy),
               order_growth=float(nu_max))[:, 0]
    return out + tl
