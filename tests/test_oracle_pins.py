"""Pins for the CPU oracle, taken from mathematics rather than from the oracle
itself (Section 2: the fractional ABM predictor-corrector and its weights).

Each test would fail under a plausible slip in the oracle:
  * weights vs quadrature of the product-integration rules   (sign of b, Gamma factors, indices)
  * telescoping sums of the weights                           (every weight at once)
  * exactness for forcing linear in t                         (corrector indexing, c_n f_0 term)
  * Mittag-Leffler convergence order                          (whole scheme)
  * alpha = 1 two-term recurrence                             (predictor/corrector coupling)
  * 50-digit brute force on tiny N, weights by quadrature     (every step, every rhs)
  * equilibrium invariance                                     (rhs formulas, spurious history terms)
  * per-component orders: uncoupled components equal scalar runs, closed
    forms per component, brute force with one order per component
                                                               (order / weight table of the wrong component)
  * orders in (1, 2]: the start term x0 + t x1 of eq. abm by closed forms,
    Mittag-Leffler / harmonic-oscillator convergence, alpha = 2 weights exact
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


# ---------------------------------------------------------------- weights
def _quad_weights(alpha, n, dps=30):
    """Product-integration weights of step n+1 by numerical quadrature.

    Predictor (product rectangle rule): weight of f_j is
        (1/Gamma(alpha)) * int_j^{j+1} (n+1-u)^(alpha-1) du       -> b_{n-j}
    Corrector (product trapezoid rule): weight of f_j is
        (1/Gamma(alpha)) * int_0^{n+1} (n+1-u)^(alpha-1) phi_j(u) du
    with phi_j the piecewise-linear hat at node j:  j=0 -> c_n,
    1<=j<=n -> a_{n-j}, j=n+1 -> 1/Gamma(alpha+2).
    The integrals are taken in v = n+1-u, the distance to the singular end
    point, and then in w = v^alpha, which turns v^(alpha-1) dv into dw/alpha
    and leaves a smooth integrand for the quadrature.
    """
    with mp.workdps(dps):
        al = mp.mpf(alpha)
        ga = mp.gamma(al)
        pred = [_kq(al, lambda v: 1, n - j, n + 1 - j) / ga for j in range(n + 1)]
        corr = []
        for j in range(n + 2):
            vj = n + 1 - j     # node j sits at v = n+1-j
            tot = mp.mpf(0)
            if j >= 1:      # u in [j-1, j]  <->  v in [vj, vj+1]
                tot += _kq(al, lambda v: vj + 1 - v, vj, vj + 1)
            if j <= n:      # u in [j, j+1]  <->  v in [vj-1, vj]
                tot += _kq(al, lambda v: v - (vj - 1), vj - 1, vj)
            corr.append(tot / ga)
        return [float(x) for x in pred], [float(x) for x in corr]


def _kq(al, g, v0, v1):
    """int_{v0}^{v1} v^(al-1) g(v) dv by quadrature in w = v^al."""
    inv = 1 / al
    return mp.quad(lambda w: g(w ** inv), [mp.mpf(v0) ** al, mp.mpf(v1) ** al]) / al


@pytest.mark.parametrize("alpha", [0.3, 0.8, 0.95, 1.0, 1.4, 2.0])
def test_weights_match_quadrature(alpha):
    nmax = 4
    b, a, c = O.weights(alpha, nmax + 1)
    for n in range(nmax + 1):
        pred, corr = _quad_weights(alpha, n)
        for j in range(n + 1):
            assert b[n - j] == pytest.approx(pred[j], rel=2e-15, abs=0)
        assert c[n] == pytest.approx(corr[0], rel=2e-15, abs=0)
        for j in range(1, n + 1):
            assert a[n - j] == pytest.approx(corr[j], rel=2e-15, abs=0)
        assert corr[n + 1] == pytest.approx(1.0 / math.gamma(alpha + 2.0), rel=2e-15)


def test_printed_plus_sign_of_b_is_not_the_rule():
    # The predictor weight is printed with a "+" between the powers; the
    # product-rectangle rule gives the difference.  At alpha=0.8, n=1 the
    # quadrature value is 0.79570; the "+" form would give 2.943.
    pred, _ = _quad_weights(0.8, 1)
    plus = (2 ** 0.8 + 1 ** 0.8) / math.gamma(1.8)
    minus = (2 ** 0.8 - 1 ** 0.8) / math.gamma(1.8)
    assert pred[0] == pytest.approx(minus, rel=1e-14)
    assert abs(pred[0] - plus) > 1.0
    b, _, _ = O.weights(0.8, 2)
    assert b[1] == pytest.approx(pred[0], rel=1e-15)


@pytest.mark.parametrize("alpha,k0", [(0.8, 65536), (0.9, 262144), (0.95, 3_000_000),
                                      (0.5, 1_000_000), (1.5, 1_000_000), (1.9, 65536)])
def test_weights_large_index_50_digits(alpha, k0):
    """Cancellation in the differences of powers grows like k^2; the oracle's
    quad evaluation must still be within a few ulp of a 50-digit value."""
    n = 4
    b, a, c = O.weights(alpha, n, k0=k0)
    with mp.workdps(50):
        al = mp.mpf(alpha)
        g1, g2 = mp.gamma(al + 1), mp.gamma(al + 2)
        for i in range(n):
            k = mp.mpf(k0 + i)
            bb = ((k + 1) ** al - k ** al) / g1
            aa = ((k + 2) ** (al + 1) - 2 * (k + 1) ** (al + 1) + k ** (al + 1)) / g2
            cc = (k ** (al + 1) - (k - al) * (k + 1) ** al) / g2
            # Gamma is taken in double on the oracle side: allow its 1-2 ulp.
            assert b[i] == pytest.approx(float(bb), rel=8e-16)
            assert a[i] == pytest.approx(float(aa), rel=8e-16)
            assert c[i] == pytest.approx(float(cc), rel=8e-16)


@pytest.mark.parametrize("alpha", [0.2, 0.55, 0.8, 0.9, 0.99, 1.0, 1.3, 1.75, 2.0])
def test_weight_sums_telescope(alpha):
    """Both quadrature rules integrate f == 1 exactly:
       sum_{k=0..n} b_k                        = (n+1)^alpha / Gamma(alpha+1)
       c_n + sum_{k=0..n-1} a_k + 1/Gamma(alpha+2) = (n+1)^alpha / Gamma(alpha+1)"""
    nmax = 5000
    b, a, c = O.weights(alpha, nmax + 1)
    g1 = math.gamma(alpha + 1.0)
    g2 = math.gamma(alpha + 2.0)
    for n in [0, 1, 2, 7, 100, 1234, nmax]:
        exact = (n + 1) ** alpha / g1
        sb = math.fsum(b[: n + 1])
        sc = math.fsum(list(a[:n]) + [c[n], 1.0 / g2])
        assert sb == pytest.approx(exact, rel=4e-15)
        assert sc == pytest.approx(exact, rel=4e-15)


def test_alpha_one_weights_exact():
    b, a, c = O.weights(1.0, 1000)
    assert np.all(b == 1.0)
    assert np.all(a == 1.0)
    assert np.all(c[1:] == 0.5)
    assert c[0] == 0.5  # c_0 = alpha / Gamma(alpha+2) = 1/2


def test_alpha_two_weights_exact():
    """At alpha = 2 the differences of powers are polynomials in k:
    b_k = (2k+1)/2, a_k = (6k+6)/6 = k+1, c_k = (3k+2)/6 (c_0 = 2/6)."""
    n = 4000
    b, a, c = O.weights(2.0, n)
    k = np.arange(n, dtype=np.float64)
    assert np.array_equal(b, (2 * k + 1) / 2)
    assert np.array_equal(a, k + 1)
    assert np.max(np.abs(c - (3 * k + 2) / 6) / ((3 * k + 2) / 6)) <= 2.3e-16


# ---------------------------------------------------------------- whole scheme
@pytest.mark.parametrize("alpha", [0.35, 0.8, 1.0])
def test_linear_in_t_forcing_is_integrated_exactly(alpha):
    """f = c0 + c1 t does not depend on y, so the corrector (product
    trapezoid rule, exact for piecewise-linear integrands) reproduces
    y(t) = y0 + c0 t^a/Gamma(a+1) + c1 t^(a+1)/Gamma(a+2) at every node."""
    c0, c1, y0, h, N = 0.7, -0.3, 0.25, 1.0 / 64, 300
    y = O.solve(O.RHS_POLY, alpha, h, N, [y0], [c0, c1], out_stride=1)[:, 0]
    t = np.arange(N + 1) * h
    exact = y0 + c0 * t ** alpha / math.gamma(alpha + 1) + c1 * t ** (alpha + 1) / math.gamma(alpha + 2)
    assert np.max(np.abs(y - exact)) <= 2e-14 * np.max(np.abs(exact))


def _mittag_leffler(alpha, z, dps=60):
    with mp.workdps(dps):
        z = mp.mpf(z)
        return float(mp.nsum(lambda k: z ** k / mp.gamma(alpha * k + 1), [0, mp.inf]))


@pytest.mark.parametrize("alpha", [0.5, 0.8])
def test_mittag_leffler_convergence_order(alpha):
    """D^a y = -y, y(0)=1 has y = E_a(-t^a).  The ABM error at fixed T decays
    like h^(1+a) for a < 1 (the observed order of the product-trapezoid
    corrector on this smooth-in-t^a solution)."""
    T = 8.0
    exact = _mittag_leffler(alpha, -T ** alpha)
    errs = []
    hs = [2.0 ** -k for k in (5, 6, 7, 8, 9)]
    for h in hs:
        N = int(round(T / h))
        y = O.solve(O.RHS_LINEAR, alpha, h, N, [1.0], [1.0], out_stride=0)[0, 0]
        errs.append(abs(y - exact))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - (1 + alpha)) < 0.08, orders


def test_mittag_leffler_at_the_linear_workload():
    """alpha=0.8, h=2^-10, N=8192: the ABM value sits within 2e-8 of
    E_0.8(-8^0.8) (error of order h^1.8)."""
    exact = _mittag_leffler(0.8, -8.0 ** 0.8)
    y = O.solve(O.RHS_LINEAR, 0.8, 2.0 ** -10, 8192, [1.0], [1.0], out_stride=0)[0, 0]
    assert 1e-9 < abs(y - exact) < 2e-8


def _volterra_alpha1(rhs_fn, x0, h, N):
    """At alpha = 1 the scheme collapses to a two-term recurrence:
       yP_{n+1} = yP_n + h f_n                      (yP_0 = x0)
       y_{n+1}  = y_n + h (f_n + (fP_{n+1} - fP_n)/2)  with fP_0 = f_0."""
    x0 = np.asarray(x0, float)
    y = [x0.copy()]
    f = [rhs_fn(0.0, x0)]
    yP = x0.copy()
    fP_prev = f[0]
    for n in range(N):
        t1 = (n + 1) * h
        yP = yP + h * f[n]
        fP = rhs_fn(t1, yP)
        ynew = y[n] + h * (f[n] + (fP - fP_prev) / 2.0)
        y.append(ynew)
        f.append(rhs_fn(t1, ynew))
        fP_prev = fP
    return np.array(y)


def _duffing(p):
    d_, A, w = p
    return lambda t, y: np.array([y[1], -d_ * y[1] - y[0] - y[0] ** 3 + A * math.cos(w * t)])


def test_alpha_one_is_the_volterra_recurrence():
    p = (0.1, 0.3, 1.2)
    h, N = 1.0 / 128, 1024
    y = O.solve(O.RHS_DUFFING, 1.0, h, N, [0.1, 0.0], p, out_stride=1)
    ref = _volterra_alpha1(_duffing(p), [0.1, 0.0], h, N)
    assert np.max(np.abs(y - ref)) <= 3e-14 * np.max(np.abs(ref))


def test_alpha_one_vs_classical_trapezoid_pece():
    """Classical trapezoidal PECE (y_{n+1} = y_n + h/2 (f_n + f(t_{n+1}, y_n + h f_n)))
    coincides with the alpha=1 scheme only when f ignores y; otherwise the two
    differ by O(h^2)."""
    # f independent of y: identical up to rounding
    h, N = 1.0 / 64, 256
    y = O.solve(O.RHS_POLY, 1.0, h, N, [0.5], [0.7, -0.3], out_stride=1)[:, 0]
    t = np.arange(N + 1) * h
    z = 0.5 + 0.7 * t - 0.15 * t * t
    assert np.max(np.abs(y - z)) < 1e-13
    # y-dependent f: the gap shrinks about 4x per halving of h
    p = (0.1, 0.3, 1.2)
    fn = _duffing(p)
    gaps = []
    for h in (2.0 ** -5, 2.0 ** -6, 2.0 ** -7):
        N = int(4 / h)
        ya = O.solve(O.RHS_DUFFING, 1.0, h, N, [0.1, 0.0], p, out_stride=0)[0]
        yc = np.array([0.1, 0.0])
        for n in range(N):
            f0 = fn(n * h, yc)
            yc = yc + h / 2 * (f0 + fn((n + 1) * h, yc + h * f0))
        gaps.append(np.max(np.abs(ya - yc)))
    assert gaps[0] > 1e-6
    r1, r2 = gaps[0] / gaps[1], gaps[1] / gaps[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, gaps


# ---------------------------------------------------------------- brute force
def _rhs_mp(name, p):
    if name == "LINEAR":
        return lambda t, y: [-p[0] * y[0]]
    if name == "DUFFING":
        return lambda t, y: [y[1], -p[0] * y[1] - y[0] - y[0] ** 3 + p[1] * mp.cos(p[2] * t)]
    if name == "LORENZ":
        return lambda t, y: [p[0] * (y[1] - y[0]), y[0] * (p[1] - y[2]) - y[1],
                             y[0] * y[1] - p[2] * y[2]]
    if name == "LCR":
        def g(x):
            if x <= -1:
                return p[3] * x - p[2] + p[3]
            if x >= 1:
                return p[3] * x + p[2] - p[3]
            return p[2] * x
        return lambda t, y: [y[1] - g(y[0]), -p[0] * y[1] - y[0] + p[4] * mp.sin(p[1] * t)]
    if name == "DIAG":
        return lambda t, y: [-p[0] * y[0] + p[2], -p[1] * y[1] + p[3]]
    raise KeyError(name)


def _quad_rules(al, n):
    """Product-rectangle and product-trapezoid weights of step n+1 for order
    al by quadrature (v = t_{n+1}/h - u, kernel v^(al-1), node j at v = n+1-j)."""
    ga = mp.gamma(al)
    pw = [_kq(al, lambda v: 1, n - j, n + 1 - j) / ga for j in range(n + 1)]
    cw = []
    for j in range(n + 2):
        vj = n + 1 - j
        tot = mp.mpf(0)
        if j >= 1:
            tot += _kq(al, lambda v: vj + 1 - v, vj, vj + 1)
        if j <= n:
            tot += _kq(al, lambda v: v - (vj - 1), vj - 1, vj)
        cw.append(tot / ga)
    return pw, cw


def _brute_force(name, alpha, h, N, x0, p, x1=None):
    """_brute_force_mp rounded to double."""
    return np.array([[float(v) for v in y] for y in _brute_force_mp(name, alpha, h, N, x0, p, x1)])


def _brute_force_mp(name, alpha, h, N, x0, p, x1=None):
    """50-digit ABM for tiny N with weights from quadrature of the
    product-integration rules (no closed-form weight is used).  alpha is one
    order or one per component; components of order above 1 start from
    x0 + t x1 (the Taylor sum over the ceil(alpha) initial values).  Returns
    the states as lists of 50-digit values."""
    d = len(x0)
    alphas = list(alpha) if np.ndim(alpha) else [alpha] * d
    with mp.workdps(50):
        als = [mp.mpf(a) for a in alphas]
        hh = mp.mpf(h)
        fn = _rhs_mp(name, [mp.mpf(v) for v in p])
        x0m = [mp.mpf(v) for v in x0]
        x1m = [mp.mpf(v) for v in (x1 if x1 is not None else [0.0] * d)]
        ha = [hh ** al for al in als]
        F = [fn(mp.mpf(0), x0m)]
        ys = [x0m]
        for n in range(N):
            rules = {}
            for al in set(als):
                rules[al] = _quad_rules(al, n)
            t1 = (n + 1) * hh
            T = [x0m[i] + (t1 * x1m[i] if alphas[i] > 1 else 0) for i in range(d)]
            yP = [T[i] + ha[i] * mp.fsum(rules[als[i]][0][j] * F[j][i] for j in range(n + 1))
                  for i in range(d)]
            fP = fn(t1, yP)
            y1 = []
            for i in range(d):
                cw = rules[als[i]][1]
                y1.append(T[i] + ha[i] * (mp.fsum(cw[j] * F[j][i] for j in range(n + 1))
                                          + cw[n + 1] * fP[i]))
            ys.append(y1)
            F.append(fn(t1, y1))
        return ys


@pytest.mark.parametrize("name,alpha,h,x0,p", [
    ("LINEAR", 0.7, 0.125, [1.0], [1.3]),
    ("DUFFING", 0.9, 0.05, [0.1, 0.0], [0.1, 0.3, 1.2]),
    ("LORENZ", 0.95, 0.01, [1.0, 1.0, 1.0], [10.0, 28.0, 8.0 / 3.0]),
    ("LCR", 0.9, 0.25, [1.2, -0.4], [1.015, 0.55, -1.02, -0.58, 0.117]),
])
def test_tiny_n_brute_force(name, alpha, h, x0, p):
    N = 10
    rid = {"LINEAR": O.RHS_LINEAR, "DUFFING": O.RHS_DUFFING, "LORENZ": O.RHS_LORENZ,
           "LCR": O.RHS_LCR}[name]
    y = O.solve(rid, alpha, h, N, x0, p, out_stride=1)
    ref = _brute_force(name, alpha, h, N, x0, p)
    assert np.max(np.abs(y - ref)) <= 2e-15 * max(1.0, np.max(np.abs(ref)))


_RID = {"LINEAR": O.RHS_LINEAR, "DUFFING": O.RHS_DUFFING, "LORENZ": O.RHS_LORENZ,
        "LCR": O.RHS_LCR, "DIAG": O.RHS_DIAG}


@pytest.mark.parametrize("name,alpha,h,x0,x1,p", [
    # incommensurate orders (eq. sys.LRC with alpha_1 != alpha_2)
    ("LCR", (0.9, 0.8), 0.25, [1.2, -0.4], None, [1.015, 0.55, -1.02, -0.58, 0.117]),
    ("LORENZ", (0.95, 0.9, 0.85), 0.01, [1.0, 1.0, 1.0], None, [10.0, 28.0, 8.0 / 3.0]),
    ("DIAG", (0.6, 0.95), 0.1, [1.0, -0.5], None, [1.3, 0.7, 0.2, -0.1]),
    # orders above 1: start term x0 + t x1
    ("LINEAR", 1.5, 0.125, [1.0], [0.5], [1.3]),
    ("DUFFING", (1.3, 0.9), 0.05, [0.1, 0.0], [0.4, 0.0], [0.1, 0.3, 1.2]),
    ("DIAG", (2.0, 1.7), 0.1, [1.0, 0.0], [0.0, 1.0], [1.0, 2.0, 0.0, 0.3]),
])
def test_tiny_n_brute_force_general_orders(name, alpha, h, x0, x1, p):
    N = 8
    y = O.solve(_RID[name], alpha, h, N, x0, p, out_stride=1, x1=x1)
    ref = _brute_force(name, alpha, h, N, x0, p, x1=x1)
    assert np.max(np.abs(y - ref)) <= 4e-15 * max(1.0, np.max(np.abs(ref)))


# ---------------------------------------------------------------- general orders
def test_uncoupled_components_equal_scalar_runs():
    """DIAG with m = 0 is two scalar problems D^(a_i) y_i = -l_i y_i; with
    different orders each component must be, bit for bit, the scalar LINEAR
    run of its own order (a component reading the other's weights, h^a or
    Gamma factor fails this)."""
    h, N = 2.0 ** -6, 700
    al, lam, x0 = (0.55, 0.9), (1.3, 0.4), (1.0, -2.0)
    y = O.solve(O.RHS_DIAG, al, h, N, x0, [lam[0], lam[1], 0.0, 0.0], out_stride=1)
    for i in range(2):
        yi = O.solve(O.RHS_LINEAR, al[i], h, N, [x0[i]], [lam[i]], out_stride=1)[:, 0]
        assert np.array_equal(y[:, i], yi), i


@pytest.mark.parametrize("alphas", [(0.6, 1.7), (1.0, 0.35), (2.0, 1.25)])
def test_constant_forcing_closed_form_per_component(alphas):
    """f = m (no dependence on y): both product rules integrate a constant
    exactly, so component i is y_i(t) = x0_i + [a_i > 1] x1_i t
    + m_i t^(a_i) / Gamma(a_i + 1) at every node, each with its own order."""
    h, N = 1.0 / 64, 400
    x0, x1, m = (0.25, -1.0), (0.5, 2.0), (0.7, -0.3)
    y = O.solve(O.RHS_DIAG, alphas, h, N, x0, [0.0, 0.0, m[0], m[1]], out_stride=1, x1=x1)
    t = np.arange(N + 1) * h
    for i in range(2):
        exact = x0[i] + m[i] * t ** alphas[i] / math.gamma(alphas[i] + 1)
        if alphas[i] > 1:
            exact = exact + x1[i] * t
        assert np.max(np.abs(y[:, i] - exact)) <= 2e-14 * np.max(np.abs(exact)), i


@pytest.mark.parametrize("alpha", [1.25, 1.6, 2.0])
def test_linear_in_t_forcing_exact_above_one(alpha):
    """D^a y = c0 + c1 t, y(0) = y0, y'(0) = y1 (1 < a <= 2):
    y = y0 + y1 t + c0 t^a/Gamma(a+1) + c1 t^(a+1)/Gamma(a+2), reproduced at
    every node (the start term of eq. abm plus exact product integration)."""
    c0, c1, y0, y1, h, N = 0.7, -0.3, 0.25, -0.8, 1.0 / 64, 300
    y = O.solve(O.RHS_POLY, alpha, h, N, [y0], [c0, c1], out_stride=1, x1=[y1])[:, 0]
    t = np.arange(N + 1) * h
    exact = (y0 + y1 * t + c0 * t ** alpha / math.gamma(alpha + 1)
             + c1 * t ** (alpha + 1) / math.gamma(alpha + 2))
    assert np.max(np.abs(y - exact)) <= 2e-14 * np.max(np.abs(exact))


def test_mittag_leffler_above_one_converges_at_order_two():
    """D^1.5 y = -y, y(0) = 1, y'(0) = 0 has y = E_1.5(-t^1.5); the scheme's
    error at fixed T falls like h^2 (order min(2, 1 + a))."""
    alpha, T = 1.5, 4.0
    exact = _mittag_leffler(alpha, -T ** alpha)
    errs = []
    for k in (5, 6, 7, 8):
        h = 2.0 ** -k
        y = O.solve(O.RHS_LINEAR, alpha, h, int(round(T / h)), [1.0], [1.0], out_stride=0,
                    x1=[0.0])[0, 0]
        errs.append(abs(y - exact))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - 2.0) < 0.1, orders


def test_alpha_two_is_the_harmonic_oscillator():
    """At a = 2, D^2 y = -w^2 y with y(0) = 0, y'(0) = 1 is sin(w t)/w; the
    error at T = 5 falls like h^2."""
    w, T = 1.7, 5.0
    errs = []
    for k in (5, 6, 7, 8):
        h = 2.0 ** -k
        N = int(round(T / h))
        y = O.solve(O.RHS_LINEAR, 2.0, h, N, [0.0], [w * w], out_stride=1, x1=[1.0])[:, 0]
        t = np.arange(N + 1) * h
        errs.append(np.max(np.abs(y - np.sin(w * t) / w)))
    assert errs[0] < 5e-3
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(abs(o - 2.0) < 0.1 for o in orders), orders


# ---------------------------------------------------------------- invariants
def _lcr_equilibria(sigma, a, b):
    """Equilibria of the unforced LCR system (f = 0), as given in the
    "Numerical experiment" section: E0 = (0,0) and
    E+- = (+-sigma(a-b)/(1+sigma b), +-(b-a)/(1+sigma b))."""
    den = 1 + sigma * b
    return [(0.0, 0.0), (sigma * (a - b) / den, (b - a) / den),
            (-sigma * (a - b) / den, -(b - a) / den)]


@pytest.mark.parametrize("case", ["lorenz0", "lorenz+", "lorenz-", "duffing0", "lcr0", "lcr+",
                                  "lcr-", "lcr+ incommensurate", "lcr- incommensurate"])
def test_equilibrium_is_invariant(case):
    alpha, h, N = 0.9, 1.0 / 256, 512
    if case.endswith("incommensurate"):
        alpha = (0.9, 0.75)
    if case.startswith("lorenz"):
        s, r, bb = 10.0, 28.0, 8.0 / 3.0
        q = math.sqrt(bb * (r - 1))
        x0 = {"lorenz0": (0, 0, 0), "lorenz+": (q, q, r - 1), "lorenz-": (-q, -q, r - 1)}[case]
        y = O.solve(O.RHS_LORENZ, alpha, h, N, x0, (s, r, bb), out_stride=1)
    elif case == "duffing0":
        x0 = (0.0, 0.0)
        y = O.solve(O.RHS_DUFFING, alpha, h, N, x0, (0.1, 0.0, 1.2), out_stride=1)
    else:
        E = _lcr_equilibria(1.015, -1.02, -0.58)
        x0 = E[{"lcr0": 0, "lcr+": 1, "lcr-": 2}[case.split()[0]]]
        y = O.solve(O.RHS_LCR, alpha, h, N, x0, (1.015, 0.55, -1.02, -0.58, 0.0), out_stride=1)
    dev = np.max(np.abs(y - np.asarray(x0)[None, :]))
    assert dev <= 1e-12 * max(1.0, np.max(np.abs(x0))), dev


def test_steps_from_states_reproduce_a_run():
    pr = dict(rhs=O.RHS_DUFFING, alpha=0.9, h=1e-2, x0=[0.1, 0.0], p=[0.1, 0.3, 1.2])
    N = 700
    y = O.solve(pr["rhs"], pr["alpha"], pr["h"], N, pr["x0"], pr["p"], out_stride=1)
    s_list = [1, 2, 63, 64, 65, 699, 700]
    ys = O.steps_from_states(pr["rhs"], pr["alpha"], pr["h"], pr["x0"], pr["p"], y, s_list)
    assert np.array_equal(ys, y[s_list])
    # the compensated recompute reproduces the compensated run
    yc = O.solve(pr["rhs"], pr["alpha"], pr["h"], N, pr["x0"], pr["p"], out_stride=1,
                 compensated=True)
    ys = O.steps_from_states(pr["rhs"], pr["alpha"], pr["h"], pr["x0"], pr["p"], yc, s_list,
                             compensated=True)
    assert np.array_equal(ys, yc[s_list])


def test_rounding_noise_floor_is_far_below_parity_tolerance():
    """Whether 1e-12 agreement is well posed: perturbing x0 by 1e-14 or
    switching to compensated summation moves the trajectory by far less."""
    base = dict(alpha=0.95, h=2.0 ** -8, N=4096, p=[0.1, 0.45, 1.2])
    y0 = O.solve(O.RHS_DUFFING, base["alpha"], base["h"], base["N"], [0.1, 0.0], base["p"])
    y1 = O.solve(O.RHS_DUFFING, base["alpha"], base["h"], base["N"], [0.1 + 1e-14, 0.0], base["p"])
    y2 = O.solve(O.RHS_DUFFING, base["alpha"], base["h"], base["N"], [0.1, 0.0], base["p"],
                 compensated=True)
    scale = np.max(np.abs(y0))
    assert np.max(np.abs(y1 - y0)) / scale < 1e-13
    assert np.max(np.abs(y2 - y0)) / scale < 1e-13


def test_batch_equals_single(orc):
    probs = [(O.RHS_DUFFING, 0.95, 2 ** -6, 300, [0.1, 0.0], [0.1, A, 1.2]) for A in (0.1, 0.35, 0.6)]
    probs.append((O.RHS_LORENZ, 0.93, 2 ** -8, 257, [1.0, 1.0, 1.0], [10.0, 28.0, 8 / 3]))
    outs = O.solve_batch([q[0] for q in probs], [q[1] for q in probs], [q[2] for q in probs],
                         [q[3] for q in probs], [q[4] for q in probs], [q[5] for q in probs],
                         out_stride=7)
    for q, o in zip(probs, outs):
        assert np.array_equal(o, O.solve(*q, out_stride=7))


def test_invalid_arguments_rejected():
    with pytest.raises(ValueError):
        O.solve(O.RHS_LINEAR, 2.5, 0.1, 10, [1.0], [1.0])
    with pytest.raises(ValueError):
        O.solve(O.RHS_DIAG, (0.5, 0.0), 0.1, 10, [1.0, 1.0], [1.0])
    with pytest.raises(ValueError):
        O.solve(O.RHS_DIAG, (0.5, 0.6, 0.7), 0.1, 10, [1.0, 1.0], [1.0])
    with pytest.raises(ValueError):
        O.solve(O.RHS_LINEAR, 0.5, -0.1, 10, [1.0], [1.0])
    with pytest.raises(ValueError):
        O.solve(O.RHS_LINEAR, 0.5, 0.1, 0, [1.0], [1.0])


def _ill_conditioned_sum(seed, n):
    """Weights that are powers of two (so every product w[n-k] F[k] is exact
    in double) and a history of large terms that cancel, plus a small
    remainder: the exact sum is tiny beside the terms."""
    rng = np.random.default_rng(seed)
    w = np.ldexp(1.0, rng.integers(-3, 4, n + 1)).astype(np.float64)
    # products in groups of four: two full-precision terms of order one,
    # then +B_j and -B_j (B_j ~ 2^40, an integer).  Adding B_j to a running
    # sum that carries fine bits drops them to B_j's grid (2^-12), and the
    # term added is then the larger one, the case that separates Neumaier's
    # compensation from Kahan's
    big = np.ldexp(rng.integers(1 << 19, 1 << 20, n // 4 + 1).astype(np.float64), 20)
    k = np.arange(n + 1)
    prod = rng.uniform(-1.0, 1.0, n + 1)
    prod[k % 4 == 2] = big[k[k % 4 == 2] // 4]
    prod[k % 4 == 3] = -big[k[k % 4 == 3] // 4]
    F = prod / w[n - k]                     # exact: w is a power of two
    terms = [float(w[n - j]) * float(F[j]) for j in range(n + 1)]
    return w, F, terms


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_compensated_history_sum_matches_exactly_rounded_sum(seed):
    """The compensated history sum (Neumaier's variant of Kahan summation) on a
    sum whose terms reach ~2^40 and cancel to ~10: the plain ascending sum
    loses at least six digits, the compensated one stays within a few ulp of
    the exactly rounded sum (math.fsum, Shewchuk's algorithm).  A wrong sign
    in the compensation, Kahan's single branch in place of Neumaier's two, or
    a compensation that is never added back fails the second assertion."""
    n = 399                                  # 100 groups of four terms
    w, F, terms = _ill_conditioned_sum(seed, n)
    exact = math.fsum(terms)
    # the condition number sum|t| / |sum t|
    assert sum(abs(t) for t in terms) / abs(exact) > 1e9
    plain = O.history_sum(w, F, 0, n, compensated=False)
    comp = O.history_sum(w, F, 0, n, compensated=True)
    assert abs(plain - exact) / abs(exact) > 1e-10
    assert abs(comp - exact) <= 4 * np.spacing(abs(exact)), (comp, exact)


def test_history_sum_index_order_and_lower_limit():
    """sum_{k=k_lo..n} w[n-k] F[k]: the weight index runs against the history
    index, and k_lo = 1 drops F[0] (the corrector's sum, whose k = 0 term
    enters through c_n).  Both variants, checked against a 50-digit sum."""
    rng = np.random.default_rng(7)
    n = 37
    w = rng.uniform(0.1, 1.0, n + 1)
    F = rng.uniform(-1.0, 1.0, n + 1)
    for k_lo in (0, 1):
        with mp.workdps(50):
            ref = mp.fsum(mp.mpf(float(w[n - k])) * mp.mpf(float(F[k])) for k in range(k_lo, n + 1))
        for comp in (False, True):
            got = O.history_sum(w, F, k_lo, n, compensated=comp)
            assert abs(got - float(ref)) <= 1e-14 * float(mp.fsum(abs(x) for x in F)), (k_lo, comp)


@pytest.mark.parametrize("alpha", [0.45, 0.9, 1.0])
def test_step_recompute_term_size_closed_form(alpha):
    """With f = c0 > 0 every history term is positive, so the size of the
    terms equals the sums themselves: h^a sum b_{n-k} c0 = c0 t^a / Gamma(a+1)
    (the product-rectangle rule is exact for constants) and
    h^a (c_n c0 + sum a_{n-k} c0) = c0 t^a / Gamma(a+1) - h^a c0 / Gamma(a+2)
    (the product-trapezoid rule too, less the weight of f at t_s itself).
    A missing |c_n F_0| term, a missing sum or a wrong h^a fails this."""
    c0, h, N = 0.7, 2.0 ** -6, 500
    y = O.solve(O.RHS_POLY, alpha, h, N, [0.3], [c0, 0.0], out_stride=1)
    s_list = [1, 2, 17, 256, 499, 500]
    ys, scale = O.steps_from_states(O.RHS_POLY, alpha, h, [0.3], [c0, 0.0], y[:-1], s_list,
                                    return_scale=True)
    assert np.array_equal(ys, y[s_list])
    for j, s in enumerate(s_list):
        t = s * h
        ref = 2 * c0 * t ** alpha / math.gamma(alpha + 1) - h ** alpha * c0 / math.gamma(alpha + 2)
        assert abs(scale[j, 0] - ref) <= 1e-13 * ref, (s, scale[j, 0], ref)



# ------------------------------------------------- the scheme in quad precision
# oracle_solve_quad runs every quantity in __float128 (the oracle of the
# double-double mode); its pins are the double oracle's, at quad tolerances.
def _pairs_mp(y):
    """(hi, lo) pairs as 50-digit values."""
    with mp.workdps(50):
        return [[mp.mpf(float(c[0])) + mp.mpf(float(c[1])) for c in st] for st in y]


def _max_rel_mp(a, b):
    with mp.workdps(50):
        scale = max(max(abs(v) for v in st) for st in b)
        return float(max(abs(x - y) for sa, sb in zip(a, b) for x, y in zip(sa, sb)) / max(scale, 1))


@pytest.mark.parametrize("name,alpha,h,x0,p,x1", [
    ("LINEAR", 0.7, 0.125, [1.0], [1.3], None),
    ("DUFFING", 0.9, 0.05, [0.1, 0.0], [0.1, 0.3, 1.2], None),
    ("LORENZ", 0.95, 0.01, [1.0, 1.0, 1.0], [10.0, 28.0, 8.0 / 3.0], None),
    ("LCR", 0.9, 0.25, [1.2, -0.4], [1.015, 0.55, -1.02, -0.58, 0.117], None),
    ("LCR", (0.9, 0.8), 0.25, [1.2, -0.4], [1.015, 0.55, -1.02, -0.58, 0.117], None),
    ("LINEAR", 1.5, 0.125, [1.0], [1.3], [0.5]),
])
def test_quad_tiny_n_brute_force(name, alpha, h, x0, p, x1):
    """The quad scheme against the 50-digit brute force with quadrature
    weights, to 1e-30 (quad rounding is ~1e-34 per operation; a double-rounded
    weight, Gamma factor, h^alpha or cos/sin would show at 1e-16)."""
    N = 10
    y = O.solve_quad(_RID[name], alpha, h, N, x0, p, out_stride=1, x1=x1)
    ref = _brute_force_mp(name, alpha, h, N, x0, p, x1)
    assert _max_rel_mp(_pairs_mp(y), ref) <= 1e-30


@pytest.mark.parametrize("alpha", [0.35, 0.8, 1.0])
def test_quad_linear_in_t_forcing_is_exact(alpha):
    """f = c0 + c1 t is integrated exactly by the product-trapezoid corrector,
    so y_s = x0 + c0 t^a / Gamma(a+1) + c1 t^(a+1) / Gamma(a+2) to quad
    rounding over 400 steps."""
    c0, c1, h, N, x0 = 0.7, -0.3, 1.0 / 64, 400, 0.25
    y = O.solve_quad(O.RHS_POLY, alpha, h, N, [x0], [c0, c1], out_stride=1)
    got = _pairs_mp(y)
    with mp.workdps(50):
        a = mp.mpf(alpha)
        ref = [[mp.mpf(x0) + mp.mpf(c0) * (s * mp.mpf(h)) ** a / mp.gamma(a + 1)
                + mp.mpf(c1) * (s * mp.mpf(h)) ** (a + 1) / mp.gamma(a + 2)] for s in range(N + 1)]
    assert _max_rel_mp(got, ref) <= 1e-30


@pytest.mark.parametrize("alpha", [0.3, 0.95, 1.5, 2.0])
@pytest.mark.parametrize("k0", [0, 2, 1000, 262144, 3000000])
def test_quad_weights_50_digits(alpha, k0):
    """Quad weights against 50-digit evaluations of the literal formulas.  The
    quad oracle writes the differences of powers through expm1 / log1p
    (exact identities), which lose about log10(k) digits where the literal
    forms would lose 2 log10(k) for a and c; with libquadmath good to a few
    quad ulp and the (hi, lo) pair keeping 106 bits, the bound is
    1e-32 (k+2) relative (measured up to 2.5e-33 (k+2))."""
    n = 6
    b, a, c = O.weights_quad(alpha, n, k0=k0)
    with mp.workdps(50):
        al = mp.mpf(alpha)
        g1, g2 = mp.gamma(al + 1), mp.gamma(al + 2)
        for i in range(n):
            k = mp.mpf(k0 + i)
            rb = ((k + 1) ** al - (k ** al if k0 + i else 0)) / g1
            ra = ((k + 2) ** (al + 1) - 2 * (k + 1) ** (al + 1) + (k ** (al + 1) if k0 + i else 0)) / g2
            rc = ((k ** (al + 1) if k0 + i else 0) - (k - al) * (k + 1) ** al) / g2
            kk = float(k0 + i + 2)
            for got, ref, tol in ((b[i], rb, 1e-32 * kk), (a[i], ra, 1e-32 * kk),
                                  (c[i], rc, 1e-32 * kk)):
                v = mp.mpf(float(got[0])) + mp.mpf(float(got[1]))
                assert abs(v - ref) <= tol * abs(ref), (k0 + i, float(abs(v - ref) / abs(ref)))


def test_quad_steps_from_states_reproduce_a_run():
    pr = dict(rhs=O.RHS_LCR, alpha=(0.9, 0.8), h=0.05, x0=[1.2, -0.4],
              p=[1.015, 0.55, -1.02, -0.58, 0.117])
    N = 600
    y = O.solve_quad(pr["rhs"], pr["alpha"], pr["h"], N, pr["x0"], pr["p"], out_stride=1)
    s_list = [1, 2, 63, 64, 65, 599, 600]
    ys = O.steps_from_states_quad(pr["rhs"], pr["alpha"], pr["h"], pr["x0"], pr["p"], y, s_list)
    # the history enters as (hi, lo) pairs, 106 of its 113 bits
    assert _max_rel_mp(_pairs_mp(ys), _pairs_mp(y[s_list])) <= 1e-30


@pytest.mark.parametrize("rhs,alpha,h,N,x0,p", [
    (O.RHS_DUFFING, 0.95, 2.0 ** -8, 3000, [0.1, 0.0], [0.1, 0.45, 1.2]),
    (O.RHS_LORENZ, 0.93, 2.0 ** -8, 1500, [1.0, 1.0, 1.0], [10.0, 28.0, 8.0 / 3.0]),
    (O.RHS_LCR, (0.9, 0.8), 0.01, 2000, [1.2, -0.4], [1.015, 0.55, -1.02, -0.58, 0.117]),
])
def test_quad_and_double_schemes_agree(rhs, alpha, h, N, x0, p):
    """The quad and double schemes differ only by rounding (the double
    oracle's is ~1e-15 here): a wrong right-hand side or weight in either
    would differ at order one."""
    yq = O.solve_quad(rhs, alpha, h, N, x0, p, out_stride=7)
    yd = O.solve(rhs, alpha, h, N, x0, p, out_stride=7)
    assert np.max(np.abs(yq[..., 0] + yq[..., 1] - yd)) <= 1e-13 * np.max(np.abs(yd))
