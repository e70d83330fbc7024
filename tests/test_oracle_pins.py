"""Pins for the CPU oracle: closed forms, invariants and special cases fixed by the mathematics.

Each test checks the oracle against something other than its own formulas:
  * unit-circle spectra of S and D (Fourier series of log|e^{it} - e^{is}|),
  * Gauss's identity for D applied to the constant density,
  * Green's representation formula (the paper's accuracy test, Sec. 5.1),
  * the special case "center = target", where eq. (qbx) reduces to the plain quadrature sum of
    the layer-potential definitions (eqs. slp/dlp) written here in real-vector form,
  * Taylor-remainder bounds for a single source (wrong indices or factorials violate them),
  * far/near-field bounds for the brute-force multipole and local expansions (eqs. multipole,
    local).
"""
import math

import numpy as np
import pytest

import gq_inputs as gi
import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def test_gauss_legendre_exact_on_polynomials():
    for n in (4, 16, 33):
        x, w = gi.gauss_legendre(n)
        for deg in range(0, 2 * n):
            exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
            assert abs(np.dot(w, x ** deg) - exact) < 1e-13


def test_geometry_normals_and_area():
    g = gi.unit_circle(32)
    assert np.allclose(np.hypot(*g.src_nrm.T), 1.0, atol=1e-15)
    # divergence theorem: area = 1/2 int x . n ds > 0 iff normals point outward
    area = 0.5 * np.sum(g.src_w * np.einsum("ij,ij->i", g.src_xy, g.src_nrm))
    assert abs(area - math.pi) < 1e-12
    assert abs(g.src_w.sum() - 2 * math.pi) < 1e-12
    star = gi.starfish_c1()
    a = 0.5 * np.sum(star.src_w * np.einsum("ij,ij->i", star.src_xy, star.src_nrm))
    # area of r = 1 + 0.25 cos 5t is pi (1 + 0.25^2 / 2)
    assert abs(a - math.pi * (1 + 0.25 ** 2 / 2)) < 1e-12


@pytest.mark.parametrize("k", [1, 3, 6])
def test_circle_single_layer_interior_is_exact(k):
    # interior side: the potential r^k cos(k t)/(2k) is a polynomial, no truncation error for k <= p
    g = gi.unit_circle(64, order=32)
    mu = np.cos(k * g.theta)
    u = oracle.qbx_eval(g.one_sided(-1), oracle.S, mu, p_qbx=8)
    assert np.abs(u - np.cos(k * g.theta) / (2 * k)).max() < 2e-14


def test_circle_single_layer_exterior_converges_in_p():
    g = gi.unit_circle(64, order=32)
    k = 3
    mu = np.cos(k * g.theta)
    exact = np.cos(k * g.theta) / (2 * k)
    r = g.ctr_r[1]
    errs = []
    for p in (4, 6, 8, 10):
        u = oracle.qbx_eval(g.one_sided(+1), oracle.S, mu, p_qbx=p)
        errs.append(np.abs(u - exact).max())
        # exterior potential Re z^{-k}/(2k) expanded about |c| = 1 + r, evaluated at distance r:
        # Taylor tail of (1+r+w)^{-k} bounded by a geometric series in rho = r/(1+r)
        rho = r / (1 + r)
        bound = math.comb(p + k, p + 1) * rho ** (p + 1) / (1 - rho) ** (p + k + 1) / (2 * k)
        assert errs[-1] <= 1.05 * bound + 1e-14
    assert errs[-1] < 1e-11
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


@pytest.mark.parametrize("k", [2, 5])
def test_circle_double_layer_jump(k):
    g = gi.unit_circle(64, order=32)
    mu = np.cos(k * g.theta)
    ref = 0.5 * np.cos(k * g.theta)
    dm = oracle.qbx_eval(g.one_sided(-1), oracle.D, mu, p_qbx=12)
    dp = oracle.qbx_eval(g.one_sided(+1), oracle.D, mu, p_qbx=12)
    da = oracle.qbx_eval(g, oracle.D, mu, p_qbx=12)
    assert np.abs(dm + ref).max() < 1e-12
    assert np.abs(dp - ref).max() < 1e-12
    assert np.abs(da).max() < 1e-12


def test_gauss_identity_starfish():
    g = gi.discretize([gi.StarCurve(amp=0.25, arms=5)], 64, order=32)
    one = np.ones(g.n_src)
    dm = oracle.qbx_eval(g.one_sided(-1), oracle.D, one, p_qbx=10)
    dp = oracle.qbx_eval(g.one_sided(+1), oracle.D, one, p_qbx=10)
    da = oracle.qbx_eval(g, oracle.D, one, p_qbx=10)
    assert np.abs(dm + 1.0).max() < 1e-9
    assert np.abs(dp).max() < 1e-9
    assert np.abs(da + 0.5).max() < 1e-9


def test_green_representation_starfish():
    # S(du/dn) - D(u) = u/2 on the curve (average of sides), u inside, 0 outside, for u harmonic
    # inside: u = log|x - x0| with the charge x0 = (2, 1) outside (the paper's Sec. 5.1 test).
    g = gi.discretize([gi.StarCurve(amp=0.25, arms=5)], 64, order=32)
    sig, tau, u = gi.green_test_field(g, (2.0, 1.0))
    avg = oracle.qbx_eval(g, oracle.S_MINUS_D, sig, tau, p_qbx=10)
    inn = oracle.qbx_eval(g.one_sided(-1), oracle.S_MINUS_D, sig, tau, p_qbx=10)
    out = oracle.qbx_eval(g.one_sided(+1), oracle.S_MINUS_D, sig, tau, p_qbx=10)
    scale = np.abs(u).max()
    assert np.abs(avg - u / 2).max() / scale < 1e-9
    assert np.abs(inn - u).max() / scale < 1e-9
    assert np.abs(out).max() / scale < 1e-9


def test_green_representation_multi_curve():
    # several disjoint curves: for a point on one curve the others contribute their exterior value 0
    g = gi.random_stars(n_curves=3, panels_per_curve=96, seed=7, box=10.0, order=32)
    sig, tau, u = gi.green_test_field(g, (-3.0, -2.0))
    avg = oracle.qbx_eval(g, oracle.S_MINUS_D, sig, tau, p_qbx=10)
    assert np.abs(avg - u / 2).max() / np.abs(u).max() < 1e-11


def _direct_real_vector(g, dens1, dens2, x):
    """Layer potentials by plain quadrature, eqs. (slp)/(dlp) in real-vector form."""
    d = g.src_xy - x[None, :]
    r2 = np.einsum("ij,ij->i", d, d)
    s = -np.sum(g.src_w * dens1 * 0.5 * np.log(r2)) / (2 * np.pi)
    dd = -np.sum(g.src_w * dens2 * np.einsum("ij,ij->i", g.src_nrm, d) / r2) / (2 * np.pi)
    return s, dd


def test_center_at_target_reduces_to_plain_quadrature():
    g = gi.starfish_c1()
    rng = np.random.default_rng(5)
    mu1 = rng.normal(size=g.n_src)
    mu2 = rng.normal(size=g.n_src)
    pts = np.array([[3.0, 0.5], [0.1, -0.2], [-2.0, 2.5]])
    for p in (0, 5):
        for x in pts:
            tc = np.array([[0, -1]], dtype=np.int32)
            gg = gi.Geometry(**{k: getattr(g, k) for k in g.__dataclass_fields__})
            gg.ctr_xy = x[None, :].copy()
            gg.ctr_r = np.array([0.1])
            s = oracle.qbx_eval(gg, oracle.S, mu1, p_qbx=p, tgt_xy=x[None], tgt_ctr=tc)[0]
            d = oracle.qbx_eval(gg, oracle.D, mu2, p_qbx=p, tgt_xy=x[None], tgt_ctr=tc)[0]
            sd = oracle.qbx_eval(gg, oracle.S_MINUS_D, mu1, mu2, p_qbx=p, tgt_xy=x[None],
                                 tgt_ctr=tc)[0]
            s_ref, d_ref = _direct_real_vector(g, mu1, mu2, x)
            assert abs(s - s_ref) < 1e-13 * max(1.0, abs(s_ref))
            assert abs(d - d_ref) < 1e-13 * max(1.0, abs(d_ref))
            assert abs(sd - (s_ref - d_ref)) < 1e-13 * max(1.0, abs(s_ref) + abs(d_ref))
            # a target with no center is a conventional point target: plain quadrature sum
            none = np.array([[-1, -1]], dtype=np.int32)
            s2 = oracle.qbx_eval(gg, oracle.S, mu1, p_qbx=p, tgt_xy=x[None], tgt_ctr=none)[0]
            assert abs(s2 - s_ref) < 1e-13 * max(1.0, abs(s_ref))


def _single_source_geom(y, n, w=1.0):
    return gi.Geometry(src_xy=np.array([y], float), src_nrm=np.array([n], float),
                       src_w=np.array([w]), theta=np.zeros(1), curve_id=np.zeros(1, np.int32),
                       panel_id=np.zeros(1, np.int32), panel_len=np.ones(1),
                       ctr_xy=np.zeros((1, 2)), ctr_r=np.ones(1), tgt_xy=np.zeros((1, 2)),
                       tgt_ctr=np.zeros((1, 2), np.int32))


@pytest.mark.parametrize("p", [0, 1, 3, 7, 12])
def test_single_source_taylor_remainder(p):
    rng = np.random.default_rng(p)
    for _ in range(20):
        y = rng.uniform(-1, 1, 2)
        nrm = rng.normal(size=2)
        nrm /= np.linalg.norm(nrm)
        g = _single_source_geom(y, nrm)
        c = y + rng.uniform(0.5, 1.0) * rng.normal(size=2)
        R = np.linalg.norm(y - c)
        x = c + rng.uniform(0.1, 0.6) * R * rng.normal(size=2) / math.sqrt(2)
        rho = np.linalg.norm(x - c) / R
        if rho >= 0.8:
            continue
        tc = np.array([[0, -1]], dtype=np.int32)
        g.ctr_xy = c[None, :]
        s = oracle.qbx_eval(g, oracle.S, np.ones(1), p_qbx=p, tgt_xy=x[None], tgt_ctr=tc)[0]
        d = oracle.qbx_eval(g, oracle.D, np.ones(1), p_qbx=p, tgt_xy=x[None], tgt_ctr=tc)[0]
        dx = y - x
        s_true = -math.log(np.linalg.norm(dx)) / (2 * math.pi)
        d_true = -np.dot(nrm, dx) / np.dot(dx, dx) / (2 * math.pi)
        # log(1 - t) tail: sum_{m>p} t^m/m; 1/(1-t) tail: sum_{m>p} t^m (divided by R)
        s_bound = rho ** (p + 1) / ((p + 1) * (1 - rho)) / (2 * math.pi)
        d_bound = rho ** (p + 1) / (1 - rho) / R / (2 * math.pi)
        assert abs(s - s_true) <= s_bound * (1 + 1e-9) + 1e-15
        assert abs(d - d_true) <= d_bound * (1 + 1e-9) + 1e-15
        # and the error is not much smaller than the leading neglected term would allow
        # (a dropped or duplicated term would overshoot or vanish)
        if rho > 0.3 and p < 8:
            assert abs(s - s_true) > 1e-3 * s_bound


def _box_sources(rng, n, half, center=(0.0, 0.0)):
    xy = np.asarray(center) + rng.uniform(-half, half, size=(n, 2))
    nrm = rng.normal(size=(n, 2))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    g = gi.Geometry(src_xy=xy, src_nrm=nrm, src_w=rng.uniform(0.5, 1.5, n), theta=np.zeros(n),
                    curve_id=np.zeros(n, np.int32), panel_id=np.zeros(n, np.int32),
                    panel_len=np.ones(n), ctr_xy=np.zeros((1, 2)), ctr_r=np.ones(1),
                    tgt_xy=np.zeros((1, 2)), tgt_ctr=np.zeros((1, 2), np.int32))
    return g


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_multipole_far_field_bound(kind):
    rng = np.random.default_rng(11 + kind)
    g = _box_sources(rng, 40, 0.5, (0.3, -0.2))
    m1, m2 = rng.normal(size=40), rng.normal(size=40)
    ctr = np.array([0.3, -0.2])
    R = math.sqrt(2) * 0.5
    far = ctr + np.array([[3.0, 0.4], [-2.0, -2.5], [0.0, 2.0]])
    exact = oracle.point_potential(g, kind, m1, m2, tgt_xy=far)
    q = np.abs(g.src_w * m1) if kind != 2 else np.zeros(40)
    dl = np.abs(g.src_w * (m2 if kind == 3 else m1)) if kind != 1 else np.zeros(40)
    for p in (5, 10, 20):
        a = oracle.multipole(g, kind, m1, m2, ctr, p)
        approx = oracle.eval_multipole(a, ctr, far)
        for j, x in enumerate(far):
            t = R / np.linalg.norm(x - ctr)
            bound = (q.sum() / (p + 1) + dl.sum() / R) * t ** (p + 1) / (1 - t) / (2 * math.pi)
            assert abs(approx[j] - exact[j]) <= bound * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_local_expansion_near_bound(kind):
    rng = np.random.default_rng(21 + kind)
    g = _box_sources(rng, 40, 0.5, (4.0, 1.0))
    m1, m2 = rng.normal(size=40), rng.normal(size=40)
    ctr = np.array([0.0, 0.0])
    dmin = np.linalg.norm(g.src_xy - ctr, axis=1).min()
    pts = rng.uniform(-0.7, 0.7, size=(6, 2))
    exact = oracle.point_potential(g, kind, m1, m2, tgt_xy=pts)
    q = np.abs(g.src_w * m1) if kind != 2 else np.zeros(40)
    dl = np.abs(g.src_w * (m2 if kind == 3 else m1)) if kind != 1 else np.zeros(40)
    for p in (4, 10, 20):
        b = oracle.local(g, kind, m1, m2, ctr, p)
        approx = oracle.eval_local(b, ctr, pts)
        for j, x in enumerate(pts):
            t = np.linalg.norm(x - ctr) / dmin
            bound = (q.sum() / (p + 1) + dl.sum() / dmin) * t ** (p + 1) / (1 - t) / (2 * math.pi)
            assert abs(approx[j] - exact[j]) <= bound * (1 + 1e-9) + 1e-14


def test_qbx_coeffs_match_local_and_eval():
    # the per-center coefficients and the per-target evaluation are two entry points of one
    # definition; a target evaluated from the returned coefficients must agree
    g = gi.starfish_c1()
    mu = gi.fourier_density(g, seed=0)
    al = oracle.qbx_coeffs(g, oracle.S, mu, p_qbx=8)
    x = g.tgt_xy[:16]
    vals = []
    for t in range(16):
        v = 0.0
        for j in g.tgt_ctr[t]:
            v += oracle.eval_local(al[j], g.ctr_xy[j], x[t:t + 1])[0]
        vals.append(v / 2)
    ref = oracle.qbx_eval(g, oracle.S, mu, p_qbx=8)[:16]
    assert np.abs(np.array(vals) - ref).max() < 1e-14 * np.abs(ref).max() + 1e-15


def test_compensated_sum_is_order_independent():
    g = gi.starfish_c1()
    mu = gi.fourier_density(g, seed=3)
    u1 = oracle.qbx_eval(g, oracle.S, mu, p_qbx=8)
    perm = np.random.default_rng(0).permutation(g.n_src)
    gp = gi.Geometry(**{k: getattr(g, k) for k in g.__dataclass_fields__})
    gp.src_xy, gp.src_nrm, gp.src_w = g.src_xy[perm], g.src_nrm[perm], g.src_w[perm]
    u2 = oracle.qbx_eval(gp, oracle.S, mu[perm], p_qbx=8)
    assert np.abs(u1 - u2).max() <= 4e-16 * np.abs(u1).max() * 8


def test_rough_m2l_estimate_order8():
    """Sec. 2.4, eq. (rough-m2l-error): for boxes of side 1 one box apart, the furthest target of
    the target box lies sqrt(2)/2 from its center and the closest source at least (4 - sqrt 2)/2,
    so an order-8 local expansion errs by about (sqrt 2/(4 - sqrt 2))^9 = 4.4e-3. A unit charge on
    the source box's circumscribed circle, nearest the target box, and a target at the corner
    distance on the same ray are the worst case: the error of the oracle's order-8 local
    expansion there (in units of log|x - y|) is the log series tail sum_{n>8} w^n/n with w the
    distance ratio, below the paper's estimate and within a factor of ten of it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")) as f:
        est = json.load(f)["rough_m2l_estimate_order8"]["value"]
    s2 = math.sqrt(2.0)
    w = s2 / (4 - s2)
    assert abs(w ** 9 - est) < 5e-5  # the paper prints two digits
    g = _single_source_geom(np.array([(4 - s2) / 2, 0.0]), np.array([1.0, 0.0]))
    x = np.array([[s2 / 2, 0.0]])
    b = oracle.local(g, oracle.S, np.ones(1), None, (0.0, 0.0), 8)
    err = abs(oracle.eval_local(b, (0.0, 0.0), x)[0]
              - oracle.point_potential(g, oracle.S, np.ones(1), tgt_xy=x)[0]) * 2 * math.pi
    tail = -math.log1p(-w) - sum(w ** n / n for n in range(1, 9))
    assert err == pytest.approx(tail, rel=1e-9)
    assert est / 10 < err < est


# ---- S' (normal derivative of the single layer potential, Sec. 1 eq. (ext-neumann-ie)) ----

def _sp(g, mu, p, side=0):
    gg = g if side == 0 else g.one_sided(side)
    return oracle.qbx_normal_derivative(gg, mu, p_qbx=p, tgt_nrm=g.src_nrm)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_circle_normal_derivative_one_sided_limits(k):
    """Unit circle, density cos k t: S mu = r^k cos(k t)/(2k) inside and r^-k cos(k t)/(2k)
    outside, so the radial derivative at r = 1 is +cos(k t)/2 from inside (a polynomial: exact
    for p >= k) and -cos(k t)/2 from outside (converging in p); the average (the principal value
    S' mu) is 0. Beyond p ~ 12 the quadrature error of the high coefficients (centers at half a
    panel length, amplified by the factor m of the derivative) takes over, so p stays <= 12."""
    g = gi.unit_circle(64, order=32)
    mu = np.cos(k * g.theta)
    half = 0.5 * np.cos(k * g.theta)
    assert np.abs(_sp(g, mu, 8, -1) - half).max() < 1e-13
    errs = [np.abs(_sp(g, mu, p, +1) + half).max() for p in (4, 8, 12)]
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    assert errs[-1] < 1e-11
    assert np.abs(_sp(g, mu, 12)).max() < 1e-11


def test_circle_normal_derivative_of_constant():
    """S 1 = 0 inside the unit circle and -log r outside: S' 1 is 0 from inside, -1 from outside,
    -1/2 on the curve."""
    g = gi.unit_circle(64, order=32)
    one = np.ones(g.n_src)
    assert np.abs(_sp(g, one, 8, -1)).max() < 1e-13
    assert np.abs(_sp(g, one, 12, +1) + 1.0).max() < 1e-11
    assert np.abs(_sp(g, one, 12) + 0.5).max() < 1e-11


def test_starfish_normal_derivative_jump_and_adjoint_identity():
    """On a starfish with a smooth density: the one-sided limits differ by the density (the jump
    of the single layer's normal derivative), and sum_i w_i S' mu(x_i) = -1/2 sum_i w_i mu_i,
    since S' is the adjoint of the double layer operator and D 1 = -1/2 on the curve (Gauss)."""
    g = gi.discretize([gi.StarCurve(amp=0.25, arms=5)], 256, order=32)
    mu = 1.0 + 0.3 * np.cos(2 * g.theta) - 0.2 * np.sin(5 * g.theta)
    inner, outer = _sp(g, mu, 12, -1), _sp(g, mu, 12, +1)
    assert np.abs((inner - outer) - mu).max() < 1e-9
    avg = _sp(g, mu, 12)
    assert abs(np.sum(g.src_w * avg) + 0.5 * np.sum(g.src_w * mu)) < 1e-12 * np.sum(g.src_w)


def test_normal_derivative_matches_finite_differences():
    """Both branches against central differences of the oracle's potentials along the normal:
    a point target with no center (plain quadrature) and an off-surface target with one
    center (the differentiated expansion against the expansion's own values)."""
    g = gi.discretize([gi.StarCurve(amp=0.25, arms=5)], 32, order=16)
    mu = np.cos(3 * g.theta)
    x = np.array([[2.1, 0.7]])
    nu = np.array([[0.6, 0.8]])
    h = 1e-5
    none = np.full((1, 2), -1, dtype=np.int32)
    got = oracle.qbx_normal_derivative(g, mu, p_qbx=8, tgt_xy=x, tgt_nrm=nu, tgt_ctr=none)
    up = oracle.point_potential(g, oracle.S, mu, tgt_xy=x + h * nu)
    dn = oracle.point_potential(g, oracle.S, mu, tgt_xy=x - h * nu)
    assert abs(got[0] - (up[0] - dn[0]) / (2 * h)) < 1e-8
    j = 7  # an exterior center; a target inside its disk
    c, r = g.ctr_xy[2 * j + 1], g.ctr_r[2 * j + 1]
    xt = (c + 0.5 * r * np.array([0.8, -0.6]))[None, :]
    one = np.array([[2 * j + 1, -1]], dtype=np.int32)
    got = oracle.qbx_normal_derivative(g, mu, p_qbx=10, tgt_xy=xt, tgt_nrm=nu, tgt_ctr=one)
    hh = 1e-6 * r
    up = oracle.qbx_eval(g, oracle.S, mu, p_qbx=10, tgt_xy=xt + hh * nu, tgt_ctr=one)
    dn = oracle.qbx_eval(g, oracle.S, mu, p_qbx=10, tgt_xy=xt - hh * nu, tgt_ctr=one)
    assert abs(got[0] - (up[0] - dn[0]) / (2 * hh)) < 1e-6 * max(1.0, abs(got[0]))
