"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it does not compute: hand-derived traces of
the update rules (tests/golden), closed forms of the recurrences, library routines
(scipy.signal.lfilter, pandas ewm, scikit-learn), exact special cases and invariants. Chosen
so that a dropped term, a wrong sign or index, or a transposed operand fails at least one.
"""
import math

import numpy as np
import pandas as pd
import pytest
import scipy.signal
import torch

from oracle import MixParams, MixtureOracle, ScalarMixture, FusionOracle, fuse_step, round_to_storage
from oracle import metrics
from tests.goldens import mixture_trace, fusion_traces

TRACE_PARAMS = dict(alpha=0.5, k=2.5, T=0.7, sigma0=10.0, var_min=1.0, w_init=0.5)


def _ranks(o: MixtureOracle, pix=0):
    out = []
    for r in range(o.p.M):
        if o.w[r, pix] == 0.0:
            out.append(None)
        else:
            out.append((tuple(o.mu[r, :, pix]), o.var[r, pix], o.w[r, pix]))
    return out


def _check_trace(rows, C, M):
    p = MixParams(M=M, **TRACE_PARAMS)
    vec = MixtureOracle(p, C, 1)
    sca = ScalarMixture(p, C)
    for t, (x, comps, B, fg) in enumerate(rows):
        info = vec.step(np.array([x], dtype=np.float64))
        fg_s = sca.step(x)
        got = _ranks(vec)
        for r, (exp, g) in enumerate(zip(comps, got)):
            if exp is None:
                assert g is None, (t, r, g)
                continue
            assert g is not None, (t, r)
            np.testing.assert_allclose(g[0], exp[0], rtol=0, atol=1e-12, err_msg=f"t{t} r{r} mu")
            assert g[1] == pytest.approx(exp[1], abs=1e-12), (t, r, "var")
            assert g[2] == pytest.approx(exp[2], abs=1e-12), (t, r, "w")
        assert int(info.B[0]) == B, (t, "B")
        assert bool(info.fg[0]) == bool(fg), (t, "fg")
        assert bool(fg_s) == bool(fg), (t, "fg scalar")
        mu_s, var_s, w_s = sca.state()
        for r in range(M):
            assert w_s[r] == pytest.approx(vec.w[r, 0], abs=1e-12)
            if w_s[r] > 0:
                assert var_s[r] == pytest.approx(vec.var[r, 0], abs=1e-12)
                np.testing.assert_allclose(mu_s[r], vec.mu[r, :, 0], atol=1e-12)


def test_depth_trace_hand_derived():
    _check_trace(mixture_trace("trace_depth_m3.txt", 1), C=1, M=3)


def test_rgb_trace_hand_derived():
    _check_trace(mixture_trace("trace_rgb_m2.txt", 3), C=3, M=2)


@pytest.mark.parametrize("C", [1, 3])
def test_constant_stream_closed_form(C):
    # x == c forever: the first frame creates one component (w=1, fg=1); afterwards mu = c
    # exactly, w = 1, fg = 0 and var_t = max(var_min, (1-a)^t sigma0^2)
    a, s0, vmin = 0.1, 50.0, 25.0
    p = MixParams(M=3, alpha=a, k=2.5, T=0.7, sigma0=s0, var_min=vmin, w_init=a)
    o = MixtureOracle(p, C, 1)
    c = np.array([[1234.0] * C])
    floor_t = math.ceil(math.log(vmin / s0 ** 2) / math.log(1 - a))
    assert floor_t == 44
    for t in range(80):
        info = o.step(c)
        assert bool(info.fg[0]) == (t == 0)
        assert o.w[0, 0] == pytest.approx(1.0, abs=1e-15)
        assert np.all(o.w[1:, 0] == 0.0)
        np.testing.assert_allclose(o.mu[0, :, 0], 1234.0, rtol=1e-14)
        expect = max(vmin, (1 - a) ** t * s0 ** 2)
        assert o.var[0, 0] == pytest.approx(expect, rel=1e-12)
        if t >= floor_t:
            assert o.var[0, 0] == vmin


def test_single_component_mean_is_exponential_moving_average():
    # M=1 with an unreachable threshold: every frame matches, so the mean is an EMA and the
    # variance an EMA of squared residuals about the new mean.
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 255, size=200)
    a = 0.07
    p = MixParams(M=1, alpha=a, k=1e9, T=0.7, sigma0=30.0, var_min=1e-300, w_init=a)
    o = MixtureOracle(p, 1, 1)
    mus, vars_ = [], []
    for t in range(len(x)):
        info = o.step(x[t:t + 1])
        assert bool(info.fg[0]) == (t == 0)
        mus.append(o.mu[0, 0, 0])
        vars_.append(o.var[0, 0])
    ewm = pd.Series(x).ewm(alpha=a, adjust=False).mean().to_numpy()
    np.testing.assert_allclose(mus, ewm, rtol=1e-12)
    lf, _ = scipy.signal.lfilter([a], [1.0, a - 1.0], x[1:], zi=[(1 - a) * x[0]])
    np.testing.assert_allclose(mus[1:], lf, rtol=1e-12)
    r2 = (x[1:] - ewm[1:]) ** 2
    v, _ = scipy.signal.lfilter([a], [1.0, a - 1.0], r2, zi=[(1 - a) * 30.0 ** 2])
    np.testing.assert_allclose(vars_[1:], v, rtol=1e-10)
    assert vars_[0] == 900.0


def test_match_boundary_is_strict():
    # mu=100, var=100, k=2.5: x=125 gives d2 = 625 = k^2 var exactly -> no match
    p = MixParams(M=3, alpha=0.01, k=2.5, T=0.7, sigma0=30.0, var_min=9.0, w_init=0.01)
    for x, expect_match in ((125.0, False), (124.0, True), (75.0, False), (76.0, True)):
        o = MixtureOracle(p, 1, 1)
        o.set_state(np.array([100.0, 0, 0]).reshape(3, 1, 1), np.array([100.0, 900, 900]).reshape(3, 1),
                    np.array([1.0, 0, 0]).reshape(3, 1))
        info = o.step(np.array([[x]]))
        assert bool(info.matched[0]) == expect_match
        assert bool(info.fg[0]) == (not expect_match)
        s = ScalarMixture(p, 1)
        s.comps = [[[100.0], 100.0, 1.0], [[0.0], 900.0, 0.0], [[0.0], 900.0, 0.0]]
        assert s.step([x]) == (not expect_match)


def test_grey_colour_equals_scaled_single_channel():
    # colour input (x,x,x) with grey means behaves like one channel sqrt(3) x: same variances,
    # weights and masks, means scaled by sqrt(3). Catches a dropped or mis-indexed channel term.
    rng = np.random.default_rng(11)
    n, T = 64, 40
    p = MixParams(M=4, alpha=0.05, k=2.5, T=0.7, sigma0=30.0, var_min=9.0, w_init=0.05)
    col = MixtureOracle(p, 3, n)
    one = MixtureOracle(p, 1, n)
    base = rng.uniform(20, 230, size=n)
    s3 = math.sqrt(3.0)
    for t in range(T):
        g = base + rng.normal(0, 6, size=n) + (60 * (rng.random(n) < 0.15))
        i3 = col.step(np.repeat(g[:, None], 3, axis=1))
        i1 = one.step(s3 * g[:, None])
        np.testing.assert_array_equal(i3.fg, i1.fg)
        np.testing.assert_allclose(col.var, one.var, rtol=1e-9)
        np.testing.assert_allclose(col.w, one.w, rtol=1e-9, atol=1e-15)
        for c in range(3):
            np.testing.assert_allclose(s3 * col.mu[:, c, :], one.mu[:, 0, :], rtol=1e-9, atol=1e-9)


def _random_stream(rng, n, C, T, spread):
    centres = rng.uniform(50, 200, size=(3, n, C))
    xs = []
    for t in range(T):
        which = rng.integers(0, 3, size=n)
        noise = rng.normal(0, spread, size=(n, C))
        xs.append(np.round(np.clip(centres[which, np.arange(n)] + noise, 0, 255)))
    return xs


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("C", [1, 3])
def test_vectorised_equals_scalar(M, C):
    rng = np.random.default_rng(100 * M + C)
    n, T = 16, 30
    p = MixParams(M=M, alpha=float(rng.uniform(0.05, 0.4)), k=float(rng.uniform(1.5, 3.0)),
                  T=float(rng.uniform(0.4, 0.9)), sigma0=float(rng.uniform(8, 30)), var_min=4.0,
                  w_init=float(rng.uniform(0.05, 0.3)))
    vec = MixtureOracle(p, C, n)
    sca = [ScalarMixture(p, C) for _ in range(n)]
    n_match = n_nomatch = 0
    for x in _random_stream(rng, n, C, T, spread=6.0):
        info = vec.step(x)
        for i in range(n):
            fg = sca[i].step(x[i])
            assert fg == bool(info.fg[i])
            mu_s, var_s, w_s = sca[i].state()
            np.testing.assert_allclose(w_s, vec.w[:, i], rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(var_s, vec.var[:, i], rtol=1e-12)
            np.testing.assert_allclose(np.array(mu_s), vec.mu[:, :, i], rtol=1e-12, atol=1e-12)
        n_match += int(info.matched.sum())
        n_nomatch += int((~info.matched).sum())
    assert n_match > 0 and n_nomatch > n  # both branches exercised


def _live(o):
    return o.w > 0


def test_invariants_on_generated_stream():
    from paper_2110_14934_amd.synth import Stream, workload
    wl = workload("plain-160x120")
    spec = wl.streams[0]
    st = Stream(spec)
    mp = wl.mix
    n = spec.npix
    pc = MixParams(M=mp.M, alpha=mp.alpha, k=mp.k, T=mp.T, sigma0=mp.sigma0_rgb, var_min=mp.var_min_rgb,
                   w_init=mp.w_init)
    pd_ = MixParams(M=mp.M, alpha=mp.alpha, k=mp.k, T=mp.T, sigma0=mp.sigma0_depth, var_min=mp.var_min_depth,
                    w_init=mp.w_init, hole_skip=True)
    oc, od = MixtureOracle(pc, 3, n), MixtureOracle(pd_, 1, n)
    lo_c = np.full((3, n), np.inf); hi_c = np.full((3, n), -np.inf)
    lo_d = np.full(n, np.inf); hi_d = np.full(n, -np.inf)
    prev_live_c = np.zeros(n, int); prev_live_d = np.zeros(n, int)
    for t in range(25):
        rgb = st.rgb(t).reshape(-1, 3).numpy().astype(np.float64)
        dep = st.depth(t).reshape(-1).numpy().astype(np.float64)
        lo_c = np.minimum(lo_c, rgb.T); hi_c = np.maximum(hi_c, rgb.T)
        ok = dep > 0
        lo_d = np.where(ok, np.minimum(lo_d, dep), lo_d); hi_d = np.where(ok, np.maximum(hi_d, dep), hi_d)
        for o, x, pp, prev in ((oc, rgb, pc, prev_live_c), (od, dep, pd_, prev_live_d)):
            info = o.step(x)
            live = _live(o)
            ws = o.w.sum(axis=0)
            touched = live.any(axis=0)
            np.testing.assert_allclose(ws[touched], 1.0, atol=1e-12)
            assert np.all(o.w >= 0)
            nl = live.sum(axis=0)
            assert np.all(nl >= prev) and np.all(nl <= pp.M)
            prev[:] = nl
            key = o.w / np.sqrt(o.var)
            assert np.all(np.diff(key, axis=0) <= 0)
            assert np.all(o.var[live] >= pp.var_min)
            assert np.all(info.fg[~info.matched & ~info.hole])
            # live components come first
            assert np.all(np.diff(live.astype(int), axis=0) <= 0)
        # means are convex combinations of the pixel's inputs
        for r in range(mp.M):
            lv = oc.w[r] > 0
            assert np.all(oc.mu[r][:, lv] >= lo_c[:, lv] - 1e-9) and np.all(oc.mu[r][:, lv] <= hi_c[:, lv] + 1e-9)
            lv = od.w[r] > 0
            assert np.all(od.mu[r, 0, lv] >= lo_d[lv] - 1e-9) and np.all(od.mu[r, 0, lv] <= hi_d[lv] + 1e-9)


def test_depth_holes_leave_state_untouched():
    p = MixParams(M=3, alpha=0.2, k=2.5, T=0.7, sigma0=50.0, var_min=25.0, w_init=0.2, hole_skip=True)
    o = MixtureOracle(p, 1, 4)
    o.step(np.array([[2000.0], [2001.0], [1500.0], [1999.0]]))
    o.step(np.array([[2010.0], [1990.0], [1200.0], [2000.0]]))
    before = o.get_state()
    info = o.step(np.array([[0.0], [2000.0], [0.0], [0.0]]))
    after = o.get_state()
    for b, a in zip(before, after):
        np.testing.assert_array_equal(b[..., [0, 2, 3]], a[..., [0, 2, 3]])
    assert not info.fg[[0, 2, 3]].any()
    assert info.hole.tolist() == [True, False, True, True]
    # with the policy off, 0 is an ordinary (far) reading: no match, so foreground
    p2 = MixParams(**{**p.__dict__, "hole_skip": False})
    o2 = MixtureOracle(p2, 1, 1)
    o2.step(np.array([[2000.0]]))
    assert bool(o2.step(np.array([[0.0]])).fg[0])


def test_pixel_permutation_commutes():
    rng = np.random.default_rng(5)
    n = 40
    p = MixParams(M=3, alpha=0.1, k=2.5, T=0.7, sigma0=20.0, var_min=4.0, w_init=0.1)
    perm = rng.permutation(n)
    a, b = MixtureOracle(p, 3, n), MixtureOracle(p, 3, n)
    for x in _random_stream(rng, n, 3, 20, spread=8.0):
        ia = a.step(x)
        ib = b.step(x[perm])
        np.testing.assert_array_equal(ia.fg[perm], ib.fg)
        np.testing.assert_array_equal(a.mu[:, :, perm], b.mu)
        np.testing.assert_array_equal(a.w[:, perm], b.w)


# ---- fusion ------------------------------------------------------------------------------

def test_fusion_hand_traces():
    for name, (inputs, states) in fusion_traces().items():
        f = FusionOracle(1)
        for (r, d), (I, c) in zip(inputs, states):
            out = f.step(np.array([r]), np.array([d]))
            assert (int(f.I[0]), int(f.cpt[0])) == (I, c), name
            assert bool(out[0]) == bool(I)


def test_fusion_exhaustive_properties():
    # every sequence of 8 (r, d) pairs, one per pixel: 4^8 = 65536 sequences
    L = 8
    n = 4 ** L
    codes = np.arange(n)
    I = np.zeros(n, np.int64)
    c = np.zeros(n, np.int64)
    for s in range(L):
        sym = (codes >> (2 * s)) & 3
        r, d = sym & 1, sym >> 1
        I2, c2 = fuse_step(r, d, I, c)
        assert np.all((c2 >= -3) & (c2 <= 3))
        agree = r == d
        # agreement: the fused bit is the common vote and the counter resets
        assert np.all(I2[agree] == d[agree]) and np.all(c2[agree] == 0)
        # the fused bit can only change on agreement or when a saturated counter is met
        changed = I2 != I
        assert np.all(agree[changed] | (np.abs(c[changed]) == 3))
        # a saturated counter meeting a disagreement always resets
        sat = ~agree & (np.abs(c) == 3)
        assert np.all(c2[sat] == 0)
        # unsaturated disagreement moves the counter by exactly one step
        mv = ~agree & (np.abs(c) < 3)
        assert np.all(np.abs(c2[mv] - c[mv]) == 1) and np.all(I2[mv] == I[mv])
        I, c = I2, c2


@pytest.mark.parametrize("r,d", [(1, 0), (0, 1)])
@pytest.mark.parametrize("I0", [0, 1])
@pytest.mark.parametrize("c0", [-3, -2, -1, 0, 1, 2, 3])
def test_persistent_disagreement_never_flips_a_settled_bit(r, d, I0, c0):
    # The prose rule of Sec. III.C: a pixel keeps its state under lasting incoherence between
    # the two modalities. Under List 1 that holds once the counter has reset; only a counter
    # already saturated in the opposite sense can flip the bit, once.
    I, c = np.array([I0]), np.array([c0])
    flips = 0
    for _ in range(40):
        I2, c = fuse_step(np.array([r]), np.array([d]), I, c)
        flips += int(I2[0] != I[0])
        I = I2
    assert flips <= 1
    Is = []
    for _ in range(12):
        I, c = fuse_step(np.array([r]), np.array([d]), I, c)
        Is.append(int(I[0]))
    assert len(set(Is)) == 1


# ---- metrics (Eqs. 1-3) ------------------------------------------------------------------

def test_metrics_hand_counted():
    pred = np.array([1, 1, 1, 0, 0, 0, 1, 0], bool)
    truth = np.array([1, 1, 0, 1, 0, 0, 1, 1], bool)
    # TP = 3 (0,1,6), FP = 1 (2), FN = 2 (3,7), TN = 2
    assert metrics.confusion(pred, truth) == (3, 1, 2, 2)
    assert metrics.recall(pred, truth) == pytest.approx(3 / 5)
    assert metrics.precision(pred, truth) == pytest.approx(3 / 4)
    assert metrics.f1_score(pred, truth) == pytest.approx(2 * 0.75 * 0.6 / 1.35)
    assert math.isnan(metrics.precision(np.zeros(4, bool), np.ones(4, bool)))


def test_metrics_match_scikit_learn():
    sk = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(9)
    for _ in range(20):
        truth = rng.random(500) < rng.uniform(0.05, 0.5)
        pred = truth ^ (rng.random(500) < rng.uniform(0.01, 0.3))
        assert metrics.recall(pred, truth) == pytest.approx(sk.recall_score(truth, pred))
        assert metrics.precision(pred, truth) == pytest.approx(sk.precision_score(truth, pred))
        assert metrics.f1_score(pred, truth) == pytest.approx(sk.f1_score(truth, pred))


# ---- storage rounding used by the reduced-precision emulation ---------------------------

def test_storage_rounding_matches_torch_conversions():
    rng = np.random.default_rng(2)
    v32 = np.concatenate([
        rng.uniform(-300, 300, 4000), rng.uniform(0, 1, 4000), 2.0 ** rng.uniform(-140, 120, 4000),
        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 65504.0, 2.0 ** -24]),
    ]).astype(np.float32)
    v = v32.astype(np.float64)   # float32-exact inputs: torch's float32 conversions round once
    bf_t = torch.from_numpy(v32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_to_storage(v, "bf16"), bf_t)
    small = v[np.abs(v) < 60000]
    f16_t = torch.from_numpy(small.astype(np.float32)).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_to_storage(small, "f16"), f16_t)
    assert round_to_storage(np.array([1 + 2 ** -8]), "bf16")[0] == 1.0          # tie -> even
    assert round_to_storage(np.array([1 + 3 * 2 ** -8]), "bf16")[0] == 1 + 2 ** -6


# ---- the ablation variants: density rate, four-channel augmentation ----------------------

@pytest.mark.parametrize("C", [1, 3, 4])
def test_density_rate_matches_scipy_gaussian_pdf(C):
    # One live component, x inside k sigma: the mean moves towards x by the fraction rho, which
    # must equal alpha times scipy's multivariate normal density N(x | mu, var I) (an independent
    # evaluation of the density: normalisation, power of 2 pi, the 1/2 in the exponent).
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(40 + C)
    n, a = 24, 0.3
    p = MixParams(M=2, alpha=a, k=2.5, T=0.7, sigma0=30.0, var_min=1e-6, w_init=a, rho="density")
    o = MixtureOracle(p, C, n)
    mu = rng.uniform(50, 200, size=(n, C))
    var = rng.uniform(0.5, 40.0, size=n)                        # small variances: rho up to ~0.1
    o.set_state(np.stack([mu.T, np.zeros((C, n))]), np.stack([var, np.full(n, 900.0)]),
                np.stack([np.ones(n), np.zeros(n)]))
    x = mu + rng.normal(0, 1, size=(n, C)) * np.sqrt(var)[:, None] * 0.8
    x[0] = mu[0]                                                # d = 0: rho = alpha (2 pi var)^(-C/2)
    info = o.step(x)
    for i in range(n):
        d2 = float(((x[i] - mu[i]) ** 2).sum())
        if d2 >= 6.25 * var[i]:
            assert not info.matched[i]
            continue
        assert info.matched[i]
        pdf = multivariate_normal.pdf(x[i], mean=mu[i], cov=var[i] * np.eye(C))
        r = 0 if o.w[0, i] > o.w[1, i] and o.var[0, i] != 900.0 else 1
        new_mu = o.mu[r, :, i]
        if i == 0:
            np.testing.assert_allclose(new_mu, mu[0], rtol=0, atol=1e-12)
            continue
        c = int(np.argmax(np.abs(x[i] - mu[i])))
        rho = (new_mu[c] - mu[i, c]) / (x[i, c] - mu[i, c])
        assert rho == pytest.approx(a * pdf, rel=1e-9), i
        # every channel moves by the same fraction
        np.testing.assert_allclose(new_mu - mu[i], rho * (x[i] - mu[i]), rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("C", [1, 3, 4])
@pytest.mark.parametrize("M", [3, 5])
def test_density_rate_vectorised_equals_scalar(M, C):
    rng = np.random.default_rng(700 + 10 * M + C)
    n, T = 16, 40
    p = MixParams(M=M, alpha=0.3, k=2.5, T=0.6, sigma0=6.0, var_min=0.25, w_init=0.2, rho="density")
    vec = MixtureOracle(p, C, n)
    sca = [ScalarMixture(p, C) for _ in range(n)]
    for x in _random_stream(rng, n, C, T, spread=1.5):
        info = vec.step(x)
        for i in range(n):
            assert sca[i].step(x[i]) == bool(info.fg[i])
            mu_s, var_s, w_s = sca[i].state()
            np.testing.assert_allclose(w_s, vec.w[:, i], rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(var_s, vec.var[:, i], rtol=1e-12)
            np.testing.assert_allclose(np.array(mu_s), vec.mu[:, :, i], rtol=1e-12, atol=1e-12)


def test_density_rate_differs_from_alpha_rate():
    # the two readings of rho must give different means on the same input (a variant that
    # silently fell back to alpha would pass every other density pin with rho = alpha ...
    # except this one)
    rng = np.random.default_rng(5)
    n = 32
    xs = _random_stream(rng, n, 3, 20, spread=3.0)
    base = dict(M=3, alpha=0.1, k=2.5, T=0.7, sigma0=20.0, var_min=4.0, w_init=0.1)
    oa = MixtureOracle(MixParams(**base), 3, n)
    od = MixtureOracle(MixParams(**base, rho="density"), 3, n)
    for x in xs:
        oa.step(x)
        od.step(x)
    assert np.abs(oa.mu - od.mu).max() > 0.1


def test_depth_byte_hand_values():
    from oracle import depth_byte
    d = np.array([0, 1, 15, 16, 17, 31, 32, 1200, 2000, 4079, 4080, 4095, 4096, 65535])
    assert depth_byte(d).tolist() == [0, 0, 0, 1, 1, 1, 2, 75, 125, 254, 255, 255, 255, 255]


def test_vectorised_equals_scalar_four_channels():
    rng = np.random.default_rng(404)
    n, T = 16, 30
    p = MixParams(M=4, alpha=0.2, k=2.5, T=0.7, sigma0=15.0, var_min=4.0, w_init=0.1)
    vec = MixtureOracle(p, 4, n)
    sca = [ScalarMixture(p, 4) for _ in range(n)]
    for x in _random_stream(rng, n, 4, T, spread=6.0):
        info = vec.step(x)
        for i in range(n):
            assert sca[i].step(x[i]) == bool(info.fg[i])
            mu_s, var_s, w_s = sca[i].state()
            np.testing.assert_allclose(w_s, vec.w[:, i], rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(var_s, vec.var[:, i], rtol=1e-12)
            np.testing.assert_allclose(np.array(mu_s), vec.mu[:, :, i], rtol=1e-12, atol=1e-12)


def test_augmented_with_constant_depth_is_the_colour_model():
    # A depth byte that never changes adds nothing to any distance once a component holds it,
    # so the four-channel model must reproduce the three-channel colour model: same masks,
    # variances, weights and colour means; the depth mean stays at the byte.
    from oracle import AugmentedOracle
    rng = np.random.default_rng(8)
    n, T = 48, 40
    p = MixParams(M=4, alpha=0.05, k=2.5, T=0.7, sigma0=30.0, var_min=9.0, w_init=0.05, hole_skip=True)
    aug = AugmentedOracle(p, n)
    col = MixtureOracle(p, 3, n)
    depth = np.full(n, 2000, dtype=np.uint16)              # byte 125
    for rgb in _random_stream(rng, n, 3, T, spread=5.0):
        ia = aug.step(rgb, depth)
        ic = col.step(rgb)
        np.testing.assert_array_equal(ia.fg, ic.fg)
        mu, var, w = aug.get_state()
        np.testing.assert_allclose(var, col.var, rtol=1e-12)
        np.testing.assert_allclose(w, col.w, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(mu[:, :3], col.mu, rtol=1e-12, atol=1e-12)
        live = w > 0
        np.testing.assert_allclose(mu[:, 3][live], 125.0, rtol=1e-12)


def test_augmented_depth_change_alone_is_foreground_and_holes_are_skipped():
    # fixed colour; after the background settles, a depth jump of 400 mm (25 bytes) alone must
    # make the pixel foreground (25^2 = 625 > k^2 var with var at its floor 9 is not needed:
    # the settled variance is at the floor); a hole leaves the state untouched, background
    from oracle import AugmentedOracle
    p = MixParams(M=3, alpha=0.05, k=2.5, T=0.7, sigma0=30.0, var_min=9.0, w_init=0.05, hole_skip=True)
    aug = AugmentedOracle(p, 1)
    rgb = np.array([[100, 120, 140]])
    for _ in range(200):
        info = aug.step(rgb, np.array([2000]))
    assert not info.fg[0]
    before = [a.copy() for a in aug.get_state()]
    info = aug.step(rgb, np.array([0]))
    assert info.hole[0] and not info.fg[0]
    for a, b in zip(aug.get_state(), before):
        np.testing.assert_array_equal(a, b)
    info = aug.step(rgb, np.array([1600]))
    assert info.fg[0] and not info.matched[0]
