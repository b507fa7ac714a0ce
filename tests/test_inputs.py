"""The seeded input generators (CPU): determinism, shapes and the physical
structure each stand-in claims (no step of the scheme is checked here)."""
import numpy as np

from paper_0901_4107_amd.inputs import configs


def test_riemann_problems_seeded_and_valid():
    a = configs.riemann_problems(n=4096)
    b = configs.riemann_problems(n=4096)
    assert a.shape == (6, 4096)
    assert np.array_equal(a, b)
    assert np.all(np.isfinite(a))
    assert np.all(a[[0, 3]] > 0) and np.all(a[[2, 5]] > 0)
    c = configs.riemann_problems(n=4096, seed=5)
    assert not np.array_equal(a, c)


def test_harvest_sampling_follows_the_histograms():
    """Problems drawn from one source's histograms land in its bins with the
    bins' frequencies (a chi-square-like check on the joint histogram's
    largest bins), and the drawn features reproduce the histogram's
    quantities: x0 = ln(rho_R/rho_L), x1 = ln(P_R/P_L),
    x2 = (u_R - u_L)/(c_L + c_R) and u_L / c_L inside the edges; no problem
    generates vacuum (x2 < 2/(gamma - 1))."""
    h = configs.load_harvest()
    g = float(h["gamma"])
    rng = np.random.default_rng(11)
    for src in configs.HARVEST_SOURCES:
        n = 200000
        S = configs.sample_harvest(h, src, n, g, rng)
        rl, ul, pl, rr, ur, pr = S
        cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
        f = np.stack([np.log(rr / rl), np.log(pr / pl), (ur - ul) / (cl + cr)], axis=1)
        assert np.all(f[:, 2] < 2.0 / (g - 1.0))
        e = [h["edges_x0"], h["edges_x1"], h["edges_x2"]]
        got, _ = np.histogramdd(f, bins=e)
        want = h[f"{src}_joint"].astype(np.float64)
        want *= n / want.sum()
        big = want > 2000
        assert np.all(np.abs(got[big] - want[big]) <= 5 * np.sqrt(want[big])), src
        assert got[want == 0].sum() <= 1e-4 * n, src   # only round-off of exp and log at bin edges
        m = ul / cl
        assert np.all((m >= h["edges_m"][0]) & (m <= h["edges_m"][-1]))
        assert int(h[f"{src}_problems"]) > 10 ** 5


def test_riemann_tails_reach_the_stated_extremes():
    g = 5.0 / 3.0
    t = configs.riemann_tails(20000, g, np.random.default_rng(3))
    rl, ul, pl, rr, ur, pr = t
    h = t.shape[1] // 2
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    frac = (ur - ul) / (2 * (cl + cr) / (g - 1))          # share of the vacuum threshold
    assert np.all((frac[:h] >= 0.8) & (frac[:h] < 1.0))
    ratio = np.maximum(pl[h:] / pr[h:], pr[h:] / pl[h:])
    assert ratio.min() >= 1e2 * (1 - 1e-12) and ratio.max() <= 1e6 * (1 + 1e-12)
    assert ratio.max() > 1e5                                # the range is covered
    assert np.all(ur[h:] <= ul[h:])                         # colliding flows
