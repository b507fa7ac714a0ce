"""The seeded input generators (CPU): determinism, shapes and the physical
structure each stand-in claims (no step of the scheme is checked here)."""
import numpy as np

from paper_0901_4107_amd.inputs import configs


def test_riemann_problems_seeded_and_valid():
    a = configs.riemann_problems(n=4096, side=12, nthreads=4)
    b = configs.riemann_problems(n=4096, side=12, nthreads=4)
    assert a.shape == (6, 4096)
    assert np.array_equal(a, b)
    assert np.all(np.isfinite(a))
    assert np.all(a[[0, 3]] > 0) and np.all(a[[2, 5]] > 0)
    c = configs.riemann_problems(n=4096, side=12, seed=5, nthreads=4)
    assert not np.array_equal(a, c)


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


def test_blast_shell_jump_conditions():
    """Just inside the shock the stand-in's state is the strong-shock
    post-shock state: mass and momentum fluxes through the moving shock
    balance (Rankine-Hugoniot), and the density jump is (g+1)/(g-1)."""
    g = 5.0 / 3.0
    wl = configs.sedov3d(n_side=24, nthreads=4)
    rho, vel, P = configs.blast_shell_states(wl.mesh, g, r_shock=0.2)
    d = wl.mesh.positions - 0.5
    r = np.sqrt(np.sum(d * d, axis=1))
    inside = r < 0.2
    assert np.all(P[~inside] == 1e-5) and np.all(rho[~inside] == 1.0)
    assert np.all(vel[:, ~inside] == 0.0)
    # radial velocity, outward, growing with r inside
    vr = np.sum(vel * (d / r[:, None]).T, axis=0)
    assert np.all(vr[inside] >= 0)
    # extrapolate the interior profile to x = 1: the post-shock state
    xi0, E, rho0 = 1.15, 1.0, 1.0
    t = (0.2 / xi0) ** 2.5 * np.sqrt(rho0 / E)
    vs = 0.4 * 0.2 / t
    edge = inside & (r > 0.19)
    x = r[edge] / 0.2
    rho2 = np.max(rho[edge] / x ** (3 / (g - 1)))
    v2 = np.max(vr[edge] / x)
    p2 = np.max(P[edge] / (0.3 + 0.7 * x ** 5))
    assert abs(rho2 / rho0 - (g + 1) / (g - 1)) < 1e-12
    assert abs(rho0 * vs - rho2 * (vs - v2)) <= 1e-12 * rho0 * vs            # mass
    assert abs((p2 - 1e-5) - rho0 * vs * v2) <= 1e-4 * p2                     # momentum (strong shock)
