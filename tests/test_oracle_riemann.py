"""Pins of the oracle's exact Riemann solver against facts fixed outside it:
textbook and paper values, closed forms of special wave patterns, the
Rankine-Hugoniot conditions and the isentropic fan relations checked on the
whole self-similar solution, and symmetries of the Euler equations."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def solve(g, L, R):
    r = O.riemann(g, L[0], L[1], L[2], R[0], R[1], R[2])
    return {k: v[0] for k, v in r.items()}


def sample_at(g, L, R, S):
    """The self-similar solution at x/t = S: solve the problem seen from a
    frame moving with speed S (the exact Riemann solution is Galilean
    invariant) and shift the sampled velocity back."""
    r = solve(g, (L[0], L[1] - S, L[2]), (R[0], R[1] - S, R[2]))
    return r["rho"], r["u"] + S, r["P"]


def sample_many(g, L, R, S):
    r = O.riemann(g, L[0], L[1] - S, L[2], R[0], R[1] - S, R[2])
    return r["rho"], r["u"] + S, r["P"]


def test_golden_star_states():
    """Published star states (Sod's problem; the paper's shock tube)."""
    with open(os.path.join(GOLD, "riemann_star.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        r = solve(c["gamma"], c["L"], c["R"])
        for key in ("pstar", "ustar", "rho_star_L", "rho_star_R"):
            if key not in c:
                continue
            if key == "rho_star_L":
                val = sample_at(c["gamma"], c["L"], c["R"], r["ustar"] - 1e-9)[0]
            elif key == "rho_star_R":
                val = sample_at(c["gamma"], c["L"], c["R"], r["ustar"] + 1e-9)[0]
            else:
                val = r[key]
            assert abs(val - c[key]) <= 0.5 * 10.0 ** (-c["digits"]) + 1e-12, (c["name"], key, val)


def test_paper_shock_tube_mach():
    """Section 8.2: rho,P = 1,1 | 0.25,0.1795, gamma 1.4 gives a shock of Mach
    number 1.48 running into the right state; the post-shock density jump
    must match the paper's f_rho(M) = (g+1) M^2 / ((g-1) M^2 + 2)."""
    g = 1.4
    L, R = (1.0, 0.0, 1.0), (0.25, 0.0, 0.1795)
    r = solve(g, L, R)
    cR = np.sqrt(g * R[2] / R[0])
    # locate the shock by scanning the sampled density to the right of u*
    S = np.linspace(r["ustar"] + 1e-6, 3.0, 300001)
    rho = sample_many(g, L, R, S)[0]
    jump = np.argmax(np.abs(np.diff(rho)))
    S_shock = 0.5 * (S[jump] + S[jump + 1])
    mach = (S_shock - R[1]) / cR
    assert round(mach, 2) == 1.48
    rho2 = sample_at(g, L, R, r["ustar"] + 1e-6)[0]
    # refine the Mach number from the density jump itself (no solver formula)
    f_rho = rho2 / R[0]
    M2 = 2.0 * f_rho / ((g + 1.0) - (g - 1.0) * f_rho)
    assert abs(np.sqrt(M2) - mach) < 2e-3


def test_equal_states():
    for g in (1.4, 5.0 / 3.0):
        for (rho, u, P) in [(1.0, 0.0, 1.0), (0.3, -2.0, 7.0), (1e-2, 5.0, 1e2)]:
            r = solve(g, (rho, u, P), (rho, u, P))
            assert abs(r["pstar"] - P) <= 1e-14 * P
            assert abs(r["ustar"] - u) <= 1e-14 * (abs(u) + np.sqrt(g * P / rho))


def test_two_rarefaction_closed_form():
    """When both waves are rarefactions the star pressure has the closed form
    p* = [(cL + cR - (g-1)/2 (uR-uL)) / (cL PL^-z + cR PR^-z)]^(1/z),
    z = (g-1)/(2g), from the two isentropic Riemann invariants."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        g = rng.choice([1.4, 5.0 / 3.0])
        rhoL, rhoR = 10 ** rng.uniform(-2, 2, 2)
        PL, PR = 10 ** rng.uniform(-2, 2, 2)
        cL, cR = np.sqrt(g * PL / rhoL), np.sqrt(g * PR / rhoR)
        z = (g - 1) / (2 * g)
        vmax = 2 * (cL + cR) / (g - 1)
        du = rng.uniform(0.0, 0.95) * vmax
        uL = rng.normal()
        p_tr = ((cL + cR - 0.5 * (g - 1) * du) / (cL / PL ** z + cR / PR ** z)) ** (1 / z)
        if p_tr > min(PL, PR):
            continue  # not a two-rarefaction pattern
        r = solve(g, (rhoL, uL, PL), (rhoR, uL + du, PR))
        assert abs(r["pstar"] - p_tr) <= 1e-12 * p_tr


def test_symmetric_two_shock_closed_form():
    """Identical states colliding at +-U: both waves are shocks of equal
    strength, u* = 0, and p* solves (p-P)^2 A = U^2 (p+B) with
    A = 2/((g+1) rho), B = (g-1)/(g+1) P (Rankine-Hugoniot)."""
    for g in (1.4, 5.0 / 3.0):
        for (rho, P, U) in [(1.0, 1.0, 1.0), (0.1, 3.0, 20.0), (50.0, 0.01, 0.5)]:
            A = 2 / ((g + 1) * rho)
            B = (g - 1) / (g + 1) * P
            # A p^2 - (2 A P + U^2) p + (A P^2 - U^2 B) = 0, larger root
            a, b, c = A, -(2 * A * P + U * U), A * P * P - U * U * B
            p = (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)
            r = solve(g, (rho, U, P), (rho, -U, P))
            assert abs(r["pstar"] - p) <= 1e-12 * p
            assert abs(r["ustar"]) <= 1e-12 * U


def _conserved(g, rho, u, P):
    return np.array([rho, rho * u, P / (g - 1) + 0.5 * rho * u * u])


def _flux(g, rho, u, P):
    E = P / (g - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + P, (E + P) * u])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_whole_solution_conservation_laws(seed):
    """Sample the full self-similar solution and check it against the Euler
    equations themselves: across every jump the Rankine-Hugoniot conditions
    F(U+) - F(U-) = S (U+ - U-) hold; inside fans the entropy P/rho^g and the
    Riemann invariant are constant; at the contact u and P are continuous."""
    rng = np.random.default_rng(seed)
    g = 5.0 / 3.0
    checked_shocks = 0
    for _ in range(40):
        rhoL, rhoR = 10 ** rng.uniform(-2, 2, 2)
        PL, PR = 10 ** rng.uniform(-2, 2, 2)
        cL, cR = np.sqrt(g * PL / rhoL), np.sqrt(g * PR / rhoR)
        uL, uR = rng.normal(0, 1.5 * cL), rng.normal(0, 1.5 * cR)
        if uR - uL >= 2 * (cL + cR) / (g - 1):
            continue
        L, R = (rhoL, uL, PL), (rhoR, uR, PR)
        r = solve(g, L, R)
        smax = 4 * (abs(uL) + abs(uR) + cL + cR)
        S = np.linspace(-smax, smax, 4001)
        rho, u, P = sample_many(g, L, R, S)
        st = np.stack([rho, u, P], axis=1)
        # far field
        assert np.allclose(st[0], L, rtol=1e-12) and np.allclose(st[-1], R, rtol=1e-12)
        # contact: u and P continuous through u*
        a = sample_at(g, L, R, r["ustar"] - 1e-10 * smax)
        b = sample_at(g, L, R, r["ustar"] + 1e-10 * smax)
        assert abs(a[1] - b[1]) <= 1e-8 * smax and abs(a[2] - b[2]) <= 1e-8 * max(PL, PR)
        # jumps: any density step larger than the local fan gradient is a shock
        drho = np.abs(np.diff(rho)) / np.maximum(rho[:-1], rho[1:])
        for k in np.where(drho > 0.02)[0]:
            s_mid = 0.5 * (S[k] + S[k + 1])
            if abs(s_mid - r["ustar"]) < 2 * (S[1] - S[0]):
                continue  # the contact
            lo, hi = S[k], S[k + 1]
            for _ in range(60):  # bisect the jump location on the sampled state
                mid = 0.5 * (lo + hi)
                if abs(sample_at(g, L, R, mid)[0] - sample_at(g, L, R, lo)[0]) < 1e-9 * rho[k]:
                    lo = mid
                else:
                    hi = mid
            Um = sample_at(g, L, R, lo)
            Up = sample_at(g, L, R, hi)
            Sshock = 0.5 * (lo + hi)
            lhs = _flux(g, *Up) - _flux(g, *Um)
            rhs = Sshock * (_conserved(g, *Up) - _conserved(g, *Um))
            scale = np.abs(_flux(g, *Up)) + np.abs(_flux(g, *Um)) + abs(Sshock) * np.abs(_conserved(g, *Um))
            assert np.all(np.abs(lhs - rhs) <= 1e-6 * scale + 1e-300), (L, R, lhs, rhs)
            checked_shocks += 1
        # left fan (if the left wave is a rarefaction): entropy and the
        # Riemann invariant u + 2c/(g-1) stay at their left-state values
        if r["pstar"] < PL:
            star_rho = sample_at(g, L, R, r["ustar"] - 1e-9 * smax)[0]
            fan = (S < r["ustar"]) & (np.abs(rho - rhoL) > 1e-9 * rhoL) & (np.abs(rho - star_rho) > 1e-9 * star_rho)
            assert np.any(fan)
            ent = P[fan] / rho[fan] ** g
            inv = u[fan] + 2 * np.sqrt(g * P[fan] / rho[fan]) / (g - 1)
            assert np.allclose(ent, PL / rhoL ** g, rtol=1e-10)
            assert np.allclose(inv, uL + 2 * cL / (g - 1), rtol=1e-10, atol=1e-10 * cL)
    assert checked_shocks > 5


def test_mirror_symmetry():
    """Reflecting x -> -x swaps the states and negates velocities: the sampled
    state at x/t = 0 is mirrored and comes from the other side."""
    rng = np.random.default_rng(11)
    g = 5.0 / 3.0
    n = 2000
    rhoL, rhoR, PL, PR = (10 ** rng.uniform(-2, 2, n) for _ in range(4))
    uL, uR = rng.normal(0, 3, n), rng.normal(0, 3, n)
    a = O.riemann(g, rhoL, uL, PL, rhoR, uR, PR)
    b = O.riemann(g, rhoR, -uR, PR, rhoL, -uL, PL)
    ok = a["ustar"] != 0.0
    assert np.allclose(a["rho"][ok], b["rho"][ok], rtol=1e-12, atol=0)
    assert np.allclose(a["P"][ok], b["P"][ok], rtol=1e-12, atol=0)
    assert np.allclose(a["u"][ok], -b["u"][ok], rtol=1e-12, atol=1e-12 * np.abs(a["u"][ok]).max())
    both = ok & (a["case"] == 0)
    assert np.all(a["side"][both] + b["side"][both] == 1)


def test_root_is_root_and_guess_independent():
    """p* is a zero of the pressure function (checked by an independent
    bisection that never calls the solver's loop) to round-off."""
    rng = np.random.default_rng(5)
    g = 1.4
    for _ in range(100):
        L = (10 ** rng.uniform(-2, 2), rng.normal(0, 2), 10 ** rng.uniform(-2, 2))
        R = (10 ** rng.uniform(-2, 2), rng.normal(0, 2), 10 ** rng.uniform(-2, 2))
        cL, cR = np.sqrt(g * L[2] / L[0]), np.sqrt(g * R[2] / R[0])
        if R[1] - L[1] >= 2 * (cL + cR) / (g - 1):
            continue
        r = solve(g, L, R)
        lo, hi = 0.0, max(L[2], R[2])
        while O.pressure_function(g, L, R, hi) <= 0:
            hi *= 2
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid == lo or mid == hi:
                break
            if O.pressure_function(g, L, R, mid) < 0:
                lo = mid
            else:
                hi = mid
        assert abs(r["pstar"] - 0.5 * (lo + hi)) <= 1e-13 * r["pstar"]


def test_vacuum_cases():
    g = 1.4
    # generated vacuum: u_R - u_L >= 2 (cL + cR)/(g-1)
    L, R = (1.0, -10.0, 1.0), (1.0, 10.0, 1.0)
    r = solve(g, L, R)
    assert r["case"] == 3 and r["rho"] == 0.0 and r["P"] == 0.0
    # just below the threshold: tiny but positive star pressure
    c = np.sqrt(g)
    du = 0.999 * 2 * (2 * c) / (g - 1)
    r = solve(g, (1.0, -du / 2, 1.0), (1.0, du / 2, 1.0))
    assert r["case"] == 0 and 0 < r["pstar"] < 1e-3
    # vacuum on one side: state at the face follows the fan; rho -> 0 at front
    r = solve(g, (0.0, 0.0, 0.0), (1.0, 0.0, 1.0))
    assert r["case"] == 1 and r["side"] == 1
    # sample at the right state's vacuum front: density vanishes
    front = 0.0 - 2 * c / (g - 1)
    assert sample_at(g, (0.0, 0.0, 0.0), (1.0, 0.0, 1.0), front + 1e-12)[0] < 1e-12
    r = solve(g, (1.0, 0.0, 1.0), (0.0, 0.0, 0.0))
    assert r["case"] == 2 and r["side"] == 0
    r = solve(g, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    assert r["case"] == 4 and r["rho"] == 0.0


def test_galilean_invariance_of_star_state():
    """The exact Riemann solution is Galilean invariant: a common boost shifts
    u* and leaves p* unchanged (the sampling at x/t=0 is what is not
    invariant, which is why the scheme samples in the face frame)."""
    rng = np.random.default_rng(3)
    g = 5.0 / 3.0
    n = 500
    rhoL, rhoR, PL, PR = (10 ** rng.uniform(-2, 2, n) for _ in range(4))
    uL, uR = rng.normal(0, 2, n), rng.normal(0, 2, n)
    v = 37.0
    a = O.riemann(g, rhoL, uL, PL, rhoR, uR, PR)
    b = O.riemann(g, rhoL, uL + v, PL, rhoR, uR + v, PR)
    ok = a["case"] == 0
    assert np.allclose(a["pstar"][ok], b["pstar"][ok], rtol=1e-10)
    assert np.allclose(a["ustar"][ok] + v, b["ustar"][ok], rtol=1e-12, atol=1e-10 * v)
