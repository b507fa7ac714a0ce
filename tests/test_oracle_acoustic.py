"""Pin of the oracle's order of accuracy: the one-dimensional sound wave of
Section 8.1 (relative amplitude 1e-6, P = 3/5, gamma = 5/3, so that the
sound speed is 1), travelling once through the periodic box on a fixed
Cartesian mesh. The exact solution after one crossing is the initial
state; the paper finds the L1 error falling as N^-2, where a first-order
scheme's would fall as N^-1."""
import numpy as np

from oracle import oracle as O
from paper_0901_4107_amd.inputs.configs import conserved_from_primitive
from tests.test_oracle_entropy import lattice_2d

GAMMA = 5.0 / 3.0
AMP = 1e-6


def wave(x, t):
    """Right-moving linear sound wave: drho = dP / c^2 = rho0 dv / c, c = 1."""
    s = AMP * np.sin(2 * np.pi * (x - t))
    return 1.0 + s, s, 0.6 + s


def crossing(nx, step=None):
    """L1 density error after one crossing (t = 1) on an nx x nx lattice;
    `step(mesh, Q, dt)` advances one step (the oracle's by default)."""
    mesh, x, _ = lattice_2d(nx)
    n = mesh.n_cells
    rho, vx, P = wave(x, 0.0)
    Q = conserved_from_primitive(mesh.volume, rho, np.stack([vx, np.zeros(n)]), P, GAMMA)
    t = 0.0
    while t < 1.0 - 1e-14:
        dt = min(O.cfl_dt(mesh, GAMMA, 0.4, O.prim(2, GAMMA, mesh.volume, Q)), 1.0 - t)
        Q = O.hydro_step(mesh, GAMMA, 0.4, Q, dt=dt)[0] if step is None else step(mesh, Q, dt)
        t += dt
    W = O.prim(2, GAMMA, mesh.volume, Q)
    return float(np.mean(np.abs(W[0] - wave(x, 1.0)[0]))), mesh, Q


def test_sound_wave_converges_at_second_order():
    """L1 on 16^2, 32^2, 64^2: about 4.7e-8, 1.4e-8, 3.5e-9 (falling 3.4x
    and 3.9x, approaching the factor 4 of second order), far above the
    round-off of the unit density."""
    l1 = [crossing(nx)[0] for nx in (16, 32, 64)]
    assert l1[0] < 1e-7
    assert l1[0] / l1[1] > 3.2 and l1[1] / l1[2] > 3.7, l1
