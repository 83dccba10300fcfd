"""Pins of the oracle's NPT integrator (eq. Langevin_NPT, diagonal h) against
what the mathematics fixes: the exact flow of the drift, the moments of the
Ornstein-Uhlenbeck step, free flight, the second order of the splitting and
equipartition of the kinetic pressure."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as orc


def _zero_forces(n):
    return lambda pos, L, step: (np.zeros((n, 3)), np.zeros((3, 3)))


def test_drift_is_the_exact_flow_of_its_equations():
    rng = np.random.default_rng(3)
    n = 5
    pos = rng.uniform(0, 20, (n, 3)); mom = rng.normal(size=(n, 3)); mass = rng.uniform(1, 16, n)
    L = np.array([20.0, 22.0, 25.0]); ph = np.array([3.0, -2.0, 5.0]); M = 7.0; t = 0.8
    groups = orc.COUPLINGS[0]

    def rhs(_, y):
        Lt = y[:3]; r = y[3:3 + 3 * n].reshape(n, 3); p = y[3 + 3 * n:].reshape(n, 3)
        Ld = ph / M
        return np.concatenate([Ld, (p / mass[:, None] + Ld / Lt * r).ravel(), (-(Ld / Lt) * p).ravel()])

    y0 = np.concatenate([L, pos.ravel(), mom.ravel()])
    sol = solve_ivp(rhs, (0, t), y0, rtol=1e-12, atol=1e-12)
    ref = sol.y[:, -1]
    p2, m2, L2 = pos.copy(), mom.copy(), L.copy()
    orc.npt_drift(p2, m2, mass, L2, ph.copy(), groups, M, t)
    assert np.allclose(L2, ref[:3], rtol=1e-10)
    assert np.allclose(p2.ravel(), ref[3:3 + 3 * n], rtol=1e-9, atol=1e-9)
    assert np.allclose(m2.ravel(), ref[3 + 3 * n:], rtol=1e-9, atol=1e-9)


def test_coupled_axes_keep_equal_lengths():
    pos = np.zeros((1, 3)); mom = np.zeros((1, 3)); mass = np.ones(1)
    L = np.array([30.0, 30.0, 40.0]); ph = np.array([4.0, 1.0])
    orc.npt_drift(pos, mom, mass, L, ph, orc.COUPLINGS[1], 2.0, 0.5)
    assert L[0] == L[1] == 30.0 + 0.5 * 4.0 / (2 * 2.0) and L[2] == 40.0 + 0.5 * 1.0 / 2.0


def test_ou_step_moments_and_noise_normals():
    n = 200_000
    z, zb = orc.npt_normals(9, 1, 17, n)
    assert abs(z.mean()) < 5e-3 and abs(z.var() - 1.0) < 5e-3
    rng = np.random.default_rng(1)
    mass = rng.uniform(1, 30, n); mom = rng.normal(size=(n, 3)) * np.sqrt(mass)[:, None]
    kT, c1 = 2.5, np.exp(-0.3)
    before = (mom ** 2 / mass[:, None]).mean()
    m2 = mom.copy()
    orc.npt_ou(m2, mass, np.zeros(3), orc.COUPLINGS[0], 1.0, kT, c1, 1.0, z, zb)
    after = (m2 ** 2 / mass[:, None]).mean()
    expect = c1 * c1 * before + (1 - c1 * c1) * kT
    assert abs(after / expect - 1) < 1e-2
    # no noise: pure damping
    m3 = mom.copy()
    orc.npt_ou(m3, mass, np.zeros(3), orc.COUPLINGS[0], 1.0, 0.0, c1, 1.0, z, zb)
    assert np.allclose(m3, c1 * mom, rtol=1e-15)


def test_free_flight_with_a_frozen_box():
    rng = np.random.default_rng(5)
    n = 50
    pos = rng.uniform(0, 30, (n, 3)); mom = rng.normal(size=(n, 3)); mass = rng.uniform(1, 16, n)
    prm = dict(dt=0.01, kT=0.0, gamma=0.0, gamma_box=0.0, box_mass=1e300, p_ext=0.0, coupling=0)
    out = orc.npt_run(np.zeros(n), pos, mom, mass, [30.0, 30.0, 30.0], np.zeros(3), prm, None, 0, 0, 0, 0, 20,
                      evaluate=_zero_forces(n))
    assert np.allclose(out[0], pos + 20 * 0.01 * mom / mass[:, None], rtol=1e-13, atol=1e-13)
    assert np.array_equal(out[1], mom)


def test_splitting_is_second_order():
    """Harmonic forces, frozen box, no friction: velocity Verlet, energy error
    of order dt^2."""
    rng = np.random.default_rng(2)
    n = 8
    k = rng.uniform(0.5, 2.0, n)
    pos0 = rng.normal(size=(n, 3)); mom0 = rng.normal(size=(n, 3)); mass = rng.uniform(1, 4, n)

    def energy(x, p):
        return 0.5 * (k[:, None] * x * x).sum() + 0.5 * (p * p / mass[:, None]).sum()

    ev = lambda x, L, step: (-k[:, None] * x, np.zeros((3, 3)))
    errs = []
    for dt in (0.02, 0.01):
        prm = dict(dt=dt, kT=0.0, gamma=0.0, gamma_box=0.0, box_mass=1e300, p_ext=0.0, coupling=0)
        out = orc.npt_run(np.zeros(n), pos0, mom0, mass, [50.0, 50.0, 50.0], np.zeros(3), prm, None, 0, 0, 0, 0,
                          int(round(2.0 / dt)), evaluate=ev)
        errs.append(abs(energy(out[0], out[1]) - energy(pos0, mom0)))
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.0, ratio


def test_kinetic_pressure_reaches_equipartition():
    """Free particles under the Langevin thermostat: <P_kin,mumu> = N kT / V."""
    rng = np.random.default_rng(4)
    n = 4000
    mass = rng.uniform(1, 16, n)
    kT = 1.7
    L = np.array([40.0, 40.0, 40.0])
    prm = dict(dt=0.1, kT=kT, gamma=5.0, gamma_box=0.0, box_mass=1e300, p_ext=0.0, coupling=2)
    pos = rng.uniform(0, 40, (n, 3)); mom = np.zeros((n, 3))
    acc = []
    for blk in range(20):
        pos, mom, L2, _, Pi, Pk = orc.npt_run(np.zeros(n), pos, mom, mass, L, np.zeros(3), prm, None, 0, 6, 0, 10 * blk,
                                             10, evaluate=_zero_forces(n))
        if blk >= 2:
            acc.append(np.diag(Pk))
    got = np.mean(acc)
    assert abs(got / (n * kT / np.prod(L)) - 1) < 0.02
