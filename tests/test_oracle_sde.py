"""Pins for the oracle's particle SDEs against closed forms of the explicit
Euler-Maruyama scheme.

* Ornstein-Uhlenbeck limit of the Langevin equation (frozen statistics):
  stationary variance C0 eps / (-2G - G^2 dt) per component.
* Decaying homogeneous turbulence under the simplified Langevin model, which
  satisfies the energy constraint eq:constraint-on-c0:
  k_n = k_0 (1 - <omega> dt + G^2 dt^2)^n.
* Stationary frequency of eq:frequency-model with frozen <omega> = Omega and
  S_omega = 0: mean Omega, variance C4 Omega^2 / (1 - C3 Omega dt / 2),
  distribution close to Gamma(1/C4, C4 Omega).
* IEM (eq:IEM) with a frozen mean: every particle relaxes as
  psi_n - <phi> = (1 - dt C_phi <omega>/2)^n (psi_0 - <phi>).
* Generalized Langevin model in isotropic frozen turbulence with the local
  elliptic-relaxation right-hand side: G = -(C1/2)<omega>, C0 = 2(C1-1)/3.
* No-slip trajectory (b) (eq:fw): the probability of the wall condition.
"""
import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _frozen(mesh, ppe, U=(0, 0, 0), R_diag=(2 / 3,) * 3, Om=1.0, Phi=0.5, seed=0, psi_mode=0,
            init_var=0.01, **pk):
    o = O.Oracle(mesh, CF.params(frozen=1, **pk))
    U0, R0, Om0 = CF._iso(mesh.n_nodes, U, init_var, Om)
    o.seed(dict(ppe=ppe, seed=seed, psi_mode=psi_mode, U0=U0, R0=R0, Om0=Om0))
    o.set_stats(CF.frozen_stats_for(mesh, U=U, R_diag=R_diag, Om=Om, Phi=Phi))
    return o


def _velocity_var(o):
    return o.state[2:5].var(axis=1)


def test_ou_stationary_variance_slm():
    mesh = M.periodic_square(8)
    dt = 0.01
    o = _frozen(mesh, 200, U=(1.0, 0.0, 0.0), C0=2.1, C3=1.0)
    G = -(0.5 + 0.75 * 2.1)
    expect = 2.1 * 1.0 / (-2 * G - G * G * dt)
    assert abs(expect - 0.511329) < 1e-6
    snaps = []
    for n in range(450):
        o.step(dt)
        if n >= 200 and n % 50 == 0:
            snaps.append(_velocity_var(o))
    v = np.mean(snaps)
    # ~1.3e5 particles x 3 components x 5 weakly correlated snapshots
    assert abs(v - expect) / expect < 0.006
    assert abs(v - 2.1 / 4.15) / (2.1 / 4.15) > 0.004  # resolves the O(dt) discrete bias


def test_glm_isotropic_local_wp_closed_form():
    mesh = M.periodic_square(8)
    dt = 0.01
    o = _frozen(mesh, 200, model=CF.MODEL_GLM, wp_source=CF.WP_LOCAL, omega_source=0, C3=1.0,
                init_var=0.3)
    C1 = CF.PAPER_CONSTANTS["C1"]
    G = -0.5 * C1
    C0 = 2.0 * (C1 - 1.0) / 3.0
    # energy constraint eq:constraint-on-c0 holds: (1 + 1.5 C0) eps + G_ij R_ij = 0
    assert abs((1 + 1.5 * C0) * 1.0 + G * 2.0) < 1e-14
    expect = C0 * 1.0 / (-2 * G - G * G * dt)
    snaps = []
    for n in range(400):
        o.step(dt)
        if n >= 200 and n % 40 == 0:
            snaps.append(_velocity_var(o))
    v = np.mean(snaps)
    assert abs(v - expect) / expect < 0.008


def test_decaying_turbulence_energy():
    """Unfrozen run of the periodic-square workload (SLM, S_omega = 0): the
    kinetic energy decays as (1 - <omega> dt + G^2 dt^2)^n."""
    w = CF.periodic_square(n=16, ppe=200, steps=100, var=0.01)
    o = O.Oracle(w.mesh, w.params)
    o.seed(w.seed)
    k0 = 0.5 * o.state[2:5].var(axis=1).sum()
    for _ in range(100):
        o.step(w.dt)
    k100 = 0.5 * o.state[2:5].var(axis=1).sum()
    om = o.stats[3].mean()
    G = -(0.5 + 0.75 * 2.1) * om
    expect = (1.0 - om * w.dt + G * G * w.dt ** 2) ** 100
    assert abs(expect - 0.382299) < 2e-3
    # finite particle number: relative bias O(1 / particles per node support)
    assert abs(k100 / k0 - expect) / expect < 0.03


def test_frequency_stationary_gamma():
    mesh = M.periodic_square(8)
    dt, C3, C4 = 0.01, 1.0, 0.25
    o = _frozen(mesh, 200, Om=1.0, C3=C3, C4=C4, omega_source=0)
    snaps_m, snaps_v = [], []
    for n in range(500):
        o.step(dt)
        if n >= 300 and n % 40 == 0:
            snaps_m.append(o.state[5].mean())
            snaps_v.append(o.state[5].var())
    expect_v = C4 / (1.0 - C3 * dt / 2.0)
    assert abs(expect_v - 0.251256) < 1e-6
    assert abs(np.mean(snaps_m) - 1.0) < 0.004
    assert abs(np.mean(snaps_v) - expect_v) / expect_v < 0.012
    assert stats.kstest(o.state[5, :5000], stats.gamma(1 / C4, scale=C4).cdf).pvalue > 1e-3


def test_iem_exact_relaxation_with_frozen_mean():
    mesh = M.periodic_square(8)
    dt, Cphi, Om, Phi = 0.01, 2.0, 1.0, 0.5
    o = _frozen(mesh, 50, Om=Om, Phi=Phi, psi_mode=CF.PSI_BERNOULLI, Cphi=Cphi)
    psi0 = o.state[6].copy()
    v0 = psi0.var()
    for _ in range(100):
        o.step(dt)
    r = (1.0 - dt * 0.5 * Cphi * Om) ** 100
    assert np.abs(o.state[6] - (Phi + r * (psi0 - Phi))).max() < 1e-13
    assert abs(o.state[6].var() / v0 - 0.99 ** 200) < 1e-12
    assert abs(0.99 ** 200 - 0.133980) < 1e-6


@pytest.mark.parametrize("d0", [0.002, 0.005])
def test_noslip_trajectory_b_probability(d0):
    """Particles at rest at distance d0 from a flat no-slip wall with nu > 0:
    after one step, the wall condition of trajectory (b) is applied with
    probability E[exp(-d0 d1 / (nu dt)); d1 >= 0], d1 = d0 + sqrt(2 nu dt) xi."""
    mesh = M.graded_channel(8, 6, 6.0, 1.0, 0.0, 0)
    nu, dt = 1e-3, 1e-2
    o = O.Oracle(mesh, CF.params(frozen=1, nu=nu, wall_b=1))
    U0, R0, Om0 = CF._iso(mesh.n_nodes)
    o.seed(dict(ppe=1, seed=9, psi_mode=0, U0=U0, R0=R0, Om0=Om0))
    o.set_stats(CF.frozen_stats_for(mesh, U=(0, 0, 0), R_diag=(0, 0, 0), Om=1.0))
    n = 40000
    rng = np.random.default_rng(3)
    x = rng.uniform(0.5, 5.5, n)
    om = O.OracleMesh(mesh)
    e = np.array([om.locate_brute(a, d0) for a in x])
    o.state = np.zeros((7, n))
    o.state[0], o.state[1], o.state[5] = x, d0, 1.0
    o.elem = e.astype(np.int32)
    o.id = np.arange(n, dtype=np.uint32)
    o.step(dt)
    s = np.sqrt(2 * nu * dt)
    p_b = integrate.quad(lambda z: np.exp(-d0 * (d0 + s * z) / (nu * dt)) * stats.norm.pdf(z),
                         -d0 / s, np.inf)[0]
    p_a = stats.norm.cdf(-d0 / s)
    cnt = o.counter_dict()
    # trajectory (a): behind the wall after the move -> reflected
    assert abs(cnt["reflect"] / n - p_a) < 5 * np.sqrt(p_a / n) + 1e-3
    assert abs(cnt["noslip_b"] / n - p_b) < 5 * np.sqrt(p_b / n)
    # every wall condition zeroes the velocity; all other particles received
    # the nonzero noise sqrt(C0 eps) dW' (eps > 0 through the nu C_T^2 <omega> term)
    hit = (o.state[2] == 0) & (o.state[3] == 0) & (o.state[4] == 0)
    assert hit.sum() == cnt["reflect"] + cnt["noslip_b"]
