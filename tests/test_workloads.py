"""Checks of the synthetic workload generators (no method arithmetic)."""
import numpy as np

from paper_2504_08157_amd import workloads as W


def test_vortex_profile_peak():
    # Eq. (initial-velocity): Gaussian vorticity gives V(r) = zeta0 L^2 (1 - e^{-r^2/L^2})/(2r).
    r = np.linspace(1.0, 300e3, 300001)
    V = W.vortex_profile(r, vmax=20.0, rmax=50e3)
    i = np.argmax(V)
    assert abs(r[i] - 50e3) < 200.0 and abs(V[i] - 20.0) < 0.01
    # the paper's peak vorticity 1.5e-3 1/s at r_max = 50 km integrates to ~21.4 m/s
    # (printed as 21.5 m/s in Sec. 4.1)
    L = 50e3 / 1.120906
    v = 1.5e-3 * L * L * (1 - np.exp(-r * r / L / L)) / (2 * r)
    assert abs(v.max() - 21.5) < 0.2


def test_reference_profiles_hydrostatic():
    z = np.linspace(0, 20e3, 2001)
    for rho0, th0, ex in ((*W.constant_n_reference(z), W.exner_constant_n(z)),
                          (*W.isentropic_reference(z), W.exner_isentropic(z))):
        p0 = W.PA * ex ** (W.CP / W.RD)
        dp = np.gradient(p0, z)
        np.testing.assert_allclose(dp[5:-5], -rho0[5:-5] * W.G, rtol=1e-5)
        # equation of state consistency p0 = p_a (rho0 R theta0 / p_a)^gamma
        np.testing.assert_allclose(p0, W.PA * (rho0 * W.RD * th0 / W.PA) ** (W.CP / W.CV), rtol=1e-13)


def test_heating_bursts_bounded_and_seeded():
    x = np.linspace(-100e3, 100e3, 81); z = np.linspace(0, 20e3, 21)
    s1 = W.burst_schedule(seed=2); s2 = W.burst_schedule(seed=2)
    np.testing.assert_array_equal(s1.tb, s2.tb)
    t, Q = W.heating_snapshots(x, x, z, 3600.0, s1)
    assert Q.shape == (11, 21, 81, 81) and t[-1] == 3600.0
    assert Q.min() >= 0 and Q.max() <= 12 * 10 / 3600.0
    assert np.all(Q[:, z >= 15e3] == 0)


def test_ensemble_members():
    sizes = [W.cfg_ensemble_member(i).mesh for i in range(48)]
    assert sizes[0].nel == (8, 8, 8) and sizes[1].nel == (40, 40, 16)
    assert all(m.order in (3, 4, 5) for m in sizes)
    assert all(8 <= m.nel[0] <= 40 and 8 <= m.nel[2] <= 16 for m in sizes)
