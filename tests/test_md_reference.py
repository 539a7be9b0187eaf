"""Pins of the MD reference helpers (tests/md_reference.py) on the CPU, so
that the GPU trajectory tests compare against integrators that are checked
on their own: the short-range forces against plain pair loops and finite
differences, the virial against the volume-scaling derivative, and the
integrators against their defining properties (RESPA with one inner step is
velocity Verlet; a thermostat of infinite mass does nothing; reversibility;
second-order energy error; the Nose-Hoover extended energy).  The long-range
forces are a smooth periodic stand-in here (no oracle needed)."""
import numpy as np
import pytest

from md_reference import (K6, cpu_nose_hoover, cpu_respa, cpu_verlet, lattice_system, lj_numpy, nh_half,
                          rdf_numpy)


def stand_in(box, amp=0.5):
    """Smooth periodic external potential U = amp sum_i sum_k cos(2 pi x_ik /
    L_k) and its forces: plays the role of the Coulomb part."""
    w = 2 * np.pi / box

    def f(x):
        return amp * w * np.sin(w * x), amp * np.cos(w * x).sum()
    return f


def lj_loops(x, box, slab, eps=1.0, sig=1.0, weps=0.0, wsig=1.0):
    """WCA pairs and walls by the definition, one pair at a time."""
    n = len(x)
    rc = K6 * sig
    f = np.zeros_like(x)
    e = w = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            d = x[i] - x[j]
            for k in range(2 if slab else 3):
                d[k] -= box[k] * round(d[k] / box[k])
            r = float(np.sqrt(d @ d))
            if r >= rc:
                continue
            u = 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6) + eps
            fr = 24 * eps * (2 * (sig / r) ** 12 - (sig / r) ** 6) / r  # -dU/dr
            f[i] += fr * d / r
            f[j] -= fr * d / r
            e += u
            w += fr * r
    if slab and weps > 0:
        for i in range(n):
            for dist, sgn in ((x[i, 2], 1.0), (box[2] - x[i, 2], -1.0)):
                if dist >= K6 * wsig:
                    continue
                e += 4 * weps * ((wsig / dist) ** 12 - (wsig / dist) ** 6) + weps
                f[i, 2] += sgn * 24 * weps * (2 * (wsig / dist) ** 12 - (wsig / dist) ** 6) / dist
    return f, e, w


def dense_system(seed, slab=False):
    """27 ions in a box of 3.3 (lattice spacing 1.1, below the WCA cut-off
    1.12): every ion in contact with its neighbours, also across the
    periodic boundary; the slab variant sits between walls at 0 and 3.6."""
    box = np.array([3.3, 3.3, 3.6 if slab else 3.3])
    pos, q, v, m = lattice_system((3, 3, 3), box, seed, z_lo=0.15 if slab else 0.0,
                                  z_hi=3.45 if slab else None, jitter=0.05)
    return box, pos, q, v, m


@pytest.mark.parametrize("slab", [False, True])
def test_lj_numpy_matches_pair_loops(slab):
    box, x, _, _, _ = dense_system(1, slab)
    weps, wsig = (1.0, 0.5) if slab else (0.0, 1.0)
    f, e, w = lj_numpy(x, box, slab, weps=weps, wsig=wsig)
    fl, el, wl = lj_loops(x, box, slab, weps=weps, wsig=wsig)
    assert e > 1.0 and np.abs(fl).max() > 1.0  # pairs in contact
    assert np.abs(f - fl).max() <= 1e-12 * np.abs(fl).max()
    assert abs(e - el) <= 1e-12 * abs(el) and abs(w - wl) <= 1e-12 * abs(wl)


@pytest.mark.parametrize("slab", [False, True])
def test_lj_numpy_forces_are_minus_the_gradient(slab):
    box, x, _, _, _ = dense_system(2, slab)
    weps, wsig = (1.0, 0.5) if slab else (0.0, 1.0)
    f, _, _ = lj_numpy(x, box, slab, weps=weps, wsig=wsig)
    h = 1e-6
    g = np.zeros_like(x)
    for i in range(len(x)):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            g[i, k] = (lj_numpy(xp, box, slab, weps=weps, wsig=wsig)[1] -
                       lj_numpy(xm, box, slab, weps=weps, wsig=wsig)[1]) / (2 * h)
    assert np.abs(f + g).max() <= 1e-6 * np.abs(f).max()


def test_lj_numpy_virial_is_the_scaling_derivative():
    """sum over pairs r . F = -d/ds E(s x, s L) at s = 1 (the pair part of
    the pressure virial)."""
    box, x, _, _, _ = dense_system(3)
    _, _, w = lj_numpy(x, box, False)
    h = 1e-6
    ep = lj_numpy(x * (1 + h), box * (1 + h), False)[1]
    em = lj_numpy(x * (1 - h), box * (1 - h), False)[1]
    assert abs(w + (ep - em) / (2 * h)) <= 1e-6 * abs(w)


def test_respa_with_one_inner_step_is_velocity_verlet():
    box, x, q, v, m = dense_system(4)
    lr = stand_in(box)
    xr, vr, rr = cpu_respa(x, v, q, m, box, lr, 0.002, 1, 30)
    xv, vv, rv = cpu_verlet(x, v, q, m, box, lr, 0.002, 30)
    assert np.abs(xr - xv).max() <= 1e-12 and np.abs(vr - vv).max() <= 1e-11
    assert np.abs(rr[:, :3] - rv[:, :3]).max() <= 1e-11 * np.abs(rv[:, :3]).max()
    p = (2 * rv[:, 2] + rv[:, 3] + rv[:, 0]) / (3 * box.prod())
    assert np.abs(rr[:, 3] - p).max() <= 1e-11 * np.abs(p).max()


def test_thermostat_of_infinite_mass_is_velocity_verlet():
    box, x, q, v, m = dense_system(5)
    lr = stand_in(box)
    xn, vn, rn, nh = cpu_nose_hoover(x, v, q, m, box, lr, 0.002, 30, kT=1.5, tau=1e9)
    xv, vv, rv = cpu_verlet(x, v, q, m, box, lr, 0.002, 30)
    assert np.abs(xn - xv).max() <= 1e-12 and np.abs(vn - vv).max() <= 1e-11
    assert np.abs(rn[:, :3] - rv[:, :3]).max() <= 1e-11 * np.abs(rv[:, :3]).max()
    assert np.abs(nh[:, 0]).max() < 1e-15


def test_nose_hoover_half_step_values():
    """One half step from xi = 0 by hand: xi1 = dt/4 G(K), s = exp(-dt/2 xi1),
    eta = dt/2 xi1, xi = xi1 + dt/4 G(K s^2)."""
    K, nf, kT, Q, dt = 30.0, 24, 1.5, 0.6, 0.01
    xi, eta, s = nh_half(0.0, 0.0, K, nf, kT, Q, dt)
    xi1 = 0.25 * dt * (2 * K - nf * kT) / Q
    assert s == pytest.approx(np.exp(-0.5 * dt * xi1), rel=1e-15)
    assert eta == pytest.approx(0.5 * dt * xi1, rel=1e-15)
    assert xi == pytest.approx(xi1 + 0.25 * dt * (2 * K * s * s - nf * kT) / Q, rel=1e-15)
    # hotter than the target: the thermostat removes energy (s < 1)
    assert xi > 0 and s < 1


def test_respa_is_time_reversible():
    """k = 3 inner steps: 20 outer steps forward, velocities reversed, 20
    steps again return to the start (rounding only)."""
    box, x, q, v, m = dense_system(6)
    lr = stand_in(box)
    x1, v1, _ = cpu_respa(x, v, q, m, box, lr, 0.006, 3, 20)
    x2, v2, _ = cpu_respa(x1, -v1, q, m, box, lr, 0.006, 3, 20)
    d = x2 - x
    d -= box * np.rint(d / box)
    assert np.abs(d).max() <= 1e-10 and np.abs(v2 + v).max() <= 1e-9
    assert np.abs(x1 - x).max() > 0.01  # it moved


def energy_fluctuation(run, dt, T):
    nsteps = int(round(T / dt))
    H0, H = run(dt, nsteps)
    return np.sqrt(np.mean((H - H0) ** 2))


@pytest.mark.parametrize("integrator", ["verlet", "respa", "nose_hoover"])
def test_energy_error_is_second_order(integrator):
    """The conserved quantity's fluctuation about its start falls about 4x
    (3x to 6.5x; a first-order error would give 2x) when the step is halved
    over the same time: E_long + E_LJ + E_kin for
    velocity Verlet and RESPA (3 inner steps), plus Q xi^2 / 2 + nf kT eta
    for Nose-Hoover (kT 1.5 from a start at 1, tau 0.1)."""
    box, x, q, v, m = dense_system(7)
    lr = stand_in(box)
    fc, ec = lr(x)
    _, el, _ = lj_numpy(x, box, False)
    H0 = ec + el + 0.5 * (m[:, None] * v * v).sum()

    def run(dt, nsteps):
        if integrator == "verlet":
            _, _, r = cpu_verlet(x, v, q, m, box, lr, dt, nsteps)
            return H0, r[:, 0] + r[:, 1] + r[:, 2]
        if integrator == "respa":
            _, _, r = cpu_respa(x, v, q, m, box, lr, dt, 3, nsteps)
            return H0, r[:, 0] + r[:, 1] + r[:, 2]
        _, _, r, nh = cpu_nose_hoover(x, v, q, m, box, lr, dt, nsteps, kT=1.5, tau=0.1)
        assert np.abs(nh[:, 2]).max() > 1.0  # the thermostat exchanges energy
        return H0, r[:, 0] + r[:, 1] + r[:, 2] + nh[:, 2]

    dt = 0.006 if integrator == "respa" else 0.002
    f1 = energy_fluctuation(run, dt, 0.6)
    f2 = energy_fluctuation(run, dt / 2, 0.6)
    assert 3.0 <= f1 / f2 <= 6.5
    assert f2 <= 1e-3 * abs(H0)


def test_rdf_numpy_matches_pair_loops():
    rng = np.random.default_rng(8)
    box = np.array([5.0, 6.0, 4.5])
    x = rng.uniform(0, 1, (60, 3)) * box
    q = rng.choice([1.0, -1.0, 2.0, 0.0], 60)
    for slab in (False, True):
        nb, rmax = 40, 2.2
        h = rdf_numpy(x, q, box, nb, rmax, slab)
        ref = np.zeros((3, nb), np.int64)
        for i in range(60):
            for j in range(i + 1, 60):
                if q[i] == 0 or q[j] == 0:
                    continue
                d = x[i] - x[j]
                for k in range(2 if slab else 3):
                    d[k] -= box[k] * round(d[k] / box[k])
                r = float(np.sqrt(d @ d))
                if r < rmax:
                    c = 1 if (q[i] > 0) != (q[j] > 0) else (0 if q[i] > 0 else 2)
                    ref[c, min(nb - 1, int(r / (rmax / nb)))] += 1
        assert np.array_equal(h, ref) and ref.sum() > 100
