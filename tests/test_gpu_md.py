"""Molecular dynamics on the GPU (hsma_md_*): velocity-Verlet trajectories
of charged soft spheres against the same integration on the CPU driven by
the FP64 oracle's forces, energy conservation, the slab with walls, and the
pressure virial."""
import sys

import numpy as np
import pytest

from md_reference import (cpu_nose_hoover, cpu_respa, cpu_verlet, lattice_system, lj_numpy,
                          min_image_diff, rdf_numpy)
from oracle import hsma as ohsma

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2104_05260_amd")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", [0, 1])
def test_md_trajectory_matches_cpu_3d(prec):
    """216 ions (+-1 WCA soft spheres, about 100 pairs in contact, Coulomb
    prefactor 2) in a periodic box L = 7, p = 8, dt = 0.002, 25 steps: positions, velocities and the per
    step energies against the CPU integration with the oracle's forces (FP64
    path: 1e-9; FP32C: 1e-5 of the box and the 1e-6 energy bar)."""
    import torch
    box = np.array([7.0, 7.0, 7.0])
    pos, q, v0, m = lattice_system((6, 6, 6), box, 11, jitter=0.05)
    kc = 2.0
    params = hs.Params(precision=prec, p=8, K=162, F=512, lam=1.5, coulomb_k=kc)
    dev = torch.device("cuda:0")
    x = torch.tensor(pos, device=dev)
    v = torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq = torch.tensor(q, device=dev)
    mm = torch.tensor(m, device=dev)
    nsteps, dt = 25, 0.002
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt) as md:
        md.run(x, v, f, qq, mm, nsteps, forces_valid=False, thermo=th)
        torch.cuda.synchronize()
    xg, vg, tg = x.cpu().numpy(), v.cpu().numpy(), th.cpu().numpy()

    def coulomb(xx):
        r = ohsma.hsma3d(xx, q, np.zeros(3), box, 8, 162, 512, 1.5)
        return kc * r.force, kc * r.energy

    xc, vc, rc = cpu_verlet(pos, v0, q, m, box, coulomb, dt, nsteps)
    dx = min_image_diff(xg, xc, box) / box[0]
    dv = np.abs(vg - vc).max() / np.abs(vc).max()
    de = np.abs(tg[:, 0] - rc[:, 0]).max() / np.abs(rc[:, 0]).max()
    dl = np.abs(tg[:, 1] - rc[:, 1]).max() / max(1e-12, np.abs(rc[:, 1]).max())
    dk = np.abs(tg[:, 2] - rc[:, 2]).max() / np.abs(rc[:, 2]).max()
    vol = box.prod()
    p_ref = (2 * rc[:, 2] + rc[:, 3] + rc[:, 0]) / (3 * vol)
    dp = np.abs(tg[:, 3] - p_ref).max() / np.abs(p_ref).max()
    note(f"   prec {prec}: positions {dx:.2e} velocities {dv:.2e}; E_C {de:.2e} E_LJ {dl:.2e} E_kin {dk:.2e} P {dp:.2e}")
    tol = 1e-9 if prec == 0 else 1e-5
    assert dx <= tol and dv <= tol
    assert de <= (1e-10 if prec == 0 else 1e-6) and dk <= tol and dl <= tol and dp <= tol


def test_nose_hoover_trajectory_matches_cpu():
    """NVT (Nose-Hoover, target kT = 1.5 from a start at kT = 1, tau = 0.05):
    216 ions, FP64 path, 25 steps: positions, velocities, the per step rows
    (E_kin and pressure after the thermostat's closing half) and the
    thermostat's state against the same splitting on the CPU with the
    oracle's forces (1e-9)."""
    import torch
    box = np.array([7.0, 7.0, 7.0])
    pos, q, v0, m = lattice_system((6, 6, 6), box, 11, jitter=0.05)
    kc, kT, tau = 2.0, 1.5, 0.05
    params = hs.Params(precision=0, p=8, K=162, F=512, lam=1.5, coulomb_k=kc)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nsteps, dt = 25, 0.002
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    st = torch.zeros(3, dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt, nh_kT=kT, nh_damping=tau) as md:
        md.run(x, v, f, qq, mm, nsteps, thermo=th)
        md.thermostat(st)
        torch.cuda.synchronize()
    xg, vg, tg, sg = x.cpu().numpy(), v.cpu().numpy(), th.cpu().numpy(), st.cpu().numpy()

    def coulomb(xx):
        r = ohsma.hsma3d(xx, q, np.zeros(3), box, 8, 162, 512, 1.5)
        return kc * r.force, kc * r.energy

    xc, vc, rc, nc = cpu_nose_hoover(pos, v0, q, m, box, coulomb, dt, nsteps, kT, tau)
    dx = min_image_diff(xg, xc, box) / box[0]
    dv = np.abs(vg - vc).max() / np.abs(vc).max()
    dr = (np.abs(tg - rc) / np.abs(rc).max(0)).max()
    dn = np.abs(sg - nc[-1]).max() / np.abs(nc[-1]).max()
    note(f"   positions {dx:.2e} velocities {dv:.2e} rows {dr:.2e} thermostat {dn:.2e}; "
         f"E_kin {rc[0, 2]:.3f} -> {rc[-1, 2]:.3f}, xi {nc[-1, 0]:.4f}")
    assert dx <= 1e-9 and dv <= 1e-9 and dr <= 1e-9 and dn <= 1e-9
    assert nc[-1, 0] < 0.0  # colder than the target: the thermostat heats (xi < 0)


@pytest.mark.parametrize("nh", [False, True])
def test_respa_trajectory_matches_cpu(nh):
    """Multiple time steps (respa_inner = 3: Coulomb forces every 0.006,
    short-range forces every 0.002), 216 ions, FP64, 10 outer steps, NVE
    and NVT: positions, velocities and rows against the same integrator on
    the CPU with the oracle's forces (1e-9); forces_valid = 1 continues
    from the driver's own force parts."""
    import torch
    box = np.array([7.0, 7.0, 7.0])
    pos, q, v0, m = lattice_system((6, 6, 6), box, 11, jitter=0.05)
    kc = 2.0
    params = hs.Params(precision=0, p=8, K=162, F=512, lam=1.5, coulomb_k=kc)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nsteps, dt, k = 10, 0.006, 3
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    kw = dict(nh_kT=1.5, nh_damping=0.05) if nh else {}
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt, respa_inner=k, **kw) as md:
        md.run(x, v, f, qq, mm, 4, thermo=th[:4])
        md.run(x, v, f, qq, mm, nsteps - 4, forces_valid=True, thermo=th[4:])
        torch.cuda.synchronize()
    xg, vg, tg = x.cpu().numpy(), v.cpu().numpy(), th.cpu().numpy()

    def coulomb(xx):
        r = ohsma.hsma3d(xx, q, np.zeros(3), box, 8, 162, 512, 1.5)
        return kc * r.force, kc * r.energy

    xc, vc, rc = cpu_respa(pos, v0, q, m, box, coulomb, dt, k, nsteps, *( (1.5, 0.05) if nh else ()))
    dx = min_image_diff(xg, xc, box) / box[0]
    dv = np.abs(vg - vc).max() / np.abs(vc).max()
    dr = (np.abs(tg - rc) / np.abs(rc).max(0)).max()
    note(f"   nh={nh}: positions {dx:.2e} velocities {dv:.2e} rows {dr:.2e}")
    assert dx <= 1e-9 and dv <= 1e-9 and dr <= 1e-9


def test_respa_slab_with_walls_matches_cpu():
    """Multiple time steps between the dielectric interfaces (the slab
    test's 100 ions, walls of sigma 0.5 among the short-range forces,
    respa_inner = 4, NVT): 8 outer steps against the numpy integrator with
    the oracle's slab forces (FP64, 1e-9)."""
    import torch
    box = np.array([10.0, 10.0, 8.0])
    pos, q, v0, m = lattice_system((5, 5, 4), box, 31, z_lo=1.2, z_hi=6.8)
    kc = 1.5
    params = hs.Params(geometry=1, precision=0, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=-0.5, gamma_low=0.3,
                       nz=40, coulomb_k=kc)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nsteps, dt, k = 8, 0.008, 4
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, \
            hs.MD(plan, len(q), dt, wall_epsilon=1.0, wall_sigma=0.5, nh_kT=1.5, nh_damping=0.05,
                  respa_inner=k) as md:
        md.run(x, v, f, qq, mm, nsteps, thermo=th)
        torch.cuda.synchronize()
    xg, tg = x.cpu().numpy(), th.cpu().numpy()

    def coulomb(xx):
        r = ohsma.hsma2d(xx, q, np.zeros(3), box, 8, 200, 512, 1.6, 6, -0.5, 0.3, 40)
        return kc * r.force, kc * r.energy

    xc, vc, rc = cpu_respa(pos, v0, q, m, box, coulomb, dt, k, nsteps, 1.5, 0.05, slab=True, weps=1.0, wsig=0.5)
    dx = min_image_diff(xg, xc, box, axes=2) / box[0]
    dr = (np.abs(tg - rc) / np.maximum(np.abs(rc).max(0), 1e-12)).max()
    note(f"   slab RESPA: positions {dx:.2e} rows {dr:.2e}")
    assert dx <= 1e-9 and dr <= 1e-9


def test_respa_energy_conservation_dt2():
    """NVE with multiple time steps (3 short-range steps per Coulomb step):
    the total energy's fluctuation falls like dt^2 when both steps are
    halved together (FP64, p = 10, the system of the velocity-Verlet test)."""
    import torch
    box = np.array([11.0, 11.0, 11.0])
    pos, q, v0, m = lattice_system((4, 4, 6), box, 21)
    params = hs.Params(precision=0, p=10, K=242, F=800, lam=1.5, coulomb_k=1.0)
    dev = torch.device("cuda:0")
    T, fluct = 0.96, []
    for dt in (0.012, 0.006):
        nsteps = int(round(T / dt))
        x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
        f = torch.zeros_like(x)
        qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
        th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
        row0 = torch.zeros(4, dtype=torch.float64, device=dev)
        with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt, respa_inner=3) as md:
            md.forces(x, v, f, qq, mm, thermo_row=row0)
            md.run(x, v, f, qq, mm, nsteps, forces_valid=True, thermo=th)
            torch.cuda.synchronize()
        t, r0 = th.cpu().numpy(), row0.cpu().numpy()
        H0 = r0[0] + r0[1] + r0[2]
        H = t[:, 0] + t[:, 1] + t[:, 2]
        fluct.append(np.sqrt(np.mean((H - H0) ** 2)))
        note(f"   outer dt {dt}: {nsteps} steps, rms(H - H0) {fluct[-1]:.3e} ({fluct[-1] / abs(r0[2]):.2e} of E_kin)")
    ratio = fluct[0] / fluct[1]
    note(f"   fluctuation ratio dt / (dt/2): {ratio:.2f}")
    assert 2.5 <= ratio <= 6.5
    assert fluct[1] <= 1e-3 * abs(r0[2])


def test_md_energy_conservation_dt2():
    """NVE: the total energy's fluctuation about its start falls like dt^2
    (velocity Verlet), and stays small, over the same time with dt and
    dt / 2 (FP64 path, p = 10)."""
    import torch
    box = np.array([11.0, 11.0, 11.0])
    pos, q, v0, m = lattice_system((4, 4, 6), box, 21)
    params = hs.Params(precision=0, p=10, K=242, F=800, lam=1.5, coulomb_k=1.0)
    dev = torch.device("cuda:0")
    T = 0.8
    fluct = []
    for dt in (0.004, 0.002):
        nsteps = int(round(T / dt))
        x = torch.tensor(pos, device=dev)
        v = torch.tensor(v0, device=dev)
        f = torch.zeros_like(x)
        qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
        th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
        row0 = torch.zeros(4, dtype=torch.float64, device=dev)
        with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt) as md:
            md.forces(x, v, f, qq, mm, thermo_row=row0)
            md.run(x, v, f, qq, mm, nsteps, forces_valid=True, thermo=th)
            torch.cuda.synchronize()
        t = th.cpu().numpy()
        r0 = row0.cpu().numpy()
        H0 = r0[0] + r0[1] + r0[2]
        H = t[:, 0] + t[:, 1] + t[:, 2]
        fl = np.sqrt(np.mean((H - H0) ** 2))
        fluct.append(fl)
        note(f"   dt {dt}: {nsteps} steps, H0 {H0:.8f}, rms(H - H0) {fl:.3e} ({fl / abs(r0[2]):.2e} of E_kin)")
    ratio = fluct[0] / fluct[1]
    note(f"   fluctuation ratio dt / (dt/2): {ratio:.2f}")
    assert 2.5 <= ratio <= 6.5
    assert fluct[1] <= 1e-3 * abs(r0[2])


def test_nose_hoover_extended_energy_dt2():
    """NVT conserves the extended energy E_C + E_LJ + E_kin + Q xi^2 / 2 +
    nf kT eta: its fluctuation about the start falls like dt^2 (the splitting
    is second order) over the same time with dt and dt / 2, while the
    thermostat exchanges energy with the system (FP64 path, p = 10, target
    kT = 1.6, tau = 0.1)."""
    import torch
    box = np.array([11.0, 11.0, 11.0])
    pos, q, v0, m = lattice_system((4, 4, 6), box, 21)
    params = hs.Params(precision=0, p=10, K=242, F=800, lam=1.5, coulomb_k=1.0)
    dev = torch.device("cuda:0")
    T = 0.8
    fluct, moved = [], []
    for dt in (0.004, 0.002):
        nsteps = int(round(T / dt))
        x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
        f = torch.zeros_like(x)
        qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
        th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
        st = torch.zeros((nsteps, 3), dtype=torch.float64, device=dev)
        row0 = torch.zeros(4, dtype=torch.float64, device=dev)
        with hs.Plan(params, (0, 0, 0), box) as plan, \
                hs.MD(plan, len(q), dt, nh_kT=1.6, nh_damping=0.1) as md:
            md.forces(x, v, f, qq, mm, thermo_row=row0)
            for i in range(nsteps):
                md.run(x, v, f, qq, mm, 1, forces_valid=True, thermo=th[i])
                md.thermostat(st[i])
            torch.cuda.synchronize()
        t, sn, r0 = th.cpu().numpy(), st.cpu().numpy(), row0.cpu().numpy()
        H0 = r0[0] + r0[1] + r0[2]
        H = t[:, 0] + t[:, 1] + t[:, 2] + sn[:, 2]
        fl = np.sqrt(np.mean((H - H0) ** 2))
        fluct.append(fl)
        moved.append(np.abs(sn[:, 2]).max())
        note(f"   dt {dt}: {nsteps} steps, H0 {H0:.8f}, rms(H - H0) {fl:.3e}, max |E_thermostat| {moved[-1]:.3e}, "
             f"E_kin {t[0, 2]:.3f} -> {t[-1, 2]:.3f}")
    ratio = fluct[0] / fluct[1]
    note(f"   fluctuation ratio dt / (dt/2): {ratio:.2f}")
    assert 2.5 <= ratio <= 6.5
    assert fluct[1] <= 1e-3 * moved[1]


def test_nose_hoover_mean_temperature_is_the_target():
    """Over a Nose-Hoover run the thermostat's momentum obeys
    Q dxi/dt = 2 E_kin - nf kT, so the time average of 2 E_kin / nf equals
    kT up to Q (xi_end - xi_start) / (nf time) whatever the dynamics: 96 ions
    from kT = 1 thermostatted to kT = 1.5 (tau = 0.1, 1000 steps of 0.004),
    the average over the last 750 steps within 3 percent of the target."""
    import torch
    box = np.array([11.0, 11.0, 11.0])
    pos, q, v0, m = lattice_system((4, 4, 6), box, 23)
    params = hs.Params(precision=0, p=8, K=162, F=512, lam=1.5, coulomb_k=1.0)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nsteps, dt, kT = 1000, 0.004, 1.5
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt, nh_kT=kT, nh_damping=0.1) as md:
        md.run(x, v, f, qq, mm, nsteps, thermo=th)
        torch.cuda.synchronize()
    t = th.cpu().numpy()
    nf = 3 * len(q) - 3
    temp = 2 * t[:, 2] / nf
    mean = temp[250:].mean()
    note(f"   kinetic temperature: first step {temp[0]:.3f}, mean over the last 750 steps {mean:.4f} (target {kT})")
    assert abs(mean - kT) <= 0.03 * kT


def test_md_slab_with_walls_matches_cpu():
    """100 ions between two dielectric interfaces (gamma_up = -0.5,
    gamma_low = 0.3, M = 6) kept inside by WCA walls, 15 steps: against the
    CPU integration with the oracle's slab forces (FP64)."""
    import torch
    box = np.array([10.0, 10.0, 8.0])
    pos, q, v0, m = lattice_system((5, 5, 4), box, 31, z_lo=1.2, z_hi=6.8)
    kc = 1.5
    params = hs.Params(geometry=1, precision=0, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=-0.5, gamma_low=0.3,
                       nz=40, coulomb_k=kc)
    dev = torch.device("cuda:0")
    x = torch.tensor(pos, device=dev)
    v = torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nsteps, dt = 15, 0.002
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt, wall_epsilon=1.0, wall_sigma=1.0) as md:
        md.run(x, v, f, qq, mm, nsteps, thermo=th)
        torch.cuda.synchronize()
    xg, tg = x.cpu().numpy(), th.cpu().numpy()

    def coulomb(xx):
        r = ohsma.hsma2d(xx, q, np.zeros(3), box, 8, 200, 512, 1.6, 6, -0.5, 0.3, 40)
        return kc * r.force, kc * r.energy

    xc, vc, rc = cpu_verlet(pos, v0, q, m, box, coulomb, dt, nsteps, slab=True, weps=1.0)
    dx = min_image_diff(xg, xc, box, axes=2) / box[0]
    de = np.abs(tg[:, 0] - rc[:, 0]).max() / np.abs(rc[:, 0]).max()
    dl = np.abs(tg[:, 1] - rc[:, 1]).max() / max(1e-12, np.abs(rc[:, 1]).max())
    note(f"   slab: positions {dx:.2e}; E_C {de:.2e} E_LJ {dl:.2e}; z range {xg[:, 2].min():.3f} .. {xg[:, 2].max():.3f}")
    assert dx <= 1e-9 and de <= 1e-10 and dl <= 1e-9


def test_nose_hoover_slab_with_walls_matches_cpu():
    """NVT between the dielectric interfaces (the slab test's 100 ions and
    walls; Nose-Hoover at kT = 1.5, tau = 0.05, nf = 3n - 2 since the walls
    take up momentum along z), 15 steps: positions, rows and thermostat
    state against the numpy integrator with the oracle's slab forces
    (FP64)."""
    import torch
    box = np.array([10.0, 10.0, 8.0])
    pos, q, v0, m = lattice_system((5, 5, 4), box, 31, z_lo=1.2, z_hi=6.8)
    kc, kT, tau = 1.5, 1.5, 0.05
    params = hs.Params(geometry=1, precision=0, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=-0.5, gamma_low=0.3,
                       nz=40, coulomb_k=kc)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nsteps, dt = 15, 0.002
    th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
    st = torch.zeros(3, dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, \
            hs.MD(plan, len(q), dt, wall_epsilon=1.0, wall_sigma=1.0, nh_kT=kT, nh_damping=tau) as md:
        md.run(x, v, f, qq, mm, nsteps, thermo=th)
        md.thermostat(st)
        torch.cuda.synchronize()
    xg, tg, sg = x.cpu().numpy(), th.cpu().numpy(), st.cpu().numpy()

    def coulomb(xx):
        r = ohsma.hsma2d(xx, q, np.zeros(3), box, 8, 200, 512, 1.6, 6, -0.5, 0.3, 40)
        return kc * r.force, kc * r.energy

    xc, vc, rc, nc = cpu_nose_hoover(pos, v0, q, m, box, coulomb, dt, nsteps, kT, tau, slab=True, weps=1.0)
    dx = min_image_diff(xg, xc, box, axes=2) / box[0]
    dr = (np.abs(tg - rc) / np.maximum(np.abs(rc).max(0), 1e-12)).max()
    dn = np.abs(sg - nc[-1]).max() / np.abs(nc[-1]).max()
    note(f"   slab NVT: positions {dx:.2e} rows {dr:.2e} thermostat {dn:.2e}; xi {nc[-1, 0]:.4f}")
    assert dx <= 1e-9 and dr <= 1e-9 and dn <= 1e-9


@pytest.mark.parametrize("slab", [False, True])
def test_rdf_and_zprofile_counts_exact(slab):
    """Pair-distance and z-density counts on 700 ions (three target blocks,
    three source chunks, a ragged end; charges +-1, +2 and some zero) with
    r_max at half the box edge: equal, count for count, to the definition
    evaluated in numpy; and accumulated over two calls."""
    import torch
    rng = np.random.default_rng(5)
    box = np.array([9.0, 11.0, 8.0])
    n = 700
    x = rng.uniform(0, 1, (n, 3)) * box
    if slab:
        x[:, 2] = 0.5 + rng.uniform(0, 1, n) * (box[2] - 1.0)
    q = rng.choice([1.0, -1.0, 2.0, 0.0], n, p=[0.45, 0.4, 0.1, 0.05])
    dev = torch.device("cuda:0")
    xt, qt = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
    nbins, rmax = 300, 4.0  # half the smallest periodic edge in 3D (L_z = 8)
    h = torch.zeros((3, nbins), dtype=torch.int64, device=dev)
    zh = torch.zeros((2, 64), dtype=torch.int64, device=dev)
    with hs.MD(None, n, 0.001, geometry=hs.GEOM_2D if slab else hs.GEOM_3D, box_lo=(0, 0, 0), box_len=box) as md:
        md.rdf(xt, qt, rmax, h)
        md.rdf(xt, qt, rmax, h)
        md.zprofile(xt, qt, zh)
        with pytest.raises(hs.HSMAError):
            md.rdf(xt, qt, 4.6, h)  # beyond half the smallest periodic edge (3D: 4; slab: 4.5)
        torch.cuda.synchronize()
    ref = rdf_numpy(x, q, box, nbins, rmax, slab)
    hg = h.cpu().numpy()
    zref = np.zeros((2, 64), np.int64)
    zb = np.clip(np.floor((x[:, 2] - 0.0) / (box[2] / 64)).astype(np.int64), 0, 63)
    for c, sel in enumerate((q > 0, q < 0)):
        np.add.at(zref[c], zb[sel], 1)
    note(f"   slab={slab}: {ref.sum()} pairs within r_max; classes {ref.sum(1).tolist()}")
    assert np.array_equal(hg, 2 * ref)
    assert np.array_equal(zh.cpu().numpy(), zref)


def test_electrolyte_rdf_contacts():
    """The 216-ion melt of the trajectory test (Bjerrum length 2), thermostatted
    at kT = 1 for 1,000 steps and sampled every 50: unlike charges are in
    contact more often than like ones (pair-normalised counts below 1.3
    sigma; measured 1.65 times as often in this dense melt, asserted with a
    margin of 1.25 over the sampling noise of about 3 percent), and every
    count stays within its pair total."""
    import torch
    box = np.array([7.0, 7.0, 7.0])
    pos, q, v0, m = lattice_system((6, 6, 6), box, 11, jitter=0.05)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, coulomb_k=2.0)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
    nbins, rmax = 70, 3.5
    h = torch.zeros((3, nbins), dtype=torch.int64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), 0.005, nh_kT=1.0, nh_damping=0.1) as md:
        md.run(x, v, f, qq, mm, 200, forces_valid=False)
        for _ in range(16):
            md.run(x, v, f, qq, mm, 50, forces_valid=True)
            md.rdf(x, qq, rmax, h)
        torch.cuda.synchronize()
    hc = h.cpu().numpy()
    npos, nneg = int((q > 0).sum()), int((q < 0).sum())
    pairs = np.array([npos * (npos - 1) / 2, npos * nneg, nneg * (nneg - 1) / 2]) * 16
    close = hc[:, : int(1.3 / (rmax / nbins))].sum(1) / pairs
    note(f"   contacts per pair below 1.3 sigma: ++ {close[0]:.4f}, +- {close[1]:.4f}, -- {close[2]:.4f}")
    assert close[1] > 1.25 * max(close[0], close[2])
    assert (hc.sum(1) <= pairs).all()


def test_slab_dielectric_depletion():
    """The paper's slab experiment in miniature (Sec. 4.3: ions between two
    interfaces with gamma = 0.939 on both sides, WCA walls of sigma 0.5 at
    the interfaces, Bjerrum length 3.5, NVT): repulsive polarisation
    depletes the ions near the interfaces.  100 ions in 10 x 10 x 8, 1,000
    steps of equilibration then 60 z profiles 50 steps apart
    (hsma_md_zprofile), with gamma = 0.939 and with gamma = 0: fewer ions
    within 1 sigma of an interface with the images (FP32C, p = 8)."""
    import torch
    box = np.array([10.0, 10.0, 8.0])
    pos, q, v0, m = lattice_system((5, 5, 4), box, 31, z_lo=1.2, z_hi=6.8)
    dev = torch.device("cuda:0")
    near = {}
    for g in (0.939, 0.0):
        params = hs.Params(geometry=1, precision=1, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=g, gamma_low=g,
                           nz=40, coulomb_k=3.5)
        x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
        f = torch.zeros_like(x)
        qq, mm = torch.tensor(q, device=dev), torch.tensor(m, device=dev)
        zh = torch.zeros((2, 16), dtype=torch.int64, device=dev)  # bins of 0.5 sigma
        with hs.Plan(params, (0, 0, 0), box) as plan, \
                hs.MD(plan, len(q), 0.005, wall_epsilon=1.0, wall_sigma=0.5, nh_kT=1.0, nh_damping=0.05) as md:
            md.run(x, v, f, qq, mm, 1000, forces_valid=False)
            for _ in range(60):
                md.run(x, v, f, qq, mm, 50, forces_valid=True)
                md.zprofile(x, qq, zh)
            torch.cuda.synchronize()
        h = zh.cpu().numpy().sum(0)
        near[g] = (h[:2].sum() + h[-2:].sum()) / h.sum()
        note(f"   gamma {g}: profile {h.tolist()}; fraction within 1 sigma of an interface {near[g]:.4f}")
    assert near[0.939] < 0.8 * near[0.0]


def test_coulomb_virial_is_the_energy():
    """The pressure's Coulomb virial W_C = -dE/ds at s = 1 under scaling of
    positions and box together equals E_C (the HSMA energy is homogeneous of
    degree -1): checked on the oracle by a central difference, and the
    driver's pressure uses it with the LJ pair virial."""
    import torch
    box = np.array([12.0, 12.0, 12.0])
    pos, q, v0, m = lattice_system((4, 4, 4), box, 41)
    e = lambda s: ohsma.hsma3d(pos * s, q, np.zeros(3), box * s, 8, 162, 512, 1.5).energy
    h = 1e-4
    w = -(e(1 + h) - e(1 - h)) / (2 * h)
    e1 = e(1.0)
    note(f"   W_C {w:.12g}, E_C {e1:.12g}, rel {abs(w - e1) / abs(e1):.2e}")
    assert abs(w - e1) <= 1e-7 * abs(e1)
    params = hs.Params(precision=0, p=8, K=162, F=512, lam=1.5)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    row = torch.zeros(4, dtype=torch.float64, device=dev)
    with hs.Plan(params, (0, 0, 0), box) as plan, hs.MD(plan, len(q), 0.001) as md:
        md.forces(x, v, f, torch.tensor(q, device=dev), torch.tensor(m, device=dev), thermo_row=row)
        torch.cuda.synchronize()
    r = row.cpu().numpy()
    _, el, wl = lj_numpy(pos, box, False)
    ke = 0.5 * (v0 * v0).sum()
    p_ref = (2 * ke + wl + e1) / (3 * box.prod())
    note(f"   pressure {r[3]:.12g} reference {p_ref:.12g}")
    assert abs(r[0] - e1) <= 1e-10 * abs(e1) and abs(r[3] - p_ref) <= 1e-10 * abs(p_ref)


@pytest.mark.parametrize("nh", [False, True])
def test_replica_ensemble_on_the_server(nh):
    """Four MD replicas on the serving loop (device-resident state, Coulomb
    forces by device requests with system ids, drift and finish on the
    device; NVE, or NVT with a Nose-Hoover thermostat per replica):
    trajectories and thermo rows equal each replica integrated by its own
    plan to 1e-9 (FP64; the server re-targets a unit-box plan), and the
    replicas' steps are replayed from captured graphs."""
    import torch
    th_kw = dict(nh_kT=1.5, nh_damping=0.05) if nh else {}
    dev = torch.device("cuda:0")
    prm = hs.Params(precision=0, p=8, K=162, F=512, lam=1.5)
    reps, refs = [], []
    nsteps, dt = 10, 0.002
    for i, L in enumerate((7.0, 7.1, 7.2, 7.3)):
        box = np.array([L, L, L])
        pos, q, v0, m = lattice_system((6, 6, 6), box, 50 + i, jitter=0.05)
        reps.append(dict(x=torch.tensor(pos, device=dev), v=torch.tensor(v0, device=dev),
                         q=torch.tensor(q, device=dev), m=torch.tensor(m, device=dev), box_lo=(0.0, 0.0, 0.0),
                         box_len=tuple(box)))
        # reference: the replica on its own plan
        x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
        f = torch.zeros_like(x)
        th = torch.zeros((nsteps, 4), dtype=torch.float64, device=dev)
        with hs.Plan(prm, (0, 0, 0), box) as plan, hs.MD(plan, len(q), dt, **th_kw) as md:
            md.run(x, v, f, torch.tensor(q, device=dev), torch.tensor(m, device=dev), nsteps, thermo=th)
            torch.cuda.synchronize()
        refs.append((x.cpu().numpy(), th.cpu().numpy(), box))
    with hs.Server(prm, (1.0, 1.0, 1.0), max_n=216, max_slots=4) as sv:
        ens = hs.ReplicaEnsemble(sv, reps, dt, **th_kw)
        rows = [[torch.zeros(4, dtype=torch.float64, device=dev) for _ in reps] for _ in range(nsteps)]
        for s in range(nsteps):
            res = ens.step(rows[s])
            assert all(r["status"] == 0 for r in res)
        torch.cuda.synchronize()
        st = sv.stats()
        ens.close()
    note(f"   server stats {st}")
    for k, (r, (xr, thr, box)) in enumerate(zip(reps, refs)):
        dx = min_image_diff(r["x"].cpu().numpy(), xr, box) / box[0]
        tg = np.array([[rows[s][k][c].item() for c in range(4)] for s in range(nsteps)])
        dth = np.abs(tg - thr).max() / np.abs(thr).max()
        note(f"   replica {k}: positions {dx:.2e} thermo {dth:.2e}")
        assert dx <= 1e-9 and dth <= 1e-9
    assert st["graph_replays"] >= 4 * (nsteps - 2)
