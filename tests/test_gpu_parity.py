"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs."""
import math
import sys

import numpy as np
import pytest

import workloads
from oracle import geometry as ogeo
from oracle import hsma as ohsma
from oracle import native

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2104_05260_amd")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def run_gpu(params, pos, q, lo, L):
    with hs.Plan(params, lo, L) as plan:
        return plan.compute(pos, q)


def oracle_run(params, pos, q, lo, L, targets=None):
    # near rule 2 (treecode) approximates the 27-cell sums of rule 0: the
    # oracle computes those exactly
    rule = 0 if params.near_rule == 2 else params.near_rule
    if params.geometry == 0:
        return ohsma.hsma3d(pos, q, lo, L, params.p, params.K, params.F, params.lam, params.Fw,
                            params.surface_rule, targets, rule)
    return ohsma.hsma2d(pos, q, lo, L, params.p, params.K, params.F, params.lam, params.M, params.gamma_up,
                        params.gamma_low, params.nz, params.Fw, params.surface_rule, targets, rule)


# FP64 path: agreement to 1e-10 relative (energy, potentials, forces).
# FP32 compensated path: 1e-5 relative RMS force and max potential, and
# the energy to 1e-6 relative (FP32C_E) on every benchmark system (100,
# 50,000, the 20,000-ion slab and 999,999 ions; measured 1.3e-7 to 6.3e-7).
# Small random test systems (the ragged sizes, the boundary and clustered
# cases) have energies that are a small remainder of their terms (|E| / S
# = 0.02 to 0.05 at 1000 ions, S = 1/2 sum |q_i Phi_i|), and every pair
# term carries a few units of FP32 rounding that does not cancel, so the
# energy error is a random walk that scales with S, not with E.  For those
# systems the bar is 1e-6 |E| + FP32_E_FLOOR S.
TOL64 = 1e-10
FP32C_E = 1e-6
FP32_E_FLOOR = 1e-7


def fp32_energy_bar(E, S):
    """Energy bar of the small cancelling test systems (not used for the
    benchmark systems, which are held to FP32C_E |E|)."""
    return FP32C_E * abs(E) + FP32_E_FLOOR * S


# Treecode (near rule 2) against the oracle's exact 27-cell sums: the FP32
# bars for energy and force, and 5e-5 on the largest potential error (the
# truncation of the multipole expansions; measured up to 1.7e-5 at order
# 8, theta 0.5 on the 50,000-ion system).  At the default order 12, theta
# 0.5 the benchmark systems meet the FP32C energy bar (50,000 ions 4.5e-7,
# 999,999 ions 1.5e-7; the slab, whose multipoles are evaluated in FP64,
# 9.7e-7, and 5.3e-7 at theta 0.45).
TREE_POT = 5e-5


def check(params, pos, q, lo, L, fp32=False, label="", pot_bar=1e-5, cancel_floor=True):
    """GPU against oracle on the whole system.  cancel_floor: the FP32 energy
    bar of the small cancelling test systems (fp32_energy_bar); False holds
    the energy to FP32C_E |E| alone."""
    note(f"[parity] {label} n={len(q)} geometry={params.geometry} precision={params.precision}")
    e, pot, f = run_gpu(params, pos, q, lo, L)
    r = oracle_run(params, pos, q, lo, L)
    de = abs(e - r.energy) / abs(r.energy)
    dp = np.abs(pot - r.potential).max() / np.abs(r.potential).max()
    df = rel_rms(f, r.force)
    dfmax = np.abs(f - r.force).max() / np.abs(r.force).max()
    note(f"   energy {e:.15g} oracle {r.energy:.15g}: rel {de:.2e}; potential max rel {dp:.2e}; "
         f"force rms rel {df:.2e}, max rel {dfmax:.2e}")
    if fp32:
        S = 0.5 * np.abs(q * r.potential).sum()
        bar = fp32_energy_bar(r.energy, S) if cancel_floor else FP32C_E * abs(r.energy)
        note(f"   energy scale S {S:.6g}; |dE| {abs(e - r.energy):.3g}, bar {bar:.3g}; |dE|/S {abs(e - r.energy) / S:.2e}")
        assert abs(e - r.energy) <= bar and df <= 1e-5 and dp <= pot_bar
    else:
        assert de <= TOL64 and dp <= TOL64 and dfmax <= TOL64 * 10 and df <= TOL64
    return e, pot, f, r


def test_c1_fp64_matches_oracle():
    w = workloads.C1
    pos, q, lo, L = workloads.make_system(w)
    check(hs.Params.from_workload(w, precision=hs.FP64), pos, q, lo, L, label="C1 fp64")


def test_c1_fp32c_matches_oracle():
    w = workloads.C1
    pos, q, lo, L = workloads.make_system(w)
    check(hs.Params.from_workload(w, precision=hs.FP32C), pos, q, lo, L, fp32=True, label="C1 fp32c",
          cancel_floor=False)


@pytest.mark.parametrize("n", [2, 64, 130, 1000, 4096, 4098])
@pytest.mark.parametrize("prec", [0, 1])
def test_ragged_sizes_3d(n, prec):
    """Sizes around the 64-source tile and the 64-target group: empty
    tails, one partial tile, several tiles with a ragged end; 4096 is the
    largest system sorted in one block, 4098 the smallest above it (radix
    sort across blocks)."""
    L = 3.0 * (n / 2.0) ** (1 / 3) + 2.0
    pos, q, lo, box = workloads.small_system(n, (L, L * 1.1, L * 0.9), 100 + n)
    lo = np.array([-1.0, 2.0, 0.5])
    pos = pos + lo
    params = hs.Params(precision=prec, p=6, K=100, F=200, lam=1.4)
    check(params, pos, q, lo, box, fp32=prec == 1, label=f"3d ragged n={n}")


@pytest.mark.parametrize("prec,rule", [(0, 0), (1, 0), (1, 2)])
def test_boundary_and_wrapped_positions(prec, rule):
    """Ions exactly on box faces, edges and corners, and ions given one or
    two box lengths outside the box (wrapped into it by both sides)."""
    L = np.array([9.0, 10.0, 11.0])
    lo = np.array([-2.0, 1.0, 0.5])
    pos, q, _, _ = workloads.small_system(200, tuple(L), 17)
    pos = pos + lo
    rng = np.random.default_rng(3)
    for i in range(0, 24):           # faces (one coordinate) and edges (two)
        for k in rng.choice(3, 1 + i % 2, replace=False):
            pos[i, k] = lo[k] + (L[k] if rng.random() < 0.5 else 0.0)
    pos[24] = lo + L                 # one corner (all corners are one point)
    for i in range(25, 48):          # one or two periods outside
        pos[i] += rng.integers(-2, 3, 3) * L
    params = hs.Params(precision=prec, p=6, K=100, F=200, lam=1.4, near_rule=rule)
    check(params, pos, q, lo, L, fp32=prec == 1, label=f"boundary and wrapped positions, near rule {rule}",
          pot_bar=TREE_POT if rule == 2 else 1e-5)


def test_single_neutral_particle():
    """n = 1 with zero charge: neutral, every output zero."""
    L = np.array([5.0, 5.0, 5.0])
    with hs.Plan(hs.Params(precision=0, p=4, K=60, F=200, lam=1.5), [0, 0, 0], L) as plan:
        e, pot, f = plan.compute(np.array([[1.0, 2.0, 3.0]]), np.array([0.0]))
    assert e == 0.0 and np.all(pot == 0.0) and np.all(f == 0.0)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gam", [(0.0, 0.0), (-0.94, -0.94), (0.5, -0.3)])
def test_slab_matches_oracle(prec, gam):
    pos, q, lo, L = workloads.small_system(300, (20.0, 20.0, 10.0), 21, geometry=1)
    params = hs.Params(geometry=1, precision=prec, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=gam[0],
                       gamma_low=gam[1], nz=40)
    check(params, pos, q, lo, L, fp32=prec == 1, label=f"slab gamma={gam}")


# ---- sphere near set (near_rule=1): only the images inside the sphere.
# The inside/outside decision is taken in FP64 on the same image positions
# and the same R on both sides, so the parity bars are those above.
def test_c1_sphere_near_set():
    w = workloads.C1
    pos, q, lo, L = workloads.make_system(w)
    for prec in (0, 1):
        params = hs.Params.from_workload(w, precision=prec)
        params.near_rule = 1
        check(params, pos, q, lo, L, fp32=prec == 1, label=f"C1 sphere near set prec={prec}")


@pytest.mark.parametrize("n", [2, 130, 1000, 4098])
@pytest.mark.parametrize("prec", [0, 1])
def test_sphere_near_set_ragged_3d(n, prec):
    L = 3.0 * (n / 2.0) ** (1 / 3) + 2.0
    pos, q, lo, box = workloads.small_system(n, (L, L * 1.1, L * 0.9), 300 + n)
    lo = np.array([0.5, -2.0, 1.0])
    pos = pos + lo
    params = hs.Params(precision=prec, p=8, K=162, F=512, lam=1.4, near_rule=1)
    check(params, pos, q, lo, box, fp32=prec == 1, label=f"3d sphere near set n={n}")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gam", [(-0.94, -0.94), (0.5, -0.3)])
def test_sphere_near_set_slab(prec, gam):
    pos, q, lo, L = workloads.small_system(300, (20.0, 20.0, 10.0), 23, geometry=1)
    params = hs.Params(geometry=1, precision=prec, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=gam[0],
                       gamma_low=gam[1], nz=40, near_rule=1)
    check(params, pos, q, lo, L, fp32=prec == 1, label=f"slab sphere near set gamma={gam}")


def test_sphere_near_set_pair_count():
    """Plan info reports the pairs the sphere near set actually sums: every
    particle against every image inside the sphere, self pairs excluded
    (counted here directly from the positions)."""
    pos, q, lo, L = workloads.small_system(3000, (25.0, 25.0, 25.0), 8)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, near_rule=1)
    with hs.Plan(params, lo, L) as plan:
        plan.compute(pos, q)
        info = plan.info()
    x = ogeo.centre_and_wrap(pos, lo, L)
    R = ohsma._radius(L, 1.5)
    inside = 0
    for k in ogeo.shifts_3d() * L:
        y = x + k
        inside += int((((y[:, 0] * y[:, 0] + y[:, 1] * y[:, 1]) + y[:, 2] * y[:, 2]) < R * R).sum())
    assert info["near_pairs"] == len(q) * inside - len(q)
    assert info["check_pairs"] == info["n_check"] * inside


def test_deterministic_and_permutation():
    pos, q, lo, L = workloads.small_system(3000, (25.0, 25.0, 25.0), 7)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5)
    with hs.Plan(params, lo, L) as plan:
        a = plan.compute(pos, q)
        b = plan.compute(pos, q)
        perm = np.random.default_rng(0).permutation(len(q))
        c = plan.compute(pos[perm], q[perm])
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert abs(c[0] - a[0]) <= 1e-12 * abs(a[0])
    assert np.abs(c[2] - a[2][perm]).max() <= 1e-6 * np.abs(a[2]).max()


def test_invalid_inputs():
    import torch
    pos, q, lo, L = workloads.small_system(200, (8.0, 8.0, 8.0), 3)
    params = hs.Params(precision=1, p=6, K=100, F=200, lam=1.5)
    with hs.Plan(params, lo, L) as plan:
        with pytest.raises(hs.HSMAError) as e:
            plan.compute(pos, q + 0.01)
        assert e.value.name == "HSMA_ERR_NOT_NEUTRAL"
        bad = pos.copy()
        bad[3, 1] = np.nan
        with pytest.raises(hs.HSMAError) as e:
            plan.compute(bad, q)
        assert e.value.name == "HSMA_ERR_OUT_OF_DOMAIN"
        with pytest.raises(hs.HSMAError):
            plan.compute(pos[:0], q[:0])
        # device path: validation on the GPU, NaN outputs, status afterwards
        dev = torch.device("cuda:0")
        x = torch.tensor(pos, device=dev)
        qq = torch.tensor(q + 0.01, device=dev)
        en = torch.zeros(1, dtype=torch.float64, device=dev)
        pot = torch.zeros(len(q), dtype=torch.float64, device=dev)
        f = torch.zeros((len(q), 3), dtype=torch.float64, device=dev)
        plan.compute_device(x, qq, en, pot, f)
        assert hs.STATUS[plan.device_status()] == "HSMA_ERR_NOT_NEUTRAL"
        assert torch.isnan(pot).all() and torch.isnan(f).all()
        # and a valid call afterwards works again
        qq = torch.tensor(q, device=dev)
        plan.compute_device(x, qq, en, pot, f)
        assert plan.device_status() == 0
        e_host, pot_h, f_h = plan.compute(pos, q)
        torch.cuda.synchronize()
        assert abs(en.item() - e_host) <= 1e-12 * abs(e_host)
        assert np.array_equal(f.cpu().numpy(), f_h)
    # slab: particle on the interface
    pos2, q2, lo2, L2 = workloads.small_system(50, (10.0, 10.0, 5.0), 4, geometry=1)
    pos2[0, 2] = 5.0
    with hs.Plan(hs.Params(geometry=1, p=4, K=60, F=200, lam=1.6, M=4, nz=20), lo2, L2) as plan:
        with pytest.raises(hs.HSMAError) as e:
            plan.compute(pos2, q2)
        assert e.value.name == "HSMA_ERR_OUT_OF_DOMAIN"


@pytest.mark.parametrize("prec,rule", [(0, 0), (1, 0), (1, 2)])
def test_coincident_charges(prec, rule):
    """Two charges at zero distance (here one ion placed on a periodic image
    of another, one box length away) have no finite energy: the call
    completes, the energy and the two ions' forces are not finite, and the
    plan computes the next, valid system as if nothing had happened."""
    pos, q, lo, L = workloads.small_system(200, (8.0, 8.0, 8.0), 3)
    params = hs.Params(precision=prec, p=6, K=100, F=200, lam=1.5, near_rule=rule)
    bad = pos.copy()
    i, j = int(np.argmax(q > 0)), int(np.argmax(q < 0))
    # dyadic coordinates: the wrap of ion j onto ion i is exact
    bad[i] = lo + np.array([1.5, 2.25, 3.125])
    bad[j] = bad[i] + np.array([L[0], 0.0, 0.0])
    with hs.Plan(params, lo, L) as plan:
        e, pot, f = plan.compute(bad, q)
        assert not np.isfinite(e)
        assert not np.isfinite(f[[i, j]]).all()
        e2, pot2, f2 = plan.compute(pos, q)
    with hs.Plan(params, lo, L) as fresh:
        e3, pot3, f3 = fresh.compute(pos, q)
    assert np.isfinite(e2) and e2 == e3 and np.array_equal(pot2, pot3) and np.array_equal(f2, f3)


@pytest.mark.parametrize("rule,limit", [(0, (1 << 30) - 1), (1, 1 << 26), (2, 1 << 26)])
def test_particle_count_limits(rule, limit):
    """A count above the per-call limit is refused on the host before any
    buffer is read or any work is enqueued (the buffers passed here hold
    three particles); a server whose slots would exceed it is refused at
    creation.  The plan then still computes a valid system."""
    import ctypes
    import torch
    pos, q, lo, L = workloads.small_system(200, (8.0, 8.0, 8.0), 3)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, near_rule=rule)
    dev = torch.device("cuda:0")
    x = torch.zeros((3, 3), dtype=torch.float64, device=dev)
    qq = torch.zeros(3, dtype=torch.float64, device=dev)
    out = torch.zeros(9, dtype=torch.float64, device=dev)
    xh, qh = np.zeros((3, 3)), np.zeros(3)
    with hs.Plan(params, lo, L) as plan:
        lib = plan._lib
        vp = lambda t: ctypes.c_void_p(t.data_ptr())
        st = lib.hsma_compute_device(plan._p, None, limit + 1, vp(x), vp(qq), vp(out), vp(out), vp(out))
        assert hs.STATUS[st] == "HSMA_ERR_INVALID_ARG"
        assert b"too many particles" in lib.hsma_last_error()
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st = lib.hsma_compute(plan._p, limit + 1, dp(xh), dp(qh), None, None, None)
        assert hs.STATUS[st] == "HSMA_ERR_INVALID_ARG"
        torch.cuda.synchronize()
        e, pot, f = plan.compute(pos, q)
        assert np.isfinite(e) and np.isfinite(f).all()
    with pytest.raises(hs.HSMAError) as err:
        hs.Server(params, (8.0, 8.0, 8.0), max_n=limit + 1, max_slots=1)
    assert err.value.name == "HSMA_ERR_INVALID_ARG"


def _sampled_oracle(w, params, pos, q, lo, L, sample):
    """Oracle at full size, evaluated only at the sampled particles (the
    check-point sums and the fit use every particle)."""
    return oracle_run(params, pos, q, lo, L, targets=sample)


def test_c2_full_size_sampled():
    """The 50,000-ion system in the launch configuration the benchmark
    times: FP32 compensated and FP64 GPU paths against the oracle at 256
    sampled particles, and against each other everywhere."""
    w = workloads.C2
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(5).choice(w.n, 256, replace=False)
    note("[parity] C2 oracle (sampled)")
    r = _sampled_oracle(w, hs.Params.from_workload(w), pos, q, lo, L, sample)
    res = {}
    for prec in (1, 0):
        note(f"[parity] C2 gpu precision={prec}")
        e, pot, f = run_gpu(hs.Params.from_workload(w, precision=prec), pos, q, lo, L)
        res[prec] = (e, pot, f)
        dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
        df = rel_rms(f[sample], r.force)
        note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}")
        if prec == 0:
            assert dp < 1e-10 and df < 1e-10
        else:
            assert dp < 1e-5 and df < 1e-5
    e32, e64 = res[1][0], res[0][0]
    S = 0.5 * np.abs(q * res[0][1]).sum()
    note(f"   energy fp32c {e32:.12g} fp64 {e64:.12g} rel {abs(e32 - e64) / abs(e64):.2e}; "
         f"S {S:.6g}, |E|/S {abs(e64) / S:.2e}, dE/S {abs(e32 - e64) / S:.2e}")
    assert abs(e32 - e64) <= FP32C_E * abs(e64)
    assert rel_rms(res[1][2], res[0][2]) <= 1e-5
    # net force of a periodic system vanishes within the method error
    assert np.abs(res[0][2].sum(0)).max() <= 1e-4 * np.sqrt((res[0][2] ** 2).sum())


def test_c2_sphere_near_set_sampled():
    """The 50,000-ion system with the sphere near set, in the configuration
    the benchmark times for it: both precisions against the oracle at 256
    sampled particles."""
    w = workloads.C2
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(6).choice(w.n, 256, replace=False)
    params = hs.Params.from_workload(w)
    params.near_rule = 1
    note("[parity] C2 sphere near set: oracle (sampled)")
    r = _sampled_oracle(w, params, pos, q, lo, L, sample)
    for prec in (1, 0):
        params.precision = prec
        note(f"[parity] C2 sphere near set gpu precision={prec}")
        e, pot, f = run_gpu(params, pos, q, lo, L)
        dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
        df = rel_rms(f[sample], r.force)
        note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}")
        assert (dp < 1e-10 and df < 1e-10) if prec == 0 else (dp < 1e-5 and df < 1e-5)


def test_c3_slab_full_size_sampled():
    """The 20,000-ion dielectric slab (gamma = -0.94, M = 10 image layers,
    80 x 80 interface grids) against the oracle at 256 sampled particles."""
    w = workloads.C3
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(6).choice(w.n, 256, replace=False)
    note("[parity] C3 oracle (sampled)")
    r = _sampled_oracle(w, hs.Params.from_workload(w), pos, q, lo, L, sample)
    res = {}
    for prec in (1, 0):
        note(f"[parity] C3 gpu precision={prec}")
        e, pot, f = run_gpu(hs.Params.from_workload(w, precision=prec), pos, q, lo, L)
        res[prec] = (e, pot, f)
        dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
        df = rel_rms(f[sample], r.force)
        note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}")
        if prec == 0:
            assert dp < 1e-10 and df < 1e-10
        else:
            assert dp < 1e-5 and df < 1e-5
    e32, e64 = res[1][0], res[0][0]
    S = 0.5 * np.abs(q * res[0][1]).sum()
    note(f"   energy fp32c {e32:.12g} fp64 {e64:.12g} rel {abs(e32 - e64) / abs(e64):.2e}; S {S:.6g}, "
         f"dE/S {abs(e32 - e64) / S:.2e}")
    assert abs(e32 - e64) <= FP32C_E * abs(e64)
    assert rel_rms(res[1][2], res[0][2]) <= 1e-5
    # in-plane net force vanishes within the method error
    f64 = res[0][2]
    assert np.abs(f64[:, :2].sum(0)).max() <= 1e-3 * np.sqrt((f64 ** 2).sum())


def test_c3_sphere_near_set_sampled():
    """The 20,000-ion slab with the sphere near set at p = 14: FP64 face rows
    and FP32 interface rows in one partial buffer (65,536 check slots),
    both precisions against the oracle at 128 sampled ions."""
    import dataclasses
    w = dataclasses.replace(workloads.C3, near_rule=1, p=14, K=450, F=1152)
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(8).choice(w.n, 128, replace=False)
    note("[parity] C3 sphere near set: oracle (sampled)")
    r = _sampled_oracle(w, hs.Params.from_workload(w), pos, q, lo, L, sample)
    for prec in (1, 0):
        note(f"[parity] C3 sphere near set gpu precision={prec}")
        e, pot, f = run_gpu(hs.Params.from_workload(w, precision=prec), pos, q, lo, L)
        dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
        df = rel_rms(f[sample], r.force)
        note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}")
        assert (dp < 1e-10 and df < 1e-10) if prec == 0 else (dp < 1e-5 and df < 1e-5)


def test_c5_million_ions_sampled():
    """999,999 ions (2:1 valence) in L = 200, p = 12, F = 1152, K = 800: the
    FP64 and FP32 compensated paths with the 27 cells summed directly, and
    the FP32 path with the treecode, against the oracle at 128 sampled
    particles (the oracle's check sums and fit use every particle); the
    FP32 energy against the FP64 path's over the whole system."""
    w = workloads.C5
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(7).choice(w.n, 128, replace=False)
    note("[parity] C5 oracle (sampled)")
    r = _sampled_oracle(w, hs.Params.from_workload(w), pos, q, lo, L, sample)
    res = {}
    for prec in (1, 0):
        note(f"[parity] C5 gpu precision={prec}")
        e, pot, f = run_gpu(hs.Params.from_workload(w, precision=prec), pos, q, lo, L)
        res[prec] = (e, pot, f)
        dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
        df = rel_rms(f[sample], r.force)
        dfm = np.abs(f[sample] - r.force).max() / np.abs(r.force).max()
        note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}, force max rel {dfm:.2e}")
        if prec == 0:
            assert dp < 1e-10 and df < 1e-10
        else:
            assert dp < 1e-5 and df < 1e-5
        assert np.isfinite(e)
        assert np.abs(f.sum(0)).max() <= 1e-3 * np.sqrt((f ** 2).sum())
    (e, pot, f), (e64, pot64, f64) = res[1], res[0]
    S = 0.5 * np.abs(q * pot64).sum()
    note(f"   energy fp32c {e:.12g} fp64 {e64:.12g} rel {abs(e - e64) / abs(e64):.2e}; dE/S {abs(e - e64) / S:.2e}; "
         f"force rms rel {rel_rms(f, f64):.2e}")
    assert abs(e - e64) <= FP32C_E * abs(e64)
    assert rel_rms(f, f64) <= 1e-5
    note("[parity] C5 gpu treecode")
    params = hs.Params.from_workload(w, precision=1)
    params.near_rule = 2
    et, pt, ft = run_gpu(params, pos, q, lo, L)
    dp = np.abs(pt[sample] - r.potential).max() / np.abs(r.potential).max()
    df = rel_rms(ft[sample], r.force)
    note(f"   treecode sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}; energy {et:.12g} "
         f"(fp64 direct {e64:.12g}, rel {abs(et - e64) / abs(e64):.2e}, dE/S {abs(et - e64) / S:.2e}); "
         f"force rms rel to fp64 direct {rel_rms(ft, f64):.2e}")
    assert dp < TREE_POT and df < 1e-5
    assert rel_rms(ft, f64) <= 1e-5
    assert abs(et - e64) <= FP32C_E * abs(e64)


@pytest.mark.parametrize("near_rule", [0, 1, 2])
def test_step_graph_replays_match_eager(near_rule):
    """A plan in graph mode captures the step on the second identical call
    and replays it; every replay (new positions each time, eager work and
    synchronisations in between) equals the eager result bitwise.  With the
    sphere near set the graph also holds the mask and list kernels."""
    import torch
    dev = torch.device("cuda:0")
    pos0, q, lo, L = workloads.small_system(2000, (20.0, 20.0, 20.0), 31)
    rng = np.random.default_rng(4)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, near_rule=near_rule)
    stream = torch.cuda.Stream()
    with hs.Plan(params, lo, L) as eager, hs.Plan(params, lo, L) as graphed:
        graphed.set_graph(True)
        x = torch.empty((len(q), 3), dtype=torch.float64, device=dev)
        qq = torch.tensor(q, device=dev)
        en = torch.zeros(1, dtype=torch.float64, device=dev)
        pot = torch.zeros(len(q), dtype=torch.float64, device=dev)
        f = torch.zeros((len(q), 3), dtype=torch.float64, device=dev)
        for it in range(6):
            pos = pos0 + rng.normal(0, 0.05, pos0.shape)
            with torch.cuda.stream(stream):
                x.copy_(torch.tensor(pos, device=dev))
                graphed.compute_device(x, qq, en, pot, f, stream=stream.cuda_stream)
                junk = torch.randn(1000, device=dev).sum()   # eager work on the same stream
            stream.synchronize()
            e_ref, p_ref, f_ref = eager.compute(pos, q)
            assert en.item() == e_ref, it
            assert np.array_equal(pot.cpu().numpy(), p_ref), it
            assert np.array_equal(f.cpu().numpy(), f_ref), it
            del junk
        assert graphed.device_status() == 0


# ---- treecode (near_rule=2): far nodes of the 27-cell sums through their
# multipole expansions, the rest direct.  Sizes cover one tile (no tree
# level), a partial level-1 node, and several levels with ragged ends.
@pytest.mark.parametrize("n", [2, 130, 1000, 4098])
def test_tree_ragged_3d(n):
    L = 3.0 * (n / 2.0) ** (1 / 3) + 2.0
    pos, q, lo, box = workloads.small_system(n, (L, L * 1.1, L * 0.9), 400 + n)
    lo = np.array([0.5, -2.0, 1.0])
    pos = pos + lo
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.4, near_rule=2)
    check(params, pos, q, lo, box, fp32=True, label=f"3d treecode n={n}", pot_bar=TREE_POT)


@pytest.mark.parametrize("order,theta", [(4, 0.25), (6, 0.4), (8, 0.5), (10, 0.5), (12, 0.35)])
def test_tree_orders(order, theta):
    """Every compiled expansion order; the error falls with the order and
    the opening parameter (order 12, theta 0.35 is within the FP32 floor)."""
    pos, q, lo, L = workloads.small_system(3000, (25.0, 25.0, 25.0), 9)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, near_rule=2, tree_order=order, tree_theta=theta)
    e, pot, f, r = check(params, pos, q, lo, L, fp32=True, label=f"treecode order {order} theta {theta}",
                         pot_bar=TREE_POT)
    if order == 12:
        assert rel_rms(f, r.force) <= 1e-6


@pytest.mark.parametrize("gam", [(0.0, 0.0), (-0.94, -0.94), (0.5, -0.3)])
def test_tree_slab(gam):
    """The slab's image layers through the treecode: mirrored images act as
    the node at the mirrored point, scaled by the layer strength."""
    pos, q, lo, L = workloads.small_system(2000, (40.0, 40.0, 20.0), 25, geometry=1)
    params = hs.Params(geometry=1, precision=1, p=8, K=200, F=512, lam=1.6, M=6, gamma_up=gam[0],
                       gamma_low=gam[1], nz=40, near_rule=2)
    check(params, pos, q, lo, L, fp32=True, label=f"slab treecode gamma={gam}", pot_bar=TREE_POT)


def test_c3_slab_treecode_sampled():
    """The 20,000-ion slab with the treecode: against the oracle at 256
    sampled particles and against the FP64 stencil GPU path everywhere."""
    w = workloads.C3
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(8).choice(w.n, 256, replace=False)
    params = hs.Params.from_workload(w)
    params.near_rule = 2
    note("[parity] C3 slab treecode: oracle (sampled)")
    r = _sampled_oracle(w, params, pos, q, lo, L, sample)
    e, pot, f = run_gpu(params, pos, q, lo, L)
    dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
    df = rel_rms(f[sample], r.force)
    note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}")
    assert dp < TREE_POT and df < 1e-5
    e64, pot64, f64 = run_gpu(hs.Params.from_workload(w, precision=0), pos, q, lo, L)
    S = 0.5 * np.abs(q * pot64).sum()
    note(f"   energy tree {e:.12g} fp64 {e64:.12g} rel {abs(e - e64) / abs(e64):.2e}; dE/S {abs(e - e64) / S:.2e}; "
         f"force rms rel {rel_rms(f, f64):.2e}")
    assert abs(e - e64) <= FP32C_E * abs(e64)
    assert rel_rms(f, f64) <= 1e-5


def test_tree_clustered():
    """Strongly non-uniform sources (a tight cluster across a box corner, a
    thin sheet, a uniform rest): elongated and tiny nodes, many close pairs
    through the checked loop."""
    rng = np.random.default_rng(12)
    L = np.array([24.0, 24.0, 24.0])
    a = rng.normal(0.0, 0.6, (1000, 3)) % L                      # around the corner, wrapped
    b = np.column_stack([rng.random(1000) * 24.0, rng.random(1000) * 24.0, 12.0 + rng.normal(0, 0.05, 1000)])
    c = rng.random((1000, 3)) * L
    pos = np.vstack([a, b, c])
    q = np.where(np.arange(3000) % 2 == 0, 1.0, -1.0)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, near_rule=2)
    check(params, pos, q, np.zeros(3), L, fp32=True, label="treecode clustered", pot_bar=TREE_POT)


def test_tree_deterministic():
    pos, q, lo, L = workloads.small_system(3000, (25.0, 25.0, 25.0), 10)
    params = hs.Params(precision=1, p=8, K=162, F=512, lam=1.5, near_rule=2)
    with hs.Plan(params, lo, L) as plan:
        a = plan.compute(pos, q)
        b = plan.compute(pos, q)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_c2_treecode_sampled():
    """The 50,000-ion system with the treecode, in the configuration the
    benchmark times for it: against the oracle at 256 sampled particles
    and against the FP64 27-cell GPU path everywhere."""
    w = workloads.C2
    pos, q, lo, L = workloads.make_system(w)
    sample = np.random.default_rng(7).choice(w.n, 256, replace=False)
    params = hs.Params.from_workload(w)
    params.near_rule = 2
    note("[parity] C2 treecode: oracle (sampled)")
    r = _sampled_oracle(w, params, pos, q, lo, L, sample)
    e, pot, f = run_gpu(params, pos, q, lo, L)
    dp = np.abs(pot[sample] - r.potential).max() / np.abs(r.potential).max()
    df = rel_rms(f[sample], r.force)
    note(f"   sampled: potential max rel {dp:.2e}, force rms rel {df:.2e}")
    assert dp < TREE_POT and df < 1e-5
    e64, pot64, f64 = run_gpu(hs.Params.from_workload(w, precision=0), pos, q, lo, L)
    S = 0.5 * np.abs(q * pot64).sum()
    note(f"   energy tree {e:.12g} fp64 {e64:.12g} rel {abs(e - e64) / abs(e64):.2e}; dE/S {abs(e - e64) / S:.2e}; "
         f"force rms rel {rel_rms(f, f64):.2e}")
    assert abs(e - e64) <= FP32C_E * abs(e64)
    assert rel_rms(f, f64) <= 1e-5
    assert np.abs(pot - pot64).max() <= TREE_POT * np.abs(pot64).max()


@pytest.mark.parametrize("name", ["c2_hsma3d_n50000_fp32c", "c3_hsma2d_n20000_slab"])
def test_near_rules_agree_at_full_size(name):
    """Both near sets are exact splittings of the same potential: the sphere
    near set at p = 14 (K = 450, F = 1152) and the cell/layer stencil at the
    workload's p = 10 give the same forces to the 1e-5 bar (FP64 paths;
    measured 9e-6 on the 50,000-ion system, 4.5e-6 on the slab)."""
    import dataclasses
    w = workloads.CONFIGS[name]
    pos, q, lo, L = workloads.make_system(w)
    with hs.Plan(hs.Params.from_workload(w, precision=0), lo, L) as plan:
        _, _, f0 = plan.compute(pos, q)
    ws = dataclasses.replace(w, near_rule=1, p=14, K=450, F=1152)
    with hs.Plan(hs.Params.from_workload(ws, precision=0), lo, L) as plan:
        _, _, f1 = plan.compute(pos, q)
    d = rel_rms(f1, f0)
    note(f"[rules] {name}: sphere p=14 vs stencil p=10 force rms rel {d:.2e}")
    assert d < 1.5e-5
