"""Serving form on the GPU: continuous batching of independent systems."""
import sys

import numpy as np
import pytest

import workloads
from oracle import hsma as ohsma

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2104_05260_amd")

UNIT = (1.0, 1.0, 1.0)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mix(count=6, seed0=2000, n_lo=300, n_hi=3000):
    """Serving-shaped systems: N uniform, L = (N / 0.05)^(1/3), +-1."""
    ws = workloads.serving_systems(count, n_lo, n_hi, seed0=seed0)
    out = []
    for w in ws:
        pos, q, lo, L = workloads.make_system(w)
        out.append((w, pos + 1.5, q, lo + 1.5, L[0]))
    return ws[0], out


def params(prec=1):
    return hs.Params(precision=prec, p=8, K=162, F=512, lam=1.5)


def test_alone_equals_mix_bitwise():
    w0, systems = mix()
    nmax = max(len(q) for _, _, q, _, _ in systems)
    note(f"[serving] {len(systems)} systems, n up to {nmax}")
    with hs.Server(params(), UNIT, max_n=nmax, max_slots=4) as sv:
        alone = []
        for _, pos, q, lo, L in systems:
            alone.append(sv.wait(sv.submit(pos, q, lo, L)))
        tickets = [sv.submit(pos, q, lo, L) for _, pos, q, lo, L in systems]
        together = [sv.wait(t) for t in tickets]
    slots_used = {r["slot"] for r in together}
    note(f"   slots used in the mix: {sorted(slots_used)}")
    assert len(slots_used) > 1
    for a, b in zip(alone, together):
        assert a["status"] == 0 and b["status"] == 0
        assert a["energy"] == b["energy"]
        assert np.array_equal(a["potential"], b["potential"]) and np.array_equal(a["force"], b["force"])


@pytest.mark.parametrize("prec", [0, 1])
def test_served_results_match_plan_and_oracle(prec):
    _, systems = mix(count=3, seed0=2100)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    with hs.Server(params(prec), UNIT, max_n=nmax, max_slots=3) as sv:
        tickets = [sv.submit(pos, q, lo, L) for _, pos, q, lo, L in systems]
        res = [sv.wait(t) for t in tickets]
    for (w, pos, q, lo, L), r in zip(systems, res):
        ref = ohsma.hsma3d(pos, q, lo, np.array([L, L, L]), 8, 162, 512, 1.5)
        with hs.Plan(params(prec), lo, [L, L, L]) as plan:
            e1, p1, f1 = plan.compute(pos, q)
        de = abs(r["energy"] - ref.energy)
        S = 0.5 * np.abs(q * ref.potential).sum()
        df = np.sqrt(((r["force"] - ref.force) ** 2).sum() / (ref.force ** 2).sum())
        note(f"   n={len(q)} L={L:.3f}: energy {r['energy']:.12g} oracle {ref.energy:.12g} dE/S {de / S:.2e} "
             f"force rel {df:.2e}; vs direct plan dE {abs(r['energy'] - e1):.2e}")
        if prec == 0:
            assert de <= 1e-10 * S and df <= 1e-10
        else:
            assert de <= 1e-6 * abs(ref.energy) + 1e-7 * S and df <= 1e-5  # FP32 pair-term floor
        # a server slot re-targets a unit-box plan; a plan built for the box
        # itself agrees to rounding
        assert abs(r["energy"] - e1) <= 1e-10 * S
        assert np.abs(r["force"] - f1).max() <= 1e-6 * np.abs(f1).max()


def test_budget_and_per_request_errors():
    _, systems = mix(count=4, seed0=2200)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    with hs.Server(params(), UNIT, max_n=nmax, max_slots=8) as probe:
        n_full, per = probe.slots()
    note(f"   bytes per slot {per}, slots with default budget {n_full}")
    # a budget of two slots admits two requests at a time; everything completes
    with hs.Server(params(), UNIT, max_n=nmax, max_slots=8, hbm_budget=2 * per + per // 2) as sv:
        assert sv.slots()[0] == 2
        big = np.zeros((nmax + 1, 3))
        qbig = np.zeros(nmax + 1)
        with pytest.raises(hs.HSMAError) as e:
            sv.submit(big, qbig, (0, 0, 0), 10.0)
        assert e.value.name == "HSMA_ERR_OOM"
        w, pos, q, lo, L = systems[0]
        with pytest.raises(hs.HSMAError) as e:
            sv.submit(pos, q + 0.5, lo, L)
        assert e.value.name == "HSMA_ERR_NOT_NEUTRAL"
        tickets = [sv.submit(pos, q, lo, L) for _, pos, q, lo, L in systems]
        res = [sv.wait(t) for t in tickets]
        assert all(r["status"] == 0 for r in res)
        assert {r["slot"] for r in res} <= {0, 1}
    with pytest.raises(hs.HSMAError) as e:
        hs.Server(params(), UNIT, max_n=nmax, max_slots=2, hbm_budget=per // 2)
    assert e.value.name == "HSMA_ERR_OOM"


def test_shutdown_cancels_queued_requests():
    _, systems = mix(count=3, seed0=2300, n_lo=2000, n_hi=3000)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    sv = hs.Server(params(0), UNIT, max_n=nmax, max_slots=1)
    tickets = []
    for _ in range(10):
        for _, pos, q, lo, L in systems:
            tickets.append(sv.submit(pos, q, lo, L))
    sv.shutdown()
    with pytest.raises(hs.HSMAError) as e:
        sv.submit(systems[0][1], systems[0][2], systems[0][3], systems[0][4])
    assert e.value.name == "HSMA_ERR_CANCELLED"
    codes = [sv.wait(t)["status"] for t in tickets]
    note(f"   statuses after shutdown: {codes.count(0)} done, {codes.count(-10)} cancelled")
    assert set(codes) <= {0, -10} and codes.count(-10) >= 1
    sv.close()


def test_served_sphere_near_set():
    """The sphere near set through the server: FP64 results agree with the
    oracle to the parity bar, and every result is the same alone and in the
    mix."""
    _, systems = mix(count=3, seed0=2200)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    prm = params(0)
    prm.near_rule = 1
    with hs.Server(prm, UNIT, max_n=nmax, max_slots=3) as sv:
        alone = [sv.wait(sv.submit(pos, q, lo, L)) for _, pos, q, lo, L in systems]
        tickets = [sv.submit(pos, q, lo, L) for _, pos, q, lo, L in systems]
        together = [sv.wait(t) for t in tickets]
    for (w, pos, q, lo, L), a, b in zip(systems, alone, together):
        assert a["status"] == 0 and b["status"] == 0
        assert a["energy"] == b["energy"] and np.array_equal(a["force"], b["force"])
        ref = ohsma.hsma3d(pos, q, lo, np.array([L, L, L]), 8, 162, 512, 1.5, near_rule=1)
        S = 0.5 * np.abs(q * ref.potential).sum()
        df = np.sqrt(((b["force"] - ref.force) ** 2).sum() / (ref.force ** 2).sum())
        note(f"   sphere near set n={len(q)}: dE/S {abs(b['energy'] - ref.energy) / S:.2e} force rel {df:.2e}")
        assert abs(b["energy"] - ref.energy) <= 1e-10 * S and df <= 1e-10


def test_served_treecode():
    """The treecode (near rule 2, FP32C) through the server: results within
    the FP32 bars of the oracle's exact 27-cell sums (5e-5 on the largest
    potential error, the treecode's truncation), and every result the same
    alone and in the mix."""
    _, systems = mix(count=3, seed0=2300)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    prm = params(1)
    prm.near_rule = 2
    with hs.Server(prm, UNIT, max_n=nmax, max_slots=3) as sv:
        alone = [sv.wait(sv.submit(pos, q, lo, L)) for _, pos, q, lo, L in systems]
        tickets = [sv.submit(pos, q, lo, L) for _, pos, q, lo, L in systems]
        together = [sv.wait(t) for t in tickets]
    for (w, pos, q, lo, L), a, b in zip(systems, alone, together):
        assert a["status"] == 0 and b["status"] == 0
        assert a["energy"] == b["energy"] and np.array_equal(a["force"], b["force"])
        ref = ohsma.hsma3d(pos, q, lo, np.array([L, L, L]), 8, 162, 512, 1.5)
        S = 0.5 * np.abs(q * ref.potential).sum()
        df = np.sqrt(((b["force"] - ref.force) ** 2).sum() / (ref.force ** 2).sum())
        dp = np.abs(b["potential"] - ref.potential).max() / np.abs(ref.potential).max()
        note(f"   treecode n={len(q)}: dE/S {abs(b['energy'] - ref.energy) / S:.2e} force rel {df:.2e} "
             f"potential max rel {dp:.2e}")
        assert abs(b["energy"] - ref.energy) <= 1e-6 * abs(ref.energy) + 1e-7 * S
        assert df <= 1e-5 and dp <= 5e-5


def _noncubic_params(prec=1, lsq=0):
    # lambda 1.3: the sphere must stay inside the near cells of the shortest edge
    return hs.Params(precision=prec, p=10, K=242, F=800, lam=1.3, lsq_solver=lsq)


def _noncubic_system(n, L, seed):
    box = (L, 1.2 * L, 0.9 * L)
    pos, q, lo, _ = workloads.small_system(n, box, seed)
    return pos + 0.7, q, lo + 0.7, box


def test_two_class_mix_bitwise_and_oracle():
    """Per-request parameters and box shapes through one server: p = 8 in
    cubic boxes (the server's default class) and p = 10 in 1 : 1.2 : 0.9
    boxes, two plan classes; every result is the same alone and in the mix
    and agrees with the oracle (FP64 path, 1e-10)."""
    _, cubic = mix(count=3, seed0=2400, n_lo=400, n_hi=1600)
    other = [_noncubic_system(n, (n / 0.05) ** (1 / 3), 2500 + n) for n in (700, 1300)]
    nmax = max([len(q) for _, _, q, _, _ in cubic] + [len(q) for _, q, _, _ in other])
    prm_b = _noncubic_params(prec=0)

    def submit_all(sv):
        t = [sv.submit(pos, q, lo, L) for _, pos, q, lo, L in cubic]
        t += [sv.submit(pos, q, lo, box_len=box, params=prm_b) for pos, q, lo, box in other]
        return t

    with hs.Server(params(0), UNIT, max_n=nmax, max_slots=4) as sv:
        alone = [sv.wait(t) for t in submit_all(sv)]
        together_t = submit_all(sv)
        together = [sv.wait(t) for t in together_t]
        st = sv.stats()
    note(f"   server stats {st}; classes of the results {[r['plan_class'] for r in together]}")
    assert st["classes"] == 2
    assert [r["plan_class"] for r in together] == [0, 0, 0, 1, 1]
    for a, b in zip(alone, together):
        assert a["status"] == 0 and b["status"] == 0
        assert a["energy"] == b["energy"] and np.array_equal(a["force"], b["force"])
    refs = [ohsma.hsma3d(pos, q, lo, np.array([L, L, L]), 8, 162, 512, 1.5) for _, pos, q, lo, L in cubic]
    refs += [ohsma.hsma3d(pos, q, lo, np.array(box), 10, 242, 800, 1.3) for pos, q, lo, box in other]
    qs = [q for _, _, q, _, _ in cubic] + [q for _, q, _, _ in other]
    for r, ref, q in zip(together, refs, qs):
        S = 0.5 * np.abs(q * ref.potential).sum()
        df = np.sqrt(((r["force"] - ref.force) ** 2).sum() / (ref.force ** 2).sum())
        note(f"   n={len(q)} class {r['plan_class']}: dE/S {abs(r['energy'] - ref.energy) / S:.2e} force rel {df:.2e}")
        assert abs(r["energy"] - ref.energy) <= 1e-10 * S and df <= 1e-10


def test_one_slot_alternating_classes():
    """One slot whose two plan classes share its arena: the same request
    before and after a request of the other class gives bitwise the same
    result (each plan uploads its check schedule again after the other
    class has used the arena), and the repeated request's result equals
    that of a server that runs it alone."""
    _, cubic = mix(count=1, seed0=2600, n_lo=900, n_hi=900)
    other = _noncubic_system(1100, (1100 / 0.05) ** (1 / 3), 2601)
    _, pos_a, q_a, lo_a, L_a = cubic[0]
    pos_b, q_b, lo_b, box_b = other
    prm_b = _noncubic_params(prec=1)
    nmax = max(len(q_a), len(q_b))
    with hs.Server(params(1), UNIT, max_n=nmax, max_slots=1, classes=[(prm_b, tuple(np.array(box_b) / box_b[0]))]) as sv:
        seq = []
        for k in range(3):
            ra = sv.wait(sv.submit(pos_a, q_a, lo_a, L_a))
            rb = sv.wait(sv.submit(pos_b, q_b, lo_b, box_len=box_b, params=prm_b))
            seq.append((ra, rb))
        st = sv.stats()
    with hs.Server(params(1), UNIT, max_n=nmax, max_slots=1) as sv:
        alone = sv.wait(sv.submit(pos_a, q_a, lo_a, L_a))
    note(f"   server stats {st}; classes {[(a['plan_class'], b['plan_class']) for a, b in seq]}")
    assert all(a["status"] == 0 and b["status"] == 0 for a, b in seq)
    assert all(a["plan_class"] == 0 and b["plan_class"] == 1 for a, b in seq)
    for a, b in seq[1:]:
        assert a["energy"] == seq[0][0]["energy"] and np.array_equal(a["force"], seq[0][0]["force"])
        assert b["energy"] == seq[0][1]["energy"] and np.array_equal(b["force"], seq[0][1]["force"])
    assert alone["energy"] == seq[0][0]["energy"] and np.array_equal(alone["force"], seq[0][0]["force"])


def test_device_resident_replicas_replay_graphs():
    """Device-resident requests: positions and charges stay in HBM and the
    outputs are written in place; the results equal the host requests'
    bitwise.  Replicas resubmitted with their system ids return to their
    slots, and from the third round on each step is a graph replay that
    still reads the updated positions."""
    import torch
    dev = torch.device("cuda:0")
    _, systems = mix(count=4, seed0=2600, n_lo=600, n_hi=2400)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    reps = []
    for _, pos, q, lo, L in systems:
        n = len(q)
        reps.append(dict(x=torch.tensor(pos, device=dev), q=torch.tensor(q, device=dev), lo=lo, L=L,
                         pot=torch.zeros(n, dtype=torch.float64, device=dev),
                         f=torch.zeros((n, 3), dtype=torch.float64, device=dev),
                         e=torch.zeros(1, dtype=torch.float64, device=dev)))
    rng = np.random.default_rng(5)
    # the host-request references run on a second server, so that the
    # replicas' slots see only their own systems
    ref_sv = hs.Server(params(1), UNIT, max_n=nmax, max_slots=2)
    with hs.Server(params(1), UNIT, max_n=nmax, max_slots=4) as sv:
        for rnd in range(4):
            torch.cuda.synchronize()  # the inputs are complete before submit
            tickets = [sv.submit_device(r["x"], r["q"], r["lo"], r["L"], potential=r["pot"], force=r["f"],
                                        energy=r["e"], system_id=i + 1) for i, r in enumerate(reps)]
            res = [sv.wait(t) for t in tickets]
            for i, (r, out) in enumerate(zip(reps, res)):
                assert out["status"] == 0
                if rnd >= 2:
                    assert out["replayed"] == 1
                # the same configuration as a host request: bitwise equal
                href = ref_sv.wait(ref_sv.submit(r["x"].cpu().numpy(), r["q"].cpu().numpy(), r["lo"], r["L"]))
                assert href["energy"] == out["energy"] == r["e"].item()
                assert np.array_equal(href["force"], r["f"].cpu().numpy())
                assert np.array_equal(href["potential"], r["pot"].cpu().numpy())
            note(f"   round {rnd}: slots {[o['slot'] for o in res]} replayed {[o['replayed'] for o in res]}")
            # move every replica on the device (as an MD or MC step would)
            for r in reps:
                r["x"] += torch.tensor(rng.normal(0, 0.01, tuple(r["x"].shape)), device=dev)
        st = sv.stats()
    ref_sv.close()
    note(f"   stats {st}")
    assert st["graph_replays"] >= 8 and st["affinity_hits"] >= 8


def test_more_replicas_than_slots_replay():
    """Twelve device-resident replicas on four slots, all submitted at once
    each round: a slot keeps the steps of its last eight systems, and a
    replica goes preferably to a free slot that recently ran it, so from
    the third round on most steps are replays; every result stays equal to
    the same replica served by a server of its own (bitwise)."""
    import torch
    dev = torch.device("cuda:0")
    _, systems = mix(count=12, seed0=2700, n_lo=300, n_hi=1500)
    nmax = max(len(q) for _, _, q, _, _ in systems)
    reps = [dict(x=torch.tensor(pos, device=dev), q=torch.tensor(q, device=dev), lo=lo, L=L,
                 f=torch.zeros((len(q), 3), dtype=torch.float64, device=dev),
                 e=torch.zeros(1, dtype=torch.float64, device=dev)) for _, pos, q, lo, L in systems]
    with hs.Server(params(1), UNIT, max_n=nmax, max_slots=4) as sv:
        replayed = []
        for rnd in range(5):
            torch.cuda.synchronize()
            tickets = [sv.submit_device(r["x"], r["q"], r["lo"], r["L"], force=r["f"], energy=r["e"],
                                        system_id=i + 1) for i, r in enumerate(reps)]
            res = [sv.wait(t) for t in tickets]
            assert all(o["status"] == 0 for o in res)
            replayed.append(sum(o["replayed"] for o in res))
            note(f"   round {rnd}: slots {[o['slot'] for o in res]} replayed {[o['replayed'] for o in res]}")
        st = sv.stats()
        energies = [r["e"].item() for r in reps]
        forces = [r["f"].cpu().numpy() for r in reps]
    note(f"   stats {st}")
    with hs.Server(params(1), UNIT, max_n=nmax, max_slots=1) as ref:
        for r, e, f in zip(reps, energies, forces):
            out = ref.wait(ref.submit(r["x"].cpu().numpy(), r["q"].cpu().numpy(), r["lo"], r["L"], potential=False))
            assert out["energy"] == e and np.array_equal(out["force"], f)
    # (arrival order and sizes repeat each round, so the slots' histories
    # mostly hold their replicas; at least a quarter of the steps must hit)
    assert st["affinity_hits"] >= 12
    assert sum(replayed[2:]) >= 9


@pytest.mark.parametrize("case", ["3d_p6", "3d_p10", "3d_p12_K800", "noncubic_p8", "slab_p10"])
def test_device_lsq_matches_host_qr(case):
    """The fit's pseudo-inverse from the device CholeskyQR2 (FP64 Gram
    matrices on the matrix cores) against the host Householder QR: the
    folded maps Praw agree to 1e-9 of their largest entry (condition numbers
    up to 1e4), the condition estimates to 1e-6."""
    box = (10.0, 10.0, 10.0)
    if case == "3d_p6":
        kw = dict(p=6, K=100, F=200, lam=1.5)
    elif case == "3d_p10":
        kw = dict(p=10, K=400, F=800, lam=1.5)
    elif case == "3d_p12_K800":
        kw = dict(p=12, K=800, F=1152, lam=1.5)
    elif case == "noncubic_p8":
        kw = dict(p=8, K=162, F=512, lam=1.3)
        box = (10.0, 12.0, 9.0)
    else:
        kw = dict(geometry=1, p=10, K=400, F=800, lam=1.6, M=6, gamma_up=-0.94, gamma_low=-0.94, nz=40)
        box = (40.0, 40.0, 20.0)
    ph = hs.HostPlan(hs.Params(**kw, lsq_solver=0), (0, 0, 0), box)
    pd = hs.HostPlan(hs.Params(**kw, lsq_solver=1), (0, 0, 0), box)
    a, b = ph.get("Praw"), pd.get("Praw")
    ca, cb = ph.get("scalars")[3], pd.get("scalars")[3]
    err = np.abs(a - b).max() / np.abs(a).max()
    note(f"   {case}: Praw rel diff {err:.2e}; cond host {ca:.4g} device {cb:.4g}")
    assert err <= 1e-9 and abs(ca - cb) <= 1e-6 * ca


def test_server_classes_grouped_device_lsq():
    """Classes declared at server creation with the device solver: their
    factorisations run together (grouped launches).  Results agree with
    plans built by the host QR to 1e-10 (FP64 path)."""
    decl = [(hs.Params(precision=0, p=6, K=100, F=200, lam=1.5, lsq_solver=1), (1.0, 1.0, 1.0)),
            (hs.Params(precision=0, p=10, K=242, F=800, lam=1.3, lsq_solver=1), (1.0, 1.2, 0.9)),
            (hs.Params(precision=0, p=8, K=200, F=512, lam=1.6, lsq_solver=1, geometry=1, M=6, gamma_up=-0.5,
                       gamma_low=0.3, nz=40), (2.0, 2.0, 1.0))]
    systems = [workloads.small_system(800, (20.0, 20.0, 20.0), 71),
               workloads.small_system(900, (20.0, 24.0, 18.0), 72),
               workloads.small_system(1000, (30.0, 30.0, 15.0), 73, geometry=1)]
    boxes = [(20.0, 20.0, 20.0), (20.0, 24.0, 18.0), (30.0, 30.0, 15.0)]
    with hs.Server(decl[0][0], decl[0][1], max_n=1000, max_slots=3, classes=decl[1:]) as sv:
        assert sv.stats()["classes"] == 3
        tickets = [sv.submit(pos, q, lo, box_len=box, params=prm)
                   for (prm, _), (pos, q, lo, _), box in zip(decl, systems, boxes)]
        res = [sv.wait(t) for t in tickets]
        assert sv.stats()["classes"] == 3
    for (prm, _), (pos, q, lo, _), box, r in zip(decl, systems, boxes, res):
        import dataclasses
        with hs.Plan(dataclasses.replace(prm, lsq_solver=0), lo, box) as plan:
            e, pot, f = plan.compute(pos, q)
        df = np.sqrt(((r["force"] - f) ** 2).sum() / (f ** 2).sum())
        note(f"   class {r['plan_class']} n={len(q)}: energy {r['energy']:.15g} host-QR plan {e:.15g} force rel {df:.2e}")
        assert r["status"] == 0 and abs(r["energy"] - e) <= 1e-10 * abs(e) and df <= 1e-10


def test_served_parity_at_mix_sizes():
    """Served FP32C results at the serving mix's largest sizes (about 20,000
    and 12,000 ions) against the oracle at 96 sampled ions (its check sums
    and fit use every ion), and the served FP32C energy against the served
    FP64 energy to 1e-6."""
    ws = [w for w in workloads.serving_systems(256) if w.n >= 12000][:2]
    systems = []
    for w in ws:
        pos, q, lo, L = workloads.make_system(w)
        systems.append((pos, q, lo, L[0]))
    nmax = max(len(q) for _, q, _, _ in systems)
    out = {}
    for prec in (1, 0):
        with hs.Server(params(prec), UNIT, max_n=nmax, max_slots=2) as sv:
            tickets = [sv.submit(pos, q, lo, L) for pos, q, lo, L in systems]
            out[prec] = [sv.wait(t) for t in tickets]
    for (pos, q, lo, L), r32, r64 in zip(systems, out[1], out[0]):
        sample = np.random.default_rng(len(q)).choice(len(q), 96, replace=False)
        note(f"[serving] oracle at n={len(q)} (sampled)")
        ref = ohsma.hsma3d(pos, q, lo, np.array([L, L, L]), 8, 162, 512, 1.5, targets=sample)
        dp = np.abs(r32["potential"][sample] - ref.potential).max() / np.abs(ref.potential).max()
        df = np.sqrt(((r32["force"][sample] - ref.force) ** 2).sum() / (ref.force ** 2).sum())
        dp64 = np.abs(r64["potential"][sample] - ref.potential).max() / np.abs(ref.potential).max()
        de = abs(r32["energy"] - r64["energy"]) / abs(r64["energy"])
        note(f"   n={len(q)}: fp32c potential max rel {dp:.2e} force rms rel {df:.2e}; fp64 potential {dp64:.2e}; "
             f"energy fp32c vs fp64 {de:.2e}")
        assert dp <= 1e-5 and df <= 1e-5 and dp64 <= 1e-10 and de <= 1e-6
