#!/usr/bin/env python3
"""Benchmark of the HSMA hot path on one MI355X.

One step = one full evaluation (energy, potentials, forces) of the largest
single-GPU system: 999,999 ions of a 2:1 electrolyte (+2 / -1) in a periodic
box L = 200, p = 12, F = 1152, K = 800, lambda 1.5, 27 near cells summed
directly, in the FP32-compensated path, inputs resident in HBM: ingest and
sort, check-point sums, least-squares fit, sphere sources, particle near-set
and sphere sums, forces and energy.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]

Besides the throughput it reports the dominant kernel's roofline position
(FP32 VALU bound; algorithmic 20 flop per near pair over its HIP-event
duration), the error against the FP64 GPU path on the same system and that
path's speed, the same system with the 27 cells summed by the treecode, the
50,000-ion system (27 cells; its FP64 path, the sphere near set, the
treecode, the slab's near sets), and the FP64 CPU oracle timed as a CPU
baseline (a bounded sample scaled to the step).  With --serving it also
measures the request server (serving mix, device-resident replicas, an MD
ensemble); that part is off by default.

For profiling, the same timed loop runs alone on any named configuration,
optionally with another near set and other p, K, F:

  python bench.py --workload c2_hsma3d_n50000_fp32c
  python bench.py --workload c3_hsma2d_n20000_slab [--near-rule 1 --p 14 --K 450 --F 1152]
  python bench.py --workload c5_hsma3d_n999999_2to1 --near-rule 2   (treecode)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak (published)
PEAK_FP64_TFLOPS = 78.6           # MI355X FP64 vector peak (published)
FLOP_PER_NEAR_PAIR = 20           # algorithmic convention for one Coulomb pair (potential + field)


def progress(msg: str):
    """One line per phase on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2104_05260_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ent = t.get(kernel, {}).get(workload)
    if not ent or ent.get("kernels_hip_sha256_16") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def measured_valu(kernel: str, workload: str):
    """FP32 and FP64 VALU flop per launch of `kernel` from the committed
    rocprofv3 counter summary (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32/F64
    x 64 lanes, FMA counted twice), if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "valu_counters.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ent = t.get(kernel, {}).get(workload)
    if not ent or ent.get("kernels_hip_sha256_16") != kernel_source_hash():
        return None
    return ent


def tree_roofline(workload: str, launch_ms: float):
    """Position of the treecode's particle kernel (k_tree_far, the dominant
    kernel of near rule 2): its VALU flop per launch from the committed
    counters over its live HIP-event duration, and its HBM bytes per
    launch from the committed FETCH_SIZE / WRITE_SIZE counters.  Its work
    is not a fixed count of pair terms (accepted nodes and opened tiles
    depend on the configuration), so the flop count is what the kernel
    issued.  frac is
    the share of the VALU peak: FP32 flop at 157.3 TFLOP/s plus FP64 flop
    at 78.6 TFLOP/s."""
    c = measured_valu("k_tree_far_particles", workload)
    out = {"kernel": "k_tree_far<P,false,false> (treecode sums at the particles)", "bound": "alu",
           "launch_ms": launch_ms, "peak": PEAK_FP32_TFLOPS, "fp64_peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
           "traffic": measured_traffic("k_tree_far_particles", workload)}
    if c is None or not launch_ms:
        out.update({"achieved": None, "frac": None, "flop_source": "no counters for this kernel source"})
        return out
    a32 = c["fp32_flop_per_launch"] / (launch_ms * 1e-3) / 1e12
    a64 = c["fp64_flop_per_launch"] / (launch_ms * 1e-3) / 1e12
    out.update({"achieved": a32, "fp64_achieved": a64, "frac": a32 / PEAK_FP32_TFLOPS + a64 / PEAK_FP64_TFLOPS,
                "fp32_flop_per_launch": c["fp32_flop_per_launch"], "fp64_flop_per_launch": c["fp64_flop_per_launch"],
                "flop_source": "rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32/F64 of one launch, x 64 lanes "
                               "(FMA x 2), profiles/valu_counters.json"})
    return out


def cpu_baseline(w, pos, q, lo, L, sample_n=4096, full_limit_s=30.0):
    """The FP64 oracle timed on the same step.  First its fixed part
    (check-point sums over all particles, least-squares fit, sphere
    sources) and the particle sums at `sample_n` particles give an
    estimate linear in the number of particles evaluated; when that
    estimate is within `full_limit_s`, one full step (every particle) is
    then measured and reported, else the estimate is.  A first, untimed
    call keeps one-time start-up costs out of the fixed part, where they
    would bias the estimate low."""
    import numpy as np
    from oracle import hsma as ohsma

    # the treecode (near rule 2) approximates the cell stencil's sums: the
    # oracle computes those sums exactly (near rule 0)
    near = 0 if w.near_rule == 2 else w.near_rule

    def run(targets):
        # the oracle on the arrays already generated (generation is not timed)
        if w.geometry == 0:
            return ohsma.hsma3d(pos, q, lo, L, w.p, w.K, w.F, w.lam, w.Fw, w.surface_rule, targets, near)
        return ohsma.hsma2d(pos, q, lo, L, w.p, w.K, w.F, w.lam, w.M, w.gamma_up, w.gamma_low, w.nz,
                            w.Fw, w.surface_rule, targets, near)

    rng = np.random.default_rng(11)
    run(np.arange(1))  # untimed: loads the oracle's C sums and warms its caches
    t0 = time.perf_counter()
    run(np.arange(1))
    t1 = time.perf_counter()
    sample = rng.choice(w.n, sample_n, replace=False)
    run(sample)
    t2 = time.perf_counter()
    fixed = t1 - t0
    per_particle = max((t2 - t1) - fixed, 1e-9) / (sample_n - 1)
    est_step = fixed + per_particle * w.n
    if est_step <= full_limit_s:
        t3 = time.perf_counter()
        r = run(None)
        step = time.perf_counter() - t3
        assert np.isfinite(r.energy)
        how = (f"FP64 oracle: one full step (all {w.n} particles: check sums, fit, sphere sources, "
               f"particle sums, energy) measured, {step:.1f} s (a {sample_n}-particle sample had estimated "
               f"{est_step:.1f} s)")
    else:
        step = est_step
        how = (f"FP64 oracle: fixed part (all check sums + fit + sphere sources) {fixed:.2f} s measured, "
               f"particle sums at {sample_n} sampled particles measured and scaled to all {w.n}; "
               f"estimated {est_step:.1f} s per step")
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    if near != w.near_rule:
        how += "; the GPU step sums the cell stencil by the treecode, the oracle sums it directly"
    return {
        "value": w.n / step, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
        "cpu_model": model, "nproc": os.cpu_count(), "sample": how,
    }


def serving_bench(hs, workloads, n_systems=256, slots=8, loads=(0.5, 0.8, 0.95), seed=77):
    """The serving mix: independent cubic systems (N uniform in [500, 20000],
    L = (N/0.05)^(1/3), +-1, p 8, F 512, K 162) through the continuous
    batching server.  Saturated throughput with every request queued at
    once, the same with one slot (no overlap), then Poisson arrivals at
    fractions of the saturated rate with p50/p99 submit-to-result latency."""
    import numpy as np
    ws = workloads.serving_systems(n_systems)
    systems = []
    for w in ws:
        pos, q, lo, L = workloads.make_system(w)
        systems.append((pos, q, lo, L[0]))
    nmax = max(len(q) for _, q, _, _ in systems)
    total_particles = sum(len(q) for _, q, _, _ in systems)
    prm = hs.Params(precision=hs.FP32C, p=8, K=162, F=512, lam=1.5)
    out = {"systems": n_systems, "particles": total_particles, "n_range": [min(len(q) for _, q, _, _ in systems), nmax]}

    def run_all(sv):
        t0 = time.perf_counter()
        tickets = [sv.submit(pos, q, lo, L, potential=False) for pos, q, lo, L in systems]
        res = [sv.wait(t) for t in tickets]
        dt = time.perf_counter() - t0
        assert all(r["status"] == 0 for r in res)
        return dt, res

    progress("serving: one slot")
    with hs.Server(prm, (1.0, 1.0, 1.0), max_n=nmax, max_slots=1) as sv1:
        run_all(sv1)  # warm-up
        dt1, _ = run_all(sv1)
    progress(f"serving: {slots} slots, saturated then Poisson arrivals")
    with hs.Server(prm, (1.0, 1.0, 1.0), max_n=nmax, max_slots=slots) as sv:
        nslots, per = sv.slots()
        run_all(sv)  # warm-up
        dt, res = run_all(sv)
        rate = n_systems / dt
        out.update({"slots": nslots, "bytes_per_slot": per,
                    "saturated_requests_per_s": rate, "saturated_particle_steps_per_s": total_particles / dt,
                    "one_slot_requests_per_s": n_systems / dt1, "batching_speedup": dt1 / dt})
        rng = np.random.default_rng(seed)
        out["poisson"] = []
        for f in loads:
            lam = f * rate
            gaps = rng.exponential(1.0 / lam, n_systems)
            order = rng.permutation(n_systems)
            t0 = time.perf_counter()
            arrivals = t0 + np.cumsum(gaps)
            tickets = []
            for k, i in enumerate(order):
                delay = arrivals[k] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                pos, q, lo, L = systems[i]
                tickets.append(sv.submit(pos, q, lo, L, potential=False))
            rs = [sv.wait(t) for t in tickets]
            lat = np.array([r["t_done"] - r["t_submit"] for r in rs]) * 1e3
            span = max(r["t_done"] for r in rs) - min(r["t_submit"] for r in rs)
            out["poisson"].append({"offered_fraction": f, "offered_requests_per_s": lam,
                                   "achieved_requests_per_s": n_systems / span,
                                   "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))})
    # the same mix with the stencil summed by the treecode (saturated rate)
    prm2 = hs.Params(precision=hs.FP32C, p=8, K=162, F=512, lam=1.5, near_rule=2)
    progress("serving: treecode")
    with hs.Server(prm2, (1.0, 1.0, 1.0), max_n=nmax, max_slots=slots) as sv:
        run_all(sv)  # warm-up
        dt2, _ = run_all(sv)
        out["treecode"] = {"saturated_requests_per_s": n_systems / dt2,
                           "saturated_particle_steps_per_s": total_particles / dt2}
    # two plan classes in one server: half the systems at p = 8 in cubic
    # boxes, half at p = 10 in 1 : 1.2 : 0.9 boxes (lambda 1.3), host requests
    prm_b = hs.Params(precision=hs.FP32C, p=10, K=242, F=800, lam=1.3)
    progress("serving: two plan classes")
    with hs.Server(prm, (1.0, 1.0, 1.0), max_n=nmax, max_slots=slots, classes=[(prm_b, (1.0, 1.2, 0.9))]) as sv:
        def run_two():
            t0 = time.perf_counter()
            tk = []
            for k, (pos, q, lo, L) in enumerate(systems):
                if k % 2 == 0:
                    tk.append(sv.submit(pos, q, lo, L, potential=False))
                else:
                    box = (L, 1.2 * L, 0.9 * L)
                    tk.append(sv.submit(pos * np.array([1.0, 1.2, 0.9]), q, lo, box_len=box, params=prm_b,
                                        potential=False))
            rs = [sv.wait(t) for t in tk]
            assert all(r["status"] == 0 for r in rs)
            return time.perf_counter() - t0
        run_two()
        dt3 = run_two()
        out["two_classes"] = {"classes": sv.stats()["classes"], "saturated_requests_per_s": n_systems / dt3,
                              "saturated_particle_steps_per_s": total_particles / dt3,
                              "mix": "p 8 cubic and p 10 in 1 : 1.2 : 0.9 boxes, alternating"}
    out["replicas"] = replica_bench(hs, workloads, slots=slots, loads=loads, seed=seed)
    return out


def replica_bench(hs, workloads, n_rep=64, rounds=6, slots=8, loads=(0.5, 0.8, 0.95), seed=78):
    """Device-resident replicas (Monte Carlo / MD ensembles): the first
    n_rep systems of the serving mix stay in HBM; every round submits each
    replica once as a device request with its system id (after a small move
    of its positions on the device), so its slot replays a captured step.
    Saturated rounds, then Poisson arrivals at fractions of that rate with
    p50/p99 latency; graph replays and slot-affinity hits counted by the
    server."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    ws = workloads.serving_systems(n_rep)
    reps = []
    for w in ws:
        pos, q, lo, L = workloads.make_system(w)
        reps.append(dict(x=torch.tensor(pos, device=dev), q=torch.tensor(q, device=dev), lo=lo, L=L[0],
                         f=torch.zeros((w.n, 3), dtype=torch.float64, device=dev)))
    nmax = max(w.n for w in ws)
    total = sum(w.n for w in ws)
    prm = hs.Params(precision=hs.FP32C, p=8, K=162, F=512, lam=1.5)
    gen = torch.Generator(device=dev).manual_seed(seed)

    def move():
        for r in reps:  # every replica moves a little on the device
            r["x"].add_(torch.randn(r["x"].shape, generator=gen, device=dev, dtype=torch.float64), alpha=1e-3)
            r["x"].remainder_(r["L"])
        torch.cuda.synchronize()

    def round_(sv):
        move()
        t0 = time.perf_counter()
        tk = [sv.submit_device(r["x"], r["q"], r["lo"], r["L"], force=r["f"], system_id=i + 1)
              for i, r in enumerate(reps)]
        rs = [sv.wait(t) for t in tk]
        assert all(r["status"] == 0 for r in rs)
        return time.perf_counter() - t0, rs

    out = {"replicas": n_rep, "particles": total, "n_range": [min(w.n for w in ws), nmax], "rounds": rounds}
    progress(f"serving: {n_rep} device-resident replicas")
    with hs.Server(prm, (1.0, 1.0, 1.0), max_n=nmax, max_slots=slots) as sv:
        for _ in range(2):
            round_(sv)  # capture the replicas' steps
        st0 = sv.stats()
        dts = [round_(sv)[0] for _ in range(rounds)]
        st1 = sv.stats()
        dt = float(np.median(dts))
        rate = n_rep / dt
        out.update({"saturated_requests_per_s": rate, "saturated_particle_steps_per_s": total / dt,
                    "graph_replays_in_timed_rounds": st1["graph_replays"] - st0["graph_replays"],
                    "requests_in_timed_rounds": n_rep * rounds,
                    "affinity_hits_in_timed_rounds": st1["affinity_hits"] - st0["affinity_hits"]})
        rng = np.random.default_rng(seed)
        out["poisson"] = []
        for fr in loads:
            lam = fr * rate
            lat = []
            t_first, t_last = None, 0.0
            for _ in range(2):
                move()
                gaps = rng.exponential(1.0 / lam, n_rep)
                order = rng.permutation(n_rep)
                t0 = time.perf_counter()
                arrivals = t0 + np.cumsum(gaps)
                tk = []
                for k, i in enumerate(order):
                    delay = arrivals[k] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    r = reps[i]
                    tk.append(sv.submit_device(r["x"], r["q"], r["lo"], r["L"], force=r["f"], system_id=int(i) + 1))
                rs = [sv.wait(t) for t in tk]
                lat += [(r["t_done"] - r["t_submit"]) * 1e3 for r in rs]
                t_first = min(r["t_submit"] for r in rs) if t_first is None else t_first
                t_last = max(t_last, max(r["t_done"] for r in rs))
            out["poisson"].append({"offered_fraction": fr, "offered_requests_per_s": lam,
                                   "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                                   "replayed_fraction": float(np.mean([r["replayed"] for r in rs]))})
    # molecular dynamics of 16 replicas on the serving loop (drift, Coulomb
    # forces by device requests, finish), steps per second of the ensemble
    md_reps = []
    for r, w in list(zip(reps, ws))[:16]:
        md_reps.append(dict(x=r["x"].clone(), v=torch.zeros_like(r["x"]), q=r["q"],
                            m=torch.ones(w.n, dtype=torch.float64, device=dev), box_lo=(0.0, 0.0, 0.0),
                            box_len=(r["L"],) * 3))
    progress(f"serving: MD ensemble of {len(md_reps)} replicas")
    with hs.Server(prm, (1.0, 1.0, 1.0), max_n=nmax, max_slots=slots) as sv:
        ens = hs.ReplicaEnsemble(sv, md_reps, 0.001, lj_epsilon=0.0)
        for _ in range(3):
            ens.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 10
        for _ in range(steps):
            ens.step()
        torch.cuda.synchronize()
        dtm = (time.perf_counter() - t0) / steps
        ens.close()
        n_md = sum(r["x"].shape[0] for r in md_reps)
        out["md_ensemble"] = {"replicas": len(md_reps), "particles": n_md, "ms_per_ensemble_step": dtm * 1e3,
                              "particle_steps_per_s": n_md / dtm, "graph_replays": sv.stats()["graph_replays"]}
    return out


def single_system_latency(hs, workloads, sizes=(500, 2000, 10000, 20000), steps=60, warmup=5):
    """Latency of one request of the serving shape on an otherwise idle GPU,
    through a plan of its own (no server): systems of the serving mix's
    recipe (L = (N/0.05)^(1/3), +-1, p 8, K 162, F 512, FP32C), inputs in
    HBM, the step replayed from its captured graph.  Per step: the device
    time between HIP events around it, and the host round trip (enqueue to
    results available: launch plus a stream synchronisation); p50 and p99
    over `steps` steps."""
    import numpy as np
    import torch
    from workloads import Workload
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()  # a stream of its own (steps on it are captured and replayed)
    out = []
    for n in sizes:
        Lb = (n / 0.05) ** (1.0 / 3.0)
        w = Workload(f"latency_{n}", 0, (Lb, Lb, Lb), n, 4000 + n, p=8, F=512, K=162, lam=1.5)
        pos, q, lo, L = workloads.make_system(w)
        x = torch.tensor(pos, device=dev)
        qq = torch.tensor(q, device=dev)
        en = torch.zeros(1, dtype=torch.float64, device=dev)
        f = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        with hs.Plan(hs.Params(precision=hs.FP32C, p=8, K=162, F=512, lam=1.5), lo, L) as plan:
            plan.set_graph(True)
            torch.cuda.synchronize()
            for _ in range(warmup):
                plan.compute_device(x, qq, en, None, f, stream=stream.cuda_stream)
            stream.synchronize()
            dev_ms, wall_ms = [], []
            for _ in range(steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                e0.record(stream)
                plan.compute_device(x, qq, en, None, f, stream=stream.cuda_stream)
                e1.record(stream)
                stream.synchronize()
                wall_ms.append((time.perf_counter() - t0) * 1e3)
                dev_ms.append(e0.elapsed_time(e1))
        out.append({"n": n, "device_p50_ms": float(np.percentile(dev_ms, 50)),
                    "device_p99_ms": float(np.percentile(dev_ms, 99)),
                    "round_trip_p50_ms": float(np.percentile(wall_ms, 50)),
                    "round_trip_p99_ms": float(np.percentile(wall_ms, 99))})
        torch.cuda.synchronize()
        del x, qq, en, f
    return {"note": "one request on an idle GPU through its own plan (no server, graph replay), p50/p99 over "
                    f"{steps} steps", "sizes": out}


def md_bench(hs, steps=200, warmup=20, seed=91):
    """The MD driver on the 3D electrolyte of the paper's accuracy study
    (Sec. 4.1, monovalent case): 1,500 cations and 1,500 anions, WCA soft
    spheres (sigma 1, epsilon kT) in a periodic box of 25 sigma, Bjerrum
    length 3.5 sigma (Coulomb prefactor 3.5 kT sigma / e^2), time step
    0.01 tau, Nose-Hoover thermostat at kT = 1 (damping time 0.1 tau: the
    paper's 0.01 tau equals the time step, a thermostat period of about
    four steps; the rate does not depend on it); HSMA FP32C with p 8,
    K 162, F 512.  Ions on 3,000 random sites of a
    15^3 lattice (no contacts at the start), Maxwell velocities.  `warmup`
    steps (the Coulomb step is captured into a graph), then `steps` steps
    in one hsma_md_run, timed with HIP events on the driver's stream.
    Reported beside the rate: the mean kinetic temperature of the timed
    steps, the drift of the extended energy (E_C + E_LJ + E_kin + the
    thermostat's) over them, the peaks of the radial distribution
    functions g_++, g_+- and g_-- over a further 1,000 steps, and the rate
    of two-level RESPA (Coulomb forces every 0.02 tau, short-range forces
    every 0.01 tau) from the state reached."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    L, m_side, n = 25.0, 15, 3000
    g = (np.stack(np.meshgrid(*(np.arange(m_side),) * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) * (L / m_side)
    pos = g[rng.choice(len(g), n, replace=False)]
    q = np.where(rng.permutation(n) % 2 == 0, 1.0, -1.0)
    v0 = rng.normal(0.0, 1.0, (n, 3))
    v0 -= v0.mean(0)
    dev = torch.device("cuda:0")
    x, v = torch.tensor(pos, device=dev), torch.tensor(v0, device=dev)
    f = torch.zeros_like(x)
    qq, mm = torch.tensor(q, device=dev), torch.ones(n, dtype=torch.float64, device=dev)
    th = torch.zeros((steps, 4), dtype=torch.float64, device=dev)
    th0 = torch.zeros((warmup, 4), dtype=torch.float64, device=dev)
    s0, s1 = (torch.zeros(3, dtype=torch.float64, device=dev) for _ in range(2))
    stream = torch.cuda.Stream()
    prm = hs.Params(precision=hs.FP32C, p=8, K=162, F=512, lam=1.5, coulomb_k=3.5)
    dt = 0.01
    with hs.Plan(prm, (0.0, 0.0, 0.0), (L, L, L)) as plan, \
            hs.MD(plan, n, dt, nh_kT=1.0, nh_damping=0.1) as md:
        torch.cuda.synchronize()
        md.run(x, v, f, qq, mm, warmup, forces_valid=False, thermo=th0, stream=stream.cuda_stream)
        md.thermostat(s0, stream=stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        md.run(x, v, f, qq, mm, steps, forces_valid=True, thermo=th, stream=stream.cuda_stream)
        e1.record(stream)
        md.thermostat(s1, stream=stream.cuda_stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # radial distribution functions over a further 10 tau, sampled every
        # 0.2 tau (hsma_md_rdf), as in the paper's accuracy study
        nbins, rmax, samples = 120, 6.0, 50
        hist = torch.zeros((3, nbins), dtype=torch.int64, device=dev)
        for _ in range(samples):
            md.run(x, v, f, qq, mm, 20, forces_valid=True, stream=stream.cuda_stream)
            md.rdf(x, qq, rmax, hist, stream=stream.cuda_stream)
        stream.synchronize()
    # multiple time steps (reversible RESPA, as the paper's slab runs): the
    # Coulomb forces every 0.02 tau, the short-range ones every 0.01 tau
    # (the velocity-Verlet step above), from the same state
    rs = {}
    with hs.Plan(prm, (0.0, 0.0, 0.0), (L, L, L)) as plan2, \
            hs.MD(plan2, n, 2 * dt, nh_kT=1.0, nh_damping=0.1, respa_inner=2) as md2:
        th2 = torch.zeros((steps, 4), dtype=torch.float64, device=dev)
        md2.run(x, v, f, qq, mm, warmup, forces_valid=False, stream=stream.cuda_stream)
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        md2.run(x, v, f, qq, mm, steps, forces_valid=True, thermo=th2, stream=stream.cuda_stream)
        e3.record(stream)
        stream.synchronize()
        ms2 = e2.elapsed_time(e3) / steps
        t2 = th2.cpu().numpy()
        rs = {"respa_inner": 2, "outer_dt": 2 * dt, "ms_per_outer_step": ms2,
              "simulated_tau_per_s": 2 * dt / (ms2 * 1e-3), "velocity_verlet_tau_per_s": dt / (ms * 1e-3),
              "mean_kT": float(np.mean(2 * t2[:, 2] / (3 * n - 3)))}
    t, t0, a, b = th.cpu().numpy(), th0.cpu().numpy(), s0.cpu().numpy(), s1.cpu().numpy()
    nf = 3 * n - 3
    h0 = t0[-1, :3].sum() + a[2]
    h1 = t[-1, :3].sum() + b[2]
    hc = hist.cpu().numpy().astype(np.float64)
    dr = rmax / nbins
    edges = np.arange(nbins + 1) * dr
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    npos, nneg = int((q > 0).sum()), int((q < 0).sum())
    pairs = np.array([npos * (npos - 1) / 2, npos * nneg, nneg * (nneg - 1) / 2])
    g = hc / (samples * pairs[:, None] * shell[None, :] / L ** 3)
    centre = edges[:-1] + 0.5 * dr
    peaks = {name: {"g_max": float(g[c].max()), "r_at_max": float(centre[int(g[c].argmax())])}
             for c, name in enumerate(("++", "+-", "--"))}
    return {"system": "3D electrolyte, 3,000 ions (+-1), L 25 sigma, Bjerrum length 3.5 sigma, WCA; "
                      "NVT (Nose-Hoover kT 1, damping 0.1 tau), dt 0.01 tau; FP32C p 8",
            "n": n, "steps": steps, "ms_per_step": ms, "particle_steps_per_s": n / (ms * 1e-3),
            "mean_kT": float(np.mean(2 * t[:, 2] / nf)),
            "extended_energy_drift_per_step": float((h1 - h0) / steps),
            "extended_energy": float(h0),
            "rdf": {"samples": samples, "every_steps": 20, "r_max": rmax, "bins": nbins, "peaks": peaks,
                    "g_at_large_r": float(g[1][centre > 5.0].mean())},
            "respa": rs}


def sphere_rule_bench(hs, w, pos, q, lo, L, x, qq, en, pot, f, stream, ms_cells, f64_cells, steps=10):
    """The same system with the sphere near set (images inside the sphere
    only, Sec. 2.2) at parameters that reach the same 1e-5 force bar:
    p = 14, K = 450, F = 1152 (measured against Ewald on the 100-ion
    system: 6e-6 RMS force error, the 27-cell set at p = 10 gives 2e-6)."""
    import dataclasses
    import numpy as np
    import torch
    ws = dataclasses.replace(w, p=14, K=450, F=1152, near_rule=1)
    plan = hs.Plan(hs.Params.from_workload(ws, precision=hs.FP32C), lo, L)
    for _ in range(2):
        plan.compute_device(x, qq, en, pot, f)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.compute_device(x, qq, en, pot, f)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    pairs = plan.info()["near_pairs"]
    plan.close()
    out = {"near_rule": 1, "p": ws.p, "K": ws.K, "F": ws.F, "lambda": ws.lam, "precision": "fp32-compensated",
           "ms_per_step": ms, "particle_steps_per_s": w.n / (ms * 1e-3), "speedup_vs_27_cells": ms_cells / ms,
           "near_pairs": pairs, "near_pairs_27_cells": 27 * w.n * w.n - w.n}
    if f64_cells is not None:
        fs = f.cpu().numpy()
        out["rel_rms_force_diff_vs_27_cells_fp64"] = float(np.sqrt(((fs - f64_cells) ** 2).sum() / (f64_cells ** 2).sum()))
    return out


def slab_near_sets_bench(hs, workloads, steps=5):
    """The 20,000-ion slab with the near sets: the 189-entry stencil at the
    workload's p = 10, the sphere near set at p = 14 (K = 450, F = 1152),
    and the stencil by the treecode (order 12, theta 0.5), FP32 compensated,
    timed on the current stream; their differences from the stencil's FP64
    result."""
    import dataclasses
    import numpy as np
    import torch
    w = workloads.C3
    pos, q, lo, L = workloads.make_system(w)
    dev = torch.device("cuda:0")
    x = torch.tensor(pos, device=dev)
    qq = torch.tensor(q, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    pot = torch.zeros(w.n, dtype=torch.float64, device=dev)
    f = torch.zeros((w.n, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(ww, prec, k):
        plan = hs.Plan(hs.Params.from_workload(ww, precision=prec), lo, L)
        plan.compute_device(x, qq, en, pot, f)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(k):
            plan.compute_device(x, qq, en, pot, f)
        ev1.record(stream)
        torch.cuda.synchronize()
        pairs = plan.info()["near_pairs"]
        plan.close()
        return ev0.elapsed_time(ev1) / k, f.cpu().numpy(), pairs

    ws = dataclasses.replace(w, p=14, K=450, F=1152, near_rule=1)
    wt = dataclasses.replace(w, near_rule=2)
    ms_cells, _, pairs_cells = timed(w, hs.FP32C, steps)
    _, f64_cells, _ = timed(w, hs.FP64, 1)
    e64 = en.item()
    ms_sphere, f_sphere, pairs_sphere = timed(ws, hs.FP32C, steps)
    ms_tree, f_tree, _ = timed(wt, hs.FP32C, steps)
    e_tree = en.item()

    def rms(a):
        return float(np.sqrt(((a - f64_cells) ** 2).sum() / (f64_cells ** 2).sum()))

    return {"workload": w.name, "stencil_ms_per_step": ms_cells, "sphere_ms_per_step": ms_sphere,
            "speedup": ms_cells / ms_sphere, "stencil_near_pairs": pairs_cells, "sphere_near_pairs": pairs_sphere,
            "sphere_p": ws.p, "sphere_K": ws.K, "sphere_F": ws.F,
            "rel_rms_force_diff_vs_stencil_fp64": rms(f_sphere),
            "tree": {"ms_per_step": ms_tree, "speedup": ms_cells / ms_tree, "tree_order": 12, "tree_theta": 0.5,
                     "rel_energy_err_vs_stencil_fp64": abs(e_tree - e64) / abs(e64),
                     "rel_rms_force_err_vs_stencil_fp64": rms(f_tree)}}


def timed_loop(hs, w, lo, L, x, qq, en, pot, f, steps, warmup, stream):
    """W untimed warm-up steps, then exactly K steps on `stream` between two
    device synchronisations; one HIP event between consecutive steps (no
    synchronisation inside the timed region).  The plan's stage events
    (HIP events on the call's stream) give the dominant kernel's time."""
    import numpy as np
    import torch
    plan = hs.Plan(hs.Params.from_workload(w, precision=hs.FP32C), lo, L)
    for _ in range(warmup):
        plan.compute_device(x, qq, en, pot, f)
    torch.cuda.synchronize()
    if plan.device_status() != 0:
        raise SystemExit("device-side validation failed")
    plan.set_timing(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        plan.compute_device(x, qq, en, pot, f)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    tm = plan.timing()
    info = plan.info()
    plan.close()
    calls = max(1, tm["calls"])
    near_ms = tm["near_ms"] / calls
    near_flop = FLOP_PER_NEAR_PAIR * info["near_pairs"]
    ms = evs[0].elapsed_time(evs[-1]) / steps
    return {
        "ms": ms, "median": float(np.median(per_step)), "p90": float(np.percentile(per_step, 90)),
        "wall_ms": (wall1 - wall0) * 1e3 / steps, "near_ms": near_ms, "info": info,
        "stage_ms": {"step": tm["step_ms"] / calls, "near": near_ms, "check": tm["check_ms"] / calls,
                     "sphere": tm["sphere_ms"] / calls},
        "achieved_tflops": near_flop / (near_ms * 1e-3) / 1e12, "near_flop": near_flop,
    }


def roofline(w, r):
    return {
        "kernel": "k_pair<float,false,true> (far near-set sums at the particles)",
        "bound": "alu", "achieved": r["achieved_tflops"], "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": r["achieved_tflops"] / PEAK_FP32_TFLOPS,
        "traffic": measured_traffic("k_pair_float_particles", w.name),
        "flop_per_launch": r["near_flop"], "pairs_per_launch": r["info"]["near_pairs"],
        "flop_per_pair": FLOP_PER_NEAR_PAIR, "launch_ms": r["near_ms"],
    }


def fp64_leg(hs, w, lo, L, x, qq, en, pot, f, e32, f32, ms32, stream, steps=1):
    """The plain FP64 single-system GPU path on the same system: one call to
    warm the plan where it is cheap, then `steps` timed calls; its energy
    and forces are the reference of the FP32-compensated result."""
    import numpy as np
    import torch
    p64 = hs.Plan(hs.Params.from_workload(w, precision=hs.FP64), lo, L)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if w.n <= 100_000:
        p64.compute_device(x, qq, en, pot, f)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        p64.compute_device(x, qq, en, pot, f)
    ev1.record(stream)
    torch.cuda.synchronize()
    p64.close()
    ms64 = ev0.elapsed_time(ev1) / steps
    e64 = en.item()
    f64 = f.cpu().numpy()
    return {
        "ms_per_step": ms64, "speedup_fp32c_over_fp64": ms64 / ms32,
        "rel_energy_err": abs(e32 - e64) / abs(e64),
        "rel_rms_force_err": float(np.sqrt(((f32 - f64) ** 2).sum() / (f64 ** 2).sum())),
        "max_force_err_rel_to_max": float(np.abs(f32 - f64).max() / np.abs(f64).max()),
    }, e64, f64


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison")
    ap.add_argument("--serving", action="store_true",
                    help="also measure the serving mix, device replicas and the MD ensemble through the "
                         "request server (off by default)")
    ap.add_argument("--no-sphere-rule", action="store_true",
                    help="skip the sphere-near-set measurement (near_rule=1 at matched accuracy)")
    ap.add_argument("--no-tree", action="store_true", help="skip the treecode measurement (near_rule=2)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 50,000-ion system and every other secondary measurement")
    ap.add_argument("--workload", default="c5_hsma3d_n999999_2to1",
                    help="configuration to time (default: the 999,999-ion system, the largest one)")
    ap.add_argument("--near-rule", type=int, default=None, help="override the near set (0 cells, 1 sphere, 2 treecode)")
    ap.add_argument("--p", type=int, default=None, help="override the harmonic degree")
    ap.add_argument("--K", type=int, default=None, help="override the check-point pairs")
    ap.add_argument("--F", type=int, default=None, help="override the sphere points")
    ap.add_argument("--profile-pass", action="store_true",
                    help="for counter runs: one 512 MiB device copy (calibration of the byte counters) "
                         "then warmup + steps of the benchmarked step, nothing else")
    ap.add_argument("--md-only", action="store_true",
                    help="only the MD driver measurement (for kernel traces of the MD step); prints its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method would shard by target ranges). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one process per run; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    import paper_2104_05260_amd as hs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.md_only:
        print(json.dumps({"md": md_bench(hs)}), flush=True)
        return
    import dataclasses
    w = workloads.CONFIGS[args.workload]
    over = {k: v for k, v in (("near_rule", args.near_rule), ("p", args.p), ("K", args.K), ("F", args.F))
            if v is not None}
    default_run = args.workload == workloads.C5.name and not over
    if over:
        w = dataclasses.replace(w, **over)
    if not default_run:
        # a profiling run of another configuration: the timed loop only
        args.no_fp64 = args.no_sphere_rule = args.no_tree = args.no_secondary = True
        args.serving = False
    pos, q, lo, L = workloads.make_system(w)
    dev = torch.device("cuda:0")
    x = torch.tensor(pos, device=dev)
    qq = torch.tensor(q, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    pot = torch.zeros(w.n, dtype=torch.float64, device=dev)
    f = torch.zeros((w.n, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    if args.profile_pass:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)           # plain copy kernel: 512 MiB read + 512 MiB written
        torch.cuda.synchronize()
        del src, dst
        plan = hs.Plan(hs.Params.from_workload(w, precision=hs.FP32C), lo, L)
        for _ in range(args.warmup + args.steps):
            plan.compute_device(x, qq, en, pot, f)
        torch.cuda.synchronize()
        plan.close()
        print(json.dumps({"profile_pass": True, "copy_bytes": 512 * 1024 * 1024, "steps": args.warmup + args.steps}))
        return

    progress(f"{w.name}: {args.warmup} warm-up + {args.steps} timed steps")
    r = timed_loop(hs, w, lo, L, x, qq, en, pot, f, args.steps, args.warmup, stream)
    ms = r["ms"]
    info = r["info"]
    e32 = en.item()
    f32 = f.cpu().numpy()
    out = {
        "metric": "particle-steps/s (E+F) at 1e-5 rel force err; pair-int/s % FP32 peak; p50/p99",
        "value": w.n / (ms * 1e-3),
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "ms_per_step_median": r["median"], "ms_per_step_p90": r["p90"],
        "wall_ms_per_step": r["wall_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "box": list(w.box), "p": w.p, "F": w.F, "K": w.K,
                   "lambda": w.lam, "charges": w.charges,
                   "near_set": "images inside the sphere" if w.near_rule == 1 else
                               ("27 cells by the treecode" if w.near_rule == 2 else
                                ("27 cells" if w.geometry == 0 else f"9 cells x {2 * w.M + 1} layers")),
                   "precision": "fp32-compensated (FP64 potential accumulation, FP64 fit and energy)",
                   "parallelism": "single-gpu"},
        "pair_interactions_per_s": (info["near_pairs"] + info["check_pairs"] + info["surface_pairs"]) / (ms * 1e-3),
        "pairs_per_step": {"near_set": info["near_pairs"], "check_points": info["check_pairs"],
                           "sphere_sources": info["surface_pairs"]},
        "stage_ms": r["stage_ms"],
        "roofline": roofline(w, r) if w.near_rule != 2 else tree_roofline(w.name, r["near_ms"]),
    }
    progress(f"timed: {ms:.3f} ms per step")
    if not args.no_fp64:
        progress("FP64 path on the same system")
        out["fp64_gpu"], e64_large, f64_large = fp64_leg(hs, w, lo, L, x, qq, en, pot, f, e32, f32, ms, stream)
        progress(f"fp64: rel energy err {out['fp64_gpu']['rel_energy_err']:.2e}")
    if not args.no_tree:
        progress("treecode on the same system")
        params = hs.Params.from_workload(w, precision=hs.FP32C)
        params.near_rule = 2
        out["tree_near_set_large"] = tree_entry(hs, params, w, lo, L, x, qq, en, pot, f, stream, ms, 5,
                                                None if args.no_fp64 else e64_large,
                                                None if args.no_fp64 else f64_large)
    if not args.no_sphere_rule:
        progress("sphere near set on the same system")
        out["sphere_near_set_large"] = sphere_rule_bench(hs, w, pos, q, lo, L, x, qq, en, pot, f, stream, ms,
                                                         None if args.no_fp64 else f64_large, steps=2)
    del x, qq, pot, f
    torch.cuda.empty_cache()
    if not args.no_secondary:
        progress("50,000-ion system (27 cells)")
        out["c2_50000"] = c2_bench(hs, workloads, args)
        progress("single-request latency at serving sizes")
        out["single_system_latency"] = single_system_latency(hs, workloads)
        progress("MD driver: 3,000-ion electrolyte, NVT")
        out["md"] = md_bench(hs)
    if args.serving:
        progress("serving mix")
        out["serving"] = serving_bench(hs, workloads)
    if not args.no_cpu_baseline:
        progress("CPU oracle (bounded: a sample scaled to the step, or one full step if it fits 30 s)")
        out["cpu_baseline"] = cpu_baseline(w, pos, q, lo, L)
    print(json.dumps(out), flush=True)


def tree_entry(hs, params, w, lo, L, x, qq, en, pot, f, stream, ms_cells, steps, e64=None, f64=None):
    """The 27-cell sums by the treecode (near_rule=2) on the same arrays:
    time per step and, when given, the error against the FP64 27-cell
    result."""
    import numpy as np
    import torch
    plan = hs.Plan(params, lo, L)
    for _ in range(2):
        plan.compute_device(x, qq, en, pot, f)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.compute_device(x, qq, en, pot, f)
    ev1.record(stream)
    torch.cuda.synchronize()
    # then a few calls with the plan's stage events: k_tree_far's duration
    plan.set_timing(True)
    for _ in range(3):
        plan.compute_device(x, qq, en, pot, f)
    torch.cuda.synchronize()
    tm = plan.timing()
    plan.close()
    tree_ms = tm["near_ms"] / max(1, tm["calls"])
    ms = ev0.elapsed_time(ev1) / steps
    o = {"near_rule": 2, "tree_order": params.tree_order, "tree_theta": params.tree_theta,
         "precision": "fp32-compensated", "ms_per_step": ms, "particle_steps_per_s": w.n / (ms * 1e-3),
         "speedup_vs_27_cells": ms_cells / ms,
         "roofline": tree_roofline(w.name if params.tree_order == 12 else f"{w.name}_order{params.tree_order}",
                                   tree_ms)}
    if e64 is not None:
        fs = f.cpu().numpy()
        o["rel_energy_err_vs_27_cells_fp64"] = abs(en.item() - e64) / abs(e64)
        o["rel_rms_force_err_vs_27_cells_fp64"] = float(np.sqrt(((fs - f64) ** 2).sum() / (f64 ** 2).sum()))
    return o


def c2_bench(hs, workloads, args, steps=20):
    """The 50,000-ion system (27 cells, FP32 compensated): step time and the
    far kernel's roofline position, the FP64 path, the sphere near set, the
    treecode, and the slab's near sets."""
    import dataclasses
    import torch
    w = workloads.C2
    pos, q, lo, L = workloads.make_system(w)
    dev = torch.device("cuda:0")
    x = torch.tensor(pos, device=dev)
    qq = torch.tensor(q, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    pot = torch.zeros(w.n, dtype=torch.float64, device=dev)
    f = torch.zeros((w.n, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    r = timed_loop(hs, w, lo, L, x, qq, en, pot, f, steps, 3, stream)
    ms = r["ms"]
    e32, f32 = en.item(), f.cpu().numpy()
    out = {"workload": w.name, "n": w.n, "ms_per_step": ms, "particle_steps_per_s": w.n / (ms * 1e-3),
           "stage_ms": r["stage_ms"], "roofline": roofline(w, r)}
    e64 = f64 = None
    if not args.no_fp64:
        out["fp64_gpu"], e64, f64 = fp64_leg(hs, w, lo, L, x, qq, en, pot, f, e32, f32, ms, stream, steps=3)
    if not args.no_sphere_rule:
        out["sphere_near_set"] = sphere_rule_bench(hs, w, pos, q, lo, L, x, qq, en, pot, f, stream, ms, f64)
        out["sphere_near_set_slab"] = slab_near_sets_bench(hs, workloads)
    if not args.no_tree:
        params = hs.Params.from_workload(w, precision=hs.FP32C)
        params.near_rule = 2
        out["tree_near_set"] = tree_entry(hs, params, w, lo, L, x, qq, en, pot, f, stream, ms, 10, e64, f64)
        out["tree_near_set"]["order8"] = tree_entry(hs, dataclasses.replace(params, tree_order=8), w, lo, L,
                                                     x, qq, en, pot, f, stream, ms, 10, e64, f64)
    return out


if __name__ == "__main__":
    main()
