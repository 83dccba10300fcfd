"""Benchmark of the RBSOG force + pressure step on one MI355X.

A step is one full pass of the hot path: FP64 box rescale of the positions
on the device, mode sampling (both MH chains), binning and sort, short-range
pair kernel, structure factors, estimators and the long-range force scatter,
then the pressure tensor back on the host.  Inputs are resident in HBM before
the timed region starts.

Prints one JSON line: atom-steps/s, the roofline of the dominant kernel (the
pair kernel) from HIP-event timings taken inside the timed region, and the
FP64 oracle timed on the host cores on a bounded sample of the same workload.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config slab-1m]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RBSOG force+pressure atom-steps/s at 1e6 atoms, P=100; served p50/p99 latency"

# MI355X FP32 vector peak: 157.3 TFLOP/s = 256 CUs x 4 SIMDs x 32 FMA lanes per
# clock x 2.4 GHz x 2 flops, i.e. 78.6e12 FP32 lane-ops (FMA, add, mul) per second.
VALU_LANE_OPS_PER_S = 256 * 4 * 32 * 2.4e9
# A transcendental (v_exp/v_rsq/v_sin/v_cos) occupies the issue of this many
# FP32 lane-ops; measured by the probe in every run (this value only when the
# probe is skipped).
TRANS_WEIGHT_DEFAULT = 3.4


def pair_work(trans_weight, M=10):
    """Algorithmic work of one unordered in-cutoff pair, in FP32 lane-op
    equivalents, for the paper's form of the SOG kernels: about 42 FMA-class
    operations (2M for the two weighted Gaussian sums, about 22 for distance,
    cutoff, N~, force on both atoms, 6 virial components and energy) and M + 1
    transcendentals (M exponentials and r^-1)."""
    return 42 + trans_weight * (M + 1)


def pair_work_implemented(trans_weight):
    """The FP32C polynomial form as implemented: displacement 9, r^2 3, cutoff
    1, r^-3 2, t 1, degree-10 Horner 10, N~ 1, q_i q_j and f 2, f r 3, force on
    both atoms 6, virial 6 (no energy in the timed step), one transcendental."""
    return 44 + trans_weight * 1


def mode_work(trans_weight):
    """Work per (atom, distinct mode): structure factor (3 integer
    multiply-adds, convert, 2 FMA + sin, cos) and force scatter (3
    multiply-adds, convert, 2 + 3 FMA + sin, cos)."""
    return 6 + 2 * trans_weight, 9 + 2 * trans_weight


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2602_23582_amd import workloads as W
    if name == "slab-1m":
        d = W.slab()
        desc = ("slab-1m: 1,000,000 atoms in a 200 x 200 x 500 A box, two +-0.7e dipole layers at z_c +- 20 A "
                "in 330,000 three-site water-like molecules, rc 12 A, P 100")
    elif name == "slab-1m-p400":
        d = W.slab(P=400)
        desc = "slab-1m at P 400"
    elif name == "electrolyte-10m":
        d = W.electrolyte()
        desc = "electrolyte-10m: 10,000,000 atoms, 1 M ion pairs in water-like molecules, 467.5 A cube, rc 10, P 100"
    elif name == "sheared-slab-1m":
        # the slab's fractional positions in a general (triclinic) cell: the
        # columns of h are the cell vectors (200, 0, 0), (30, 200, 0), (0, 20, 500)
        d = W.slab()
        h = np.array([[200.0, 30.0, 0.0], [0.0, 200.0, 20.0], [0.0, 0.0, 500.0]])
        d["pos"] = (d["pos"] / np.asarray(d["L"])) @ h.T
        d["h"] = h
        desc = ("sheared-slab-1m: slab-1m's fractional positions in the general cell with vectors (200, 0, 0), "
                "(30, 200, 0), (0, 20, 500) A, rc 12 A, P 100 (general-cell sampler and exact pair path)")
    elif name == "water-30k":
        d = W.water_box()
        desc = "water-30k: 10,000 three-site molecules at 1 g/cm^3 (66.9 A cube), rc 10, P 100"
    elif name == "lattice-1k":
        d = W.c1_lattice()
        desc = "lattice-1k: 1,000 +-1e charges on a jittered 10^3 lattice, 30 A cube, rc 10, P 100"
    else:
        raise SystemExit(f"unknown config {name}")
    return d, desc


def kernel_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip",):
        with open(os.path.join(ROOT, "paper_2602_23582_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counters(config):
    """The committed counter summary of the pair kernel (name -> value text), if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"pair_kernel_{config}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.split("#")[0].strip()
    if vals.get("kernels_sha256") != kernel_hash():
        return None
    return vals


def read_traffic(config):
    """HBM bytes per pair-kernel launch from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    vals = read_counters(config)
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def read_issued(config, tw):
    """VALU lane-instructions the pair kernel issues per launch (transcendentals
    weighed by tw, FP32 lane-op equivalents), from the same counter summary."""
    vals = read_counters(config)
    try:
        valu, trans = float(vals["SQ_INSTS_VALU"]), float(vals["SQ_INSTS_VALU_TRANS_F32"])
    except (TypeError, KeyError, ValueError):
        return None
    return 64.0 * ((valu - trans) + trans * tw)


PROBE_KINDS = [  # (name, FP32 FMA per iteration, transcendentals per iteration), per lane
    ("fma", 8, 0), ("exp", 0, 8), ("rsq", 0, 8), ("sin", 0, 8),
    ("exp+4fma", 32, 8), ("exp+2fma", 16, 8), ("exp+1fma", 8, 8), ("exp+8fma", 64, 8)]


def valu_probe(iters=32768, blocks=2048):
    """Issue rates behind the ALU roofline, measured on this GPU: wave
    instructions per second of FP32 FMA, of v_exp/v_rsq/v_sin, and of mixes,
    from paper_2602_23582_amd/csrc/valu_probe.hip (8 independent chains per
    lane, 4 waves per workgroup)."""
    import ctypes as C
    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_2602_23582_amd", "libvaluprobe.so"))
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    waves = blocks * 4
    simd_cycles_per_s = 256 * 4 * 2.4e9
    res = {}
    for kind, (name, nv, nt) in enumerate(PROBE_KINDS):
        ms = C.c_float()
        rc = lib.valu_probe(kind, iters, blocks, C.c_void_p(out.data_ptr()), C.byref(ms))
        if rc != 0:
            raise RuntimeError(f"valu_probe kind {kind}: error {rc}")
        t = ms.value * 1e-3
        v = waves * iters * nv / t
        tr = waves * iters * nt / t
        res[name] = {"ms": ms.value, "valu_per_simd_cycle": v / simd_cycles_per_s,
                     "trans_per_simd_cycle": tr / simd_cycles_per_s}
    return res


def served_bench(n_req, seed, pool_bytes, lam_fracs=(0.5, 0.8, 0.95), nsteps=10, growth=0.001):
    """The served stream: n_req independent systems (sizes log-uniform in
    [500, 50,000] atoms, +-1e on jittered lattices at 0.1 A^-3, P from
    {50, 100, 200}), each a request of nsteps steps under L_k = L_0 (1 + g k).
    Capacity is measured with every request submitted at once; then requests
    arrive as Poisson streams at each fraction of that capacity.  Each stream
    runs with continuous batching (all admitted requests per tick); one
    request at a time (the same server with one slot) runs at capacity and at
    the middle fraction, on the same GPU and at the same accuracy; every
    request is a force + pressure solve (no energy sum).  Latency =
    completion - submission.  The pool is small enough that admission by
    memory binds at capacity."""
    from paper_2602_23582_amd import rbsog
    from paper_2602_23582_amd import workloads as W
    sizes, seeds = W.served_stream(n_req, seed=seed)
    reqs = [W.ionic_system(int(n), int(sd)) for n, sd in zip(sizes, seeds)]
    atom_steps = float(sum(len(r["q"]) for r in reqs)) * nsteps

    def run(max_active, arrivals):
        with rbsog.Server(max_active=max_active, pool_bytes=pool_bytes, energy=False) as sv:
            t0 = time.perf_counter()
            tickets = []
            for i, (r, ta) in enumerate(zip(reqs, arrivals)):
                dt = ta - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets.append(sv.submit(r["q"], r["pos"], r["L"], r["rc"], nsteps=nsteps, growth=growth, P=r["P"],
                                         seed=int(seeds[i]), system_id=i))
            res = [sv.wait(t) for t in tickets]
            wall = time.perf_counter() - t0
            st = sv.stats()
        lat = np.array([x["latency_s"] for x in res])
        return {"p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "atom_steps_per_s": atom_steps / wall, "requests_per_s": n_req / wall, "wall_s": wall,
                "ticks": st["ticks"], "peak_active": st["peak_active"], "peak_pool_mib": st["peak_pool_bytes"] / 2**20,
                "tick_ms": {k: 1e3 * st[k + "_s"] / max(st["ticks"], 1) for k in ("admit", "launch", "wait")}}

    burst = np.zeros(n_req)
    sat = run(65536, burst)
    streams = {}
    mid = lam_fracs[len(lam_fracs) // 2]
    solo = None
    for frac in lam_fracs:
        lam = frac * sat["requests_per_s"]
        arrivals = np.cumsum(np.random.default_rng(seed).exponential(1.0 / lam, n_req))
        r = run(65536, arrivals)
        r["arrival_rate_per_s"] = lam
        streams[f"{frac:g}"] = r
        if frac == mid:
            solo = run(1, arrivals)
            solo["arrival_rate_per_s"] = lam
    solo_sat = run(1, burst)
    return {"requests": n_req, "steps_per_request": nsteps, "pool_mib": pool_bytes / 2**20, "energy": False,
            "atoms": int(sum(len(r["q"]) for r in reqs)),
            "continuous_batching_by_load": streams,
            "one_at_a_time": {"load": mid, **solo},
            "capacity": {"continuous_batching": sat, "one_at_a_time": solo_sat}}


def host_cpu():
    """Model name and logical CPUs of the host, and the CPUs this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def oracle_step_time(orc, d, P, seed, sample_atoms):
    """Seconds of one oracle step (Algorithm O) on the workload: mode
    sampling, structure factors of all atoms for the 2P sampled modes and the
    estimators, then short- and long-range forces of sample_atoms atoms; the
    per-atom force time is scaled to all atoms (no scaling when the sample is
    every atom)."""
    n = len(d["q"])
    p = orc.sog(d["rc"], row=2, M=10)
    rng = np.random.default_rng(0)
    k = min(n, sample_atoms) if sample_atoms > 0 else n
    smp = None if k == n else np.sort(rng.choice(n, k, replace=False))
    t0 = time.perf_counter()
    m_r, m_nr, _ = orc.sample_modes(d["L"], p, P, seed, 0, 0)
    Sr, Snr = orc.norm_consts(d["L"], p)
    t1 = time.perf_counter()
    orc.long_range_rb(d["q"], d["pos"], d["L"], m_r, m_nr, Sr, Snr, forces=False)  # all rho + estimators
    t2 = time.perf_counter()
    orc.short_range(d["q"], d["pos"], d["L"], p, method="cells", sample=smp)
    orc.long_range_rb(d["q"], d["pos"], d["L"], m_r, m_nr, Sr, Snr, forces=True, sample=smp)
    t3 = time.perf_counter()
    # the second long_range_rb re-evaluates rho: subtract one full rho pass
    per_atom = max(t3 - t2 - (t2 - t1), 0.0) / k
    return (t1 - t0) + (t2 - t1) + per_atom * n, k, t3 - t0


def cpu_baseline(d, P, seed, sample_atoms, single_sample):
    """The oracle as it stands, timed on the host: every OpenMP thread it is
    given on sample_atoms atoms (0: all of them, one full step), then one
    thread on single_sample atoms."""
    from oracle import oracle as orc
    n = len(d["q"])
    threads = orc.num_threads()
    t_step, k, wall = oracle_step_time(orc, d, P, seed, sample_atoms)
    out = {"value": n / t_step, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
           "sample": (f"one full step of all {n} atoms (sampling, structure factors of the {2 * P} sampled modes, "
                      f"estimators, short- and long-range forces)" if k == n else
                      f"{k} of {n} atoms for short- and long-range forces, structure factors of all atoms for "
                      f"the {2 * P} sampled modes, one step; per-atom time scaled to all atoms"),
           "seconds": wall, "host": host_cpu()}
    if single_sample > 0:
        orc.set_num_threads(1)
        try:
            t1, k1, w1 = oracle_step_time(orc, d, P, seed, single_sample)
        finally:
            orc.set_num_threads(threads)
        out["single_core"] = {"value": n / t1, "cores": 1, "seconds": w1,
                              "sample": f"{k1} of {n} atoms for the forces, structure factors of all atoms; "
                                        f"per-atom time scaled to all atoms"}
    return out


def npt_bench(torch, ctx, d, x, y, z, nsteps, force_ms):
    """Langevin NPT steps (rbsog_npt_run, semi-isotropic for a box with Lx = Ly)
    from the benchmark's final positions and box with thermal momenta; synthetic masses (16 for
    negative sites, 1 for positive).  Reports time per NPT step and what it adds
    to the force + pressure evaluation."""
    from paper_2602_23582_amd import rbsog
    q = d["q"]
    m = np.where(q < 0, 16.0, 1.0)
    rng = np.random.default_rng(7)
    kT = 0.6
    mom = rng.normal(size=(len(q), 3)) * np.sqrt(m * kT)[:, None]
    xs, ys, zs = (t.clone() for t in (x, y, z))
    px, py, pz = (torch.tensor(np.ascontiguousarray(mom[:, k]), dtype=torch.float64, device="cuda") for k in range(3))
    L = np.asarray(ctx.box, dtype=np.float64)   # the box the positions were last rescaled to
    coupling = rbsog.COUPLE_SEMI if L[0] == L[1] else rbsog.COUPLE_ANISO
    ctx.npt_init(m, dt=0.002, kT=kT, gamma=1.0, gamma_box=0.5, box_mass=1e4, p_ext=0.0, coupling=coupling)
    pbox = np.zeros(3)
    box, pbox, _, _ = ctx.npt_run(xs, ys, zs, px, py, pz, 1000, 2, pbox)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    box, pbox, Pi, Pk = ctx.npt_run(xs, ys, zs, px, py, pz, 1002, nsteps, pbox)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # one call evaluates the starting state first: nsteps + 1 evaluations
    ms = 1e3 * (t1 - t0) / nsteps
    return {"steps": nsteps, "ms_per_npt_step": ms, "atom_steps_per_s": len(q) * nsteps / (t1 - t0),
            "force_pressure_ms_per_step": force_ms, "coupling": "semi-isotropic" if coupling else "anisotropic",
            "final_box": box.tolist(), "P_ins_diag": np.diag(Pi).tolist(), "P_kin_diag": np.diag(Pk).tolist(),
            "note": "per call the starting state is evaluated once more (nsteps + 1 evaluations)"}


SAMPLERS = {0: "recalibrated (as printed)", 1: "recalibrated (exchange form)", 2: "shared proposal, no recalibration",
            3: "independent chain (2P structure factors)"}


def variance_study(torch, reps, Ps=(50, 100, 200), sizes=(2000, 16000)):
    """Variance of the long-range pressure estimator P^{F,r*} + P^{F,nr*}
    under the four samplers of the non-radial modes (Sec. 3.2), against P and
    N: seeded disordered ionic systems at 0.1 A^-3 (rc 10 A).  For each sampler, P and
    system size, reps steps (the step index draws the modes) give the variance
    of every tensor component about its mean; reported as the mean over the
    diagonal and over the off-diagonal components, with the mean number of
    distinct modes (structure factors) per step and their product
    (variance x work).  The radial estimator and the force are the same under
    every sampler."""
    from paper_2602_23582_amd import rbsog
    from paper_2602_23582_amd import workloads as W
    rows = []
    ref_path = os.path.join(ROOT, "tests", "golden", "variance_reference.json")
    ref = json.load(open(ref_path))["systems"] if os.path.exists(ref_path) else {}
    for n in sizes:
        d = W.ionic_melt(n, seed=11)
        x, y, z = (torch.tensor(np.ascontiguousarray(d["pos"][:, k]), dtype=torch.float64, device="cuda")
                   for k in range(3))
        fx, fy, fz = (torch.empty_like(x) for _ in range(3))
        for variant in SAMPLERS:
            for P in Ps:
                vals, nd = [], []
                with rbsog.Context(d["q"], d["L"], d["rc"], P=P, seed=31, system_id=n,
                                   recalibration=variant) as ctx:
                    for step in range(reps):
                        ctx.sample_modes(step, d["L"])
                        ctx.force_virial(x, y, z, fx, fy, fz, energy=False)
                        _, parts = ctx.pressure()
                        vals.append((parts[1] + parts[2]).ravel())
                        nd.append(ctx.step_info()["nd"])
                a = np.array(vals)
                v = np.var(a, axis=0, ddof=1)
                # standard error of each component's variance from its fourth central moment
                m4 = np.mean((a - a.mean(0)) ** 4, axis=0)
                se = np.sqrt(np.maximum(m4 - v * v, 0.0) / len(a))
                vd, vo = float(v[[0, 4, 8]].mean()), float(v[[1, 2, 5]].mean())
                row = {"n": n, "sampler": SAMPLERS[variant], "P": P, "var_diag": vd, "var_offdiag": vo,
                       "var_diag_rel_se": float(se[[0, 4, 8]].mean() / 3 ** 0.5 / vd),
                       "modes_per_step": float(np.mean(nd)), "var_diag_x_modes": vd * float(np.mean(nd))}
                if str(n) in ref:
                    # bias of the batch mean against the deterministic P^F, its
                    # z-score, and the mean squared error per step var + bias^2
                    PF = np.asarray(ref[str(n)]["PF"])
                    bias = a.mean(0) - PF
                    zsc = bias / np.sqrt(v / len(a))
                    mse = v + bias ** 2
                    row.update({"bias_diag": bias[[0, 4, 8]].tolist(), "bias_offdiag": bias[[1, 2, 5]].tolist(),
                                "bias_rel_norm": float(np.linalg.norm(bias) / np.linalg.norm(PF)),
                                "bias_max_abs_z": float(np.abs(zsc).max()),
                                "mse_diag": float(mse[[0, 4, 8]].mean()), "mse_offdiag": float(mse[[1, 2, 5]].mean())})
                rows.append(row)
    return {"system": "ionic, 0.1 A^-3, rc 10 A, +-1e at uniform random positions", "reps": reps, "rows": rows,
            "reference": "P^F by the full k-space sum, tests/golden/variance_reference.json"}


def pipelined(args):
    """The default stepping: each step queued with rbsog_step_async and its
    pressure read (rbsog_step_wait) once the next step is queued."""
    return not (args.graph or args.separate_calls or args.sync_steps)


def run_queued(c, steps, mu_of, arrays):
    """Step context c through the step indices `steps` with rbsog_step_async,
    reading each step's pressure after the next step is queued; returns the
    host time at which each step's pressure had arrived."""
    x, y, z, fx, fy, fz = arrays
    marks, pending = [], None
    for s in steps:
        t = c.step_async(s, mu_of(s), x, y, z, fx, fy, fz)
        if pending is not None:
            c.step_wait(pending)
            marks.append(time.perf_counter())
        pending = t
    if pending is not None:
        c.step_wait(pending)
        marks.append(time.perf_counter())
    return marks


def extra_workload(torch, name, args, tw):
    """Another workload through the same step (context calls, HIP events on the
    pair launches): ms per step with its spread, atom-steps/s and the pair
    kernel's roofline fraction."""
    from paper_2602_23582_amd import rbsog
    d, desc = make_workload(name)
    n = len(d["q"])
    x, y, z = (torch.tensor(np.ascontiguousarray(d["pos"][:, k]), dtype=torch.float64, device="cuda")
               for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    L0 = np.asarray(d["L"], dtype=np.float64)
    cell = d.get("h")
    with rbsog.Context(d["q"], L0 if cell is None else np.diag(cell).copy(), d["rc"], P=int(d["P"]),
                       seed=args.seed) as c:
        def step(s):
            if cell is None:
                mu = L0 * (1.0 + 0.001 * (s % 10)) / c.box
                if not args.separate_calls:
                    return c.step(s, mu, x, y, z, fx, fy, fz)[0]
                c.rescale(mu, x, y, z)
                c.sample_modes(s, c.box)
            else:  # a general cell: fixed cell and positions (the device rescale is diagonal)
                c.sample_modes_cell(s, cell)
            c.force_virial(x, y, z, fx, fy, fz, energy=False)
            return c.pressure()[0]
        queued = pipelined(args) and cell is None
        mu_of = lambda s: L0 * (1.0 + 0.001 * (s % 10)) / c.box
        for s in range(3):
            step(s)
        torch.cuda.synchronize()
        c.set_timing(2)  # the pair kernel's launches only
        t0 = time.perf_counter()
        if queued:
            marks = run_queued(c, range(3, 3 + args.extra_steps), mu_of, (x, y, z, fx, fy, fz))
        else:
            marks = []
            for s in range(3, 3 + args.extra_steps):
                step(s)
                marks.append(time.perf_counter())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        timing = c.get_timing()
        info = c.step_info()
        c.set_timing(False)
    per_step = 1e3 * np.diff(np.concatenate([[t0], marks]))
    pair_ms, pair_cnt = timing.get("pair", (0.0, 1))
    t_pair = pair_ms / max(pair_cnt, 1) * 1e-3
    work = info["npairs"] * pair_work(tw)
    del x, y, z, fx, fy, fz
    torch.cuda.empty_cache()
    return {"workload": desc, "n_atoms": n, "steps": args.extra_steps, "ms_per_step": 1e3 * (t1 - t0) / args.extra_steps,
            "ms_per_step_percentiles": {"p10": float(np.percentile(per_step, 10)),
                                        "median": float(np.percentile(per_step, 50)),
                                        "p90": float(np.percentile(per_step, 90))},
            "atom_steps_per_s": n * args.extra_steps / (t1 - t0),
            "roofline": {"bound": "alu", "kernel": "k_pair (with its neighbourhood and gather launches)",
                         "avg_launch_ms": 1e3 * t_pair, "unordered_pairs_per_launch": info["npairs"],
                         "achieved": work / t_pair / 1e12 if t_pair > 0 else 0.0,
                         "peak": VALU_LANE_OPS_PER_S / 1e12, "unit": "T FP32 lane-op/s",
                         "frac": work / t_pair / VALU_LANE_OPS_PER_S if t_pair > 0 else 0.0},
            "distinct_modes": info["nd"],
            **({"note": "general cell: cell and positions fixed between steps"} if cell is not None else {})}


SHELL_FLAGS = {"auto": 0, "full": 2, "half": 4}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="slab-1m")
    ap.add_argument("--seed", type=int, default=2026)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="atoms whose forces the oracle computes on all host threads (0: every atom, one full step)")
    ap.add_argument("--cpu-single-sample", type=int, default=20_000,
                    help="atoms of the single-thread oracle timing (0: skip)")
    ap.add_argument("--extra", default="electrolyte-10m,sheared-slab-1m",
                    help="comma-separated further workloads timed after the main one (none: skip)")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--shell", choices=["auto", "full", "half"], default="auto",
                    help="pair kernel: the library's choice, or force the full or the half shell")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-valu-probe", action="store_true")
    ap.add_argument("--sync-steps", action="store_true",
                    help="read each step's pressure before queuing the next (rbsog_step) instead of one step "
                         "later (rbsog_step_async / rbsog_step_wait)")
    ap.add_argument("--separate-calls", action="store_true",
                    help="step with rbsog_rescale, rbsog_sample_modes, rbsog_force_virial and rbsog_pressure "
                         "instead of the one-call rbsog_step")
    ap.add_argument("--graph", action="store_true",
                    help="run the step as a batch of one replaying a captured HIP graph")
    ap.add_argument("--served", type=int, default=4096, help="requests of the served-stream run (0: skip)")
    ap.add_argument("--npt-steps", type=int, default=20, help="Langevin NPT steps timed after the main run (0: skip)")
    ap.add_argument("--served-pool-mib", type=int, default=1024)
    ap.add_argument("--other-p", type=int, default=400,
                    help="also time the workload at this batch size P (0: skip)")
    ap.add_argument("--variance-reps", type=int, default=1000,
                    help="steps per sampler, P and size in the estimator-variance study (0: skip)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the multi-GPU decomposition "
              "is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_23582_amd import rbsog

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    d, desc = make_workload(args.config)
    log(f"workload {args.config} ready: {len(d['q'])} atoms")
    n = len(d["q"])
    P = int(d["P"])
    dev = "cuda"
    x, y, z = (torch.tensor(np.ascontiguousarray(d["pos"][:, k]), dtype=torch.float64, device=dev)
               for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    L0 = np.asarray(d["L"], dtype=np.float64)
    if args.graph:
        # one system as a batch of one; the step's launches replay a captured graph
        ctx = rbsog.Batch([dict(q=d["q"], box=L0, rc=d["rc"], P=P, seed=args.seed)])
        ctx.set_options(schedule=rbsog.SCHED_STATIC, graph=True)
        last = {}

        def step(s):
            target = L0 * (1.0 + 0.001 * (s % 10))
            mu = target / ctx.boxes[0]
            ctx.rescale(mu[None, :], x, y, z)
            Pb, _, inf = ctx.step(s, ctx.boxes, x, y, z, fx, fy, fz, energy=False)
            last["info"] = inf[0]
            return Pb[0]
    else:
        ctx = rbsog.Context(d["q"], L0, d["rc"], P=P, seed=args.seed, precision=rbsog.PREC_FP32C,
                            flags=SHELL_FLAGS[args.shell])

        def step(s):
            target = L0 * (1.0 + 0.001 * (s % 10))
            mu = target / ctx.box
            if not args.separate_calls:
                # rbsog_step: rescale, sampling, forces and pressure in one call
                return ctx.step(s, mu, x, y, z, fx, fy, fz)[0]
            ctx.rescale(mu, x, y, z)
            ctx.sample_modes(s, ctx.box)
            ctx.force_virial(x, y, z, fx, fy, fz, energy=False)
            return ctx.pressure()[0]

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    if not args.graph:
        ctx.set_timing(2)  # events around the pair kernel only: each recorded event delays the next launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if pipelined(args):
        # every step's pressure reaches the host, read once the next step is queued
        marks = run_queued(ctx, range(args.warmup, args.warmup + args.steps),
                           lambda s: L0 * (1.0 + 0.001 * (s % 10)) / ctx.box, (x, y, z, fx, fy, fz))
    else:
        marks = []
        for s in range(args.warmup, args.warmup + args.steps):
            step(s)  # ends with the pressure copied to the host (a stream synchronisation)
            marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_step = 1e3 * np.diff(np.concatenate([[t0], marks]))
    if not args.graph:
        timing_pair = ctx.get_timing()["pair"]
        info = ctx.step_info()
        # the other kernels' times from a few more steps with every launch timed
        ctx.set_timing(1)
        for s in range(args.warmup + args.steps, args.warmup + args.steps + 5):
            step(s)
        torch.cuda.synchronize()
        timing = ctx.get_timing()
        timing["pair"] = timing_pair
        ctx.set_timing(False)
    else:
        # per-kernel times from a few eager steps of the same launches (events
        # cannot be recorded inside the replayed graph)
        ctx.set_timing(True)
        for s in range(args.warmup + args.steps, args.warmup + args.steps + 3):
            step(s)
        torch.cuda.synchronize()
        timing = ctx.get_timing()
        ctx.set_timing(False)
        inf = last["info"]
        info = dict(nd=int(inf[0]), acc_r=int(inf[1]), acc_nr=int(inf[2]), npairs=int(inf[3]))
    T = t1 - t0
    ms_step = 1e3 * T / args.steps
    value = n * args.steps / T

    log(f"{args.steps} timed steps: {ms_step:.3f} ms/step")
    probe = None if args.no_valu_probe else valu_probe()
    tw = TRANS_WEIGHT_DEFAULT
    if probe:
        tw = probe["fma"]["valu_per_simd_cycle"] / probe["exp"]["trans_per_simd_cycle"]
    pair_ms, pair_cnt = timing.get("pair", (0.0, 1))
    t_pair = pair_ms / max(pair_cnt, 1) * 1e-3
    work = info["npairs"] * pair_work(tw)
    achieved = work / t_pair if t_pair > 0 else 0.0
    work_impl = info["npairs"] * pair_work_implemented(tw)
    traffic = read_traffic(args.config)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_LANE_OPS_PER_S / 1e12,
                "unit": "T FP32 lane-op/s", "frac": achieved / VALU_LANE_OPS_PER_S, "traffic": traffic,
                "kernel": "k_pair", "unordered_pairs_per_launch": info["npairs"],
                "work_per_pair": pair_work(tw), "trans_weight": tw, "avg_launch_ms": 1e3 * t_pair,
                "implemented_form": {"work_per_pair": pair_work_implemented(tw),
                                     "frac": work_impl / t_pair / VALU_LANE_OPS_PER_S if t_pair > 0 else 0.0}}
    issued = read_issued(args.config, tw)
    if issued is not None and t_pair > 0:
        # every VALU instruction the kernel issues (filter, walk, staging, both
        # sides of each pair), from the committed counters of this source
        roofline["issued"] = {"lane_ops_per_launch": issued, "per_unordered_pair": issued / info["npairs"],
                              "frac": issued / t_pair / VALU_LANE_OPS_PER_S}
    sk_w, fo_w = mode_work(tw)
    kernels = {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in timing.items()}
    for k, per in (("sk", sk_w), ("force", fo_w)):
        if k in kernels and kernels[k]["avg_ms"] > 0:
            kernels[k]["frac_valu"] = n * info["nd"] * per / (kernels[k]["avg_ms"] * 1e-3) / VALU_LANE_OPS_PER_S
    cpu = None
    if not args.no_cpu_baseline:
        log("oracle on the host cores")
        cpu = cpu_baseline(d, P, args.seed, args.cpu_sample, args.cpu_single_sample)
    out = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step,
        "ms_per_step_percentiles": {"p10": float(np.percentile(per_step, 10)),
                                    "median": float(np.percentile(per_step, 50)),
                                    "p90": float(np.percentile(per_step, 90))},
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "n_atoms": n, "box": L0.tolist(), "rc": d["rc"], "P": P,
                   "precision": "FP32C (FP32 arithmetic, FP64 partial sums and reductions)",
                   "parallelism": "single GPU",
                   "api": "batch of one, HIP graph" if args.graph else
                          ("context, four calls a step" if args.separate_calls else
                           ("context, rbsog_step" if args.sync_steps else
                            "context, rbsog_step_async (each step's pressure read once the next step is queued)"))},
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kernels,
        "distinct_modes": info["nd"], "valu_probe": probe,
    }
    if args.other_p > 0 and not args.graph:
        # the same workload at another batch size (the slab config names P = 100 and 400)
        log(f"P = {args.other_p}: {args.steps} steps")
        with rbsog.Context(d["q"], ctx.box, d["rc"], P=args.other_p, seed=args.seed) as c2:
            def step2(s):
                if not args.separate_calls:
                    return c2.step(s, None, x, y, z, fx, fy, fz)[0]
                c2.sample_modes(s, c2.box)
                c2.force_virial(x, y, z, fx, fy, fz, energy=False)
                return c2.pressure()[0]
            for s in range(args.warmup):
                step2(s)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            if pipelined(args):
                run_queued(c2, range(args.warmup, args.warmup + args.steps), lambda s: None, (x, y, z, fx, fy, fz))
            else:
                for s in range(args.warmup, args.warmup + args.steps):
                    step2(s)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            out["other_P"] = {"P": args.other_p, "ms_per_step": 1e3 * (tb - ta) / args.steps,
                              "atom_steps_per_s": n * args.steps / (tb - ta),
                              "distinct_modes": c2.step_info()["nd"],
                              "note": "no box rescale between these steps"}
    if args.extra and args.extra != "none" and not args.graph:
        out["extra"] = {}
        for name in args.extra.split(","):
            log(f"workload {name}: {args.extra_steps} steps")
            out["extra"][name] = extra_workload(torch, name, args, tw)
    if args.npt_steps > 0 and not args.graph:
        log(f"NPT integration: {args.npt_steps} steps")
        out["npt"] = npt_bench(torch, ctx, d, x, y, z, args.npt_steps, ms_step)
    if args.variance_reps > 0 and not args.graph:
        log(f"estimator variance: {args.variance_reps} steps per sampler, P and size")
        out["variance"] = variance_study(torch, args.variance_reps)
    if args.served > 0:
        log(f"served stream: {args.served} requests")
        out["served"] = served_bench(args.served, 5, args.served_pool_mib << 20)
    ctx.close()
    if args.calibration_copy_mib > 0:
        src = torch.ones(args.calibration_copy_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
