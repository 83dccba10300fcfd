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

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = VALU issue slots per second
# (one non-packed FP32 lane-op per slot; transcendentals take 4 slots).
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
TRANS_SLOTS = 4


def pair_slots(M):
    """VALU slots of one unordered in-cutoff pair in the paper's M-exp form:
    displacement 3, r^2 3, cutoff test 1, r^-3 from r^-1 2, exponent scaling M,
    two weighted Gaussian sums 2M, N~ and N 2, q_i q_j and f 2, force on both
    atoms 9, virial 6, energy 1; transcendentals: r^-1 and M exponentials."""
    ops = 29 + 3 * M
    trans = 1 + M
    return ops + TRANS_SLOTS * trans


def mode_slots():
    """VALU slots per (atom, distinct mode) of the structure factor (3 integer
    multiply-adds, convert, 2 FMA + sin, cos) and of the force scatter (3
    multiply-adds, convert, 2 + 3 FMA + sin, cos)."""
    return (6 + 2 * TRANS_SLOTS), (9 + 2 * TRANS_SLOTS)


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


def read_traffic(config):
    """HBM bytes per pair-kernel launch from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"pair_kernel_{config}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernels_sha256") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def cpu_baseline(d, P, seed, sample_atoms):
    """The oracle as it stands on a bounded sample: long-range structure factors
    of all atoms for every sampled mode (2P evaluations), short-range and
    long-range forces of a random subset of atoms; the time scales to a full
    step by the subset fraction."""
    from oracle import oracle as orc
    n = len(d["q"])
    p = orc.sog(d["rc"], row=2, M=10)
    rng = np.random.default_rng(0)
    k = min(n, sample_atoms)
    smp = np.sort(rng.choice(n, k, replace=False))
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
    t_step = (t1 - t0) + (t2 - t1) + per_atom * n
    return {"value": n / t_step, "unit": "atom-steps/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{k} of {n} atoms for short- and long-range forces, structure factors of all atoms for "
                      f"the {2 * P} sampled modes, one step; per-atom time scaled to all atoms",
            "seconds": t3 - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="slab-1m")
    ap.add_argument("--seed", type=int, default=2026)
    ap.add_argument("--cpu-sample", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-valu-probe", action="store_true")
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
    n = len(d["q"])
    P = int(d["P"])
    dev = "cuda"
    x, y, z = (torch.tensor(np.ascontiguousarray(d["pos"][:, k]), dtype=torch.float64, device=dev)
               for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    L0 = np.asarray(d["L"], dtype=np.float64)
    ctx = rbsog.Context(d["q"], L0, d["rc"], P=P, seed=args.seed, precision=rbsog.PREC_FP32C)

    def step(s):
        target = L0 * (1.0 + 0.001 * (s % 10))
        mu = target / ctx.box
        ctx.rescale(mu, x, y, z)
        ctx.sample_modes(s, ctx.box)
        ctx.force_virial(x, y, z, fx, fy, fz, energy=False)
        return ctx.pressure()

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        step(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = ctx.get_timing()
    info = ctx.step_info()
    ctx.set_timing(False)
    T = t1 - t0
    ms_step = 1e3 * T / args.steps
    value = n * args.steps / T

    pair_ms, pair_cnt = timing.get("pair", (0.0, 1))
    t_pair = pair_ms / max(pair_cnt, 1) * 1e-3
    slots = info["npairs"] * pair_slots(10)
    achieved = slots / t_pair if t_pair > 0 else 0.0
    traffic = read_traffic(args.config)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_SLOTS_PER_S / 1e12,
                "unit": "T VALU-slot/s", "frac": achieved / VALU_SLOTS_PER_S, "traffic": traffic,
                "kernel": "k_pair", "unordered_pairs_per_launch": info["npairs"],
                "slots_per_pair": pair_slots(10), "avg_launch_ms": 1e3 * t_pair}
    sk_slots, fo_slots = mode_slots()
    kernels = {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in timing.items()}
    for k, per in (("sk", sk_slots), ("force", fo_slots)):
        if k in kernels and kernels[k]["avg_ms"] > 0:
            kernels[k]["frac_valu"] = n * info["nd"] * per / (kernels[k]["avg_ms"] * 1e-3) / VALU_SLOTS_PER_S
    probe = None if args.no_valu_probe else valu_probe()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d, P, args.seed, args.cpu_sample)
    out = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "n_atoms": n, "box": L0.tolist(), "rc": d["rc"], "P": P,
                   "precision": "FP32C (FP32 arithmetic, FP64 partial sums and reductions)",
                   "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kernels,
        "distinct_modes": info["nd"], "valu_probe": probe,
    }
    ctx.close()
    if args.calibration_copy_mib > 0:
        src = torch.ones(args.calibration_copy_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
