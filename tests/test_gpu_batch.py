"""Batched and served forms through the C ABI.

A system's results do not depend on the company it keeps: every system of a
batch, and every request of the server, must give the same bits as the same
system evaluated alone through the single-system calls (which are checked
against the FP64 oracle in test_gpu_parity.py).  A few systems of the batch
are also checked against the oracle directly.  Launch options (static or
persistent pair schedule, HIP-graph replay, the autotuner's choice) must not
change a single bit either.
"""
import numpy as np
import pytest

from paper_2602_23582_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FP32C = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


@pytest.fixture(scope="module")
def rb():
    from paper_2602_23582_amd import rbsog
    rbsog.load()
    return rbsog


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _systems():
    """Uneven systems: served-stream sizes, the lattice, a small slab-like box."""
    out = []
    for n, seed in [(500, 11), (2_400, 12), (9_000, 13), (31_000, 14)]:
        d = W.ionic_system(n, seed)
        out.append(dict(q=d["q"], pos=d["pos"], box=d["L"], rc=d["rc"], P=d["P"], seed=seed, system_id=n))
    d = W.c1_lattice()
    out.append(dict(q=d["q"], pos=d["pos"], box=d["L"], rc=d["rc"], P=100, seed=7, system_id=0))
    return out


def _alone(torch, rb, spec, step, box):
    """One step of one system through the single-system calls."""
    with rb.Context(spec["q"], spec["box"], spec["rc"], P=spec["P"], seed=spec["seed"],
                    system_id=spec["system_id"], M=spec.get("M", 10), flags=spec.get("flags", 0),
                    recalibration=spec.get("recalibration", rb.RECAL_EXCHANGE)) as ctx:
        x, y, z = (_dev(torch, spec["pos"][:, k]) for k in range(3))
        fx, fy, fz = (torch.empty_like(x) for _ in range(3))
        ctx.sample_modes(step, box)
        e, _ = ctx.force_virial(x, y, z, fx, fy, fz)
        P, _ = ctx.pressure()
        return torch.stack([fx, fy, fz], 1).cpu().numpy(), P, e


def _concat(torch, systems):
    pos = np.concatenate([s["pos"] for s in systems])
    x, y, z = (_dev(torch, pos[:, k]) for k in range(3))
    fx, fy, fz = (torch.zeros_like(x) for _ in range(3))
    return (x, y, z), (fx, fy, fz)


def _split(torch, f, offsets):
    F = torch.stack(f, 1).cpu().numpy()
    return [F[offsets[s]:offsets[s + 1]] for s in range(len(offsets) - 1)]


def test_batch_equals_each_system_alone(torch, rb):
    systems = _systems()
    steps = [3, 0, 17, 5, 2]
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P, U, info = b.step(steps, boxes, x, y, z, *f)
        Fs = _split(torch, f, b.offsets)
    for s, spec in enumerate(systems):
        F1, P1, e1 = _alone(torch, rb, spec, steps[s], spec["box"])
        print(f"system {s}: n {len(spec['q'])} modes {info[s, 0]} pairs {info[s, 3]}", flush=True)
        assert np.array_equal(Fs[s], F1), f"system {s}: forces differ from the system alone"
        assert np.array_equal(P[s], P1), f"system {s}: pressure differs from the system alone"
        assert np.array_equal(U[s], e1), f"system {s}: energies differ from the system alone"


def test_batch_systems_match_oracle(torch, rb, orc):
    systems = _systems()[:3]
    steps = [1, 2, 3]
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P, U, _ = b.step(steps, boxes, x, y, z, *f)
        Fs = _split(torch, f, b.offsets)
    for s, spec in enumerate(systems):
        p = orc.sog(spec["rc"], row=2, M=10)
        o = orc.rbsog_step(spec["q"], spec["pos"], spec["box"], p, spec["P"], spec["seed"], spec["system_id"],
                           steps[s])
        fr = np.sqrt(((Fs[s] - o["F"]) ** 2).sum() / (o["F"] ** 2).sum())
        pr = np.linalg.norm(P[s] - o["P"]) / np.linalg.norm(o["P"])
        u = U[s, 0] + U[s, 1] - U[s, 2]
        ur = abs(u - o["U"]) / abs(o["U"])
        print(f"system {s}: F {fr:.2e} P {pr:.2e} U {ur:.2e}", flush=True)
        assert fr <= TOL_FP32C and pr <= TOL_FP32C and ur <= TOL_FP32C


@pytest.mark.parametrize("schedule,wg", [(1, 4), (1, 16), (1, 64)])
def test_pair_schedules_are_bitwise_identical(torch, rb, schedule, wg):
    systems = _systems()
    steps = [4] * len(systems)
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P0, U0, _ = b.step(steps, boxes, x, y, z, *f)
        F0 = torch.stack(f, 1).clone()
        b.set_options(schedule=schedule, wg_per_cu=wg)
        P1, U1, _ = b.step(steps, boxes, x, y, z, *f)
        assert torch.equal(F0, torch.stack(f, 1))
        assert np.array_equal(P0, P1) and np.array_equal(U0, U1)


def test_graph_replays_match_eager_steps(torch, rb):
    systems = _systems()[:4]
    boxes0 = np.array([s["box"] for s in systems])
    (x, y, z), f = _concat(torch, systems)
    x2, y2, z2 = x.clone(), y.clone(), z.clone()
    f2 = tuple(torch.zeros_like(x) for _ in range(3))
    with rb.Batch(systems) as eager, rb.Batch(systems) as graph:
        graph.set_options(schedule=1, wg_per_cu=16, graph=True)
        for k in range(4):
            # eager work between the replays: a rescale of both position sets
            mu = 1.0 + 0.001 * k
            if k:
                eager.rescale([mu, mu, mu], x, y, z)
                graph.rescale([mu, mu, mu], x2, y2, z2)
            Pe, Ue, _ = eager.step(k, eager.boxes, x, y, z, *f)
            Pg, Ug, _ = graph.step(k, graph.boxes, x2, y2, z2, *f2)
            torch.cuda.synchronize()
            assert np.array_equal(Pe, Pg) and np.array_equal(Ue, Ug), f"replay {k}"
            assert torch.equal(torch.stack(f, 1), torch.stack(f2, 1)), f"replay {k}"
        assert np.allclose(eager.boxes, boxes0 * 1.001 * 1.002 * 1.003, rtol=1e-14)


def test_autotune_keeps_results(torch, rb):
    systems = _systems()
    steps = [9] * len(systems)
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        # the autotuner's timed steps leave the energy sum out
        P0, U0, _ = b.step(steps, boxes, x, y, z, *f, energy=False)
        F0 = torch.stack(f, 1).clone()
        choice, ms = b.autotune(steps, boxes, x, y, z, *f, reps=2)
        print("autotune", choice, ms, flush=True)
        assert 0 <= choice < len(rb.AUTOTUNE_CANDIDATES) and np.all(ms > 0)
        assert torch.equal(F0, torch.stack(f, 1))
        P1, U1, _ = b.step(steps, boxes, x, y, z, *f, energy=False)
        assert np.array_equal(P0, P1) and np.array_equal(U0, U1)


def test_cached_autotune_reads_back_its_choice(torch, rb, tmp_path):
    """rbsog_batch_autotune_cached: a first call times the ten candidates
    (schedules with and without graph replay) and appends the fastest to the
    cache file; a second call for the same key applies it without timing; a
    forced call times again.  Results are bitwise the same under every
    choice."""
    systems = _systems()
    steps = [9] * len(systems)
    boxes = np.array([s["box"] for s in systems])
    path = tmp_path / "tune.txt"
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P0, U0, _ = b.step(steps, boxes, x, y, z, *f, energy=False)
        F0 = torch.stack(f, 1).clone()
        c1, ms1, hit1 = b.autotune_cached(path, steps, boxes, x, y, z, *f, reps=2)
        print("autotune_cached", c1, rb.TUNE_CANDIDATES[c1], ms1, flush=True)
        assert not hit1 and 0 <= c1 < len(rb.TUNE_CANDIDATES) and np.all(ms1 > 0)
        assert ms1[c1] == ms1.min()
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and lines[0].split("|")[1].split()[0] == str(c1)
        P1, U1, _ = b.step(steps, boxes, x, y, z, *f, energy=False)
        assert np.array_equal(P0, P1) and np.array_equal(U0, U1) and torch.equal(F0, torch.stack(f, 1))
        c2, ms2, hit2 = b.autotune_cached(path, steps, boxes, x, y, z, *f, reps=2)
        assert hit2 and c2 == c1 and abs(ms2[c1] - ms1[c1]) < 1e-5 and np.count_nonzero(ms2) == 1
        assert len(path.read_text().splitlines()) == 1
        P2, U2, _ = b.step(steps, boxes, x, y, z, *f, energy=False)
        assert np.array_equal(P0, P2) and np.array_equal(U0, U2) and torch.equal(F0, torch.stack(f, 1))
        c3, ms3, hit3 = b.autotune_cached(path, steps, boxes, x, y, z, *f, reps=1, force=True)
        assert not hit3 and np.all(ms3 > 0) and len(path.read_text().splitlines()) == 2
    # a batch of another size bucket is a key of its own
    with rb.Batch(systems[:1]) as b1:
        (x, y, z), f = _concat(torch, systems[:1])
        _, _, hit = b1.autotune_cached(path, steps[:1], boxes[:1], x, y, z, *f, reps=1)
        keys = [l.split("|")[0] for l in path.read_text().splitlines()]
        assert not hit and len(set(keys)) == 2


def test_energy_request_keeps_forces_and_pressure(torch, rb):
    """With the energy sum the fast path takes pair displacements from exact
    fixed-point differences, without it from FP32 block-relative coordinates:
    forces and pressure agree to the rounding of those coordinates, and each
    setting is bitwise reproducible."""
    spec = _systems()[3]
    with rb.Context(spec["q"], spec["box"], spec["rc"], P=spec["P"], seed=spec["seed"]) as ctx:
        x, y, z = (_dev(torch, spec["pos"][:, k]) for k in range(3))
        out = []
        for energy in (True, False, True):
            fx, fy, fz = (torch.empty_like(x) for _ in range(3))
            ctx.sample_modes(5, spec["box"])
            ctx.force_virial(x, y, z, fx, fy, fz, energy=energy)
            out.append((torch.stack([fx, fy, fz], 1).cpu().numpy(), ctx.pressure()[0]))
    assert np.array_equal(out[2][0], out[0][0]) and np.array_equal(out[2][1], out[0][1])
    F0, P0 = out[0]
    F1, P1 = out[1]
    fr = np.sqrt(((F1 - F0) ** 2).sum() / (F0 ** 2).sum())
    pr = np.linalg.norm(P1 - P0) / np.linalg.norm(P0)
    print(f"energy on/off: force rel RMS {fr:.2e}, pressure {pr:.2e}", flush=True)
    assert fr < 2e-6 and pr < 1e-6


def test_mixed_forms_keep_each_system_exact(torch, rb):
    """Polynomial and exponential FP32C forms in one batch."""
    systems = _systems()[:4]
    systems[2] = dict(systems[2], flags=rb.FLAG_EXP_FORM)
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P, U, _ = b.step([6] * 4, boxes, x, y, z, *f)
        Fs = _split(torch, f, b.offsets)
    for s, spec in enumerate(systems):
        F1, P1, e1 = _alone(torch, rb, spec, 6, spec["box"])
        assert np.array_equal(Fs[s], F1) and np.array_equal(P[s], P1) and np.array_equal(U[s], e1), f"system {s}"


def test_mixed_term_counts_keep_each_system_exact(torch, rb):
    systems = _systems()[:3]
    systems[1] = dict(systems[1], M=12)
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P, U, _ = b.step([2, 2, 2], boxes, x, y, z, *f)
        Fs = _split(torch, f, b.offsets)
    for s, spec in enumerate(systems):
        F1, P1, _ = _alone(torch, rb, spec, 2, spec["box"])
        assert np.array_equal(Fs[s], F1) and np.array_equal(P[s], P1), f"system {s}"


def test_mixed_samplers_keep_each_system_exact(torch, rb):
    """All four non-radial samplers in one batch: the independent chain's
    systems hold 2P + 1 mode slots beside systems holding P + 1."""
    systems = _systems()[:4]
    for s, v in enumerate([rb.RECAL_INDEPENDENT, rb.RECAL_PRINTED, rb.RECAL_SHARED, rb.RECAL_EXCHANGE]):
        systems[s] = dict(systems[s], recalibration=v)
    boxes = np.array([s["box"] for s in systems])
    with rb.Batch(systems) as b:
        (x, y, z), f = _concat(torch, systems)
        P, U, info = b.step([4] * 4, boxes, x, y, z, *f)
        Fs = _split(torch, f, b.offsets)
    assert info[0, 0] <= 2 * systems[0]["P"] + 1
    for s, spec in enumerate(systems):
        F1, P1, e1 = _alone(torch, rb, spec, 4, spec["box"])
        assert np.array_equal(Fs[s], F1) and np.array_equal(P[s], P1) and np.array_equal(U[s], e1), f"system {s}"


# --------------------------------------------------------------------------
# served form
# --------------------------------------------------------------------------

@pytest.mark.parametrize("graph", [False, True])
def test_batch_grid_growth_matches_fresh_batches(torch, rb, graph):
    """Boxes that grow past cell boundaries re-carve the cell arrays inside a
    batch (eager and graph replay); each step equals a fresh batch at that box."""
    d = W.water_box(n_mol=8000, seed=21)
    spec = dict(q=d["q"], box=d["L"], rc=d["rc"], P=100, seed=9)
    b = rb.Batch([spec])
    b.set_options(graph=graph)
    for k, g in enumerate([1.0, 1.15, 1.30, 1.0, 1.45, 1.15]):
        box = d["L"] * g
        print(f"graph {graph} growth {g}", flush=True)
        (x, y, z), f = _concat(torch, [dict(pos=d["pos"] * g)])
        P, _, _ = b.step(k, box[None, :], x, y, z, *f)
        fresh = rb.Batch([dict(spec, box=box)])
        (x2, y2, z2), f2 = _concat(torch, [dict(pos=d["pos"] * g)])
        P2, _, _ = fresh.step(k, box[None, :], x2, y2, z2, *f2)
        fresh.close()
        assert np.array_equal(_split(torch, f, [0, len(d["q"])])[0], _split(torch, f2, [0, len(d["q"])])[0])
        assert np.array_equal(P, P2)
    b.close()


def _requests(k=6, seed=3):
    sizes, seeds = W.served_stream(k, seed=seed, n_max=12_000)
    out = []
    for n, sd in zip(sizes, seeds):
        d = W.ionic_system(int(n), int(sd))
        out.append(dict(q=d["q"], pos=d["pos"], box=d["L"], rc=d["rc"], P=d["P"], seed=int(sd),
                        system_id=int(n)))
    return out


def _alone_steps(torch, rb, spec, nsteps, growth, energy=True):
    """The request's box law run through the single-system calls."""
    box = np.array(spec["box"], dtype=np.float64)
    with rb.Context(spec["q"], box, spec["rc"], P=spec["P"], seed=spec["seed"], system_id=spec["system_id"]) as ctx:
        x, y, z = (_dev(torch, spec["pos"][:, k]) for k in range(3))
        fx, fy, fz = (torch.empty_like(x) for _ in range(3))
        Ps = []
        for k in range(nsteps):
            if k:
                mu = (1.0 + growth * k) / (1.0 + growth * (k - 1))
                ctx.rescale([mu, mu, mu], x, y, z)
            ctx.sample_modes(k, ctx.box)
            ctx.force_virial(x, y, z, fx, fy, fz, energy=energy)
            Ps.append(ctx.pressure()[0])
        return torch.stack([fx, fy, fz], 1).cpu().numpy(), np.array(Ps)


@pytest.mark.parametrize("energy", [True, False])
def test_server_results_alone_equal_results_in_the_mix(torch, rb, energy):
    reqs = _requests()
    nsteps, growth = 3, 0.001
    with rb.Server(max_active=64, energy=energy) as sv:
        tickets = [sv.submit(r["q"], r["pos"], r["box"], r["rc"], nsteps=nsteps, growth=growth, P=r["P"],
                             seed=r["seed"], system_id=r["system_id"]) for r in reqs]
        mix = [sv.wait(t, timeout=120.0) for t in tickets]
        st = sv.stats()
    print("server stats", st, flush=True)
    assert all(m is not None for m in mix)
    assert st["completed"] == len(reqs) and st["peak_active"] >= 2
    assert sum(m["shared_ticks"] for m in mix) > 0
    for r, m in zip(reqs, mix):
        F1, P1 = _alone_steps(torch, rb, r, nsteps, growth, energy)
        assert np.array_equal(m["forces"], F1), "forces in the mix differ from the request alone"
        assert np.array_equal(m["P"], P1), "pressures in the mix differ from the request alone"
        assert energy or not np.any(m["U"]), "energies reported although the server skips them"
    # one request at a time gives the same bits too
    with rb.Server(max_active=1, energy=energy) as sv:
        t = sv.submit(reqs[0]["q"], reqs[0]["pos"], reqs[0]["box"], reqs[0]["rc"], nsteps=nsteps, growth=growth,
                      P=reqs[0]["P"], seed=reqs[0]["seed"], system_id=reqs[0]["system_id"])
        solo = sv.wait(t, timeout=60.0)
    assert solo["shared_ticks"] == 0
    assert np.array_equal(solo["forces"], mix[0]["forces"]) and np.array_equal(solo["P"], mix[0]["P"])


def test_full_served_stream_sampled(torch, rb, orc):
    """The served workload at full size, in the configuration the benchmark
    times at capacity: 4,096 requests of 500-50,000 atoms (stream seed 5), 10
    steps each under L_k = L_(k-1) (1 + 0.001 k) / (1 + 0.001 (k - 1)), force +
    pressure solves from a 4 GiB pool, all submitted at once.  Sampled
    requests: the smallest, the largest and four more give the same bits alone
    as in the mix; three of at most 6,000 atoms match the oracle at their last
    step within 1e-5."""
    nsteps, growth, nreq = 10, 0.001, 4096
    sizes, seeds = W.served_stream(nreq, seed=5)
    reqs = [W.ionic_system(int(n), int(sd)) for n, sd in zip(sizes, seeds)]
    print(f"served stream: {nreq} requests, {int(sizes.sum())} atoms", flush=True)
    with rb.Server(max_active=65536, pool_bytes=4 << 30, energy=False) as sv:
        tickets = [sv.submit(r["q"], r["pos"], r["L"], r["rc"], nsteps=nsteps, growth=growth, P=r["P"],
                             seed=int(seeds[i]), system_id=i) for i, r in enumerate(reqs)]
        res = [sv.wait(t, timeout=300.0) for t in tickets]
        st = sv.stats()
    print("server stats", st, flush=True)
    assert all(m is not None for m in res) and st["completed"] == nreq and st["peak_active"] > 1000
    rng = np.random.default_rng(11)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *rng.choice(nreq, 4, replace=False).tolist()})
    for i in pick:
        r = reqs[i]
        spec = dict(q=r["q"], pos=r["pos"], box=r["L"], rc=r["rc"], P=r["P"], seed=int(seeds[i]), system_id=i)
        F1, P1 = _alone_steps(torch, rb, spec, nsteps, growth, energy=False)
        print(f"request {i}: {len(r['q'])} atoms, alone vs mix", flush=True)
        assert np.array_equal(res[i]["forces"], F1) and np.array_equal(res[i]["P"], P1), i
    small = [int(i) for i in rng.permutation(nreq) if sizes[i] <= 6000][:3]
    for i in small:
        r = reqs[i]
        L, pos = np.array(r["L"], dtype=np.float64), np.array(r["pos"], dtype=np.float64)
        for k in range(1, nsteps):  # the server's box law and device rescale, both in FP64
            m = (1.0 + growth * k) / (1.0 + growth * (k - 1))
            L, pos = L * m, pos * m
        o = orc.rbsog_step(r["q"], pos, L, orc.sog(r["rc"], row=2, M=10), r["P"], int(seeds[i]), i, nsteps - 1)
        F, P = res[i]["forces"], res[i]["P"][-1]
        fr = np.sqrt(((F - o["F"]) ** 2).sum() / (o["F"] ** 2).sum())
        pr = np.linalg.norm(P - o["P"]) / np.linalg.norm(o["P"])
        print(f"request {i}: {len(r['q'])} atoms vs oracle: F {fr:.2e} P {pr:.2e}", flush=True)
        assert fr < TOL_FP32C and pr < TOL_FP32C, (i, fr, pr)


def test_server_admission_is_bounded_by_the_memory_pool(torch, rb):
    reqs = _requests(8, seed=9)
    # a pool that holds only a few of these requests at once
    pool = 24 << 20
    with rb.Server(pool_bytes=pool, max_active=64) as sv:
        tickets = [sv.submit(r["q"], r["pos"], r["box"], r["rc"], nsteps=2, P=r["P"], seed=r["seed"],
                             system_id=r["system_id"]) for r in reqs]
        res = [sv.wait(t, timeout=120.0) for t in tickets]
        st = sv.stats()
    print("bounded pool", st, flush=True)
    assert all(r is not None for r in res)
    assert st["peak_pool_bytes"] <= pool
    assert st["completed"] == len(reqs)


def test_server_energy_setting_is_fixed_after_the_first_request(torch, rb):
    r = _requests(1, seed=4)[0]
    with rb.Server(max_active=4) as sv:
        sv.set_energy(False)
        sv.set_energy(True)
        t = sv.submit(r["q"], r["pos"], r["box"], r["rc"], nsteps=1, P=r["P"], seed=r["seed"])
        with pytest.raises(rb.RBSOGError) as ei:
            sv.set_energy(False)
        assert ei.value.code == -6
        assert sv.wait(t, timeout=60.0) is not None


def test_server_rejects_a_request_larger_than_the_pool(torch, rb):
    r = _requests(1, seed=4)[0]
    with rb.Server(pool_bytes=1 << 16, max_active=4) as sv:
        with pytest.raises(rb.RBSOGError) as ei:
            sv.submit(r["q"], r["pos"], r["box"], r["rc"], nsteps=2, P=r["P"], seed=r["seed"])
        assert ei.value.code == -7
