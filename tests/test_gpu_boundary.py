"""The C-ABI boundary beyond one context's step: a batch of existing contexts
admitted by device memory (rbsog_batch_create/admit/release, rbsog_stage,
rbsog_batch_step), the energy's own term count (M_energy), and the argument
checks on position and force arrays (NaN/Inf on the device, host and device
arrays mixed, wrong lengths)."""
import numpy as np
import pytest

from paper_2602_23582_amd import workloads as W
from test_gpu_parity import TOL_FP32C, TOL_FP64, _dev, check, gpu_step

pytestmark = pytest.mark.gpu


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


def _systems(rb):
    d1 = W.water_box(n_mol=5000, seed=3)
    d2 = W.ionic_system(12000, seed=12)
    d3 = W.ionic_system(2000, seed=20)
    return [dict(d=d1, P=100, seed=3, sid=0, flags=rb.FLAG_HALF_SHELL, step=3),
            dict(d=d2, P=50, seed=12, sid=1, flags=0, step=4),
            dict(d=d3, P=200, seed=20, sid=2, flags=0, step=5)]


def _ctx(rb, s):
    d = s["d"]
    return rb.Context(d["q"], d["L"], d["rc"], P=s["P"], seed=s["seed"], system_id=s["sid"], flags=s["flags"])


def test_context_batch_admits_by_memory_and_matches_alone(torch, rb):
    """Three contexts admitted to one batch give, after one batched step,
    bitwise the forces, pressures and energies each gives alone; a budget too
    small refuses admission with RBSOG_EAGAIN; an admitted context refuses its
    own evaluation calls; a released context works alone again."""
    systems = _systems(rb)
    alone = []
    for s in systems:
        with _ctx(rb, s) as c:
            alone.append(gpu_step(torch, c, s["d"]["pos"], s["step"], s["d"]["L"]))
    ctxs = [_ctx(rb, s) for s in systems]
    with rb.ContextBatch(1) as tiny:
        assert tiny.admit(ctxs[2]) is False  # one byte of budget: refused
    arrays = []
    with rb.ContextBatch(1 << 30) as b:
        for c in ctxs:
            assert b.admit(c)
        with pytest.raises(rb.RBSOGError) as e:
            ctxs[0].sample_modes(0, systems[0]["d"]["L"])
        assert e.value.code == -6
        for c, s in zip(ctxs, systems):
            d = s["d"]
            x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
            f = [torch.empty_like(x) for _ in range(3)]
            arrays.append((x, y, z, f))
            c.stage(s["step"], d["L"], x, y, z, *f)
        P, U, info = b.step()
        for k, (c, a) in enumerate(zip(ctxs, alone)):
            F = torch.stack(arrays[k][3], 1).cpu().numpy()
            assert np.array_equal(F, a["F"]), k
            assert np.array_equal(P[k], a["P"]), k
            assert U[k, 0] + U[k, 1] - U[k, 2] == a["U"], k
            Pc, parts = c.pressure()
            assert np.array_equal(Pc, a["P"]) and np.array_equal(parts[0], a["PN"]), k
        # release the first; the other two step again from new staged inputs
        b.release(ctxs[0])
        for c, s, arr in zip(ctxs[1:], systems[1:], arrays[1:]):
            c.stage(s["step"], s["d"]["L"], *arr[:3], *arr[3])
        P2, _, _ = b.step()
        assert np.array_equal(P2[0], alone[1]["P"]) and np.array_equal(P2[1], alone[2]["P"])
    # released (and the batch closed): the contexts work alone again
    g = gpu_step(torch, ctxs[0], systems[0]["d"]["pos"], systems[0]["step"], systems[0]["d"]["L"])
    assert np.array_equal(g["F"], alone[0]["F"])
    for c in ctxs:
        c.close()


def test_context_batch_refuses_a_step_with_unstaged_members(torch, rb):
    s = _systems(rb)[2]
    with _ctx(rb, s) as c, rb.ContextBatch(1 << 30) as b:
        assert b.admit(c)
        with pytest.raises(rb.RBSOGError) as e:
            b.step()
        assert e.value.code == -6


def test_nan_device_positions_are_rejected(torch, rb):
    """A NaN or an infinity in device position arrays is flagged by the binning
    kernel and reported as RBSOG_EINVAL; the next call with finite positions
    is unaffected."""
    d = W.ionic_system(3000, seed=4)
    with rb.Context(d["q"], d["L"], d["rc"], P=50, seed=1) as c:
        good = gpu_step(torch, c, d["pos"], 1, d["L"])
        for bad in (np.nan, np.inf):
            pos = d["pos"].copy()
            pos[1234, 1] = bad
            with pytest.raises(rb.RBSOGError) as e:
                gpu_step(torch, c, pos, 1, d["L"])
            assert e.value.code == -1
        again = gpu_step(torch, c, d["pos"], 1, d["L"])
    assert np.array_equal(good["F"], again["F"]) and np.array_equal(good["P"], again["P"])


def test_mixed_host_device_arrays_and_wrong_lengths_are_rejected(torch, rb):
    d = W.ionic_system(3000, seed=4)
    with rb.Context(d["q"], d["L"], d["rc"], P=50, seed=1) as c:
        c.sample_modes(0, d["L"])
        x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
        f = [torch.empty_like(x) for _ in range(3)]
        with pytest.raises(rb.RBSOGError) as e:
            c.force_virial(x, np.ascontiguousarray(d["pos"][:, 1]), z, *f)
        assert e.value.code == -1
        with pytest.raises(ValueError):
            c.force_virial(x[:-1], y[:-1], z[:-1], *f)
        with pytest.raises(ValueError):
            c.force_virial(x, y, z, f[0][:10], f[1], f[2])


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_energy_term_count(torch, rb, orc, precision):
    """M_energy = 25 (Table 1 row 2's energy column) with M = 10: U^N and
    U_self take 25 Gaussians, U^{F*} the 25-term energy kernel sampled under
    the 10-term proposal; forces, pressure and the modes stay those of M = 10."""
    if precision == "fp64":
        d = W.c1_lattice(seed=1, jitter=0.2)
        prec, tol = rb.PREC_FP64, TOL_FP64
    else:
        d = W.water_box(n_mol=3000, seed=9)
        prec, tol = rb.PREC_FP32C, TOL_FP32C
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=6, precision=prec, M_energy=25) as c:
        g = gpu_step(torch, c, d["pos"], 2, d["L"])
    p = orc.sog(d["rc"], row=2, M=10)
    pe = orc.sog(d["rc"], row=2, M=25)
    o = orc.rbsog_step(d["q"], d["pos"], d["L"], p, 100, 6, 0, 2)
    gf = dict(g)
    gf["U"] = None  # forces, pressure and parts against the M = 10 oracle
    check(gf, o, tol, f"M_energy 25 {precision}: forces and pressure")
    _, _, UN = orc.short_range(d["q"], d["pos"], d["L"], pe)
    US = orc.self_energy(pe, d["q"])
    UF = orc.uf_rb_energy(d["q"], d["pos"], d["L"], o["m_r"], o["Sr"], p, pe)
    U = UN + UF - US
    for name, a, b in (("UN", g["UN"], UN), ("UF", g["UF"], UF), ("Uself", g["Uself"], US), ("U", g["U"], U)):
        err = abs(a - b) / abs(U)
        print(f"M_energy 25 {precision}: {name} {a:.10e} vs {b:.10e}, {err:.2e} of |U|", flush=True)
        assert err < tol, name
    # the extra wide terms change the energy, not the forces
    assert abs(g["U"] - o["U"]) > 10 * tol * abs(U)
