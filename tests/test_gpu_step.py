"""rbsog_step (rescale, sampling, forces and pressure in one call) against the
four separate calls it stands for: positions, boxes, forces, pressures and
energies bitwise equal over several steps, with and without the rescale and
the energy sum, on the fast (FP32C, at least four cells per edge) and exact
paths; and its refusals."""
import numpy as np
import pytest

from paper_2602_23582_amd import workloads as W

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


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _run(torch, rb, d, precision, fused, mus, energy):
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    out = []
    with rb.Context(d["q"], d["L"], d["rc"], P=60, seed=5, precision=precision) as ctx:
        for s, mu in enumerate(mus):
            if fused:
                P, e = ctx.step(s, mu, x, y, z, fx, fy, fz, energy=energy)
            else:
                if mu is not None:
                    ctx.rescale(mu, x, y, z)
                ctx.sample_modes(s, ctx.box)
                e, _ = ctx.force_virial(x, y, z, fx, fy, fz, energy=energy)
                P, _ = ctx.pressure()
            out.append(dict(box=ctx.box.copy(), P=P.copy(), e=None if e is None else e.copy(),
                            F=torch.stack([fx, fy, fz], 1).cpu().numpy(),
                            X=torch.stack([x, y, z], 1).cpu().numpy(), info=ctx.step_info()))
    return out


@pytest.mark.parametrize("energy", [False, True])
@pytest.mark.parametrize("case", ["fast", "exact", "fp64"])
def test_step_equals_the_separate_calls(torch, rb, case, energy):
    if case == "fast":
        d = W.ionic_system(20000, seed=3)  # at least four cells per edge: the relative-coordinate path
    else:
        d = W.ionic_system(3000, seed=3)
    precision = rb.PREC_FP64 if case == "fp64" else rb.PREC_FP32C
    mus = [None, np.array([1.002, 1.002, 0.999]), np.array([0.998, 1.0, 1.001]), None]
    a = _run(torch, rb, d, precision, False, mus, energy)
    b = _run(torch, rb, d, precision, True, mus, energy)
    for k, (u, v) in enumerate(zip(a, b)):
        assert np.array_equal(u["box"], v["box"]), (case, k)
        assert np.array_equal(u["X"], v["X"]), (case, k)
        assert np.array_equal(u["F"], v["F"]), (case, k)
        assert np.array_equal(u["P"], v["P"]), (case, k)
        assert u["info"] == v["info"], (case, k)
        if energy:
            assert np.array_equal(u["e"], v["e"]), (case, k)
    assert np.abs(a[-1]["F"]).max() > 0


def test_step_refusals(torch, rb):
    d = W.ionic_system(3000, seed=1)
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    with rb.Context(d["q"], d["L"], d["rc"], P=30, seed=1) as ctx:
        box0 = ctx.box.copy()
        with pytest.raises(rb.RBSOGError) as e:
            ctx.step(0, np.array([1.0, -1.0, 1.0]), x, y, z, fx, fy, fz)
        assert e.value.code == -1
        assert np.array_equal(ctx.box, box0)
        hx = np.ascontiguousarray(d["pos"][:, 0])
        with pytest.raises(rb.RBSOGError) as e:
            ctx.step(0, None, hx, y, z, fx, fy, fz)
        assert e.value.code == -1
        # a scale that leaves the cut-off more than half the box
        with pytest.raises(rb.RBSOGError) as e:
            ctx.step(0, np.array([0.1, 1.0, 1.0]), x, y, z, fx, fy, fz)
        assert e.value.code == -3
        assert np.array_equal(ctx.box, box0)
        assert np.array_equal(x.cpu().numpy(), d["pos"][:, 0])
        P, _ = ctx.step(0, None, x, y, z, fx, fy, fz)
        assert np.all(np.isfinite(P))


@pytest.mark.parametrize("energy", [False, True])
def test_queued_steps_equal_the_one_call_step(torch, rb, energy):
    """rbsog_step_async + rbsog_step_wait, each pressure read one step late:
    the same pressures, energies, forces and positions as rbsog_step."""
    d = W.ionic_system(20000, seed=7)
    mus = [None, np.array([1.001, 1.001, 1.0]), np.array([0.999, 1.0, 1.002]), None, np.array([1.0, 0.999, 1.0]),
           None]
    ref = []
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    with rb.Context(d["q"], d["L"], d["rc"], P=60, seed=5) as ctx:
        for s, mu in enumerate(mus):
            P, e = ctx.step(s, mu, x, y, z, fx, fy, fz, energy=energy)
            ref.append((P.copy(), None if e is None else e.copy(), ctx.box.copy()))
        F_ref = torch.stack([fx, fy, fz], 1).cpu().numpy()
        X_ref = torch.stack([x, y, z], 1).cpu().numpy()
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    got = []
    with rb.Context(d["q"], d["L"], d["rc"], P=60, seed=5) as ctx:
        tickets = []
        for s, mu in enumerate(mus):
            tickets.append((ctx.step_async(s, mu, x, y, z, fx, fy, fz, energy=energy), ctx.box.copy()))
            if len(tickets) > 1:
                t, box = tickets.pop(0)
                got.append((*ctx.step_wait(t, energy=energy), box))
        t, box = tickets.pop(0)
        got.append((*ctx.step_wait(t, energy=energy), box))
        # a ticket may be read again while its slot holds it
        P_again, _ = ctx.step_wait(t)
        assert np.array_equal(P_again, got[-1][0])
        # slots are reused after four steps
        with pytest.raises(rb.RBSOGError) as err:
            ctx.step_wait(0)
        assert err.value.code == -1
        with pytest.raises(rb.RBSOGError):
            ctx.step_wait(t + 1)  # never issued
        assert np.array_equal(torch.stack([fx, fy, fz], 1).cpu().numpy(), F_ref)
        assert np.array_equal(torch.stack([x, y, z], 1).cpu().numpy(), X_ref)
    assert len(got) == len(ref)
    for k, ((P1, e1, b1), (P2, e2, b2)) in enumerate(zip(ref, got)):
        assert np.array_equal(P1, P2), k
        assert np.array_equal(b1, b2), k
        if energy:
            assert np.array_equal(e1, e2), k
