"""The half-shell pair kernel (Newton's third law on the FP32 fast path):
parity with the oracle, agreement with the full shell, bitwise
reproducibility, the batch, and the full-shell fallback when a block's
neighbourhood outgrows the partial buffer.  The half shell is taken only on
request (RBSOG_FLAG_HALF_SHELL)."""
import numpy as np
import pytest

from paper_2602_23582_amd import workloads as W
from test_gpu_parity import TOL_FP32C, _dev, check, gpu_step, oracle_step

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


def _shell_pair(torch, rb, d, P, seed, step, energy, form=0, system_id=0):
    """The same evaluation with the half shell and with the full shell."""
    out = {}
    for name, flag in (("half", rb.FLAG_HALF_SHELL), ("full", rb.FLAG_FULL_SHELL)):
        with rb.Context(d["q"], d["L"], d["rc"], P=P, seed=seed, system_id=system_id, flags=form | flag) as ctx:
            g = gpu_step(torch, ctx, d["pos"], step, d["L"], energy=energy)
            g["npairs"] = ctx.step_info()["npairs"]
        out[name] = g
    return out["half"], out["full"]


def _agree(h, f, what):
    fr = np.sqrt(((h["F"] - f["F"]) ** 2).sum() / (f["F"] ** 2).sum())
    pr = np.linalg.norm(h["P"] - f["P"]) / np.linalg.norm(f["P"])
    print(f"{what}: half vs full shell F {fr:.2e} P {pr:.2e}, pairs {h['npairs']} / {f['npairs']}", flush=True)
    # the full shell tests a pair from both atoms with FP32 block-relative
    # coordinates of two different block origins; a pair within rounding of
    # rc can fall on different sides of it (counted 1/2), the half shell tests
    # it once
    assert abs(h["npairs"] - f["npairs"]) <= 2 + 1e-6 * f["npairs"]
    assert fr < 2e-6 and pr < 1e-6, (fr, pr)
    assert np.array_equal(h["Pr"], f["Pr"]) and np.array_equal(h["Pnr"], f["Pnr"])


@pytest.mark.parametrize("energy", [False, True])
@pytest.mark.parametrize("form", [0, 1])
def test_half_shell_water(torch, rb, orc, form, energy):
    """Bulk water (6 cells per edge, rc 10): half shell against the oracle and
    against the full shell on the same modes."""
    d = W.water_box()
    h, f = _shell_pair(torch, rb, d, 100, 2, 1, energy, form=form)
    o = oracle_step(orc, d, d["L"], d["pos"], 100, 2, 0, 1)
    check(h, o, TOL_FP32C, f"half-shell water form {form} energy {energy}")
    _agree(h, f, f"water form {form} energy {energy}")


@pytest.mark.parametrize("energy", [False, True])
def test_half_shell_small_slab(torch, rb, orc, energy):
    """Slab with dipole layers and vacuum (5 x 5 x 12 cells, rc 12): segments
    of several cells, blocks thin in z near the layers, empty columns."""
    d = W.slab(Lx=60.0, n_water=8000, layer_grid=15, seed=6)
    h, f = _shell_pair(torch, rb, d, 100, 31, 4, energy)
    o = oracle_step(orc, d, d["L"], d["pos"], 100, 31, 0, 4)
    check(h, o, TOL_FP32C, f"half-shell slab energy {energy}")
    _agree(h, f, f"slab energy {energy}")


@pytest.mark.parametrize("n", [9000, 20000])
def test_half_shell_fewest_cells(torch, rb, orc, n):
    """Ionic systems at 0.1 A^-3: 9,000 atoms give 4 cells per edge (the fewest
    the fast path takes: each forward column and its reverse are distinct,
    and the own column's window wraps the periodic seam), 20,000 give 5."""
    d = W.ionic_system(n, seed=n)
    h, f = _shell_pair(torch, rb, d, d["P"], n, 1, False, system_id=3)
    o = oracle_step(orc, d, d["L"], d["pos"], d["P"], n, 3, 1)
    check(h, o, TOL_FP32C, f"half-shell ionic n={n}")
    _agree(h, f, f"ionic n={n}")


def test_half_shell_bitwise_reproducible(torch, rb):
    """Reactions meet in per-wavefront FP64 LDS sums and a fixed-order gather:
    two runs give the same bits."""
    d = W.water_box(n_mol=5000, seed=8)
    out = []
    for _ in range(2):
        with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=4, flags=rb.FLAG_HALF_SHELL) as ctx:
            g = gpu_step(torch, ctx, d["pos"], 6, d["L"])
            g2 = gpu_step(torch, ctx, d["pos"], 6, d["L"], energy=False)
        out.append((g, g2))
    for k in range(2):
        assert np.array_equal(out[0][k]["F"], out[1][k]["F"])
        assert np.array_equal(out[0][k]["P"], out[1][k]["P"])
    assert out[0][0]["U"] == out[1][0]["U"]


def test_half_shell_overflow_runs_the_full_shell(torch, rb, orc):
    """At 0.5 atoms/A^3 (above the 0.15 the partial buffer is sized for) the
    blocks' neighbourhoods outgrow the buffer: the step runs the full-shell
    fast path, bit for bit what the full-shell flag gives, and matches the
    oracle."""
    d = W.ionic_system(34000, seed=77, density=0.5, P=50)
    assert d["L"][0] >= 4 * d["rc"]
    h, f = _shell_pair(torch, rb, d, 50, 77, 2, True, system_id=5)
    assert np.array_equal(h["F"], f["F"]) and np.array_equal(h["P"], f["P"]) and h["U"] == f["U"]
    o = oracle_step(orc, d, d["L"], d["pos"], 50, 77, 5, 2)
    check(h, o, TOL_FP32C, "dense half-shell request on the full shell")


def test_half_shell_in_a_batch_equals_alone(torch, rb):
    """A half-shell system gives the same bits alone and in a batch beside a
    full-shell fast-path system and an exact-path one."""
    specs = []
    d1 = W.water_box(n_mol=5000, seed=3)
    specs.append(dict(q=d1["q"], pos=d1["pos"], box=d1["L"], rc=d1["rc"], P=100, seed=3, system_id=0,
                      flags=rb.FLAG_HALF_SHELL))
    d2 = W.ionic_system(12000, seed=12)
    specs.append(dict(q=d2["q"], pos=d2["pos"], box=d2["L"], rc=d2["rc"], P=50, seed=12, system_id=1, flags=0))
    d3 = W.ionic_system(2000, seed=20)
    specs.append(dict(q=d3["q"], pos=d3["pos"], box=d3["L"], rc=d3["rc"], P=200, seed=20, system_id=2, flags=0))
    steps = np.array([3, 4, 5], dtype=np.int64)
    boxes = np.stack([s["box"] for s in specs])
    xs = [torch.tensor(np.concatenate([s["pos"][:, k] for s in specs]), dtype=torch.float64, device="cuda")
          for k in range(3)]
    fs = [torch.empty_like(xs[0]) for _ in range(3)]
    with rb.Batch(specs) as b:
        P, U, _ = b.step(steps, boxes, *xs, *fs)
        off = b.offsets
    F = torch.stack(fs, 1).cpu().numpy()
    for s, spec in enumerate(specs):
        with rb.Context(spec["q"], spec["box"], spec["rc"], P=spec["P"], seed=spec["seed"],
                        system_id=spec["system_id"], flags=spec["flags"]) as ctx:
            g = gpu_step(torch, ctx, spec["pos"], int(steps[s]), spec["box"])
        assert np.array_equal(g["F"], F[off[s]:off[s + 1]]), s
        assert np.array_equal(g["P"], P[s]), s
        assert g["U"] == U[s, 0] + U[s, 1] - U[s, 2], s
