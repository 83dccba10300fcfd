"""General (triclinic) cells through the C ABI (rbsog_sample_modes_cell):
modes bit-exact and forces, energies and the full pressure tensor (shear
components included) against the oracle's general-cell functions, in FP64 and
FP32C; a diagonal cell against the box call; the refusals."""
import numpy as np
import pytest

from test_gpu_parity import TOL_ATOM_FP32C, TOL_ATOM_FP64, TOL_FP32C, TOL_FP64, _dev, force_errors

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


# columns are the cell vectors
CELLS = {
    "sheared": np.array([[21.0, 4.0, 2.0], [0.0, 20.0, -3.5], [0.0, 0.0, 22.0]]),
    "skewed": np.array([[24.0, -6.0, 5.0], [0.0, 22.0, 4.0], [1.5, 0.0, 23.0]]),
    "thin": np.array([[13.0, 3.0, 0.0], [0.0, 14.0, 2.0], [0.0, 0.0, 15.0]]),  # fewer than 3 cells per edge
    # four or more cells per edge: FP32C takes the relative-coordinate filter and evaluation
    "wide": np.array([[30.0, 5.0, 3.0], [0.0, 28.0, -4.0], [2.0, 0.0, 32.0]]),
}


def _system(h, seed, density=0.1):
    rng = np.random.default_rng(seed)
    n = 2 * int(0.5 * density * abs(np.linalg.det(h)))
    s = rng.uniform(0.0, 1.0, (n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return q, s @ h.T


def _widths(h):
    return 1.0 / np.linalg.norm(np.linalg.inv(h), axis=1)


def _gpu_step(torch, rb, q, pos, h, rc, P, seed, step, precision, energy=True):
    with rb.Context(q, np.diag(h).copy(), rc, P=P, seed=seed, system_id=2, precision=precision) as ctx:
        m_r, m_nr, S = ctx.sample_modes_cell(step, h, return_modes=True)
        x, y, z = (_dev(torch, pos[:, k]) for k in range(3))
        f = [torch.empty_like(x) for _ in range(3)]
        e, v = ctx.force_virial(x, y, z, *f, energy=energy)
        P_, parts = ctx.pressure()
        g = [torch.empty_like(x) for _ in range(3)]
        ctx.debug_long_range_force(*g)
        return dict(m_r=m_r, m_nr=m_nr, Sr=S[0], Snr=S[1], F=torch.stack(f, 1).cpu().numpy(),
                    FF=torch.stack(g, 1).cpu().numpy(), P=P_, PN=parts[0], Pr=parts[1], Pnr=parts[2],
                    U=(e[0] + e[1] - e[2]) if energy else None, UN=e[0] if energy else None,
                    UF=e[1] if energy else None)


def _oracle(orc, q, pos, h, rc, P, seed, step):
    p = orc.sog(rc, row=2, M=10)
    return orc.tri_rbsog_step(q, pos, h, p, P, seed, 2, step)


def _check(g, o, tol, atol, what):
    assert np.array_equal(g["m_r"], o["m_r"]), f"{what}: r-chain modes"
    assert np.array_equal(g["m_nr"], o["m_nr"]), f"{what}: nr-chain modes"
    assert abs(g["Sr"] / o["Sr"] - 1) < 1e-13 and abs(g["Snr"] / o["Snr"] - 1) < 1e-13, what
    fr, fa = force_errors(g["F"], o["F"])
    lr, la = force_errors(g["FF"], o["FF"])
    pn = np.linalg.norm(o["P"])
    pr = np.linalg.norm(g["P"] - o["P"]) / pn
    shear = np.abs(g["P"] - o["P"])[[0, 0, 1], [1, 2, 2]].max() / pn
    print(f"{what}: F {fr:.2e} (atom {fa:.2e}) FF {lr:.2e} P {pr:.2e} shear {shear:.2e}"
          f" |P_shear|/|P| {np.abs(o['P'][[0, 0, 1], [1, 2, 2]]).max() / pn:.2e}", flush=True)
    assert fr <= tol and fa <= atol, what
    assert lr <= tol and la <= atol, what
    assert pr <= tol, what
    for k in ("PN", "Pr", "Pnr"):
        assert np.linalg.norm(g[k] - o[k]) / pn <= tol, (what, k)
    if g["U"] is not None:
        assert abs(g["U"] - o["U"]) <= tol * abs(o["U"]), what


@pytest.mark.parametrize("cell", ["sheared", "skewed", "thin", "wide"])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_cell_matches_oracle(torch, rb, orc, cell, precision):
    h = CELLS[cell]
    rc = 6.0
    assert 2 * rc <= _widths(h).min()
    q, pos = _system(h, seed=len(cell))
    prec, tol, atol = ((rb.PREC_FP64, TOL_FP64, TOL_ATOM_FP64) if precision == "fp64"
                       else (rb.PREC_FP32C, TOL_FP32C, TOL_ATOM_FP32C))
    g = _gpu_step(torch, rb, q, pos, h, rc, 100, 7, 3, prec)
    o = _oracle(orc, q, pos, h, rc, 100, 7, 3)
    _check(g, o, tol, atol, f"{cell} {precision} n={len(q)}")


def test_cell_several_steps_and_samplers(torch, rb, orc):
    """The exchange, printed, shared and independent samplers on a sheared
    cell, several steps: modes bit-exact against the oracle's chains."""
    h = CELLS["skewed"]
    rc = 6.0
    q, pos = _system(h, seed=5)
    p = orc.sog(rc, row=2, M=10)
    for variant in (0, 1, 2, 3):
        with rb.Context(q, np.diag(h).copy(), rc, P=50, seed=11, system_id=4, precision=rb.PREC_FP64,
                        recalibration=variant) as ctx:
            for step in (0, 1, 17):
                m_r, m_nr, _ = ctx.sample_modes_cell(step, h, return_modes=True)
                o_r, o_nr, _ = orc.tri_sample_modes(h, p, 50, 11, 4, step, variant)
                assert np.array_equal(m_r, o_r) and np.array_equal(m_nr, o_nr), (variant, step)


def test_diagonal_cell_is_the_box(torch, rb):
    """A diagonal cell tensor takes the box path: bitwise the results of
    rbsog_sample_modes with its diagonal."""
    from paper_2602_23582_amd import workloads as W
    d = W.ionic_system(3000, seed=4)
    h = np.diag(d["L"])
    out = []
    for use_cell in (False, True):
        with rb.Context(d["q"], d["L"], d["rc"], P=50, seed=1) as ctx:
            if use_cell:
                ctx.sample_modes_cell(2, h)
            else:
                ctx.sample_modes(2, d["L"])
            x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
            f = [torch.empty_like(x) for _ in range(3)]
            ctx.force_virial(x, y, z, *f)
            out.append((torch.stack(f, 1).cpu().numpy(), ctx.pressure()[0]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_cell_refusals(torch, rb):
    h = CELLS["thin"]
    q, pos = _system(h, seed=2)
    with rb.Context(q, np.diag(h).copy(), 6.0, P=50, seed=1) as ctx:
        # r_c above half the smallest perpendicular width
        wide = h.copy()
        wide[0, 1] = 11.0
        assert 2 * 6.0 > _widths(wide).min()
        with pytest.raises(rb.RBSOGError) as e:
            ctx.sample_modes_cell(0, wide)
        assert e.value.code == -3
        flipped = h.copy()
        flipped[:, 0] *= -1.0
        with pytest.raises(rb.RBSOGError):
            ctx.sample_modes_cell(0, flipped)  # det h < 0
        ctx.sample_modes_cell(0, h)
        x, y, z = (_dev(torch, pos[:, k]) for k in range(3))
        with pytest.raises(rb.RBSOGError) as e:
            ctx.rescale(np.array([1.01, 1.0, 1.0]), x, y, z)
        assert e.value.code == -6
