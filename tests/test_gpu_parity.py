"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer outputs (sampled modes, cell ids) must match bit for bit.  Floating
point results are compared on the same sampled modes: FP64 path within 1e-12,
FP32C path within 1e-5 (force relative RMS, Frobenius relative pressure error,
relative energy), the gate stated for the method.
"""
import numpy as np
import pytest

from paper_2602_23582_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12
TOL_FP32C = 1e-5
# Per-atom force error, max_i |dF_i| / rms|F|: an atom's force is a sum of
# about 700 pair terms each rounded to FP32 (relative 6e-8), and a pair force
# can be ten times the rms net force, so sqrt(700) * 6e-8 * 10 = 1.6e-5 is the
# scale of the largest rounding error; the gate allows 6x that.
TOL_ATOM_FP32C = 1e-4
TOL_ATOM_FP64 = 1e-10
# Structure factors in FP32C: the hardware sine/cosine (input in revolutions)
# carry an absolute error of at most 1.25e-7 per term (measured over 2^24
# arguments), the phase's rounding to FP32 up to 2^-25 revolutions, and the
# terms are summed in FP64; with random signs |d rho| grows like that times
# sqrt(sum q^2).
RHO_TOL = 1e-6


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


def gpu_step(torch, ctx, pos, step, box, energy=True, lr=True):
    """One step; energy=False is the force + pressure call the benchmark times
    (the FP32 fast path then takes pair displacements from block-relative
    coordinates).  lr: also fetch the long-range force F^{F*} alone."""
    x, y, z = (_dev(torch, pos[:, k]) for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    m_r, m_nr, S = ctx.sample_modes(step, box, return_modes=True)
    e, v = ctx.force_virial(x, y, z, fx, fy, fz, energy=energy)
    P, parts = ctx.pressure()
    F = torch.stack([fx, fy, fz], 1).cpu().numpy()
    out = dict(F=F, P=P, PN=parts[0], Pr=parts[1], Pnr=parts[2], m_r=m_r, m_nr=m_nr, Sr=S[0], Snr=S[1], U=None)
    if lr:
        gx, gy, gz = (torch.empty_like(x) for _ in range(3))
        ctx.debug_long_range_force(gx, gy, gz)
        out["FF"] = torch.stack([gx, gy, gz], 1).cpu().numpy()
    if energy:
        out.update(UN=e[0], UF=e[1], Uself=e[2], U=e[0] + e[1] - e[2], vir=v)
    return out


def oracle_step(orc, d, box, pos, P, seed, sys, step, variant=1, sample=None):
    p = orc.sog(d["rc"], row=2, M=10)
    return orc.rbsog_step(d["q"], pos, box, p, P, seed, sys, step, sample=sample, variant=variant)


def force_errors(F, Fo):
    """Relative RMS error and the largest per-atom error over the rms force."""
    d = F - Fo
    rms = np.sqrt((Fo ** 2).sum(1).mean())
    return np.sqrt((d ** 2).sum() / (Fo ** 2).sum()), np.sqrt((d ** 2).sum(1)).max() / rms


def check(g, o, tol, what=""):
    assert np.array_equal(g["m_r"], o["m_r"]), f"{what}: r-chain modes differ"
    assert np.array_equal(g["m_nr"], o["m_nr"]), f"{what}: nr-chain modes differ"
    assert abs(g["Sr"] / o["Sr"] - 1) < 1e-13 and abs(g["Snr"] / o["Snr"] - 1) < 1e-13
    fr, fa = force_errors(g["F"], o["F"])
    atol = TOL_ATOM_FP64 if tol <= TOL_FP64 else TOL_ATOM_FP32C
    pn = np.linalg.norm(o["P"])
    pr = np.linalg.norm(g["P"] - o["P"]) / pn
    parts = {k: np.linalg.norm(g[k] - o[k]) / pn for k in ("PN", "Pr", "Pnr")}
    lr = ""
    if "FF" in g and "FF" in o:
        # the long-range force on its own: on water it is under a tenth of the
        # total, so the total's gate alone would let a large error in it pass
        lr_r, lr_a = force_errors(g["FF"], o["FF"])
        lr = f" FF {lr_r:.2e} (atom {lr_a:.2e})"
        assert lr_r <= tol and lr_a <= atol, f"{what}: long-range force{lr}"
    assert fa <= atol, f"{what}: per-atom force error {fa:.2e}"
    if g["U"] is None:  # forces and pressure only
        msg = f"{what}: F {fr:.2e} (atom {fa:.2e}){lr} P {pr:.2e} parts {parts}"
        print(msg, flush=True)
        assert fr <= tol and pr <= tol and all(v <= tol for v in parts.values()), msg
        return
    ur = abs(g["U"] - o["U"]) / abs(o["U"])
    un = abs(g["UN"] - o["UN"]) / abs(o["U"])
    uf = abs(g["UF"] - o["UF"]) / abs(o["U"])
    us = abs(g["Uself"] - o["Uself"]) / abs(o["Uself"])
    msg = f"{what}: F {fr:.2e} (atom {fa:.2e}){lr} P {pr:.2e} parts {parts} U {ur:.2e} UN {un:.2e} UF {uf:.2e} Us {us:.2e}"
    print(msg, flush=True)
    assert fr <= tol and pr <= tol and ur <= tol and un <= tol and uf <= tol and us <= tol, msg
    assert all(v <= tol for v in parts.values()), msg


# --------------------------------------------------------------------------
# bit-exact integer work
# --------------------------------------------------------------------------

@pytest.mark.parametrize("box,rc,P", [((30.0, 30.0, 30.0), 10.0, 100), ((200.0, 200.0, 500.0), 12.0, 400),
                                      ((17.1, 17.1, 17.1), 8.55, 50), ((66.88, 66.88, 66.88), 10.0, 1024),
                                      ((41.0, 23.0, 60.0), 11.0, 200)])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_modes_bit_exact(torch, rb, orc, box, rc, P, variant):
    q = np.array([1.0, -1.0, 0.5, -0.5])
    box = np.array(box)
    p = orc.sog(rc, row=2, M=10)
    if variant == 3 and P > 512:
        # the independent chain's proposals need P more mode slots
        with pytest.raises(rb.RBSOGError) as ei:
            rb.Context(q, box, rc, P=P, recalibration=variant)
        assert ei.value.code == -1
        return
    for seed, sys in ((1, 0), (12345, 7), (2**40 + 3, 99)):
        with rb.Context(q, box, rc, P=P, seed=seed, system_id=sys, recalibration=variant) as ctx:
            for step in (0, 1, 17, 4_000_000_000):
                m_r, m_nr, S = ctx.sample_modes(step, box, return_modes=True)
                o_r, o_nr, _ = orc.sample_modes(box, p, P, seed, sys, step, variant)
                assert np.array_equal(m_r, o_r), (seed, sys, step)
                assert np.array_equal(m_nr, o_nr), (seed, sys, step)
                Sr, Snr = orc.norm_consts(box, p)
                assert abs(S[0] / Sr - 1) < 1e-13 and abs(S[1] / Snr - 1) < 1e-13
                modes, counts, _ = ctx.debug_modes(with_rho=False)
                # distinct set: every sampled mode appears once, multiplicities add up to P
                assert len({tuple(m) for m in modes}) == len(modes)
                assert counts[:, 0].sum() == P and counts[:, 1].sum() == P
                lookup = {tuple(m): i for i, m in enumerate(modes)}
                cr = np.zeros(len(modes), int)
                cn = np.zeros(len(modes), int)
                for m in o_r:
                    cr[lookup[tuple(m)]] += 1
                for m in o_nr:
                    cn[lookup[tuple(m)]] += 1
                assert np.array_equal(cr, counts[:, 0]) and np.array_equal(cn, counts[:, 1])


@pytest.mark.parametrize("case", ["lattice", "water", "small"])
def test_cell_binning_bit_exact(torch, rb, orc, case):
    d = {"lattice": lambda: W.c1_lattice(jitter=0.2), "water": lambda: W.water_box(n_mol=3000, seed=4),
         "small": lambda: W.ionic_system(500, seed=3)}[case]()
    # include images far outside the box and points on the cell faces
    pos = d["pos"].copy()
    pos[::7] -= d["L"]
    pos[1::11] += 2 * d["L"]
    pos[2, 0] = 0.0
    pos[3, 1] = d["L"][1]
    with rb.Context(d["q"], d["L"], d["rc"], P=8) as ctx:
        gpu_step(torch, ctx, pos, 0, d["L"])
        cell, nc = ctx.debug_cells()
    ref = orc.cell_ids(pos, d["L"], nc)
    assert np.array_equal(cell, ref)


# --------------------------------------------------------------------------
# floating-point parity on identical modes
# --------------------------------------------------------------------------

def test_fp64_lattice_ten_steps_with_rescale(torch, rb, orc):
    """1,000 charges, FP64 path, 10 steps on L_n = 30 (1 + 0.001 n), r <- mu r."""
    d = W.c1_lattice(jitter=0.2)
    pos0 = d["pos"]
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=5, precision=rb.PREC_FP64) as ctx:
        for step in range(10):
            box = W.rescale_schedule(d["L"], step)
            pos = pos0 * (box / d["L"])
            g = gpu_step(torch, ctx, pos, step, box)
            o = oracle_step(orc, d, box, pos, 100, 5, 0, step)
            check(g, o, TOL_FP64, f"fp64 step {step}")


def test_device_rescale_matches_host_rescale(torch, rb):
    d = W.c1_lattice(jitter=0.2)
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    with rb.Context(d["q"], d["L"], d["rc"], P=10) as ctx:
        mu = np.array([1.001, 1.001, 1.002])
        box = ctx.rescale(mu, x, y, z)
        torch.cuda.synchronize()
    np.testing.assert_array_equal(box, d["L"] * mu)
    np.testing.assert_array_equal(x.cpu().numpy(), d["pos"][:, 0] * mu[0])
    np.testing.assert_array_equal(z.cpu().numpy(), d["pos"][:, 2] * mu[2])


# FP32C evaluates the SOG sums either as polynomials in r^2 (default) or as
# the M exponentials (flag); both are checked against the oracle
FORMS = [0, 1]


@pytest.mark.parametrize("variant", [2, 3])
def test_fp64_lattice_comparison_samplers(torch, rb, orc, variant):
    """The shared-proposal and independent-chain samplers of the non-radial
    modes, FP64 path, two steps."""
    d = W.c1_lattice(jitter=0.2)
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=5, precision=rb.PREC_FP64, recalibration=variant) as ctx:
        for step in (0, 7):
            g = gpu_step(torch, ctx, d["pos"], step, d["L"])
            o = oracle_step(orc, d, d["L"], d["pos"], 100, 5, 0, step, variant=variant)
            check(g, o, TOL_FP64, f"fp64 sampler {variant} step {step}")


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_fp32c_lattice(torch, rb, orc, variant, form):
    d = W.c1_lattice(jitter=0.2)
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=9, recalibration=variant, flags=form) as ctx:
        for step in (0, 3):
            g = gpu_step(torch, ctx, d["pos"], step, d["L"])
            o = oracle_step(orc, d, d["L"], d["pos"], 100, 9, 0, step, variant=variant)
            check(g, o, TOL_FP32C, f"fp32c lattice v{variant} form {form} step {step}")


@pytest.mark.parametrize("M,P,precision", [(4, 100, "fp64"), (25, 100, "fp32c"), (64, 100, "fp32c"),
                                         (64, 1024, "fp64"), (10, 1024, "fp32c")])
def test_term_counts_and_the_largest_batch(torch, rb, orc, M, P, precision):
    """Term counts other than M = 10, up to the largest (64): the kernels
    with M read at run time, or the FP32C polynomial where its fit holds.
    And the largest batch, P = 1024 (1,025 mode slots).  Jittered lattice,
    energy included, Table 1 row 2 with its printed omega at every M."""
    d = W.c1_lattice(jitter=0.2)
    prec = rb.PREC_FP32C if precision == "fp32c" else rb.PREC_FP64
    with rb.Context(d["q"], d["L"], d["rc"], P=P, seed=13, M=M, precision=prec) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 1, d["L"])
    o = orc.rbsog_step(d["q"], d["pos"], d["L"], orc.sog(d["rc"], row=2, M=M), P, 13, 0, 1)
    check(g, o, TOL_FP32C if precision == "fp32c" else TOL_FP64, f"M={M} P={P} {precision}")


@pytest.mark.parametrize("row,M,precision", [(1, 4, "fp32c"), (3, 27, "fp32c"), (3, 27, "fp64"), (4, 64, "fp32c")])
def test_other_table1_rows(torch, rb, orc, row, M, precision):
    """The other parameter sets of Table 1 (b, sigma scaled to rc, omega as
    printed) at their pressure term counts M~ (row 4 asks 69; the largest
    allowed, 64, is used): jittered lattice, energy included."""
    b, s9, om = orc.TABLE1[row][:3]
    d = W.c1_lattice(jitter=0.2)
    prec = rb.PREC_FP32C if precision == "fp32c" else rb.PREC_FP64
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=14, M=M, b=b, sigma=s9 * d["rc"] / orc.TABLE1_RC, omega=om,
                    precision=prec) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 2, d["L"])
    o = orc.rbsog_step(d["q"], d["pos"], d["L"], orc.sog(d["rc"], row=row, M=M), 100, 14, 0, 2)
    check(g, o, TOL_FP32C if precision == "fp32c" else TOL_FP64, f"Table 1 row {row} M={M} {precision}")


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_coulomb_prefactor_scales_every_result(torch, rb, orc, precision):
    """With the prefactor k (here 332.0637, kcal/mol A per e^2) every force,
    pressure part and energy term is k times the oracle's (which works in
    units of k = 1); the sampled modes do not depend on it."""
    k = 332.0637
    d = W.c1_lattice(jitter=0.2)
    prec = rb.PREC_FP32C if precision == "fp32c" else rb.PREC_FP64
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=15, coulomb_k=k, precision=prec) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 3, d["L"])
    o = oracle_step(orc, d, d["L"], d["pos"], 100, 15, 0, 3)
    for key in ("F", "FF", "P", "PN", "Pr", "Pnr"):
        o[key] = k * o[key]
    for key in ("UN", "UF", "Uself", "U"):
        o[key] = k * o[key]
    check(g, o, TOL_FP32C if precision == "fp32c" else TOL_FP64, f"coulomb_k {precision}")


@pytest.mark.parametrize("M", [7, 10])
def test_omega_solved_at_the_given_term_count(torch, rb, orc, M):
    """omega <= 0 asks the library for the C0 root of the 1/r^3 split at rc
    and the given M (eq. continuity); the oracle solves the same equation
    with its own code, and the FP64 results agree to 1e-12."""
    d = W.c1_lattice(jitter=0.2)
    p2 = orc.sog(d["rc"], row=2, M=M)
    om = orc.omega_c0(p2.b, p2.sigma, d["rc"], M)
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=16, M=M, omega=0.0, precision=rb.PREC_FP64) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 1, d["L"])
    o = orc.rbsog_step(d["q"], d["pos"], d["L"], orc.sog(d["rc"], row=2, M=M, omega=om), 100, 16, 0, 1)
    check(g, o, TOL_FP64, f"omega solved, M={M}")


@pytest.mark.parametrize("energy", [True, False])
@pytest.mark.parametrize("form", FORMS)
def test_fp32c_water_30k(torch, rb, orc, form, energy):
    """10,000 three-site molecules at 1 g/cm^3 (L = 66.9 A), rc 10, P 100."""
    d = W.water_box()
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=2, flags=form) as ctx:
        for step in range(3):
            box = W.rescale_schedule(d["L"], step)
            pos = d["pos"] * (box / d["L"])
            g = gpu_step(torch, ctx, pos, step, box, energy=energy)
            o = oracle_step(orc, d, box, pos, 100, 2, 0, step)
            check(g, o, TOL_FP32C, f"water form {form} energy {energy} step {step}")


def test_fp32c_water_100_steps_with_rescale(torch, rb, orc):
    """The bulk-water workload for 100 steps under L_n = L_0 (1 + 0.001 n),
    positions rescaled on the device each step (the grid grows from 6 to 7
    cells per edge on the way); steps 0, 57 and 99 against the oracle."""
    d = W.water_box()
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    fx, fy, fz = (torch.empty_like(x) for _ in range(3))
    grids = set()
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=4) as ctx:
        for step in range(100):
            if step:
                mu = (1.0 + 0.001 * step) / (1.0 + 0.001 * (step - 1))
                ctx.rescale([mu, mu, mu], x, y, z)
            box = ctx.box.copy()
            ctx.sample_modes(step, box)
            ctx.force_virial(x, y, z, fx, fy, fz, energy=False)
            P, parts = ctx.pressure()
            grids.add(int(ctx.debug_cells()[1][0]))
            if step in (0, 57, 99):
                pos = torch.stack([x, y, z], 1).cpu().numpy()
                o = oracle_step(orc, d, box, pos, 100, 4, 0, step)
                F = torch.stack([fx, fy, fz], 1).cpu().numpy()
                fr = np.sqrt(((F - o["F"]) ** 2).sum() / (o["F"] ** 2).sum())
                pr = np.linalg.norm(P - o["P"]) / np.linalg.norm(o["P"])
                print(f"water step {step} box {box[0]:.3f}: F {fr:.2e} P {pr:.2e}", flush=True)
                assert fr < TOL_FP32C and pr < TOL_FP32C, (step, fr, pr)
    assert grids == {6, 7}, grids


@pytest.mark.parametrize("energy", [True, False])
@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("P", [100, 400])
def test_fp32c_small_slab(torch, rb, orc, P, form, energy):
    """Anisotropic slab (60 x 60 x 150 A) with dipole layers, rc 12."""
    d = W.slab(Lx=60.0, n_water=8000, layer_grid=15, seed=6)
    with rb.Context(d["q"], d["L"], d["rc"], P=P, seed=31, flags=form) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 4, d["L"], energy=energy)
    o = oracle_step(orc, d, d["L"], d["pos"], P, 31, 0, 4)
    check(g, o, TOL_FP32C, f"slab P={P} form {form} energy {energy}")


@pytest.mark.parametrize("energy", [True, False])
@pytest.mark.parametrize("n", [500, 2000, 2600, 6000, 9000])
def test_fp32c_small_boxes_collapsed_cells(torch, rb, orc, n, energy):
    """Served-stream systems.  Fewer than three cells of rc per edge make the
    whole box one cell: 500 atoms (L = 17.1 A, rc = L/2), 2,000 and 2,600
    (L < 3 rc; 2,600 keys are ordered by three workgroups of 1,024).  6,000
    gives 3 cells per edge; 9,000 gives 4, the fewest the FP32
    relative-coordinate filter takes."""
    d = W.ionic_system(n, seed=n)
    with rb.Context(d["q"], d["L"], d["rc"], P=d["P"], seed=n, system_id=3) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 1, d["L"], energy=energy)
    o = oracle_step(orc, d, d["L"], d["pos"], d["P"], n, 3, 1)
    check(g, o, TOL_FP32C, f"ionic n={n} energy {energy}")


@pytest.mark.parametrize("box", [(45.0, 45.0, 25.0), (25.0, 45.0, 60.0), (33.0, 61.0, 47.0)])
def test_fp32c_anisotropic_exact_path(torch, rb, orc, box):
    """Orthorhombic boxes on the exact path: (45, 45, 25) has 4 x 4 x 1 cells
    (nine columns, each whole in z and cut to the block's z-window);
    (25, 45, 60) has 1 x 4 x 6 (three columns, runs of cells); (33, 61, 47)
    has 3 x 6 x 4.  The 16-bit filter's units differ per axis in all three."""
    rng = np.random.default_rng(int(sum(box)))
    L = np.array(box)
    n = 2 * int(0.05 * np.prod(L))
    pos = rng.uniform(0, 1, (n, 3)) * L
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    d = dict(q=q, pos=pos, L=L, rc=10.0)
    with rb.Context(q, L, 10.0, P=100, seed=8, system_id=2) as ctx:
        for energy in (True, False):
            g = gpu_step(torch, ctx, pos, 3, L, energy=energy)
            o = oracle_step(orc, d, L, pos, 100, 8, 2, 3)
            check(g, o, TOL_FP32C, f"anisotropic {box} energy {energy}")


@pytest.mark.parametrize("n,precision", [(9000, "fp32c"), (9000, "fp64"), (30000, "fp32c")])
def test_dense_cells_ordered_in_passes(torch, rb, orc, n, precision):
    """Charges at 1 per cubic angstrom, rc 10.  9,000 (L = 20.8 A): one cell
    of 9,000 atoms, its keys ranked by nine workgroups over LDS tiles of all
    9,000.  30,000 (L = 31.1 A): 27 cells of about 1,110 atoms, each ranked by
    one workgroup in two passes."""
    d = W.ionic_system(n, seed=n, density=1.0, P=50)
    assert d["L"][0] < (3 if n == 9000 else 4) * d["rc"]
    prec = rb.PREC_FP32C if precision == "fp32c" else rb.PREC_FP64
    with rb.Context(d["q"], d["L"], d["rc"], P=50, seed=n, system_id=1, precision=prec) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 2, d["L"])
    o = oracle_step(orc, d, d["L"], d["pos"], 50, n, 1, 2)
    check(g, o, TOL_FP32C if precision == "fp32c" else TOL_FP64, f"dense cells n={n} {precision}")


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_degenerate_systems(torch, rb, orc, precision):
    """The smallest inputs the method takes.  An ion pair 3 A apart in a 25 A
    cube (one collapsed cell, one pair block with 62 idle lanes) at P = 1: one
    mode per chain.  A lattice with every charge zero: neutral, so accepted,
    and every force, pressure part and energy term is exactly zero on both
    sides."""
    prec = rb.PREC_FP32C if precision == "fp32c" else rb.PREC_FP64
    tol = TOL_FP32C if precision == "fp32c" else TOL_FP64
    L = np.full(3, 25.0)
    d = dict(q=np.array([1.0, -1.0]), pos=np.array([[11.0, 12.0, 12.5], [13.0, 14.0, 13.5]]), L=L, rc=10.0)
    with rb.Context(d["q"], L, 10.0, P=1, seed=17, precision=prec) as ctx:
        for step in (0, 1):
            g = gpu_step(torch, ctx, d["pos"], step, L)
            o = oracle_step(orc, d, L, d["pos"], 1, 17, 0, step)
            assert len(g["m_r"]) == 1 and len(g["m_nr"]) == 1
            check(g, o, tol, f"ion pair {precision} step {step}")
    z = W.c1_lattice(jitter=0.2)
    z["q"] = np.zeros_like(z["q"])
    with rb.Context(z["q"], z["L"], z["rc"], P=50, seed=5, precision=prec) as ctx:
        g = gpu_step(torch, ctx, z["pos"], 2, z["L"])
    o = oracle_step(orc, z, z["L"], z["pos"], 50, 5, 0, 2)
    assert np.array_equal(g["m_r"], o["m_r"]) and np.array_equal(g["m_nr"], o["m_nr"])
    for k in ("F", "P", "PN", "Pr", "Pnr", "UN", "UF", "Uself"):
        assert not np.any(np.asarray(g[k])), (k, g[k])
        assert not np.any(np.asarray(o[k])), (k, o[k])


def test_rho_of_distinct_modes(torch, rb, orc):
    d = W.water_box(n_mol=4000, seed=12)
    with rb.Context(d["q"], d["L"], d["rc"], P=200, seed=3) as ctx:
        gpu_step(torch, ctx, d["pos"], 0, d["L"])
        modes, counts, rho = ctx.debug_modes()
    ref = orc.rho(d["q"], d["pos"], d["L"], modes)
    scale = np.sqrt(np.sum(d["q"] ** 2))
    err = np.abs(rho - ref).max() / scale
    print("rho max err / sqrt(sum q^2):", err)
    assert err < RHO_TOL


def test_host_arrays_match_device_arrays(torch, rb):
    d = W.c1_lattice(jitter=0.2)
    with rb.Context(d["q"], d["L"], d["rc"], P=50, seed=1) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 2, d["L"])
        x, y, z = (np.ascontiguousarray(d["pos"][:, k]) for k in range(3))
        fx, fy, fz = (np.zeros(len(x)) for _ in range(3))
        ctx.sample_modes(2, d["L"])
        e, v = ctx.force_virial(x, y, z, fx, fy, fz)
        P, _ = ctx.pressure()
    np.testing.assert_array_equal(np.stack([fx, fy, fz], 1), g["F"])
    np.testing.assert_array_equal(P, g["P"])


def test_bitwise_reproducible(torch, rb):
    d = W.water_box(n_mol=5000, seed=8)
    out = []
    for _ in range(2):
        with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=4) as ctx:
            out.append(gpu_step(torch, ctx, d["pos"], 6, d["L"]))
    assert np.array_equal(out[0]["F"], out[1]["F"])
    assert np.array_equal(out[0]["P"], out[1]["P"])
    assert out[0]["U"] == out[1]["U"]


def test_timing_levels(torch, rb):
    """rbsog_set_timing: level 1 times every kernel group, level 2 the pair
    kernel alone; timing never changes a result."""
    d = W.water_box(n_mol=3000, seed=3)
    out = []
    for level in (0, 1, 2):
        with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=4) as ctx:
            if level:
                ctx.set_timing(level)
            out.append(gpu_step(torch, ctx, d["pos"], 2, d["L"]))
            if level:
                t = ctx.get_timing()
                if level == 1:
                    assert {"sampler", "bin", "pair", "sk", "reduce", "force"} <= set(t), t
                else:
                    assert set(t) == {"pair"}, t
                assert t["pair"][1] == 1 and t["pair"][0] > 0
    for o in out[1:]:
        assert np.array_equal(o["F"], out[0]["F"]) and np.array_equal(o["P"], out[0]["P"])


GROWTH = [1.0, 1.15, 1.30, 1.0, 1.45, 1.15]  # 6, 7, 8, 6, 9, 7 cells per edge at rc 10


def test_grid_growth_reuploads_cell_arrays(torch, rb):
    """A box that grows past a cell boundary re-carves the cell arrays; every
    step must equal a fresh context built at that box (bit for bit)."""
    d = W.water_box(n_mol=8000, seed=21)
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=9) as ctx:
        for k, g in enumerate(GROWTH):
            box = d["L"] * g
            pos = d["pos"] * g
            print(f"growth {g}: box {box[0]:.2f}", flush=True)
            a = gpu_step(torch, ctx, pos, k, box)
            with rb.Context(d["q"], box, d["rc"], P=100, seed=9) as fresh:
                b = gpu_step(torch, fresh, pos, k, box)
            assert np.array_equal(a["F"], b["F"]), f"growth {g}: forces differ from a fresh context"
            assert np.array_equal(a["P"], b["P"]), f"growth {g}: pressure differs from a fresh context"


def test_state_errors(torch, rb):
    d = W.c1_lattice()
    x, y, z = (_dev(torch, d["pos"][:, k]) for k in range(3))
    f = [torch.empty_like(x) for _ in range(3)]
    with rb.Context(d["q"], d["L"], d["rc"], P=10) as ctx:
        with pytest.raises(rb.RBSOGError) as e:
            ctx.force_virial(x, y, z, *f)
        assert e.value.code == -6
        with pytest.raises(rb.RBSOGError) as e:
            ctx.pressure()
        assert e.value.code == -6
        with pytest.raises(rb.RBSOGError) as e:
            ctx.sample_modes(0, np.array([30.0, 30.0, 15.0]))
        assert e.value.code == -3
        with pytest.raises(rb.RBSOGError) as e:
            ctx.sample_modes(-1, d["L"])
        assert e.value.code == -1


# --------------------------------------------------------------------------
# full-size slab (1,000,000 atoms): sampled forces, all rho, full pressure
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def slab_1m():
    return W.slab()


@pytest.mark.parametrize("P", [100, 400])
def test_full_size_slab_sampled(torch, rb, orc, slab_1m, P):
    d = slab_1m
    rng = np.random.default_rng(0)
    smp = np.sort(rng.choice(len(d["q"]), 400, replace=False))
    smp = np.concatenate([smp, np.arange(990000, 990040)])  # layer atoms
    with rb.Context(d["q"], d["L"], d["rc"], P=P, seed=11) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 0, d["L"], energy=False)  # the benchmark's call
        modes, counts, rho = ctx.debug_modes()
        ge = gpu_step(torch, ctx, d["pos"], 0, d["L"])
    p = orc.sog(d["rc"], row=2, M=10)
    m_r, m_nr, _ = orc.sample_modes(d["L"], p, P, 11, 0, 0)
    assert np.array_equal(g["m_r"], m_r) and np.array_equal(g["m_nr"], m_nr)
    ref = orc.rho(d["q"], d["pos"], d["L"], modes)
    err = np.abs(rho - ref).max() / np.sqrt(np.sum(d["q"] ** 2))
    print("1M slab rho max err / sqrt(sum q^2):", err)
    assert err < RHO_TOL
    o = orc.rbsog_step(d["q"], d["pos"], d["L"], p, P, 11, 0, 0, modes=(m_r, m_nr), sample=smp)
    Fo = o["F"]
    Fg = g["F"][smp]
    fr, fa = force_errors(Fg, Fo)
    lr, la = force_errors(g["FF"][smp], o["FF"])
    print(f"1M slab sampled force rel RMS {fr:.2e} (atom {fa:.2e}), long-range {lr:.2e} (atom {la:.2e})")
    assert fr < TOL_FP32C and fa < TOL_ATOM_FP32C
    assert lr < TOL_FP32C and la < TOL_ATOM_FP32C
    # long-range parts are global: compare against the oracle's estimators
    pn = np.linalg.norm(g["P"])
    assert np.linalg.norm(g["Pr"] - o["Pr"]) / pn < TOL_FP32C
    assert np.linalg.norm(g["Pnr"] - o["Pnr"]) / pn < TOL_FP32C
    assert abs(ge["UF"] - o["UF"]) / abs(o["UF"]) < TOL_FP32C
    fre = np.sqrt(((ge["F"][smp] - Fo) ** 2).sum() / (Fo ** 2).sum())
    print("1M slab sampled force rel RMS with the energy sum", fre)
    assert fre < TOL_FP32C


@pytest.mark.slow
def test_full_size_electrolyte_sampled(torch, rb, orc):
    """The 10^7-atom electrolyte (467.5 A cube, rc 10, P 100) in the call the
    benchmark times: modes bit-exact, rho of every distinct mode, forces of
    sampled atoms and the long-range estimators against the oracle."""
    d = W.electrolyte()
    rng = np.random.default_rng(3)
    smp = np.sort(rng.choice(len(d["q"]), 300, replace=False))
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=13) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 0, d["L"], energy=False)
        modes, counts, rho = ctx.debug_modes()
    p = orc.sog(d["rc"], row=2, M=10)
    m_r, m_nr, _ = orc.sample_modes(d["L"], p, 100, 13, 0, 0)
    assert np.array_equal(g["m_r"], m_r) and np.array_equal(g["m_nr"], m_nr)
    ref = orc.rho(d["q"], d["pos"], d["L"], modes)
    err = np.abs(rho - ref).max() / np.sqrt(np.sum(d["q"] ** 2))
    print("10M electrolyte rho max err / sqrt(sum q^2):", err)
    assert err < RHO_TOL
    o = orc.rbsog_step(d["q"], d["pos"], d["L"], p, 100, 13, 0, 0, modes=(m_r, m_nr), sample=smp)
    fr, fa = force_errors(g["F"][smp], o["F"])
    lr, la = force_errors(g["FF"][smp], o["FF"])
    print(f"10M electrolyte sampled force rel RMS {fr:.2e} (atom {fa:.2e}), long-range {lr:.2e} (atom {la:.2e})")
    assert fr < TOL_FP32C and fa < TOL_ATOM_FP32C
    assert lr < TOL_FP32C and la < TOL_ATOM_FP32C
    pn = np.linalg.norm(g["P"])
    assert np.linalg.norm(g["Pr"] - o["Pr"]) / pn < TOL_FP32C
    assert np.linalg.norm(g["Pnr"] - o["Pnr"]) / pn < TOL_FP32C


@pytest.mark.slow
def test_full_size_slab_pressure(torch, rb, orc, slab_1m):
    """Short-range virial and energy of all 1,000,000 atoms against the oracle."""
    d = slab_1m
    with rb.Context(d["q"], d["L"], d["rc"], P=100, seed=11) as ctx:
        g = gpu_step(torch, ctx, d["pos"], 0, d["L"])
        gf = gpu_step(torch, ctx, d["pos"], 0, d["L"], energy=False)
    o = oracle_step(orc, d, d["L"], d["pos"], 100, 11, 0, 0)
    check(g, o, TOL_FP32C, "1M slab full")
    check(gf, o, TOL_FP32C, "1M slab full, no energy")
