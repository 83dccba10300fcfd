"""Pins of the oracle's general-cell (triclinic) functions, h = [h_1, h_2, h_3]
with r = h s and k = 2 pi h^-T m (Sec. 2.1, eq. FourierTransform), each
against something other than its own formula:
- at h = diag(L) every function against the orthorhombic oracle (closed-form
  erf proposal, per-axis sums, minimum image);
- invariance under h -> h U for unimodular U (the same lattice, so the same
  physics);
- the direct lattice sums against the Poisson forms of Prop. 1;
- the proposal pmf of eq. proposal against its normalisation and against
  rounded draws;
- the rock-salt Madelung constant in a primitive (rhombohedral) fcc cell;
- the start bound against enumerated ratios, the start draws and the
  estimators against enumerated expectations, batch means against Theorem 1;
- finite-difference shear strains against the off-diagonal pressure."""
import numpy as np
import pytest

from paper_2602_23582_amd import workloads as W

SHEARED = [
    np.array([[9.0, 2.0, 1.0], [0.0, 8.5, -1.5], [0.0, 0.0, 10.0]]),
    np.array([[11.0, -3.0, 0.5], [0.0, 10.0, 2.5], [0.0, 0.0, 9.0]]),
]


def _golden_madelung():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "nacl_madelung.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return float(rows[0][0])


def _ionic_in_cell(h, n=64, seed=3):
    """n alternating unit charges at seeded uniform fractional positions of cell h."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.0, 1.0, (n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return q, s @ h.T


def _widths(h):
    hi = np.linalg.inv(h)
    return 1.0 / np.linalg.norm(hi, axis=1)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _vir(v):
    xx, yy, zz, xy, xz, yz = v
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def test_tri_reduces_to_orthorhombic(orc):
    """At h = diag(L) the general-cell functions give the orthorhombic ones:
    the lattice sums, the quadrature proposal pmf against the erf product,
    the rounded proposal, the chains (from the orthorhombic start states),
    structure factors, estimators, short-range and full k-space sums, Ewald."""
    L = np.array([16.0, 13.0, 19.0])
    h = np.diag(L)
    p = orc.sog(6.0, row=2, M=10)
    for l in range(p.M):
        for form, name in ((1, "direct"), (2, "poisson")):
            a = orc.tri_H(h, p.wt[l], p.s[l], form)
            b = orc.H(L, p.wt[l], p.s[l], name)
            assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0]) and abs(a[1] - b[1]) <= 1e-13 * abs(b[1]), (l, name)
    sr, snr = orc.norm_consts(L, p)
    tr, tnr = orc.tri_norm_consts(h, p)
    assert abs(tr / sr - 1) < 1e-13 and abs(tnr / snr - 1) < 1e-13
    rng = np.random.default_rng(1)
    for m in rng.integers(-6, 7, (40, 3)).astype(np.int32):
        for s0 in (p.s[0], p.s[0] / np.sqrt(2)):
            a, b = orc.proposal_pmf(m, L, s0), orc.tri_proposal_pmf(m, h, s0)
            assert abs(b / a - 1) < 1e-12, (m, a, b)
        if np.any(m != 0):
            assert abs(orc.tri_target_r(m, h, p) / orc.target_r(m, L, p) - 1) < 1e-14
            assert abs(orc.tri_ratio_nr(m, h, p) / orc.ratio_nr(m, L, p) - 1) < 1e-14
    for t in range(200):
        z = orc.draw_proposal(3, 1, 2, t)[0]
        sig = L / (np.sqrt(2) * np.pi * p.s[0])
        m = np.where(sig * z >= 0, np.floor(sig * z + 0.5), -np.floor(-sig * z + 0.5))
        assert np.array_equal(orc.tri_round(z, h, p.s[0]), m.astype(np.int32))
    for step in range(6):
        a, b = orc.start_states(L, p, 5, 1, step)
        for v in range(4):
            t = orc.tri_chains(h, p, 60, 5, 1, step, v, a, b)
            o = orc.sample_modes(L, p, 60, 5, 1, step, v)
            assert np.array_equal(t[0], o[0]) and np.array_equal(t[1], o[1]) and np.array_equal(t[2], o[2])
    q, pos = _ionic_in_cell(h, n=80, seed=4)
    m_r, m_nr, _ = orc.sample_modes(L, p, 40, 2, 0, 3)
    assert _rel(orc.tri_rho(q, pos, h, m_r), orc.rho(q, pos, L, m_r)) < 1e-13
    Ft, Prt, Pnrt, Ut = orc.tri_long_range_rb(q, pos, h, m_r, m_nr, sr, snr)
    Fo, Pro, Pnro, Uo = orc.long_range_rb(q, pos, L, m_r, m_nr, sr, snr)
    assert _rel(Ft, Fo) < 1e-12 and _rel(Prt, Pro) < 1e-12 and _rel(Pnrt, Pnro) < 1e-12 and abs(Ut / Uo - 1) < 1e-12
    Ft, vt, ut = orc.tri_short_range(q, pos, h, p)
    Fo, vo, uo = orc.short_range(q, pos, L, p, method="brute")
    assert _rel(Ft, Fo) < 1e-12 and _rel(vt, vo) < 1e-12 and abs(ut / uo - 1) < 1e-12
    Ft, Pt, ut = orc.tri_sog_kspace_full(q, pos, h, p)
    Fo, Po, uo = orc.sog_kspace_full(q, pos, L, p)
    assert _rel(Ft, Fo) < 1e-12 and _rel(Pt, Po) < 1e-12 and abs(ut / uo - 1) < 1e-12
    beta = 6.5 / (0.9 * L.min())
    Ft, Pt, ut = orc.tri_ewald(q, pos, h, beta, 6.5 / beta, 2 * beta * 6.7)
    Fo, Po, uo = orc.ewald(q, pos, L)
    assert _rel(Ft, Fo) < 1e-12 and _rel(Pt, Po) < 1e-12 and abs(ut / uo - 1) < 1e-12


@pytest.mark.parametrize("U", [np.array([[1, 1, 0], [0, 1, 0], [0, 0, 1]]),
                               np.array([[1, 0, 1], [1, 1, 1], [0, 1, 1]])])
def test_tri_unimodular_invariance(orc, U):
    """h and h U (det U = 1, integer) describe the same periodic lattice, so the
    lattice sums S^r, S^nr, the full k-space SOG energy, forces and pressure,
    the short-range sums over every image and Ewald are unchanged."""
    assert round(abs(np.linalg.det(U))) == 1
    h0 = SHEARED[0]
    h1 = h0 @ U
    p = orc.sog(4.0, row=2, M=10)
    assert 2 * p.rc <= _widths(h0).min()
    q, pos = _ionic_in_cell(h0, n=48, seed=9)
    a, b = orc.tri_norm_consts(h0, p, form=1), orc.tri_norm_consts(h1, p, form=1)
    assert abs(a[0] / b[0] - 1) < 1e-12 and abs(a[1] / b[1] - 1) < 1e-12
    F0, P0, u0 = orc.tri_sog_kspace_full(q, pos, h0, p)
    F1, P1, u1 = orc.tri_sog_kspace_full(q, pos, h1, p)
    assert _rel(F1, F0) < 1e-11 and _rel(P1, P0) < 1e-11 and abs(u1 / u0 - 1) < 1e-12
    F0, v0, u0 = orc.tri_short_range(q, pos, h0, p)
    F1, v1, u1 = orc.tri_short_range(q, pos, h1, p)
    assert _rel(F1, F0) < 1e-12 and _rel(v1, v0) < 1e-12 and abs(u1 / u0 - 1) < 1e-12
    beta = 0.6
    E0 = orc.tri_ewald(q, pos, h0, beta, 6.5 / beta, 2 * beta * 6.7)
    E1 = orc.tri_ewald(q, pos, h1, beta, 6.5 / beta, 2 * beta * 6.7)
    assert _rel(E1[0], E0[0]) < 1e-11 and _rel(E1[1], E0[1]) < 1e-11 and abs(E1[2] / E0[2] - 1) < 1e-12


@pytest.mark.parametrize("h", SHEARED)
def test_tri_direct_sums_equal_poisson_forms(orc, h):
    """Prop. 1 on a sheared cell: H^r_l and H^nr_l by the reciprocal-lattice sums
    of eqs. Sr, Snr equal the real-space forms of eqs. H2, H2r."""
    p = orc.sog(4.0, row=2, M=10)
    w = _widths(h).min()
    used = 0
    for l in range(p.M):
        if p.s[l] > 0.8 * w or p.s[l] < 0.05 * w:
            continue  # Poisson cancels for s >~ the cell; the direct sum needs too many terms for s << it
        a = orc.tri_H(h, p.wt[l], p.s[l], 1)
        b = orc.tri_H(h, p.wt[l], p.s[l], 2)
        assert abs(a[0] / b[0] - 1) < 1e-11 and abs(a[1] / b[1] - 1) < 1e-11, l
        used += 1
    assert used >= 2


def _enumerate(h, p, pad=2):
    kmax = np.sqrt(4 * 60.0) / p.s[0]
    mmax = [int(np.ceil(np.linalg.norm(h[:, j]) * kmax / (2 * np.pi))) + 1 + pad for j in range(3)]
    g = [np.arange(-mmax[k], mmax[k] + 1) for k in range(3)]
    return np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.int32)


@pytest.mark.parametrize("h", SHEARED)
def test_tri_proposal_pmf_normalised_and_matches_draws(orc, h):
    """Eq. proposal on a sheared cell: the quadrature pmf sums to one over the
    lattice, and 40,000 draws of round(h^T u) from the generator's normals
    follow it (chi^2 over the cells expected to hold at least 20 draws)."""
    p = orc.sog(4.0, row=2, M=10)
    s0 = p.s[0]
    hi = np.linalg.inv(h)
    sig_max = np.linalg.norm(h, axis=0).max() / (np.sqrt(2) * np.pi * s0)
    r = int(np.ceil(12 * sig_max)) + 1
    g = np.arange(-r, r + 1)
    ms = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.int32)
    pmf = np.array([orc.tri_proposal_pmf(m, h, s0) for m in ms])
    assert abs(pmf.sum() - 1.0) < 1e-11
    draws = np.array([orc.tri_round(orc.draw_proposal(11, 2, 7, t)[0], h, s0) for t in range(40000)])
    keys = {tuple(m): i for i, m in enumerate(ms)}
    cnt = np.zeros(len(ms))
    for m in draws:
        cnt[keys[tuple(m)]] += 1
    exp = pmf * len(draws)
    keep = exp > 20
    chi2 = np.sum((cnt[keep] - exp[keep]) ** 2 / exp[keep])
    dof = keep.sum() - 1
    assert (chi2 - dof) / np.sqrt(2 * dof) < 5, (chi2, dof)
    assert hi is not None


def _nacl_primitive(n, d=3.0):
    """Rock salt in n^3 primitive fcc cells: h = n [a1 a2 a3], a1 = (a/2)(0,1,1),
    a2 = (a/2)(1,0,1), a3 = (a/2)(1,1,0) with a = 2 d; Na at the lattice
    points, Cl at fractional (1/2, 1/2, 1/2) of each primitive cell."""
    a = 2.0 * d
    prim = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]]).T
    h = n * prim
    pos, q = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                base = prim @ np.array([i, j, k], dtype=float)
                pos.append(base)
                q.append(1.0)
                pos.append(base + prim @ np.array([0.5, 0.5, 0.5]))
                q.append(-1.0)
    return np.array(q), np.array(pos), h


def test_tri_rock_salt_madelung_in_primitive_fcc_cell(orc):
    """Rock salt in a supercell of the primitive rhombohedral fcc cell (angles
    of 60 degrees): the Ewald energy is -(N/2) M / d with the Madelung constant
    M of the rock-salt structure, the forces vanish and the pressure is
    isotropic, U / (3V).  The SOG total (Table 1 row 2, r_c = 4 A) of the
    same crystal in the primitive cell equals, per ion, the orthorhombic
    oracle's SOG total in the cubic 10^3-site cell, and so does its pressure:
    both cells tile the same infinite crystal."""
    d = 3.0
    q, pos, h = _nacl_primitive(3, d)
    V = abs(np.linalg.det(h))
    M = _golden_madelung()
    beta = 0.55
    F, P, U = orc.tri_ewald(q, pos, h, beta, 6.5 / beta, 2 * beta * 6.7)
    assert abs(U / (-0.5 * len(q) * M / d) - 1) < 1e-10
    assert np.abs(F).max() < 1e-10
    np.testing.assert_allclose(P, np.eye(3) * U / (3 * V), rtol=0, atol=1e-13)
    p = orc.sog(4.0, row=2, M=10)
    assert 2 * p.rc <= _widths(h).min()
    FN, vir, UN = orc.tri_short_range(q, pos, h, p)
    FF, PF, UF = orc.tri_sog_kspace_full(q, pos, h, p)
    Us = UN + UF - orc.self_energy(p, q)
    Ps = _vir(vir) / V + PF
    c = W.c1_lattice(jitter=0.0)  # the same crystal (d = 3 A) in its cubic cell
    assert np.isclose(c["L"][0] / 10, d)
    r = orc.sog_deterministic(c["q"], c["pos"], c["L"], p)
    assert abs((Us / len(q)) / (r["U"] / len(c["q"])) - 1) < 1e-11
    assert _rel(Ps, r["P"]) < 1e-10
    assert np.abs(FN + FF).max() < 1e-10


@pytest.mark.parametrize("h", SHEARED)
def test_tri_start_bound_exceeds_every_lattice_ratio(orc, h):
    """The rejection constant of the start draws on a sheared cell lies above
    g_p(m)/q'(m) at every lattice point (the widened proposal, width
    s_0/sqrt2), and within a modest factor of the largest ratio."""
    p = orc.sog(4.0, row=2, M=10)
    ms = _enumerate(h, p)
    ms = ms[np.any(ms != 0, axis=1)]
    sp = p.s[0] / np.sqrt(2)
    for power in (2, 4):
        B = orc.tri_start_bound(h, p, power)
        best = 0.0
        for m in ms:
            g = orc.tri_target_r(m, h, p)
            if power == 4:
                g *= orc.tri_ratio_nr(m, h, p)
            best = max(best, g / orc.tri_proposal_pmf(m, h, sp))
        assert best < B < 50 * best, (power, best, B)


def test_tri_start_states_are_exact_draws_of_their_targets(orc):
    """The start draws on a sheared cell follow P^r and P^nr (chi^2 over
    4,000 steps against the enumerated targets)."""
    h = SHEARED[0]
    p = orc.sog(4.0, row=2, M=10)
    ms = _enumerate(h, p)
    ms = ms[np.any(ms != 0, axis=1)]
    gr = np.array([orc.tri_target_r(m, h, p) for m in ms])
    gn = gr * np.array([orc.tri_ratio_nr(m, h, p) for m in ms])
    keys = {tuple(m): i for i, m in enumerate(ms)}
    cr = np.zeros(len(ms)); cn = np.zeros(len(ms))
    R = 4000
    for step in range(R):
        a, b = orc.tri_start_states(h, p, 17, 4, step)
        cr[keys[tuple(a)]] += 1
        cn[keys[tuple(b)]] += 1
    for c, g in ((cr, gr), (cn, gn)):
        exp = g / g.sum() * R
        keep = exp > 15
        chi2 = np.sum((c[keep] - exp[keep]) ** 2 / exp[keep])
        dof = keep.sum() - 1
        assert (chi2 - dof) / np.sqrt(2 * dof) < 5, (chi2, dof)
        assert c[~keep].sum() <= 3 * max(exp[~keep].sum(), 1.0) + 10


def test_tri_estimators_are_exactly_unbiased(orc):
    """On a sheared cell, the expectations over P^r and P^nr of the
    single-sample estimators (eqs. P_approx_r, P_approx_nr, f_approx and the
    energy) equal the full k-space sums of Theorem 1 and App. A."""
    h = SHEARED[1]
    p = orc.sog(4.0, row=2, M=10)
    q, pos = _ionic_in_cell(h, n=24, seed=21)
    Sr, Snr = orc.tri_norm_consts(h, p)
    ms = _enumerate(h, p, pad=0)
    ms = ms[np.any(ms != 0, axis=1)]
    gr = np.array([orc.tri_target_r(m, h, p) for m in ms])
    prob_r = np.pi ** 1.5 * gr / Sr
    assert abs(prob_r.sum() - 1.0) < 1e-12
    gn = gr * np.array([orc.tri_ratio_nr(m, h, p) for m in ms])
    prob_nr = gn / gn.sum()
    EF = np.zeros((len(q), 3)); EPr = np.zeros((3, 3)); EPnr = np.zeros((3, 3)); EU = 0.0
    for m, a, b in zip(ms, prob_r, prob_nr):
        F, Pr, _, U = orc.tri_long_range_rb(q, pos, h, m[None], m[None], Sr, Snr)
        _, _, Pnr, _ = orc.tri_long_range_rb(q, pos, h, m[None], m[None], Sr, Snr, forces=False)
        EF += a * F; EPr += a * Pr; EU += a * U; EPnr += b * Pnr
    FF, PF, UF = orc.tri_sog_kspace_full(q, pos, h, p)
    assert _rel(EF, FF) < 1e-10
    assert _rel(EPr + EPnr, PF) < 1e-10
    assert abs(EU / UF - 1) < 1e-10


def test_tri_batch_mean_is_unbiased(orc):
    """Batch means of P^{F,r*} + P^{F,nr*} (exchange recalibration, exact
    starts) over independent steps on a sheared cell converge to the full
    k-space P^F of Theorem 1."""
    h = SHEARED[0]
    p = orc.sog(4.0, row=2, M=10)
    q, pos = _ionic_in_cell(h, n=48, seed=5)
    Sr, Snr = orc.tri_norm_consts(h, p)
    _, PF, _ = orc.tri_sog_kspace_full(q, pos, h, p, forces=False)
    R = 6000
    acc = np.empty((R, 9))
    for step in range(R):
        m_r, m_nr, _ = orc.tri_sample_modes(h, p, 20, 1234, 7, step, orc.RECAL_EXCHANGE)
        _, Pr, Pnr, _ = orc.tri_long_range_rb(q, pos, h, m_r, m_nr, Sr, Snr, forces=False)
        acc[step] = (Pr + Pnr).ravel()
    mean, sem = acc.mean(0), acc.std(0, ddof=1) / np.sqrt(R)
    z = (mean - PF.ravel()) / np.maximum(sem, 1e-300)
    assert np.all(np.abs(z) < 4.5), z


def test_tri_pressure_is_the_strain_derivative(orc):
    """The deterministic SOG total on a sheared cell: P_ab = -(1/V) dU/d eps_ab
    for the strain r -> (I + eps E_ab) r, h -> (I + eps E_ab) h, including the
    off-diagonal (shear) components, and F = -dU/dr."""
    h = SHEARED[1]
    p = orc.sog(4.0, row=2, M=10)
    q, pos = _ionic_in_cell(h, n=32, seed=8)
    V = abs(np.linalg.det(h))

    def total(pos_, h_):
        FN, vir, UN = orc.tri_short_range(q, pos_, h_, p)
        FF, PF, UF = orc.tri_sog_kspace_full(q, pos_, h_, p)
        return UN + UF, FN + FF, _vir(vir) / V + PF

    U0, F0, P0 = total(pos, h)
    eps = 1e-5
    for a, b in ((0, 0), (2, 2), (0, 1), (1, 2), (2, 0)):
        E = np.zeros((3, 3)); E[a, b] = 1.0
        up = [total(pos @ (np.eye(3) + s * eps * E).T, (np.eye(3) + s * eps * E) @ h)[0] for s in (1, -1)]
        dU = (up[0] - up[1]) / (2 * eps)
        assert abs(-dU / V - P0[a, b]) < 2e-7 * np.abs(P0).max(), (a, b, -dU / V, P0[a, b])
    for i in (0, 7):
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, k] += 1e-5
            pm[i, k] -= 1e-5
            fd = -(total(pp, h)[0] - total(pm, h)[0]) / 2e-5
            assert abs(fd - F0[i, k]) < 2e-7 * np.abs(F0).max()
