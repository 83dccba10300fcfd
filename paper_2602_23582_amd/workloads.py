"""Seeded synthetic inputs shaped like the paper's workloads.

The paper measures on SPC/E water, LiTFSI electrolytes and a DPPC membrane
(Sec. 4); none of those structures ship with it.  These generators stand in
for them with the same kinds of shapes: charge-neutral point-charge systems on
jittered lattices, rigid three-site water-like molecules at liquid density, an
anisotropic slab with charged dipole layers, a 1 M ion/water mixture and a
stream of independent small systems.

This module holds no part of the method's arithmetic (no SOG weights, no
sampling, no forces): it only places charges in boxes.  Both the oracle-based
tests and the HIP path read their inputs from here.

Every generator returns a dict with
    q    (n,)  float64 charges in units of e, summing to zero,
    pos  (n,3) float64 positions in Angstrom, wrapped into [0, L),
    L    (3,)  float64 orthorhombic box edges,
    rc   float cutoff, P int batch size (the configuration's defaults).
"""
from __future__ import annotations

import numpy as np

Q_O = -0.8476
Q_H = 0.4238
R_OH = 1.0
ANGLE_HOH = np.deg2rad(109.47)
WATER_MASS_AMU = 18.01528
AVOGADRO_PER_ANG3_GCM3 = 0.602214076  # molecules/A^3 per (g/cm^3 / amu)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _wrap(pos, L):
    return np.mod(pos, L)


def _random_rotations(rng, n):
    """Uniform random rotation matrices from unit quaternions of four normals."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_frame():
    h = 0.5 * ANGLE_HOH
    return np.array([[0.0, 0.0, 0.0],
                     [R_OH * np.sin(h), 0.0, R_OH * np.cos(h)],
                     [-R_OH * np.sin(h), 0.0, R_OH * np.cos(h)]])


def _place_waters(rng, centres, L, fixed_pos=None, min_dist=1.5, max_iter=60):
    """Three-site molecules with random orientations around the given O sites;
    a molecule is re-oriented while any of its atoms is closer than min_dist to
    an atom of another molecule (or to a fixed atom)."""
    nm = centres.shape[0]
    frame = _water_frame()
    R = _random_rotations(rng, nm)
    body = np.einsum("mij,aj->mai", R, frame)
    if min_dist is None or min_dist <= 0:
        return _wrap(centres[:, None, :] + body, L).reshape(-1, 3)
    from scipy.spatial import cKDTree
    nfix = 0 if fixed_pos is None else fixed_pos.shape[0]
    owner = np.concatenate([np.arange(3 * nm) // 3, -1 - np.arange(nfix)])
    movers = None
    for _ in range(max_iter):
        pos = _wrap(centres[:, None, :] + body, L).reshape(-1, 3)
        allpos = pos if nfix == 0 else np.concatenate([pos, fixed_pos])
        allpos = np.minimum(allpos, np.nextafter(L, 0))
        tree = cKDTree(allpos, boxsize=L)
        if movers is None:
            pairs = tree.query_pairs(min_dist, output_type="ndarray")
            oi, oj = owner[pairs[:, 0]], owner[pairs[:, 1]]
            bad = oi != oj
            cand = np.unique(np.concatenate([oi[bad], oj[bad]]))
        else:
            atoms = (3 * movers[:, None] + np.arange(3)).ravel()
            hits = tree.query_ball_point(allpos[atoms], min_dist)
            cand = []
            for a, hl in zip(atoms, hits):
                for h in hl:
                    if owner[h] != owner[a]:
                        cand.append(owner[a])
                        if owner[h] >= 0:
                            cand.append(owner[h])
            cand = np.unique(np.array(cand, dtype=np.int64))
        movers = cand[cand >= 0]
        if movers.size == 0:
            return pos
        Rn = _random_rotations(rng, movers.size)
        body[movers] = np.einsum("mij,aj->mai", Rn, frame)
    return _wrap(centres[:, None, :] + body, L).reshape(-1, 3)


def _sc_lattice(nside, spacing, offset):
    g = np.arange(nside) * spacing + offset
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1), np.stack(
        np.meshgrid(np.arange(nside), np.arange(nside), np.arange(nside), indexing="ij"), axis=-1
    ).reshape(-1, 3)


def c1_lattice(seed: int = 1, jitter: float = 0.2, nside: int = 10, spacing: float = 3.0):
    """1,000 point charges, +-1e alternating on a 10^3 simple-cubic lattice
    (spacing 3 A, origin 1.5 A) in a 30 A cube, each coordinate jittered by
    U(-jitter, +jitter) * spacing.  jitter = 0 gives the rock-salt lattice."""
    rng = _rng(seed)
    pos, idx = _sc_lattice(nside, spacing, 0.5 * spacing)
    q = np.where(idx.sum(axis=1) % 2 == 0, 1.0, -1.0)
    pos = pos + rng.uniform(-jitter * spacing, jitter * spacing, pos.shape)
    L = np.full(3, nside * spacing)
    return dict(name="lattice-1k", q=q, pos=_wrap(pos, L), L=L, rc=10.0, P=100)


def water_box(n_mol: int = 10_000, seed: int = 2, density_gcm3: float = 1.0, jitter: float = 0.1,
              rc: float = 10.0, P: int = 100, min_dist: float = 1.5):
    """Rigid three-site water-like molecules (O -0.8476e, H +0.4238e, O-H 1 A,
    H-O-H 109.47 deg) with random orientations, centres on a jittered cubic
    lattice (first n_mol sites of a seeded permutation), cubic box at the given
    mass density.  10,000 molecules at 1 g/cm^3 give L = 66.89 A."""
    rng = _rng(seed)
    L1 = (n_mol * WATER_MASS_AMU / (AVOGADRO_PER_ANG3_GCM3 * density_gcm3)) ** (1.0 / 3.0)
    nside = int(np.ceil(n_mol ** (1.0 / 3.0)))
    a = L1 / nside
    sites, _ = _sc_lattice(nside, a, 0.5 * a)
    sites = sites[rng.permutation(sites.shape[0])[:n_mol]]
    sites = sites + rng.uniform(-jitter * a, jitter * a, sites.shape)
    L = np.full(3, L1)
    pos = _place_waters(rng, sites, L, min_dist=min_dist)
    q = np.tile([Q_O, Q_H, Q_H], n_mol)
    return dict(name=f"water-{3 * n_mol}", q=q, pos=pos, L=L, rc=rc, P=P)


def slab(Lx: float = 200.0, Lz_factor: float = 2.5, n_water: int = 330_000, layer_grid: int = 50,
         layer_spacing: float = 4.0, layer_offset: float = 20.0, pair_sep: float = 0.5,
         pair_charge: float = 0.7, water_density: float = 0.0334, seed: int = 3, jitter: float = 0.1,
         rc: float = 12.0, P: int = 100, min_dist: float = 1.5):
    """Anisotropic slab: box Lx x Lx x 2.5 Lx.  Two layers of +-0.7e dipole
    pairs (0.5 A apart along z, 50x50 grid of 4 A) at z_c +- 20 A, the upper
    layer +z-oriented and the lower -z-oriented, inside a neutral background of
    water-like molecules on a jittered lattice at 0.0334 molecules/A^3 filling a
    band around z_c (lattice planes within 2 A of a layer are left empty),
    vacuum elsewhere.  Defaults: 1,000,000 atoms in 200 x 200 x 500 A."""
    rng = _rng(seed)
    Lz = Lz_factor * Lx
    L = np.array([Lx, Lx, Lz])
    zc = 0.5 * Lz
    g = (np.arange(layer_grid) + 0.5) * layer_spacing
    GX, GY = np.meshgrid(g, g, indexing="ij")
    gx, gy = GX.ravel(), GY.ravel()
    layer_pos, layer_q = [], []
    for zl, sign in ((zc + layer_offset, 1.0), (zc - layer_offset, -1.0)):
        lo = np.stack([gx, gy, np.full_like(gx, zl - 0.5 * pair_sep)], axis=1)
        hi = np.stack([gx, gy, np.full_like(gx, zl + 0.5 * pair_sep)], axis=1)
        layer_pos += [lo, hi]
        layer_q += [np.full(gx.size, -sign * pair_charge), np.full(gx.size, sign * pair_charge)]
    layer_pos = _wrap(np.concatenate(layer_pos), L)
    layer_q = np.concatenate(layer_q)
    nxy = int(round(Lx * water_density ** (1.0 / 3.0)))
    axy = Lx / nxy
    az = 1.0 / (water_density * axy * axy)
    gxy = (np.arange(nxy) + 0.5) * axy
    PX, PY = np.meshgrid(gxy, gxy, indexing="ij")
    plane = np.stack([PX.ravel(), PY.ravel()], axis=1)
    planes = []
    k = 0
    while sum(p.shape[0] for p in planes) < n_water:
        for zp in (zc + (k + 0.5) * az, zc - (k + 0.5) * az):
            if min(abs(zp - zc - layer_offset), abs(zp - zc + layer_offset)) < 2.0:
                continue
            planes.append(np.column_stack([plane, np.full(plane.shape[0], zp)]))
        k += 1
    sites = np.concatenate(planes)
    # keep complete inner planes, pick the remainder of the outermost planes at random
    full = sites[: n_water - (n_water % plane.shape[0])] if n_water % plane.shape[0] else sites[:n_water]
    if full.shape[0] < n_water:
        rest = sites[full.shape[0]:]
        rest = rest[rng.permutation(rest.shape[0])[: n_water - full.shape[0]]]
        sites = np.concatenate([full, rest])
    else:
        sites = full
    a = np.array([axy, axy, az])
    sites = sites + rng.uniform(-1.0, 1.0, sites.shape) * jitter * a
    wpos = _place_waters(rng, sites, L, fixed_pos=layer_pos, min_dist=min_dist)
    q = np.concatenate([np.tile([Q_O, Q_H, Q_H], n_water), layer_q])
    pos = np.concatenate([wpos, layer_pos])
    return dict(name=f"slab-{q.size}", q=q, pos=pos, L=L, rc=rc, P=P)


def electrolyte(n_atoms: int = 10_000_000, waters_per_pair: float = 55.5, site_density: float = 0.0334,
                seed: int = 4, jitter: float = 0.1, rc: float = 10.0, P: int = 100):
    """1 M monovalent ion pairs in water-like three-site molecules: sites of a
    jittered cubic lattice at 0.0334 sites/A^3 hold either one ion or one
    water; ion sites are chosen by a seeded permutation.  Defaults: 59,348
    pairs + 3,293,768 waters = 10,000,000 atoms in a 467.5 A cube."""
    rng = _rng(seed)
    n_pairs = int(round(n_atoms / (2 + 3 * waters_per_pair)))
    n_wat = (n_atoms - 2 * n_pairs) // 3
    n_pairs = (n_atoms - 3 * n_wat) // 2
    n_sites = 2 * n_pairs + n_wat
    L1 = (n_sites / site_density) ** (1.0 / 3.0)
    nside = int(np.ceil(n_sites ** (1.0 / 3.0)))
    a = L1 / nside
    sites, _ = _sc_lattice(nside, a, 0.5 * a)
    sites = sites[rng.permutation(sites.shape[0])[:n_sites]]
    sites = sites + rng.uniform(-jitter * a, jitter * a, sites.shape)
    L = np.full(3, L1)
    ion = sites[: 2 * n_pairs]
    wat = sites[2 * n_pairs:]
    ion_q = np.where(np.arange(2 * n_pairs) % 2 == 0, 1.0, -1.0)
    wpos = _place_waters(rng, wat, L, min_dist=None)
    q = np.concatenate([ion_q, np.tile([Q_O, Q_H, Q_H], n_wat)])
    pos = np.concatenate([_wrap(ion, L), wpos])
    return dict(name=f"electrolyte-{q.size}", q=q, pos=pos, L=L, rc=rc, P=P)


def ionic_system(n: int, seed: int, density: float = 0.1, jitter: float = 0.1, rc_max: float = 10.0,
                 P: int | None = None):
    """One system of the served stream: n (even) charges +-1e alternating over
    the first n sites of a jittered simple-cubic lattice (ceil(n^(1/3)) per
    side), cubic box at number density 0.1 A^-3, cutoff min(10 A, L/2), batch
    size drawn from {50, 100, 200} by the seed unless given."""
    rng = _rng(seed)
    n = 2 * (n // 2)
    L1 = (n / density) ** (1.0 / 3.0)
    nside = int(np.ceil(n ** (1.0 / 3.0)))
    a = L1 / nside
    sites, _ = _sc_lattice(nside, a, 0.5 * a)
    sites = sites[:n] + rng.uniform(-jitter * a, jitter * a, (n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    L = np.full(3, L1)
    if P is None:
        P = int(rng.choice([50, 100, 200]))
    return dict(name=f"ionic-{n}", q=q, pos=_wrap(sites, L), L=L, rc=min(rc_max, 0.5 * L1), P=P)


def ionic_melt(n: int, seed: int, density: float = 0.1, rc_max: float = 10.0, P: int = 100):
    """n (even) charges +-1e at independent uniform positions in a cubic box
    at number density 0.1 A^-3, cutoff min(10 A, L/2): a disordered ionic
    system without the lattice's Bragg peaks.  (On the jittered lattices of
    ionic_system with an even number of sites per side the alternating
    charges form layers, and |rho(k)|^2 ~ n^2 at the layers' wave vector, far
    in the tail of the radial proposal.)"""
    rng = _rng(seed)
    n = 2 * (n // 2)
    L1 = (n / density) ** (1.0 / 3.0)
    L = np.full(3, L1)
    pos = rng.uniform(0.0, 1.0, (n, 3)) * L
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return dict(name=f"melt-{n}", q=q, pos=_wrap(pos, L), L=L, rc=min(rc_max, 0.5 * L1), P=P)


def served_stream(n_systems: int = 4096, seed: int = 5, n_min: int = 500, n_max: int = 50_000):
    """Sizes, seeds and batch sizes of the served stream: sizes log-uniform in
    [500, 50,000] (rounded down to even), one seed per system."""
    rng = _rng(seed)
    sizes = 2 * (np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_systems)) // 2).astype(np.int64)
    seeds = rng.integers(1, 2**31 - 1, n_systems)
    return sizes, seeds


def rescale_schedule(L0, step: int):
    """Deterministic isotropic box schedule used for multi-step runs:
    L_n = L_0 (1 + 0.001 n)."""
    return np.asarray(L0, dtype=np.float64) * (1.0 + 0.001 * step)


CONFIGS = {
    "lattice-1k": c1_lattice,
    "water-30k": water_box,
    "slab-1m": slab,
    "electrolyte-10m": electrolyte,
}
