"""rbsog_force_virial_noalloc (the entry point that allocates nothing):
through the C ABI, its forces, energies, virial and pressure against those of
rbsog_force_virial on the same context, step and positions, on two calls in
a row with the second on a smaller system (the scratch is shared); and the
clear errors for a system beyond the scratch and for host arrays."""
import ctypes as C

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
    L = rbsog.load()
    f = L.rbsog_force_virial_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p] * 7 + [C.POINTER(C.c_double)] * 2
    return rbsog


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _run(torch, rb, ctx, pos, step, box, noalloc):
    x, y, z = (_dev(torch, pos[:, k]) for k in range(3))
    f = [torch.full_like(x, np.nan) for _ in range(3)]
    ctx.sample_modes(step, box)
    e = np.zeros(3)
    v = np.zeros(6)
    if noalloc:
        rc = rb.load().rbsog_force_virial_noalloc(ctx._h, *(C.c_void_p(t.data_ptr()) for t in (x, y, z, *f)),
                                                   rb._pd(e), rb._pd(v))
        ctx._check(rc, "rbsog_force_virial_noalloc")
    else:
        e, v = ctx.force_virial(x, y, z, *f)
    P, parts = ctx.pressure()
    return torch.stack(f, 1).cpu().numpy(), e, v, P


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_force_virial_on_two_calls(torch, rb, order):
    systems = [(W.water_box(n_mol=10_000, seed=2), 100, 0),          # 30,000 atoms, fast path
               (W.ionic_system(3000, seed=4), 50, rb.FLAG_FULL_SHELL)]  # smaller, exact path
    ctxs = [rb.Context(d["q"], d["L"], d["rc"], P=P, seed=9, flags=fl) for d, P, fl in systems]
    try:
        ref = []
        for c, (d, P, fl) in zip(ctxs, systems):
            ref.append(_run(torch, rb, c, d["pos"], 3, d["L"], noalloc=False))
        for rep in range(2):  # the same two calls twice: the scratch keeps the last call's contents
            for c, (d, P, fl), r in zip(ctxs, systems, ref):
                got = _run(torch, rb, c, d["pos"], 3, d["L"], noalloc=True)
                assert np.array_equal(got[0], r[0])
                assert np.array_equal(got[1], r[1]) and np.array_equal(got[2], r[2])
                assert np.array_equal(got[3], r[3])
        # the regular call on the same context afterwards is unchanged
        again = _run(torch, rb, ctxs[0], systems[0][0]["pos"], 3, systems[0][0]["L"], noalloc=False)
        assert np.array_equal(again[0], ref[0][0]) and np.array_equal(again[3], ref[0][3])
    finally:
        for c in ctxs:
            c.close()


def test_noalloc_refuses_host_arrays_and_oversized_systems(torch, rb):
    d = W.ionic_system(3000, seed=4)
    with rb.Context(d["q"], d["L"], d["rc"], P=50, seed=1) as c:
        c.sample_modes(0, d["L"])
        h = [np.zeros(len(d["q"])) for _ in range(6)]
        rc = rb.load().rbsog_force_virial_noalloc(c._h, *(C.c_void_p(a.ctypes.data) for a in h), None, None)
        assert rc == -1
    # 3,000,000 atoms at P = 1024: structure-factor partials of 2,930 blocks x
    # 1,026 mode slots x 16 B = 48 MB, beyond the 32 MiB scratch
    n = 3_000_000
    rng = np.random.default_rng(0)
    L = np.full(3, (n / 0.1) ** (1 / 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    pos = rng.uniform(0, 1, (n, 3)) * L
    with rb.Context(q, L, 10.0, P=1024, seed=1, flags=rb.FLAG_FULL_SHELL) as c:
        c.sample_modes(0, L)
        x, y, z = (_dev(torch, pos[:, k]) for k in range(3))
        f = [torch.empty_like(x) for _ in range(3)]
        rc = rb.load().rbsog_force_virial_noalloc(c._h, *(C.c_void_p(t.data_ptr()) for t in (x, y, z, *f)),
                                                  None, None)
        assert rc == -1
        assert b"scratch" in rb.load().rbsog_last_error(c._h)
