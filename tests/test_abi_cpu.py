"""Host-side checks of libnbody.so that need no GPU: the library loads, exports
every entry point include/nbody.h declares, and rejects bad arguments on the
host before any HIP call (every error path below returns before touching the
device)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nb():
    import paper_2511_02655_amd as nb
    if not os.path.exists(nb.LIB_PATH):
        pytest.fail("libnbody.so is not built; run python -m paper_2511_02655_amd.build")
    nb.lib()
    return nb


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "nbody.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(nb):
    syms = declared_symbols()
    assert len(syms) >= 11
    L = ctypes.CDLL(nb.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(nb.EXPORTED)


def test_abi_version(nb):
    assert nb.lib().nbody_abi_version() == nb.NBODY_ABI_VERSION


def test_tile_variants_listed(nb):
    for k in nb.KERNELS:
        for p in nb.PRECISIONS:
            v = nb.tile_variants(k, p)
            assert len(v) >= 2 and all(x.startswith("bs=") for x in v)


def _cfg(nb, **kw):
    c = nb.NBodyConfig()
    c.abi_version = kw.get("abi", nb.NBODY_ABI_VERSION)
    c.precision = kw.get("precision", 2)
    c.G = kw.get("G", 1.0)
    c.eps = kw.get("eps", 1e-2)
    off = kw.get("offsets")
    if off is not None:
        arr = np.ascontiguousarray(off, dtype=np.int64)
        c._keep = arr
        c.n_systems = len(arr) - 1
        c.offsets = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    else:
        c.n_systems = kw.get("n_systems", 1)
        c.offsets = None
    c.workspace = kw.get("ws", None)
    c.workspace_bytes = kw.get("ws_bytes", 0)
    c.stream = None
    c.flags = kw.get("flags", 0)
    c.reserved = kw.get("reserved", 0)
    return c


def _ws_size(nb, c, n, steps=0, ck=0):
    b = ctypes.c_size_t()
    rc = nb.lib().nbody_workspace_size(ctypes.byref(c), n, steps, ck, ctypes.byref(b))
    return rc, b.value


def test_workspace_size_grows_with_n_and_backward(nb):
    rc, a = _ws_size(nb, _cfg(nb), 1000)
    assert rc == 0 and a > 0
    rc, b = _ws_size(nb, _cfg(nb), 100000)
    assert rc == 0 and b > a
    rc, c = _ws_size(nb, _cfg(nb), 100000, 200, 20)
    assert rc == 0 and c > b
    rc, z = _ws_size(nb, _cfg(nb), 0)
    assert rc == 0


def test_workspace_covers_batched_partials(nb):
    """Persistent batched passes always write one partial-sum slot per j-chunk: the
    planned workspace must hold at least 4 planes (force) / 8 planes (adjoint) of n
    doubles on top of the j-array, even when every system fits in one chunk."""
    off = [0, 100, 300, 301, 700]
    n = 700
    rc, fw = _ws_size(nb, _cfg(nb, offsets=off, precision=2), n)
    assert rc == 0 and fw >= n * 16 + 4 * n * 8
    rc, bw = _ws_size(nb, _cfg(nb, offsets=off, precision=0), n, 6, 3)
    assert rc == 0 and bw >= 2 * n * 32 + 8 * n * 8 + 4 * 3 * n * 8


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("kw,code,needle", [
    (dict(abi=99), 1, "abi_version"),
    (dict(precision=7), 1, "precision"),
    (dict(eps=0.0), 1, "eps"),
    (dict(eps=-1.0), 1, "eps"),
    (dict(eps=float("nan")), 1, "eps"),
    (dict(eps=1e-12), 1, "FP32"),
    (dict(G=float("inf")), 1, "G"),
    (dict(n_systems=0), 1, "n_systems"),
    (dict(n_systems=2), 1, "offsets"),
    (dict(offsets=[0, 5, 3, 10]), 1, "non-decreasing"),
    (dict(offsets=[1, 5, 10]), 1, "offsets[0]"),
    (dict(offsets=[0, 5, 9]), 1, "must equal n"),
    (dict(flags=16), 1, "flags"),
    (dict(flags=32), 1, "flags"),
    (dict(flags=15 | 64), 1, "flags"),
    (dict(reserved=1), 1, "reserved"),
    (dict(), 4, "workspace is NULL"),
    (dict(ws=0x1000, ws_bytes=10), 4, "too small"),
    (dict(ws=0x1001, ws_bytes=1 << 40), 4, "aligned"),
])
def test_forces_argument_errors(nb, kw, code, needle):
    c = _cfg(nb, **kw)
    rc = nb.lib().nbody_forces(ctypes.byref(c), 10, FAKE, FAKE, FAKE, None)
    assert rc == code
    assert needle in nb.lib().nbody_last_error().decode()


def test_other_entry_point_errors(nb):
    L = nb.lib()
    c = _cfg(nb, ws=0x1000, ws_bytes=1 << 40)
    assert L.nbody_forces(ctypes.byref(c), -1, FAKE, FAKE, FAKE, None) == 1
    assert L.nbody_forces(None, 10, FAKE, FAKE, FAKE, None) == 1
    assert L.nbody_forces(ctypes.byref(c), 10, None, FAKE, FAKE, None) == 1
    assert L.nbody_step(ctypes.byref(c), 10, float("nan"), FAKE, FAKE, FAKE, FAKE, None) == 1
    assert L.nbody_rollout(ctypes.byref(c), 10, 1e-3, -1, 0, FAKE, FAKE, FAKE, FAKE, None, None) == 1
    assert L.nbody_rollout(ctypes.byref(c), 10, 1e-3, 5, 0, FAKE, FAKE, FAKE, FAKE, FAKE, None) == 1
    assert L.nbody_rollout_backward(ctypes.byref(c), 10, 1e-3, 5, 0, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE) == 1
    assert L.nbody_rollout_backward(ctypes.byref(c), 10, 1e-3, 5, 2, None, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE) == 1
    assert L.nbody_rollout_backward_reversible(ctypes.byref(c), 10, float("inf"), 5, FAKE, FAKE, FAKE, FAKE, FAKE,
                                               FAKE, FAKE, FAKE) == 1
    assert L.nbody_rollout_backward_reversible(ctypes.byref(c), 10, 1e-3, -1, FAKE, FAKE, FAKE, FAKE, FAKE,
                                               FAKE, FAKE, FAKE) == 1
    assert L.nbody_rollout_backward_reversible(ctypes.byref(c), 10, 1e-3, 5, FAKE, None, FAKE, FAKE, FAKE,
                                               FAKE, FAKE, FAKE) == 1
    assert L.nbody_energy_momentum(ctypes.byref(c), 10, FAKE, FAKE, FAKE, None, None) == 1
    assert "out" in L.nbody_last_error().decode()
    # n == 0 is a valid no-op that touches nothing
    assert L.nbody_forces(ctypes.byref(_cfg(nb)), 0, None, None, None, None) == 0
    assert L.nbody_step(ctypes.byref(_cfg(nb)), 0, 1e-3, None, None, None, None, None) == 0


def test_tile_table_validation(nb):
    good = [dict(kernel="force", precision="fp32c", n_min=0, n_max=1 << 40, variant=0, j_split=1)]
    nb.set_tile_table(good)
    assert nb.tile_lookup("force", "fp32c", 5000) == (0, 1)
    with pytest.raises(nb.NBodyError):
        nb.set_tile_table([dict(kernel="force", precision="fp32c", n_min=0, n_max=10, variant=99, j_split=1)])
    with pytest.raises(nb.NBodyError):
        nb.set_tile_table([dict(kernel="force", precision="fp32c", n_min=5, n_max=1, variant=0, j_split=1)])
    nb.restore_tile_table()
    v, s = nb.tile_lookup("force", "fp32c", 1 << 20)
    assert v >= 0 and s >= 1


def _lj(nb, **kw):
    p = nb.lj_params(kw.get("sigma", 1.0), kw.get("epsilon", 1.0), kw.get("soft", 0.0), kw.get("box"))
    if "reserved" in kw:
        p.reserved = kw["reserved"]
    if "walls" in kw:
        p.walls = kw["walls"]
    return p


def test_lj_params_layout(nb):
    """nbody_lj_params: 3 doubles, 2 int32, 6 doubles = 80 bytes, no padding."""
    assert ctypes.sizeof(nb.LJParams) == 80
    assert nb.LJParams.lo.offset == 32 and nb.LJParams.hi.offset == 56


@pytest.mark.parametrize("kw,needle", [
    (dict(sigma=0.0), "sigma"),
    (dict(sigma=float("nan")), "sigma"),
    (dict(epsilon=float("inf")), "epsilon"),
    (dict(soft=-0.1), "soft"),
    (dict(soft=1e-12), "soft/sigma"),
    (dict(reserved=3), "reserved"),
    (dict(walls=2), "walls"),
    (dict(box=([0, 0, 0], [1, 1, 0])), "box"),
    (dict(box=([0, 0, float("nan")], [1, 1, 1])), "box"),
])
def test_lj_argument_errors_cpu(nb, kw, needle):
    c = _cfg(nb, ws=0x1000, ws_bytes=1 << 40)
    lj = _lj(nb, **kw)
    rc = nb.lib().nbody_lj_rollout(ctypes.byref(c), ctypes.byref(lj), 10, 1e-3, 1, FAKE, FAKE, FAKE, FAKE, None)
    assert rc == 1
    assert needle in nb.lib().nbody_last_error().decode()


def test_lj_ignores_gravity_constants(nb):
    """G and eps are not used by the Lennard-Jones calls, so they are not checked there
    (n == 0 returns before any device work); the workspace size ignores them too."""
    c = _cfg(nb, eps=0.0, G=float("nan"))
    assert nb.lib().nbody_lj_forces(ctypes.byref(c), ctypes.byref(_lj(nb)), 0, None, None, None, None) == 0
    assert nb.lib().nbody_lj_forces(None, ctypes.byref(_lj(nb)), 0, None, None, None, None) == 1
    assert nb.lib().nbody_lj_forces(ctypes.byref(c), None, 0, None, None, None, None) == 1
    rc, b = _ws_size(nb, c, 1000)
    assert rc == 0 and b > 0
    rc, b2 = _ws_size(nb, _cfg(nb), 1000)
    assert b == b2


def test_known_flags_accepted(nb):
    """The per-system loop and the whole-rollout flags pass validation (the call then stops
    at the missing workspace, the first check after the configuration)."""
    for flags in (nb.FLAG_LOOP_SYSTEMS, nb.FLAG_WHOLE_ROLLOUT, nb.FLAG_PER_PASS, nb.FLAG_SYM_ROUNDS, 15):
        c = _cfg(nb, flags=flags)
        assert nb.lib().nbody_forces(ctypes.byref(c), 10, FAKE, FAKE, FAKE, None) == 4
        assert "workspace is NULL" in nb.lib().nbody_last_error().decode()


def test_workspace_size_covers_whole_rollout_tables(nb):
    """A batch's workspace, which holds the whole-rollout tables (unit copy, reduction tasks,
    per-system counters), does not depend on the flags."""
    import numpy as np
    sizes = [0, 1, 300, 5000, 9000, 64]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    b = []
    for flags in (0, nb.FLAG_WHOLE_ROLLOUT):
        c = _cfg(nb, n_systems=len(sizes), offsets=list(off), flags=flags)
        out = ctypes.c_size_t()
        assert nb.lib().nbody_workspace_size(ctypes.byref(c), int(off[-1]), 10, 0, ctypes.byref(out)) == 0
        b.append(out.value)
    assert b[0] == b[1] and b[0] > 0


def test_wait_limit_argument(nb):
    assert nb.lib().nbody_set_wait_limit(0) == 1
    assert "probes" in nb.lib().nbody_last_error().decode()
    assert nb.lib().nbody_set_wait_limit(-5) == 1
    assert nb.lib().nbody_set_wait_limit(1 << 24) == 0


def test_tuned_table_names_the_variants_it_was_tuned_with(nb):
    """Every entry of the tuned table records the description of the variant it chose; the
    index must still name that variant in this build (variant lists only ever grow at the end)."""
    import json
    import os
    path = os.path.join(os.path.dirname(nb.__file__), "tune", "gfx950.json")
    for e in json.load(open(path))["entries"]:
        assert nb.tile_variants(e["kernel"], e["precision"])[e["variant"]] == e["desc"], e


def test_restore_tile_table(nb):
    """An empty table selects the built-in defaults; restore_tile_table reloads the tuned
    table the binding loaded at start-up."""
    import json
    import os
    path = os.path.join(os.path.dirname(nb.__file__), "tune", "gfx950.json")
    tuned = [e for e in json.load(open(path))["entries"]
             if e["kernel"] == "force" and e["precision"] == "fp32c" and e["n_min"] <= (1 << 20) <= e["n_max"]][0]
    try:
        nb.set_tile_table([])
        builtin = nb.tile_lookup("force", "fp32c", 1 << 20)
        nb.restore_tile_table()
        assert nb.tile_lookup("force", "fp32c", 1 << 20) == (tuned["variant"], 1)
        assert builtin != (tuned["variant"], 1)
    finally:
        nb.restore_tile_table()


def test_autotune_bucket_bounds_tile_the_size_axis():
    """Tuned buckets split the particle-count axis at geometric midpoints, cover it from 0 to
    2^40 without gaps or overlaps, and a partial re-tune keeps the standard list's ranges."""
    from paper_2511_02655_amd import autotune as at
    b = at.FORCE_BUCKETS
    rng = [at._bounds(b, k) for k in range(len(b))]
    assert rng[0][0] == 0 and rng[-1][1] == 1 << 40
    for (lo, hi), (lo2, _) in zip(rng, rng[1:]):
        assert lo2 == hi + 1
    for k, n in enumerate(b):
        assert rng[k][0] <= n <= rng[k][1]
    assert at._bounds(b, 2) == (int((4096 * 16384) ** 0.5) + 1, int((16384 * 65536) ** 0.5))
    # re-tuning one bucket alone against the standard list gives it the same range
    assert at._bounds([16384], 0, b) == rng[2]


def test_autotune_pick_prefers_larger_symmetric_blocks_within_slack():
    """Among candidates within 1% of the fastest, the largest symmetric block wins (half the
    partial-sum workspace per doubling); outside the slack the fastest wins."""
    from paper_2511_02655_amd import autotune as at
    descs = ["bs=256,i=1,tj=256", "bs=256,i=4,sym=1024,rot=lds", "bs=256,i=8,sym=2048,rot=lds,pipe"]
    assert at._pick([(1.000, 0), (1.005, 1), (1.009, 2)], descs)[1] == 2
    assert at._pick([(1.000, 0), (1.005, 1), (1.02, 2)], descs)[1] == 1
    assert at._pick([(1.000, 1), (1.05, 2), (0.98, 0)], descs)[1] == 0
    assert at._sym_edge(descs[2]) == 2048 and at._sym_edge(descs[0]) == 0


def test_step_noalloc_rejections_before_device_work(nb):
    """The allocation-free step refuses, on the host and before any HIP call, a caller workspace,
    batches, and systems whose step needs more than the static scratch."""
    L = nb.lib()
    z = ctypes.c_void_p(0)
    c = _cfg(nb, ws=ctypes.c_void_p(256), ws_bytes=1 << 20)
    assert L.nbody_step_noalloc(ctypes.byref(c), 10, 1e-3, z, z, z, z, None) == 1
    assert b"workspace" in L.nbody_last_error()
    c = _cfg(nb, offsets=[0, 5, 10])
    assert L.nbody_step_noalloc(ctypes.byref(c), 10, 1e-3, z, z, z, z, None) == 3
    c = _cfg(nb)
    assert L.nbody_step_noalloc(ctypes.byref(c), 1 << 23, 1e-3, z, z, z, z, None) == 4
    assert b"static scratch" in L.nbody_last_error()
    # zero particles: nothing to do, OK without touching a device
    assert L.nbody_step_noalloc(ctypes.byref(c), 0, 1e-3, z, z, z, z, None) == 0


def test_workspace_stays_linear_beyond_the_symmetric_cap(nb):
    """Symmetric tiles keep O(n^2 / block) float slots; past 16 GiB of them a single-system force
    pass runs on the round schedule (per-particle accumulators) and the adjoint one-sided, so the
    workspace of a 4M-particle call is O(n) (and smaller than at 1M)."""
    for prec in (1, 2, 4):  # plain, compensated, adaptive FP32
        rc, w1m = _ws_size(nb, _cfg(nb, precision=prec), 1 << 20)
        assert rc == 0 and w1m > (1 << 33)  # ~8.6 GB of tile partials on the tuned 2048-particle tiles
        rc, w4m = _ws_size(nb, _cfg(nb, precision=prec), 1 << 22)
        assert rc == 0 and w4m < 240 * (1 << 22) and w4m < w1m  # 4 accumulator copies: 128 B per particle
        rc, wb = _ws_size(nb, _cfg(nb, precision=prec), 1 << 22, 10, 5)  # with a backward pass
        assert rc == 0 and wb < 1000 * (1 << 22)
    v = ctypes.c_int32()
    sp = ctypes.c_int32()
    for kernel in (0, 1):
        assert nb.lib().nbody_tile_lookup(kernel, 2, 1 << 22, ctypes.byref(v), ctypes.byref(sp)) == 0
        assert "sym=" not in nb.tile_variants(["force", "adjoint"][kernel], "fp32c")[v.value]


def test_round_schedule_flag_workspace(nb):
    """NBODY_FLAG_SYM_ROUNDS (8) is accepted and puts a single-system FP32 pass on per-particle
    accumulators: 4 copies of 32 bytes per particle instead of the slot planes (8.6 GB at 1M)."""
    n = 1 << 20
    for prec in (1, 2, 3, 4):
        rc, slots = _ws_size(nb, _cfg(nb, precision=prec), n)
        rc2, rounds = _ws_size(nb, _cfg(nb, precision=prec, flags=8), n)
        assert rc == 0 and rc2 == 0
        assert 128 * n < rounds < 240 * n < slots, (prec, rounds, slots)
    rc, w64 = _ws_size(nb, _cfg(nb, precision=0, flags=8), n)  # FP64 has no symmetric tiles
    rc2, w64b = _ws_size(nb, _cfg(nb, precision=0), n)
    assert rc == 0 and rc2 == 0 and w64 == w64b


def test_forces_shard_arguments(nb):
    """nbody_forces_shard (one GPU's share of the ring decomposition): its workspace is the
    j-array plus one [4][n] double plane set per j-block (none for P = 1); P < 1, g outside
    [0, P) and batches are rejected before any device work."""
    L = nb.lib()
    n = 1 << 20
    b = ctypes.c_size_t()
    for prec, jb in ((2, 16), (3, 32), (0, 32)):
        assert L.nbody_forces_shard_workspace_size(ctypes.byref(_cfg(nb, precision=prec)), n, 8, ctypes.byref(b)) == 0
        assert jb * n + 8 * 32 * n <= b.value < jb * n + 8 * 32 * n + 1024, (prec, b.value)
        assert L.nbody_forces_shard_workspace_size(ctypes.byref(_cfg(nb, precision=prec)), n, 1, ctypes.byref(b)) == 0
        assert jb * n <= b.value < jb * n + 512, (prec, b.value)
    # 1000 particles are four 256-particle j-tiles: at most four blocks carry partial planes
    assert L.nbody_forces_shard_workspace_size(ctypes.byref(_cfg(nb)), 1000, 8, ctypes.byref(b)) == 0
    assert b.value < 16 * 1000 + 4 * 32 * 1000 + 1024
    assert L.nbody_forces_shard_workspace_size(ctypes.byref(_cfg(nb)), n, 0, ctypes.byref(b)) == 1
    z = np.zeros(3)
    zp = z.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for P, g in ((0, 0), (8, 8), (8, -1)):
        assert L.nbody_forces_shard(ctypes.byref(_cfg(nb)), 10, P, g, zp, zp, zp, None) == 1, (P, g)
    batched = _cfg(nb, offsets=[0, 5, 10])
    assert L.nbody_forces_shard_workspace_size(ctypes.byref(batched), 10, 2, ctypes.byref(b)) == 3
    assert L.nbody_forces_shard(ctypes.byref(batched), 10, 2, 0, zp, zp, zp, None) == 3
