"""MI355X (gfx950) all-pairs N-body hot path: Python binding of libnbody.so.

Every step of the path runs in the HIP kernels of libnbody.so (built from
csrc/ with ``python -m paper_2511_02655_amd.build``); this module only
marshals torch tensors (device memory, the current HIP stream) through the
C ABI declared in include/nbody.h. There is no CPU fallback: if the library
is missing or no GPU is present the calls raise.

Arrays: positions/velocities/accelerations are float64 tensors of shape (3, n)
on the GPU (SoA planes), masses float64 of shape (n,).

Precision names: "fp64", "fp32", "fp32c" (FP32 pair math with compensated
accumulation), "fp32ds" (compensated, with double-float separations). State,
updates and reductions are FP64 in every mode.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnbody.so")

NBODY_ABI_VERSION = 1
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32c": 2, "fp32ds": 3, "fp32a": 4}
KERNELS = {"force": 0, "adjoint": 1, "force_batched": 2, "adjoint_batched": 3, "lj_force": 4,
           "lj_force_batched": 5}
FLAG_LOOP_SYSTEMS = 1
FLAG_WHOLE_ROLLOUT = 2  # batched symmetric rollouts: every step in one launch
FLAG_PER_PASS = 4  # batched rollouts: one launch per pass even where one launch for all steps is chosen
FLAG_SYM_ROUNDS = 8  # single-system FP32 force passes on the round schedule (workspace linear in n)
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "DEVICE", 3: "UNSUPPORTED", 4: "WORKSPACE"}

EXPORTED = ("nbody_abi_version", "nbody_last_error", "nbody_workspace_size", "nbody_forces", "nbody_step",
            "nbody_rollout", "nbody_energy_momentum", "nbody_rollout_backward", "nbody_set_tile_table",
            "nbody_tile_variants", "nbody_tile_lookup", "nbody_lj_forces", "nbody_lj_rollout",
            "nbody_rollout_backward_reversible", "nbody_diagnostics", "nbody_set_wait_limit",
            "nbody_step_noalloc", "nbody_forces_shard_workspace_size", "nbody_forces_shard")


class NBodyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("nbody status %d (%s): %s" % (code, STATUS.get(code, "?"), msg))
        self.code = code


class NBodyConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("G", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("n_systems", ctypes.c_int64),
        ("offsets", ctypes.POINTER(ctypes.c_int64)),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class LJParams(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double),
        ("epsilon", ctypes.c_double),
        ("soft", ctypes.c_double),
        ("walls", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
    ]


class TileEntry(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_min", ctypes.c_int64),
        ("n_max", ctypes.c_int64),
        ("variant", ctypes.c_int32),
        ("j_split", ctypes.c_int32),
    ]


_lib_handle = None


def lib():
    """Load libnbody.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libnbody.so is not built (%s); run python -m paper_2511_02655_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    C = ctypes.POINTER(NBodyConfig)
    sig = {
        "nbody_abi_version": ([], ctypes.c_int),
        "nbody_last_error": ([], ctypes.c_char_p),
        "nbody_workspace_size": ([C, I64, I64, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "nbody_forces": ([C, I64, P, P, P, P], ctypes.c_int),
        "nbody_forces_shard_workspace_size": ([C, I64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "nbody_forces_shard": ([C, I64, ctypes.c_int32, ctypes.c_int32, P, P, P, P], ctypes.c_int),
        "nbody_step": ([C, I64, D, P, P, P, P, P], ctypes.c_int),
        "nbody_step_noalloc": ([C, I64, D, P, P, P, P, P], ctypes.c_int),
        "nbody_rollout": ([C, I64, D, I64, I64, P, P, P, P, P, P], ctypes.c_int),
        "nbody_energy_momentum": ([C, I64, P, P, P, P, P], ctypes.c_int),
        "nbody_diagnostics": ([C, I64, P, P, P, P, P, P], ctypes.c_int),
        "nbody_rollout_backward": ([C, I64, D, I64, I64, P, P, P, P, P, P, P], ctypes.c_int),
        "nbody_rollout_backward_reversible": ([C, I64, D, I64, P, P, P, P, P, P, P, P], ctypes.c_int),
        "nbody_set_tile_table": ([ctypes.POINTER(TileEntry), I64], ctypes.c_int),
        "nbody_tile_variants": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
        "nbody_tile_lookup": ([ctypes.c_int32, ctypes.c_int32, I64, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "nbody_lj_forces": ([C, ctypes.POINTER(LJParams), I64, P, P, P, P], ctypes.c_int),
        "nbody_lj_rollout": ([C, ctypes.POINTER(LJParams), I64, D, I64, P, P, P, P, P], ctypes.c_int),
        "nbody_set_wait_limit": ([I64], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if L.nbody_abi_version() != NBODY_ABI_VERSION:
        raise RuntimeError("libnbody ABI %d != binding ABI %d" % (L.nbody_abi_version(), NBODY_ABI_VERSION))
    _lib_handle = L
    _load_default_tiles(L)
    return L


def _check(rc: int):
    if rc != 0:
        raise NBodyError(rc, lib().nbody_last_error().decode(errors="replace"))


# ------------------------------------------------------------------ tile table

TUNE_DIR = os.path.join(_PKG, "tune")


def _load_default_tiles(L):
    path = os.environ.get("NBODY_TILE_TABLE", os.path.join(TUNE_DIR, "gfx950.json"))
    if os.path.exists(path):
        import json
        with open(path) as f:
            entries = json.load(f).get("entries", [])
        _set_table(L, entries)


def _set_table(L, entries):
    arr = (TileEntry * max(len(entries), 1))()
    for k, e in enumerate(entries):
        arr[k] = TileEntry(KERNELS[e["kernel"]] if isinstance(e["kernel"], str) else e["kernel"],
                           PRECISIONS[e["precision"]] if isinstance(e["precision"], str) else e["precision"],
                           int(e["n_min"]), int(e["n_max"]), int(e["variant"]), int(e["j_split"]))
    rc = L.nbody_set_tile_table(arr, len(entries))
    if rc != 0:
        raise NBodyError(rc, L.nbody_last_error().decode())


def set_tile_table(entries: Sequence[dict]):
    """Replace the tile table; entries are dicts with kernel, precision, n_min, n_max, variant, j_split.
    An empty list selects the library's built-in defaults (restore_tile_table reloads the tuned table)."""
    _set_table(lib(), list(entries))


def restore_tile_table():
    """Reload the table loaded at start-up (NBODY_TILE_TABLE or tune/gfx950.json; the built-in
    defaults when there is none)."""
    L = lib()
    _set_table(L, [])
    _load_default_tiles(L)


def tile_variants(kernel: str, precision: str):
    buf = ctypes.create_string_buffer(4096)
    nv = lib().nbody_tile_variants(KERNELS[kernel], PRECISIONS[precision], buf, len(buf))
    if nv < 0:
        raise NBodyError(1, lib().nbody_last_error().decode())
    return [s.decode() for s in buf.raw.split(b"\0")[:nv]]


def set_wait_limit(probes: int = 1 << 24) -> None:
    """Probes a whole-rollout wait makes before it gives up (default 2^24)."""
    _check(lib().nbody_set_wait_limit(int(probes)))


def tile_lookup(kernel: str, precision: str, n: int):
    v = ctypes.c_int32()
    s = ctypes.c_int32()
    _check(lib().nbody_tile_lookup(KERNELS[kernel], PRECISIONS[precision], n, ctypes.byref(v), ctypes.byref(s)))
    return v.value, s.value


# ------------------------------------------------------------------ workspace / config

_ws_cache = {}


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _Cfg:
    """A filled NBodyConfig plus the host offsets array it points to (kept alive)."""

    def __init__(self, precision="fp32c", G=1.0, eps=1e-2, offsets=None, flags=0, stream=None):
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % list(PRECISIONS))
        self.cfg = NBodyConfig()
        self.cfg.abi_version = NBODY_ABI_VERSION
        self.cfg.precision = PRECISIONS[precision]
        self.cfg.G = float(G)
        self.cfg.eps = float(eps)
        self.offsets = None
        if offsets is not None:
            import numpy as np
            off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
            self.offsets = off
            self.cfg.n_systems = int(off.shape[0] - 1)
            self.cfg.offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        else:
            self.cfg.n_systems = 1
            self.cfg.offsets = None
        self.cfg.flags = int(flags)
        self.cfg.reserved = 0
        self.cfg.stream = _stream_ptr(stream)
        self.cfg.workspace = None
        self.cfg.workspace_bytes = 0

    def workspace(self, n, steps=0, ckpt_every=0, device=None, shard_P=0):
        need = ctypes.c_size_t()
        if shard_P:
            _check(lib().nbody_forces_shard_workspace_size(ctypes.byref(self.cfg), n, shard_P, ctypes.byref(need)))
        else:
            _check(lib().nbody_workspace_size(ctypes.byref(self.cfg), n, steps, ckpt_every, ctypes.byref(need)))
        nbytes = int(need.value)
        torch = _torch()
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        key = (str(dev), self.cfg.stream.value if hasattr(self.cfg.stream, "value") else self.cfg.stream)
        buf = _ws_cache.get(key)
        if buf is None or buf.numel() < nbytes + 256:
            buf = torch.empty(max(nbytes + 256, 1 << 16), dtype=torch.uint8, device=dev)
            _ws_cache[key] = buf
        base = buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.cfg.workspace = ctypes.c_void_p(aligned)
        self.cfg.workspace_bytes = nbytes
        self._ws = buf
        return nbytes


def _dptr(t, name, shape=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64 (got %s)" % (name, t.dtype))
    if t.device.type != "cuda":
        raise ValueError("%s must be on the GPU (got %s)" % (name, t.device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _n_of(mass):
    if mass.dim() != 1:
        raise ValueError("mass must be 1-D")
    return int(mass.shape[0])


# ------------------------------------------------------------------ entry points

def forces(pos, mass, *, G=1.0, eps=1e-2, precision="fp32c", want_pot=False, offsets=None, flags=0,
           out_acc=None, out_pot=None, stream=None):
    """All-pairs accelerations (3, n) and optionally potentials (n,)."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    acc = out_acc if out_acc is not None else torch.empty((3, n), dtype=torch.float64, device=mass.device)
    pot = (out_pot if out_pot is not None else torch.empty(n, dtype=torch.float64, device=mass.device)) \
        if want_pot else None
    _check(lib().nbody_forces(ctypes.byref(c.cfg), n, _dptr(pos, "pos", (3, n)), _dptr(mass, "mass"),
                              _dptr(acc, "acc", (3, n)), _dptr(pot, "pot", (n,))))
    return acc, pot


def forces_shard(pos, mass, P, g, *, G=1.0, eps=1e-2, precision="fp32c", want_pot=False, out_acc=None,
                 out_pot=None, stream=None):
    """Share g of P of the ring decomposition: the rows of block g of (3, n) accelerations (and
    (n,) potentials) from all n particles; the other rows of out_acc / out_pot are left as they
    are (zeros when the arrays are allocated here). Returns (acc, pot, (i0, i1))."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, None, 0, stream)
    c.workspace(n, device=mass.device, shard_P=P)
    acc = out_acc if out_acc is not None else torch.zeros((3, n), dtype=torch.float64, device=mass.device)
    pot = (out_pot if out_pot is not None else torch.zeros(n, dtype=torch.float64, device=mass.device)) \
        if want_pot else None
    _check(lib().nbody_forces_shard(ctypes.byref(c.cfg), n, int(P), int(g), _dptr(pos, "pos", (3, n)),
                                    _dptr(mass, "mass"), _dptr(acc, "acc", (3, n)), _dptr(pot, "pot", (n,))))
    return acc, pot, shard_range(n, P, g)


def shard_range(n, P, g):
    """Rows [i0, i1) of share g of P: blocks of s = 256 ceil(t / min(P, t)) particles, t = ceil(n / 256)."""
    t = max(1, -(-n // 256))
    s = 256 * -(-t // min(P, t))
    i0 = min(n, g * s)
    return i0, min(n, i0 + s)


def step(pos, vel, mass, acc, dt, *, G=1.0, eps=1e-2, precision="fp32c", offsets=None, flags=0, out_pot=None,
         stream=None):
    """One KDK step in place (acc: in a(x_n), out a(x_{n+1})); out_pot (n,), when given,
    receives the potential at x_{n+1} from the same force pass."""
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    _check(lib().nbody_step(ctypes.byref(c.cfg), n, float(dt), _dptr(pos, "pos", (3, n)), _dptr(vel, "vel", (3, n)),
                            _dptr(mass, "mass"), _dptr(acc, "acc", (3, n)), _dptr(out_pot, "pot", (n,))))


def step_noalloc(pos, vel, mass, acc, dt, *, G=1.0, eps=1e-2, precision="fp32c", out_pot=None, stream=None):
    """nbody_step without a workspace: the library's static device scratch serves it (single
    systems whose step fits NBODY_NOALLOC_SCRATCH_BYTES)."""
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, None, 0, stream)
    _check(lib().nbody_step_noalloc(ctypes.byref(c.cfg), n, float(dt), _dptr(pos, "pos", (3, n)),
                                    _dptr(vel, "vel", (3, n)), _dptr(mass, "mass"), _dptr(acc, "acc", (3, n)),
                                    _dptr(out_pot, "pot", (n,))))


def rollout(pos, vel, mass, acc, dt, steps, *, ckpt_every=0, energy_trace=False, G=1.0, eps=1e-2,
            precision="fp32c", offsets=None, flags=0, ckpt=None, stream=None):
    """`steps` KDK steps in place. Returns (ckpt or None, energy trace (steps+1, S, 5) or None)."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    S = c.cfg.n_systems
    if ckpt_every and ckpt is None:
        ckpt = torch.empty((steps // ckpt_every + 1, 6, n), dtype=torch.float64, device=mass.device)
    if ckpt is not None and ckpt_every:
        if tuple(ckpt.shape) != (steps // ckpt_every + 1, 6, n):
            raise ValueError("ckpt must have shape %s" % ((steps // ckpt_every + 1, 6, n),))
    trace = torch.empty((steps + 1, S, 5), dtype=torch.float64, device=mass.device) if energy_trace else None
    _check(lib().nbody_rollout(ctypes.byref(c.cfg), n, float(dt), int(steps), int(ckpt_every),
                               _dptr(pos, "pos", (3, n)), _dptr(vel, "vel", (3, n)), _dptr(mass, "mass"),
                               _dptr(acc, "acc", (3, n)), _dptr(ckpt, "ckpt") if ckpt_every else None,
                               _dptr(trace, "energy_trace")))
    return (ckpt if ckpt_every else None), trace


def energy_momentum(pos, vel, mass, pot=None, *, G=1.0, eps=1e-2, precision="fp32c", offsets=None, flags=0,
                    stream=None):
    """(n_systems, 5) tensor of KE, PE, Px, Py, Pz."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    out = torch.empty((c.cfg.n_systems, 5), dtype=torch.float64, device=mass.device)
    _check(lib().nbody_energy_momentum(ctypes.byref(c.cfg), n, _dptr(pos, "pos", (3, n)), _dptr(vel, "vel", (3, n)),
                                       _dptr(mass, "mass"), _dptr(pot, "pot", (n,)), _dptr(out, "out")))
    return out


def rollout_backward(mass, ckpt, gpos_final, gvel_final, dt, steps, ckpt_every, *, G=1.0, eps=1e-2,
                     precision="fp32c", offsets=None, flags=0, stream=None):
    """Discrete-adjoint gradients (gpos0 (3, n), gvel0 (3, n), gmass (n,))."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, offsets, flags, stream)
    c.workspace(n, steps, ckpt_every, device=mass.device)
    gx = torch.empty((3, n), dtype=torch.float64, device=mass.device)
    gv = torch.empty((3, n), dtype=torch.float64, device=mass.device)
    gm = torch.empty(n, dtype=torch.float64, device=mass.device)
    _check(lib().nbody_rollout_backward(ctypes.byref(c.cfg), n, float(dt), int(steps), int(ckpt_every),
                                        _dptr(mass, "mass"), _dptr(ckpt, "ckpt"),
                                        _dptr(gpos_final, "gpos_final", (3, n)),
                                        _dptr(gvel_final, "gvel_final", (3, n)), _dptr(gx, "gpos0"),
                                        _dptr(gv, "gvel0"), _dptr(gm, "gmass")))
    return gx, gv, gm


# ------------------------------------------------------------------ Lennard-Jones gas (Eq. (1))

def lj_params(sigma=1.0, epsilon=1.0, soft=0.0, box=None) -> LJParams:
    """Pair-law parameters; box = (lo[3], hi[3]) turns on the reflective walls."""
    p = LJParams()
    p.sigma, p.epsilon, p.soft = float(sigma), float(epsilon), float(soft)
    p.reserved = 0
    if box is not None:
        p.walls = 1
        for c in range(3):
            p.lo[c] = float(box[0][c])
            p.hi[c] = float(box[1][c])
    else:
        p.walls = 0
    return p


def lj_forces(pos, mass, *, sigma=1.0, epsilon=1.0, soft=0.0, precision="fp32c", want_pot=False, offsets=None,
              flags=0, out_acc=None, out_pot=None, stream=None):
    """Lennard-Jones accelerations F_i/m_i (3, n) and optionally potentials per unit mass (n,)."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, 1.0, 1.0, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    lj = lj_params(sigma, epsilon, soft)
    acc = out_acc if out_acc is not None else torch.empty((3, n), dtype=torch.float64, device=mass.device)
    pot = (out_pot if out_pot is not None else torch.empty(n, dtype=torch.float64, device=mass.device)) \
        if want_pot else None
    _check(lib().nbody_lj_forces(ctypes.byref(c.cfg), ctypes.byref(lj), n, _dptr(pos, "pos", (3, n)),
                                 _dptr(mass, "mass"), _dptr(acc, "acc", (3, n)), _dptr(pot, "pot", (n,))))
    return acc, pot


def lj_rollout(pos, vel, mass, acc, dt, steps, *, sigma=1.0, epsilon=1.0, soft=0.0, box=None,
               energy_trace=False, precision="fp32c", offsets=None, flags=0, stream=None):
    """`steps` KDK steps of the Lennard-Jones gas in place (reflective walls when box is
    given). Returns the energy trace (steps+1, S, 5) or None."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, 1.0, 1.0, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    lj = lj_params(sigma, epsilon, soft, box)
    trace = torch.empty((steps + 1, c.cfg.n_systems, 5), dtype=torch.float64, device=mass.device) \
        if energy_trace else None
    _check(lib().nbody_lj_rollout(ctypes.byref(c.cfg), ctypes.byref(lj), n, float(dt), int(steps),
                                  _dptr(pos, "pos", (3, n)), _dptr(vel, "vel", (3, n)), _dptr(mass, "mass"),
                                  _dptr(acc, "acc", (3, n)), _dptr(trace, "energy_trace")))
    return trace


DIAGNOSTICS = ("KE", "PE", "Px", "Py", "Pz", "Lx", "Ly", "Lz", "W", "M")


def diagnostics(pos, vel, mass, pot, acc, *, precision="fp32c", offsets=None, flags=0, stream=None):
    """(S, 10) per system: KE, PE, Px, Py, Pz, Lx, Ly, Lz, W = sum m x.a, M (see DIAGNOSTICS),
    from the state and the pot / acc of a force call (either pair law)."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, 1.0, 1.0, offsets, flags, stream)
    c.workspace(n, device=mass.device)
    out = torch.empty((c.cfg.n_systems, 10), dtype=torch.float64, device=mass.device)
    _check(lib().nbody_diagnostics(ctypes.byref(c.cfg), n, _dptr(pos, "pos", (3, n)), _dptr(vel, "vel", (3, n)),
                                   _dptr(mass, "mass"), _dptr(pot, "pot", (n,)), _dptr(acc, "acc", (3, n)),
                                   _dptr(out, "out")))
    return out


def rollout_backward_reversible(mass, pos_final, vel_final, gpos_final, gvel_final, dt, steps, *, G=1.0, eps=1e-2,
                                precision="fp32c", offsets=None, flags=0, stream=None):
    """Discrete-adjoint gradients without checkpoints: the trajectory is rebuilt by
    integrating backwards from (pos_final, vel_final). Returns (gpos0, gvel0, gmass)."""
    torch = _torch()
    n = _n_of(mass)
    c = _Cfg(precision, G, eps, offsets, flags, stream)
    c.workspace(n, steps, 1, device=mass.device)
    gx = torch.empty((3, n), dtype=torch.float64, device=mass.device)
    gv = torch.empty((3, n), dtype=torch.float64, device=mass.device)
    gm = torch.empty(n, dtype=torch.float64, device=mass.device)
    _check(lib().nbody_rollout_backward_reversible(ctypes.byref(c.cfg), n, float(dt), int(steps), _dptr(mass, "mass"),
                                                   _dptr(pos_final, "pos_final", (3, n)),
                                                   _dptr(vel_final, "vel_final", (3, n)),
                                                   _dptr(gpos_final, "gpos_final", (3, n)),
                                                   _dptr(gvel_final, "gvel_final", (3, n)), _dptr(gx, "gpos0"),
                                                   _dptr(gv, "gvel0"), _dptr(gm, "gmass")))
    return gx, gv, gm


from .autograd import NBodyRollout, rollout_fn  # noqa: E402,F401
