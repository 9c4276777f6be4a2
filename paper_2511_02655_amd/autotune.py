"""Tile autotuner for libnbody.so.

For every (kernel, precision, particle-count bucket) it times each compiled tile
variant (and, for the split kernels, a few j-split / j-chunk settings) through
the C ABI on the current GPU, keeps the fastest, and writes the winners as a
tile table (JSON) that the library loads at start-up (tune/<arch>.json, or the
file named by NBODY_TILE_TABLE).

Timing: HIP events on the current stream around `reps` back-to-back calls after
one warm-up call; the median of `trials` such measurements is the score.

Usage (on the GPU): python -m paper_2511_02655_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

FORCE_BUCKETS = [1024, 4096, 16384, 65536, 262144, 1048576]
LJ_BUCKETS = [1024, 4096, 10000, 32768, 131072]
SYM_PART_LIMIT = 16.0 * 2 ** 30  # workspace bytes a symmetric tile may ask for
ADJ_BUCKETS = [1024, 4096, 16384, 65536, 262144]
J_SPLITS = [1, 2, 4, 8, 16, 32, 64]
BATCH_JCHUNK = [512, 1024, 2048, 4096]


def _bounds(buckets, k, standard=()):
    """n-range of bucket k: geometric midpoints to its neighbours, taken from the union of
    the tuned buckets and the standard list, so a partial re-tune keeps the table's ranges."""
    grid = sorted(set(buckets) | set(standard))
    j = grid.index(buckets[k])
    lo = 0 if j == 0 else int(math.sqrt(grid[j - 1] * grid[j])) + 1
    hi = (1 << 40) if j == len(grid) - 1 else int(math.sqrt(grid[j] * grid[j + 1]))
    return lo, hi


def _time(fn, reps, trials=3):
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(trials):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / reps)
    return float(np.median(out))


def _reps_for(n):
    work = float(n) * n
    return int(min(50, max(2, 2e11 / max(work, 1.0))))


def _sym_edge(desc):
    return int(desc.split("sym=")[1].split(",")[0]) if "sym=" in desc else 0


def _pick(cands, descs, slack=0.01):
    """Fastest candidate; among those within `slack` of it, the one with the largest
    symmetric block (fewer partial-sum slots: half the workspace per doubling)."""
    tmin = min(c[0] for c in cands)
    near = [c for c in cands if c[0] <= tmin * (1.0 + slack)]
    return max(near, key=lambda c: (_sym_edge(descs[c[1]]), -c[0]))


def tune_force(nb, torch, precision, buckets, log, law="gravity"):
    """Single-system force pass: gravity on Plummer spheres, or (law="lj") the
    Lennard-Jones gas on its lattice (tile-table kernel "lj_force")."""
    from . import inputs
    entries = []
    kname = "lj_force" if law == "lj" else "force"
    nvar = len(nb.tile_variants(kname, precision))
    for k, n in enumerate(buckets):
        if law == "lj":
            s = inputs.lj_gas(n, 100 + k)[0]
        else:
            s = inputs.plummer(n, 100 + k)
        pos = torch.from_numpy(s.pos).cuda()
        mass = torch.from_numpy(s.mass).cuda()
        acc = torch.empty((3, n), dtype=torch.float64, device="cuda")
        reps = _reps_for(n)
        cands = []
        descs = nb.tile_variants(kname, precision)
        if law == "lj":
            call = lambda: nb.lj_forces(pos, mass, precision=precision, out_acc=acc)
        else:
            call = lambda: nb.forces(pos, mass, eps=1e-2, precision=precision, out_acc=acc)
        for v in range(nvar):
            sym = "sym=" in descs[v]
            if sym and n < 4096:
                continue
            if sym and -(-n // _sym_edge(descs[v])) * 16.0 * n > SYM_PART_LIMIT:
                continue  # float partials of nb slots x 4 components per particle
            for js in ([1] if sym else J_SPLITS):
                if js > 1 and n >= 262144:
                    continue
                nb.set_tile_table([dict(kernel=kname, precision=precision, n_min=0, n_max=1 << 40, variant=v,
                                        j_split=js)])
                t = _time(call, reps)
                rate = float(n) * n / (t * 1e-3)
                log("%s %s n=%d variant %d (%s) j_split %d: %.3f ms  %.3e inter/s" % (kname, precision, n, v, descs[v],
                                                                                   js, t, rate))
                cands.append((t, v, js, rate))
        best = _pick(cands, descs)
        lo, hi = _bounds(buckets, k, LJ_BUCKETS if law == "lj" else FORCE_BUCKETS)
        entries.append(dict(kernel=kname, precision=precision, n_min=lo, n_max=hi, variant=best[1],
                            desc=descs[best[1]], j_split=best[2], tuned_n=n, ms=best[0],
                            interactions_per_s=best[3]))
        nb.set_tile_table([])
    return entries


def tune_adjoint(nb, torch, precision, buckets, log):
    """Times one adjoint pass (backward of a 1-step rollout, dominated by two adjoint
    passes and one recomputed force pass) per variant."""
    from . import inputs
    entries = []
    descs = nb.tile_variants("adjoint", precision)
    for k, n in enumerate(buckets):
        s = inputs.plummer(n, 200 + k)
        pos = torch.from_numpy(s.pos).cuda()
        vel = torch.from_numpy(s.vel).cuda()
        mass = torch.from_numpy(s.mass).cuda()
        acc, _ = nb.forces(pos, mass, precision=precision)
        ckpt, _ = nb.rollout(pos.clone(), vel.clone(), mass, acc.clone(), 1e-3, 1, ckpt_every=1, precision=precision)
        g = torch.ones((3, n), dtype=torch.float64, device="cuda")
        reps = max(1, _reps_for(n) // 2)
        best = None
        for v in range(len(descs)):
            sym = "sym=" in descs[v]
            if sym and (n < 2048 or -(-n // _sym_edge(descs[v])) * 16.0 * n > SYM_PART_LIMIT):
                continue
            for js in ([1] if sym else J_SPLITS):
                nb.set_tile_table([dict(kernel="adjoint", precision=precision, n_min=0, n_max=1 << 40, variant=v,
                                        j_split=js)])
                t = _time(lambda: nb.rollout_backward(mass, ckpt, g, g, 1e-3, 1, 1, precision=precision), reps)
                log("adjoint %s n=%d variant %d (%s) j_split %d: %.3f ms" % (precision, n, v, descs[v], js, t))
                if best is None or t < best[0]:
                    best = (t, v, js)
        lo, hi = _bounds(buckets, k, ADJ_BUCKETS)
        entries.append(dict(kernel="adjoint", precision=precision, n_min=lo, n_max=hi, variant=best[1],
                            desc=descs[best[1]], j_split=best[2], tuned_n=n, ms=best[0]))
        nb.set_tile_table([])
    return entries


# batched mixes tuned separately, keyed by their largest system (systems, smallest, largest, seed)
BATCH_MIXES = [(4096, 16, 256, 7), (1024, 64, 2048, 8), (512, 64, 8192, 6)]


def tune_batched(nb, torch, precision, log, mixes=BATCH_MIXES):
    """Batched force and adjoint passes on mixes of uneven systems (N_s
    log-uniform), one table bucket per mix keyed by its largest system. Each candidate is
    timed inside a 10-step rollout (force) or a 10-step backward (adjoint), so the library's
    per-call host work (work-unit lists, uploads) is paid once per 10 passes as in use."""
    from . import inputs
    results = []  # (kernel, nmax, best, description of the best variant)
    for S, lo_n, hi_n, seed in mixes:
        b = inputs.batched_mix(S, seed, nmin=lo_n, nmax=hi_n)
        off = b.offsets
        pos = torch.from_numpy(b.pos).cuda()
        vel = torch.from_numpy(b.vel).cuda()
        mass = torch.from_numpy(b.mass).cuda()
        nmax = int(np.max(np.diff(off)))
        for kernel in ("force_batched", "adjoint_batched"):
            descs = nb.tile_variants(kernel, precision)
            best = None
            if kernel == "adjoint_batched":
                a0, _ = nb.forces(pos, mass, precision=precision, offsets=off)
                ckpt, _ = nb.rollout(pos.clone(), vel.clone(), mass, a0, 1e-3, 10, ckpt_every=10, precision=precision,
                                     offsets=off)
                g = torch.ones_like(pos)
            else:
                p, v = pos.clone(), vel.clone()
                a, _ = nb.forces(p, mass, precision=precision, offsets=off)
            for var in range(len(descs)):
                for jc in ([1] if "sym=" in descs[var] else BATCH_JCHUNK):  # symmetric units: whole tiles
                    nb.set_tile_table([dict(kernel=kernel, precision=precision, n_min=0, n_max=1 << 40, variant=var,
                                            j_split=jc)])
                    if kernel == "force_batched":
                        fn = lambda: nb.rollout(p, v, mass, a, 1e-3, 10, precision=precision, offsets=off)
                    else:
                        fn = lambda: nb.rollout_backward(mass, ckpt, g, g, 1e-3, 10, 10, precision=precision,
                                                         offsets=off)
                    t = _time(fn, 2) / 10.0
                    log("%s %s mix %d x [%d, %d] variant %d (%s) j_chunk %d: %.3f ms per pass" % (
                        kernel, precision, S, lo_n, hi_n, var, descs[var], jc, t))
                    if best is None or t < best[0]:
                        best = (t, var, jc)
            results.append((kernel, nmax, best, descs[best[1]]))
            nb.set_tile_table([])
    entries = []
    for kernel in ("force_batched", "adjoint_batched"):
        rows = sorted([(nm, bst, d) for k, nm, bst, d in results if k == kernel])
        sizes = [nm for nm, _, _ in rows]
        for k, (nm, bst, d) in enumerate(rows):
            lo, hi = _bounds(sizes, k)
            entries.append(dict(kernel=kernel, precision=precision, n_min=lo, n_max=hi, variant=bst[1],
                                desc=d, j_split=bst[2], tuned_n=nm, ms=bst[0]))
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="FP32-compensated force buckets only")
    ap.add_argument("--precisions", default=None, help="comma list (default: all)")
    ap.add_argument("--kernels", default="force,adjoint,batched,lj_force",
                    help="comma list of force, adjoint, batched, lj_force")
    ap.add_argument("--merge", default=None,
                    help="existing table: keep its entries for every (kernel, precision, bucket) not re-tuned")
    ap.add_argument("--force-buckets", default=None, help="comma list of particle counts for the force buckets")
    args = ap.parse_args()
    import torch
    import paper_2511_02655_amd as nb
    nb.lib()
    nb.set_tile_table([])

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    entries = []
    precs = ["fp32c"] if args.quick else ["fp32c", "fp32", "fp32ds", "fp64"]
    if args.precisions:
        precs = args.precisions.split(",")
    kernels = ["force"] if args.quick else args.kernels.split(",")
    fb = [int(x) for x in args.force_buckets.split(",")] if args.force_buckets else FORCE_BUCKETS
    if "force" in kernels:
        for p in precs:
            entries += tune_force(nb, torch, p, fb, log)
    if "adjoint" in kernels:
        for p in precs:
            if p != "fp32ds":  # adjoint passes of the double-float mode run the compensated kernels
                entries += tune_adjoint(nb, torch, p, ADJ_BUCKETS, log)
    if "batched" in kernels:
        for p in precs:
            entries += tune_batched(nb, torch, p, log)
    if "lj_force" in kernels:
        lb = [int(x) for x in args.force_buckets.split(",")] if args.force_buckets else LJ_BUCKETS
        for p in precs:
            entries += tune_force(nb, torch, p, lb, log, law="lj")
    if args.merge and os.path.exists(args.merge):
        with open(args.merge) as f:
            old = json.load(f).get("entries", [])
        tuned = {(e["kernel"], e["precision"], e.get("tuned_n")) for e in entries}
        entries = [e for e in old if (e["kernel"], e["precision"], e.get("tuned_n")) not in tuned] + entries
        entries.sort(key=lambda e: (e["kernel"], e["precision"], e["n_min"]))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    table = {"arch": arch, "tuned_in_s": time.time() - t0, "entries": entries}
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", arch + ".json")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    log("wrote %s (%d entries, %.0f s)" % (out, len(entries), time.time() - t0))


if __name__ == "__main__":
    sys.exit(main())
