"""Benchmark of the all-pairs N-body hot path on one MI355X.

One timed step = the Plummer N = 1,048,576 workload (eps = 1e-3): one force pass with
the fused potential, the energy/momentum reduction at t = 0, 10 kick-drift-kick steps
of dt = 5e-4 (one force pass each, through nbody_step; the last one also emits the
potential), and the energy/momentum reduction at the end: 11 all-pairs evaluations,
FP32 pair math with compensated accumulation and adaptive separations (the particles are
Morton-sorted on the device at every pass and sub-block pairs closer than X_max / 256 take
double-float separations: max force error <= 1e-5 on every particle), FP64 state and
reductions. Inputs are resident on the GPU before the timed region.

Printed: ONE JSON line with the throughput in pair interactions/s, the roofline of the
dominant kernel (the FP32 force pass, 20 flop per interaction against the 157.3
TFLOP/s FP32 vector peak), the force error of this run against the FP64 GPU path and
the CPU oracle, the adjoint and batched legs, and the CPU oracle timed on a bounded
sample of the same workload.

Also reported (not part of the timed step): the paper's own workload, a Lennard-Jones
gas of 10 000 particles in a box with reflective walls run for 2500 KDK steps, with and
without the per-step energy reduction, in FP64 and FP32 (the "lj10k" leg); and the same
force pass on the round schedule, whose workspace is linear in N, beside the default slot
schedule (the "round_schedule" leg: time, workspace, max error on every particle); and one
GPU's share of the paper's ring decomposition at its real shape, 1/8 of the particles against
all (the "ring_share" leg).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
       python bench.py --lj-only     (only the Lennard-Jones leg, printed as one JSON line)
       python bench.py --adjoint-1m-only  (only the adjoint pass at the headline size)
       python bench.py --round-schedule-only  (only the headline pass on the round schedule)
       python bench.py --merger-only  (only the two-sphere merger forward and backward, no oracle)
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12          # MI355X FP32 vector, FLOP/s
FLOP_PER_INTERACTION = 20.0   # forward pair-interaction convention
LJ_FLOP_PER_INTERACTION = 22.0  # Lennard-Jones pair: 3 sub, 3 FMA (r^2), rcp, 2 mul (u^3), FMA, 2 mul, 3 FMA
# adjoint interaction (one ordered pair's share of the force VJP): 3 sub, 3 FMA (r^2), rsq
# (2, as in the forward convention), 2 mul (r^-2, r^-3), 2 mul (3 r^-5), two dot products
# d.l_j and d.l_k (5 each), 4 FMA (r^-3 l_j, m_j r^-3), w = m_k (d.l_j) - m_j (d.l_k) (3), mul,
# 4 FMA (C, M)
ADJ_FLOP_PER_INTERACTION = 45.0
METRIC = "pair interactions/s (fwd & adjoint), % FP32 vector peak, at stated error"
KERNEL_SRC = os.path.join(ROOT, "paper_2511_02655_amd", "csrc", "nbody_kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_fp32a_plummer1m_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SYM_BEGIN = "// ----------------------------------------------------------------- symmetric force pass (FP32)"
SYM_END = "// ----------------------------------------------------------------- symmetric pass: per-particle reduction"


def kernel_hash():
    """Hash of the symmetric force kernel's source (lane rotation, tile mapping and
    force_sym_kernel: the kernel the stored counters describe)."""
    with open(KERNEL_SRC) as f:
        src = f.read()
    if SYM_BEGIN in src and SYM_END in src:
        src = src[src.index(SYM_BEGIN):src.index(SYM_END)]
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def stored_traffic(per_launch_n2):
    """HBM bytes per force launch from the stored rocprofv3 counter runs, or None when
    the kernel source has changed since they were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32a", choices=["fp32a", "fp32c", "fp32", "fp32ds", "fp64"])
    ap.add_argument("--n", type=int, default=1048576)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--lj-only", action="store_true")
    ap.add_argument("--adjoint-1m-only", action="store_true")
    ap.add_argument("--round-schedule-only", action="store_true")
    ap.add_argument("--merger-only", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the whole system on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2511_02655_amd as nb
    from paper_2511_02655_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    nb.lib()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.lj_only:
        print(json.dumps({"lj10k": lj_leg(nb, torch, np, inputs, dev)}), flush=True)
        return
    if args.merger_only:
        print(json.dumps({"adjoint": adjoint_leg(nb, torch, np, inputs, dev, with_oracle=False)}), flush=True)
        return

    W = inputs.WORKLOADS["plummer1m"]
    n, eps, dt, ksteps = args.n, W["eps"], W["dt"], W["steps"]
    prec = args.precision
    log("generating Plummer n=%d" % n)
    s = inputs.plummer(n, W["seed"])
    pos0 = torch.from_numpy(s.pos).to(dev)
    vel0 = torch.from_numpy(s.vel).to(dev)
    mass = torch.from_numpy(s.mass).to(dev)
    if args.round_schedule_only:
        leg = round_schedule_leg(nb, torch, np, pos0, mass, eps, prec, n, warm=1, reps=3)
        print(json.dumps({"round_schedule": leg}), flush=True)
        return
    if args.adjoint_1m_only:
        print(json.dumps({"adjoint_1m": adjoint_1m_leg(nb, torch, np, pos0, mass, s, eps, prec)}), flush=True)
        return
    pos, vel = pos0.clone(), vel0.clone()
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    evals_per_step = 1 + ksteps
    inter_per_step = evals_per_step * float(n) * float(n)

    pot_events = []   # force pass with the fused potential (2 per step)
    step_events = []  # KDK steps: kick/drift/stage + force pass + closing kick (10 per step)

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def one_step(timed):
        pos.copy_(pos0)
        vel.copy_(vel0)
        e0 = ev() if timed else None
        nb.forces(pos, mass, eps=eps, precision=prec, want_pot=True, out_acc=acc, out_pot=pot)
        if timed:
            pot_events.append((e0, ev()))
        em0 = nb.energy_momentum(pos, vel, mass, pot, eps=eps, precision=prec)
        for k in range(ksteps):
            last = k == ksteps - 1
            e0 = ev() if (timed and not last) else None
            # the last step's force pass also yields the potential for the closing energy reduction
            nb.step(pos, vel, mass, acc, dt, eps=eps, precision=prec, out_pot=pot if last else None)
            if timed and not last:
                step_events.append((e0, ev()))
        em1 = nb.energy_momentum(pos, vel, mass, pot, eps=eps, precision=prec)
        return em0, em1

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for k in range(args.steps):
        em0, em1 = one_step(True)
        torch.cuda.synchronize()
        log("  step %d done" % k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = inter_per_step * args.steps / elapsed
    force_ms = float(np.mean([a.elapsed_time(b) for a, b in step_events]))
    pot_ms = float(np.mean([a.elapsed_time(b) for a, b in pot_events]))
    achieved = FLOP_PER_INTERACTION * float(n) * float(n) / (force_ms * 1e-3)
    vid, _ = nb.tile_lookup("force", prec, n)
    kdesc = nb.tile_variants("force", prec)[vid]
    em0 = em0.cpu().numpy()[0]
    em1 = em1.cpu().numpy()[0]
    E0, E1 = em0[0] + em0[1], em1[0] + em1[1]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec != "fp64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "plummer1m: Plummer sphere N=%d (M=1, a=1, seed %d), eps=%g; per step 1 force pass with "
                        "potential + energy/momentum, %d KDK steps dt=%g (the last one also yields the potential), "
                        "energy/momentum at the end (%d all-pairs evaluations); %s pair math, FP64 state and reductions"
                        % (n, W["seed"], eps, ksteps, dt, evals_per_step, prec),
            "n": n, "eps": eps, "dt": dt, "kdk_steps": ksteps, "evaluations_per_step": evals_per_step,
            "precision": prec,
        },
        "pct_fp32_peak": 100.0 * FLOP_PER_INTERACTION * value / PEAK_FP32,
        "roofline": {
            "bound": "alu",
            "kernel": "%s force pass (%s, %s), no potential; timed per KDK step (kick/drift + %sforce + "
                      "closing kick, > 99%% force)" % ("symmetric" if "sym=" in kdesc else "one-sided", kdesc, prec,
                                                      "Morton sort and sorted staging + " if prec == "fp32a" else
                                                      "staging + "),
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": stored_traffic(n),
            "avg_launch_ms": force_ms,
            "avg_launch_ms_with_potential": pot_ms,
            "frac_with_potential": FLOP_PER_INTERACTION * float(n) * float(n) / (pot_ms * 1e-3) / PEAK_FP32,
            "flop_per_interaction": FLOP_PER_INTERACTION,
            "interactions_per_launch": float(n) * float(n),
        },
        "energy": {"E0": E0, "E_end": E1, "rel_drift": abs(E1 - E0) / abs(E0),
                   "P_end": [float(x) for x in em1[2:]]},
    }

    out["force_pass_reps"] = force_pass_reps(nb, torch, np, pos0, mass, eps, prec, n)
    if not args.no_extras:
        out["error"] = force_errors(nb, torch, np, pos0, mass, s, eps, prec)
        if prec != "fp64":
            out["round_schedule"] = round_schedule_leg(nb, torch, np, pos0, mass, eps, prec, n)
        out["ring_share"] = ring_share_leg(nb, torch, np, pos0, mass, eps, n)
        out["cube1k"] = cube1k_leg(nb, torch, np, inputs, dev)
        out["plummer64k"] = plummer64k_leg(nb, torch, np, inputs, dev)
        out["adjoint"] = adjoint_leg(nb, torch, np, inputs, dev)
        out["adjoint_1m"] = adjoint_1m_leg(nb, torch, np, pos0, mass, s, eps, prec)
        out["batched"] = batched_leg(nb, torch, np, inputs, dev)
        out["lj10k"] = lj_leg(nb, torch, np, inputs, dev)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(np, s, eps)
    print(json.dumps(out), flush=True)


def sample_sclk():
    """Current GPU engine clock in MHz from rocm-smi (None when it cannot be read, and
    under rocprofv3, which preloads its GPU-initialising library into every child process:
    rocm-smi's interpreter would then be started by exec from an initialised process)."""
    import re
    import subprocess
    if "ROCPROF_OUTPUT_PATH" in os.environ:
        return None
    try:
        r = subprocess.run(["rocm-smi", "-g", "--json"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                           text=True, timeout=20)
        cards = json.loads(r.stdout)
    except Exception:
        return None
    for card in cards.values():
        if not isinstance(card, dict):
            continue
        for key, val in card.items():
            m = re.search(r"\((\d+(?:\.\d+)?)\s*mhz\)", str(val), re.I)
            if "sclk" in key.lower() and m:
                return float(m.group(1))
    return None


def force_pass_reps(nb, torch, np, pos0, mass, eps, prec, n, warm=2, reps=10):
    """The headline force pass alone (staging, pair pass and per-particle reduction, no
    potential): `warm` untimed launches, then `reps` launches timed one by one with HIP
    events; median, min and max. The engine clock is sampled with rocm-smi while they run."""
    log("force pass: %d warm-up + %d timed launches" % (warm, reps))
    acc = torch.empty((3, n), dtype=torch.float64, device=pos0.device)
    for _ in range(warm):
        nb.forces(pos0, mass, eps=eps, precision=prec, out_acc=acc)
    torch.cuda.synchronize()
    evs = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nb.forces(pos0, mass, eps=eps, precision=prec, out_acc=acc)
        e1.record()
        evs.append((e0, e1))
    sclk = [c for c in (sample_sclk() for _ in range(3)) if c]  # the launches are still running
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in evs])
    med = float(np.median(ms))
    flops = FLOP_PER_INTERACTION * float(n) * float(n) / (med * 1e-3)
    out = {"median_ms": med, "min_ms": float(ms.min()), "max_ms": float(ms.max()), "reps": reps, "warmup": warm,
           "interactions_per_s": float(n) * float(n) / (med * 1e-3), "pct_fp32_peak": 100.0 * flops / PEAK_FP32,
           "sclk_mhz_samples": sclk}
    if sclk:
        # peak at the sampled clock: 256 CUs x 128 FMA lanes x 2 flop per clock
        peak_at_clk = 256 * 256 * float(np.median(sclk)) * 1e6
        out["pct_fp32_peak_at_sampled_sclk"] = 100.0 * flops / peak_at_clk
    return out


def round_schedule_leg(nb, torch, np, pos0, mass, eps, prec, n, warm=1, reps=5):
    """The headline force pass on the round schedule (NBODY_FLAG_SYM_ROUNDS: per-particle double
    accumulators, workspace linear in N) beside the default slot schedule: one step's workspace
    under each, the pass timed as in force_pass_reps, and its max relative error on every
    particle against the FP64 GPU path."""
    import ctypes
    log("round schedule: %d warm-up + %d timed launches" % (warm, reps))
    lib = nb.lib()

    def ws(flags):
        c = nb._Cfg(prec, 1.0, eps, None, flags, None)
        b = ctypes.c_size_t()
        rc = lib.nbody_workspace_size(ctypes.byref(c.cfg), n, 1, 0, ctypes.byref(b))
        return int(b.value) if rc == 0 else None

    F = nb.FLAG_SYM_ROUNDS
    acc = torch.empty((3, n), dtype=torch.float64, device=pos0.device)
    for _ in range(warm):
        nb.forces(pos0, mass, eps=eps, precision=prec, out_acc=acc, flags=F)
    torch.cuda.synchronize()
    evs = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nb.forces(pos0, mass, eps=eps, precision=prec, out_acc=acc, flags=F)
        e1.record()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in evs])
    med = float(np.median(ms))
    a64, _ = nb.forces(pos0, mass, eps=eps, precision="fp64")
    mag = torch.sqrt((a64 ** 2).sum(0))
    floor = 1e-6 * float(torch.sqrt((mag ** 2).mean()))
    e = torch.sqrt(((acc - a64) ** 2).sum(0)) / torch.clamp(mag, min=floor)
    return {"median_ms": med, "min_ms": float(ms.min()), "max_ms": float(ms.max()), "reps": reps,
            "pct_fp32_peak": 100.0 * FLOP_PER_INTERACTION * float(n) * float(n) / (med * 1e-3) / PEAK_FP32,
            "max_e_all_particles": float(e.max()), "workspace_bytes_step": ws(F),
            "workspace_bytes_step_slot_schedule": ws(0)}


def ring_share_leg(nb, torch, np, pos0, mass, eps, n, P=8, reps=3):
    """One GPU's share of the paper's ring decomposition at its real shape: share 0 of P (its
    n / P particles against all n, the j-range in P blocks) through nbody_forces_shard, timed
    with HIP events, in the compensated and the double-float mode."""
    log("ring share: 0 of %d" % P)
    out = {"P": P, "share": 0}
    acc = torch.zeros((3, n), dtype=torch.float64, device=pos0.device)
    for prec in ("fp32c", "fp32ds"):
        _, _, (i0, i1) = nb.forces_shard(pos0, mass, P, 0, eps=eps, precision=prec, out_acc=acc)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nb.forces_shard(pos0, mass, P, 0, eps=eps, precision=prec, out_acc=acc)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        inter = float(i1 - i0) * float(n)
        out[prec] = {"rows": [i0, i1], "median_ms": med, "interactions_per_s": inter / (med * 1e-3),
                     "pct_fp32_peak": 100.0 * FLOP_PER_INTERACTION * inter / (med * 1e-3) / PEAK_FP32}
    return out


def adjoint_1m_leg(nb, torch, np, pos0, mass, s, eps, prec):
    """The adjoint pair pass at the headline size: a one-step backward (two adjoint passes
    and one recomputed force pass, with their staging and reductions) timed with HIP events,
    less one force pass timed the same way, halved."""
    log("adjoint 1M leg")
    dt = 5e-4
    pos, vel = pos0.clone(), torch.from_numpy(s.vel).to(pos0.device)
    acc, _ = nb.forces(pos, mass, eps=eps, precision=prec)
    ckpt, _ = nb.rollout(pos, vel, mass, acc, dt, 1, ckpt_every=1, eps=eps, precision=prec)
    gx = torch.ones_like(pos)
    gv = torch.zeros_like(pos)
    nb.rollout_backward(mass, ckpt, gx, gv, dt, 1, 1, eps=eps, precision=prec)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    nb.forces(pos0, mass, eps=eps, precision=prec, out_acc=acc)
    ev[1].record()
    nb.rollout_backward(mass, ckpt, gx, gv, dt, 1, 1, eps=eps, precision=prec)
    ev[2].record()
    torch.cuda.synchronize()
    f_ms, b_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    adj_ms = 0.5 * (b_ms - f_ms)
    n2 = float(s.n) ** 2
    vid, _ = nb.tile_lookup("adjoint", prec, s.n)
    return {"workload": "plummer1m state, one-step backward (dt=%g) with a unit position cotangent, %s" % (dt, prec),
            "kernel": nb.tile_variants("adjoint", prec)[vid],
            "backward_1step_ms": b_ms, "force_pass_ms": f_ms, "adjoint_pass_ms": adj_ms,
            "adjoint_interactions_per_s": n2 / (adj_ms * 1e-3),
            "flop_per_adjoint_interaction": ADJ_FLOP_PER_INTERACTION,
            "pct_fp32_peak": 100.0 * ADJ_FLOP_PER_INTERACTION * n2 / (adj_ms * 1e-3) / PEAK_FP32,
            "adjoint_over_forward_time": adj_ms / f_ms}


def force_errors(nb, torch, np, pos0, mass, s, eps, prec):
    """Force error of every pair-math mode: each mode's force pass (without the potential)
    timed once and compared on every particle with the FP64 GPU path; every mode's 64 worst
    particles and a random sample also against the FP64 CPU oracle."""
    log("error leg")
    a64, p64 = nb.forces(pos0, mass, eps=eps, precision="fp64", want_pot=True)
    m = torch.sqrt((a64 ** 2).sum(0))
    rms = torch.sqrt((m ** 2).mean())
    n2 = float(s.n) ** 2
    modes = {}
    results = {}
    worst = set()
    for mode in ("fp32", "fp32c", "fp32ds", "fp32a", "fp64"):
        a32, p32 = nb.forces(pos0, mass, eps=eps, precision=mode, want_pot=True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        nb.forces(pos0, mass, eps=eps, precision=mode, want_pot=False, out_acc=a32)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        d = torch.sqrt(((a32 - a64) ** 2).sum(0))
        e = d / torch.clamp(m, min=1e-6 * rms.item())
        modes[mode] = {"force_ms": ms, "interactions_per_s": n2 / (ms * 1e-3),
                       "pct_fp32_peak": 100.0 * FLOP_PER_INTERACTION * n2 / (ms * 1e-3) / PEAK_FP32,
                       "max_e": float(e.max()), "p999_e": float(torch.quantile(e.float(), 0.999)),
                       "max_abs_over_rms": float((d / rms).max()),
                       "phi_max_rel": float((torch.abs(p32 - p64) / torch.abs(p64)).max())}
        results[mode] = a32.cpu().numpy()
        if mode != "fp64":
            worst.update(torch.argsort(e)[-64:].cpu().numpy().tolist())
    return {
        "vs_fp64_gpu_all": modes[prec] if prec in modes else None,
        "modes_vs_fp64_gpu_all": modes,
        "vs_oracle_worst_and_sample": oracle_check(np, s, eps, {k: v for k, v in results.items()}, worst),
        "metric": "e_i = |a_i - a_i^ref| / max(|a_i^ref|, 1e-6 rms|a^ref|), all N particles unless noted",
    }


def oracle_check(np, s, eps, results, worst, n_random=64):
    """Each mode's worst particles (from the all-particle comparison with the FP64 GPU path)
    plus a random sample and both ends against the CPU oracle: max e_i, and the largest ratio
    of |da_i| to the per-particle rounding bound B_i of the FP32 pair paths."""
    import oracle
    from oracle import bounds
    g = np.random.Generator(np.random.PCG64(7))
    idx = np.unique(np.concatenate([np.asarray(sorted(worst), dtype=np.int64), g.choice(s.n, n_random, replace=False),
                                    [0, s.n - 1]]))
    ar, _ = oracle.forces_sample(s.pos, s.mass, idx, eps=eps)
    mm = np.sqrt((ar ** 2).sum(0))
    floor = 1e-6 * math.sqrt(np.mean(mm ** 2))
    out = {"particles": int(idx.size)}
    for name, a_host in results.items():
        a = a_host[:, idx]
        dd = np.sqrt(((a - ar) ** 2).sum(0))
        r = {"max_e": float(np.max(dd / np.maximum(mm, floor)))}
        if name != "fp64":
            B = bounds.fp32_force_bound(s.pos, s.mass, eps, accumulate_plain=(name == "fp32"),
                                        exact_coords=(name == "fp32ds"), adaptive=(name == "fp32a"), idx=idx)
            r["max_err_over_bound"] = float(np.max(dd / B))
        out[name] = r
    return out


def cube1k_leg(nb, torch, np, inputs, dev):
    """Uniform cube N = 1024, eps = 1e-2, 10 KDK steps dt = 1e-3 in FP64 on the GPU against
    the CPU oracle: forces, final state, energy and momentum."""
    import oracle
    log("cube1k leg")
    W = inputs.WORKLOADS["cube1k"]
    s = inputs.make("cube1k")
    pos = torch.from_numpy(s.pos).to(dev)
    vel = torch.from_numpy(s.vel).to(dev)
    m = torch.from_numpy(s.mass).to(dev)
    acc, pot = nb.forces(pos, m, eps=W["eps"], precision="fp64", want_pot=True)
    a_ref, p_ref = oracle.forces(s.pos, s.mass, eps=W["eps"])
    a = acc.cpu().numpy()
    rms = math.sqrt(np.mean(np.sum(a_ref ** 2, axis=0)))
    e = np.sqrt(np.sum((a - a_ref) ** 2, axis=0)) / np.maximum(np.sqrt(np.sum(a_ref ** 2, axis=0)), 1e-6 * rms)
    _, trace = nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], energy_trace=True, eps=W["eps"], precision="fp64")
    xr, vr, _, er = oracle.kdk(s.pos, s.vel, s.mass, W["dt"], W["steps"], eps=W["eps"], want_energy=True)
    tr = trace.cpu().numpy()[:, 0, :]
    E, Er = tr[:, 0] + tr[:, 1], er[:, 0] + er[:, 1]
    return {"workload": "cube1k: uniform cube N=1024, eps=1e-2, 10 KDK steps dt=1e-3, FP64 GPU vs CPU oracle",
            "force_max_e": float(e.max()),
            "phi_max_rel": float(np.max(np.abs(pot.cpu().numpy() - p_ref) / np.abs(p_ref))),
            "final_x_max_abs_diff": float(np.max(np.abs(pos.cpu().numpy() - xr))),
            "final_v_max_abs_diff": float(np.max(np.abs(vel.cpu().numpy() - vr))),
            "energy_max_rel_diff": float(np.max(np.abs(E - Er) / abs(Er[0]))),
            "momentum_max_abs_diff": float(np.max(np.abs(tr[:, 2:] - er[:, 2:]))),
            "energy_drift_gpu": float(np.max(np.abs(E - E[0])) / abs(E[0]))}


def plummer64k_leg(nb, torch, np, inputs, dev):
    """Plummer sphere N = 65536, eps = 1e-2, 100 KDK steps dt = 1e-3 in every pair-math mode
    with an energy trace: energy drift, final-state error against the FP64 GPU path, time;
    the initial energy also against the CPU oracle."""
    import oracle
    log("plummer64k leg")
    W = inputs.WORKLOADS["plummer64k"]
    s = inputs.make("plummer64k")
    x0 = torch.from_numpy(s.pos).to(dev)
    v0 = torch.from_numpy(s.vel).to(dev)
    m = torch.from_numpy(s.mass).to(dev)
    res = {"workload": "plummer64k: Plummer N=65536, eps=1e-2, 100 KDK steps dt=1e-3"}
    # forces at t = 0: every particle of every FP32 mode against the FP64 GPU path, and the
    # worst particles of each against the oracle
    a64, _ = nb.forces(x0, m, eps=W["eps"], precision="fp64")
    mag = torch.sqrt((a64 ** 2).sum(0))
    floor = 1e-6 * float(torch.sqrt((mag ** 2).mean()))
    results, worst, ferr = {"fp64": a64.cpu().numpy()}, set(), {}
    for mode in ("fp32c", "fp32ds", "fp32", "fp32a"):
        a, _ = nb.forces(x0, m, eps=W["eps"], precision=mode)
        e = torch.sqrt(((a - a64) ** 2).sum(0)) / torch.clamp(mag, min=floor)
        ferr[mode] = {"max_e": float(e.max()), "p999_e": float(torch.quantile(e.float(), 0.999))}
        results[mode] = a.cpu().numpy()
        worst.update(torch.argsort(e)[-64:].cpu().numpy().tolist())
    res["force_error_vs_fp64_gpu_all"] = ferr
    res["force_error_vs_oracle_worst_and_sample"] = oracle_check(np, s, W["eps"], results, worst)
    finals = {}
    for mode in ("fp64", "fp32c", "fp32ds", "fp32", "fp32a"):
        pos, vel = x0.clone(), v0.clone()
        acc, _ = nb.forces(pos, m, eps=W["eps"], precision=mode)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, trace = nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], energy_trace=True, eps=W["eps"],
                              precision=mode)
        e1.record()
        torch.cuda.synchronize()
        tr = trace.cpu().numpy()[:, 0, :]
        E = tr[:, 0] + tr[:, 1]
        finals[mode] = (pos, vel, E)
        res[mode] = {"rollout_ms": e0.elapsed_time(e1),
                     "interactions_per_s_with_potential": (W["steps"] + 1) * 65536.0 ** 2 / (e0.elapsed_time(e1) * 1e-3),
                     "energy_drift": float(np.max(np.abs(E - E[0])) / abs(E[0])),
                     "momentum_drift": float(np.max(np.abs(tr[:, 2:] - tr[0, 2:])))}
    x64, v64, E64 = finals["fp64"]
    rmsx = float(torch.sqrt((x64 ** 2).mean()))
    for mode in ("fp32c", "fp32ds", "fp32", "fp32a"):
        x, v, E = finals[mode]
        res[mode]["final_x_max_abs_diff_over_rms_vs_fp64_gpu"] = float(torch.max(torch.abs(x - x64))) / rmsx
        res[mode]["energy_trace_max_rel_diff_vs_fp64_gpu"] = float(np.max(np.abs(E - E64) / abs(E64[0])))
    em = oracle.energy_momentum(s.pos, s.vel, s.mass, eps=W["eps"])
    res["fp64"]["E0_rel_diff_vs_oracle"] = float(abs(E64[0] - (em[0] + em[1])) / abs(em[0] + em[1]))
    return res


def adjoint_leg(nb, torch, np, inputs, dev, with_oracle=True):
    """Two-sphere merger N = 2 x 8192, eps = 1e-2, 200 KDK steps dt = 1e-3, checkpoints
    every 20; loss = mean squared distance of the final positions to a Gaussian target
    set; gradient w.r.t. initial positions, velocities and masses (FP32 compensated)."""
    log("adjoint leg")
    W = inputs.WORKLOADS["merger2x8k"]
    s = inputs.make("merger2x8k")
    y = torch.from_numpy(inputs.gaussian_targets(s.n, W["target_seed"])).to(dev)
    x0 = torch.from_numpy(s.pos).to(dev)
    v0 = torch.from_numpy(s.vel).to(dev)
    m = torch.from_numpy(s.mass).to(dev)
    prec = "fp32c"

    # forward + backward timing (backward includes the recomputation between checkpoints)
    ckpt_every = W["ckpt"]
    pos, vel = x0.clone(), v0.clone()
    acc, _ = nb.forces(pos, m, eps=W["eps"], precision=prec)
    ckpt, _ = nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], ckpt_every=ckpt_every, eps=W["eps"], precision=prec)
    gxK = (2.0 / s.n) * (pos - y)
    gvK = torch.zeros_like(gxK)
    nb.rollout_backward(m, ckpt, gxK, gvK, W["dt"], W["steps"], ckpt_every, eps=W["eps"], precision=prec)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    reps = 3
    e0.record()
    for _ in range(reps):
        pos.copy_(x0)
        vel.copy_(v0)
        nb.forces(pos, m, eps=W["eps"], precision=prec, out_acc=acc)
        nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], ckpt_every=ckpt_every, eps=W["eps"], precision=prec,
                   ckpt=ckpt)
    e1.record()
    for _ in range(reps):
        g32 = nb.rollout_backward(m, ckpt, gxK, gvK, W["dt"], W["steps"], ckpt_every, eps=W["eps"], precision=prec)
    e2.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    bwd_ms = e1.elapsed_time(e2) / reps
    n2 = float(s.n) ** 2
    adj_passes = W["steps"] + 1
    # FP64 GPU reference gradient for the error statement
    pos64, vel64 = x0.clone(), v0.clone()
    acc64, _ = nb.forces(pos64, m, eps=W["eps"], precision="fp64")
    ck64, _ = nb.rollout(pos64, vel64, m, acc64, W["dt"], W["steps"], ckpt_every=ckpt_every, eps=W["eps"],
                         precision="fp64")
    gxK64 = (2.0 / s.n) * (pos64 - y)
    g64 = nb.rollout_backward(m, ck64, gxK64, torch.zeros_like(gxK64), W["dt"], W["steps"], ckpt_every,
                              eps=W["eps"], precision="fp64")
    rel = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(g32, g64)]

    # checkpoint-free backward: the trajectory rebuilt by stepping back from the final state
    pos.copy_(x0)
    vel.copy_(v0)
    nb.forces(pos, m, eps=W["eps"], precision=prec, out_acc=acc)
    nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], eps=W["eps"], precision=prec)
    nb.rollout_backward_reversible(m, pos, vel, gxK, gvK, W["dt"], W["steps"], eps=W["eps"], precision=prec)
    torch.cuda.synchronize()
    e3, e4 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e3.record()
    for _ in range(reps):
        grev = nb.rollout_backward_reversible(m, pos, vel, gxK, gvK, W["dt"], W["steps"], eps=W["eps"],
                                              precision=prec)
    e4.record()
    torch.cuda.synchronize()
    rev_ms = e3.elapsed_time(e4) / reps
    rel_rev = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(grev, g32)]

    # FP64 finite differences of the loss along random directions (central, h relative to the group scale)
    def loss64(xa, va, ma):
        p, v = xa.clone(), va.clone()
        a, _ = nb.forces(p, ma, eps=W["eps"], precision="fp64")
        nb.rollout(p, v, ma, a, W["dt"], W["steps"], eps=W["eps"], precision="fp64")
        return float(((p - y) ** 2).sum()) / s.n

    gen = torch.Generator(device="cpu").manual_seed(9)
    fd = {}
    for k, (name, scale) in enumerate((("x0", 1.0), ("v0", 0.3), ("m", float(m.mean())))):
        base = (x0, v0, m)[k]
        d = torch.randn(base.shape, generator=gen, dtype=torch.float64).to(dev)
        h = 1e-6 * scale
        args_p = [x0, v0, m]
        args_m = [x0, v0, m]
        args_p[k] = base + h * d
        args_m[k] = base - h * d
        fdv = (loss64(*args_p) - loss64(*args_m)) / (2 * h)
        fd[name] = {"fd": fdv, "adjoint_fp32c": float((g32[k] * d).sum()), "adjoint_fp64": float((g64[k] * d).sum()),
                    "rel_err_fp32c": abs(float((g32[k] * d).sum()) - fdv) / abs(fdv),
                    "rel_err_fp64": abs(float((g64[k] * d).sum()) - fdv) / abs(fdv)}
    # the CPU oracle's discrete adjoint at the full configuration (its own FP64 forward
    # trajectory and loss seed): rel-L2 and per particle
    out = {
        "workload": "merger2x8k: two Plummer spheres N=2x8192, eps=1e-2, 200 KDK steps dt=1e-3, ckpt every 20, "
                    "MSD loss to Gaussian targets; FP32 compensated",
        "forward_ms": fwd_ms,
        "backward_ms": bwd_ms,
        "adjoint_passes": adj_passes,
        "recompute_force_passes": W["steps"],
        "adjoint_interactions_per_s_incl_recompute": adj_passes * n2 / (bwd_ms * 1e-3),
        "forward_interactions_per_s": (W["steps"] + 1) * n2 / (fwd_ms * 1e-3),
        "grad_rel_l2_vs_fp64_gpu": {"x0": rel[0], "v0": rel[1], "m": rel[2]},
        "reversible_backward_ms": rev_ms,
        "reversible_grad_rel_l2_vs_checkpointed": {"x0": rel_rev[0], "v0": rel_rev[1], "m": rel_rev[2]},
        "checkpoint_bytes": int(ckpt.numel() * 8),
        "directional_vs_fp64_finite_differences": fd,
    }
    if not with_oracle:
        return out
    import oracle
    log("adjoint leg: oracle gradient (full configuration)")
    t0 = time.perf_counter()
    xr, _, _, _ = oracle.kdk(s.pos, s.vel, s.mass, W["dt"], W["steps"], eps=W["eps"])
    _, gxr = oracle.loss_msd(xr, inputs.gaussian_targets(s.n, W["target_seed"]))
    ref = oracle.rollout_adjoint(s.pos, s.vel, s.mass, W["dt"], W["steps"], gxr, np.zeros_like(gxr), eps=W["eps"])
    out["oracle_seconds"] = time.perf_counter() - t0
    out["oracle_threads"] = oracle.num_threads()
    out["grad_vs_oracle"] = {
        pname: {k: grad_errors(np, t.cpu().numpy(), r) for k, t, r in zip(("x0", "v0", "m"), gg, ref)}
        for pname, gg in (("fp32c", g32), ("fp64", g64))}
    return out


def grad_errors(np, a, b):
    """rel-L2 of a against b and the per-particle error max_k |a_k - b_k| / max(|b_k|, f rms|b|)
    (columns of (3, n) arrays are vectors) for the floors f = 1e-6 and 1e-3."""
    d = np.sqrt(((a - b) ** 2).sum(0)) if b.ndim == 2 else np.abs(a - b)
    mb = np.sqrt((b ** 2).sum(0)) if b.ndim == 2 else np.abs(b)
    rms = math.sqrt(float(np.mean(mb ** 2)))
    return {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "per_particle_floor_1e-6": float(np.max(d / np.maximum(mb, 1e-6 * rms))),
            "per_particle_floor_1e-3": float(np.max(d / np.maximum(mb, 1e-3 * rms)))}


def batched_leg(nb, torch, np, inputs, dev):
    """512 independent systems, N per system log-uniform in [64, 8192], cube or Plummer;
    eps = 1e-2, dt = 1e-3, 50 KDK steps, FP32 compensated forward + adjoint: one
    launch per batched pass against looping the single-system kernels."""
    log("batched leg")
    W = inputs.WORKLOADS["batch512"]
    b = inputs.make("batch512")
    off = b.offsets
    sizes = np.diff(off)
    sum_n2 = float(np.sum(sizes.astype(np.float64) ** 2))
    x0 = torch.from_numpy(b.pos).to(dev)
    v0 = torch.from_numpy(b.vel).to(dev)
    m = torch.from_numpy(b.mass).to(dev)
    res = {"workload": "batch512: 512 systems, N_s log-uniform [64, 8192] (sum N = %d, sum N^2 = %.3e), eps=1e-2, "
                       "50 KDK steps dt=1e-3, FP32 compensated" % (int(off[-1]), sum_n2)}
    for name, flags in (("one_launch", 0), ("looped", nb.FLAG_LOOP_SYSTEMS)):
        pos, vel = x0.clone(), v0.clone()
        acc, _ = nb.forces(pos, m, eps=W["eps"], precision="fp32c", offsets=off, flags=flags)
        ckpt, _ = nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], ckpt_every=10, eps=W["eps"], precision="fp32c",
                             offsets=off, flags=flags)
        gx = torch.ones_like(pos)
        gv = torch.zeros_like(pos)
        nb.rollout_backward(m, ckpt, gx, gv, W["dt"], W["steps"], 10, eps=W["eps"], precision="fp32c", offsets=off,
                            flags=flags)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        pos.copy_(x0)
        vel.copy_(v0)
        nb.forces(pos, m, eps=W["eps"], precision="fp32c", offsets=off, flags=flags, out_acc=acc)
        nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], ckpt_every=10, eps=W["eps"], precision="fp32c",
                   offsets=off, flags=flags, ckpt=ckpt)
        e1.record()
        g = nb.rollout_backward(m, ckpt, gx, gv, W["dt"], W["steps"], 10, eps=W["eps"], precision="fp32c",
                                offsets=off, flags=flags)
        e2.record()
        torch.cuda.synchronize()
        f_ms = e0.elapsed_time(e1)
        b_ms = e1.elapsed_time(e2)
        res[name] = {"forward_ms": f_ms, "backward_ms": b_ms,
                     "forward_interactions_per_s": (W["steps"] + 1) * sum_n2 / (f_ms * 1e-3),
                     "adjoint_interactions_per_s_incl_recompute": (W["steps"] + 1) * sum_n2 / (b_ms * 1e-3)}
        res[name + "_final_pos"] = pos
    d = float(torch.max(torch.abs(res["one_launch_final_pos"] - res["looped_final_pos"])))
    del res["one_launch_final_pos"], res["looped_final_pos"]
    res["max_abs_pos_diff_one_launch_vs_looped"] = d
    res["speedup_forward"] = res["looped"]["forward_ms"] / res["one_launch"]["forward_ms"]
    res["speedup_backward"] = res["looped"]["backward_ms"] / res["one_launch"]["backward_ms"]
    # forward without checkpoints: one launch per pass against every step in one launch,
    # on this mix and on a mix of tiny systems (4096 systems of 16-256 particles)
    res["rollout_no_checkpoints"] = whole_rollout_compare(nb, torch, np, b, W, sum_n2)
    tiny = inputs.batched_mix(4096, 7, nmin=16, nmax=256)
    tiny_n2 = float(np.sum(np.diff(tiny.offsets).astype(np.float64) ** 2))
    res["rollout_no_checkpoints_tiny"] = whole_rollout_compare(nb, torch, np, tiny, W, tiny_n2)
    res["rollout_no_checkpoints_tiny"]["workload"] = ("4096 systems, N_s log-uniform [16, 256] (sum N^2 = %.3e), "
                                                      "50 KDK steps, FP32 compensated" % tiny_n2)
    return res


def whole_rollout_compare(nb, torch, np, b, W, sum_n2):
    """50-step forward of batch b without checkpoints: one launch per pass against every step
    in one launch (NBODY_FLAG_WHOLE_ROLLOUT); median of 3, and the final states compared."""
    off = b.offsets
    x0 = torch.from_numpy(b.pos).cuda()
    v0 = torch.from_numpy(b.vel).cuda()
    m = torch.from_numpy(b.mass).cuda()
    wr = {}
    for name, flags in (("per_pass", nb.FLAG_PER_PASS), ("whole_rollout", nb.FLAG_WHOLE_ROLLOUT)):
        pos, vel = x0.clone(), v0.clone()
        acc, _ = nb.forces(pos, m, eps=W["eps"], precision="fp32c", offsets=off)
        nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], eps=W["eps"], precision="fp32c", offsets=off, flags=flags)
        ts = []
        for _ in range(3):
            pos.copy_(x0)
            vel.copy_(v0)
            nb.forces(pos, m, eps=W["eps"], precision="fp32c", offsets=off, out_acc=acc)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nb.rollout(pos, vel, m, acc, W["dt"], W["steps"], eps=W["eps"], precision="fp32c", offsets=off,
                       flags=flags)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        wr[name] = {"ms": ms, "interactions_per_s": W["steps"] * sum_n2 / (ms * 1e-3), "final_pos": pos.clone()}
    wr["bitwise_equal"] = bool(torch.equal(wr["per_pass"].pop("final_pos"), wr["whole_rollout"].pop("final_pos")))
    wr["speedup"] = wr["per_pass"]["ms"] / wr["whole_rollout"]["ms"]
    return wr


def lj_leg(nb, torch, np, inputs, dev):
    """The paper's experiment size with its own pair law: a Lennard-Jones gas of N = 10 000
    (sigma = epsilon = m = 1, simple cubic lattice of spacing 1.5 sigma, kT = 1) in a box
    with reflective walls, 2500 KDK steps of dt = 0.002, with the energy reduction after
    every step ("with reduction") and without it. Also: the force pass alone (roofline) and
    the first 20 steps against the CPU oracle."""
    import oracle
    log("lj10k leg")
    W = inputs.WORKLOADS["lj10k"]
    s, box = inputs.make("lj10k")
    n, dt, steps = s.n, W["dt"], W["steps"]
    bx = (box.lo, box.hi)
    x0 = torch.from_numpy(s.pos).to(dev)
    v0 = torch.from_numpy(s.vel).to(dev)
    m = torch.from_numpy(s.mass).to(dev)
    res = {"workload": "lj10k: Lennard-Jones gas N=%d (sigma=eps=m=1, sc lattice spacing 1.5, kT=1, seed %d) in a "
                       "reflective box of edge %.1f; %d KDK steps dt=%g, no cutoff" % (n, W["seed"], box.hi[0], steps, dt),
           "flop_per_interaction": LJ_FLOP_PER_INTERACTION}
    for prec in ("fp64", "fp32", "fp32c"):
        r = {}
        pos, vel = x0.clone(), v0.clone()
        acc, _ = nb.lj_forces(pos, m, precision=prec)
        nb.lj_rollout(pos, vel, m, acc, dt, 20, box=bx, precision=prec)  # warm-up
        for label, trace in (("no_reduction", False), ("with_reduction", True)):
            pos.copy_(x0)
            vel.copy_(v0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nb.lj_forces(pos, m, precision=prec, out_acc=acc)
            tr = nb.lj_rollout(pos, vel, m, acc, dt, steps, box=bx, energy_trace=trace, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            r[label] = {"seconds": ms * 1e-3, "ms_per_step": ms / steps,
                        "interactions_per_s": (steps + 1) * float(n) * n / (ms * 1e-3)}
            if trace:
                t = tr.cpu().numpy()[:, 0, :]
                E = t[:, 0] + t[:, 1]
                r[label]["energy_rel_drift_max"] = float(np.max(np.abs(E - E[0])) / abs(t[0, 0]))
                r[label]["in_box"] = bool(torch.all(pos >= torch.from_numpy(box.lo).to(dev)[:, None]).item()
                                          and torch.all(pos <= torch.from_numpy(box.hi).to(dev)[:, None]).item())
        # the force pass alone: 200 back-to-back launches on the current stream
        reps = 200
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        for want_pot in (False, True):
            nb.lj_forces(x0, m, precision=prec, out_acc=acc, want_pot=want_pot, out_pot=pot if want_pot else None)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                nb.lj_forces(x0, m, precision=prec, out_acc=acc, want_pot=want_pot, out_pot=pot if want_pot else None)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            flops = LJ_FLOP_PER_INTERACTION * float(n) * n / (ms * 1e-3)
            r["force_call_us" + ("_with_potential" if want_pot else "")] = ms * 1e3
            r["force_frac_fp32_peak" + ("_with_potential" if want_pot else "")] = flops / PEAK_FP32
        vid, jsplit = nb.tile_lookup("lj_force", prec, n)
        r["tile"] = "%s, j_split=%d" % (nb.tile_variants("lj_force", prec)[vid], jsplit)
        res[prec] = r
    # parity: 20 steps against the oracle (FP64 and compensated FP32)
    k = 20
    t0 = time.perf_counter()
    pr, vr, _ = oracle.lj_kdk(s.pos, s.vel, s.mass, dt, k, box=bx)
    res["oracle_20_steps_s"] = time.perf_counter() - t0
    for prec in ("fp64", "fp32c"):
        pos, vel = x0.clone(), v0.clone()
        acc, _ = nb.lj_forces(pos, m, precision=prec)
        nb.lj_rollout(pos, vel, m, acc, dt, k, box=bx, precision=prec)
        res[prec]["max_abs_pos_err_vs_oracle_20_steps"] = float(np.max(np.abs(pos.cpu().numpy() - pr)))
        res[prec]["max_abs_vel_err_vs_oracle_20_steps"] = float(np.max(np.abs(vel.cpu().numpy() - vr)))
    res["paper_context"] = ("the paper reports 19.02 s (best, with the energy reduction) and 8.96 s (best, "
                            "without) for this size on four A100 GPUs of one node; its box, lattice and dt are "
                            "not stated, so the workloads match in N and steps only")
    return res


def cpu_baseline(np, s, eps, target_s=12.0):
    """The CPU oracle (FP64, OpenMP over particles) on a bounded sample of the same
    workload: k particles against all N, k scaled to about target_s seconds."""
    import oracle
    log("cpu baseline")
    threads = oracle.num_threads()
    g = np.random.Generator(np.random.PCG64(11))
    k = 64
    idx = np.sort(g.choice(s.n, k, replace=False))
    t0 = time.perf_counter()
    oracle.forces_sample(s.pos, s.mass, idx, eps=eps)
    t1 = time.perf_counter() - t0
    k2 = int(min(s.n, max(k, k * target_s / max(t1, 1e-3))))
    idx = np.sort(g.choice(s.n, k2, replace=False))
    t0 = time.perf_counter()
    oracle.forces_sample(s.pos, s.mass, idx, eps=eps)
    t2 = time.perf_counter() - t0
    # the same oracle on one thread, on a smaller sample (about target_s / 4 seconds)
    oracle.set_threads(1)
    k1 = int(min(s.n, max(8, k2 * (target_s / 4.0) / max(t2 * threads, 1e-3))))
    idx1 = np.sort(g.choice(s.n, k1, replace=False))
    t0 = time.perf_counter()
    oracle.forces_sample(s.pos, s.mass, idx1, eps=eps)
    t3 = time.perf_counter() - t0
    oracle.set_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": k2 * float(s.n) / t2, "unit": "pair interactions/s", "cores": threads, "kind": "oracle",
            "sample": "%d random particles of the Plummer N=%d system against all N (one FP64 force evaluation "
                      "restricted to the sample), %.1f s" % (k2, s.n, t2),
            "value_1_thread": k1 * float(s.n) / t3, "sample_1_thread": "%d particles, %.1f s" % (k1, t3),
            "host_cpus_visible": os.cpu_count(), "cpu_model": model,
            "build": "gcc -O3 -march=x86-64-v3 -fopenmp -ffp-contract=off -fno-fast-math (oracle/__init__.py), OpenMP over target particles"}


if __name__ == "__main__":
    main()
