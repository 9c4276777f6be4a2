/*
 * nbody.h - C ABI of libnbody.so, the MI355X (gfx950) all-pairs N-body hot path.
 *
 * What is computed (per system; systems never interact):
 *   The paper's N-body miniapp evaluates the force between every pair of
 *   particles, N_p^2 pair interactions per evaluation (Sec. V-B), moves the
 *   particles with a Verlet half-step integrator (Sec. II-A) and reduces the
 *   total energy over all particles inside the force pass (Sec. VI, with and
 *   without that reduction). This library keeps that structure with
 *   Plummer-softened gravity as the pair law in place of Eq. (1):
 *       d_ij  = x_j - x_i,   s_ij = |d_ij|^2 + eps^2
 *       a_i   =  G sum_{j != i} m_j d_ij s_ij^{-3/2}
 *       phi_i = -G sum_{j != i} m_j s_ij^{-1/2}
 *   and reads the Verlet half-step scheme as kick-drift-kick leapfrog with
 *   force reuse. Energy/momentum per system: KE = 1/2 sum m|v|^2,
 *   PE = 1/2 sum m phi, P = sum m v (all reduced in FP64, deterministically,
 *   without atomics).
 *   The paper's own Lennard-Jones gas (Eq. (1)) runs through the same tile
 *   engine: nbody_lj_forces / nbody_lj_rollout at the end of this header.
 *
 * Conventions (all entry points):
 *   - Array pointers are DEVICE pointers owned by the caller, unless a comment
 *     says HOST. Positions, velocities, accelerations and their gradients are
 *     SoA planes of doubles, [3][n] (all x, then all y, then all z).
 *   - The library allocates no device memory. Scratch space comes from the
 *     caller's workspace (nbody_config.workspace), whose size
 *     nbody_workspace_size() returns (nbody_step_noalloc: a static device array
 *     of the library instead).
 *   - Calls are asynchronous on nbody_config.stream (a hipStream_t; NULL = the
 *     null stream). The round schedule (NBODY_FLAG_SYM_ROUNDS) also runs work
 *     on two streams of the library, ordered before and after the call's other
 *     work on nbody_config.stream by events. Host arguments (offsets, the
 *     config itself) may be reused as soon as the call returns.
 *   - Every call returns an nbody_status. Argument errors are detected on the
 *     host before any HIP call and leave device memory untouched; a failed
 *     launch returns NBODY_ERR_DEVICE. nbody_last_error() describes the last
 *     failure of the calling thread. Device faults surface at the caller's
 *     next synchronisation.
 *   - n == 0 is valid and does nothing.
 *   - Results are deterministic: the same inputs, configuration and tile
 *     table give bitwise-equal outputs (fixed summation orders; the round
 *     schedule's atomic adds reach each accumulator word once per launch, so
 *     their order is fixed as well).
 *   - Outputs must not alias inputs except where a parameter is documented as
 *     in/out.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBODY_ABI_VERSION 1

typedef enum {
  NBODY_OK = 0,
  NBODY_ERR_INVALID_ARG = 1, /* bad pointer, size, softening, step, offsets ... */
  NBODY_ERR_DEVICE = 2,      /* a HIP call failed (message in nbody_last_error) */
  NBODY_ERR_UNSUPPORTED = 3, /* valid request this build cannot serve */
  NBODY_ERR_WORKSPACE = 4    /* workspace missing or smaller than required */
} nbody_status;

/* Arithmetic of the pair interactions. State, position/velocity updates and
 * every reduction are FP64 in all modes.
 *   NBODY_FP64       pair math in double.
 *   NBODY_FP32       pair math in float; per-particle float accumulators.
 *   NBODY_FP32_COMP  pair math in float; per-particle accumulation blocked and
 *                    compensated: no float sum spans more than one tile of
 *                    j-particles, and the tile sums are combined without
 *                    rounding loss - folded with an error-free TwoSum into a
 *                    float (hi, lo) pair, or added in double.
 *   NBODY_FP32_DS    as NBODY_FP32_COMP, and every separation is formed from
 *                    double-float coordinates (x = hi + lo, two floats), so it is
 *                    exact to the float rounding of the separation itself instead
 *                    of the coordinates; costs about 6 more float operations per
 *                    pair (adjoint passes run as NBODY_FP32_COMP).
 *   NBODY_FP32_ADAPT as NBODY_FP32_COMP, with double-float separations only where
 *                    they matter: a single system on symmetric tiles is ordered along a
 *                    Morton curve on the device at every force pass (deterministic:
 *                    unique keys), and only the 64-particle sub-block pairs whose
 *                    bounding boxes lie within T = X_max / 256 of each other (X_max: the
 *                    largest coordinate magnitude) take double-float separations; every
 *                    other pair is at least T apart, so its float separation errs by at
 *                    most 2 u X_max / T < 3.1e-5 relative. Results come back in the
 *                    caller's order. Other paths (batches, one-sided small-n passes) run
 *                    as NBODY_FP32_DS; adjoint passes as NBODY_FP32_COMP. A rollout with
 *                    an energy trace reduces the energy in a separate pass. */
typedef enum {
  NBODY_FP64 = 0,
  NBODY_FP32 = 1,
  NBODY_FP32_COMP = 2,
  NBODY_FP32_DS = 3,
  NBODY_FP32_ADAPT = 4
} nbody_precision;

/* config.flags */
#define NBODY_FLAG_LOOP_SYSTEMS 1u /* batched calls: one plain launch per system
                                      instead of one launch for all systems (baseline) */
#define NBODY_FLAG_WHOLE_ROLLOUT 2u /* nbody_rollout / nbody_lj_rollout of a batch on
                                      symmetric tiles without an energy trace or
                                      checkpoints: every step in one launch, systems
                                      advancing independently (per-system waits on
                                      device counters); the trajectory is bitwise that
                                      of the per-step path. When some system spans
                                      several tiles the call waits for the launch to
                                      finish (it reads back a device error word).
                                      Ignored where it does not apply. A batch whose
                                      systems all fit one tile takes this path without
                                      the flag (no waits, no read-back). */
#define NBODY_FLAG_PER_PASS 4u      /* batched rollouts: one launch per pass even where
                                      every step in one launch would be chosen (the
                                      baseline of that choice; results are identical) */
#define NBODY_FLAG_SYM_ROUNDS 8u    /* single-system FP32 force and adjoint passes on the
                                      round schedule: symmetric tiles of 1024-particle
                                      blocks run in rounds of disjoint block pairs (circle
                                      method), each tile adding its sums to per-particle
                                      double accumulators, so the workspace is linear in n
                                      (32 K bytes per particle for K accumulator copies:
                                      K = 4 where the workspace allows, else 2 or 1) instead
                                      of one float slot per particle and block. With K >= 2
                                      the launches (K/2 rounds each) alternate between two
                                      streams the library creates per device and keeps; the
                                      call's stream waits for both. Deterministic for a
                                      given K; not bitwise the slot schedule's sums (another
                                      order). The library takes this schedule by itself
                                      where the slot schedule's partial sums would exceed
                                      its cap (16 GiB: forces near 1.5 million particles,
                                      the adjoint just above 1 million). The adaptive mode
                                      sorts and runs its adaptive tiles on it as well. */

typedef struct {
  int32_t abi_version;     /* must equal NBODY_ABI_VERSION */
  int32_t precision;       /* nbody_precision */
  double G;                /* gravitational constant, finite */
  double eps;              /* Plummer softening length; eps > 0, and eps >= 1e-10 for
                              the FP32 modes (eps^2 must be a normal float) */
  int64_t n_systems;       /* >= 1 */
  const int64_t *offsets;  /* HOST, n_systems + 1 entries: offsets[0] = 0,
                              non-decreasing, offsets[n_systems] = n. System s owns
                              particles offsets[s] .. offsets[s+1]-1. May be NULL
                              only when n_systems == 1. */
  void *workspace;         /* DEVICE scratch, caller-owned, 256-byte aligned */
  size_t workspace_bytes;  /* >= nbody_workspace_size(...) for the call */
  void *stream;            /* hipStream_t (NULL = null stream) */
  uint32_t flags;          /* NBODY_FLAG_* */
  uint32_t reserved;       /* must be 0 */
} nbody_config;

/* Bytes of workspace any call below needs for n particles (in cfg's systems).
 * For nbody_rollout_backward pass its ckpt_every (>= 1; the size grows with it);
 * pass 0 when no backward pass is planned. `steps` must be >= 0. The size depends
 * on cfg->precision, cfg->n_systems/offsets and the tile table (not on G, eps or
 * the pair law: the same size serves the Lennard-Jones calls).
 * Returns NBODY_OK and writes *bytes. */
int nbody_workspace_size(const nbody_config *cfg, int64_t n, int64_t steps, int64_t ckpt_every,
                         size_t *bytes);

/* All-pairs acceleration and, optionally, potential of every particle
 * (the force pass of Sec. V-B; pot != NULL adds the fused per-particle
 * potential that the Sec. VI energy reduction needs, pot == NULL is the
 * variant without it).
 *   pos  [3][n] double, mass [n] double (any finite values; mass may be 0)
 *   acc  [3][n] double, out
 *   pot  [n] double, out, nullable */
int nbody_forces(const nbody_config *cfg, int64_t n, const double *pos, const double *mass,
                 double *acc, double *pot);

/* One GPU's share of the paper's ring decomposition (Sec. V-B, Fig. 1), run on this GPU: with P
 * GPUs each owning one block of the particles while the j-blocks travel around the ring, GPU g
 * evaluates its own particles against all n, one j-block per hop. This call computes share g:
 * the accelerations (and potentials) of block g's particles from all n particles, with the
 * j-range taken in the same P blocks, one double partial sum per block, added in block order
 * (what a ring implementation that keeps one partial per arriving block computes, whatever the
 * order of arrival). Blocks hold s = 256 ceil(t / min(P, t)) particles, t = ceil(n / 256), so
 * block g is [g s, min(n, (g + 1) s)) (empty when g s >= n). The rows equal, bitwise, those of
 * nbody_forces on the one-sided tile "bs=256,i=1,tj=256" (tile variant 0) with P j-ranges.
 * Gravity, single systems; FP32 modes and FP64 (the adaptive mode runs as the double-float
 * mode).
 *   P >= 1, 0 <= g < P (else NBODY_ERR_INVALID_ARG); n_systems == 1 (else UNSUPPORTED);
 *   pos [3][n], mass [n]; acc [3][n], pot [n] (nullable): only block g's rows are written;
 *   the workspace: nbody_forces_shard_workspace_size bytes (the j-array and, for P > 1,
 *   P [4][n] double partial planes). */
int nbody_forces_shard_workspace_size(const nbody_config *cfg, int64_t n, int32_t P, size_t *bytes);
int nbody_forces_shard(const nbody_config *cfg, int64_t n, int32_t P, int32_t g, const double *pos,
                       const double *mass, double *acc, double *pot);

/* One kick-drift-kick step of size dt with force reuse (the Verlet
 * half-step update of Sec. II-A):
 *   v += dt/2 a;  x += dt v;  a = a(x);  v += dt/2 a
 *   pos, vel [3][n] in/out; acc [3][n] in: a(x_n), out: a(x_{n+1});
 *   pot [n] nullable, out: the potential at x_{n+1} from the same force pass
 *   (for an energy reduction after the step without another pass). */
int nbody_step(const nbody_config *cfg, int64_t n, double dt, double *pos, double *vel,
               const double *mass, double *acc, double *pot);

/* ---- allocation-free step ----
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. The same step as nbody_step with its workspace taken
 * from a static device array of NBODY_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
 * until the process ends; the library neither allocates nor frees memory in this call (the
 * first call on a device only looks up the array's device address).
 * Tiles: the first of these whose whole workspace fits the array: the tile nbody_step would use
 * (bitwise the same results); the tile table's tile for the largest systems (its largest block,
 * fewest partial sums); the round schedule (NBODY_FLAG_SYM_ROUNDS: workspace linear in n); the
 * one-sided pass with as many j-ranges as fit (FP64, which has no symmetric tiles, takes its
 * tuned tile or this one). The later ones differ from nbody_step only in the order of the
 * floating-point sums.
 *   cfg->workspace must be NULL and cfg->workspace_bytes 0 (else NBODY_ERR_INVALID_ARG);
 *   a single system only (n_systems == 1, offsets NULL; else NBODY_ERR_UNSUPPORTED);
 *   n whose step needs more than NBODY_NOALLOC_SCRATCH_BYTES of workspace even one-sided
 *   with one j-range (beyond about 1.95 million particles in FP64 and in the double-float and
 *   adaptive modes, 2.6 million in the other FP32 modes; the round schedule serves up to about
 *   1.2-1.6 million, by mode) returns NBODY_ERR_WORKSPACE before any device work.
 * Every call on one GPU shares that GPU's array (nothing in it needs to start at zero): calls
 * that overlap on one GPU (other host threads, other streams without ordering) race.
 * The step creates no stream or event and records only kernel launches on the caller's stream
 * (the round schedule's launches, which nbody_step alternates between two library streams, go in
 * order on it, with the same results), also under stream capture. */
#define NBODY_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int nbody_step_noalloc(const nbody_config *cfg, int64_t n, double dt, double *pos, double *vel,
                       const double *mass, double *acc, double *pot);

/* `steps` KDK steps (steps >= 0), state in place.
 *   acc   in: a(x_0) (e.g. from nbody_forces), out: a(x_steps)
 *   ckpt  nullable, [steps/ckpt_every + 1][6][n] doubles: (x planes, v planes)
 *         at steps 0, ckpt_every, 2 ckpt_every, ... (ckpt_every >= 1 when given;
 *         ignored when NULL)
 *   energy_trace nullable, [steps + 1][n_systems][5] doubles: (KE, PE, Px, Py, Pz)
 *         of every system at every integer step (costs the potential in every
 *         force pass). */
int nbody_rollout(const nbody_config *cfg, int64_t n, double dt, int64_t steps, int64_t ckpt_every,
                  double *pos, double *vel, const double *mass, double *acc, double *ckpt,
                  double *energy_trace);

/* Energy and linear momentum of every system (the energy reduction of Sec. VI).
 *   pot  nullable: the per-particle potential from nbody_forces (or, for the
 *        Lennard-Jones gas, from nbody_lj_forces); when NULL it is computed here
 *        with one gravity force pass at cfg->precision.
 *   out  [n_systems][5] double: KE, PE, Px, Py, Pz. */
int nbody_energy_momentum(const nbody_config *cfg, int64_t n, const double *pos, const double *vel,
                          const double *mass, const double *pot, double *out);

/* Diagnostics of every system from its state and a force evaluation of any pair law
 * (the pot and acc written by nbody_forces or nbody_lj_forces for these positions):
 *   out [n_systems][10] double: KE, PE, Px, Py, Pz, Lx, Ly, Lz, W, M with
 *   L = sum m x cross v (angular momentum about the origin), W = sum m x . a (the virial
 *   of the pair forces; for a gas in a box it gives the pressure), M = sum m.
 * Reduced in FP64 by the same deterministic two-pass tree as the energy. G and eps
 * are not used. */
int nbody_diagnostics(const nbody_config *cfg, int64_t n, const double *pos, const double *vel,
                      const double *mass, const double *pot, const double *acc, double *out);

/* Reverse-mode gradient of a function of the final state of a rollout made by
 * nbody_rollout(cfg, n, dt, steps, ckpt_every, ...) with the same cfg:
 * the exact adjoint of the discrete KDK map (discretise, then differentiate).
 *   ckpt        [steps/ckpt_every + 1][6][n] checkpoints written by that rollout
 *   gpos_final, gvel_final [3][n]: dL/dx_steps, dL/dv_steps
 *   gpos0, gvel0 [3][n] out: dL/dx_0, dL/dv_0;  gmass [n] out: dL/dm.
 * Positions between checkpoints are recomputed (bitwise equal to the forward
 * pass). Each step costs one adjoint pair pass
 *   gx_k += G sum_j T(d_kj)(m_k l_j - m_j l_k),  gm_k += -G sum_j s^{-3/2} d_kj . l_j,
 *   T(d) = s^{-3/2} I - 3 s^{-5/2} d d^T,  l = w * (velocity cotangent)
 * at cfg->precision, plus one recomputed force pass. */
int nbody_rollout_backward(const nbody_config *cfg, int64_t n, double dt, int64_t steps,
                           int64_t ckpt_every, const double *mass, const double *ckpt,
                           const double *gpos_final, const double *gvel_final, double *gpos0,
                           double *gvel0, double *gmass);

/* The same gradient without checkpoints: the positions x_{steps-1} .. x_0 are rebuilt
 * by integrating backwards from the final state (the kick-drift-kick map is time
 * reversible: a step of -dt undoes a step of dt up to rounding), so only O(n) memory
 * is held. Costs the same as nbody_rollout_backward (one force pass and one adjoint pass
 * per step). The rebuilt positions differ from the forward ones by rounding that
 * chaotic dynamics amplify over many steps, so the gradient is exact only to that level.
 *   pos_final, vel_final [3][n]: the state after the rollout (x_steps, v_steps). */
int nbody_rollout_backward_reversible(const nbody_config *cfg, int64_t n, double dt, int64_t steps,
                                      const double *mass, const double *pos_final, const double *vel_final,
                                      const double *gpos_final, const double *gvel_final, double *gpos0,
                                      double *gvel0, double *gmass);

/* ---- the paper's pair law: Lennard-Jones gas (Eq. (1)) ----
 *
 *   V(r) = 4 epsilon [(sigma/r)^12 - (sigma/r)^6],
 *   F_i  = sum_{j != i} 24 epsilon [2 sigma^12 / r^13 - sigma^6 / r^7] r_hat_ji
 *          (r_hat_ji: unit vector from x_j to x_i; repulsive below 2^{1/6} sigma),
 *   a_i  = F_i / m_i,   pot_i = (1/m_i) sum_{j != i} V(r_ij)
 * so that PE = 1/2 sum m pot exactly as for gravity (nbody_energy_momentum with
 * this pot gives the gas's energy). An optional softening w replaces r^2 by
 * r^2 + w^2 (w = 0 is the plain law; then no two particles may coincide, and
 * masses must be nonzero). No cutoff: every pair interacts, as in the paper.
 * All nbody_config fields apply except G and eps, which these calls ignore. */
typedef struct {
  double sigma;      /* > 0 */
  double epsilon;    /* well depth, finite */
  double soft;       /* >= 0 (FP32 modes: 0 or soft/sigma >= 1e-10) */
  int32_t walls;     /* 1: reflective walls at lo/hi, 0: open space */
  int32_t reserved;  /* must be 0 */
  double lo[3];      /* box corners when walls == 1: finite, lo[c] < hi[c]; */
  double hi[3];      /* initial positions should lie inside the box */
} nbody_lj_params;

/* Lennard-Jones accelerations and (pot != NULL) per-particle potentials of every
 * system; arguments as in nbody_forces, mass [n] > 0. Pair arithmetic at
 * cfg->precision on coordinates scaled by 1/sigma; sums and constants in FP64. */
int nbody_lj_forces(const nbody_config *cfg, const nbody_lj_params *lj, int64_t n, const double *pos,
                    const double *mass, double *acc, double *pot);

/* `steps` KDK steps of the Lennard-Jones gas (steps >= 0), state in place, with the
 * boundary check after every drift when lj->walls: a coordinate that left the box
 * is mirrored back in (x -> 2 lo - x or 2 hi - x) and that velocity component
 * changes sign (elastic walls).
 *   acc in: a(x_0) (from nbody_lj_forces), out: a(x_steps)
 *   energy_trace nullable, [steps + 1][n_systems][5] doubles as in nbody_rollout
 *         (the energy reduction of every step, fused behind its force pass). */
int nbody_lj_rollout(const nbody_config *cfg, const nbody_lj_params *lj, int64_t n, double dt,
                     int64_t steps, double *pos, double *vel, const double *mass, double *acc,
                     double *energy_trace);

/* ---- tile table (written by the autotuner; built-in defaults otherwise) ---- */

typedef enum {
  NBODY_KERNEL_FORCE = 0,   /* single-system force pass */
  NBODY_KERNEL_ADJOINT = 1, /* single-system adjoint pass */
  NBODY_KERNEL_FORCE_BATCHED = 2,
  NBODY_KERNEL_ADJOINT_BATCHED = 3,
  /* Lennard-Jones force passes: the same variants as NBODY_KERNEL_FORCE(_BATCHED);
     without an entry of their own they run with that kernel's entry (or default) */
  NBODY_KERNEL_LJ_FORCE = 4,
  NBODY_KERNEL_LJ_FORCE_BATCHED = 5
} nbody_kernel;

typedef struct {
  int32_t kernel;    /* nbody_kernel */
  int32_t precision; /* nbody_precision */
  int64_t n_min;     /* entry applies when n_min <= n <= n_max (n: particles of the
                        system for single-system kernels, largest system for batched) */
  int64_t n_max;
  int32_t variant;   /* index into nbody_tile_variants() for (kernel, precision) */
  int32_t j_split;   /* single-system: number of j-ranges (>= 1, results summed in a
                        fixed order); batched: j-chunk length of one work unit */
} nbody_tile_entry;

/* Replace the tile table (copied; count 0 restores the built-in defaults). */
int nbody_set_tile_table(const nbody_tile_entry *entries, int64_t count);

/* Number of compiled tile variants for (kernel, precision); writes up to `cap`
 * descriptions "bs=256,i=2,tj=256" (NUL-separated) into `buf` when non-NULL. */
int nbody_tile_variants(int32_t kernel, int32_t precision, char *buf, size_t cap);

/* The (variant, j_split) the library would use for a call of size n. */
int nbody_tile_lookup(int32_t kernel, int32_t precision, int64_t n, int32_t *variant,
                      int32_t *j_split);

/* ---- diagnostics ---- */
const char *nbody_last_error(void); /* thread-local, valid until the next call on this thread */
int nbody_abi_version(void);

/* Probes (each a device-scope load and a short sleep) a wait of the whole-rollout launch
 * (NBODY_FLAG_WHOLE_ROLLOUT) makes before it gives up; the launch then ends early and the
 * call returns NBODY_ERR_DEVICE. Default 2^24 probes (each a sleep of 128 clocks plus the
 * load's latency: seconds of waiting). probes >= 1, else
 * NBODY_ERR_INVALID_ARG. For failure-path tests and for diagnosing a stalled launch;
 * process-wide, applies to launches made after the call. */
int nbody_set_wait_limit(int64_t probes);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
