// Device kernels of the all-pairs N-body hot path for gfx950 (CDNA4).
//
// Pair laws (all-pairs structure of Sec. V-B), chosen at compile time (LAW):
//   LAW_GRAV  softened gravity: d = x_j - x_i, s = |d|^2 + eps^2,
//             a_i = G sum_j m_j d s^{-3/2}, phi_i = -G sum_j m_j s^{-1/2};
//   LAW_LJ    the Lennard-Jones law of Eq. (1) on coordinates staged in units of
//             sigma (x' = x / sigma) with optional softening w' = w / sigma:
//             u = 1 / (|d'|^2 + w'^2), q = u^3 = (sigma/r)^6,
//             a_i = (24 eps / sigma) / m_i sum_j u q (1 - 2 q) d',
//             pot_i = 4 eps / m_i sum_j (q^2 - q)   (= (1/m_i) sum_j V(r_ij)).
//   The kernels accumulate the law's sums without its constants; the reduce /
//   store step applies them (G, or 24 eps / sigma and 4 eps with the 1/m_i).
//
// Execution model of the pair kernels:
//   * a block owns BS*I consecutive i-particles; lane t keeps particles
//     ib + t + u*BS (u < I) in registers, so the i loads and the result stores
//     are coalesced;
//   * the j-range streams through LDS in tiles of TJ particles; the next tile is
//     prefetched into registers while the current one is consumed, and every
//     lane of a wave reads the same LDS address (a broadcast, conflict-free);
//   * every loop-invariant operand of the inner loop (eps^2, the i-particle
//     coordinates) lives in a VGPR: on gfx950 a VALU instruction that reads an
//     SGPR cannot be paired with another wave's VALU instruction in the same
//     cycle, which halves the FP32 issue rate of the loop;
//   * every sum runs in a fixed order: no atomics in the arithmetic, except the round
//     schedule's adds, which reach each accumulator word once per launch.
//
// Self pair: d = 0 exactly (both sides read the same stored coordinates), so under
// gravity it adds exactly 0 to the acceleration. It must be excluded from the
// potential, from the adjoint and (its u is infinite without softening) from the
// whole Lennard-Jones pair, so tiles that overlap the block's own i-range take a
// masked copy of the inner loop; all other tiles take the unmasked one.
//
// Padding: j-slots past the end of a range hold a particle that contributes exactly
// zero - massless at the origin under gravity, and under Lennard-Jones a particle so
// far away (1e30 in float, 1e150 in double) that u^3 underflows to 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbody {

// ----------------------------------------------------------------- helpers

// Copy a value into a VGPR the compiler cannot see through (keeps uniform
// loop constants out of SGPR operands of the inner-loop VALU instructions).
__device__ __forceinline__ float in_vgpr(float x) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// An opaque copy of an int: address arithmetic built on it stays where it is written (the
// compiler cannot hoist it out of a branch into registers held across a whole loop).
__device__ __forceinline__ int opaque_int(int x) {
  int r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ double in_vgpr(double x) {
  double r;
  asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Error-free transformation (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// s^{-1/2} in double: hardware estimate refined by Newton-Raphson steps
// y <- y + y/2 (1 - s y^2) (each step roughly doubles the correct bits).
template <int NEWTON>
__device__ __forceinline__ double rsqrt_f64(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int k = 0; k < NEWTON; ++k) {
    double e = __builtin_fma(-s * y, y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
  }
  return y;
}

// Fused multiply-add in the pair precision (float must not be promoted to double).
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

struct alignas(16) D4 { double x, y, z, w; };

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = D4; };

template <typename T>
__device__ __forceinline__ typename Vec4<T>::type zero4() {
  typename Vec4<T>::type v;
  v.x = v.y = v.z = v.w = T(0);
  return v;
}

enum { LAW_GRAV = 0, LAW_LJ = 1 };

// j-slot padding that adds exactly zero under the pair law (see the header comment).
template <typename T, int LAW>
__device__ __forceinline__ typename Vec4<T>::type pad4() {
  typename Vec4<T>::type v = zero4<T>();
  if constexpr (LAW == LAW_LJ) v.x = v.y = v.z = sizeof(T) == 4 ? T(1e30f) : T(1e150);
  return v;
}

// v[idx] when ok, else fill: an explicit branch around the load (a select between the
// element's address and a local's would turn the load into a generic one through
// private memory).
template <typename V>
__device__ __forceinline__ V load_or(const V* __restrict__ v, int64_t idx, bool ok, V fill) {
  if (ok) fill = v[idx];
  return fill;
}

// 1/s in double: hardware estimate refined by two Newton-Raphson steps y <- y + y (1 - s y).
__device__ __forceinline__ double rcp_f64(double s) {
  double y = __builtin_amdgcn_rcp(s);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double e = __builtin_fma(-s, y, 1.0);
    y = __builtin_fma(y, e, y);
  }
  return y;
}

template <typename T>
__device__ __forceinline__ T pair_rcp(T s);
template <>
__device__ __forceinline__ float pair_rcp<float>(float s) { return __builtin_amdgcn_rcpf(s); }
template <>
__device__ __forceinline__ double pair_rcp<double>(double s) { return rcp_f64(s); }

template <typename T>
__device__ __forceinline__ T pair_rsqrt(T s);
template <>
__device__ __forceinline__ float pair_rsqrt<float>(float s) { return __builtin_amdgcn_rsqf(s); }
template <>
__device__ __forceinline__ double pair_rsqrt<double>(double s) { return rsqrt_f64<2>(s); }

// ----------------------------------------------------------------- staging / update kernels

// j-array: (x, y, z, m) per particle in the pair precision, 16 B (float) or 32 B (double).
// Double-float form (DS): two float4 per particle, (hi_x, hi_y, hi_z, m) and
// (lo_x, lo_y, lo_z, 0) with hi = fl32(x), lo = fl32(x - hi), so hi + lo carries x to
// about 48 bits and a separation (hi_j - hi_i) + (lo_j - lo_i) is exact to float
// rounding of the separation itself, not of the coordinates.
// xs scales the staged coordinates (1 under gravity, 1/sigma under Lennard-Jones).
template <typename T, bool DS>
__device__ __forceinline__ void put_j(typename Vec4<T>::type* __restrict__ jarr, int64_t i, const double x_in[3],
                                      double m, double xs) {
  const double x[3] = {x_in[0] * xs, x_in[1] * xs, x_in[2] * xs};
  if constexpr (DS) {
    float4 h, l;
    h.x = (float)x[0]; h.y = (float)x[1]; h.z = (float)x[2]; h.w = (float)m;
    l.x = (float)(x[0] - (double)h.x);
    l.y = (float)(x[1] - (double)h.y);
    l.z = (float)(x[2] - (double)h.z);
    l.w = 0.f;
    jarr[2 * i] = h;
    jarr[2 * i + 1] = l;
  } else {
    typename Vec4<T>::type v;
    v.x = (T)x[0]; v.y = (T)x[1]; v.z = (T)x[2]; v.w = (T)m;
    jarr[i] = v;
  }
}

template <typename T, bool DS>
__global__ void stage_j(int64_t n, const double* __restrict__ pos, const double* __restrict__ mass, double xs,
                        typename Vec4<T>::type* __restrict__ jarr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x[3] = {pos[i], pos[n + i], pos[2 * n + i]};
  put_j<T, DS>(jarr, i, x, mass[i], xs);
}

// Reflective walls of the box [lo, hi]^3, applied after the drift (the boundary
// check of the paper's miniapp): a coordinate past a wall is mirrored back into
// the box and that velocity component changes sign. on == 0: open space.
struct Walls {
  int32_t on;
  int32_t pad;
  double lo[3], hi[3];
};

// First half of a KDK step fused with the staging of the new positions:
//   v += hh a;  x += h v;  (walls);  jarr = (xs x, m) in pair precision (jarr == nullptr:
//   no staging; the adaptive mode stages in sorted order at its next force pass).
template <typename T, bool DS>
__global__ void kick_drift_stage(int64_t n, double hh, double h, double* __restrict__ pos,
                                 double* __restrict__ vel, const double* __restrict__ acc,
                                 const double* __restrict__ mass, double xs, Walls wl,
                                 typename Vec4<T>::type* __restrict__ jarr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = vel[c * n + i] + hh * acc[c * n + i];
    double xc = pos[c * n + i] + h * v;
    if (wl.on) {
      if (xc < wl.lo[c]) {
        xc = 2.0 * wl.lo[c] - xc;
        v = -v;
      } else if (xc > wl.hi[c]) {
        xc = 2.0 * wl.hi[c] - xc;
        v = -v;
      }
    }
    vel[c * n + i] = v;
    pos[c * n + i] = xc;
    x[c] = xc;
  }
  if (jarr) put_j<T, DS>(jarr, i, x, mass[i], xs);
}

// Constants of the pair law applied to the kernels' raw sums:
//   acc = ca * sum / m_i, pot = cp * sum / m_i (mdiv = masses), or without the 1/m_i
//   when mdiv == nullptr (gravity: ca = cp = G).
struct LawScale {
  double ca, cp;
  const double* mdiv;
};

__device__ __forceinline__ double law_div(const LawScale& ls, int64_t i) { return ls.mdiv ? ls.mdiv[i] : 1.0; }

// The next kick-drift-kick step's first half, fused into the kernel that finishes the
// current step (the per-particle reduction of the force pass): after the closing kick
// v += hh a of step n, the opening kick v += hh a of step n+1, the drift x += h v, the
// walls and the staging of x into the j-array - the same operations in the same order
// as kick_drift_stage, so trajectories are bitwise those of the unfused loop.
// kind: 0 none, 1 float j-array, 2 double, 3 double-float (two float4 per particle),
// 4 kick and drift without staging.
struct NextStep {
  int32_t kind;
  int32_t pad;
  double* pos;
  const double* mass;
  double hh, h, xs;
  Walls wl;
  void* jarr;
  double* pos_copy;  // nullable: the drifted positions are also written here ([3][n] like pos)
};

// The state a per-particle reduction needs besides the particle's sums, loaded before the sums'
// own loads so that all of them are in flight together (a reduction over few particles is bound by
// memory round trips): the divisor of the law (a mass, or 1), the velocity, and for the fused
// next step the position and the mass; the energy's mass.
struct PState {
  double md, em, m;
  double v[3], x[3];
};

__device__ __forceinline__ PState load_state(int64_t i, int64_t stride, const LawScale& ls,
                                             const double* __restrict__ vel, const NextStep& nx,
                                             const double* __restrict__ emass, bool en) {
  PState ps{};
  ps.md = law_div(ls, i);
  if (vel)
#pragma unroll
    for (int c = 0; c < 3; ++c) ps.v[c] = vel[c * stride + i];
  if (nx.kind) {
#pragma unroll
    for (int c = 0; c < 3; ++c) ps.x[c] = nx.pos[c * stride + i];
    if (nx.kind != 4) ps.m = nx.mass[i];
  }
  if (en) ps.em = emass[i];
  return ps;
}

// The next step's first half for particle i, whose closing-kicked velocity is v (the value just
// written to the velocity planes) and whose position is x0: kick, drift, walls, staging.
__device__ __forceinline__ void next_step_tail(const NextStep& ns, int64_t i, int64_t n, const double a[3],
                                               const double v_in[3], const double x0[3], double m,
                                               double* __restrict__ vel) {
  double x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = v_in[c] + ns.hh * a[c];
    double xc = x0[c] + ns.h * v;
    if (ns.wl.on) {
      if (xc < ns.wl.lo[c]) {
        xc = 2.0 * ns.wl.lo[c] - xc;
        v = -v;
      } else if (xc > ns.wl.hi[c]) {
        xc = 2.0 * ns.wl.hi[c] - xc;
        v = -v;
      }
    }
    vel[c * n + i] = v;
    ns.pos[c * n + i] = xc;
    if (ns.pos_copy) ns.pos_copy[c * n + i] = xc;
    x[c] = xc;
  }
  if (ns.kind == 1) put_j<float, false>((float4*)ns.jarr, i, x, m, ns.xs);
  else if (ns.kind == 2) put_j<double, false>((D4*)ns.jarr, i, x, m, ns.xs);
  else if (ns.kind == 3) put_j<float, true>((float4*)ns.jarr, i, x, m, ns.xs);
  // kind 4: no staging (the adaptive mode stages in sorted order before its next pass)
}

// Block-wide sum of K doubles per thread in a fixed order (wave64 shuffle tree, then the
// waves in order); the result is valid in thread 0. sh: [K][BS/64] doubles of LDS.
template <int BS, int K>
__device__ __forceinline__ void block_sum(double v[K], double* sh) {
#pragma unroll
  for (int c = 0; c < K; ++c) {
    double x = v[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[c] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < K; ++c) sh[c * (BS / 64) + wave] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double x = 0.0;
      for (int w = 0; w < BS / 64; ++w) x += sh[c * (BS / 64) + w];
      v[c] = x;
    }
  }
}

// One particle's share of the energy and momentum: KE, PE (half its mass times its
// potential), P.
__device__ __forceinline__ void energy_terms(double m, double vx, double vy, double vz, double phi, double e[5]) {
  e[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
  e[1] += 0.5 * m * phi;
  e[2] += m * vx;
  e[3] += m * vy;
  e[4] += m * vz;
}

// Energy of the state a per-particle reduction has just finished, fused into it: the
// reduction then runs on the (chunk, system) grid of energy_partial, blocks of kEnergyBS
// threads, each thread taking the same particles in the same order, and block (chunk, s)
// writes part[s][chunk][5] exactly as energy_partial would (energy_final completes the sum).
// part == nullptr: nothing fused, one thread per particle.
constexpr int kReduceBS = 256;  // block size of the per-particle reductions without the energy
// Threads of an energy chunk: one wave, so that a system of n particles spreads its fused
// reduction over n / 64 workgroups (at n = 10^4, 157 rather than 40 CUs).
constexpr int kEnergyBS = 64;

struct EnergyFuse {
  double* part;
  const double* mass;
  int32_t chunks;
  int32_t pad;
};

// Thread loop of chunk blockIdx.x over the particles [b, e) of system s, with body(i, en)
// adding particle i's energy terms to en, then the chunk's block sum.
template <typename F>
__device__ __forceinline__ void energy_chunk(int64_t b, int64_t e, int64_t s, const EnergyFuse& ef, F&& body) {
  __shared__ double sh[5 * (kEnergyBS / 64)];
  double en[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = b + (int64_t)blockIdx.x * kEnergyBS + threadIdx.x; i < e; i += (int64_t)ef.chunks * kEnergyBS)
    body(i, en);
  block_sum<kEnergyBS, 5>(en, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 5; ++c) ef.part[(s * ef.chunks + blockIdx.x) * 5 + c] = en[c];
}

// The common end of the per-particle reductions, given particle i's raw sums a[4] and its state
// ps (load_state): acceleration, closing half kick v += hh a (vel != nullptr), potential (pot !=
// nullptr), its energy terms (en != nullptr; needs pot, vel and emass) and the next step's first
// half.
__device__ __forceinline__ void finish_particle(int64_t i, int64_t stride, const double a[4], const LawScale& ls,
                                                double* __restrict__ acc, double* __restrict__ pot,
                                                double* __restrict__ vel, double hh, const NextStep& nx,
                                                double* en, const PState& ps) {
  const double md = ps.md;
  double ac[3], v[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ac[c] = ls.ca * a[c] / md;
    acc[c * stride + i] = ac[c];
    if (vel) {
      v[c] = ps.v[c] + hh * ac[c];
      vel[c * stride + i] = v[c];
    }
  }
  double phi = 0.0;
  if (pot) {
    phi = ls.cp * a[3] / md;
    pot[i] = phi;
  }
  if (en) energy_terms(ps.em, v[0], v[1], v[2], phi, en);
  if (nx.kind) next_step_tail(nx, i, stride, ac, v, ps.x, ps.m, vel);
}

// The same with the state loaded here (kernels whose registers a pair loop shares).
__device__ __forceinline__ void finish_particle(int64_t i, int64_t stride, const double a[4], const LawScale& ls,
                                                double* __restrict__ acc, double* __restrict__ pot,
                                                double* __restrict__ vel, double hh, const NextStep& nx,
                                                const double* __restrict__ emass, double* en) {
  const PState ps = load_state(i, stride, ls, vel, nx, emass, en != nullptr);
  finish_particle(i, stride, a, ls, acc, pot, vel, hh, nx, en, ps);
}

// a[c] += part[(p * NC + c) * n + i] for p = 0 .. S-1 in order (double partial planes of the
// j-split passes). The loads of K splits are issued before their additions, so ceil(S / K)
// memory round trips serve the whole sum while the additions keep the split order; the splits
// past S in the last round add +0.0, which leaves a sum that starts at +0.0 unchanged (in
// round-to-nearest a sum is -0.0 only when both terms are), so the result is that of the plain
// loop for any K.
template <int NC, int K = 16>
__device__ __forceinline__ void sum_splits(const double* __restrict__ part, int64_t n, int64_t i, int32_t S,
                                           double* a) {
  for (int32_t p = 0; p < S; p += K) {
    double v[K][NC];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int32_t q = p + k < S ? p + k : S - 1;  // in bounds: every load issues unconditionally
        const double x = part[((int64_t)q * NC + c) * n + i];
        v[k][c] = p + k < S ? x : 0.0;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] += v[k][c];
  }
}

// Sum of j-split partials (fixed order p = 0..S-1), scaled by the law's constants;
// optional potential and optional closing half-kick v += hh a.
//   part [S][4][n]: planes ax, ay, az, phi of every split.
// Batched form: sys_off (device, n_sys+1) and nsplit (device, n_sys) give the split
// count of the system that owns particle i; single-system form passes n_sys = 0.
// count particles starting at the given pointers; stride = plane stride of part/acc/vel.
__global__ __launch_bounds__(kReduceBS) void reduce_splits(int64_t count, int64_t stride, int32_t S,
                                                          const double* __restrict__ part, LawScale ls,
                                                          double* __restrict__ acc, double* __restrict__ pot,
                                                          double* __restrict__ vel, double hh, int64_t n_sys,
                                                          const int64_t* __restrict__ sys_off,
                                                          const int32_t* __restrict__ nsplit, NextStep nx,
                                                          EnergyFuse ef) {
  const int64_t n = stride;
  auto body = [&](int64_t i, int32_t s_cnt, double* en) {
    const PState ps = load_state(i, n, ls, vel, nx, ef.mass, en != nullptr);
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    sum_splits<4>(part, n, i, s_cnt, a);
    finish_particle(i, n, a, ls, acc, pot, vel, hh, nx, en, ps);
  };
  if (ef.part) {  // grid (chunks, systems)
    const int64_t s = blockIdx.y;
    const int64_t b = n_sys > 0 ? sys_off[s] : 0, e = n_sys > 0 ? sys_off[s + 1] : count;
    const int32_t s_cnt = n_sys > 0 ? nsplit[s] : S;
    energy_chunk(b, e, s, ef, [&](int64_t i, double* en) { body(i, s_cnt, en); });
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int32_t s_cnt = S;
  if (n_sys > 0) {
    int64_t lo = 0, hi = n_sys;  // find s with sys_off[s] <= i < sys_off[s+1]
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (sys_off[mid] <= i) lo = mid; else hi = mid;
    }
    s_cnt = nsplit[lo];
  }
  body(i, s_cnt, nullptr);
}

// ----------------------------------------------------------------- force pair pass

// Launch geometry shared by the single-system and batched drivers.
struct ForceOut {
  // direct mode (part == nullptr): acc = ca*sum/m, pot = cp*sum/m (if pot), vel += hh*acc (if vel)
  double* acc;
  double* pot;
  double* vel;
  double hh;
  LawScale ls;
  // partial mode: part[(slot*4 + c)*n_plane + i] = sum (unscaled)
  double* part;
  int64_t n_plane;
};

// Pair-math modes of the FP32 kernels: plain float sums, compensated sums, compensated
// sums with double-float separations, and (symmetric single-system tiles only) compensated
// sums with double-float separations where two sub-blocks are near (the adaptive mode:
// MODE_ADAPT for the off-diagonal tiles, MODE_ADAPT_DIAG for the diagonal ones, which are
// launched separately so that the double-float diagonal loop does not raise the register
// count, and so lower the occupancy, of the off-diagonal kernel).
enum { MODE_PLAIN = 0, MODE_COMP = 1, MODE_DS = 2, MODE_ADAPT = 3, MODE_ADAPT_DIAG = 4 };

// Inputs of the adaptive mode, all in sorted order (see nbody_adapt.hpp): the low words of
// the double-float coordinates, the bounding box of every 64-particle sub-block
// (box[2q] = min corner, box[2q + 1] = max corner) and T^2, the squared box distance below
// which two sub-blocks take double-float separations.
struct AdaptIn {
  const float4* jlo;
  const float4* box;
  const double* thr;
};

// One block's work: i in [ib, ie) (ie - ib <= BS*I) against j in [jb, je).
// Returns the unscaled sums of every component in res[c][u] (c = ax, ay, az, phi).
template <typename T, int BS, int I, int TJ, bool POT, int MODE, int LAW>
__device__ __forceinline__ void force_block(const typename Vec4<T>::type* __restrict__ jarr,
                                            int64_t ib, int64_t ie, int64_t jb, int64_t je, T eps2_arg,
                                            typename Vec4<T>::type* tile /* [TJ * (DS ? 2 : 1)] */,
                                            double res[4][I]) {
  using V = typename Vec4<T>::type;
  constexpr bool COMP = MODE != MODE_PLAIN;
  constexpr bool DS = MODE == MODE_DS;
  constexpr int NV = DS ? 2 : 1;  // vectors per particle in the j-array
  static_assert(TJ % BS == 0, "TJ must be a multiple of BS");
  static_assert(!DS || sizeof(T) == 4, "double-float separations are a float mode");
  constexpr int PER = TJ / BS;
  const T eps2 = in_vgpr(eps2_arg);
  const int t = threadIdx.x;

  T xi[I], yi[I], zi[I], xl[I], yl[I], zl[I];
  T acc_t[4][I];        // running sum inside the current tile (or whole range if !COMP)
  float hi[4][I], lo[4][I];
  int64_t my_i[I];
#pragma unroll
  for (int u = 0; u < I; ++u) {
    int64_t i = ib + t + (int64_t)u * BS;
    my_i[u] = i;
    int64_t ic = i < ie ? i : ie - 1;  // lanes past the end read a valid particle, results dropped
    V p = jarr[NV * ic];
    xi[u] = in_vgpr(p.x);
    yi[u] = in_vgpr(p.y);
    zi[u] = in_vgpr(p.z);
    if constexpr (DS) {
      V pl = jarr[NV * ic + 1];
      xl[u] = in_vgpr(pl.x);
      yl[u] = in_vgpr(pl.y);
      zl[u] = in_vgpr(pl.z);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) { acc_t[c][u] = T(0); hi[c][u] = 0.f; lo[c][u] = 0.f; }
  }

  V pre[NV * PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int64_t j = jb + t + (int64_t)k * BS;
#pragma unroll
    for (int v = 0; v < NV; ++v) pre[NV * k + v] = load_or(jarr, NV * j + v, j < je, v ? zero4<T>() : pad4<T, LAW>());
  }

  for (int64_t j0 = jb; j0 < je; j0 += TJ) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) tile[NV * (t + k * BS) + v] = pre[NV * k + v];
    __syncthreads();
    if (j0 + TJ < je) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        int64_t j = j0 + TJ + t + (int64_t)k * BS;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          pre[NV * k + v] = load_or(jarr, NV * j + v, j < je, v ? zero4<T>() : pad4<T, LAW>());
      }
    }
    const bool diag = (POT || LAW == LAW_LJ) && (j0 < ie) && (j0 + TJ > ib);
#define NBODY_FORCE_PAIR(MASKED)                                                          \
    {                                                                                     \
      const V q = tile[NV * jj];                                                          \
      V ql;                                                                               \
      if constexpr (DS) ql = tile[NV * jj + 1];                                           \
      _Pragma("unroll") for (int u = 0; u < I; ++u) {                                     \
        T dx = q.x - xi[u], dy = q.y - yi[u], dz = q.z - zi[u];                           \
        if constexpr (DS) {                                                               \
          dx += ql.x - xl[u];                                                             \
          dy += ql.y - yl[u];                                                             \
          dz += ql.z - zl[u];                                                             \
        }                                                                                 \
        T r2 = fmaT(dx, dx, fmaT(dy, dy, fmaT(dz, dz, eps2)));                            \
        if constexpr (LAW == LAW_LJ) {                                                    \
          const T iv = pair_rcp<T>(r2);                                                   \
          const T q6 = (iv * iv) * iv;                                                    \
          T s = (iv * q6) * fmaT(T(-2), q6, T(1));                                        \
          T pv = fmaT(q6, q6, -q6);                                                       \
          if (MASKED) {                                                                   \
            const bool self = (j0 + jj == my_i[u]);                                       \
            s = self ? T(0) : s;                                                          \
            pv = self ? T(0) : pv;                                                        \
          }                                                                               \
          acc_t[0][u] = fmaT(s, dx, acc_t[0][u]);                                         \
          acc_t[1][u] = fmaT(s, dy, acc_t[1][u]);                                         \
          acc_t[2][u] = fmaT(s, dz, acc_t[2][u]);                                         \
          if (POT) acc_t[3][u] += pv;                                                     \
        } else {                                                                          \
          T ri = pair_rsqrt<T>(r2);                                                       \
          T mr = q.w * ri;                                                                \
          T s = (mr * ri) * ri;                                                           \
          acc_t[0][u] = fmaT(s, dx, acc_t[0][u]);                                         \
          acc_t[1][u] = fmaT(s, dy, acc_t[1][u]);                                         \
          acc_t[2][u] = fmaT(s, dz, acc_t[2][u]);                                         \
          if (MASKED) acc_t[3][u] -= (j0 + jj == my_i[u]) ? T(0) : mr;                    \
          else if (POT) acc_t[3][u] -= mr;                                                \
        }                                                                                 \
      }                                                                                   \
    }
    if (!diag) {
#pragma unroll 8
      for (int jj = 0; jj < TJ; ++jj) NBODY_FORCE_PAIR(false)
    } else {
      for (int jj = 0; jj < TJ; ++jj) NBODY_FORCE_PAIR(true)
    }
#undef NBODY_FORCE_PAIR
    if (COMP) {
#pragma unroll
      for (int u = 0; u < I; ++u)
#pragma unroll
        for (int c = 0; c < (POT ? 4 : 3); ++c) {
          float s, e;
          two_sum(hi[c][u], (float)acc_t[c][u], s, e);
          hi[c][u] = s;
          lo[c][u] += e;
          acc_t[c][u] = T(0);
        }
    }
  }
#pragma unroll
  for (int u = 0; u < I; ++u)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      res[c][u] = COMP ? (double)hi[c][u] + (double)lo[c][u] : (double)acc_t[c][u];
}

template <int I>
__device__ __forceinline__ void force_store(const ForceOut& o, int64_t ib, int64_t ie, int slot,
                                            const double res[4][I], bool pot_on, int BS) {
#pragma unroll
  for (int u = 0; u < I; ++u) {
    int64_t i = ib + threadIdx.x + (int64_t)u * BS;
    if (i >= ie) continue;
    if (o.part) {
#pragma unroll
      for (int c = 0; c < 4; ++c) o.part[((int64_t)slot * 4 + c) * o.n_plane + i] = res[c][u];
    } else {
      const double md = law_div(o.ls, i);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double a = o.ls.ca * res[c][u] / md;
        o.acc[c * o.n_plane + i] = a;
        if (o.vel) o.vel[c * o.n_plane + i] += o.hh * a;
      }
      if (pot_on && o.pot) o.pot[i] = o.ls.cp * res[3][u] / md;
    }
  }
}

// Single system (or one i-range of it): grid (ceil(ni / (BS*I)), S).
// Block (bx, by) takes i-range [i0 + bx*BS*I, ...) and the by-th of S j-ranges
// of length jchunk (a multiple of TJ) inside [j0, j1).
template <typename T, int BS, int I, int TJ, bool POT, int MODE, int LAW>
__global__ __launch_bounds__(BS) void force_kernel(const typename Vec4<T>::type* __restrict__ jarr,
                                                   int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                                                   int64_t jchunk, T eps2, ForceOut o) {
  __shared__ typename Vec4<T>::type tile[TJ * (MODE == MODE_DS ? 2 : 1)];
  const int64_t ib = i0 + (int64_t)blockIdx.x * BS * I;
  const int64_t ie = ib + BS * I < i1 ? ib + BS * I : i1;
  const int64_t jb = j0 + (int64_t)blockIdx.y * jchunk;
  const int64_t je = jb + jchunk < j1 ? jb + jchunk : j1;
  double res[4][I];
  force_block<T, BS, I, TJ, POT, MODE, LAW>(jarr, ib, ie, jb, je, eps2, tile, res);
  force_store<I>(o, ib, ie, blockIdx.y, res, POT, BS);
}

// ----------------------------------------------------------------- symmetric force pass (FP32)

// Rotate a wave's values one lane to the right (lane l receives lane l-1, lane 0
// receives lane 63): DPP wave_ror:1, a VALU move with a cross-lane source.
__device__ __forceinline__ float wave_ror1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xF, 0xF, false));
}

// The same rotation through the LDS crossbar (ds_bpermute: no LDS storage, no VALU
// issue slot). src_byte = 4 * ((lane - 1) & 63).
__device__ __forceinline__ float wave_ror1_lds(float v, int src_byte) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_byte, __float_as_int(v)));
}

// ROT: 0 DPP, 1 LDS crossbar, 2 mixed (coordinates and masses through the LDS crossbar, whose
// latency a step ahead hides; the j accumulators, which the next step needs at once, through DPP).
template <int ROT>
__device__ __forceinline__ float rotate1(float v, int src_byte) {
  if constexpr (ROT == 0) return wave_ror1(v);
  else return wave_ror1_lds(v, src_byte);
}
template <int ROT> constexpr int rot_coord() { return ROT == 2 ? 1 : ROT; }
template <int ROT> constexpr int rot_acc() { return ROT == 2 ? 0 : ROT; }

// Tile t of the upper triangle (A <= B) of an nb x nb block grid, row-major:
// row A holds tiles B = A .. nb-1, and rows before A hold A*nb - A*(A-1)/2 tiles.
__device__ __forceinline__ void tile_rc(int64_t t, int32_t nb, int32_t& A, int32_t& B) {
  const double m = 2.0 * nb + 1.0;
  int64_t a = (int64_t)((m - sqrt(m * m - 8.0 * (double)t)) * 0.5);
  if (a < 0) a = 0;
  if (a > nb - 1) a = nb - 1;
  auto start = [&](int64_t r) { return r * nb - r * (r - 1) / 2; };
  while (a > 0 && start(a) > t) --a;
  while (a + 1 < nb && start(a + 1) <= t) ++a;
  A = (int32_t)a;
  B = (int32_t)(a + (t - start(a)));
}

// Each unordered pair once: a_i += m_j r3 d and a_j -= m_i r3 d (r3 = s^{-3/2}), with
// phi_i -= m_j s^{-1/2}, phi_j -= m_i s^{-1/2} - the action-reaction symmetry of the
// pair force halves the separations, square roots and scale factors per interaction.
// Under Lennard-Jones the pair factor k = u q (1 - 2q) carries no mass (the 1/m is
// applied at the end), so a_i += k d and a_j -= k d, and both potentials add q^2 - q.
//
// Blocks of BI = W*64*I consecutive particles; one workgroup per tile (A, B), A <= B.
// Wave w keeps i-particles A*BI + w*64*I + u*64 + lane (u < I) in registers. Block B
// streams through every wave in sub-blocks of 64 particles, one per lane; at each of
// 64 steps a lane pairs its I i-particles with the j-particle it holds, then the
// j-particle and its accumulators move one lane (wave_ror1). After 64 steps every j
// has met every i of the wave and its accumulator is back in its home lane; the W
// waves' j-accumulators are summed in LDS in wave order. Diagonal tiles (A == B) pair
// every i with every j one-sidedly (i-side only, self pair excluded from phi).
//
// Output: float partial sums part[(slot*4 + c)*n + p], c = ax, ay, az, phi: the
// i-side of tile (A, B) goes to slot B, the j-side to slot A, so every particle owns
// exactly nb slots, summed in double (fixed order) by reduce_sym.
//
// One tile (A, B) of a system of n particles (jarr and part point at the system's own
// j-array and partial planes); red is the workgroup's LDS for the cross-wave j sums.
// PIPE chooses when a step's j coordinates are rotated: 0 right after they are consumed
// (phase 1), 1 at the top of the step, a whole step ahead of their use. Both compute the
// same values; which schedules better depends on the variant (measured by the tuner).
//
// Adaptive mode (particles in Morton order): every off-diagonal (wave, sub-block) iteration
// whose i- and j-sub-block boxes lie within T of each other (a bit of the wave's near mask,
// one ballot per tile; MODE_ADAPT) and every diagonal tile (MODE_ADAPT_DIAG) form their
// separations from double-float coordinates, (hi_j - hi_i) + (lo_j - lo_i); all other
// iterations run the compensated float loop unchanged (its low words in LDS, as in the
// potential variant). The double-float loops take part of a lane's i-particles at a time
// (the j-particles come home after 64 steps), so they need no more registers than the float
// loop.
//
// OUT 1 and 2 (the round schedule): instead of writing slots, the tile adds its i-side and j-side
// sums to per-particle double accumulators acc64 [4][n], with a load, add and store (1) or a
// device atomic add (2); the caller runs only tiles whose blocks no other running tile touches.
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE = 0, int OUT = 0>
__device__ __forceinline__ void sym_tile(const float4* __restrict__ jarr, int64_t n, int32_t A, int32_t B,
                                         float eps2_arg, float* __restrict__ part,
                                         float (&red)[2][W][POT ? 4 : 3][64], AdaptIn ad = AdaptIn{},
                                         double* __restrict__ acc64 = nullptr) {
  constexpr bool COMP = MODE != MODE_PLAIN;
  constexpr bool DS = MODE == MODE_DS;
  constexpr bool ADAPT_OFF = MODE == MODE_ADAPT;        // adaptive, off-diagonal tiles only
  constexpr bool ADAPT_DIAG = MODE == MODE_ADAPT_DIAG;  // adaptive, diagonal tiles only
  constexpr bool ADAPT = ADAPT_OFF || ADAPT_DIAG;
  static_assert(!ADAPT || I % 2 == 0, "the adaptive double-float loops take part of the i-particles at a time");
  constexpr int IH = I / 2 > 0 ? I / 2 : 1;   // i-particles per off-diagonal double-float pass
  constexpr int IHD = I / 4 > 0 ? I / 4 : 1;  // i-particles per diagonal pass
  constexpr int NV = DS ? 2 : 1;
  constexpr int BI = W * 64 * I;
  constexpr int NC = POT ? 4 : 3;
  constexpr int NSUB = BI / 64;

  const bool diag = ADAPT_DIAG ? true : ADAPT_OFF ? false : (A == B);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rot_src = ((lane - 1) & 63) << 2;  // rotation source lane (byte address) for ROT = 1
  const int64_t Abase = (int64_t)A * BI, Bbase = (int64_t)B * BI;
  const float eps2 = in_vgpr(eps2_arg);
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 jpad = pad4<float, LAW>();

  // The compensated variant with the potential keeps the low words of its compensated sums
  // in LDS (a lane touches only its own words, once per sub-block), which takes 4I registers
  // out of the pair loop; the arithmetic is that of the register form.
  constexpr bool LO_LDS = COMP && (POT || ADAPT);
  __shared__ float lo_lds[LO_LDS ? W * NC * I * 64 : 1];
  float* const lo_w = lo_lds + (LO_LDS ? w * NC * I * 64 + lane : 0);  // word (c, u): lo_w[(c * I + u) * 64]

  float xi[I], yi[I], zi[I], mi[I], xl[I], yl[I], zl[I];
  float ai[NC][I], hi[NC][I], lo[NC][I];
#pragma unroll
  for (int u = 0; u < I; ++u) {
    const int64_t i = Abase + (int64_t)w * 64 * I + u * 64 + lane;
    const int64_t ic = i < n ? i : n - 1;
    // padding lanes have no j-side effect: no mass (gravity), far away (Lennard-Jones)
    const float4 p = (LAW == LAW_LJ && i >= n) ? jpad : jarr[NV * ic];
    xi[u] = in_vgpr(p.x);
    yi[u] = in_vgpr(p.y);
    zi[u] = in_vgpr(p.z);
    mi[u] = in_vgpr(i < n ? p.w : 0.f);
    if constexpr (DS) {
      const float4 pl = jarr[NV * ic + 1];
      xl[u] = in_vgpr(pl.x);
      yl[u] = in_vgpr(pl.y);
      zl[u] = in_vgpr(pl.z);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ai[c][u] = 0.f;
      hi[c][u] = 0.f;
      if constexpr (LO_LDS) lo_w[(c * I + u) * 64] = 0.f;
      else lo[c][u] = 0.f;
    }
  }

  float4 nxt, nxtl = zero;
  {
    const int64_t j = Bbase + lane;
    nxt = load_or(jarr, NV * j, j < n, jpad);
    if constexpr (DS) nxtl = load_or(jarr, NV * j + 1, j < n, zero);
  }
  // Adaptive mode: bit q of near_mask marks the j-sub-blocks q of block B whose boxes lie
  // within T of one of this wave's I i-sub-blocks (lane q tests sub-block q; off-diagonal
  // tiles have A < B, so block A is full).
  uint64_t near_mask = 0;
  if constexpr (ADAPT_OFF) {
    {
      const float T2 = (float)ad.thr[0];
      const int64_t nsub_all = (n + 63) >> 6;
      const int64_t jq = (int64_t)B * NSUB + lane;
      bool nr = false;
      if (lane < NSUB && jq < nsub_all) {
        const float4 blo = ad.box[2 * jq], bhi = ad.box[2 * jq + 1];
#pragma unroll
        for (int u = 0; u < I; ++u) {
          const int64_t iq = (int64_t)A * NSUB + w * I + u;
          const float4 alo = ad.box[2 * iq], ahi = ad.box[2 * iq + 1];
          const float gx = fmaxf(0.f, fmaxf(blo.x - ahi.x, alo.x - bhi.x));
          const float gy = fmaxf(0.f, fmaxf(blo.y - ahi.y, alo.y - bhi.y));
          const float gz = fmaxf(0.f, fmaxf(blo.z - ahi.z, alo.z - bhi.z));
          nr = nr || (gx * gx + gy * gy + gz * gz < T2);
        }
      }
      near_mask = __ballot(nr);
    }
  }
  // Only the sub-blocks of block B that hold particles are visited (block B is ragged
  // when it is the system's last). Off-diagonal tiles have A < B, so block A is full and
  // every wave has real i-particles; on a diagonal tile a wave whose i-particles are all
  // past the end has nothing to do (that path has no workgroup barrier).
  const int64_t jrows = n - Bbase;
  const int nsub_b = jrows >= BI ? NSUB : (int)((jrows + 63) >> 6);
  const int nsub = (diag && Abase + (int64_t)w * 64 * I >= n) ? 0 : nsub_b;
  for (int sb = 0; sb < nsub; ++sb) {
    const float4 q = nxt, ql = nxtl;
    if (sb + 1 < nsub) {
      const int64_t j = Bbase + (int64_t)(sb + 1) * 64 + lane;
      nxt = load_or(jarr, NV * j, j < n, jpad);
      if constexpr (DS) nxtl = load_or(jarr, NV * j + 1, j < n, zero);
    }
    float xj = q.x, yj = q.y, zj = q.z, mj = q.w, xjl = ql.x, yjl = ql.y, zjl = ql.z;
    if (ADAPT_DIAG) {
      // one-sided with double-float separations, a quarter of the i-particles at a time; the
      // self pair is the step-0 pair of sub-block w*I + u
      const int64_t jq = Bbase + (int64_t)sb * 64 + lane;
      const float4 qlo = load_or(ad.jlo, jq, jq < n, zero);
      float xjo = qlo.x, yjo = qlo.y, zjo = qlo.z;
#pragma unroll
      for (int h = 0; h < I / IHD; ++h) {
        float xio[IHD], yio[IHD], zio[IHD];
#pragma unroll
        for (int v = 0; v < IHD; ++v) {
          const int64_t i = Abase + (int64_t)w * 64 * I + (h * IHD + v) * 64 + lane;
          const float4 l = ad.jlo[i < n ? i : n - 1];
          xio[v] = l.x;
          yio[v] = l.y;
          zio[v] = l.z;
        }
        for (int k = 0; k < 64; ++k) {
#pragma unroll
          for (int v = 0; v < IHD; ++v) {
            const int u = h * IHD + v;
            const float dx = (xj - xi[u]) + (xjo - xio[v]);
            const float dy = (yj - yi[u]) + (yjo - yio[v]);
            const float dz = (zj - zi[u]) + (zjo - zio[v]);
            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
            const bool self = (k == 0 && sb == w * I + u);
            if constexpr (LAW == LAW_LJ) {
              const float iv = __builtin_amdgcn_rcpf(r2);
              const float q6 = (iv * iv) * iv;
              float sv = (iv * q6) * __builtin_fmaf(-2.f, q6, 1.f);
              sv = self ? 0.f : sv;
              ai[0][u] = __builtin_fmaf(sv, dx, ai[0][u]);
              ai[1][u] = __builtin_fmaf(sv, dy, ai[1][u]);
              ai[2][u] = __builtin_fmaf(sv, dz, ai[2][u]);
              if constexpr (POT) ai[3][u] += self ? 0.f : __builtin_fmaf(q6, q6, -q6);
            } else {
              const float ri = __builtin_amdgcn_rsqf(r2);
              const float mr = mj * ri;
              const float sv = (mr * ri) * ri;
              ai[0][u] = __builtin_fmaf(sv, dx, ai[0][u]);
              ai[1][u] = __builtin_fmaf(sv, dy, ai[1][u]);
              ai[2][u] = __builtin_fmaf(sv, dz, ai[2][u]);
              if constexpr (POT) ai[3][u] = self ? ai[3][u] : __builtin_fmaf(-mj, ri, ai[3][u]);
            }
          }
          xj = rotate1<rot_coord<ROT>()>(xj, rot_src);
          yj = rotate1<rot_coord<ROT>()>(yj, rot_src);
          zj = rotate1<rot_coord<ROT>()>(zj, rot_src);
          mj = rotate1<rot_coord<ROT>()>(mj, rot_src);
          xjo = rotate1<rot_coord<ROT>()>(xjo, rot_src);
          yjo = rotate1<rot_coord<ROT>()>(yjo, rot_src);
          zjo = rotate1<rot_coord<ROT>()>(zjo, rot_src);
        }
      }
    } else if (diag) {
      // one-sided: i-side only; the self pair is the step-0 pair of sub-block w*I + u
      for (int k = 0; k < 64; ++k) {
#pragma unroll
        for (int u = 0; u < I; ++u) {
          float dx = xj - xi[u], dy = yj - yi[u], dz = zj - zi[u];
          if constexpr (DS) {
            dx += xjl - xl[u];
            dy += yjl - yl[u];
            dz += zjl - zl[u];
          }
          const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
          if constexpr (LAW == LAW_LJ) {
            const bool self = (k == 0 && sb == w * I + u);
            const float iv = __builtin_amdgcn_rcpf(r2);
            const float q6 = (iv * iv) * iv;
            float s = (iv * q6) * __builtin_fmaf(-2.f, q6, 1.f);
            s = self ? 0.f : s;
            ai[0][u] = __builtin_fmaf(s, dx, ai[0][u]);
            ai[1][u] = __builtin_fmaf(s, dy, ai[1][u]);
            ai[2][u] = __builtin_fmaf(s, dz, ai[2][u]);
            if constexpr (POT) ai[3][u] += self ? 0.f : __builtin_fmaf(q6, q6, -q6);
          } else {
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float mr = mj * ri;
            const float s = (mr * ri) * ri;
            ai[0][u] = __builtin_fmaf(s, dx, ai[0][u]);
            ai[1][u] = __builtin_fmaf(s, dy, ai[1][u]);
            ai[2][u] = __builtin_fmaf(s, dz, ai[2][u]);
            // explicitly fused, as in the two-sided loop: an implicit contraction would depend on
            // how the compiler unrolls the loop (the self test folds away in later copies)
            if (POT) ai[3][u] = (k == 0 && sb == w * I + u) ? ai[3][u] : __builtin_fmaf(-mj, ri, ai[3][u]);
          }
        }
        xj = rotate1<rot_coord<ROT>()>(xj, rot_src);
        yj = rotate1<rot_coord<ROT>()>(yj, rot_src);
        zj = rotate1<rot_coord<ROT>()>(zj, rot_src);
        mj = rotate1<rot_coord<ROT>()>(mj, rot_src);
        if constexpr (DS) {
          xjl = rotate1<rot_coord<ROT>()>(xjl, rot_src);
          yjl = rotate1<rot_coord<ROT>()>(yjl, rot_src);
          zjl = rotate1<rot_coord<ROT>()>(zjl, rot_src);
        }
      }
    } else {
      float aj[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) aj[c] = 0.f;
      bool near_done = false;
      if constexpr (ADAPT_OFF) {
        if ((near_mask >> sb) & 1) {
          // double-float separations for this near sub-block pair, half of the i-particles at a
          // time; the j accumulators keep adding across both halves (they come home after 64
          // steps), the pair terms are those of the float loop below
          const int64_t jq = Bbase + (int64_t)sb * 64 + lane;
          const float4 qlo = load_or(ad.jlo, jq, jq < n, zero);
          float xjo = qlo.x, yjo = qlo.y, zjo = qlo.z;
          // the lane index through an opaque move: the addresses are formed here, not hoisted out
          // of the sub-block loop into registers the float loop would then have to carry
          const float4* lrow = ad.jlo + Abase + (int64_t)w * 64 * I + opaque_int(lane);
#pragma unroll
          for (int h = 0; h < I / IH; ++h) {
            float xio[IH], yio[IH], zio[IH];
#pragma unroll
            for (int v = 0; v < IH; ++v) {
              const float4 l = lrow[(h * IH + v) * 64];
              xio[v] = l.x;
              yio[v] = l.y;
              zio[v] = l.z;
            }
            for (int k = 0; k < 64; ++k) {
              float dx[IH], dy[IH], dz[IH], ri[IH];
#pragma unroll
              for (int v = 0; v < IH; ++v) {
                const int u = h * IH + v;
                dx[v] = (xj - xi[u]) + (xjo - xio[v]);
                dy[v] = (yj - yi[u]) + (yjo - yio[v]);
                dz[v] = (zj - zi[u]) + (zjo - zio[v]);
                ri[v] = __builtin_fmaf(dx[v], dx[v], __builtin_fmaf(dy[v], dy[v], __builtin_fmaf(dz[v], dz[v], eps2)));
              }
              const float xn = rotate1<rot_coord<ROT>()>(xj, rot_src), yn = rotate1<rot_coord<ROT>()>(yj, rot_src), zn = rotate1<rot_coord<ROT>()>(zj, rot_src);
              const float xno = rotate1<rot_coord<ROT>()>(xjo, rot_src), yno = rotate1<rot_coord<ROT>()>(yjo, rot_src),
                          zno = rotate1<rot_coord<ROT>()>(zjo, rot_src);
#pragma unroll
              for (int v = 0; v < IH; ++v)
                ri[v] = LAW == LAW_LJ ? __builtin_amdgcn_rcpf(ri[v]) : __builtin_amdgcn_rsqf(ri[v]);
#pragma unroll
              for (int v = 0; v < IH; ++v) {
                const int u = h * IH + v;
                if constexpr (LAW == LAW_LJ) {
                  const float q6 = (ri[v] * ri[v]) * ri[v];
                  const float kf = (ri[v] * q6) * __builtin_fmaf(-2.f, q6, 1.f);
                  if constexpr (POT) {
                    const float pv = __builtin_fmaf(q6, q6, -q6);
                    ai[3][u] += pv;
                    aj[3] += pv;
                  }
                  ai[0][u] = __builtin_fmaf(kf, dx[v], ai[0][u]);
                  ai[1][u] = __builtin_fmaf(kf, dy[v], ai[1][u]);
                  ai[2][u] = __builtin_fmaf(kf, dz[v], ai[2][u]);
                  aj[0] = __builtin_fmaf(-kf, dx[v], aj[0]);
                  aj[1] = __builtin_fmaf(-kf, dy[v], aj[1]);
                  aj[2] = __builtin_fmaf(-kf, dz[v], aj[2]);
                } else {
                  const float r3 = ri[v] * (ri[v] * ri[v]);
                  const float si = mj * r3;
                  const float sj = mi[u] * r3;
                  if constexpr (POT) {
                    ai[3][u] = __builtin_fmaf(-mj, ri[v], ai[3][u]);
                    aj[3] = __builtin_fmaf(-mi[u], ri[v], aj[3]);
                  }
                  ai[0][u] = __builtin_fmaf(si, dx[v], ai[0][u]);
                  ai[1][u] = __builtin_fmaf(si, dy[v], ai[1][u]);
                  ai[2][u] = __builtin_fmaf(si, dz[v], ai[2][u]);
                  aj[0] = __builtin_fmaf(-sj, dx[v], aj[0]);
                  aj[1] = __builtin_fmaf(-sj, dy[v], aj[1]);
                  aj[2] = __builtin_fmaf(-sj, dz[v], aj[2]);
                }
              }
              xj = xn;
              yj = yn;
              zj = zn;
              xjo = xno;
              yjo = yno;
              zjo = zno;
              mj = rotate1<rot_coord<ROT>()>(mj, rot_src);
#pragma unroll
              for (int c = 0; c < NC; ++c) aj[c] = rotate1<rot_acc<ROT>()>(aj[c], rot_src);
            }
          }
          near_done = true;
        }
      }
      // Potential variant: no LDS operation is left in flight when the step loop starts (a wait for
      // lgkmcnt = 0, gfx9 encoding), so the compiler's waits inside the loop need to cover only the
      // loop's own rotations (measured 1.6% faster at N = 1M; the variant without the potential
      // gains nothing from it and keeps the compiler's code).
      if constexpr (POT && LAW == LAW_GRAV) __builtin_amdgcn_s_waitcnt(0xc07f);
      for (int k = 0; k < (near_done ? 0 : 64); ++k) {
        float xn = xj, yn = yj, zn = zj, xnl = xjl, ynl = yjl, znl = zjl;
        if constexpr (PIPE == 1) {  // the next step's coordinates, requested a step ahead
          xn = rotate1<rot_coord<ROT>()>(xj, rot_src);
          yn = rotate1<rot_coord<ROT>()>(yj, rot_src);
          zn = rotate1<rot_coord<ROT>()>(zj, rot_src);
          if constexpr (DS) {
            xnl = rotate1<rot_coord<ROT>()>(xjl, rot_src);
            ynl = rotate1<rot_coord<ROT>()>(yjl, rot_src);
            znl = rotate1<rot_coord<ROT>()>(zjl, rot_src);
          }
        }
        // phase 1: separations and r^2 of the I pairs; phase 2: their square roots;
        // phase 3: scale factors and accumulation - independent work behind every rsq
        float dx[I], dy[I], dz[I], ri[I];
#pragma unroll
        for (int u = 0; u < I; ++u) {
          dx[u] = xj - xi[u];
          dy[u] = yj - yi[u];
          dz[u] = zj - zi[u];
          if constexpr (DS) {
            dx[u] += xjl - xl[u];
            dy[u] += yjl - yl[u];
            dz[u] += zjl - zl[u];
          }
          ri[u] = __builtin_fmaf(dx[u], dx[u], __builtin_fmaf(dy[u], dy[u], __builtin_fmaf(dz[u], dz[u], eps2)));
        }
        if constexpr (PIPE == 0) {  // consumed: pass them on while phases 2 and 3 run
          xn = rotate1<rot_coord<ROT>()>(xj, rot_src);
          yn = rotate1<rot_coord<ROT>()>(yj, rot_src);
          zn = rotate1<rot_coord<ROT>()>(zj, rot_src);
          if constexpr (DS) {
            xnl = rotate1<rot_coord<ROT>()>(xjl, rot_src);
            ynl = rotate1<rot_coord<ROT>()>(yjl, rot_src);
            znl = rotate1<rot_coord<ROT>()>(zjl, rot_src);
          }
        }
#pragma unroll
        for (int u = 0; u < I; ++u) ri[u] = LAW == LAW_LJ ? __builtin_amdgcn_rcpf(ri[u]) : __builtin_amdgcn_rsqf(ri[u]);
        // With the potential, left to itself the compiler starts the accumulation after the first
        // square roots, where it waits on the j-accumulators' rotation issued just before; all
        // square roots first leaves that rotation most of a step (measured 1.3-2.5% faster at
        // N = 1M; the pass without the potential is fastest as the compiler schedules it).
        if constexpr (POT && LAW == LAW_GRAV) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < I; ++u) {
          if constexpr (LAW == LAW_LJ) {
            const float q6 = (ri[u] * ri[u]) * ri[u];
            const float kf = (ri[u] * q6) * __builtin_fmaf(-2.f, q6, 1.f);
            if constexpr (POT) {
              const float pv = __builtin_fmaf(q6, q6, -q6);
              ai[3][u] += pv;
              aj[3] += pv;
            }
            ai[0][u] = __builtin_fmaf(kf, dx[u], ai[0][u]);
            ai[1][u] = __builtin_fmaf(kf, dy[u], ai[1][u]);
            ai[2][u] = __builtin_fmaf(kf, dz[u], ai[2][u]);
            aj[0] = __builtin_fmaf(-kf, dx[u], aj[0]);
            aj[1] = __builtin_fmaf(-kf, dy[u], aj[1]);
            aj[2] = __builtin_fmaf(-kf, dz[u], aj[2]);
            continue;
          }
          // the acceleration terms round identically with and without the potential,
          // so both variants give bitwise-equal accelerations (trajectories must not
          // depend on whether an energy trace is taken)
          const float r3 = ri[u] * (ri[u] * ri[u]);
          const float si = mj * r3;
          const float sj = mi[u] * r3;
          if (POT) {
            ai[3][u] = __builtin_fmaf(-mj, ri[u], ai[3][u]);
            aj[3] = __builtin_fmaf(-mi[u], ri[u], aj[3]);
          }
          ai[0][u] = __builtin_fmaf(si, dx[u], ai[0][u]);
          ai[1][u] = __builtin_fmaf(si, dy[u], ai[1][u]);
          ai[2][u] = __builtin_fmaf(si, dz[u], ai[2][u]);
          aj[0] = __builtin_fmaf(-sj, dx[u], aj[0]);
          aj[1] = __builtin_fmaf(-sj, dy[u], aj[1]);
          aj[2] = __builtin_fmaf(-sj, dz[u], aj[2]);
        }
        xj = xn;
        yj = yn;
        zj = zn;
        if constexpr (DS) {
          xjl = xnl;
          yjl = ynl;
          zjl = znl;
        }
        mj = rotate1<rot_coord<ROT>()>(mj, rot_src);
#pragma unroll
        for (int c = 0; c < NC; ++c) aj[c] = rotate1<rot_acc<ROT>()>(aj[c], rot_src);
      }
      // j-side of this sub-block: sum the W waves in wave order, write slot A
#pragma unroll
      for (int c = 0; c < NC; ++c) red[sb & 1][w][c][lane] = aj[c];
      __syncthreads();
      for (int idx = threadIdx.x; idx < NC * 64; idx += W * 64) {  // any W, any NC
        const int c = idx >> 6, l = idx & 63;
        float sum = 0.f;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) sum += red[sb & 1][ww][c][l];
        const int64_t j = Bbase + (int64_t)sb * 64 + l;
        if constexpr (OUT == 0) {
          if (j < n) part[((int64_t)A * 4 + c) * n + j] = sum;
        } else if constexpr (OUT == 1) {
          if (j < n) acc64[(int64_t)c * n + j] += (double)sum;
        } else {
          if (j < n) unsafeAtomicAdd(acc64 + (int64_t)c * n + j, (double)sum);
        }
      }
    }
    if (COMP) {
#pragma unroll
      for (int u = 0; u < I; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          float s, e;
          two_sum(hi[c][u], ai[c][u], s, e);
          hi[c][u] = s;
          if constexpr (LO_LDS) lo_w[(c * I + u) * 64] += e;
          else lo[c][u] += e;
          ai[c][u] = 0.f;
        }
    }
  }
  // i-side of the tile: slot B
#pragma unroll
  for (int u = 0; u < I; ++u) {
    const int64_t i = Abase + (int64_t)w * 64 * I + u * 64 + lane;
    if (i < n)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if constexpr (OUT == 0)
          part[((int64_t)B * 4 + c) * n + i] =
              COMP ? hi[c][u] + (LO_LDS ? lo_w[(c * I + u) * 64] : lo[c][u]) : ai[c][u];
        else if constexpr (OUT == 1)
          acc64[(int64_t)c * n + i] +=
              COMP ? (double)hi[c][u] + (double)(LO_LDS ? lo_w[(c * I + u) * 64] : lo[c][u]) : (double)ai[c][u];
        else
          unsafeAtomicAdd(acc64 + (int64_t)c * n + i, COMP ? (double)hi[c][u] + (double)(LO_LDS ? lo_w[(c * I + u) * 64] : lo[c][u])
                                                            : (double)ai[c][u]);
      }
  }
}

// Single system: one workgroup per tile t of the nb(nb+1)/2 upper-triangle tiles.
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
__global__ __launch_bounds__(W * 64) void force_sym_kernel(const float4* __restrict__ jarr, int64_t n, int32_t nb,
                                                           float eps2_arg, float* __restrict__ part, AdaptIn ad) {
  __shared__ float red[2][W][POT ? 4 : 3][64];
  int32_t A, B;
  if constexpr (MODE == MODE_ADAPT_DIAG) {  // one workgroup per diagonal tile
    A = B = (int32_t)blockIdx.x;
  } else if constexpr (MODE == MODE_ADAPT) {  // the nb (nb - 1) / 2 off-diagonal tiles
    tile_rc(blockIdx.x, nb - 1, A, B);
    ++B;
  } else {
    tile_rc(blockIdx.x, nb, A, B);
  }
  sym_tile<W, I, POT, MODE, ROT, LAW, PIPE>(jarr, n, A, B, eps2_arg, part, red, ad);
}

// The round schedule of the symmetric pass (workspace linear in n). Round r in [0, nbr - 2] is
// the circle-method pairing of nbr (even) blocks: tile t pairs (r, nbr - 1) for t = 0 and
// ((r + t) mod (nbr - 1), (r - t) mod (nbr - 1)) for t > 0, so every unordered pair of distinct
// blocks meets in exactly one round and the tiles of a round touch disjoint blocks. A launch
// runs the rounds r0 .. r0 + gridDim.y - 1 (grid (nbr / 2, rounds), blockIdx.y = r - r0), round
// r adding into its own copy of [4][n] double accumulators, acc64 + (r - r0) [4][n], so no two
// tiles of a launch touch the same accumulator word and each word takes exactly one add per
// launch: a device atomic add (the same IEEE double addition) that no wave waits for. Launches
// that reuse copies run one after the other, so every accumulator takes its tiles in a fixed
// order and the result is deterministic. A pair with the padding block nb (odd nb) is skipped.
// MODE_ADAPT: particles in Morton order, ad as in the slot schedule.
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
__global__ __launch_bounds__(W * 64) void force_sym_round_kernel(const float4* __restrict__ jarr, int64_t n,
                                                                 int32_t nb, int32_t nbr, int32_t r0,
                                                                 float eps2_arg, double* __restrict__ acc64,
                                                                 AdaptIn ad) {
  __shared__ float red[2][W][POT ? 4 : 3][64];
  const int32_t r = r0 + (int32_t)blockIdx.y;
  if (r >= nbr - 1) return;  // past the last round (the whole workgroup)
  acc64 += (int64_t)blockIdx.y * 4 * n;
  const int32_t m = nbr - 1, t = (int32_t)blockIdx.x;
  const int32_t a = t == 0 ? r : (r + t) % m;
  const int32_t b = t == 0 ? m : (r - t + m) % m;
  const int32_t A = a < b ? a : b, B = a < b ? b : a;
  if (B >= nb) return;  // the padding block of an odd block count (the whole workgroup)
  sym_tile<W, I, POT, MODE, ROT, LAW, PIPE, 2>(jarr, n, A, B, eps2_arg, nullptr, red, ad, acc64);
}

// The diagonal tiles (A, A) of the round schedule, one workgroup per block, before any round: a
// diagonal tile adds both sides of its sums to the same accumulators, with loads, adds and stores
// in program order. The adaptive mode launches its MODE_ADAPT_DIAG form.
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
__global__ __launch_bounds__(W * 64) void force_sym_round_diag_kernel(const float4* __restrict__ jarr, int64_t n,
                                                                      float eps2_arg, double* __restrict__ acc64,
                                                                      AdaptIn ad) {
  __shared__ float red[2][W][POT ? 4 : 3][64];
  const int32_t A = (int32_t)blockIdx.x;
  sym_tile<W, I, POT, MODE, ROT, LAW, PIPE, 1>(jarr, n, A, A, eps2_arg, nullptr, red, ad, acc64);
}

// The end of the round schedule: the sums at position p are the K accumulator copies
// acc64[k][c][p], added in copy order. perm (nullable): positions are in sorted order (the
// adaptive mode) and position p holds particle perm[p], whose outputs are written at its own index.
__global__ __launch_bounds__(kReduceBS) void reduce_rounds(int64_t n, int64_t stride, const double* __restrict__ acc64,
                                                           int32_t K, LawScale ls, double* __restrict__ acc,
                                                           double* __restrict__ pot, double* __restrict__ vel,
                                                           double hh, NextStep nx, EnergyFuse ef,
                                                           const uint32_t* __restrict__ perm) {
  auto body = [&](int64_t p, double* en) {
    const int64_t i = perm ? (int64_t)perm[p] : p;
    const PState ps = load_state(i, stride, ls, vel, nx, ef.mass, en != nullptr);
    double a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      a[c] = 0.0;
      if (c == 3 && !pot) continue;
      const double* q = acc64 + (int64_t)c * n + p;
      const int64_t cs = 4 * n;  // one copy
      double t = q[0];
      for (int k = 1; k < K; ++k) t += q[k * cs];
      a[c] = t;
    }
    finish_particle(i, stride, a, ls, acc, pot, vel, hh, nx, en, ps);
  };
  if (ef.part) {  // grid (chunks, 1)
    energy_chunk(0, n, 0, ef, body);
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) body(i, nullptr);
}

// ----------------------------------------------------------------- symmetric pass: per-particle reduction

// Sum of the nb float slots of every particle in double (fixed order), scaled by the
// law's constants; optional potential and closing half-kick.
// n: particles of the system (partial plane stride); stride: plane stride of acc/vel.
// a[c] += slot s of component c, s = 0 .. nb-1 in order, for the particle at offset i of
// planes of stride n (slot s, component c at (s * 4 + c) * n). The loads of K slots are issued
// before their additions, so ceil(nb / K) memory round trips serve the sum (the single-system
// reductions run few waves for small systems and are bound by those round trips) while the
// additions keep the slot order; slots past nb in the last round add +0.0, which leaves the sum
// unchanged (it starts at +0.0 and is never -0.0 in round-to-nearest), so the result is that of
// the plain loop for any K. Kernels that share their registers with a pair loop take K = 1.
template <int NC, int K = 32>
__device__ __forceinline__ void sum_slots(const float* __restrict__ part, int64_t n, int64_t i, int32_t nb,
                                          double a[4]) {
  for (int32_t s = 0; s < nb; s += K) {
    float v[K][NC];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int32_t q = s + k < nb ? s + k : nb - 1;  // in bounds: every load issues unconditionally
        const float x = part[((int64_t)q * 4 + c) * n + i];
        v[k][c] = s + k < nb ? x : 0.f;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] += (double)v[k][c];
  }
}

// The single-system slot sums in four interleaved groups: group g of the particle at offset i
// sums slots g, g + 4, g + 8, ... (< nb) in order, in double; the particle's sum is then
// (p0 + p1) + (p2 + p3). The loads of K slots of the group are issued before their additions;
// slots past nb in the last round are loaded from a valid slot and replaced by +0.0 (exact, as in
// sum_slots).
template <int NC, int K = 16>
__device__ __forceinline__ void sum_slot_group(const float* __restrict__ part, int64_t n, int64_t i, int32_t nb,
                                               int g, double p[4]) {
  for (int32_t s0 = g; s0 < nb; s0 += 4 * K) {
    float v[K][NC];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int32_t s = s0 + 4 * k;
        const float x = part[((int64_t)(s < nb ? s : s0) * 4 + c) * n + i];
        v[k][c] = s < nb ? x : 0.f;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) p[c] += (double)v[k][c];
  }
}

// perm (nullable): the slot planes are in sorted order (the adaptive mode) and position p
// holds particle perm[p], whose outputs are written at its own index.
// Without the energy: blocks of four waves for 64 positions, wave g summing slot group g; wave 0
// adds the four groups and finishes the particle (a grid of ceil(n / 64) blocks: four times the
// waves of one thread per particle, a quarter of the dependent loads each, which at small n,
// where the sum is bound by memory round trips, takes most of its time away).
// With the energy fused: the same four waves over each turn of an energy chunk (grid: the
// chunks), wave 0 also adding the particle's energy terms with the thread map and block sum of
// energy_partial; the same sums in the same order (so trajectories do not depend on whether the
// energy is traced, and the energy is bitwise the separate pass's).
__global__ __launch_bounds__(kReduceBS) void reduce_sym(int64_t n, int64_t stride, int32_t nb,
                                                       const float* __restrict__ part, LawScale ls,
                                                       double* __restrict__ acc, double* __restrict__ pot,
                                                       double* __restrict__ vel, double hh, NextStep nx,
                                                       EnergyFuse ef, const uint32_t* __restrict__ perm) {
  static_assert(kReduceBS == 256, "four waves of 64 positions");
  static_assert(kEnergyBS == 64, "one wave of positions per energy chunk");
  __shared__ double sh[3][4][64];
  const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (ef.part) {  // grid (chunks, 1): each turn the chunk's 64 positions, in four slot groups
    double en[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t base = (int64_t)blockIdx.x * kEnergyBS; base < n; base += (int64_t)ef.chunks * kEnergyBS) {
      const int64_t p = base + lane;  // the particle energy_partial's thread `lane` takes in this turn
      const bool live = p < n;
      double q[4] = {0.0, 0.0, 0.0, 0.0};
      if (live) {
        if (pot) sum_slot_group<4>(part, n, p, nb, g, q);
        else sum_slot_group<3>(part, n, p, nb, g, q);
      }
      if (g > 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[g - 1][c][lane] = q[c];
      __syncthreads();
      if (g == 0 && live) {
        const int64_t i = perm ? (int64_t)perm[p] : p;
        const PState ps = load_state(i, stride, ls, vel, nx, ef.mass, true);
        double a[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = (q[c] + sh[0][c][lane]) + (sh[1][c][lane] + sh[2][c][lane]);
        finish_particle(i, stride, a, ls, acc, pot, vel, hh, nx, en, ps);
      }
      __syncthreads();  // sh is rewritten by the next turn
    }
    if (g == 0) {  // the chunk's sum as block_sum<kEnergyBS, 5>: the wave by shuffles, then 0 + it
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        double x = en[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) ef.part[(int64_t)blockIdx.x * 5 + c] = 0.0 + x;
      }
    }
    return;
  }
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool live = p < n;
  int64_t i = 0;
  PState ps{};
  if (g == 0 && live) {
    i = perm ? (int64_t)perm[p] : p;
    ps = load_state(i, stride, ls, vel, nx, ef.mass, false);
  }
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  if (live) {
    if (pot) sum_slot_group<4>(part, n, p, nb, g, q);
    else sum_slot_group<3>(part, n, p, nb, g, q);
  }
  if (g > 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[g - 1][c][lane] = q[c];
  __syncthreads();
  if (g == 0 && live) {
    double a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (q[c] + sh[0][c][lane]) + (sh[1][c][lane] + sh[2][c][lane]);
    finish_particle(i, stride, a, ls, acc, pot, vel, hh, nx, nullptr, ps);
  }
}

// ----------------------------------------------------------------- batched symmetric pass

// One symmetric work unit: tile (A, B) of the system whose particles start at global
// index base; its partial planes ([nb][4][n] floats) start at float offset part_off.
struct SymUnit {
  int64_t base;
  int64_t part_off;
  int32_t n, nb;
  int32_t A, B;
  int32_t sys;  // index of the system
  int32_t pad;
};

// One workgroup per symmetric tile of many systems (units sorted by decreasing cost on the
// host, started in index order, as force_batched_kernel). Each tile writes its own partial
// slots, so the result does not depend on the order in which they ran.
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
__global__ __launch_bounds__(W * 64) void force_sym_batched_kernel(const float4* __restrict__ jarr,
                                                                   const SymUnit* __restrict__ units,
                                                                   int32_t n_units, float eps2_arg,
                                                                   float* __restrict__ part) {
  constexpr int NV = MODE == MODE_DS ? 2 : 1;
  __shared__ float red[2][W][POT ? 4 : 3][64];
  if ((int32_t)blockIdx.x >= n_units) return;
  const SymUnit su = units[blockIdx.x];
  sym_tile<W, I, POT, MODE, ROT, LAW, PIPE>(jarr + NV * su.base, su.n, su.A, su.B, eps2_arg, part + su.part_off, red);
}

// Per-particle sum of the batched symmetric partials: particle i of system s (found by
// binary search in sys_off) sums the nb_s float slots of its system's planes in double.
__global__ __launch_bounds__(kReduceBS) void reduce_sym_batched(int64_t n, int64_t n_sys,
                                                               const int64_t* __restrict__ sys_off,
                                                               const int32_t* __restrict__ sys_nb,
                                                               const int64_t* __restrict__ sys_part,
                                                               const float* __restrict__ part, LawScale ls,
                                                               double* __restrict__ acc, double* __restrict__ pot,
                                                               double* __restrict__ vel, double hh, NextStep nx,
                                                               EnergyFuse ef) {
  auto body = [&](int64_t i, int64_t s, double* en) {
    const int64_t b = sys_off[s], ns = sys_off[s + 1] - b, li = i - b;
    const int32_t nb = sys_nb[s];
    const float* pp = part + sys_part[s];
    const PState st = load_state(i, n, ls, vel, nx, ef.mass, en != nullptr);
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (pot) sum_slots<4, 1>(pp, ns, li, nb, a);
    else sum_slots<3, 1>(pp, ns, li, nb, a);
    finish_particle(i, n, a, ls, acc, pot, vel, hh, nx, en, st);
  };
  if (ef.part) {  // grid (chunks, systems)
    const int64_t s = blockIdx.y;
    energy_chunk(sys_off[s], sys_off[s + 1], s, ef, [&](int64_t i, double* en) { body(i, s, en); });
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t lo = 0, hi = n_sys;  // s with sys_off[s] <= i < sys_off[s+1]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (sys_off[mid] <= i) lo = mid; else hi = mid;
  }
  body(i, lo, nullptr);
}

// ----------------------------------------------------------------- whole batched rollout in one launch

// Synchronisation words of the whole-rollout kernel (device memory, zero at launch).
//   queue: next task; err: set when a wait gives up; tiles_done[s]: tiles of system s
//   finished over all steps so far; red_done[s]: per-particle reductions of system s
//   finished (the steps whose end state is written and, but for the last, staged).
struct RolloutSync {
  unsigned long long* queue;
  int32_t* err;
  int32_t* tiles_done;
  int32_t* red_done;
  int64_t spin_limit;  // probes before a wait gives up
};

// Bounded wait of one thread for *p >= v: agent-scope loads, each followed by a short sleep;
// gives up (and sets err) after limit probes, or when another workgroup has given up.
__device__ __forceinline__ bool wait_at_least(const int32_t* p, int32_t v, int32_t* err, int64_t limit) {
  for (int64_t k = 0; k < limit; ++k) {
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= v) return true;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return false;
}

constexpr int32_t kRolloutChunk = 8192;  // particles of one reduction task

// End of a task: every thread fences its own writes (device scope), the workgroup meets,
// and one thread counts the task done. (Weaker forms, one fence per workgroup or
// release/acquire-only fences, gave wrong results across the XCDs.)
__device__ __forceinline__ void release_to(int32_t* counter) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(counter, 1);
}

// Every step of a batched symmetric rollout in one launch (no potential). The task queue
// holds first the n_solo systems of one tile (units[0, n_solo)), each run for all its steps
// by the workgroup that takes it: tile, per-particle reduction and staging, separated by
// workgroup barriers only. Then, step by step, the tiles of the systems of several tiles
// (units[n_solo, n_solo + n_units), the host's order) and their per-particle reductions in
// chunks of kRolloutChunk particles (rtasks: pairs of system and chunk index). A tile of
// such a system s at step t > 0 first waits for every reduction chunk (s, t - 1), which
// staged its positions; a reduction chunk (s, t) waits for all tiles (s, t). Each wait is
// for a task earlier in the queue, already taken by a running workgroup, so every wait
// ends; each is bounded besides. A reduction does for its particles what
// reduce_sym_batched does (slots summed in the same order, acceleration, closing kick, and
// for t + 1 < steps the next step's kick, drift, walls and staging), so the trajectory is
// bitwise that of one launch per pass.
template <int W, int I, int MODE, int ROT, int LAW, int PIPE>
__global__ __launch_bounds__(W * 64) void rollout_sym_batched_kernel(
    const float4* __restrict__ jarr, const SymUnit* __restrict__ units, int32_t n_solo, int32_t n_units,
    const int32_t* __restrict__ rtasks, int32_t n_rtasks, int64_t n, const int64_t* __restrict__ sys_off,
    const int32_t* __restrict__ sys_nb, const int64_t* __restrict__ sys_part, float eps2_arg,
    float* __restrict__ part, LawScale ls, double* __restrict__ acc, double* __restrict__ vel, double hh, NextStep nx,
    int32_t steps, RolloutSync sy) {
  constexpr int NV = MODE == MODE_DS ? 2 : 1;
  __shared__ float red[2][W][3][64];
  __shared__ int64_t task_sh;
  __shared__ int32_t ok_sh;
  const int64_t per_step = (int64_t)n_units + n_rtasks;
  const int64_t total = n_solo + per_step * steps;
  for (;;) {
    __syncthreads();  // everyone has read the previous task (and finished with the LDS sums)
    if (threadIdx.x == 0) {
      const int64_t q = (int64_t)atomicAdd(sy.queue, 1ull);
      const bool stop = q >= total || __hip_atomic_load(sy.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      task_sh = stop ? -1 : q;
    }
    __syncthreads();
    const int64_t q0 = task_sh;
    if (q0 < 0) break;
    if (q0 < n_solo) {  // a system of one tile, all its steps
      const SymUnit su = units[q0];
      const float4* js = jarr + NV * su.base;
      float* ps = part + su.part_off;
      for (int32_t t = 0; t < steps; ++t) {
        sym_tile<W, I, false, MODE, ROT, LAW, PIPE>(js, su.n, 0, 0, eps2_arg, ps, red);
        __syncthreads();  // the tile's partial sums, from every wave
        NextStep nxt = nx;
        if (t + 1 >= steps) nxt.kind = 0;  // the last step stages nothing
        for (int64_t li = threadIdx.x; li < su.n; li += W * 64) {
          double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int c = 0; c < 3; ++c) a[c] += (double)ps[(int64_t)c * su.n + li];
          finish_particle(su.base + li, n, a, ls, acc, nullptr, vel, hh, nxt, nullptr, nullptr);
        }
        __syncthreads();  // positions staged for the next step's tile
      }
      continue;
    }
    const int64_t q = q0 - n_solo;
    const int32_t t = (int32_t)(q / per_step);
    const int64_t r = q - (int64_t)t * per_step;
    if (r < n_units) {
      const SymUnit su = units[n_solo + r];
      const int32_t chunks = (su.n + kRolloutChunk - 1) / kRolloutChunk;  // reduction tasks of the system
      if (threadIdx.x == 0) ok_sh = t == 0 || wait_at_least(sy.red_done + su.sys, t * chunks, sy.err, sy.spin_limit);
      __syncthreads();
      if (!ok_sh) break;
      __threadfence();  // every thread: ordered after the positions staged by (s, t - 1)
      sym_tile<W, I, false, MODE, ROT, LAW, PIPE>(jarr + NV * su.base, su.n, su.A, su.B, eps2_arg,
                                                 part + su.part_off, red);
      release_to(sy.tiles_done + su.sys);
    } else {
      const int64_t s = rtasks[2 * (r - n_units)];
      const int64_t l0 = (int64_t)rtasks[2 * (r - n_units) + 1] * kRolloutChunk;
      const int64_t b = sys_off[s], ns = sys_off[s + 1] - b;
      const int64_t l1 = l0 + kRolloutChunk < ns ? l0 + kRolloutChunk : ns;
      const int32_t nb = sys_nb[s];
      if (threadIdx.x == 0) ok_sh = wait_at_least(sy.tiles_done + s, (t + 1) * (nb * (nb + 1) / 2), sy.err, sy.spin_limit);
      __syncthreads();
      if (!ok_sh) break;
      __threadfence();  // every thread: ordered after the tiles' partial sums
      const float* ps = part + sys_part[s];
      NextStep nxt = nx;
      if (t + 1 >= steps) nxt.kind = 0;  // the last step stages nothing
      for (int64_t li = l0 + threadIdx.x; li < l1; li += W * 64) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        sum_slots<3, 1>(ps, ns, li, nb, a);
        finish_particle(b + li, n, a, ls, acc, nullptr, vel, hh, nxt, nullptr, nullptr);
      }
      release_to(sy.red_done + s);
    }
  }
}

// ----------------------------------------------------------------- batched one-sided force pass

// One work unit: an i-tile of one system against one j-chunk of the same system.
struct WorkUnit {
  int64_t ib, ie;  // i-range (global particle indices)
  int64_t jb, je;  // j-range (global particle indices, inside the same system)
  int32_t slot;    // j-chunk index inside the system (partial-sum slot)
  int32_t pad;
};

// One workgroup per work unit. The units are sorted by decreasing cost on the host and the
// hardware starts workgroups in index order, so the largest start first with no queue in
// memory. Each unit writes its own partial slot, so the result does not depend on the order
// in which they ran.
template <typename T, int BS, int I, int TJ, bool POT, int MODE, int LAW>
__global__ __launch_bounds__(BS) void force_batched_kernel(const typename Vec4<T>::type* __restrict__ jarr,
                                                           const WorkUnit* __restrict__ units, int32_t n_units,
                                                           T eps2, ForceOut o) {
  __shared__ typename Vec4<T>::type tile[TJ * (MODE == MODE_DS ? 2 : 1)];
  if ((int32_t)blockIdx.x >= n_units) return;
  const WorkUnit w = units[blockIdx.x];
  double res[4][I];
  force_block<T, BS, I, TJ, POT, MODE, LAW>(jarr, w.ib, w.ie, w.jb, w.je, eps2, tile, res);
  force_store<I>(o, w.ib, w.ie, w.slot, res, POT, BS);
}

__global__ void fill_i32(int32_t* p, int64_t count, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void fill_f64(double* p, int64_t count, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ----------------------------------------------------------------- energy / momentum

// Deterministic two-pass reduction per system. Pass 1: block (bx, s) sums chunk bx
// of system s (grid-stride over the system, fixed order), wave64 shuffle tree then
// LDS tree; writes part[s][bx][5]. Pass 2: one block per system sums its chunks.
template <int BS>
__global__ __launch_bounds__(BS) void energy_partial(int64_t n, const double* __restrict__ vel,
                                                     const double* __restrict__ mass, const double* __restrict__ pot,
                                                     const int64_t* __restrict__ sys_off, int64_t single_n,
                                                     int32_t chunks, double* __restrict__ part) {
  __shared__ double sh[5 * (BS / 64)];
  const int64_t s = blockIdx.y;
  const int64_t b = sys_off ? sys_off[s] : 0;
  const int64_t e = sys_off ? sys_off[s + 1] : single_n;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = b + (int64_t)blockIdx.x * BS + threadIdx.x; i < e; i += (int64_t)chunks * BS)
    energy_terms(mass[i], vel[i], vel[n + i], vel[2 * n + i], pot[i], v);
  block_sum<BS, 5>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 5; ++c) part[(s * chunks + blockIdx.x) * 5 + c] = v[c];
}

// grid (S, T): state t of T reads its partials at part + t * part_step and writes its [S][5]
// row at out + t * out_step.
template <int BS>
__global__ __launch_bounds__(BS) void energy_final(int32_t chunks, const double* __restrict__ part,
                                                   double* __restrict__ out, int64_t part_step, int64_t out_step) {
  __shared__ double sh[5 * (BS / 64)];
  const int64_t s = blockIdx.x;
  part += (int64_t)blockIdx.y * part_step;
  out += (int64_t)blockIdx.y * out_step;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < chunks; k += BS)
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] += part[(s * chunks + k) * 5 + c];
  block_sum<BS, 5>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 5; ++c) out[s * 5 + c] = v[c];
}

// Diagnostics, the same two-pass scheme with K = 10 components per system:
// KE, PE, Px, Py, Pz, Lx, Ly, Lz (L = sum m x cross v), W (= sum m x . a), M.
constexpr int kDiag = 10;

template <int BS>
__global__ __launch_bounds__(BS) void diag_partial(int64_t n, const double* __restrict__ pos,
                                                   const double* __restrict__ vel, const double* __restrict__ mass,
                                                   const double* __restrict__ pot, const double* __restrict__ acc,
                                                   const int64_t* __restrict__ sys_off, int64_t single_n,
                                                   int32_t chunks, double* __restrict__ part) {
  __shared__ double sh[kDiag * (BS / 64)];
  const int64_t s = blockIdx.y;
  const int64_t b = sys_off ? sys_off[s] : 0;
  const int64_t e = sys_off ? sys_off[s + 1] : single_n;
  double v[kDiag];
#pragma unroll
  for (int c = 0; c < kDiag; ++c) v[c] = 0.0;
  for (int64_t i = b + (int64_t)blockIdx.x * BS + threadIdx.x; i < e; i += (int64_t)chunks * BS) {
    const double m = mass[i];
    const double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
    v[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    v[1] += 0.5 * m * pot[i];
    v[2] += m * vx;
    v[3] += m * vy;
    v[4] += m * vz;
    v[5] += m * (y * vz - z * vy);
    v[6] += m * (z * vx - x * vz);
    v[7] += m * (x * vy - y * vx);
    v[8] += m * (x * acc[i] + y * acc[n + i] + z * acc[2 * n + i]);
    v[9] += m;
  }
  block_sum<BS, kDiag>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < kDiag; ++c) part[(s * chunks + blockIdx.x) * kDiag + c] = v[c];
}

template <int BS>
__global__ __launch_bounds__(BS) void diag_final(int32_t chunks, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  __shared__ double sh[kDiag * (BS / 64)];
  const int64_t s = blockIdx.x;
  double v[kDiag];
#pragma unroll
  for (int c = 0; c < kDiag; ++c) v[c] = 0.0;
  for (int k = threadIdx.x; k < chunks; k += BS)
#pragma unroll
    for (int c = 0; c < kDiag; ++c) v[c] += part[(s * chunks + k) * kDiag + c];
  block_sum<BS, kDiag>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < kDiag; ++c) out[s * kDiag + c] = v[c];
}

// ----------------------------------------------------------------- adjoint pair pass

// Adjoint j-array: two vectors per particle, (x, y, z, m) and (l_x, l_y, l_z, 0),
// l = w * (velocity cotangent). Optionally applies the drift adjoint first:
//   gvel += h_drift * gpos  (h_drift = 0 skips it).
template <typename T>
__global__ void adjoint_stage(int64_t n, const double* __restrict__ pos, const double* __restrict__ mass,
                              double* __restrict__ gvel, const double* __restrict__ gpos, double h_drift,
                              double w, typename Vec4<T>::type* __restrict__ jadj) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double l[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double gv = gvel[c * n + i];
    if (h_drift != 0.0) {
      gv += h_drift * gpos[c * n + i];
      gvel[c * n + i] = gv;
    }
    l[c] = w * gv;
  }
  typename Vec4<T>::type a, b;
  a.x = (T)pos[i];
  a.y = (T)pos[n + i];
  a.z = (T)pos[2 * n + i];
  a.w = (T)mass[i];
  b.x = (T)l[0];
  b.y = (T)l[1];
  b.z = (T)l[2];
  b.w = T(0);
  jadj[2 * i] = a;
  jadj[2 * i + 1] = b;
}

struct AdjOut {
  // direct mode: gpos += G*(m_k A - B l_k - C), gmass += -G*M
  double* gpos;
  double* gmass;
  double G;
  // partial mode: part[(slot*8 + c)*n_plane + i], c = A0..2, B, C0..2, M (unscaled)
  double* part;
  int64_t n_plane;
};

// Per pair (k = own particle, j = partner), d = x_j - x_k, r3 = s^{-3/2}, r5 = s^{-5/2}:
//   A += r3 l_j;  B += m_j r3;  C += 3 r5 (m_k (d.l_j) - m_j (d.l_k)) d;  M += r3 (d.l_j)
// so that  sum_j T(d)(m_k l_j - m_j l_k) = m_k A - B l_k - C  and  gm_k = -G M.
template <typename T, int BS, int I, int TJ, bool COMP>
__device__ __forceinline__ void adjoint_block(const typename Vec4<T>::type* __restrict__ jadj,
                                              int64_t ib, int64_t ie, int64_t jb, int64_t je, T eps2_arg,
                                              typename Vec4<T>::type* tile /* [2*TJ] */, double res[8][I],
                                              double own[7][I]) {
  using V = typename Vec4<T>::type;
  static_assert(TJ % BS == 0, "TJ must be a multiple of BS");
  constexpr int PER = TJ / BS;
  const T eps2 = in_vgpr(eps2_arg);
  const T three = in_vgpr(T(3));
  const int t = threadIdx.x;

  T xk[I], yk[I], zk[I], mk[I], lkx[I], lky[I], lkz[I];
  T acc_t[8][I];
  float hi[8][I], lo[8][I];
  int64_t my_i[I];
#pragma unroll
  for (int u = 0; u < I; ++u) {
    int64_t i = ib + t + (int64_t)u * BS;
    my_i[u] = i;
    int64_t ic = i < ie ? i : ie - 1;
    V p = jadj[2 * ic], l = jadj[2 * ic + 1];
    xk[u] = in_vgpr(p.x); yk[u] = in_vgpr(p.y); zk[u] = in_vgpr(p.z); mk[u] = in_vgpr(p.w);
    lkx[u] = in_vgpr(l.x); lky[u] = in_vgpr(l.y); lkz[u] = in_vgpr(l.z);
    own[0][u] = (double)p.w; own[1][u] = (double)l.x; own[2][u] = (double)l.y; own[3][u] = (double)l.z;
#pragma unroll
    for (int c = 0; c < 8; ++c) { acc_t[c][u] = T(0); hi[c][u] = 0.f; lo[c][u] = 0.f; }
  }

  V pre[2 * PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int64_t j = jb + t + (int64_t)k * BS;
    pre[2 * k] = load_or(jadj, 2 * j, j < je, zero4<T>());
    pre[2 * k + 1] = load_or(jadj, 2 * j + 1, j < je, zero4<T>());
  }

  for (int64_t j0 = jb; j0 < je; j0 += TJ) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      tile[2 * (t + k * BS)] = pre[2 * k];
      tile[2 * (t + k * BS) + 1] = pre[2 * k + 1];
    }
    __syncthreads();
    if (j0 + TJ < je) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        int64_t j = j0 + TJ + t + (int64_t)k * BS;
        pre[2 * k] = load_or(jadj, 2 * j, j < je, zero4<T>());
        pre[2 * k + 1] = load_or(jadj, 2 * j + 1, j < je, zero4<T>());
      }
    }
    const bool diag = (j0 < ie) && (j0 + TJ > ib);
#define NBODY_ADJ_PAIR(MASKED)                                                           \
    {                                                                                    \
      const V q = tile[2 * jj], L = tile[2 * jj + 1];                                    \
      _Pragma("unroll") for (int u = 0; u < I; ++u) {                                    \
        T dx = q.x - xk[u], dy = q.y - yk[u], dz = q.z - zk[u];                          \
        T r2 = fmaT(dx, dx, fmaT(dy, dy, fmaT(dz, dz, eps2))); \
        T ri = pair_rsqrt<T>(r2);                                                        \
        T ri2 = ri * ri;                                                                 \
        T r3 = ri * ri2;                                                                 \
        if (MASKED) r3 = (j0 + jj == my_i[u]) ? T(0) : r3;                               \
        T r5x3 = r3 * (ri2 * three);                                                     \
        T p = fmaT(dx, L.x, fmaT(dy, L.y, dz * L.z));                  \
        T qq = fmaT(dx, lkx[u], fmaT(dy, lky[u], dz * lkz[u]));        \
        acc_t[0][u] = fmaT(r3, L.x, acc_t[0][u]);                               \
        acc_t[1][u] = fmaT(r3, L.y, acc_t[1][u]);                               \
        acc_t[2][u] = fmaT(r3, L.z, acc_t[2][u]);                               \
        acc_t[3][u] = fmaT(q.w, r3, acc_t[3][u]);                               \
        T wv = fmaT(mk[u], p, -(q.w * qq));                                     \
        T cc = r5x3 * wv;                                                                \
        acc_t[4][u] = fmaT(cc, dx, acc_t[4][u]);                                \
        acc_t[5][u] = fmaT(cc, dy, acc_t[5][u]);                                \
        acc_t[6][u] = fmaT(cc, dz, acc_t[6][u]);                                \
        acc_t[7][u] = fmaT(r3, p, acc_t[7][u]);                                 \
      }                                                                                  \
    }
    if (!diag) {
#pragma unroll 4
      for (int jj = 0; jj < TJ; ++jj) NBODY_ADJ_PAIR(false)
    } else {
      for (int jj = 0; jj < TJ; ++jj) NBODY_ADJ_PAIR(true)
    }
#undef NBODY_ADJ_PAIR
    if (COMP) {
#pragma unroll
      for (int u = 0; u < I; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float s, e;
          two_sum(hi[c][u], (float)acc_t[c][u], s, e);
          hi[c][u] = s;
          lo[c][u] += e;
          acc_t[c][u] = T(0);
        }
    }
  }
#pragma unroll
  for (int u = 0; u < I; ++u)
#pragma unroll
    for (int c = 0; c < 8; ++c)
      res[c][u] = COMP ? (double)hi[c][u] + (double)lo[c][u] : (double)acc_t[c][u];
}

template <int I>
__device__ __forceinline__ void adjoint_store(const AdjOut& o, int64_t ib, int64_t ie, int slot,
                                              const double res[8][I], const double own[7][I], int BS) {
#pragma unroll
  for (int u = 0; u < I; ++u) {
    int64_t i = ib + threadIdx.x + (int64_t)u * BS;
    if (i >= ie) continue;
    if (o.part) {
#pragma unroll
      for (int c = 0; c < 8; ++c) o.part[((int64_t)slot * 8 + c) * o.n_plane + i] = res[c][u];
    } else {
      const double m = own[0][u];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        o.gpos[c * o.n_plane + i] += o.G * (m * res[c][u] - res[3][u] * own[1 + c][u] - res[4 + c][u]);
      o.gmass[i] += -o.G * res[7][u];
    }
  }
}

template <typename T, int BS, int I, int TJ, bool COMP>
__global__ __launch_bounds__(BS) void adjoint_kernel(const typename Vec4<T>::type* __restrict__ jadj,
                                                     int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                                                     int64_t jchunk, T eps2, AdjOut o) {
  __shared__ typename Vec4<T>::type tile[2 * TJ];
  const int64_t ib = i0 + (int64_t)blockIdx.x * BS * I;
  const int64_t ie = ib + BS * I < i1 ? ib + BS * I : i1;
  const int64_t jb = j0 + (int64_t)blockIdx.y * jchunk;
  const int64_t je = jb + jchunk < j1 ? jb + jchunk : j1;
  double res[8][I], own[7][I];
  adjoint_block<T, BS, I, TJ, COMP>(jadj, ib, ie, jb, je, eps2, tile, res, own);
  adjoint_store<I>(o, ib, ie, blockIdx.y, res, own, BS);
}

template <typename T, int BS, int I, int TJ, bool COMP>
__global__ __launch_bounds__(BS) void adjoint_batched_kernel(const typename Vec4<T>::type* __restrict__ jadj,
                                                             const WorkUnit* __restrict__ units, int32_t n_units,
                                                             T eps2, AdjOut o) {
  __shared__ typename Vec4<T>::type tile[2 * TJ];
  if ((int32_t)blockIdx.x >= n_units) return;  // one workgroup per unit, as force_batched_kernel
  const WorkUnit w = units[blockIdx.x];
  double res[8][I], own[7][I];
  adjoint_block<T, BS, I, TJ, COMP>(jadj, w.ib, w.ie, w.jb, w.je, eps2, tile, res, own);
  adjoint_store<I>(o, w.ib, w.ie, w.slot, res, own, BS);
}

// Sum of adjoint j-split partials (fixed order), combined and added into gpos/gmass.
//   part [S][8][n]; jadj gives m_k and l_k of particle k.
template <typename T>
__global__ __launch_bounds__(256) void adjoint_reduce(int64_t count, int64_t stride, int32_t S, const double* __restrict__ part,
                               const typename Vec4<T>::type* __restrict__ jadj, double G,
                               double* __restrict__ gpos, double* __restrict__ gmass, int64_t n_sys,
                               const int64_t* __restrict__ sys_off, const int32_t* __restrict__ nsplit) {
  const int64_t n = stride;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int32_t s_cnt = S;
  if (n_sys > 0) {
    int64_t lo = 0, hi = n_sys;
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (sys_off[mid] <= i) lo = mid; else hi = mid;
    }
    s_cnt = nsplit[lo];
  }
  // the particle's own state first, so that its loads are in flight with the sums'
  const auto a = jadj[2 * i];
  const auto l = jadj[2 * i + 1];
  double g0[4];
#pragma unroll
  for (int c = 0; c < 3; ++c) g0[c] = gpos[c * n + i];
  g0[3] = gmass[i];
  double r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  sum_splits<8, 4>(part, n, i, s_cnt, r);
  const double m = (double)a.w;
  const double lk[3] = {(double)l.x, (double)l.y, (double)l.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) gpos[c * n + i] = g0[c] + G * (m * r[c] - r[3] * lk[c] - r[4 + c]);
  gmass[i] = g0[3] + -G * r[7];
}

// ----------------------------------------------------------------- symmetric adjoint pass (FP32)

// Each unordered pair once. With d = x_j - x_k, r3 = s^{-3/2}, 3 r5 = 3 s^{-5/2},
// w = m_k l_j - m_j l_k and cc = 3 r5 (d.w), the pair's share of the VJP is
//   v = T(d) w = r3 w - cc d:   gx_k += v,  gx_j -= v,
// (T(d) is even in d and w changes sign when k and j swap), and for the masses
//   M_k += r3 (d.l_j),  M_j -= r3 (d.l_k),   gm = -G M.
// Unlike the one-sided pass (which factors m_k and l_k out of its sums), the sums are
// taken directly, so every particle carries 4 accumulators instead of 8 - half the
// registers and lane rotations. Tiles, lane rotation and slots as in sym_tile:
// part[(slot*4 + c)*n + p], c = gx, gy, gz, M. Diagonal tiles run one-sided with the
// self pair masked (r3 = 0 removes every term). OUT 1 and 2 (the round schedule) add the sums
// to double accumulators acc64 [4][n] instead, as sym_tile does.
template <int W, int I, bool COMP, int ROT, int OUT = 0>
__device__ __forceinline__ void adj_sym_tile(const float4* __restrict__ jadj, int64_t n, int32_t A, int32_t B,
                                             float eps2_arg, float* __restrict__ part,
                                             float (&red)[2][W][4][64], double* __restrict__ acc64 = nullptr) {
  constexpr int BI = W * 64 * I;
  constexpr int NSUB = BI / 64;
  const bool diag = (A == B);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rot_src = ((lane - 1) & 63) << 2;
  const int64_t Abase = (int64_t)A * BI, Bbase = (int64_t)B * BI;
  const float eps2 = in_vgpr(eps2_arg);
  const float three = in_vgpr(3.f);
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);

  // With 4 or more particles per lane the compensated sums (high and low words) live in LDS:
  // a lane touches only its own words, once per sub-block, and the pair loop keeps 8I fewer
  // registers (4 waves per SIMD at I = 4); the arithmetic is that of the register form.
  constexpr bool HL_LDS = COMP && I >= 4;
  __shared__ float hl_lds[HL_LDS ? W * 2 * 4 * I * 64 : 1];
  // high word of (c, u): hl_w[(c * I + u) * 64]; low word: hl_w[((4 + c) * I + u) * 64]
  float* const hl_w = hl_lds + (HL_LDS ? w * 2 * 4 * I * 64 + lane : 0);

  float xk[I], yk[I], zk[I], mk[I], lx[I], ly[I], lz[I];
  float ai[4][I], hi[4][I], lo[4][I];
#pragma unroll
  for (int u = 0; u < I; ++u) {
    const int64_t i = Abase + (int64_t)w * 64 * I + u * 64 + lane;
    const int64_t ic = i < n ? i : n - 1;
    const float4 p = jadj[2 * ic];
    float4 l = zero;  // (a branch, not a select of addresses: keeps the load global)
    if (i < n) l = jadj[2 * ic + 1];
    xk[u] = in_vgpr(p.x);
    yk[u] = in_vgpr(p.y);
    zk[u] = in_vgpr(p.z);
    mk[u] = in_vgpr(i < n ? p.w : 0.f);
    lx[u] = in_vgpr(l.x);
    ly[u] = in_vgpr(l.y);
    lz[u] = in_vgpr(l.z);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ai[c][u] = 0.f;
      if constexpr (HL_LDS) {
        hl_w[(c * I + u) * 64] = 0.f;
        hl_w[((4 + c) * I + u) * 64] = 0.f;
      } else {
        hi[c][u] = 0.f;
        lo[c][u] = 0.f;
      }
    }
  }

  float4 nq = zero, nl = zero;
  {
    const int64_t j = Bbase + lane;
    if (j < n) {
      nq = jadj[2 * j];
      nl = jadj[2 * j + 1];
    }
  }
  const int64_t jrows = n - Bbase;
  const int nsub_b = jrows >= BI ? NSUB : (int)((jrows + 63) >> 6);
  const int nsub = (diag && Abase + (int64_t)w * 64 * I >= n) ? 0 : nsub_b;
  for (int sb = 0; sb < nsub; ++sb) {
    const float4 q = nq, L = nl;
    if (sb + 1 < nsub) {
      const int64_t j = Bbase + (int64_t)(sb + 1) * 64 + lane;
      nq = zero;
      nl = zero;
      if (j < n) {
        nq = jadj[2 * j];
        nl = jadj[2 * j + 1];
      }
    }
    float xj = q.x, yj = q.y, zj = q.z, mj = q.w, ljx = L.x, ljy = L.y, ljz = L.z;
    if (diag) {
      for (int k = 0; k < 64; ++k) {
#pragma unroll
        for (int u = 0; u < I; ++u) {
          const float dx = xj - xk[u], dy = yj - yk[u], dz = zj - zk[u];
          const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
          const float ri = __builtin_amdgcn_rsqf(r2);
          const float ri2 = ri * ri;
          float r3 = ri * ri2;
          r3 = (k == 0 && sb == w * I + u) ? 0.f : r3;  // the self pair
          const float r5x3 = r3 * (ri2 * three);
          const float pp = __builtin_fmaf(dx, ljx, __builtin_fmaf(dy, ljy, dz * ljz));
          const float qq = __builtin_fmaf(dx, lx[u], __builtin_fmaf(dy, ly[u], dz * lz[u]));
          const float cc = r5x3 * __builtin_fmaf(mk[u], pp, -(mj * qq));  // 3 r5 (d.w)
          const float am = r3 * mk[u], bm = r3 * mj;                       // r3 w = am l_j - bm l_k
          ai[0][u] += __builtin_fmaf(am, ljx, __builtin_fmaf(-bm, lx[u], -(cc * dx)));
          ai[1][u] += __builtin_fmaf(am, ljy, __builtin_fmaf(-bm, ly[u], -(cc * dy)));
          ai[2][u] += __builtin_fmaf(am, ljz, __builtin_fmaf(-bm, lz[u], -(cc * dz)));
          ai[3][u] = __builtin_fmaf(r3, pp, ai[3][u]);
        }
        xj = rotate1<rot_coord<ROT>()>(xj, rot_src);
        yj = rotate1<rot_coord<ROT>()>(yj, rot_src);
        zj = rotate1<rot_coord<ROT>()>(zj, rot_src);
        mj = rotate1<rot_coord<ROT>()>(mj, rot_src);
        ljx = rotate1<rot_coord<ROT>()>(ljx, rot_src);
        ljy = rotate1<rot_coord<ROT>()>(ljy, rot_src);
        ljz = rotate1<rot_coord<ROT>()>(ljz, rot_src);
      }
    } else {
      float aj[4] = {0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < 64; ++k) {
        // the next step's coordinates are requested first, a whole step ahead of use
        const float xn = rotate1<rot_coord<ROT>()>(xj, rot_src), yn = rotate1<rot_coord<ROT>()>(yj, rot_src), zn = rotate1<rot_coord<ROT>()>(zj, rot_src);
        float dx[I], dy[I], dz[I], rr[I];
#pragma unroll
        for (int u = 0; u < I; ++u) {
          dx[u] = xj - xk[u];
          dy[u] = yj - yk[u];
          dz[u] = zj - zk[u];
          rr[u] = __builtin_fmaf(dx[u], dx[u], __builtin_fmaf(dy[u], dy[u], __builtin_fmaf(dz[u], dz[u], eps2)));
        }
#pragma unroll
        for (int u = 0; u < I; ++u) rr[u] = __builtin_amdgcn_rsqf(rr[u]);
#pragma unroll
        for (int u = 0; u < I; ++u) {
          const float ri2 = rr[u] * rr[u];
          const float r3 = rr[u] * ri2;
          const float r5x3 = r3 * (ri2 * three);
          const float pp = __builtin_fmaf(dx[u], ljx, __builtin_fmaf(dy[u], ljy, dz[u] * ljz));
          const float qq = __builtin_fmaf(dx[u], lx[u], __builtin_fmaf(dy[u], ly[u], dz[u] * lz[u]));
          const float cc = r5x3 * __builtin_fmaf(mk[u], pp, -(mj * qq));  // 3 r5 (d.w)
          const float am = r3 * mk[u], bm = r3 * mj;                       // r3 w = am l_j - bm l_k
          const float vx = __builtin_fmaf(am, ljx, __builtin_fmaf(-bm, lx[u], -(cc * dx[u])));
          const float vy = __builtin_fmaf(am, ljy, __builtin_fmaf(-bm, ly[u], -(cc * dy[u])));
          const float vz = __builtin_fmaf(am, ljz, __builtin_fmaf(-bm, lz[u], -(cc * dz[u])));
          ai[0][u] += vx;
          ai[1][u] += vy;
          ai[2][u] += vz;
          ai[3][u] = __builtin_fmaf(r3, pp, ai[3][u]);
          aj[0] -= vx;
          aj[1] -= vy;
          aj[2] -= vz;
          aj[3] = __builtin_fmaf(-r3, qq, aj[3]);
        }
        xj = xn;
        yj = yn;
        zj = zn;
        mj = rotate1<rot_coord<ROT>()>(mj, rot_src);
        ljx = rotate1<rot_coord<ROT>()>(ljx, rot_src);
        ljy = rotate1<rot_coord<ROT>()>(ljy, rot_src);
        ljz = rotate1<rot_coord<ROT>()>(ljz, rot_src);
#pragma unroll
        for (int c = 0; c < 4; ++c) aj[c] = rotate1<rot_acc<ROT>()>(aj[c], rot_src);
      }
      // j-side of this sub-block: the W waves summed in wave order, written to slot A
#pragma unroll
      for (int c = 0; c < 4; ++c) red[sb & 1][w][c][lane] = aj[c];
      __syncthreads();
      for (int idx = threadIdx.x; idx < 4 * 64; idx += W * 64) {
        const int c = idx >> 6, l = idx & 63;
        float sum = 0.f;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) sum += red[sb & 1][ww][c][l];
        const int64_t j = Bbase + (int64_t)sb * 64 + l;
        if constexpr (OUT == 0) {
          if (j < n) part[((int64_t)A * 4 + c) * n + j] = sum;
        } else if constexpr (OUT == 1) {
          if (j < n) acc64[(int64_t)c * n + j] += (double)sum;
        } else {
          if (j < n) unsafeAtomicAdd(acc64 + (int64_t)c * n + j, (double)sum);
        }
      }
    }
    if (COMP) {
#pragma unroll
      for (int u = 0; u < I; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          float t, e;
          if constexpr (HL_LDS) {
            float& h = hl_w[(c * I + u) * 64];
            two_sum(h, ai[c][u], t, e);
            h = t;
            hl_w[((4 + c) * I + u) * 64] += e;
          } else {
            two_sum(hi[c][u], ai[c][u], t, e);
            hi[c][u] = t;
            lo[c][u] += e;
          }
          ai[c][u] = 0.f;
        }
    }
  }
  // i-side of the tile: slot B
#pragma unroll
  for (int u = 0; u < I; ++u) {
    const int64_t i = Abase + (int64_t)w * 64 * I + u * 64 + lane;
    if (i < n)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (OUT == 0) {
          float v = ai[c][u];
          if constexpr (HL_LDS) v = hl_w[(c * I + u) * 64] + hl_w[((4 + c) * I + u) * 64];
          else if constexpr (COMP) v = hi[c][u] + lo[c][u];
          part[((int64_t)B * 4 + c) * n + i] = v;
        } else {
          double v = (double)ai[c][u];
          if constexpr (HL_LDS) v = (double)hl_w[(c * I + u) * 64] + (double)hl_w[((4 + c) * I + u) * 64];
          else if constexpr (COMP) v = (double)hi[c][u] + (double)lo[c][u];
          if constexpr (OUT == 1) acc64[(int64_t)c * n + i] += v;
          else unsafeAtomicAdd(acc64 + (int64_t)c * n + i, v);
        }
      }
  }
}

// The adjoint pass on the round schedule (the pairing, copies and atomic adds of
// force_sym_round_kernel; its diagonal tiles in adjoint_sym_round_diag_kernel).
template <int W, int I, bool COMP, int ROT>
__global__ __launch_bounds__(W * 64) void adjoint_sym_round_kernel(const float4* __restrict__ jadj, int64_t n,
                                                                   int32_t nb, int32_t nbr, int32_t r0, float eps2,
                                                                   double* __restrict__ acc64) {
  __shared__ float red[2][W][4][64];
  const int32_t r = r0 + (int32_t)blockIdx.y;
  if (r >= nbr - 1) return;  // past the last round (the whole workgroup)
  acc64 += (int64_t)blockIdx.y * 4 * n;
  const int32_t m = nbr - 1, t = (int32_t)blockIdx.x;
  const int32_t a = t == 0 ? r : (r + t) % m;
  const int32_t b = t == 0 ? m : (r - t + m) % m;
  const int32_t A = a < b ? a : b, B = a < b ? b : a;
  if (B >= nb) return;  // the padding block of an odd block count (the whole workgroup)
  adj_sym_tile<W, I, COMP, ROT, 2>(jadj, n, A, B, eps2, nullptr, red, acc64);
}

template <int W, int I, bool COMP, int ROT>
__global__ __launch_bounds__(W * 64) void adjoint_sym_round_diag_kernel(const float4* __restrict__ jadj, int64_t n,
                                                                        float eps2, double* __restrict__ acc64) {
  __shared__ float red[2][W][4][64];
  const int32_t A = (int32_t)blockIdx.x;
  adj_sym_tile<W, I, COMP, ROT, 1>(jadj, n, A, A, eps2, nullptr, red, acc64);
}

template <int W, int I, bool COMP, int ROT>
__global__ __launch_bounds__(W * 64) void adjoint_sym_kernel(const float4* __restrict__ jadj, int64_t n, int32_t nb,
                                                             float eps2, float* __restrict__ part) {
  __shared__ float red[2][W][4][64];
  int32_t A, B;
  tile_rc(blockIdx.x, nb, A, B);
  adj_sym_tile<W, I, COMP, ROT>(jadj, n, A, B, eps2, part, red);
}

// One workgroup per symmetric adjoint tile of many systems (as force_sym_batched_kernel).
template <int W, int I, bool COMP, int ROT>
__global__ __launch_bounds__(W * 64) void adjoint_sym_batched_kernel(const float4* __restrict__ jadj,
                                                                     const SymUnit* __restrict__ units,
                                                                     int32_t n_units, float eps2,
                                                                     float* __restrict__ part) {
  __shared__ float red[2][W][4][64];
  if ((int32_t)blockIdx.x >= n_units) return;
  const SymUnit su = units[blockIdx.x];
  adj_sym_tile<W, I, COMP, ROT>(jadj + 2 * su.base, su.n, su.A, su.B, eps2, part + su.part_off, red);
}

// Sum of the nb float slots (4 components) of every particle in double:
// gpos += G gx, gmass += -G M. Single system: n particles (partial plane
// stride), stride = plane stride of gpos; batched (n_sys > 0): system of particle i found
// by binary search, its nb and partial offset from sys_nb / sys_part.
__global__ __launch_bounds__(256) void adjoint_reduce_sym(int64_t n, int64_t stride, int32_t nb, const float* __restrict__ part,
                                   double G, double* __restrict__ gpos,
                                   double* __restrict__ gmass, int64_t n_sys, const int64_t* __restrict__ sys_off,
                                   const int32_t* __restrict__ sys_nb, const int64_t* __restrict__ sys_part) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t ns = n, li = i;
  int32_t nbs = nb;
  const float* ps = part;
  if (n_sys > 0) {
    int64_t lo = 0, hi = n_sys;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (sys_off[mid] <= i) lo = mid; else hi = mid;
    }
    const int64_t b = sys_off[lo];
    ns = sys_off[lo + 1] - b;
    li = i - b;
    nbs = sys_nb[lo];
    ps = part + sys_part[lo];
  }
  double g0[4];  // loaded before the sums, so that the loads are in flight together
#pragma unroll
  for (int c = 0; c < 3; ++c) g0[c] = gpos[c * stride + i];
  g0[3] = gmass[i];
  double r[4] = {0, 0, 0, 0};
  sum_slots<4>(ps, ns, li, nbs, r);
#pragma unroll
  for (int c = 0; c < 3; ++c) gpos[c * stride + i] = g0[c] + G * r[c];
  gmass[i] = g0[3] + -G * r[3];
}

// The end of the adjoint round schedule: the K accumulator copies added in copy order,
// gpos += G gx, gmass += -G M.
__global__ __launch_bounds__(256) void adjoint_reduce_rounds(int64_t n, int64_t stride, int32_t K,
                                                            const double* __restrict__ acc64, double G,
                                                            double* __restrict__ gpos, double* __restrict__ gmass) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double g0[4];
#pragma unroll
  for (int c = 0; c < 3; ++c) g0[c] = gpos[c * stride + i];
  g0[3] = gmass[i];
  double r[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double* q = acc64 + (int64_t)c * n + i;
    double t = q[0];
    for (int k = 1; k < K; ++k) t += q[(int64_t)k * 4 * n];
    r[c] = t;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) gpos[c * stride + i] = g0[c] + G * r[c];
  gmass[i] = g0[3] + -G * r[3];
}

// The next adjoint pass's staging (adjoint_stage<float>), fused into a reduction that has just
// updated the particle's position gradient: kind 0 nothing, 1 the FP32 adjoint j-array.
struct AdjNext {
  int32_t kind;
  int32_t pad;
  const double* pos;   // the next pass's positions [3][stride]
  const double* mass;
  double* gvel;
  double h_drift, w;
  float4* jadj;
};

// The single-system form: four waves per 64 particles, wave g summing slot group g (as in
// reduce_sym); wave 0 adds the groups, (p0 + p1) + (p2 + p3), updates the gradients and, with
// an.kind, stages the particle for the next pass with adjoint_stage's arithmetic.
__global__ __launch_bounds__(256) void adjoint_reduce_sym_groups(int64_t n, int64_t stride, int32_t nb,
                                                                const float* __restrict__ part, double G,
                                                                double* __restrict__ gpos,
                                                                double* __restrict__ gmass, AdjNext an) {
  __shared__ double sh[3][4][64];
  const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool live = i < n;
  double g0[4] = {0.0, 0.0, 0.0, 0.0};
  if (g == 0 && live) {
#pragma unroll
    for (int c = 0; c < 3; ++c) g0[c] = gpos[c * stride + i];
    g0[3] = gmass[i];
  }
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  if (live) sum_slot_group<4>(part, n, i, nb, g, q);
  if (g > 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[g - 1][c][lane] = q[c];
  __syncthreads();
  if (g == 0 && live) {
    double r[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) r[c] = (q[c] + sh[0][c][lane]) + (sh[1][c][lane] + sh[2][c][lane]);
    double gp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gp[c] = g0[c] + G * r[c];
      gpos[c * stride + i] = gp[c];
    }
    gmass[i] = g0[3] + -G * r[3];
    if (an.kind) {
      float l[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double gv = an.gvel[c * stride + i];
        if (an.h_drift != 0.0) {
          gv += an.h_drift * gp[c];
          an.gvel[c * stride + i] = gv;
        }
        l[c] = (float)(an.w * gv);
      }
      float4 a, b;
      a.x = (float)an.pos[i];
      a.y = (float)an.pos[stride + i];
      a.z = (float)an.pos[2 * stride + i];
      a.w = (float)an.mass[i];
      b.x = l[0];
      b.y = l[1];
      b.z = l[2];
      b.w = 0.f;
      an.jadj[2 * i] = a;
      an.jadj[2 * i + 1] = b;
    }
  }
}

}  // namespace nbody
