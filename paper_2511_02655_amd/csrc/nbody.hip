// libnbody.so: host side of the C ABI declared in include/nbody.h.
//
// Argument validation (host only, before any HIP call), workspace planning,
// tile-table lookup, kernel launches, and the rollout / reverse-rollout drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nbody.h"
#include "nbody_adapt.hpp"
#include "nbody_kernels.hpp"

using namespace nbody;

namespace {

thread_local std::string g_err;

// Probes a whole-rollout wait makes before it gives up (nbody_set_wait_limit).
std::atomic<int64_t> g_wait_limit{int64_t(1) << 24};

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(NBODY_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(what)                                                                   \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess) return fail(NBODY_ERR_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != NBODY_OK) return rc_; \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ tile variants

using ForceFn = void (*)(dim3, hipStream_t, const void* jarr, int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                         int64_t jchunk, double eps2, const ForceOut&);
using ForceBatchedFn = void (*)(dim3, hipStream_t, const void* jarr, const WorkUnit* units, int32_t n_units,
                                double eps2, const ForceOut&);
using AdjFn = void (*)(dim3, hipStream_t, const void* jadj, int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                       int64_t jchunk, double eps2, const AdjOut&);
using AdjBatchedFn = void (*)(dim3, hipStream_t, const void* jadj, const WorkUnit* units, int32_t n_units,
                              double eps2, const AdjOut&);

template <typename T, int BS, int I, int TJ, bool POT, int MODE, int LAW>
void launch_force(dim3 g, hipStream_t st, const void* jarr, int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                  int64_t jchunk, double eps2, const ForceOut& o) {
  hipLaunchKernelGGL((force_kernel<T, BS, I, TJ, POT, MODE, LAW>), g, dim3(BS), 0, st,
                     (const typename Vec4<T>::type*)jarr, i0, i1, j0, j1, jchunk, (T)eps2, o);
}
template <typename T, int BS, int I, int TJ, bool POT, int MODE, int LAW>
void launch_force_batched(dim3 g, hipStream_t st, const void* jarr, const WorkUnit* units, int32_t n_units,
                          double eps2, const ForceOut& o) {
  hipLaunchKernelGGL((force_batched_kernel<T, BS, I, TJ, POT, MODE, LAW>), g, dim3(BS), 0, st,
                     (const typename Vec4<T>::type*)jarr, units, n_units, (T)eps2, o);
}
template <typename T, int BS, int I, int TJ, bool COMP>
void launch_adj(dim3 g, hipStream_t st, const void* jadj, int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                int64_t jchunk, double eps2, const AdjOut& o) {
  hipLaunchKernelGGL((adjoint_kernel<T, BS, I, TJ, COMP>), g, dim3(BS), 0, st,
                     (const typename Vec4<T>::type*)jadj, i0, i1, j0, j1, jchunk, (T)eps2, o);
}
template <typename T, int BS, int I, int TJ, bool COMP>
void launch_adj_batched(dim3 g, hipStream_t st, const void* jadj, const WorkUnit* units, int32_t n_units,
                        double eps2, const AdjOut& o) {
  hipLaunchKernelGGL((adjoint_batched_kernel<T, BS, I, TJ, COMP>), g, dim3(BS), 0, st,
                     (const typename Vec4<T>::type*)jadj, units, n_units, (T)eps2, o);
}

struct ForceVariant {
  int bs, i, tj;
  ForceFn fn[2][2][3];            // [law][pot][mode]: plain, compensated, double-float separations
  ForceBatchedFn bfn[2][2][3];
};
struct AdjVariant {
  int bs, i, tj;
  AdjFn fn[2];                    // [comp]
  AdjBatchedFn bfn[2];
};

#define FV32_MODES(F, BS, I, TJ, POT, LAW) \
  { F<float, BS, I, TJ, POT, 0, LAW>, F<float, BS, I, TJ, POT, 1, LAW>, F<float, BS, I, TJ, POT, 2, LAW> }
#define FV32_LAW(F, BS, I, TJ, LAW) \
  { FV32_MODES(F, BS, I, TJ, false, LAW), FV32_MODES(F, BS, I, TJ, true, LAW) }
#define FV32(BS, I, TJ)                                                                                    \
  ForceVariant {                                                                                           \
    BS, I, TJ, {FV32_LAW(launch_force, BS, I, TJ, 0), FV32_LAW(launch_force, BS, I, TJ, 1)},              \
        {FV32_LAW(launch_force_batched, BS, I, TJ, 0), FV32_LAW(launch_force_batched, BS, I, TJ, 1)}      \
  }
#define FV64_LAW(F, BS, I, TJ, LAW) \
  { {F<double, BS, I, TJ, false, 0, LAW>, nullptr, nullptr}, {F<double, BS, I, TJ, true, 0, LAW>, nullptr, nullptr} }
#define FV64(BS, I, TJ)                                                                                    \
  ForceVariant {                                                                                           \
    BS, I, TJ, {FV64_LAW(launch_force, BS, I, TJ, 0), FV64_LAW(launch_force, BS, I, TJ, 1)},              \
        {FV64_LAW(launch_force_batched, BS, I, TJ, 0), FV64_LAW(launch_force_batched, BS, I, TJ, 1)}      \
  }
#define AV32(BS, I, TJ)                                                                                    \
  AdjVariant {                                                                                             \
    BS, I, TJ, {launch_adj<float, BS, I, TJ, false>, launch_adj<float, BS, I, TJ, true>},                 \
        {launch_adj_batched<float, BS, I, TJ, false>, launch_adj_batched<float, BS, I, TJ, true>}        \
  }
#define AV64(BS, I, TJ)                                                                                    \
  AdjVariant {                                                                                             \
    BS, I, TJ, {launch_adj<double, BS, I, TJ, false>, nullptr},                                            \
        {launch_adj_batched<double, BS, I, TJ, false>, nullptr}                                            \
  }

const ForceVariant kForce32[] = {FV32(256, 1, 256), FV32(512, 1, 512), FV32(256, 2, 256), FV32(128, 1, 256),
                                 FV32(64, 1, 128)};
const ForceVariant kForce64[] = {FV64(256, 1, 256), FV64(128, 1, 128), FV64(64, 1, 128)};
const AdjVariant kAdj32[] = {AV32(256, 1, 256), AV32(128, 1, 128), AV32(64, 1, 128)};
const AdjVariant kAdj64[] = {AV64(256, 1, 256), AV64(128, 1, 128), AV64(64, 1, 64)};

// Symmetric FP32 force variants (each pair once), indices kNumForce32 + k in the
// FORCE tile table.
using SymFn = void (*)(dim3, hipStream_t, const float4* jarr, int64_t n, int32_t nb, float eps2, float* part);
using SymAdaptFn = void (*)(dim3, hipStream_t, const float4* jarr, int64_t n, int32_t nb, float eps2, float* part,
                            const AdaptIn& ad);
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
void launch_sym(dim3 g, hipStream_t st, const float4* jarr, int64_t n, int32_t nb, float eps2, float* part) {
  hipLaunchKernelGGL((force_sym_kernel<W, I, POT, MODE, ROT, LAW, PIPE>), g, dim3(W * 64), 0, st, jarr, n, nb, eps2,
                     part, AdaptIn{});
}
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
void launch_sym_adapt(dim3 g, hipStream_t st, const float4* jarr, int64_t n, int32_t nb, float eps2, float* part,
                      const AdaptIn& ad) {
  hipLaunchKernelGGL((force_sym_kernel<W, I, POT, MODE, ROT, LAW, PIPE>), g, dim3(W * 64), 0, st, jarr, n, nb, eps2,
                     part, ad);
}
using SymBatchedFn = void (*)(dim3, hipStream_t, const float4* jarr, const SymUnit* units, int32_t n_units,
                              float eps2, float* part);
template <int W, int I, bool POT, int MODE, int ROT, int LAW, int PIPE>
void launch_sym_batched(dim3 g, hipStream_t st, const float4* jarr, const SymUnit* units, int32_t n_units, float eps2,
                        float* part) {
  hipLaunchKernelGGL((force_sym_batched_kernel<W, I, POT, MODE, ROT, LAW, PIPE>), g, dim3(W * 64), 0, st, jarr,
                     units, n_units, eps2, part);
}
using RolloutFn = void (*)(dim3, hipStream_t, const float4* jarr, const SymUnit* units, int32_t n_solo,
                           int32_t n_units, const int32_t* rtasks, int32_t n_rtasks, int64_t n, const int64_t* sys_off,
                           const int32_t* sys_nb, const int64_t* sys_part, float eps2, float* part, LawScale ls,
                           double* acc, double* vel, double hh, NextStep nx, int32_t steps, RolloutSync sy);
template <int W, int I, int MODE, int ROT, int LAW, int PIPE>
void launch_rollout(dim3 g, hipStream_t st, const float4* jarr, const SymUnit* units, int32_t n_solo, int32_t n_units,
                    const int32_t* rtasks, int32_t n_rtasks, int64_t n, const int64_t* sys_off, const int32_t* sys_nb,
                    const int64_t* sys_part, float eps2, float* part, LawScale ls, double* acc, double* vel, double hh,
                    NextStep nx, int32_t steps, RolloutSync sy) {
  hipLaunchKernelGGL((rollout_sym_batched_kernel<W, I, MODE, ROT, LAW, PIPE>), g, dim3(W * 64), 0, st, jarr, units,
                     n_solo, n_units, rtasks, n_rtasks, n, sys_off, sys_nb, sys_part, eps2, part, ls, acc, vel, hh, nx, steps,
                     sy);
}
template <int W, int I, int MODE, int ROT, int LAW, int PIPE>
const void* rollout_ptr() { return (const void*)&rollout_sym_batched_kernel<W, I, MODE, ROT, LAW, PIPE>; }
// The round schedule (single systems, workspace linear in n) on one fixed tile: 4 waves, 4
// particles per lane, 1024-particle blocks, LDS-crossbar rotation - at the sizes that need it
// (beyond ~1.5M particles) a round holds ~750-1000 tiles, and a launch of several rounds a
// multiple of that (four or five workgroups of this tile fit a CU, by mode: 1024-1280 on the chip).
constexpr int kRoundW = 4, kRoundI = 4, kRoundBlock = kRoundW * 64 * kRoundI;
// Accumulator copies of the round schedule (32 bytes per particle each; the rounds of a launch
// take one each, on two streams): 4 where the copies and a margin of 128 bytes per particle for
// the rest of the workspace fit the partial-sum cap, else 2, else 1. (8 copies, four rounds per
// launch, measured no faster.)
int round_copies(int64_t n, double cap) {
  const double nn = (double)std::max<int64_t>(n, 1);
  for (int k : {4, 2})
    if ((32.0 * k + 128.0) * nn <= cap) return k;
  return 1;
}
using RoundFn = void (*)(dim3, hipStream_t, const float4* jarr, int64_t n, int32_t nb, int32_t nbr, int32_t r,
                         float eps2, double* acc64, AdaptIn ad);
using RoundDiagFn = void (*)(dim3, hipStream_t, const float4* jarr, int64_t n, float eps2, double* acc64, AdaptIn ad);
template <bool POT, int MODE, int LAW>
void launch_round(dim3 g, hipStream_t st, const float4* jarr, int64_t n, int32_t nb, int32_t nbr, int32_t r, float eps2,
                  double* acc64, AdaptIn ad) {
  hipLaunchKernelGGL((force_sym_round_kernel<kRoundW, kRoundI, POT, MODE, 1, LAW, 0>), g, dim3(kRoundW * 64), 0, st,
                     jarr, n, nb, nbr, r, eps2, acc64, ad);
}
template <bool POT, int MODE, int LAW>
void launch_round_diag(dim3 g, hipStream_t st, const float4* jarr, int64_t n, float eps2, double* acc64, AdaptIn ad) {
  constexpr int DM = MODE == MODE_ADAPT ? MODE_ADAPT_DIAG : MODE;
  hipLaunchKernelGGL((force_sym_round_diag_kernel<kRoundW, kRoundI, POT, DM, 1, LAW, 0>), g, dim3(kRoundW * 64), 0,
                     st, jarr, n, eps2, acc64, ad);
}
// Two streams per device on which the round schedule's launches alternate: launches on one
// stream run one after the other, so a launch's last tiles would leave most CUs idle until the
// next launch starts; on two streams the next launch fills them. Created on first use (default
// priority, non-blocking), held until the process ends; calls from several host threads share
// them (their launches then interleave, each call still ordered by its own events).
constexpr int kRoundDevices = 64;
std::mutex g_round_mu;
hipStream_t g_round_st[kRoundDevices][2] = {};

int round_streams(hipStream_t (&out)[2]) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kRoundDevices)
    return fail(NBODY_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kRoundDevices);
  std::lock_guard<std::mutex> lk(g_round_mu);
  for (int k = 0; k < 2; ++k)
    if (!g_round_st[dev][k]) HIP_TRY(hipStreamCreateWithFlags(&g_round_st[dev][k], hipStreamNonBlocking));
  out[0] = g_round_st[dev][0];
  out[1] = g_round_st[dev][1];
  return NBODY_OK;
}

// The rounds 0 .. nbr - 2 of the round schedule after the diagonal tiles (enqueued on st), into K
// accumulator copies of 4 ns doubles from a64; launch(grid, stream, r0, copies) enqueues the
// rounds r0 .. r0 + grid.y - 1 into the copies from `copies`. K = 1: one round per launch. K >= 2:
// launch L runs the K/2 rounds from L K/2 into copies (L mod 2) K/2 .. (L mod 2) K/2 + K/2 - 1,
// on round stream L mod 2; the round streams start after st's work so far and st waits for both
// at the end, also when a launch failed (the workspace must not be reused under running tiles).
// Under stream capture, and in the allocation-free step (g_rounds_one_stream: no stream or event
// is created), the same launches go in order on st (the same sums in the same order, so the same
// results).
thread_local bool g_rounds_one_stream = false;

template <typename Launch>
int run_rounds(hipStream_t st, int64_t ns, int64_t nbr, double* a64, int K, const char* what, Launch&& launch) {
  const int64_t KH = K >= 2 ? K / 2 : 1;
  const int sets = K >= 2 ? 2 : 1;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cap));
  if (sets == 1 || cap != hipStreamCaptureStatusNone || g_rounds_one_stream) {
    int64_t L = 0;
    for (int64_t r = 0; r + 1 < nbr; r += KH, ++L) {
      const unsigned ky = (unsigned)std::min<int64_t>(KH, nbr - 1 - r);
      launch(dim3((unsigned)(nbr / 2), ky), st, (int32_t)r, a64 + (size_t)(L % sets) * KH * 4 * ns);
      LAUNCH_CHECK(what);
    }
    return NBODY_OK;
  }
  hipStream_t rs[2];
  TRY(round_streams(rs));
  struct Events {
    hipEvent_t e[3] = {};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);  // released once the waits on it are done
    }
  } ev;
  for (hipEvent_t& x : ev.e) HIP_TRY(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ev.e[0], st));
  HIP_TRY(hipStreamWaitEvent(rs[0], ev.e[0], 0));
  HIP_TRY(hipStreamWaitEvent(rs[1], ev.e[0], 0));
  hipError_t err = hipSuccess;
  int64_t L = 0;
  for (int64_t r = 0; r + 1 < nbr && err == hipSuccess; r += KH, ++L) {
    const unsigned ky = (unsigned)std::min<int64_t>(KH, nbr - 1 - r);
    launch(dim3((unsigned)(nbr / 2), ky), rs[L & 1], (int32_t)r, a64 + (size_t)(L & 1) * KH * 4 * ns);
    err = hipGetLastError();
  }
  hipError_t j0 = hipEventRecord(ev.e[1], rs[0]);
  if (j0 == hipSuccess) j0 = hipStreamWaitEvent(st, ev.e[1], 0);
  hipError_t j1 = hipEventRecord(ev.e[2], rs[1]);
  if (j1 == hipSuccess) j1 = hipStreamWaitEvent(st, ev.e[2], 0);
  if (j0 != hipSuccess || j1 != hipSuccess) {  // no ordering on st: wait here instead
    (void)hipStreamSynchronize(rs[0]);
    (void)hipStreamSynchronize(rs[1]);
    return fail(NBODY_ERR_DEVICE, "round streams: %s", hipGetErrorString(j0 != hipSuccess ? j0 : j1));
  }
  if (err != hipSuccess) return fail(NBODY_ERR_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(err));
  return NBODY_OK;
}

// The adjoint pass on the round schedule: the same tile shape, [comp].
using AdjRoundFn = void (*)(dim3, hipStream_t, const float4* jadj, int64_t n, int32_t nb, int32_t nbr, int32_t r,
                            float eps2, double* acc64);
using AdjRoundDiagFn = void (*)(dim3, hipStream_t, const float4* jadj, int64_t n, float eps2, double* acc64);
template <bool COMP>
void launch_adj_round(dim3 g, hipStream_t st, const float4* jadj, int64_t n, int32_t nb, int32_t nbr, int32_t r,
                      float eps2, double* acc64) {
  hipLaunchKernelGGL((adjoint_sym_round_kernel<kRoundW, kRoundI, COMP, 1>), g, dim3(kRoundW * 64), 0, st, jadj, n, nb,
                     nbr, r, eps2, acc64);
}
template <bool COMP>
void launch_adj_round_diag(dim3 g, hipStream_t st, const float4* jadj, int64_t n, float eps2, double* acc64) {
  hipLaunchKernelGGL((adjoint_sym_round_diag_kernel<kRoundW, kRoundI, COMP, 1>), g, dim3(kRoundW * 64), 0, st, jadj,
                     n, eps2, acc64);
}
const AdjRoundFn kAdjRound[2] = {launch_adj_round<false>, launch_adj_round<true>};
const AdjRoundDiagFn kAdjRoundDiag[2] = {launch_adj_round_diag<false>, launch_adj_round_diag<true>};

// [law][pot][mode]: modes 0-2 as force_mode, 3 the adaptive mode (sorted particles)
#define RND_POT(POT, LAW) \
  { launch_round<POT, 0, LAW>, launch_round<POT, 1, LAW>, launch_round<POT, 2, LAW>, launch_round<POT, 3, LAW> }
const RoundFn kRound[2][2][4] = {{RND_POT(false, 0), RND_POT(true, 0)}, {RND_POT(false, 1), RND_POT(true, 1)}};
#define RND_DIAG_POT(POT, LAW)                                                                      \
  {                                                                                                 \
    launch_round_diag<POT, 0, LAW>, launch_round_diag<POT, 1, LAW>, launch_round_diag<POT, 2, LAW>, \
        launch_round_diag<POT, 3, LAW>                                                              \
  }
const RoundDiagFn kRoundDiag[2][2][4] = {{RND_DIAG_POT(false, 0), RND_DIAG_POT(true, 0)},
                                         {RND_DIAG_POT(false, 1), RND_DIAG_POT(true, 1)}};
struct SymVariant {
  int w, i, rot;      // rot: 0 = DPP lane rotation, 1 = LDS-crossbar (ds_bpermute) rotation
  int pipe;           // coordinate rotation issued after phase 1 (0) or a step ahead (1)
  SymFn fn[2][2][3];  // [law][pot][mode]
  SymAdaptFn afn[2][2];  // [law][pot]: the adaptive mode's off-diagonal tiles (single systems)
  SymAdaptFn dfn[2][2];  // [law][pot]: its diagonal tiles
  SymBatchedFn bfn[2][2][3];
  RolloutFn rfn[2][3];  // whole batched rollout [law][mode] (no potential)
  const void* (*rptr[2][3])();
};
#define SV32_POT(F, W, I, R, P, POT, LAW) \
  { F<W, I, POT, 0, R, LAW, P>, F<W, I, POT, 1, R, LAW, P>, F<W, I, POT, 2, R, LAW, P> }
#define SV32_ALL(F, W, I, R, P)                                                                           \
  {{SV32_POT(F, W, I, R, P, false, 0), SV32_POT(F, W, I, R, P, true, 0)},                                 \
   {SV32_POT(F, W, I, R, P, false, 1), SV32_POT(F, W, I, R, P, true, 1)}}
#define SV32_RO(F, W, I, R, P, LAW) \
  { F<W, I, 0, R, LAW, P>, F<W, I, 1, R, LAW, P>, F<W, I, 2, R, LAW, P> }
#define SV32_AD(W, I, R, P, M)                                                                             \
  {{launch_sym_adapt<W, I, false, M, R, 0, P>, launch_sym_adapt<W, I, true, M, R, 0, P>},                  \
   {launch_sym_adapt<W, I, false, M, R, 1, P>, launch_sym_adapt<W, I, true, M, R, 1, P>}}
#define SV32P(W, I, R, P)                                                                                  \
  SymVariant { W, I, R, P, SV32_ALL(launch_sym, W, I, R, P), SV32_AD(W, I, R, P, MODE_ADAPT),              \
               SV32_AD(W, I, R, P, MODE_ADAPT_DIAG),                                                       \
               SV32_ALL(launch_sym_batched, W, I, R, P),                                                   \
               {SV32_RO(launch_rollout, W, I, R, P, 0), SV32_RO(launch_rollout, W, I, R, P, 1)},          \
               {SV32_RO(rollout_ptr, W, I, R, P, 0), SV32_RO(rollout_ptr, W, I, R, P, 1)} }
#define SV32(W, I, R) SV32P(W, I, R, 0)
const SymVariant kSym32[] = {SV32(8, 4, 0), SV32(4, 4, 0), SV32(8, 2, 0), SV32(4, 2, 0), SV32(2, 4, 0),
                             SV32(8, 4, 1), SV32(4, 4, 1), SV32(4, 8, 0), SV32(4, 8, 1), SV32(2, 4, 1),
                             SV32(4, 2, 1), SV32(2, 2, 1), SV32P(8, 4, 1, 1), SV32P(4, 8, 1, 1),
                             SV32P(4, 4, 1, 1), SV32(1, 4, 1), SV32(1, 2, 1), SV32(1, 2, 0), SV32(1, 2, 2),
                             SV32(1, 4, 2), SV32(2, 2, 2), SV32(2, 4, 2)};
constexpr int kNumSym32 = sizeof(kSym32) / sizeof(kSym32[0]);

// Symmetric FP32 adjoint variants, indices kNumAdj32 + k in the ADJOINT tables.
template <int W, int I, bool COMP, int ROT>
void launch_adj_sym(dim3 g, hipStream_t st, const float4* jadj, int64_t n, int32_t nb, float eps2, float* part) {
  hipLaunchKernelGGL((adjoint_sym_kernel<W, I, COMP, ROT>), g, dim3(W * 64), 0, st, jadj, n, nb, eps2, part);
}
template <int W, int I, bool COMP, int ROT>
void launch_adj_sym_batched(dim3 g, hipStream_t st, const float4* jadj, const SymUnit* units, int32_t n_units,
                            float eps2, float* part) {
  hipLaunchKernelGGL((adjoint_sym_batched_kernel<W, I, COMP, ROT>), g, dim3(W * 64), 0, st, jadj, units, n_units,
                     eps2, part);
}
struct AdjSymVariant {
  int w, i, rot;
  SymFn fn[2];  // [comp]
  SymBatchedFn bfn[2];
};
#define SA32(W, I, R)                                                                                     \
  AdjSymVariant {                                                                                         \
    W, I, R, {launch_adj_sym<W, I, false, R>, launch_adj_sym<W, I, true, R>},                            \
        {launch_adj_sym_batched<W, I, false, R>, launch_adj_sym_batched<W, I, true, R>}                  \
  }
const AdjSymVariant kAdjSym32[] = {SA32(4, 2, 1), SA32(2, 2, 1), SA32(4, 4, 1), SA32(2, 4, 1), SA32(8, 2, 1),
                                   SA32(4, 2, 0), SA32(2, 4, 0), SA32(1, 4, 1), SA32(1, 2, 1), SA32(1, 2, 0),
                                   SA32(1, 2, 2), SA32(1, 4, 2)};
constexpr int kNumAdjSym32 = sizeof(kAdjSym32) / sizeof(kAdjSym32[0]);

constexpr int kNumForce32 = sizeof(kForce32) / sizeof(kForce32[0]);
constexpr int kNumForce64 = sizeof(kForce64) / sizeof(kForce64[0]);
constexpr int kNumAdj32 = sizeof(kAdj32) / sizeof(kAdj32[0]);
constexpr int kNumAdj64 = sizeof(kAdj64) / sizeof(kAdj64[0]);

bool is_fp64(int prec) { return prec == NBODY_FP64; }
bool is_adapt(int prec) { return prec == NBODY_FP32_ADAPT; }
// double-float j-array layout (two float4 per particle): the double-float mode, and the
// adaptive mode wherever it runs as the double-float mode (batches, one-sided passes)
bool is_ds(int prec) { return prec == NBODY_FP32_DS || prec == NBODY_FP32_ADAPT; }
// force-kernel mode index: 0 plain float / double, 1 compensated, 2 double-float separations
// (the adaptive mode's own symmetric path is launched separately)
int force_mode(int prec) { return prec == NBODY_FP32_COMP ? 1 : is_ds(prec) ? 2 : 0; }
// adjoint kernels: compensated for every compensated mode
int adj_comp(int prec) { return prec == NBODY_FP32_COMP || is_ds(prec); }
// bytes of one particle in the force j-array and in the adjoint j-array
size_t jvec_bytes(int prec) { return is_fp64(prec) ? 32 : is_ds(prec) ? 32 : 16; }
size_t jadj_bytes(int prec) { return is_fp64(prec) ? 64 : 32; }

// The Lennard-Jones force kernels share the gravity kernels' variants (the pair law
// is a template parameter of the same tiles); only their tile-table entries differ.
int base_kernel(int kernel) {
  return kernel == NBODY_KERNEL_LJ_FORCE ? NBODY_KERNEL_FORCE
         : kernel == NBODY_KERNEL_LJ_FORCE_BATCHED ? NBODY_KERNEL_FORCE_BATCHED : kernel;
}
int force_kernel_id(int law, bool batched) {
  if (law == LAW_LJ) return batched ? NBODY_KERNEL_LJ_FORCE_BATCHED : NBODY_KERNEL_LJ_FORCE;
  return batched ? NBODY_KERNEL_FORCE_BATCHED : NBODY_KERNEL_FORCE;
}
constexpr int kNumKernels = 6;

bool is_force_kernel(int kernel) {
  kernel = base_kernel(kernel);
  return kernel == NBODY_KERNEL_FORCE || kernel == NBODY_KERNEL_FORCE_BATCHED;
}

int num_variants(int kernel, int prec) {
  const bool f = is_force_kernel(kernel);
  if (f && !is_fp64(prec)) return kNumForce32 + kNumSym32;
  if (f) return kNumForce64;
  return is_fp64(prec) ? kNumAdj64 : kNumAdj32 + kNumAdjSym32;
}

// Symmetric variant index (or -1) of a tile variant: into kSym32 for the force kernels,
// into kAdjSym32 for the adjoint kernels (FP32 modes only).
int sym_index(int kernel, int prec, int v) {
  if (is_fp64(prec)) return -1;
  const int first = is_force_kernel(kernel) ? kNumForce32 : kNumAdj32;
  return v < first ? -1 : v - first;
}

// (waves, i-particles per lane, rotation kind) of symmetric variant sv
void sym_shape(int kernel, int sv, int& w, int& i, int& rot) {
  if (is_force_kernel(kernel)) {
    w = kSym32[sv].w; i = kSym32[sv].i; rot = kSym32[sv].rot;
  } else {
    w = kAdjSym32[sv].w; i = kAdjSym32[sv].i; rot = kAdjSym32[sv].rot;
  }
}

void variant_shape(int kernel, int prec, int v, int& bs, int& i, int& tj) {
  kernel = base_kernel(kernel);
  bool f = kernel == NBODY_KERNEL_FORCE || kernel == NBODY_KERNEL_FORCE_BATCHED;
  int sv = sym_index(kernel, prec, v);
  if (sv >= 0) {
    // symmetric: block of bs = W*64 threads, i per lane, tile edge tj = W*64*I
    int w, rot;
    sym_shape(kernel, sv, w, i, rot);
    bs = w * 64;
    tj = bs * i;
    return;
  }
  if (f) {
    const ForceVariant& fv = is_fp64(prec) ? kForce64[v] : kForce32[v];
    bs = fv.bs; i = fv.i; tj = fv.tj;
  } else {
    const AdjVariant& av = is_fp64(prec) ? kAdj64[v] : kAdj32[v];
    bs = av.bs; i = av.i; tj = av.tj;
  }
}

// ------------------------------------------------------------------ tile table

std::mutex g_table_mu;
std::vector<nbody_tile_entry> g_table;

struct Tile {
  int variant;
  int bs, i, tj;
  int64_t j_split;  // single: number of j-ranges; batched: j-chunk length
  int sym = -1;     // symmetric variant index (single-system FP32 force only)
  bool rounds = false;  // single-system FP32 force on the round schedule (workspace linear in n)
};

int g_num_cu = 0;
int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      g_num_cu = cu;
    else
      g_num_cu = 256;
  }
  return g_num_cu;
}

// Built-in defaults: one lane per i-particle; the j-range is split until the grid
// holds about 8 blocks per CU; batched j-chunks of 1024.
Tile default_tile(int kernel, int prec, int64_t n) {
  kernel = base_kernel(kernel);
  Tile t{};
  bool batched = kernel == NBODY_KERNEL_FORCE_BATCHED || kernel == NBODY_KERNEL_ADJOINT_BATCHED;
  t.variant = 0;
  if (n <= 4096) t.variant = (kernel == NBODY_KERNEL_FORCE || kernel == NBODY_KERNEL_FORCE_BATCHED)
                                 ? (is_fp64(prec) ? 1 : 3) : 1;
  if (kernel == NBODY_KERNEL_FORCE && !is_fp64(prec)) {
    if (n >= 262144) t.variant = kNumForce32 + 0;      // symmetric, 2048-particle blocks
    else if (n >= 32768) t.variant = kNumForce32 + 1;  // symmetric, 1024-particle blocks
  }
  t.sym = sym_index(kernel, prec, t.variant);
  variant_shape(kernel, prec, t.variant, t.bs, t.i, t.tj);
  if (t.sym >= 0) {
    t.j_split = 1;
    return t;
  }
  if (batched) {
    t.j_split = 1024;
  } else {
    int64_t nblk = cdiv(std::max<int64_t>(n, 1), (int64_t)t.bs * t.i);
    int64_t want = (int64_t)num_cu() * 8;
    int64_t S = std::max<int64_t>(1, cdiv(want, nblk));
    S = std::min<int64_t>(S, std::max<int64_t>(1, n / (4 * t.tj)));
    S = std::min<int64_t>(S, 64);
    t.j_split = S;
  }
  return t;
}

Tile lookup_tile(int kernel, int prec, int64_t n);

// Entry of the table for exactly this kernel id (no fallback); false when none matches.
bool find_entry(int kernel, int prec, int64_t n, Tile& out);

// Symmetric tiles keep one float slot per (particle, other block): nb * 4 * n * 4 bytes, O(n^2).
// A single-system force pass whose slots would exceed the cap runs on the table's tile for the
// largest systems (the largest block, so the fewest slots) when that fits, else on the round
// schedule (4 doubles per particle) when that fits, else one-sided (no partial sums with one
// j-range); an adjoint pass on the round schedule when that fits, else one-sided. The default cap is reached near 1.5M particles by the
// tuned table's symmetric entries. The allocation-free step (on its own thread, for its own call)
// sets the cap to its static scratch and a level that skips the first choices of that order:
// 1 starts at the largest block, 2 at the round schedule, 3 at the one-sided pass.
constexpr double kSymPartCap = 16.0 * (double)(1ull << 30);
thread_local double g_sym_cap = kSymPartCap;
thread_local int g_sym_level = 0;

Tile lookup_tile_raw(int kernel, int prec, int64_t n);

// A single-system force pass on the round schedule (the fields a one-sided tile would have, so
// no path mistakes it for the slot schedule).
Tile rounds_tile(int kernel, int prec) {
  Tile r{};
  r.variant = 0;
  r.sym = -1;
  variant_shape(kernel, prec, 0, r.bs, r.i, r.tj);
  r.j_split = 1;
  r.rounds = true;
  return r;
}

Tile lookup_tile(int kernel, int prec, int64_t n) {
  Tile t = lookup_tile_raw(kernel, prec, n);
  const int bk = base_kernel(kernel);
  const bool single = bk == NBODY_KERNEL_FORCE || bk == NBODY_KERNEL_ADJOINT;
  auto slot_bytes = [&](const Tile& x) { return (double)cdiv(std::max<int64_t>(n, 1), (int64_t)x.tj) * 16.0 * (double)n; };
  if (single && t.sym >= 0 && (g_sym_level > 0 || slot_bytes(t) > g_sym_cap)) {
    if (bk == NBODY_KERNEL_FORCE) {
      const Tile big = lookup_tile_raw(kernel, prec, (int64_t)1 << 40);
      if (g_sym_level <= 1 && big.sym >= 0 && slot_bytes(big) <= g_sym_cap) return big;
    }
    // the round schedule's accumulators: 4 doubles per particle
    if (g_sym_level <= 2 && 32.0 * (double)std::max<int64_t>(n, 1) <= g_sym_cap) return rounds_tile(kernel, prec);
    // the one-sided variant of the built-in defaults, one j-range per block column
    Tile o{};
    o.variant = 0;
    o.sym = -1;
    variant_shape(kernel, prec, o.variant, o.bs, o.i, o.tj);
    o.j_split = 1;
    return o;
  }
  // one-sided: the j-range partials ([S][4][n] doubles, [S][8][n] for the adjoint) under the cap
  const double per_split = (bk == NBODY_KERNEL_ADJOINT ? 64.0 : 32.0) * (double)std::max<int64_t>(n, 1);
  if (single && t.sym < 0 && (double)t.j_split * per_split > g_sym_cap)
    t.j_split = std::max<int64_t>(1, (int64_t)(g_sym_cap / per_split));
  return t;
}

// The tile of a single-system force or adjoint pass under cfg: NBODY_FLAG_SYM_ROUNDS puts every
// FP32 pass on the round schedule.
Tile single_force_tile(const nbody_config* cfg, int kernel, int prec, int64_t n) {
  if ((cfg->flags & NBODY_FLAG_SYM_ROUNDS) && !is_fp64(prec)) return rounds_tile(kernel, prec);
  return lookup_tile(kernel, prec, n);
}
Tile single_adj_tile(const nbody_config* cfg, int prec, int64_t n) {
  return single_force_tile(cfg, NBODY_KERNEL_ADJOINT, prec, n);
}

Tile lookup_tile_raw(int kernel, int prec, int64_t n) {
  Tile t;
  // the adaptive mode without entries of its own runs with the compensated mode's tiles (its
  // float loop is the compensated one)
  for (int p : {prec, is_adapt(prec) ? (int)NBODY_FP32_COMP : -1}) {
    if (p < 0) continue;
    if (find_entry(kernel, p, n, t)) return t;
    // a Lennard-Jones kernel without its own entry runs with the gravity kernel's tile
    if (base_kernel(kernel) != kernel && find_entry(base_kernel(kernel), p, n, t)) return t;
  }
  return default_tile(kernel, prec, n);
}

bool find_entry(int kernel, int prec, int64_t n, Tile& out) {
  std::lock_guard<std::mutex> lk(g_table_mu);
  for (const auto& e : g_table) {
    if (e.kernel == kernel && e.precision == prec && n >= e.n_min && n <= e.n_max &&
        e.variant >= 0 && e.variant < num_variants(kernel, prec) && e.j_split >= 1) {
      Tile t{};
      t.variant = e.variant;
      t.sym = sym_index(kernel, prec, t.variant);
      variant_shape(kernel, prec, t.variant, t.bs, t.i, t.tj);
      t.j_split = t.sym >= 0 ? 1 : e.j_split;
      const int bk = base_kernel(kernel);
      bool batched = bk == NBODY_KERNEL_FORCE_BATCHED || bk == NBODY_KERNEL_ADJOINT_BATCHED;
      if (batched) t.j_split = std::max<int64_t>(t.tj, cdiv(t.j_split, t.tj) * t.tj);
      out = t;
      return true;
    }
  }
  return false;
}

// Effective number of j-ranges and their length (a multiple of TJ).
void split_geometry(const Tile& t, int64_t nj, int64_t& S, int64_t& jchunk) {
  S = std::max<int64_t>(1, t.j_split);
  int64_t ntiles = std::max<int64_t>(1, cdiv(nj, t.tj));
  if (S > ntiles) S = ntiles;
  jchunk = cdiv(ntiles, S) * t.tj;
  S = std::max<int64_t>(1, cdiv(std::max<int64_t>(nj, 1), jchunk));
}

// ------------------------------------------------------------------ validation

struct Systems {
  int64_t S;
  const int64_t* off;  // host
  int64_t max_n;
};

// law_checks: validate G and eps (gravity calls); the workspace size and the
// Lennard-Jones calls do not use them.
int check_cfg(const nbody_config* cfg, int64_t n, Systems& sys, bool law_checks = true) {
  if (!cfg) return fail(NBODY_ERR_INVALID_ARG, "cfg is NULL");
  if (cfg->abi_version != NBODY_ABI_VERSION)
    return fail(NBODY_ERR_INVALID_ARG, "abi_version %d does not match library ABI %d", cfg->abi_version,
                NBODY_ABI_VERSION);
  if (cfg->precision != NBODY_FP64 && cfg->precision != NBODY_FP32 && cfg->precision != NBODY_FP32_COMP &&
      cfg->precision != NBODY_FP32_DS && cfg->precision != NBODY_FP32_ADAPT)
    return fail(NBODY_ERR_INVALID_ARG, "unknown precision %d", cfg->precision);
  if (law_checks) {
    if (!std::isfinite(cfg->G)) return fail(NBODY_ERR_INVALID_ARG, "G must be finite");
    if (!(cfg->eps > 0.0) || !std::isfinite(cfg->eps))
      return fail(NBODY_ERR_INVALID_ARG, "eps must be finite and > 0 (got %g)", cfg->eps);
    if (cfg->precision != NBODY_FP64 && cfg->eps < 1e-10)
      return fail(NBODY_ERR_INVALID_ARG, "eps must be >= 1e-10 for the FP32 modes (got %g)", cfg->eps);
  }
  if (cfg->reserved != 0) return fail(NBODY_ERR_INVALID_ARG, "reserved must be 0");
  if (cfg->flags & ~(NBODY_FLAG_LOOP_SYSTEMS | NBODY_FLAG_WHOLE_ROLLOUT | NBODY_FLAG_PER_PASS | NBODY_FLAG_SYM_ROUNDS))
    return fail(NBODY_ERR_INVALID_ARG, "unknown flags 0x%x", cfg->flags);
  if (n < 0) return fail(NBODY_ERR_INVALID_ARG, "n must be >= 0 (got %lld)", (long long)n);
  if (n > ((int64_t)1 << 31)) return fail(NBODY_ERR_UNSUPPORTED, "n = %lld exceeds 2^31", (long long)n);
  if (cfg->n_systems < 1) return fail(NBODY_ERR_INVALID_ARG, "n_systems must be >= 1");
  sys.S = cfg->n_systems;
  sys.off = cfg->offsets;
  sys.max_n = n;
  if (cfg->offsets) {
    if (cfg->offsets[0] != 0) return fail(NBODY_ERR_INVALID_ARG, "offsets[0] must be 0");
    int64_t mx = 0;
    for (int64_t s = 0; s < cfg->n_systems; ++s) {
      if (cfg->offsets[s + 1] < cfg->offsets[s])
        return fail(NBODY_ERR_INVALID_ARG, "offsets must be non-decreasing (offsets[%lld] > offsets[%lld])",
                    (long long)s, (long long)(s + 1));
      mx = std::max(mx, cfg->offsets[s + 1] - cfg->offsets[s]);
    }
    if (cfg->offsets[cfg->n_systems] != n)
      return fail(NBODY_ERR_INVALID_ARG, "offsets[n_systems] = %lld must equal n = %lld",
                  (long long)cfg->offsets[cfg->n_systems], (long long)n);
    sys.max_n = mx;
  } else if (cfg->n_systems != 1) {
    return fail(NBODY_ERR_INVALID_ARG, "offsets may be NULL only when n_systems == 1");
  }
  return NBODY_OK;
}

// ------------------------------------------------------------------ workspace plan

struct Plan {
  // batched metadata
  size_t off_meta = 0, sz_meta = 0;
  size_t off_sysoff = 0, off_nsplit = 0, off_partoff = 0, off_partoff_adj = 0, off_units = 0, off_units_adj = 0,
         off_sync = 0, off_rtasks = 0, off_units_ro = 0;
  int64_t n_units_force = 0, n_units_adj = 0;
  // buffers
  size_t off_jbuf = 0, sz_jbuf = 0;
  size_t off_part = 0, sz_part = 0;
  size_t off_epart = 0, sz_epart = 0;
  size_t off_pot = 0, sz_pot = 0;
  size_t off_accs = 0, sz_accs = 0;   // scratch acc [3][n]
  size_t off_xw = 0, off_vw = 0, off_aw = 0, sz_state = 0;
  size_t off_seg = 0, sz_seg = 0;
  // adaptive mode (single system on symmetric tiles): sort keys, permutation, sub-block
  // boxes, bounding-box partials and the box with T^2
  bool adapt = false;
  int64_t adapt_padded = 0;
  int32_t adapt_bblocks = 0;
  size_t off_keys = 0, off_perm = 0, off_box = 0, off_bbpart = 0, off_bbox = 0;
  size_t total = 0;
  int32_t e_chunks = 1;
  int32_t e_steps = 1;  // steps whose energy partials a rollout keeps before one final sum
};

// A rollout with an energy trace sums the energy partials of up to this many steps in one
// launch, keeping at most this many bytes of them.
constexpr size_t kEnergySteps = 32;
constexpr size_t kEnergyBytes = (size_t)8 << 20;

struct UnitSet {
  std::vector<WorkUnit> units;     // one-sided units (i-tile x j-chunk)
  std::vector<int32_t> nsplit;     // per system: j-chunks (one-sided) or blocks nb (symmetric)
  std::vector<SymUnit> sym_units;  // symmetric units (tile (A, B) of one system)
  std::vector<int64_t> part_off;   // symmetric: float offset of each system's partial planes
  std::vector<SymUnit> ro_units;   // symmetric, whole rollout: one-tile systems, then the other units
  int64_t n_solo = 0;              //   (the first n_solo of ro_units run all their steps in one task)
  std::vector<int32_t> rtasks;     //   reduction tasks of the systems of several tiles: (system, chunk)
  int64_t part_floats = 0;         // symmetric: floats of all systems' partial planes
  bool sym = false;
  int64_t count() const { return sym ? (int64_t)sym_units.size() : (int64_t)units.size(); }
  size_t unit_bytes() const { return sym ? sym_units.size() * sizeof(SymUnit) : units.size() * sizeof(WorkUnit); }
};

// Work units of a batched pass: i-tiles of bs*i particles x j-chunks of jc particles
// inside each system, sorted by decreasing cost (longest-processing-time order).
void build_units(const Systems& sys, const Tile& t, UnitSet& us) {
  us.units.clear();
  us.nsplit.assign(sys.S, 0);
  const int64_t ti = (int64_t)t.bs * t.i, jc = t.j_split;
  for (int64_t s = 0; s < sys.S; ++s) {
    const int64_t b = sys.off[s], e = sys.off[s + 1], ns = e - b;
    if (ns == 0) continue;
    const int64_t nsp = cdiv(ns, jc);
    us.nsplit[s] = (int32_t)nsp;
    for (int64_t ib = b; ib < e; ib += ti)
      for (int64_t p = 0; p < nsp; ++p) {
        WorkUnit w{};
        w.ib = ib;
        w.ie = std::min(ib + ti, e);
        w.jb = b + p * jc;
        w.je = std::min(w.jb + jc, e);
        w.slot = (int32_t)p;
        us.units.push_back(w);
      }
  }
  std::stable_sort(us.units.begin(), us.units.end(), [](const WorkUnit& a, const WorkUnit& b) {
    return (a.ie - a.ib) * (a.je - a.jb) > (b.ie - b.ib) * (b.je - b.jb);
  });
}

// Symmetric units of a batched pass: every upper-triangle tile (A, B) of blocks of
// t.tj particles inside each system, sorted by decreasing pair count.
void build_sym_units(const Systems& sys, const Tile& t, UnitSet& us, int comps) {
  us = UnitSet{};
  us.sym = true;
  us.nsplit.assign(sys.S, 0);
  us.part_off.assign(sys.S + 1, 0);
  const int64_t bi = t.tj;
  int64_t off = 0;
  for (int64_t s = 0; s < sys.S; ++s) {
    const int64_t b = sys.off[s], ns = sys.off[s + 1] - b;
    us.part_off[s] = off;
    if (ns == 0) continue;
    const int64_t nb = cdiv(ns, bi);
    us.nsplit[s] = (int32_t)nb;
    for (int64_t A = 0; A < nb; ++A)
      for (int64_t B = A; B < nb; ++B) {
        SymUnit u{};
        u.base = b;
        u.part_off = off;
        u.n = (int32_t)ns;
        u.nb = (int32_t)nb;
        u.A = (int32_t)A;
        u.B = (int32_t)B;
        u.sys = (int32_t)s;
        us.sym_units.push_back(u);
      }
    for (int64_t ch = 0; nb > 1 && ch * kRolloutChunk < ns; ++ch) {
      us.rtasks.push_back((int32_t)s);
      us.rtasks.push_back((int32_t)ch);
    }
    off += nb * comps * ns;
  }
  us.part_off[sys.S] = off;
  us.part_floats = off;
  auto rows = [bi](const SymUnit& u, int32_t X) { return std::min<int64_t>(bi, (int64_t)u.n - (int64_t)X * bi); };
  std::stable_sort(us.sym_units.begin(), us.sym_units.end(), [&](const SymUnit& a, const SymUnit& b) {
    return rows(a, a.A) * rows(a, a.B) > rows(b, b.A) * rows(b, b.B);
  });
  // whole-rollout order: the one-tile systems (largest first), then the other units as above
  us.ro_units.clear();
  for (const SymUnit& u : us.sym_units)
    if (u.nb == 1) us.ro_units.push_back(u);
  us.n_solo = (int64_t)us.ro_units.size();
  for (const SymUnit& u : us.sym_units)
    if (u.nb > 1) us.ro_units.push_back(u);
}

int64_t max_nsplit(const UnitSet& us) {
  int64_t m = 1;
  for (auto v : us.nsplit) m = std::max<int64_t>(m, v);
  return m;
}

enum Need : unsigned { NEED_FORCE = 1, NEED_ENERGY = 2, NEED_ROLLOUT = 4, NEED_BACKWARD = 8 };

// Workspace layout of a call. The force regions are sized for the larger of the two
// pair laws' tiles, so one size (nbody_workspace_size) serves both; the batched work
// units are those of `law`.
int make_plan(const nbody_config* cfg, const Systems& sys, int64_t n, int64_t ckpt_every, unsigned need,
              Plan& p, UnitSet* uf, UnitSet* ua, int law = LAW_GRAV) {
  const int prec = cfg->precision;
  const bool bat = sys.S > 1;
  const bool loop = bat && (cfg->flags & NBODY_FLAG_LOOP_SYSTEMS);
  const size_t dsz = sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  int64_t force_S = 1, adj_S = 1;
  size_t force_part = 0, adj_part = 0;  // bytes of partial sums each pass writes
  const size_t nd = (size_t)n * dsz;
  UnitSet local_f, local_a;
  UnitSet& ufs = uf ? *uf : local_f;
  UnitSet& uas = ua ? *ua : local_a;
  // partial sums of one system of ns particles under tile t (0 when written directly)
  auto single_force_part = [&](const Tile& t, int64_t ns) -> size_t {
    if (t.rounds)  // the round schedule's accumulator copies
      return (size_t)round_copies(ns, g_sym_cap) * 4 * (size_t)ns * sizeof(double);
    if (t.sym >= 0) {
      const int64_t nb = cdiv(ns, (int64_t)t.tj);
      return (size_t)nb * 4 * (size_t)ns * sizeof(float);
    }
    int64_t S, jc;
    split_geometry(t, ns, S, jc);
    return S > 1 ? (size_t)S * 4 * nd : 0;
  };
  auto single_adj_part = [&](const Tile& t, int64_t ns) -> size_t {
    if (t.rounds)  // the round schedule's accumulator copies
      return (size_t)round_copies(ns, g_sym_cap) * 4 * (size_t)ns * sizeof(double);
    if (t.sym >= 0) {
      const int64_t nb = cdiv(ns, (int64_t)t.tj);
      return (size_t)nb * 4 * (size_t)ns * sizeof(float);
    }
    int64_t S, jc;
    split_geometry(t, ns, S, jc);
    return S > 1 ? (size_t)S * 8 * nd : 0;
  };
  size_t units_bytes = 0;  // force work-unit bytes reserved (either law, either unit kind)
  if (bat && !loop) {
    for (int lw : {LAW_GRAV, LAW_LJ}) {
      UnitSet tmp;
      const Tile tf = lookup_tile(force_kernel_id(lw, true), prec, sys.max_n);
      if (tf.sym >= 0) {
        build_sym_units(sys, tf, tmp, 4);
        force_part = std::max(force_part, (size_t)tmp.part_floats * sizeof(float));
      } else {
        build_units(sys, tf, tmp);
        force_S = std::max(force_S, max_nsplit(tmp));
        force_part = std::max(force_part, (size_t)max_nsplit(tmp) * 4 * nd);  // batched one-sided units always write partials
      }
      units_bytes = std::max(units_bytes, tmp.unit_bytes());
      if (lw == law) ufs = std::move(tmp);
    }
    p.n_units_force = ufs.count();
    if (p.n_units_force > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many batched work units");
    if (need & NEED_BACKWARD) {
      Tile ta = lookup_tile(NBODY_KERNEL_ADJOINT_BATCHED, prec, sys.max_n);
      if (ta.sym >= 0) {
        build_sym_units(sys, ta, uas, 4);
        adj_part = (size_t)uas.part_floats * sizeof(float);
      } else {
        build_units(sys, ta, uas);
        adj_S = max_nsplit(uas);
        adj_part = (size_t)adj_S * 8 * nd;
      }
      p.n_units_adj = uas.count();
      if (p.n_units_adj > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many batched work units");
    }
    p.off_meta = off;
    p.off_sysoff = take((sys.S + 1) * sizeof(int64_t));
    p.off_nsplit = take(2 * sys.S * sizeof(int32_t));  // force then adjoint split counts
    p.off_partoff = take((sys.S + 1) * sizeof(int64_t));
    p.off_partoff_adj = take((sys.S + 1) * sizeof(int64_t));
    p.off_units = take(units_bytes);
    p.off_units_adj = take(uas.unit_bytes());
    p.off_sync = take(16 + 2 * sys.S * sizeof(int32_t));  // whole-rollout queue, error word, per-system counts
    int64_t rchunks = 0;  // whole-rollout reduction tasks (the same for either law and tile)
    for (int64_t s = 0; s < sys.S; ++s) rchunks += cdiv(sys.off[s + 1] - sys.off[s], kRolloutChunk);
    p.off_rtasks = take(2 * rchunks * sizeof(int32_t));
    p.off_units_ro = take(units_bytes);  // the force units again, in whole-rollout order
    p.sz_meta = off - p.off_meta;
  } else if (loop) {
    for (int64_t s = 0; s < sys.S; ++s) {
      int64_t ns = sys.off[s + 1] - sys.off[s];
      if (ns == 0) continue;
      for (int lw : {LAW_GRAV, LAW_LJ})
        force_part =
            std::max(force_part, single_force_part(single_force_tile(cfg, force_kernel_id(lw, false), prec, ns), ns));
      if (need & NEED_BACKWARD)
        adj_part = std::max(adj_part, single_adj_part(single_adj_tile(cfg, prec, ns), ns));
    }
  } else {
    for (int lw : {LAW_GRAV, LAW_LJ})
      force_part =
          std::max(force_part, single_force_part(single_force_tile(cfg, force_kernel_id(lw, false), prec, n), n));
    if (need & NEED_BACKWARD) adj_part = single_adj_part(single_adj_tile(cfg, prec, n), n);
  }
  p.sz_jbuf = (size_t)n * std::max(jvec_bytes(prec), (need & NEED_BACKWARD) ? jadj_bytes(prec) : (size_t)0);
  p.off_jbuf = take(p.sz_jbuf);
  p.sz_part = std::max(force_part, adj_part);
  p.off_part = take(p.sz_part);
  // the adaptive mode sorts a single system whose force pass runs on symmetric tiles (the slot
  // or the round schedule)
  auto symmetric = [](const Tile& t) { return t.sym >= 0 || t.rounds; };
  p.adapt = is_adapt(prec) && !bat && n > 0 &&
            (symmetric(single_force_tile(cfg, NBODY_KERNEL_FORCE, prec, n)) ||
             symmetric(single_force_tile(cfg, NBODY_KERNEL_LJ_FORCE, prec, n)));
  if (p.adapt) {
    int64_t P = kBitonicLocal;
    while (P < n) P <<= 1;
    p.adapt_padded = P;
    p.adapt_bblocks = (int32_t)std::min<int64_t>(cdiv(n, kAdaptBS), 1024);
    p.off_keys = take((size_t)P * sizeof(uint64_t));
    p.off_perm = take((size_t)n * sizeof(uint32_t));
    p.off_box = take((size_t)cdiv(n, kSub) * 2 * sizeof(float4));
    p.off_bbpart = take((size_t)p.adapt_bblocks * 6 * sizeof(double));
    p.off_bbox = take(8 * sizeof(double));
  }
  // energy partials: chunks of kEnergyBS threads per system, about one particle per thread
  // (the energy can ride on a per-particle reduction, which needs that parallelism), with at
  // most max(16 S, 32768) chunks in all
  const int64_t chunk_cap = std::max<int64_t>(16, 32768 / std::max<int64_t>(1, sys.S));
  int64_t chunks = std::min<int64_t>(std::max<int64_t>(1, cdiv(sys.max_n, kEnergyBS)), chunk_cap);
  p.e_chunks = (int32_t)chunks;
  // a rollout with an energy trace keeps the partials of up to kEnergySteps steps (at most
  // kEnergyBytes) and sums them in one launch
  const size_t step_e = (size_t)sys.S * chunks * 5 * dsz;
  p.e_steps = (int32_t)std::max<size_t>(1, std::min<size_t>(kEnergySteps, kEnergyBytes / step_e));
  if (need & (NEED_ENERGY | NEED_ROLLOUT)) {
    // energy (5) or diagnostics (10) partials of one state, or a rollout's kept energy partials
    p.sz_epart = std::max((size_t)sys.S * chunks * kDiag * dsz, (size_t)p.e_steps * step_e);
    p.off_epart = take(p.sz_epart);
    p.sz_pot = (size_t)n * dsz;
    p.off_pot = take(p.sz_pot);
    p.sz_accs = (size_t)3 * n * dsz;
    p.off_accs = take(p.sz_accs);
  }
  if (need & NEED_BACKWARD) {
    p.sz_state = (size_t)3 * n * dsz;
    p.off_xw = take(p.sz_state);
    p.off_vw = take(p.sz_state);
    p.off_aw = take(p.sz_state);
    p.sz_seg = (size_t)(ckpt_every + 1) * 3 * n * dsz;
    p.off_seg = take(p.sz_seg);
  }
  p.total = off;
  return NBODY_OK;
}

int check_lj(const nbody_config* cfg, const nbody_lj_params* lj) {
  if (!lj) return fail(NBODY_ERR_INVALID_ARG, "lj is NULL");
  if (!(lj->sigma > 0.0) || !std::isfinite(lj->sigma))
    return fail(NBODY_ERR_INVALID_ARG, "sigma must be finite and > 0 (got %g)", lj->sigma);
  if (!std::isfinite(lj->epsilon)) return fail(NBODY_ERR_INVALID_ARG, "epsilon must be finite");
  if (!(lj->soft >= 0.0) || !std::isfinite(lj->soft))
    return fail(NBODY_ERR_INVALID_ARG, "soft must be finite and >= 0 (got %g)", lj->soft);
  if (cfg && cfg->precision != NBODY_FP64 && lj->soft > 0.0 && lj->soft / lj->sigma < 1e-10)
    return fail(NBODY_ERR_INVALID_ARG, "soft/sigma must be 0 or >= 1e-10 for the FP32 modes");
  if (lj->reserved != 0) return fail(NBODY_ERR_INVALID_ARG, "lj reserved must be 0");
  if (lj->walls != 0 && lj->walls != 1) return fail(NBODY_ERR_INVALID_ARG, "walls must be 0 or 1");
  if (lj->walls)
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(lj->lo[c]) || !std::isfinite(lj->hi[c]) || !(lj->lo[c] < lj->hi[c]))
        return fail(NBODY_ERR_INVALID_ARG, "box: need finite lo[%d] < hi[%d]", c, c);
  return NBODY_OK;
}

struct Ctx {
  const nbody_config* cfg;
  Systems sys;
  int64_t n;
  hipStream_t st;
  char* ws;
  Plan plan;
  UnitSet uf, ua;
  bool bat, loop;
  // pair law: LAW_GRAV, or LAW_LJ with coordinates staged in units of sigma
  int law = LAW_GRAV;
  double xs = 1.0;    // staging scale of the coordinates
  double eps2 = 0.0;  // softening^2 in staged units
  LawScale ls{};      // constants applied to the raw pair sums (mdiv set per call)
  Walls wl{};
  // adaptive mode on symmetric tiles: the force pass sorts and stages the positions itself,
  // from the state the last staging call named
  bool adapt = false;
  const double* src_pos = nullptr;
  const double* src_mass = nullptr;

  LawScale ls_at(int64_t b) const {
    LawScale r = ls;
    if (r.mdiv) r.mdiv += b;
    return r;
  }
};

// lj: the Lennard-Jones law (nullptr: gravity); law_free: a call that uses no pair law
// (its G and eps are not checked).
// One GPU's share of the ring decomposition: the one-sided tile "bs=256,i=1,tj=256" (variant 0)
// with P j-ranges of s particles each (S of them non-empty); the workspace holds the j-array and,
// for S > 1, one double partial-sum plane set per j-range.
int shard_plan(const nbody_config* cfg, int64_t n, int32_t P, Plan& p, Tile& t, int64_t& S, int64_t& s) {
  if (P < 1) return fail(NBODY_ERR_INVALID_ARG, "P must be >= 1 (got %d)", (int)P);
  t = Tile{};
  t.variant = 0;
  t.sym = -1;
  variant_shape(NBODY_KERNEL_FORCE, cfg->precision, 0, t.bs, t.i, t.tj);
  t.j_split = P;
  split_geometry(t, n, S, s);
  p = Plan{};
  size_t off = 0;
  p.off_jbuf = off;
  p.sz_jbuf = (size_t)n * jvec_bytes(cfg->precision);
  off += align_up(p.sz_jbuf);
  p.off_part = off;
  p.sz_part = S > 1 ? (size_t)S * 4 * (size_t)n * sizeof(double) : 0;
  off += align_up(p.sz_part);
  p.total = off;
  return NBODY_OK;
}

// shard_P > 0: the plan of one ring share of P (nbody_forces_shard), single systems only.
int prepare(Ctx& c, const nbody_config* cfg, int64_t n, int64_t ckpt_every, unsigned need,
            const nbody_lj_params* lj = nullptr, bool law_free = false, int32_t shard_P = 0) {
  TRY(check_cfg(cfg, n, c.sys, lj == nullptr && !law_free));
  if (lj) {
    TRY(check_lj(cfg, lj));
    c.law = LAW_LJ;
    c.xs = 1.0 / lj->sigma;
    c.eps2 = (lj->soft / lj->sigma) * (lj->soft / lj->sigma);
    c.ls.ca = 24.0 * lj->epsilon / lj->sigma;
    c.ls.cp = 4.0 * lj->epsilon;
    c.wl.on = lj->walls;
    for (int k = 0; k < 3; ++k) {
      c.wl.lo[k] = lj->lo[k];
      c.wl.hi[k] = lj->hi[k];
    }
  } else {
    c.law = LAW_GRAV;
    c.xs = 1.0;
    c.eps2 = cfg->eps * cfg->eps;
    c.ls.ca = c.ls.cp = cfg->G;
    c.ls.mdiv = nullptr;
    c.wl.on = 0;
  }
  c.cfg = cfg;
  c.n = n;
  c.st = (hipStream_t)cfg->stream;
  c.bat = c.sys.S > 1;
  c.loop = c.bat && (cfg->flags & NBODY_FLAG_LOOP_SYSTEMS);
  if (shard_P > 0) {
    if (c.sys.S != 1) return fail(NBODY_ERR_UNSUPPORTED, "a ring share is of a single system (n_systems == 1)");
    Tile t;
    int64_t S, s;
    TRY(shard_plan(cfg, n, shard_P, c.plan, t, S, s));
    c.adapt = false;
  } else {
    TRY(make_plan(cfg, c.sys, n, ckpt_every, need, c.plan, &c.uf, &c.ua, c.law));
    const Tile t = single_force_tile(cfg, force_kernel_id(c.law, false), cfg->precision, n);
    c.adapt = c.plan.adapt && (t.sym >= 0 || t.rounds);
  }
  if (n == 0) return NBODY_OK;
  if (!cfg->workspace) return fail(NBODY_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", c.plan.total);
  if (((uintptr_t)cfg->workspace) % kAlign)
    return fail(NBODY_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
  if (cfg->workspace_bytes < c.plan.total)
    return fail(NBODY_ERR_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", cfg->workspace_bytes,
                c.plan.total);
  c.ws = (char*)cfg->workspace;
  return NBODY_OK;
}

// Host staging for the batched metadata (system offsets, split counts, work units): a ring of
// pinned host buffers, each reused once the upload that last read it has completed (its event).
// Calls on other streams (or devices) take other buffers, so they do not wait for each other;
// a call waits only when every buffer of its device still feeds an upload in flight (then for the
// oldest). The buffers are held until the process ends.
constexpr int kStageSlots = 8;
struct StageSlot {
  void* buf = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;  // recorded after the slot's last upload
  int device = -1;
  uint64_t last_use = 0;
  bool in_use = false;  // a call is filling it (between acquire_stage and release_stage)
};
std::mutex g_stage_mu;
StageSlot g_stage[kStageSlots];
uint64_t g_stage_clock = 0;

void release_stage(StageSlot* sl);

// A slot of the current device whose last upload has completed, at least `total` bytes; the
// caller owns it until release_stage.
int acquire_stage(size_t total, StageSlot*& out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  StageSlot* pick = nullptr;
  bool wait = false;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    StageSlot* oldest = nullptr;
    for (auto& sl : g_stage) {
      if (sl.in_use || (sl.device != -1 && sl.device != dev)) continue;
      if (sl.device == -1 || hipEventQuery(sl.done) == hipSuccess) {
        pick = &sl;
        break;
      }
      if (!oldest || sl.last_use < oldest->last_use) oldest = &sl;
    }
    if (!pick && !oldest)
      return fail(NBODY_ERR_UNSUPPORTED, "host staging: all %d buffers busy or bound to other devices", kStageSlots);
    if (!pick) {  // every free slot of this device still feeds an upload: wait for the oldest
      pick = oldest;
      wait = true;
    }
    pick->last_use = ++g_stage_clock;
    pick->in_use = true;
  }
  hipError_t e = hipSuccess;
  if (wait) e = hipEventSynchronize(pick->done);
  if (e == hipSuccess && pick->device == -1) {
    e = hipEventCreateWithFlags(&pick->done, hipEventDisableTiming);
    if (e == hipSuccess) pick->device = dev;
  }
  if (e == hipSuccess && total > pick->bytes) {
    if (pick->buf) e = hipHostFree(pick->buf);
    pick->buf = nullptr;
    pick->bytes = 0;
    if (e == hipSuccess) e = hipHostMalloc(&pick->buf, total, hipHostMallocDefault);
    if (e == hipSuccess) pick->bytes = total;
  }
  if (e != hipSuccess) {
    release_stage(pick);
    return fail(NBODY_ERR_DEVICE, "host staging: %s", hipGetErrorString(e));
  }
  out = pick;
  return NBODY_OK;
}

void release_stage(StageSlot* sl) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  sl->in_use = false;
}

int upload_meta(Ctx& c) {
  if (!c.bat || c.loop) return NBODY_OK;
  const int64_t S = c.sys.S;
  const size_t b_off = (S + 1) * sizeof(int64_t);
  const size_t b_ns = 2 * S * sizeof(int32_t);
  const size_t b_poff = c.uf.sym ? (S + 1) * sizeof(int64_t) : 0;
  const size_t b_units = c.uf.unit_bytes();
  const size_t b_uadj = c.ua.unit_bytes();
  const size_t b_poffa = c.ua.sym ? (S + 1) * sizeof(int64_t) : 0;
  const size_t b_rt = c.uf.sym ? c.uf.rtasks.size() * sizeof(int32_t) : 0;
  const size_t b_ro = c.uf.sym ? c.uf.ro_units.size() * sizeof(SymUnit) : 0;
  const size_t total = align_up(b_off) + align_up(b_ns) + align_up(b_poff) + align_up(b_units) + align_up(b_uadj) +
                       align_up(b_poffa) + align_up(b_rt) + align_up(b_ro);
  StageSlot* slot = nullptr;
  TRY(acquire_stage(total, slot));
  struct Release {
    StageSlot* s;
    ~Release() { release_stage(s); }
  } release{slot};
  char* h = (char*)slot->buf;
  int64_t* h_off = (int64_t*)h;
  int32_t* h_ns = (int32_t*)(h + align_up(b_off));
  int64_t* h_poff = (int64_t*)(h + align_up(b_off) + align_up(b_ns));
  char* h_units = h + align_up(b_off) + align_up(b_ns) + align_up(b_poff);
  char* h_uadj = h_units + align_up(b_units);
  char* h_poffa = h_uadj + align_up(b_uadj);
  char* h_rt = h_poffa + align_up(b_poffa);
  char* h_ro = h_rt + align_up(b_rt);
  std::memcpy(h_off, c.sys.off, b_off);
  for (int64_t s = 0; s < S; ++s) {
    h_ns[s] = c.uf.nsplit.empty() ? 0 : c.uf.nsplit[s];
    h_ns[S + s] = c.ua.nsplit.empty() ? 0 : c.ua.nsplit[s];
  }
  if (b_poff) std::memcpy(h_poff, c.uf.part_off.data(), b_poff);
  if (b_units) std::memcpy(h_units, c.uf.sym ? (const void*)c.uf.sym_units.data() : (const void*)c.uf.units.data(),
                           b_units);
  if (b_uadj) std::memcpy(h_uadj, c.ua.sym ? (const void*)c.ua.sym_units.data() : (const void*)c.ua.units.data(),
                          b_uadj);
  if (b_poffa) std::memcpy(h_poffa, c.ua.part_off.data(), b_poffa);
  if (b_rt) std::memcpy(h_rt, c.uf.rtasks.data(), b_rt);
  if (b_ro) std::memcpy(h_ro, c.uf.ro_units.data(), b_ro);
  HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_sysoff, h_off, b_off, hipMemcpyHostToDevice, c.st));
  HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_nsplit, h_ns, b_ns, hipMemcpyHostToDevice, c.st));
  if (b_poff) HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_partoff, h_poff, b_poff, hipMemcpyHostToDevice, c.st));
  if (b_units) HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_units, h_units, b_units, hipMemcpyHostToDevice, c.st));
  if (b_uadj) HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_units_adj, h_uadj, b_uadj, hipMemcpyHostToDevice, c.st));
  if (b_poffa)
    HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_partoff_adj, h_poffa, b_poffa, hipMemcpyHostToDevice, c.st));
  if (b_rt) HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_rtasks, h_rt, b_rt, hipMemcpyHostToDevice, c.st));
  if (b_ro) HIP_TRY(hipMemcpyAsync(c.ws + c.plan.off_units_ro, h_ro, b_ro, hipMemcpyHostToDevice, c.st));
  HIP_TRY(hipEventRecord(slot->done, c.st));
  return NBODY_OK;
}

// Host-side guard: a pass about to write `planes` partial planes of n doubles must
// find them inside the planned partial-sum region.
int check_part(const Ctx& c, size_t bytes, const char* what) {
  if (bytes > c.plan.sz_part)
    return fail(NBODY_ERR_DEVICE, "internal: %s needs %zu bytes of partial sums, plan has %zu", what, bytes,
                c.plan.sz_part);
  return NBODY_OK;
}

int check_jbuf(const Ctx& c, size_t bytes_per_particle, const char* what) {
  if (c.plan.sz_jbuf < (size_t)c.n * bytes_per_particle)
    return fail(NBODY_ERR_DEVICE, "internal: %s j-array larger than the planned region", what);
  return NBODY_OK;
}

inline dim3 grid1d(int64_t n, int bs = 256) { return dim3((unsigned)cdiv(std::max<int64_t>(n, 1), bs)); }

// ------------------------------------------------------------------ passes

int stage(Ctx& c, const double* pos, const double* mass) {
  c.src_pos = pos;
  c.src_mass = mass;
  if (c.adapt) return NBODY_OK;  // sorted and staged by the force pass
  TRY(check_jbuf(c, jvec_bytes(c.cfg->precision), "stage_j"));
  void* j = c.ws + c.plan.off_jbuf;
  if (is_fp64(c.cfg->precision))
    hipLaunchKernelGGL((stage_j<double, false>), grid1d(c.n), dim3(256), 0, c.st, c.n, pos, mass, c.xs, (D4*)j);
  else if (is_ds(c.cfg->precision))
    hipLaunchKernelGGL((stage_j<float, true>), grid1d(c.n), dim3(256), 0, c.st, c.n, pos, mass, c.xs, (float4*)j);
  else
    hipLaunchKernelGGL((stage_j<float, false>), grid1d(c.n), dim3(256), 0, c.st, c.n, pos, mass, c.xs, (float4*)j);
  LAUNCH_CHECK("stage_j");
  return NBODY_OK;
}

int kick_drift(Ctx& c, double dt, double* pos, double* vel, const double* acc, const double* mass) {
  TRY(check_jbuf(c, jvec_bytes(c.cfg->precision), "kick_drift_stage"));
  c.src_pos = pos;
  c.src_mass = mass;
  void* j = c.adapt ? nullptr : c.ws + c.plan.off_jbuf;  // adaptive: staged in sorted order by the force pass
  if (is_fp64(c.cfg->precision))
    hipLaunchKernelGGL((kick_drift_stage<double, false>), grid1d(c.n), dim3(256), 0, c.st, c.n, 0.5 * dt, dt, pos, vel,
                       acc, mass, c.xs, c.wl, (D4*)j);
  else if (is_ds(c.cfg->precision))
    hipLaunchKernelGGL((kick_drift_stage<float, true>), grid1d(c.n), dim3(256), 0, c.st, c.n, 0.5 * dt, dt, pos, vel,
                       acc, mass, c.xs, c.wl, (float4*)j);
  else
    hipLaunchKernelGGL((kick_drift_stage<float, false>), grid1d(c.n), dim3(256), 0, c.st, c.n, 0.5 * dt, dt, pos, vel,
                       acc, mass, c.xs, c.wl, (float4*)j);
  LAUNCH_CHECK("kick_drift_stage");
  return NBODY_OK;
}

int persistent_grid(const void* kfn, int bs, int64_t units, unsigned& grid) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, bs, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t g = std::min<int64_t>(units, (int64_t)num_cu() * per_cu);
  grid = (unsigned)std::max<int64_t>(g, 1);
  return NBODY_OK;
}

// The first half of the next KDK step (dt), to be fused into this force pass's reduction.
NextStep next_step(const Ctx& c, double dt, double* pos, const double* mass) {
  NextStep nx{};
  const int prec = c.cfg->precision;
  nx.kind = is_fp64(prec) ? 2 : c.adapt ? 4 : is_ds(prec) ? 3 : 1;
  nx.pos = pos;
  nx.mass = mass;
  nx.hh = 0.5 * dt;
  nx.h = dt;
  nx.xs = c.xs;
  nx.wl = c.wl;
  nx.jarr = c.ws + c.plan.off_jbuf;
  return nx;
}

// The same, for the particles of a system starting at global index b (offset pointers).
NextStep next_step_at(const Ctx& c, const NextStep* nx, int64_t b) {
  NextStep r{};
  if (!nx) return r;  // kind 0: nothing fused
  r = *nx;
  r.pos += b;
  r.mass += b;
  if (r.pos_copy) r.pos_copy += b;
  r.jarr = (char*)r.jarr + (size_t)b * jvec_bytes(c.cfg->precision);
  return r;
}

// Optional work fused into a force pass's per-particle reduction.
struct Fuse {
  const NextStep* nx = nullptr;  // the next step's kick, drift, walls and staging
  double* eout = nullptr;        // energy and momentum of the new state, [S][5] (needs pot and vel)
  const double* mass = nullptr;  // masses, with eout
  int32_t eslot = -1;            // >= 0: leave the energy partials in kept slot eslot; the caller
                                 // sums them later (flush_energy) instead of this pass
  bool done = false;             // set by force_pass: the pass had such a reduction and did all of it
};

// The energy rows of `count` consecutive states from the partials kept in slots 0 .. count-1:
// out[t][S][5], one launch.
int flush_energy(Ctx& c, int32_t count, double* out) {
  if (count <= 0) return NBODY_OK;
  const int32_t chunks = c.plan.e_chunks;
  hipLaunchKernelGGL(energy_final<256>, dim3((unsigned)c.sys.S, (unsigned)count), dim3(256), 0, c.st, chunks,
                     (const double*)(c.ws + c.plan.off_epart), out, (int64_t)c.sys.S * chunks * 5,
                     (int64_t)c.sys.S * 5);
  LAUNCH_CHECK("energy_final");
  return NBODY_OK;
}

// The adaptive mode's symmetric pass over the single system (n particles) at the positions the
// last staging call named: bounding box and threshold, Morton keys, bitonic sort, sorted
// staging with sub-block boxes, the tile kernel, and the per-particle reduction in sorted
// order that writes every output at the particle's own index.
// The tiles of the round schedule over a system of ns particles whose j-array is jb: zero the K
// accumulator copies (K out), the diagonal tiles, then nbr - 1 rounds of disjoint block pairs
// (K / 2 per launch on two alternating streams). The caller adds the copies per particle.
// mode: force_mode's, or 3 for the adaptive mode (sorted particles, ad).
int round_tiles(Ctx& c, int64_t ns, const float4* jb, int law, int pot_on, int mode, const AdaptIn& ad, int& K) {
  const int64_t nb = cdiv(ns, (int64_t)kRoundBlock), nbr = nb + (nb & 1);
  if (nbr > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many blocks for the round schedule");
  K = round_copies(ns, g_sym_cap);
  TRY(check_part(c, (size_t)K * 4 * ns * sizeof(double), "force_sym_round_kernel"));
  double* a64 = (double*)(c.ws + c.plan.off_part);
  hipLaunchKernelGGL(fill_f64, grid1d(K * 4 * ns), dim3(256), 0, c.st, a64, K * 4 * ns, 0.0);
  LAUNCH_CHECK("fill_f64");
  kRoundDiag[law][pot_on][mode](dim3((unsigned)nb), c.st, jb, ns, (float)c.eps2, a64, ad);
  LAUNCH_CHECK("force_sym_round_diag_kernel");
  const RoundFn fn = kRound[law][pot_on][mode];
  const float eps2 = (float)c.eps2;
  return run_rounds(c.st, ns, nbr, a64, K, "force_sym_round_kernel",
                    [&](dim3 g, hipStream_t s, int32_t r0, double* acc) {
                      fn(g, s, jb, ns, (int32_t)nb, (int32_t)nbr, r0, eps2, acc, ad);
                    });
}

template <typename Tail>
int adapt_sym_pass(Ctx& c, const Tile& t, double* acc, double* pot, double* vel, double hh, const NextStep* nx,
                   Tail&& tail) {
  const int64_t n = c.n;
  if (!c.src_pos || !c.src_mass) return fail(NBODY_ERR_DEVICE, "internal: adaptive pass without staged positions");
  if (n > 0xffffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "the adaptive mode sorts at most 2^32 particles");
  // slot schedule: off-diagonal tiles (the diagonal ones launch apart)
  const int64_t nb = t.rounds ? 0 : cdiv(n, (int64_t)t.tj);
  const int64_t off_tiles = nb * (nb - 1) / 2;
  if (off_tiles > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many symmetric tiles");
  if (!t.rounds) TRY(check_part(c, (size_t)nb * 4 * n * sizeof(float), "force_sym_kernel (adaptive)"));
  TRY(check_jbuf(c, 2 * sizeof(float4), "adapt_stage"));
  const Plan& pl = c.plan;
  if (!pl.adapt) return fail(NBODY_ERR_DEVICE, "internal: adaptive pass without its workspace");
  uint64_t* keys = (uint64_t*)(c.ws + pl.off_keys);
  uint32_t* perm = (uint32_t*)(c.ws + pl.off_perm);
  float4* box = (float4*)(c.ws + pl.off_box);
  double* bbox = (double*)(c.ws + pl.off_bbox);
  float4* jhi = (float4*)(c.ws + pl.off_jbuf);
  float4* jlo = jhi + n;
  const int64_t P = pl.adapt_padded;
  hipLaunchKernelGGL(adapt_bbox_partial, dim3((unsigned)pl.adapt_bblocks), dim3(kAdaptBS), 0, c.st, n, c.src_pos,
                     (double*)(c.ws + pl.off_bbpart));
  LAUNCH_CHECK("adapt_bbox_partial");
  hipLaunchKernelGGL(adapt_bbox_final, dim3(1), dim3(kAdaptBS), 0, c.st, pl.adapt_bblocks,
                     (const double*)(c.ws + pl.off_bbpart), c.xs, bbox);
  LAUNCH_CHECK("adapt_bbox_final");
  hipLaunchKernelGGL(adapt_keys, grid1d(P, kAdaptBS), dim3(kAdaptBS), 0, c.st, n, P, c.src_pos, (const double*)bbox,
                     keys);
  LAUNCH_CHECK("adapt_keys");
  const unsigned lblocks = (unsigned)(P / kBitonicLocal);
  hipLaunchKernelGGL(bitonic_local, dim3(lblocks), dim3(kBitonicBS), 0, c.st, keys);
  LAUNCH_CHECK("bitonic_local");
  for (int64_t k = 2 * (int64_t)kBitonicLocal; k <= P; k <<= 1) {
    for (int64_t j = k >> 1; j >= kBitonicLocal; j >>= 1) {
      hipLaunchKernelGGL(bitonic_global, grid1d(P / 2, kAdaptBS), dim3(kAdaptBS), 0, c.st, keys, P, k, j);
      LAUNCH_CHECK("bitonic_global");
    }
    hipLaunchKernelGGL(bitonic_merge_local, dim3(lblocks), dim3(kBitonicBS), 0, c.st, keys, k);
    LAUNCH_CHECK("bitonic_merge_local");
  }
  hipLaunchKernelGGL(adapt_stage, grid1d(cdiv(n, kSub) * kSub, kAdaptBS), dim3(kAdaptBS), 0, c.st, n,
                     (const uint64_t*)keys, c.src_pos, c.src_mass, c.xs, perm, jhi, jlo, box);
  LAUNCH_CHECK("adapt_stage");
  AdaptIn ad;
  ad.jlo = jlo;
  ad.box = box;
  ad.thr = bbox + 6;
  if (t.rounds) {
    int K = 1;
    TRY(round_tiles(c, n, jhi, c.law, pot != nullptr, 3, ad, K));
    hipLaunchKernelGGL(reduce_rounds, grid1d(n), dim3(kReduceBS), 0, c.st, n, n,
                       (const double*)(c.ws + pl.off_part), (int32_t)K, c.ls, acc, pot, vel, hh,
                       nx ? *nx : NextStep{}, EnergyFuse{}, (const uint32_t*)perm);
    LAUNCH_CHECK("reduce_rounds");
    return tail();
  }
  const SymVariant& sv = kSym32[t.sym];
  float* pf = (float*)(c.ws + pl.off_part);
  sv.dfn[c.law][pot != nullptr](dim3((unsigned)nb), c.st, jhi, n, (int32_t)nb, (float)c.eps2, pf, ad);
  LAUNCH_CHECK("force_sym_kernel (adaptive, diagonal tiles)");
  if (off_tiles > 0) {
    sv.afn[c.law][pot != nullptr](dim3((unsigned)off_tiles), c.st, jhi, n, (int32_t)nb, (float)c.eps2, pf, ad);
    LAUNCH_CHECK("force_sym_kernel (adaptive)");
  }
  hipLaunchKernelGGL(reduce_sym, grid1d(n, 64), dim3(kReduceBS), 0, c.st, n, n, (int32_t)nb, (const float*)pf, c.ls, acc,
                     pot, vel, hh, nx ? *nx : NextStep{}, EnergyFuse{}, (const uint32_t*)perm);
  LAUNCH_CHECK("reduce_sym");
  return tail();
}

// Force pass on the staged j-array: acc = a, pot (nullable), vel += hh*acc when vel != NULL.
// fz (nullable): work to fuse into the pass's per-particle reduction. A pass without one (a
// one-sided pass that writes accelerations directly) or the per-system loop fuses nothing and
// leaves fz->done false; the caller then runs energy_pass and kick_drift itself.
int force_pass(Ctx& c, double* acc, double* pot, double* vel, double hh, Fuse* fz = nullptr) {
  const NextStep* nx = nullptr;
  EnergyFuse ef{};
  if (fz) {
    fz->done = false;
    if (c.loop || !vel || (fz->eout && (!pot || !fz->mass))) fz = nullptr;  // all systems or none; the
                                                                          // kick needs the velocities
    // the adaptive mode's reduction runs in sorted order, so its energy sums would not be those
    // of the separate energy pass: a traced step reduces its energy separately
    if (fz && c.adapt && fz->eout) fz = nullptr;
  }
  if (fz) {
    nx = fz->nx;
    if (fz->eout) {
      ef.part = (double*)(c.ws + c.plan.off_epart) + (fz->eslot > 0 ? (size_t)fz->eslot * c.sys.S * c.plan.e_chunks * 5 : 0);
      ef.mass = fz->mass;
      ef.chunks = c.plan.e_chunks;
    }
  }
  // the reduction's launch geometry: one thread per particle in one-wave workgroups (a small
  // system's reduction then spreads over n / 64 CUs; each thread's sum is a chain of dependent
  // loads, so the latency, not the bandwidth, sets its time), or the energy chunk grid
  auto rgrid = [&](int64_t count) {
    return ef.part ? dim3((unsigned)ef.chunks, (unsigned)c.sys.S) : grid1d(count, kEnergyBS);
  };
  const dim3 rblock(kEnergyBS);
  // after a reduction that carried the fused work, finish the energy sum
  auto fused_tail = [&]() -> int {
    if (!fz) return NBODY_OK;
    if (ef.part && fz->eslot < 0) {
      hipLaunchKernelGGL(energy_final<256>, dim3((unsigned)c.sys.S), dim3(256), 0, c.st, ef.chunks,
                         (const double*)ef.part, fz->eout, (int64_t)0, (int64_t)0);
      LAUNCH_CHECK("energy_final");
    }
    fz->done = true;
    return NBODY_OK;
  };
  const int prec = c.cfg->precision;
  const int mode = force_mode(prec);
  const int pot_on = pot != nullptr;
  const int law = c.law;
  const double eps2 = c.eps2;
  const void* jarr = c.ws + c.plan.off_jbuf;
  double* part = (double*)(c.ws + c.plan.off_part);
  const int64_t n = c.n;

  auto single = [&](int64_t b, int64_t e) -> int {
    const int64_t ns = e - b;
    if (ns == 0) return NBODY_OK;
    Tile t = single_force_tile(c.cfg, force_kernel_id(law, false), prec, ns);
    if ((t.sym >= 0 || t.rounds) && c.adapt) return adapt_sym_pass(c, t, acc, pot, vel, hh, nx, fused_tail);
    if (t.rounds) {
      // round schedule, then the per-particle end (copies added, scale, kick, next step, energy)
      int K = 1;
      TRY(round_tiles(c, ns, (const float4*)jarr + (is_ds(prec) ? 2 : 1) * b, law, pot_on, mode, AdaptIn{}, K));
      hipLaunchKernelGGL(reduce_rounds, rgrid(ns), rblock, 0, c.st, ns, n,
                         (const double*)(c.ws + c.plan.off_part), (int32_t)K, c.ls_at(b), acc + b,
                         pot ? pot + b : nullptr, vel ? vel + b : nullptr, hh, next_step_at(c, nx, b), ef,
                         (const uint32_t*)nullptr);
      LAUNCH_CHECK("reduce_rounds");
      return fused_tail();
    }
    if (t.sym >= 0) {
      const SymVariant& sv = kSym32[t.sym];
      const int64_t nb = cdiv(ns, (int64_t)t.tj);
      const int64_t tiles = nb * (nb + 1) / 2;
      if (tiles > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many symmetric tiles");
      TRY(check_part(c, (size_t)nb * 4 * ns * sizeof(float), "force_sym_kernel"));
      float* pf = (float*)(c.ws + c.plan.off_part);
      sv.fn[law][pot_on][mode](dim3((unsigned)tiles), c.st, (const float4*)jarr + (is_ds(prec) ? 2 : 1) * b, ns,
                               (int32_t)nb, (float)eps2, pf);
      LAUNCH_CHECK("force_sym_kernel");
      // reduce_sym: the energy's chunk grid, else blocks of four waves for 64 particles
      hipLaunchKernelGGL(reduce_sym, ef.part ? rgrid(ns) : grid1d(ns, 64), dim3(kReduceBS), 0, c.st, ns,
                         n, (int32_t)nb, (const float*)pf,
                         c.ls_at(b), acc + b, pot ? pot + b : nullptr, vel ? vel + b : nullptr, hh,
                         next_step_at(c, nx, b), ef, (const uint32_t*)nullptr);
      LAUNCH_CHECK("reduce_sym");
      return fused_tail();
    }
    int64_t S, jc;
    split_geometry(t, ns, S, jc);
    const ForceVariant& fv = is_fp64(prec) ? kForce64[t.variant] : kForce32[t.variant];
    ForceOut o{};
    o.ls = c.ls;  // direct stores index particles globally (i in [b, e))
    o.n_plane = n;
    dim3 g((unsigned)cdiv(ns, (int64_t)t.bs * t.i), (unsigned)S);
    if (S == 1) {
      o.acc = acc; o.pot = pot; o.vel = vel; o.hh = hh;
    } else {
      TRY(check_part(c, (size_t)S * 4 * n * sizeof(double), "force_kernel"));
      o.part = part;
    }
    fv.fn[law][pot_on][mode](g, c.st, jarr, b, e, b, e, jc, eps2, o);
    LAUNCH_CHECK("force_kernel");
    if (S > 1) {
      // reduce only this system's particle range: offset pointers into the planes
      hipLaunchKernelGGL(reduce_splits, rgrid(ns), rblock, 0, c.st, ns, n, (int32_t)S, part + b,
                         c.ls_at(b), acc + b, pot ? pot + b : nullptr, vel ? vel + b : nullptr, hh, (int64_t)0,
                         (const int64_t*)nullptr, (const int32_t*)nullptr, next_step_at(c, nx, b), ef);
      LAUNCH_CHECK("reduce_splits");
      return fused_tail();
    }
    return NBODY_OK;
  };

  if (!c.bat) return single(0, n);
  if (c.loop) {
    for (int64_t s = 0; s < c.sys.S; ++s) TRY(single(c.sys.off[s], c.sys.off[s + 1]));
    return NBODY_OK;
  }
  // batched: one launch, one workgroup per work unit (units sorted by decreasing cost)
  Tile t = lookup_tile(force_kernel_id(law, true), prec, c.sys.max_n);
  const dim3 ugrid((unsigned)std::max<int64_t>(1, c.plan.n_units_force));
  if (t.sym >= 0) {
    // symmetric tiles of every system; the unit list was built from the same tile
    if (!c.uf.sym) return fail(NBODY_ERR_DEVICE, "internal: symmetric batched tile without symmetric units");
    TRY(check_part(c, (size_t)c.uf.part_floats * sizeof(float), "force_sym_batched_kernel"));
    const SymVariant& sv = kSym32[t.sym];
    float* pf = (float*)(c.ws + c.plan.off_part);
    sv.bfn[law][pot_on][mode](ugrid, c.st, (const float4*)jarr, (const SymUnit*)(c.ws + c.plan.off_units),
                              (int32_t)c.plan.n_units_force, (float)eps2, pf);
    LAUNCH_CHECK("force_sym_batched_kernel");
    hipLaunchKernelGGL(reduce_sym_batched, rgrid(n), rblock, 0, c.st, n, c.sys.S,
                       (const int64_t*)(c.ws + c.plan.off_sysoff), (const int32_t*)(c.ws + c.plan.off_nsplit),
                       (const int64_t*)(c.ws + c.plan.off_partoff), (const float*)pf, c.ls, acc, pot, vel, hh,
                       next_step_at(c, nx, 0), ef);
    LAUNCH_CHECK("reduce_sym_batched");
    return fused_tail();
  }
  if (c.uf.sym) return fail(NBODY_ERR_DEVICE, "internal: one-sided batched tile with symmetric units");
  const ForceVariant& fv = is_fp64(prec) ? kForce64[t.variant] : kForce32[t.variant];
  TRY(check_part(c, (size_t)max_nsplit(c.uf) * 4 * n * sizeof(double), "force_batched_kernel"));
  ForceOut o{};
  o.ls = c.ls;
  o.n_plane = n;
  o.part = part;
  fv.bfn[law][pot_on][mode](ugrid, c.st, jarr, (const WorkUnit*)(c.ws + c.plan.off_units),
                            (int32_t)c.plan.n_units_force, eps2, o);
  LAUNCH_CHECK("force_batched_kernel");
  hipLaunchKernelGGL(reduce_splits, rgrid(n), rblock, 0, c.st, n, n, (int32_t)0, part, c.ls, acc, pot, vel,
                     hh, c.sys.S, (const int64_t*)(c.ws + c.plan.off_sysoff),
                     (const int32_t*)(c.ws + c.plan.off_nsplit), next_step_at(c, nx, 0), ef);
  LAUNCH_CHECK("reduce_splits");
  return fused_tail();
}

int energy_pass(Ctx& c, const double* vel, const double* mass, const double* pot, double* out) {
  const int32_t chunks = c.plan.e_chunks;
  double* ep = (double*)(c.ws + c.plan.off_epart);
  const int64_t* dev_off = c.bat ? (const int64_t*)(c.ws + c.plan.off_sysoff) : nullptr;
  if (c.bat && c.loop) {
    // the looped baseline has no device offsets: reduce system by system
    for (int64_t s = 0; s < c.sys.S; ++s) {
      const int64_t b = c.sys.off[s], ns = c.sys.off[s + 1] - b;
      // offset pointers; vel planes keep stride n, so pass a shifted view per plane
      hipLaunchKernelGGL(energy_partial<kEnergyBS>, dim3(chunks, 1), dim3(kEnergyBS), 0, c.st, c.n, vel + b, mass + b,
                         pot + b,
                         (const int64_t*)nullptr, ns, chunks, ep + s * chunks * 5);
      LAUNCH_CHECK("energy_partial");
    }
  } else {
    hipLaunchKernelGGL(energy_partial<kEnergyBS>, dim3(chunks, (unsigned)c.sys.S), dim3(kEnergyBS), 0, c.st, c.n, vel,
                       mass, pot,
                       dev_off, c.n, chunks, ep);
    LAUNCH_CHECK("energy_partial");
  }
  hipLaunchKernelGGL(energy_final<256>, dim3((unsigned)c.sys.S), dim3(256), 0, c.st, chunks, ep, out, (int64_t)0,
                     (int64_t)0);
  LAUNCH_CHECK("energy_final");
  return NBODY_OK;
}

int diag_pass(Ctx& c, const double* pos, const double* vel, const double* mass, const double* pot,
              const double* acc, double* out) {
  const int32_t chunks = c.plan.e_chunks;
  double* ep = (double*)(c.ws + c.plan.off_epart);
  const int64_t* dev_off = c.bat ? (const int64_t*)(c.ws + c.plan.off_sysoff) : nullptr;
  if (c.bat && c.loop) {
    for (int64_t s = 0; s < c.sys.S; ++s) {
      const int64_t b = c.sys.off[s], ns = c.sys.off[s + 1] - b;
      hipLaunchKernelGGL(diag_partial<256>, dim3(chunks, 1), dim3(256), 0, c.st, c.n, pos + b, vel + b, mass + b,
                         pot + b, acc + b, (const int64_t*)nullptr, ns, chunks, ep + s * chunks * kDiag);
      LAUNCH_CHECK("diag_partial");
    }
  } else {
    hipLaunchKernelGGL(diag_partial<256>, dim3(chunks, (unsigned)c.sys.S), dim3(256), 0, c.st, c.n, pos, vel, mass, pot,
                       acc, dev_off, c.n, chunks, ep);
    LAUNCH_CHECK("diag_partial");
  }
  hipLaunchKernelGGL(diag_final<256>, dim3((unsigned)c.sys.S), dim3(256), 0, c.st, chunks, ep, out);
  LAUNCH_CHECK("diag_final");
  return NBODY_OK;
}

// Adjoint pass at positions pos with l = w * gvel (after gvel += h_drift * gpos):
// gpos += G(...), gmass += -G M.
// The next adjoint pass's staging arguments, for a pass that can fuse them into its reduction.
struct AdjNextArgs {
  const double* pos;
  double h_drift, w;
};

// One adjoint pass at positions pos. staged: the j-array already holds this pass's staging (a
// previous pass fused it). next (nullable): the next pass's staging to fuse into this pass's
// reduction where it has one (a single system on symmetric tiles); *fused (nullable) says
// whether it did.
int adjoint_pass(Ctx& c, const double* pos, const double* mass, double* gvel, const double* gpos_in,
                 double h_drift, double w, double* gpos, double* gmass, const AdjNextArgs* next = nullptr,
                 bool staged = false, bool* fused = nullptr) {
  const int prec = c.cfg->precision;
  const int comp = adj_comp(prec);  // the double-float mode's adjoint runs compensated
  const double eps2 = c.cfg->eps * c.cfg->eps;
  TRY(check_jbuf(c, jadj_bytes(c.cfg->precision), "adjoint_stage"));
  void* jadj = c.ws + c.plan.off_jbuf;
  double* part = (double*)(c.ws + c.plan.off_part);
  const int64_t n = c.n;
  if (fused) *fused = false;
  if (!staged) {
    if (is_fp64(prec))
      hipLaunchKernelGGL(adjoint_stage<double>, grid1d(n), dim3(256), 0, c.st, n, pos, mass, gvel, gpos_in, h_drift,
                         w, (D4*)jadj);
    else
      hipLaunchKernelGGL(adjoint_stage<float>, grid1d(n), dim3(256), 0, c.st, n, pos, mass, gvel, gpos_in, h_drift,
                         w, (float4*)jadj);
    LAUNCH_CHECK("adjoint_stage");
  }

  auto single = [&](int64_t b, int64_t e) -> int {
    const int64_t ns = e - b;
    if (ns == 0) return NBODY_OK;
    Tile t = single_adj_tile(c.cfg, prec, ns);
    if (t.rounds) {
      // round schedule: zero the K accumulator copies, the diagonal tiles, the rounds, then the
      // per-particle update of the gradients
      const int64_t nb = cdiv(ns, (int64_t)kRoundBlock), nbr = nb + (nb & 1);
      if (nbr > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many blocks for the round schedule");
      const int K = round_copies(ns, g_sym_cap);
      TRY(check_part(c, (size_t)K * 4 * ns * sizeof(double), "adjoint_sym_round_kernel"));
      double* a64 = (double*)(c.ws + c.plan.off_part);
      hipLaunchKernelGGL(fill_f64, grid1d(K * 4 * ns), dim3(256), 0, c.st, a64, K * 4 * ns, 0.0);
      LAUNCH_CHECK("fill_f64");
      const float4* ja = (const float4*)jadj + 2 * b;
      const float e2 = (float)eps2;
      kAdjRoundDiag[comp](dim3((unsigned)nb), c.st, ja, ns, e2, a64);
      LAUNCH_CHECK("adjoint_sym_round_diag_kernel");
      const AdjRoundFn fn = kAdjRound[comp];
      TRY(run_rounds(c.st, ns, nbr, a64, K, "adjoint_sym_round_kernel",
                     [&](dim3 g, hipStream_t s, int32_t r0, double* acc) {
                       fn(g, s, ja, ns, (int32_t)nb, (int32_t)nbr, r0, e2, acc);
                     }));
      hipLaunchKernelGGL(adjoint_reduce_rounds, grid1d(ns), dim3(256), 0, c.st, ns, n, (int32_t)K,
                         (const double*)a64, c.cfg->G, gpos + b, gmass + b);
      LAUNCH_CHECK("adjoint_reduce_rounds");
      return NBODY_OK;
    }
    if (t.sym >= 0) {
      const AdjSymVariant& sv = kAdjSym32[t.sym];
      const int64_t nb = cdiv(ns, (int64_t)t.tj);
      const int64_t tiles = nb * (nb + 1) / 2;
      if (tiles > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many symmetric tiles");
      TRY(check_part(c, (size_t)nb * 4 * ns * sizeof(float), "adjoint_sym_kernel"));
      float* pf = (float*)(c.ws + c.plan.off_part);
      const float4* ja = (const float4*)jadj + 2 * b;
      sv.fn[comp](dim3((unsigned)tiles), c.st, ja, ns, (int32_t)nb, (float)eps2, pf);
      LAUNCH_CHECK("adjoint_sym_kernel");
      AdjNext an{};
      if (next && !c.bat && b == 0 && !is_fp64(prec)) {  // one system: its staging covers every particle
        an.kind = 1;
        an.pos = next->pos;
        an.mass = mass;
        an.gvel = gvel;
        an.h_drift = next->h_drift;
        an.w = next->w;
        an.jadj = (float4*)jadj;
        if (fused) *fused = true;
      }
      hipLaunchKernelGGL(adjoint_reduce_sym_groups, grid1d(ns, 64), dim3(256), 0, c.st, ns, n, (int32_t)nb,
                         (const float*)pf, c.cfg->G, gpos + b, gmass + b, an);
      LAUNCH_CHECK("adjoint_reduce_sym_groups");
      return NBODY_OK;
    }
    int64_t S, jc;
    split_geometry(t, ns, S, jc);
    const AdjVariant& av = is_fp64(prec) ? kAdj64[t.variant] : kAdj32[t.variant];
    AdjOut o{};
    o.G = c.cfg->G;
    o.n_plane = n;
    dim3 g((unsigned)cdiv(ns, (int64_t)t.bs * t.i), (unsigned)S);
    if (S == 1) {
      o.gpos = gpos; o.gmass = gmass;
    } else {
      TRY(check_part(c, (size_t)S * 8 * n * sizeof(double), "adjoint_kernel"));
      o.part = part;
    }
    av.fn[comp](g, c.st, jadj, b, e, b, e, jc, eps2, o);
    LAUNCH_CHECK("adjoint_kernel");
    if (S > 1) {
      if (is_fp64(prec))
        hipLaunchKernelGGL(adjoint_reduce<double>, grid1d(ns), dim3(256), 0, c.st, ns, n, (int32_t)S, part + b,
                           (const D4*)jadj + 2 * b, c.cfg->G, gpos + b, gmass + b, (int64_t)0,
                           (const int64_t*)nullptr, (const int32_t*)nullptr);
      else
        hipLaunchKernelGGL(adjoint_reduce<float>, grid1d(ns), dim3(256), 0, c.st, ns, n, (int32_t)S, part + b,
                           (const float4*)jadj + 2 * b, c.cfg->G, gpos + b, gmass + b, (int64_t)0,
                           (const int64_t*)nullptr, (const int32_t*)nullptr);
      LAUNCH_CHECK("adjoint_reduce");
    }
    return NBODY_OK;
  };
  if (!c.bat) return single(0, n);
  if (c.loop) {
    for (int64_t s = 0; s < c.sys.S; ++s) TRY(single(c.sys.off[s], c.sys.off[s + 1]));
    return NBODY_OK;
  }
  Tile t = lookup_tile(NBODY_KERNEL_ADJOINT_BATCHED, prec, c.sys.max_n);
  const dim3 ugrid((unsigned)std::max<int64_t>(1, c.plan.n_units_adj));  // one workgroup per work unit
  const int32_t* nsplit_adj = (const int32_t*)(c.ws + c.plan.off_nsplit) + c.sys.S;
  if (t.sym >= 0) {
    if (!c.ua.sym) return fail(NBODY_ERR_DEVICE, "internal: symmetric batched adjoint tile without symmetric units");
    TRY(check_part(c, (size_t)c.ua.part_floats * sizeof(float), "adjoint_sym_batched_kernel"));
    const AdjSymVariant& sv = kAdjSym32[t.sym];
    float* pf = (float*)(c.ws + c.plan.off_part);
    sv.bfn[comp](ugrid, c.st, (const float4*)jadj, (const SymUnit*)(c.ws + c.plan.off_units_adj),
                 (int32_t)c.plan.n_units_adj, (float)eps2, pf);
    LAUNCH_CHECK("adjoint_sym_batched_kernel");
    hipLaunchKernelGGL(adjoint_reduce_sym, grid1d(n), dim3(256), 0, c.st, n, n, (int32_t)0, (const float*)pf,
                       c.cfg->G, gpos, gmass, c.sys.S,
                       (const int64_t*)(c.ws + c.plan.off_sysoff), nsplit_adj,
                       (const int64_t*)(c.ws + c.plan.off_partoff_adj));
    LAUNCH_CHECK("adjoint_reduce_sym");
    return NBODY_OK;
  }
  if (c.ua.sym) return fail(NBODY_ERR_DEVICE, "internal: one-sided batched adjoint tile with symmetric units");
  const AdjVariant& av = is_fp64(prec) ? kAdj64[t.variant] : kAdj32[t.variant];
  TRY(check_part(c, (size_t)max_nsplit(c.ua) * 8 * n * sizeof(double), "adjoint_batched_kernel"));
  AdjOut o{};
  o.G = c.cfg->G;
  o.n_plane = n;
  o.part = part;
  av.bfn[comp](ugrid, c.st, jadj, (const WorkUnit*)(c.ws + c.plan.off_units_adj), (int32_t)c.plan.n_units_adj, eps2,
               o);
  LAUNCH_CHECK("adjoint_batched_kernel");
  if (is_fp64(prec))
    hipLaunchKernelGGL(adjoint_reduce<double>, grid1d(n), dim3(256), 0, c.st, n, n, (int32_t)0, part, (const D4*)jadj,
                       c.cfg->G, gpos, gmass, c.sys.S, (const int64_t*)(c.ws + c.plan.off_sysoff), nsplit_adj);
  else
    hipLaunchKernelGGL(adjoint_reduce<float>, grid1d(n), dim3(256), 0, c.st, n, n, (int32_t)0, part,
                       (const float4*)jadj, c.cfg->G, gpos, gmass, c.sys.S,
                       (const int64_t*)(c.ws + c.plan.off_sysoff), nsplit_adj);
  LAUNCH_CHECK("adjoint_reduce");
  return NBODY_OK;
}

int copy_d2d(Ctx& c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return NBODY_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.st));
  return NBODY_OK;
}

int zero_f64(Ctx& c, double* p, int64_t count) {
  if (count == 0) return NBODY_OK;
  hipLaunchKernelGGL(fill_f64, grid1d(count), dim3(256), 0, c.st, p, count, 0.0);
  LAUNCH_CHECK("fill_f64");
  return NBODY_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

__attribute__((visibility("default"))) int nbody_abi_version(void) { return NBODY_ABI_VERSION; }

__attribute__((visibility("default"))) int nbody_set_wait_limit(int64_t probes) {
  g_err.clear();
  if (probes < 1) return fail(NBODY_ERR_INVALID_ARG, "probes must be >= 1 (got %lld)", (long long)probes);
  g_wait_limit.store(probes);
  return NBODY_OK;
}

__attribute__((visibility("default"))) const char* nbody_last_error(void) { return g_err.c_str(); }

__attribute__((visibility("default"))) int nbody_workspace_size(const nbody_config* cfg, int64_t n, int64_t steps,
                                                                int64_t ckpt_every, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(NBODY_ERR_INVALID_ARG, "bytes is NULL");
  Systems sys;
  TRY(check_cfg(cfg, n, sys, false));  // the size does not depend on the pair law's constants
  if (steps < 0) return fail(NBODY_ERR_INVALID_ARG, "steps must be >= 0");
  if (ckpt_every < 0) return fail(NBODY_ERR_INVALID_ARG, "ckpt_every must be >= 0");
  Plan p;
  unsigned need = NEED_FORCE | NEED_ENERGY | NEED_ROLLOUT;
  if (ckpt_every > 0) need |= NEED_BACKWARD;  // what nbody_rollout_backward plans for any step count
  TRY(make_plan(cfg, sys, n, std::max<int64_t>(ckpt_every, 1), need, p, nullptr, nullptr));
  *bytes = p.total;
  return NBODY_OK;
}

__attribute__((visibility("default"))) int nbody_forces(const nbody_config* cfg, int64_t n, const double* pos,
                                                        const double* mass, double* acc, double* pot) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE));
  if (n == 0) return NBODY_OK;
  if (!pos || !mass || !acc) return fail(NBODY_ERR_INVALID_ARG, "pos, mass and acc must be non-NULL");
  TRY(upload_meta(c));
  TRY(stage(c, pos, mass));
  return force_pass(c, acc, pot, nullptr, 0.0);
}

__attribute__((visibility("default"))) int nbody_forces_shard_workspace_size(const nbody_config* cfg, int64_t n,
                                                                              int32_t P, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(NBODY_ERR_INVALID_ARG, "bytes is NULL");
  Systems sys;
  TRY(check_cfg(cfg, n, sys, true));
  if (sys.S != 1) return fail(NBODY_ERR_UNSUPPORTED, "a ring share is of a single system (n_systems == 1)");
  Plan p;
  Tile t;
  int64_t S, s;
  TRY(shard_plan(cfg, n, P, p, t, S, s));
  *bytes = p.total;
  return NBODY_OK;
}

__attribute__((visibility("default"))) int nbody_forces_shard(const nbody_config* cfg, int64_t n, int32_t P, int32_t g,
                                                              const double* pos, const double* mass, double* acc,
                                                              double* pot) {
  g_err.clear();
  if (P < 1 || g < 0 || g >= P) return fail(NBODY_ERR_INVALID_ARG, "need P >= 1 and 0 <= g < P (got P = %d, g = %d)",
                                           (int)P, (int)g);
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE, nullptr, false, P));
  if (n == 0) return NBODY_OK;
  if (!pos || !mass || !acc) return fail(NBODY_ERR_INVALID_ARG, "pos, mass and acc must be non-NULL");
  Plan p;
  Tile t;
  int64_t S, s;
  TRY(shard_plan(cfg, n, P, p, t, S, s));
  const int64_t i0 = (int64_t)g * s, i1 = std::min<int64_t>(n, i0 + s);
  if (i0 >= n) return NBODY_OK;  // a block past the particles (small n): nothing to write
  TRY(stage(c, pos, mass));
  const int prec = cfg->precision;
  const ForceVariant& fv = is_fp64(prec) ? kForce64[0] : kForce32[0];
  ForceOut o{};
  o.ls = c.ls;  // direct stores index particles globally (i in [i0, i1))
  o.n_plane = n;
  double* part = (double*)(c.ws + c.plan.off_part);
  if (S == 1) {
    o.acc = acc;
    o.pot = pot;
  } else {
    TRY(check_part(c, (size_t)S * 4 * n * sizeof(double), "force_kernel (ring share)"));
    o.part = part;
  }
  const dim3 grid((unsigned)cdiv(i1 - i0, (int64_t)t.bs * t.i), (unsigned)S);
  fv.fn[LAW_GRAV][pot != nullptr][force_mode(prec)](grid, c.st, c.ws + c.plan.off_jbuf, i0, i1, 0, n, s, c.eps2, o);
  LAUNCH_CHECK("force_kernel (ring share)");
  if (S > 1) {
    hipLaunchKernelGGL(reduce_splits, grid1d(i1 - i0), dim3(kReduceBS), 0, c.st, i1 - i0, n, (int32_t)S, part + i0,
                       c.ls_at(i0), acc + i0, pot ? pot + i0 : nullptr, (double*)nullptr, 0.0, (int64_t)0,
                       (const int64_t*)nullptr, (const int32_t*)nullptr, NextStep{}, EnergyFuse{});
    LAUNCH_CHECK("reduce_splits (ring share)");
  }
  return NBODY_OK;
}

__attribute__((visibility("default"))) int nbody_step(const nbody_config* cfg, int64_t n, double dt, double* pos,
                                                      double* vel, const double* mass, double* acc, double* pot) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE));
  if (!std::isfinite(dt)) return fail(NBODY_ERR_INVALID_ARG, "dt must be finite");
  if (n == 0) return NBODY_OK;
  if (!pos || !vel || !mass || !acc) return fail(NBODY_ERR_INVALID_ARG, "pos, vel, mass and acc must be non-NULL");
  TRY(upload_meta(c));
  TRY(kick_drift(c, dt, pos, vel, acc, mass));
  return force_pass(c, acc, pot, vel, 0.5 * dt);
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free step

// The workspace of nbody_step_noalloc: a file-scope device array, one copy per GPU the library
// runs on, held until the process ends. In host code its name is only a stand-in: its device
// address comes from hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[NBODY_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the first call on a device).
int scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NBODY_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p) % kAlign) return fail(NBODY_ERR_DEVICE, "scratch array address unusable");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NBODY_OK;
}

}  // namespace

extern "C" {

__attribute__((visibility("default"))) int nbody_step_noalloc(const nbody_config* cfg, int64_t n, double dt,
                                                              double* pos, double* vel, const double* mass,
                                                              double* acc, double* pot) {
  g_err.clear();
  if (!cfg) return fail(NBODY_ERR_INVALID_ARG, "cfg is NULL");
  if (cfg->workspace || cfg->workspace_bytes)
    return fail(NBODY_ERR_INVALID_ARG, "nbody_step_noalloc takes no workspace: workspace must be NULL and "
                                       "workspace_bytes 0");
  if (cfg->n_systems != 1 || cfg->offsets)
    return fail(NBODY_ERR_UNSUPPORTED, "nbody_step_noalloc serves a single system (n_systems == 1, offsets NULL)");
  // The first plan of the order tuned tile, largest-block tile, round schedule, one-sided pass
  // whose whole workspace fits the scratch (for the last, j-range partials that leave room for
  // the rest of the workspace, at most 128 bytes per particle). Cap and level hold for this
  // thread until the call returns.
  struct CapGuard {
    double cap = g_sym_cap;
    int level = g_sym_level;
    bool one_stream = g_rounds_one_stream;
    ~CapGuard() {
      g_sym_cap = cap;
      g_sym_level = level;
      g_rounds_one_stream = one_stream;
    }
  } cap_guard;
  g_rounds_one_stream = true;  // the round schedule's launches on the caller's stream only
  const double total = (double)NBODY_NOALLOC_SCRATCH_BYTES;
  size_t need = 0;
  for (int level = 0; level < 4; ++level) {
    g_sym_level = level;
    g_sym_cap = level < 3 ? total : std::max(0.0, total - 128.0 * (double)n);
    TRY(nbody_workspace_size(cfg, n, 1, 0, &need));
    if (need <= (size_t)NBODY_NOALLOC_SCRATCH_BYTES) break;
  }
  if (need > (size_t)NBODY_NOALLOC_SCRATCH_BYTES)
    return fail(NBODY_ERR_WORKSPACE, "n = %lld needs %zu bytes of scratch; the static scratch of "
                                     "nbody_step_noalloc holds %zu (use nbody_step with a workspace)",
                (long long)n, need, (size_t)NBODY_NOALLOC_SCRATCH_BYTES);
  if (n == 0) return NBODY_OK;
  nbody_config c = *cfg;
  TRY(scratch_address(&c.workspace));
  c.workspace_bytes = NBODY_NOALLOC_SCRATCH_BYTES;
  return nbody_step(&c, n, dt, pos, vel, mass, acc, pot);
}

}  // extern "C"

namespace {

// Every step of a batched rollout on symmetric tiles in one launch (see
// rollout_sym_batched_kernel): the first half of step 0 here, then the kernel, then a
// read-back of its error word.
int whole_rollout(Ctx& c, double dt, int64_t steps, double* pos, double* vel, const double* mass, double* acc,
                  const NextStep& nx) {
  if (steps > 0x7fffffffLL) return fail(NBODY_ERR_UNSUPPORTED, "too many steps for one launch");
  Tile t = lookup_tile(force_kernel_id(c.law, true), c.cfg->precision, c.sys.max_n);
  if (t.sym < 0 || !c.uf.sym) return fail(NBODY_ERR_DEVICE, "internal: whole rollout without symmetric units");
  TRY(check_part(c, (size_t)c.uf.part_floats * sizeof(float), "rollout_sym_batched_kernel"));
  const SymVariant& sv = kSym32[t.sym];
  const int law = c.law, mode = force_mode(c.cfg->precision);
  TRY(kick_drift(c, dt, pos, vel, acc, mass));
  int32_t* words = (int32_t*)(c.ws + c.plan.off_sync);
  const int64_t nwords = 4 + 2 * c.sys.S;
  hipLaunchKernelGGL(fill_i32, grid1d(nwords), dim3(256), 0, c.st, words, nwords, 0);
  LAUNCH_CHECK("fill_i32");
  RolloutSync sy;
  sy.queue = (unsigned long long*)words;
  sy.err = words + 2;
  sy.tiles_done = words + 4;
  sy.red_done = words + 4 + c.sys.S;
  sy.spin_limit = g_wait_limit.load();
  unsigned grid;
  const int64_t n_rtasks = (int64_t)c.uf.rtasks.size() / 2;
  const int64_t n_solo = c.uf.n_solo, n_multi = (int64_t)c.uf.ro_units.size() - n_solo;
  TRY(persistent_grid(sv.rptr[law][mode](), sv.w * 64, n_solo + (n_multi + n_rtasks) * steps, grid));
  sv.rfn[law][mode](dim3(grid), c.st, (const float4*)(c.ws + c.plan.off_jbuf),
                    (const SymUnit*)(c.ws + c.plan.off_units_ro), (int32_t)n_solo, (int32_t)n_multi,
                    (const int32_t*)(c.ws + c.plan.off_rtasks), (int32_t)n_rtasks, c.n,
                    (const int64_t*)(c.ws + c.plan.off_sysoff), (const int32_t*)(c.ws + c.plan.off_nsplit),
                    (const int64_t*)(c.ws + c.plan.off_partoff), (float)c.eps2, (float*)(c.ws + c.plan.off_part), c.ls,
                    acc, vel, 0.5 * dt, nx, (int32_t)steps, sy);
  LAUNCH_CHECK("rollout_sym_batched_kernel");
  if (n_multi == 0) return NBODY_OK;  // no task waits on another: nothing can time out
  int32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, sy.err, sizeof err, hipMemcpyDeviceToHost, c.st));
  HIP_TRY(hipStreamSynchronize(c.st));
  if (err) return fail(NBODY_ERR_DEVICE, "whole rollout: a per-system wait gave up (device error word set)");
  return NBODY_OK;
}

// The KDK loop shared by both pair laws (c prepared with NEED_FORCE | NEED_ROLLOUT).
int rollout_impl(Ctx& c, int64_t n, double dt, int64_t steps, int64_t ckpt_every, double* pos, double* vel,
                 const double* mass, double* acc, double* ckpt, double* energy_trace) {
  if (!std::isfinite(dt)) return fail(NBODY_ERR_INVALID_ARG, "dt must be finite");
  if (steps < 0) return fail(NBODY_ERR_INVALID_ARG, "steps must be >= 0");
  if (ckpt && ckpt_every < 1) return fail(NBODY_ERR_INVALID_ARG, "ckpt_every must be >= 1 when ckpt is given");
  if (n == 0) return NBODY_OK;
  if (!pos || !vel || !mass || !acc) return fail(NBODY_ERR_INVALID_ARG, "pos, vel, mass and acc must be non-NULL");
  TRY(upload_meta(c));
  const size_t plane3 = (size_t)3 * n * sizeof(double);
  const int64_t S = c.sys.S;
  double* pot = energy_trace ? (double*)(c.ws + c.plan.off_pot) : nullptr;
  if (ckpt) {
    TRY(copy_d2d(c, ckpt, pos, plane3));
    TRY(copy_d2d(c, ckpt + 3 * n, vel, plane3));
  }
  if (energy_trace) {
    // potential at x_0 (the caller's acc is left untouched)
    TRY(stage(c, pos, mass));
    TRY(force_pass(c, (double*)(c.ws + c.plan.off_accs), pot, nullptr, 0.0));
    TRY(energy_pass(c, vel, mass, pot, energy_trace));
  }
  const NextStep nx = next_step(c, dt, pos, mass);
  // every step in one launch: on request, and by default when every system fits one tile (no
  // workgroup then waits on another, and the launch beats one per pass)
  if (!energy_trace && !ckpt && steps > 0 && c.bat && !c.loop && c.uf.sym &&
      ((c.cfg->flags & NBODY_FLAG_WHOLE_ROLLOUT) ||
       (!(c.cfg->flags & NBODY_FLAG_PER_PASS) && c.uf.n_solo == (int64_t)c.uf.ro_units.size())))
    return whole_rollout(c, dt, steps, pos, vel, mass, acc, nx);
  bool staged = false;  // the previous pass already ran this step's kick, drift and staging
  int32_t kept = 0;     // fused steps whose energy partials wait in slots 0 .. kept-1
  int64_t kept_from = 0;  // the first of them (its state is s + 1 = kept_from + 1)
  for (int64_t s = 0; s < steps; ++s) {
    if (!staged) TRY(kick_drift(c, dt, pos, vel, acc, mass));
    // the next step's first half rides on this pass unless the state at s + 1 is copied out
    // in between (checkpoint) or there is no next step; the energy of the state at s + 1
    // is reduced inside the same pass, before that next kick
    const bool ckpt_due = ckpt && (s + 1) % ckpt_every == 0;
    Fuse fz;
    fz.nx = s + 1 < steps && !ckpt_due ? &nx : nullptr;
    fz.eout = energy_trace ? energy_trace + (s + 1) * S * 5 : nullptr;
    fz.mass = mass;
    if (energy_trace) {
      if (kept == 0) kept_from = s;
      fz.eslot = kept;
    }
    TRY(force_pass(c, acc, pot, vel, 0.5 * dt, &fz));
    staged = fz.done && fz.nx;
    if (energy_trace) {
      if (fz.done) ++kept;
      // energy_pass reuses slot 0: sum what is kept first
      if (!fz.done || kept == c.plan.e_steps || s + 1 == steps) {
        TRY(flush_energy(c, kept, energy_trace + (kept_from + 1) * S * 5));
        kept = 0;
      }
      if (!fz.done) TRY(energy_pass(c, vel, mass, pot, fz.eout));
    }
    if (ckpt && (s + 1) % ckpt_every == 0) {
      double* slot = ckpt + (size_t)((s + 1) / ckpt_every) * 6 * n;
      TRY(copy_d2d(c, slot, pos, plane3));
      TRY(copy_d2d(c, slot + 3 * n, vel, plane3));
    }
  }
  return NBODY_OK;
}

}  // namespace

extern "C" {

__attribute__((visibility("default"))) int nbody_rollout(const nbody_config* cfg, int64_t n, double dt, int64_t steps,
                                                         int64_t ckpt_every, double* pos, double* vel,
                                                         const double* mass, double* acc, double* ckpt,
                                                         double* energy_trace) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE | NEED_ROLLOUT));
  return rollout_impl(c, n, dt, steps, ckpt_every, pos, vel, mass, acc, ckpt, energy_trace);
}

__attribute__((visibility("default"))) int nbody_lj_forces(const nbody_config* cfg, const nbody_lj_params* lj,
                                                           int64_t n, const double* pos, const double* mass,
                                                           double* acc, double* pot) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE, lj));
  if (n == 0) return NBODY_OK;
  if (!pos || !mass || !acc) return fail(NBODY_ERR_INVALID_ARG, "pos, mass and acc must be non-NULL");
  c.ls.mdiv = mass;
  TRY(upload_meta(c));
  TRY(stage(c, pos, mass));
  return force_pass(c, acc, pot, nullptr, 0.0);
}

__attribute__((visibility("default"))) int nbody_lj_rollout(const nbody_config* cfg, const nbody_lj_params* lj,
                                                            int64_t n, double dt, int64_t steps, double* pos,
                                                            double* vel, const double* mass, double* acc,
                                                            double* energy_trace) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE | NEED_ROLLOUT, lj));
  c.ls.mdiv = mass;
  return rollout_impl(c, n, dt, steps, 0, pos, vel, mass, acc, nullptr, energy_trace);
}

__attribute__((visibility("default"))) int nbody_energy_momentum(const nbody_config* cfg, int64_t n,
                                                                 const double* pos, const double* vel,
                                                                 const double* mass, const double* pot,
                                                                 double* out) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_ENERGY | (pot ? 0u : (unsigned)NEED_FORCE)));
  if (!out) return fail(NBODY_ERR_INVALID_ARG, "out must be non-NULL");
  if (n == 0) {
    // every system is empty: zero energy and momentum
    hipLaunchKernelGGL(fill_f64, grid1d(c.sys.S * 5), dim3(256), 0, (hipStream_t)cfg->stream, out, c.sys.S * 5, 0.0);
    LAUNCH_CHECK("fill_f64");
    return NBODY_OK;
  }
  if (!vel || !mass || (!pot && !pos)) return fail(NBODY_ERR_INVALID_ARG, "vel, mass and pos (or pot) must be non-NULL");
  TRY(upload_meta(c));
  const double* p = pot;
  if (!p) {
    double* pw = (double*)(c.ws + c.plan.off_pot);
    TRY(stage(c, pos, mass));
    TRY(force_pass(c, (double*)(c.ws + c.plan.off_accs), pw, nullptr, 0.0));
    p = pw;
  }
  return energy_pass(c, vel, mass, p, out);
}

__attribute__((visibility("default"))) int nbody_diagnostics(const nbody_config* cfg, int64_t n, const double* pos,
                                                             const double* vel, const double* mass, const double* pot,
                                                             const double* acc, double* out) {
  g_err.clear();
  Ctx c;
  // law-free: pot and acc come from the caller's force pass, G and eps are not used
  TRY(prepare(c, cfg, n, 1, NEED_ENERGY, nullptr, true));
  if (!out) return fail(NBODY_ERR_INVALID_ARG, "out must be non-NULL");
  if (n == 0) {
    hipLaunchKernelGGL(fill_f64, grid1d(c.sys.S * kDiag), dim3(256), 0, c.st, out, c.sys.S * kDiag, 0.0);
    LAUNCH_CHECK("fill_f64");
    return NBODY_OK;
  }
  if (!pos || !vel || !mass || !pot || !acc)
    return fail(NBODY_ERR_INVALID_ARG, "pos, vel, mass, pot and acc must be non-NULL");
  TRY(upload_meta(c));
  return diag_pass(c, pos, vel, mass, pot, acc, out);
}

__attribute__((visibility("default"))) int nbody_rollout_backward(const nbody_config* cfg, int64_t n, double dt,
                                                                  int64_t steps, int64_t ckpt_every,
                                                                  const double* mass, const double* ckpt,
                                                                  const double* gpos_final,
                                                                  const double* gvel_final, double* gpos0,
                                                                  double* gvel0, double* gmass) {
  g_err.clear();
  if (ckpt_every < 1) return fail(NBODY_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  Ctx c;
  TRY(prepare(c, cfg, n, ckpt_every, NEED_FORCE | NEED_BACKWARD));
  if (!std::isfinite(dt)) return fail(NBODY_ERR_INVALID_ARG, "dt must be finite");
  if (steps < 0) return fail(NBODY_ERR_INVALID_ARG, "steps must be >= 0");
  if (n == 0) return NBODY_OK;
  if (!mass || !ckpt || !gpos_final || !gvel_final || !gpos0 || !gvel0 || !gmass)
    return fail(NBODY_ERR_INVALID_ARG, "mass, ckpt, gradients and outputs must be non-NULL");
  TRY(upload_meta(c));
  const size_t plane3 = (size_t)3 * n * sizeof(double);
  const double h = dt;
  double* xw = (double*)(c.ws + c.plan.off_xw);
  double* vw = (double*)(c.ws + c.plan.off_vw);
  double* aw = (double*)(c.ws + c.plan.off_aw);
  double* seg = (double*)(c.ws + c.plan.off_seg);

  TRY(copy_d2d(c, gpos0, gpos_final, plane3));
  TRY(copy_d2d(c, gvel0, gvel_final, plane3));
  TRY(zero_f64(c, gmass, n));
  if (steps == 0) return NBODY_OK;

  const int64_t nseg = cdiv(steps, ckpt_every);
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t t0 = sg * ckpt_every;
    const int64_t t1 = std::min(t0 + ckpt_every, steps);
    const bool last = (sg == nseg - 1);
    // recompute x_t0 .. x_t1 (x_t1 only needed by the last segment) into seg[0 .. t1-t0]
    const double* ck = ckpt + (size_t)sg * 6 * n;
    TRY(copy_d2d(c, xw, ck, plane3));
    TRY(copy_d2d(c, vw, ck + 3 * n, plane3));
    TRY(copy_d2d(c, seg, xw, plane3));
    const int64_t t_end = last ? t1 : t1 - 1;  // last position to recompute
    if (t_end > t0) {
      TRY(stage(c, xw, mass));
      TRY(force_pass(c, aw, nullptr, nullptr, 0.0));
      TRY(kick_drift(c, h, xw, vw, aw, mass));
      TRY(copy_d2d(c, seg + (size_t)3 * n, xw, plane3));
      NextStep nx = next_step(c, h, xw, mass);
      for (int64_t t = t0 + 1; t < t_end; ++t) {
        // the pass at x_t closes step t - 1; its reduction also runs the first half of step t,
        // writing x_{t+1} to xw and to the segment (as a rollout's fused steps do)
        double* dst = seg + (size_t)(t + 1 - t0) * 3 * n;
        nx.pos_copy = dst;
        Fuse fz;
        fz.nx = &nx;
        TRY(force_pass(c, aw, nullptr, vw, 0.5 * h, &fz));
        if (!fz.done) {  // a pass without such a reduction: the first half and the copy here
          TRY(kick_drift(c, h, xw, vw, aw, mass));
          TRY(copy_d2d(c, dst, xw, plane3));
        }
      }
    }
    // reverse sweep over this segment; a pass whose reduction can stage the next pass of the
    // segment does so (the next segment's recomputation reuses the j-array first)
    auto next_of = [&](int64_t t) {  // the staging of the pass at x_t
      return AdjNextArgs{seg + (size_t)(t - t0) * 3 * n, h, t > 0 ? h : 0.5 * h};
    };
    bool staged = false;
    if (last) {
      const double* xK = seg + (size_t)(steps - t0) * 3 * n;
      const AdjNextArgs nxt = next_of(t1 - 1);
      TRY(adjoint_pass(c, xK, mass, gvel0, gpos0, 0.0, 0.5 * h, gpos0, gmass, &nxt, false, &staged));
    }
    for (int64_t t = t1 - 1; t >= t0; --t) {
      const double* xt = seg + (size_t)(t - t0) * 3 * n;
      const double w = t > 0 ? h : 0.5 * h;
      bool fused = false;
      if (t > t0) {
        const AdjNextArgs nxt = next_of(t - 1);
        TRY(adjoint_pass(c, xt, mass, gvel0, gpos0, h, w, gpos0, gmass, &nxt, staged, &fused));
      } else {
        TRY(adjoint_pass(c, xt, mass, gvel0, gpos0, h, w, gpos0, gmass, nullptr, staged, &fused));
      }
      staged = fused;
    }
  }
  return NBODY_OK;
}

__attribute__((visibility("default"))) int nbody_rollout_backward_reversible(
    const nbody_config* cfg, int64_t n, double dt, int64_t steps, const double* mass, const double* pos_final,
    const double* vel_final, const double* gpos_final, const double* gvel_final, double* gpos0, double* gvel0,
    double* gmass) {
  g_err.clear();
  Ctx c;
  TRY(prepare(c, cfg, n, 1, NEED_FORCE | NEED_BACKWARD));
  if (!std::isfinite(dt)) return fail(NBODY_ERR_INVALID_ARG, "dt must be finite");
  if (steps < 0) return fail(NBODY_ERR_INVALID_ARG, "steps must be >= 0");
  if (n == 0) return NBODY_OK;
  if (!mass || !pos_final || !vel_final || !gpos_final || !gvel_final || !gpos0 || !gvel0 || !gmass)
    return fail(NBODY_ERR_INVALID_ARG, "mass, final state, gradients and outputs must be non-NULL");
  TRY(upload_meta(c));
  const size_t plane3 = (size_t)3 * n * sizeof(double);
  const double h = dt;
  double* xw = (double*)(c.ws + c.plan.off_xw);
  double* vw = (double*)(c.ws + c.plan.off_vw);
  double* aw = (double*)(c.ws + c.plan.off_aw);
  TRY(copy_d2d(c, gpos0, gpos_final, plane3));
  TRY(copy_d2d(c, gvel0, gvel_final, plane3));
  TRY(zero_f64(c, gmass, n));
  if (steps == 0) return NBODY_OK;
  TRY(copy_d2d(c, xw, pos_final, plane3));
  TRY(copy_d2d(c, vw, vel_final, plane3));
  TRY(stage(c, xw, mass));
  TRY(force_pass(c, aw, nullptr, nullptr, 0.0));  // a(x_K)
  TRY(adjoint_pass(c, xw, mass, gvel0, gpos0, 0.0, 0.5 * h, gpos0, gmass));
  for (int64_t t = steps - 1; t >= 0; --t) {
    // one kick-drift-kick step of -h takes (x_{t+1}, v_{t+1}, a_{t+1}) back to (x_t, v_t, a_t)
    TRY(kick_drift(c, -h, xw, vw, aw, mass));
    TRY(force_pass(c, aw, nullptr, vw, -0.5 * h));
    const double w = t > 0 ? h : 0.5 * h;
    TRY(adjoint_pass(c, xw, mass, gvel0, gpos0, h, w, gpos0, gmass));
  }
  return NBODY_OK;
}

__attribute__((visibility("default"))) int nbody_set_tile_table(const nbody_tile_entry* entries, int64_t count) {
  g_err.clear();
  if (count < 0 || (count > 0 && !entries)) return fail(NBODY_ERR_INVALID_ARG, "bad tile table");
  for (int64_t k = 0; k < count; ++k) {
    const auto& e = entries[k];
    if (e.kernel < 0 || e.kernel >= kNumKernels) return fail(NBODY_ERR_INVALID_ARG, "entry %lld: bad kernel", (long long)k);
    if (e.precision < 0 || e.precision > 4) return fail(NBODY_ERR_INVALID_ARG, "entry %lld: bad precision", (long long)k);
    if (e.variant < 0 || e.variant >= num_variants(e.kernel, e.precision))
      return fail(NBODY_ERR_INVALID_ARG, "entry %lld: variant %d out of range", (long long)k, e.variant);
    if (e.j_split < 1 || e.n_min > e.n_max) return fail(NBODY_ERR_INVALID_ARG, "entry %lld: bad range/j_split", (long long)k);
  }
  std::lock_guard<std::mutex> lk(g_table_mu);
  g_table.assign(entries, entries + count);
  return NBODY_OK;
}

__attribute__((visibility("default"))) int nbody_tile_variants(int32_t kernel, int32_t precision, char* buf,
                                                               size_t cap) {
  g_err.clear();
  if (kernel < 0 || kernel >= kNumKernels || precision < 0 || precision > 4) {
    fail(NBODY_ERR_INVALID_ARG, "bad kernel/precision");
    return -1;
  }
  int nv = num_variants(kernel, precision);
  if (buf && cap > 0) {
    size_t pos = 0;
    for (int v = 0; v < nv; ++v) {
      int bs, i, tj;
      variant_shape(kernel, precision, v, bs, i, tj);
      char tmp[64];
      const int sv = sym_index(kernel, precision, v);
      int sw = 0, si = 0, srot = 0;
      if (sv >= 0) sym_shape(kernel, sv, sw, si, srot);
      const bool pipe = sv >= 0 && is_force_kernel(kernel) && kSym32[sv].pipe;
      int len = sv >= 0 ? snprintf(tmp, sizeof tmp, "bs=%d,i=%d,sym=%d%s%s", bs, i, tj,
                                   srot == 1 ? ",rot=lds" : srot == 2 ? ",rot=mix" : "", pipe ? ",pipe" : "")
                        : snprintf(tmp, sizeof tmp, "bs=%d,i=%d,tj=%d", bs, i, tj);
      if (pos + len + 1 > cap) break;
      memcpy(buf + pos, tmp, len + 1);
      pos += len + 1;
    }
  }
  return nv;
}

__attribute__((visibility("default"))) int nbody_tile_lookup(int32_t kernel, int32_t precision, int64_t n,
                                                             int32_t* variant, int32_t* j_split) {
  g_err.clear();
  if (kernel < 0 || kernel >= kNumKernels || precision < 0 || precision > 4 || !variant || !j_split)
    return fail(NBODY_ERR_INVALID_ARG, "bad arguments");
  Tile t = lookup_tile(kernel, precision, n);
  *variant = t.variant;
  *j_split = (int32_t)t.j_split;
  return NBODY_OK;
}

}  // extern "C"
