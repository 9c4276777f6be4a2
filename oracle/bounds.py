"""Worst-case rounding-error bounds of the FP32 pair paths (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the smoke check and
the benchmark's error legs use these bounds to check a GPU result against the FP64 oracle.
Nothing here is called by the GPU product path.

Softened gravity, d = x_j - x_i, s = |d|^2 + eps^2, pair term m_j d s^{-3/2}:
  * rounding each coordinate to float moves it by at most u |x_c| per component
    (u = 2^-24), so a separation moves by at most sqrt(3) u (|x_i| + |x_j|) (taken
    componentwise, a safe over-estimate), and the float subtraction adds u |d|;
  * the Jacobian of d s^{-3/2} with respect to d has spectral norm at most 2 s^{-3/2};
  * the float pair arithmetic: r^2 by three fused multiply-adds (relative error <= 3u,
    which s^{-3/2} turns into 4.5u), the hardware reciprocal square root (<= 1 ulp = 2u,
    cubed: 6u) and three products (ri^2, ri^3, the mass): s^{-3/2} m_j is within 13.5u of
    exact; the multiply-add into the sum and the compensated fold add 2u;
  * the float sums between two compensated folds (at most 512 pair terms: one j-tile of
    the one-sided pass, a 64-step sub-block of the symmetric one) err by about
    sqrt(512) u < 23u of the sum of |term| (the usual probabilistic bound of a recursive
    sum; the worst case would be 511u);
So  B_i = u G sum_{j != i} m_j s^{-3/2} (2 sqrt(3) (|x_i| + |x_j|) + 41 |d|)
(2 + 13.5 + 2 + 23 = 40.5 <= 41). Plain float accumulation (no compensation) adds
sqrt(n) u sum_j |term|. Double-float separations round only the separation itself
(<= 2u |d| with the rounding of the low words), which replaces the coordinate term:
(4 + 13.5 + 2 + 23) |d| <= 43 |d|.
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24


def fp32_force_bound(pos, mass, eps, G=1.0, accumulate_plain=False, exact_coords=False, idx=None, chunk=512,
                     adaptive=False):
    """B_i of every particle (idx None) or of the particles idx, against all j != i.

    adaptive: the adaptive-separation mode. Every pair closer than T = X_max / 256 (X_max the
    largest coordinate magnitude) lies in sub-blocks whose boxes are closer than T, so it takes
    double-float separations (43 |d|); a pair at least T apart may take float separations, so it
    keeps the coordinate term (the larger of the two)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    rows = np.arange(n) if idx is None else np.asarray(idx, dtype=np.int64)
    xn = np.sqrt(np.sum(pos ** 2, axis=0))
    T = np.max(np.abs(pos)) / 256.0 if n else 0.0
    B = np.empty(rows.shape[0])
    # keep the temporaries near chunk * n doubles
    step = max(1, min(chunk, (1 << 24) // max(n, 1)))
    for k0 in range(0, rows.shape[0], step):
        r = rows[k0:k0 + step]
        d = pos[:, None, :] - pos[:, r, None]                # (3, len(r), n)
        dn = np.sqrt(np.sum(d * d, axis=0))
        s = dn * dn + eps * eps
        w = mass[None, :] * s ** -1.5
        w[np.arange(r.shape[0]), r] = 0.0  # the self pair adds exactly 0 on the GPU (d = 0)
        if exact_coords:
            k = 43.0 * dn
        elif adaptive:
            far = dn >= 0.999 * T  # box distances are taken on float coordinates
            k = np.where(far, 2 * math.sqrt(3.0) * (xn[r, None] + xn[None, :]) + 41.0 * dn, 43.0 * dn)
        else:
            k = 2 * math.sqrt(3.0) * (xn[r, None] + xn[None, :]) + (41 + (math.sqrt(n) if accumulate_plain else 0)) * dn
        B[k0:k0 + step] = U32 * G * np.sum(w * k, axis=1)
    return B


def fp32_vjp_bound(pos, mass, lam, eps, G=1.0, idx=None, chunk=512):
    """Worst-case rounding bounds (Bx_k, Bm_k) of the FP32 force-VJP pass for the particles
    idx (all when None):  gx_k = G sum_j T(d)(m_k l_j - m_j l_k),  gm_k = -G sum_j s^{-3/2} d.l_j.

    Mass cotangent, term t = s^{-3/2} d.l_j: |dt/dd| <= s^{-3/2} |l_j| (1 + 3 |d|^2 / s)
    <= 4 s^{-3/2} |l_j|, applied to the separation error sqrt(3) u (|x_k| + |x_j|) + u |d|;
    the arithmetic (s^{-3/2} as for the forces, 12.5u; the dot product, 3u; the cotangent and
    mass staged to float, 2u; the sums between compensated folds, 23u; the fold, 2u) stays
    below 64 u s^{-3/2} |d| |l_j|:
        Bm_k = u G sum_j s^{-3/2} |l_j| (4 sqrt(3) (|x_k| + |x_j|) + 68 |d|).
    Position cotangent, v = T(d) w with w = m_k l_j - m_j l_k: |T| <= 4 s^{-3/2} and
    |d(T w)/dd| <= 24 s^{-2} |w| (with |d| <= s^{1/2}); the arithmetic stays below
    64 u |T| |w|:
        Bx_k = u G sum_j |w| (24 s^{-2} (sqrt(3) (|x_k| + |x_j|) + |d|) + 256 s^{-3/2}).
    |w| is bounded by m_k |l_j| + m_j |l_k|."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    n = mass.shape[0]
    rows = np.arange(n) if idx is None else np.asarray(idx, dtype=np.int64)
    xn = np.sqrt(np.sum(pos ** 2, axis=0))
    ln = np.sqrt(np.sum(lam ** 2, axis=0))
    Bx = np.empty(rows.shape[0])
    Bm = np.empty(rows.shape[0])
    step = max(1, min(chunk, (1 << 24) // max(n, 1)))
    for k0 in range(0, rows.shape[0], step):
        r = rows[k0:k0 + step]
        d = pos[:, None, :] - pos[:, r, None]
        dn = np.sqrt(np.sum(d * d, axis=0))
        s = dn * dn + eps * eps
        s32 = s ** -1.5
        s32[np.arange(r.shape[0]), r] = 0.0  # no self pair
        coord = math.sqrt(3.0) * (xn[r, None] + xn[None, :])
        Bm[k0:k0 + step] = U32 * G * np.sum(s32 * ln[None, :] * (4.0 * coord + 68.0 * dn), axis=1)
        w = mass[r, None] * ln[None, :] + mass[None, :] * ln[r, None]
        Bx[k0:k0 + step] = U32 * G * np.sum(w * (24.0 * s32 / np.sqrt(s) * (coord + dn) + 256.0 * s32), axis=1)
    return Bx, Bm
