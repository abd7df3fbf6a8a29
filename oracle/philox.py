"""Oracle random numbers: Philox4x32-10, Poisson and Gaussian draws.

Test infrastructure (see the package docstring).

The paper adds photon noise and detector noise to the sub-aperture image
before the centroid (Sec. 4, "noise-added image"; Sec. 5, photon-noise
regime).  It does not say how, so the draws are keyed by counters rather
than by consumption order (reading O8):

* Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
  Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11), written
  here from its published definition.
* Poisson counts: sequential-search inversion for lambda < 20 and the
  transformed-rejection method with squeeze (PTRS) of W. Hormann, "The
  transformed rejection method for generating Poisson random variables",
  Insurance: Mathematics and Economics 12 (1993) 39-45, for lambda >= 20
  (the method holds from 10; the split is where the GPU's inversion stops
  being the cheaper one).
  Both decide an integer, so they run in FP32 arithmetic, the precision
  the GPU path takes the same decision in.
* Read noise: Box-Muller on words 2 and 3 of a pair block, both of its
  normal deviates used.

Counters (key: (seed mod 2^32, seed div 2^32)), for a sub-aperture image of
n pixels, h = ceil(n / 2), global sub-aperture g, frame f:
* pair block b < h: counter (0, b, g, f).  It serves pixels b and b + h (the
  latter if b + h < n): word 0 is the inversion uniform of pixel b, word 1
  that of pixel b + h; Box-Muller on words 2 and 3 gives r cos(theta) to
  pixel b and r sin(theta) to pixel b + h.
* rejection-sampler trial t = 1, 2, ... of pixel p: counter (t, p, g, f),
  words 0 and 1 the trial's two uniforms.
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

POISSON_SPLIT = 20.0
PTRS_MAX_TRIALS = 64
INVERSION_MAX_K = 100


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on counter (c0..c3) with key (k0, k1); uint32 arrays.

    Round: multiply words 0 and 2 by the two multipliers, 64-bit product
    split into hi/lo; new block (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key
    is bumped by the two Weyl constants before every round but the first.
    """
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK32)
    k1 = np.uint64(int(k1) & MASK32)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    s32 = np.uint64(32)
    mask = np.uint64(MASK32)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK32)
            k1 = np.uint64((int(k1) + W1) & MASK32)
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def uniform_f32(x):
    """Uniform in (0, 1) from a 32-bit word: ((x >> 9) + 1/2) * 2^-23, exact in FP32."""
    x = np.asarray(x, dtype=np.uint32)
    return ((x >> np.uint32(9)).astype(np.float32) + np.float32(0.5)) * np.float32(2.0 ** -23)


def noise_words(seed, trial, pix, gsub, frame):
    k0 = seed & MASK32
    k1 = (seed >> 32) & MASK32
    return philox4x32_10(trial, pix, gsub, frame, k0, k1)


def log_factorial_f32(k):
    """ln(k!) rounded to FP32."""
    k = np.asarray(k)
    out = np.array([math.lgamma(float(v) + 1.0) for v in k.ravel()], dtype=np.float64)
    return out.reshape(k.shape).astype(np.float32)


# 1/k rounded to FP32 (index 0 unused): the inversion multiplies by it instead of dividing by k
RCP_F32 = np.array([0.0] + [1.0 / k for k in range(1, 128)], dtype=np.float64).astype(np.float32)


def poisson_inversion_f32(lam, u):
    """Sequential-search inversion: smallest k with u <= sum_{j<=k} e^-lam lam^j / j!.

    FP32: p0 = exp(-lam); p_k = (p_{k-1} * lam) * r_k with r_k = 1/k rounded to FP32;
    F_k = F_{k-1} + p_k (reading O8).  The FP32 sum saturates a few 1e-7 below 1 for some
    lam; the search also stops at the first k whose term no longer changes F_k (the mass
    beyond it is below the sum's rounding), instead of running on to the step cap.
    """
    lam = np.asarray(lam, dtype=np.float32)
    u = np.asarray(u, dtype=np.float32)
    p = np.exp(-lam).astype(np.float32)
    F = p.copy()
    k = np.zeros(lam.shape, dtype=np.int64)
    active = u > F
    kk = 0
    while np.any(active) and kk < INVERSION_MAX_K:
        kk += 1
        p = np.where(active, (p * lam) * RCP_F32[kk], p).astype(np.float32)
        Fn = np.where(active, F + p, F).astype(np.float32)
        k = np.where(active, kk, k)
        active = active & (u > Fn) & (Fn > F)
        F = Fn
    return k


def ptrs_constants_f32(lam):
    lam = np.asarray(lam, dtype=np.float32)
    f = np.float32
    slam = np.sqrt(lam)
    loglam = np.log(lam)
    b = f(0.931) + f(2.53) * slam
    a = f(-0.059) + f(0.02483) * b
    invalpha = f(1.1239) + f(1.1328) / (b - f(3.4))
    vr = f(0.9277) - f(3.6224) / (b - f(2.0))
    return loglam, a, b, invalpha, vr


def ptrs_trial_f32(lam, u, v):
    """One PTRS trial in FP32: returns (k, accepted)."""
    f = np.float32
    lam = np.asarray(lam, dtype=np.float32)
    loglam, a, b, invalpha, vr = ptrs_constants_f32(lam)
    U = np.asarray(u, dtype=np.float32) - f(0.5)
    V = np.asarray(v, dtype=np.float32)
    us = f(0.5) - np.abs(U)
    kf = np.floor((f(2.0) * a / us + b) * U + lam + f(0.43)).astype(np.float32)
    quick = (us >= f(0.07)) & (V <= vr)
    reject = (kf < 0) | ((us < f(0.013)) & (V > us))
    kc = np.maximum(kf, 0).astype(np.int64)
    lhs = np.log(V) + np.log(invalpha) - np.log(a / (us * us) + b)
    rhs = -lam + kf * loglam - log_factorial_f32(kc)
    accept = quick | (~reject & (lhs <= rhs))
    return kc, accept


def pair_block(seed, pix, npix, gsub, frame):
    """Words of the pair block that serves each pixel, and whether the pixel is the second of its pair."""
    pix = np.asarray(pix, dtype=np.uint64)
    h = np.uint64((int(npix) + 1) // 2)
    second = pix >= h
    b = np.where(second, pix - h, pix)
    return noise_words(seed, np.zeros_like(b), b, gsub, frame), second


def _flat(shape, v):
    return np.broadcast_to(np.asarray(v, dtype=np.uint64), shape).ravel()


def poisson_counts(lam, seed, pix, gsub, frame, npix):
    """Poisson counts for expected values lam (any shape) of pixels pix of n = npix-pixel images."""
    lam = np.asarray(lam, dtype=np.float32)
    shape = lam.shape
    lam = lam.ravel()
    pix, gsub, frame = (_flat(shape, v) for v in (pix, gsub, frame))
    assert np.all(pix < np.uint64(npix))
    out = np.zeros(lam.shape, dtype=np.int64)
    w, second = pair_block(seed, pix, npix, gsub, frame)
    small = (lam > 0) & (lam < POISSON_SPLIT)
    if np.any(small):
        u = uniform_f32(np.where(second, w[1], w[0]))
        out[small] = poisson_inversion_f32(lam[small], u[small])
    big = np.nonzero(lam >= POISSON_SPLIT)[0]
    done = np.zeros(big.shape, dtype=bool)
    for t in range(1, PTRS_MAX_TRIALS + 1):
        idx = big[~done]
        if idx.size == 0:
            break
        wt = noise_words(seed, np.full(idx.shape, t, np.uint64), pix[idx], gsub[idx], frame[idx])
        k, acc = ptrs_trial_f32(lam[idx], uniform_f32(wt[0]), uniform_f32(wt[1]))
        out[idx[acc]] = k[acc]
        sel = np.nonzero(~done)[0]
        done[sel[acc]] = True
    if not np.all(done):
        rest = big[~done]
        out[rest] = np.floor(lam[rest] + np.float32(0.5)).astype(np.int64)
    return out.reshape(shape)


def read_noise(seed, pix, gsub, frame, npix):
    """Standard normal per pixel (FP64): r cos(theta) or r sin(theta) of its pair block's Box-Muller,
    r = sqrt(-2 ln u2), theta = 2 pi u3."""
    pix = np.asarray(pix, dtype=np.uint64)
    shape = np.broadcast_shapes(pix.shape, np.shape(gsub), np.shape(frame))
    pix, gsub, frame = (_flat(shape, v) for v in (pix, gsub, frame))
    assert np.all(pix < np.uint64(npix))
    w, second = pair_block(seed, pix, npix, gsub, frame)
    r = np.sqrt(-2.0 * np.log(uniform_f32(w[2]).astype(np.float64)))
    theta = 2.0 * np.pi * uniform_f32(w[3]).astype(np.float64)
    z = r * np.where(second, np.sin(theta), np.cos(theta))
    return z.reshape(shape)


def inversion_margin(lam, u):
    """FP64 distance from u to the nearest CDF boundary of Poisson(lam) (tie test)."""
    lam = float(lam)
    u = float(u)
    p = math.exp(-lam)
    F = p
    best = abs(u - F)
    for k in range(1, INVERSION_MAX_K):
        p *= lam / k
        F += p
        best = min(best, abs(u - F))
        if F > u + 0.01:
            break
    return best
