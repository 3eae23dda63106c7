"""Philox4x32-10 and the Box-Muller normal stream (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Algorithm 4 draws, for every particle and step, independent Gaussian
increments W^- and W^+ with covariance mu*tau*I_3 (the Euler-Maruyama step of
eq. ``rho_hat_update`` draws one increment with covariance 2*mu*tau*I_3).  The
paper does not fix a generator.  Both the oracle and the GPU library therefore
implement the same counter-based generator from its published definition:

  Philox4x32 with 10 rounds (J. K. Salmon, M. A. Moraes, R. O. Dror,
  D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
  a round maps counter (c0, c1, c2, c3) and key (k0, k1) to
      (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
  with M0 = 0xD2511F53, M1 = 0xCD9E8D57; between rounds the key is bumped by
  the Weyl constants (0x9E3779B9, 0xBB67AE85).

The stream contract (shared with the GPU library):

* key      = (low 32 bits of seed, high 32 bits of seed)
* counter  = (particle id, step n, slot, instance); slot 0 is W^- (or the
             single Euler-Maruyama increment), slot 1 is W^+.
* uniforms u = ((r >> 9) + 1/2) * 2^-23, an exact float32 and float64 value in
             [2^-24, 1 - 2^-24]: both sides see identical uniforms.
* normals  (z0, z1) = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1),
           z2       = sqrt(-2 ln u2)  cos 2 pi u3;  one call yields one 3-vector.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

SLOT_MINUS = 0  # W^- of the split step, or the single Euler-Maruyama increment
SLOT_PLUS = 1   # W^+ of the split step


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds; all arguments broadcastable integer arrays < 2^32.

    Returns a tuple of four uint64 arrays holding 32-bit outputs.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for _ in range(10):
        p0 = M0 * c0  # both factors < 2^32, so the product fits in 64 bits
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ k0, p1 & _MASK,
                          (p0 >> _S32) ^ c3 ^ k1, p0 & _MASK)
        k0 = (k0 + W0) & _MASK
        k1 = (k1 + W1) & _MASK
    return c0, c1, c2, c3


def seed_key(seed):
    """Key words (low, high) of a 64-bit seed."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniforms(r):
    """Map 32-bit outputs to uniforms ((r >> 9) + 1/2) 2^-23 (exact in fp32)."""
    r = np.asarray(r, dtype=np.uint64)
    return ((r >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def normals3(ids, n, slot, seed, instance=0):
    """Standard-normal 3-vectors for particle ids at step n, shape (len(ids), 3).

    One Philox call per particle: counter (id, n, slot, instance).
    """
    ids = np.asarray(ids, dtype=np.uint64)
    k0, k1 = seed_key(seed)
    r0, r1, r2, r3 = philox4x32_10(ids, n, slot, instance, k0, k1)
    u0, u1, u2, u3 = uniforms(r0), uniforms(r1), uniforms(r2), uniforms(r3)
    rad0 = np.sqrt(-2.0 * np.log(u0))
    rad2 = np.sqrt(-2.0 * np.log(u2))
    z = np.empty(ids.shape + (3,), dtype=np.float64)
    z[..., 0] = rad0 * np.cos(2.0 * np.pi * u1)
    z[..., 1] = rad0 * np.sin(2.0 * np.pi * u1)
    z[..., 2] = rad2 * np.cos(2.0 * np.pi * u3)
    return z
