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
* counter  = (particle id, step n, 0, instance): one call per particle and step.
* fields   the four outputs r0..r3 give six 21-bit fields
             f_i = r_i >> 11 (i = 0..3),
             f_4 = ((r0 & 0x7FF) << 10) | (r1 & 0x3FF),
             f_5 = ((r2 & 0x7FF) << 10) | (r3 & 0x3FF).
* uniforms u_i = (f_i + 1/2) 2^-21, an exact float32 and float64 value in
             [2^-22, 1 - 2^-22]: both sides see identical uniforms.
* normals  (z_2j, z_2j+1) = sqrt(-2 ln u_2j) (cos 2 pi u_2j+1, sin 2 pi u_2j+1),
             j = 0, 1, 2.
* increments  split step: W^- from (z0, z1, z2), W^+ from (z3, z4, z5);
             Euler-Maruyama: W from (z0, z1, z2).
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

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


def fields21(r0, r1, r2, r3):
    """The six 21-bit fields of one Philox output (uint64 arrays)."""
    r = [np.asarray(v, dtype=np.uint64) for v in (r0, r1, r2, r3)]
    s11, m11, m10 = np.uint64(11), np.uint64(0x7FF), np.uint64(0x3FF)
    f = [v >> s11 for v in r]
    f.append(((r[0] & m11) << np.uint64(10)) | (r[1] & m10))
    f.append(((r[2] & m11) << np.uint64(10)) | (r[3] & m10))
    return f


def uniforms21(f):
    """(f + 1/2) 2^-21 for 21-bit fields f (exact in float32)."""
    return (np.asarray(f, dtype=np.uint64).astype(np.float64) + 0.5) * 2.0 ** -21


def normals6_counter(c0, c1, c2, c3, seed):
    """Six standard normals per counter (c0, c1, c2, c3), shape (..., 6)."""
    k0, k1 = seed_key(seed)
    u = [uniforms21(f) for f in fields21(*philox4x32_10(c0, c1, c2, c3, k0, k1))]
    z = np.empty(np.broadcast(*u).shape + (6,), dtype=np.float64)
    for j in range(3):
        rad = np.sqrt(-2.0 * np.log(u[2 * j]))
        z[..., 2 * j] = rad * np.cos(2.0 * np.pi * u[2 * j + 1])
        z[..., 2 * j + 1] = rad * np.sin(2.0 * np.pi * u[2 * j + 1])
    return z


def normals6(ids, n, seed, instance=0):
    """The six normals of particle ids at step n, shape (len(ids), 6): counter
    (id, n, 0, instance)."""
    ids = np.asarray(ids, dtype=np.uint64)
    return normals6_counter(ids, n, 0, instance, seed)
