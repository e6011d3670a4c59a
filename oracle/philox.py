"""Philox4x32-10 counter-based generator and the draw layout of the sampler.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The generator is the one published by Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a 2x32-bit
key go through ten rounds of two 32x32->64 multiplications whose high and low
halves are permuted and xor-ed with the key; the key is bumped by two Weyl
constants between rounds.

The paper draws proposal noise from N(0, C_j) (Sec. 2.3, eq. (pCN-GM proposal)),
a mixture component with probabilities w_j, and a uniform for the
Metropolis-Hastings test (Alg. 2).  Both implementations of the sampler draw them
from this generator with one agreed layout, so that a move can be replayed
exactly on either side:

    key      = (seed mod 2^32, seed div 2^32)
    counter  = (block, particle, ctr mod 2^32, ctr div 2^32)

  * normal number i of a particle uses block i // 2: its four words give two
    53-bit uniforms u1, u2 and Box-Muller gives
        z_{2b}   = sqrt(-2 log(1 - u1)) cos(2 pi u2)
        z_{2b+1} = sqrt(-2 log(1 - u1)) sin(2 pi u2)
  * the two scalar uniforms of a move (component choice, MH test) come from
    block UNIFORM_BLOCK: U_comp from words 0,1 and U_acc from words 2,3.
  * a 53-bit uniform from words (a, b) is ((a >> 5) * 2^26 + (b >> 6)) / 2^53.

Move m of a call that starts at counter ctr uses ctr + m.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
UNIFORM_BLOCK = 0x80000000


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters.

    ctr: (..., 4) integers < 2^32; key: (..., 2) integers < 2^32 (broadcast).
    Returns (..., 4) uint64 arrays holding 32-bit words.
    """
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(k[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], c0.shape).copy()
    m32 = np.uint64(MASK32)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & m32
            k1 = (k1 + np.uint64(W1)) & m32
        p0 = np.uint64(M0) * c0          # < 2^64, exact in uint64
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & m32, lo1, (hi0 ^ c3 ^ k1) & m32, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def res53(a, b):
    """53-bit uniform in [0, 1) from two 32-bit words."""
    a = np.asarray(a, dtype=np.uint64) >> np.uint64(5)
    b = np.asarray(b, dtype=np.uint64) >> np.uint64(6)
    return (a * np.uint64(1 << 26) + b).astype(np.float64) * (2.0 ** -53)


def _key(seed):
    seed = int(seed)
    return np.array([seed & MASK32, (seed >> 32) & MASK32], dtype=np.uint64)


def _counters(blocks, particles, ctr):
    ctr = int(ctr)
    blocks = np.asarray(blocks, dtype=np.uint64)
    particles = np.asarray(particles, dtype=np.uint64)
    bb, pp = np.broadcast_arrays(blocks, particles)
    out = np.empty(bb.shape + (4,), dtype=np.uint64)
    out[..., 0] = bb
    out[..., 1] = pp
    out[..., 2] = ctr & MASK32
    out[..., 3] = (ctr >> 32) & MASK32
    return out


def normals(seed, ctr, particles, K):
    """Standard normals z[n, i], i < K, for the given particle ids."""
    particles = np.asarray(particles, dtype=np.int64)
    nb = (K + 1) // 2
    words = philox4x32_10(_counters(np.arange(nb)[None, :], particles[:, None], ctr), _key(seed))
    u1 = res53(words[..., 0], words[..., 1])
    u2 = res53(words[..., 2], words[..., 3])
    rad = np.sqrt(-2.0 * np.log(1.0 - u1))
    z = np.empty((particles.size, 2 * nb))
    z[:, 0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[:, 1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:, :K]


def move_uniforms(seed, ctr, particles):
    """(U_comp, U_acc) for the given particle ids at one counter value."""
    particles = np.asarray(particles, dtype=np.int64)
    words = philox4x32_10(_counters(np.uint64(UNIFORM_BLOCK), particles, ctr), _key(seed))
    return res53(words[..., 0], words[..., 1]), res53(words[..., 2], words[..., 3])
