"""Seeded synthetic inputs shared by the library's tests, the benchmark and the oracle checks.

This module only draws random numbers (numpy PCG64); it holds none of the
method's arithmetic, so the oracle and the device path can both consume its
outputs without sharing code.  Seeds are ``1000 * workload + stream`` with the
stream numbers below, so every array is reproducible on its own.

Workloads (the paper's datasets and trained weights are absent; uniform
integers of the same shapes stand in for them):
  1  plain CPMul-accumulate, N=2048, 2 primes: 8 ciphertexts x 8 plaintexts -> 1 ciphertext
  2  conv2d forward, N=8192, 3 primes: batch 16 of 3x32x32 activations (CIFAR-10
     image shape), 16 output channels, 3x3 kernel, stride 1, pad 1, int8 weights
  3  conv2d weight gradient, N=8192, 3 primes: batch 32, 16->16 channels, 16x16
     maps, 3x3 kernel, ciphertexts uniform mod q_i, plaintexts uniform mod t
  4  64 uneven layer jobs (conv 3->16 @32x32, 16->32 @16x16, 32->64 @8x8, FC
     256->10, FC 1024->256) over N in {4096 (2 primes), 8192 (3), 16384 (4)}
  5  serving: Poisson arrivals (mean 2000 jobs/s) drawn from workload 4's mix
"""
import numpy as np

STREAM_CT, STREAM_PT, STREAM_ACT, STREAM_SK, STREAM_A, STREAM_E, STREAM_MASK, STREAM_MIX, STREAM_ARRIVAL = range(1, 10)

T_PLAIN = 65537          # plaintext modulus t
ERR_SIGMA = 3.2          # error standard deviation
ERR_BOUND = 19           # tail cut (about 6 sigma)


def rng(workload, stream, extra=0):
    return np.random.Generator(np.random.PCG64(1000 * workload + stream + 100000 * extra))


def uniform_residues(g, lead_shape, q, N):
    """Array [*lead_shape, L, N] with plane i uniform in [0, q_i)."""
    L = len(q)
    out = np.empty(tuple(lead_shape) + (L, N), dtype=np.uint64)
    for i, qi in enumerate(q):
        out[..., i, :] = g.integers(0, int(qi), size=tuple(lead_shape) + (N,), dtype=np.uint64)
    return out


def uniform_mod_t(g, shape, t=T_PLAIN):
    return g.integers(0, t, size=shape, dtype=np.int64)


def int8_uniform(g, shape):
    return g.integers(-128, 128, size=shape, dtype=np.int64)


def ternary(g, N):
    return g.integers(-1, 2, size=N, dtype=np.int64)


def small_error(g, N, sigma=ERR_SIGMA, bound=ERR_BOUND):
    e = np.rint(g.normal(0.0, sigma, size=N))
    return np.clip(e, -bound, bound).astype(np.int64)


# Layer shapes of the uneven job mix: (kind, C_in, C_out, H, W, kernel, pad) or (kind, n_in, n_out)
MIX_LAYERS = [
    ("conv", 3, 16, 32, 32, 3, 1),
    ("conv", 16, 32, 16, 16, 3, 1),
    ("conv", 32, 64, 8, 8, 3, 1),
    ("fc", 256, 10),
    ("fc", 1024, 256),
]
MIX_RINGS = [(4096, 2), (8192, 3), (16384, 4)]


def job_mix(n_jobs=64, workload=4):
    """List of (layer index, ring index) drawn i.i.d. uniformly."""
    g = rng(workload, STREAM_MIX)
    lay = g.integers(0, len(MIX_LAYERS), size=n_jobs)
    ring = g.integers(0, len(MIX_RINGS), size=n_jobs)
    return [(int(a), int(b)) for a, b in zip(lay, ring)]


def poisson_arrivals(n, rate_per_s, workload=5):
    """Arrival times (seconds from 0) of a Poisson process."""
    g = rng(workload, STREAM_ARRIVAL)
    return np.cumsum(g.exponential(1.0 / rate_per_s, size=n))
