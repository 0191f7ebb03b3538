"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds data generators only (random draws, products of the planted factors,
noise); it contains none of DID's arithmetic.  It is the one module that both the oracle
side (tests, CPU baseline) and the GPU side (tests, bench) read, so that both consume
bit-identical inputs.

All matrices follow the paper's convention that each column of X is a sample: X is
M x N, the planted factors are B0 (M x K) and C0 (K x N).  Host arrays are returned as
float64 C-ordered NumPy arrays; ``to_f32_colmajor`` gives the float32 column-major copy
the GPU consumes, and ``as_oracle_input`` the float64 view of that very float32 data.

Recipes (seeds are the workload number unless a caller passes another):

* ``planted_lowrank`` (the 500 x 2000, K = 10 noiseless case):
  B0 ~ U[0,1]^{M x K}, C0 ~ U[0,1]^{K x N}, X = B0 C0.
* ``image_like`` (MNIST-shaped stand-in, 784 x 70000, K = 16): B0 ~ U[0,1] with each entry
  zeroed with probability 0.6, C0 ~ U[0,1], X = max(0, B0 C0 + 0.05 N(0,1)), then X is
  divided by its maximum so that X lies in [0, 1].
* ``large_halfnormal`` (5000 x 10^6, K = 50, generated block by block): B0 ~ U[0,1] from
  the parent seed, block p of C0 ~ U[0,1] and of the noise from
  ``SeedSequence(seed).spawn(n_blocks)[p]``, X = B0 C0 + |0.01 N(0,1)|.  Any prefix of
  blocks can be regenerated on its own, which is how the parity slices are built.
* ``serving_x`` (one served job): X = max(0, B0 C0 + 0.02 N(0,1)), U[0,1] factors, from
  the job's own seed; ``serving_jobs`` draws the arrival times and shapes.
* ``paper_synthetic`` (the experiments' synthetic sets, M = 5, K = 3): X = B0 C0 with
  U[0,1] factors (the paper's `rand` data; read as a product of uniform factors).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_init",
    "planted_lowrank",
    "image_like",
    "large_halfnormal",
    "large_halfnormal_device",
    "paper_synthetic",
    "paper_synthetic_device",
    "identifiable_plant",
    "to_f32_colmajor",
    "as_oracle_input",
    "serving_jobs",
    "serving_x",
    "serving_x_device",
    "round_to_bf16",
]


def uniform_init(M, N, K, seed):
    """Initial factors B ~ U[0,1]^{M x K}, C ~ U[0,1]^{K x N} for CPU-only oracle tests."""
    rng = np.random.default_rng(seed)
    return rng.random((M, K)), rng.random((K, N))


def planted_lowrank(M=500, N=2000, K=10, seed=1):
    """X = B0 C0 with B0, C0 i.i.d. U[0,1]; returns (X, B0, C0)."""
    rng = np.random.default_rng(seed)
    B0 = rng.random((M, K))
    C0 = rng.random((K, N))
    return B0 @ C0, B0, C0


def image_like(M=784, N=70000, K=16, seed=2, zero_frac=0.6, noise=0.05):
    """MNIST-shaped stand-in: sparse-ish nonnegative basis plus Gaussian noise, clipped."""
    rng = np.random.default_rng(seed)
    B0 = rng.random((M, K))
    B0[rng.random((M, K)) < zero_frac] = 0.0
    C0 = rng.random((K, N))
    X = B0 @ C0 + noise * rng.standard_normal((M, N))
    np.maximum(X, 0.0, out=X)
    X /= X.max()
    return X, B0, C0


def large_halfnormal(M=5000, N=1_000_000, K=50, seed=3, n_blocks=64, take_blocks=None, noise=0.01):
    """Block-generated X = B0 C0 + |noise N(0,1)|; returns (X, B0) for the first blocks.

    The full matrix has ``n_blocks`` contiguous column blocks of N / n_blocks columns.
    ``take_blocks`` (default all) generates only the leading blocks, so a slice of the large
    workload can be rebuilt exactly on a host that cannot hold all of it.
    """
    if N % n_blocks:
        raise ValueError("N must be a multiple of n_blocks")
    nb = N // n_blocks
    take = n_blocks if take_blocks is None else int(take_blocks)
    parent = np.random.SeedSequence(seed)
    B0 = np.random.default_rng(parent).random((M, K))
    children = parent.spawn(n_blocks)
    X = np.empty((M, take * nb))
    for p in range(take):
        rng = np.random.default_rng(children[p])
        C0p = rng.random((K, nb))
        X[:, p * nb:(p + 1) * nb] = B0 @ C0p + np.abs(noise * rng.standard_normal((M, nb)))
    return X, B0


def large_halfnormal_device(torch, M=5000, N=1_000_000, K=50, seed=3, n_blocks=64, device="cuda", noise=0.01):
    """Device-side generator with the large workload's recipe (same distributions).

    Used where the host cannot afford to build 20 GB of data quickly (the benchmark).  It
    draws from torch's device generator, so its values differ from ``large_halfnormal``;
    the recipe (shapes, distributions, block structure) is the same.  Returns a float32
    tensor ``Xt`` of shape (N, M), i.e. X in column-major storage.
    """
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    B0t = torch.rand((K, M), generator=g, device=device, dtype=torch.float32)  # B0^T
    Xt = torch.empty((N, M), device=device, dtype=torch.float32)
    nb = (N + n_blocks - 1) // n_blocks
    for a in range(0, N, nb):
        b = min(N, a + nb)
        C0t = torch.rand((b - a, K), generator=g, device=device, dtype=torch.float32)
        blk = Xt[a:b]
        torch.matmul(C0t, B0t, out=blk)
        nz = torch.randn((b - a, M), generator=g, device=device, dtype=torch.float32)
        blk.add_(nz.mul_(noise).abs_())
        del nz, C0t
    return Xt


def paper_synthetic(N, M=5, K=3, seed=4):
    """Synthetic sets of the experiments (M = 5, K = 3): X = B0 C0, U[0,1] factors."""
    rng = np.random.default_rng(seed)
    B0 = rng.random((M, K))
    C0 = rng.random((K, N))
    return B0 @ C0, B0, C0


def paper_synthetic_device(torch, N, M=5, K=3, seed=4, device="cuda"):
    """Device-side generator with ``paper_synthetic``'s recipe (U[0,1] factors, X = B0 C0)
    for sizes up to N = 10^8; draws from torch's device generator, so the values differ
    from the host generator's.  Returns X in column-major storage as an (N, M) float32
    tensor."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    B0t = torch.rand((K, M), generator=g, device=device, dtype=torch.float32)
    Xt = torch.empty((N, M), device=device, dtype=torch.float32)
    step = 1 << 24
    for a in range(0, N, step):
        b = min(N, a + step)
        C0t = torch.rand((b - a, K), generator=g, device=device, dtype=torch.float32)
        torch.matmul(C0t, B0t, out=Xt[a:b])
        del C0t
    return Xt


def identifiable_plant(M, N, K, seed):
    """Planted factors whose NMF is unique up to permutation and scaling.

    C0 holds the K columns of the identity (scaled) among uniform columns and B0 holds K
    unit rows (scaled) among uniform rows, so the cones generated by B0 and C0 are
    simplicial with extreme rays on the coordinate axes (separability).
    """
    rng = np.random.default_rng(seed)
    B0 = rng.random((M, K))
    C0 = rng.random((K, N))
    B0[:K, :] = np.diag(1.0 + rng.random(K))
    C0[:, :K] = np.diag(1.0 + rng.random(K))
    return B0 @ C0, B0, C0


def to_f32_colmajor(X):
    """float32 Fortran-ordered copy of X: the layout the GPU consumes (ld = M)."""
    return np.asfortranarray(np.asarray(X, dtype=np.float32))


def as_oracle_input(X32):
    """float64 copy of float32 data, so the oracle sees exactly what the GPU sees."""
    return np.asarray(X32, dtype=np.float32).astype(np.float64)


def serving_jobs(n_jobs, seed=5, rate=200.0, M_range=(100, 4000), N_range=(1000, 200000),
                 K_range=(5, 64)):
    """Arrival schedule of the served workload: Poisson arrivals and uneven (M, N, K).

    Returns a list of dicts with arrival time (s), M, N, K and a per-job data seed;
    M ~ U{M_lo..M_hi}, N = round(exp(U[ln N_lo, ln N_hi])), K ~ U{K_lo..K_hi}.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
    Ms = rng.integers(M_range[0], M_range[1] + 1, size=n_jobs)
    Ns = np.rint(np.exp(rng.uniform(np.log(N_range[0]), np.log(N_range[1]), size=n_jobs))).astype(int)
    Ks = rng.integers(K_range[0], K_range[1] + 1, size=n_jobs)
    seeds = rng.integers(0, 2**31 - 1, size=n_jobs)
    return [dict(t=float(t[i]), M=int(Ms[i]), N=int(Ns[i]), K=int(min(Ks[i], Ms[i], Ns[i])),
                 seed=int(seeds[i])) for i in range(n_jobs)]


def serving_x(M, N, K, seed, noise=0.02):
    """One served job's data: X = max(0, B0 C0 + noise N(0,1)) with U[0,1] factors (host)."""
    rng = np.random.default_rng(seed)
    B0 = rng.random((M, K))
    C0 = rng.random((K, N))
    X = B0 @ C0 + noise * rng.standard_normal((M, N))
    return np.maximum(X, 0.0)


def serving_x_device(torch, M, N, K, seed, noise=0.02, device="cuda", generator=None):
    """``serving_x``'s recipe on the device (torch's generator, so other values); returns a
    float32 (N, M) tensor, i.e. X in column-major storage."""
    g = generator
    if g is None:
        g = torch.Generator(device=device)
        g.manual_seed(seed)
    B0t = torch.rand((K, M), generator=g, device=device, dtype=torch.float32)
    C0t = torch.rand((N, K), generator=g, device=device, dtype=torch.float32)
    Xt = torch.matmul(C0t, B0t)
    Xt.add_(torch.randn((N, M), generator=g, device=device, dtype=torch.float32).mul_(noise)).clamp_(min=0.0)
    return Xt


def round_to_bf16(X):
    """Values of bf16(X) (round to nearest even) as float64: the data the reduced-precision
    storage form of X holds.  Finite inputs only (a storage format conversion, done on bits)."""
    x32 = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(x32.shape)
