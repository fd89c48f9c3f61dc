"""Seeded synthetic inputs for the partitioned-reduction workloads.

This module only draws random numbers and sizes.  It holds none of the
reduction's arithmetic, no codec and no partitioning rule, so that the GPU
path and the CPU oracle can both be fed from it without sharing any code.

Workloads (one seed per workload: SEED + its number):
  1 plain       4 ranks, FP32, 262144 elements per rank, uniform [-1, 1),
                8 partitions readied in order.
  2 sweep       8 ranks, FP32, 2^k elements per rank (k = 0..26), N(0, 1),
                partition counts {1, 4, 16, 64}, a seeded random arrival order.
  3 batched     8 ranks, 64 buckets of log-uniform byte sizes in
                [64 KiB, 64 MiB], BF16 payload drawn as FP32 N(0, 1e-3)
                (standard deviation 1e-3), 32 partitions per bucket.
  4 integer     16 ranks, int32, 2^24 elements per rank, uniform integers in
                [-2^20, 2^20], 256 partitions in a seeded random order.
  5 fp8         8 ranks, 128 buckets totalling 2^30 elements per rank,
                log-uniform sizes, FP32 N(0, 1e-2) with each element an
                outlier at 50x its draw with probability 0.01.

Tensors are drawn with torch generators (CPU or GPU, the caller picks);
sizes and permutations with numpy's default_rng.  Ranks are drawn in order
r = 0..P-1 from one generator.
"""
import math

import numpy as np
import torch

SEED = 22228


def seed_for(workload):
    return SEED + int(workload)


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def uniform_f32(nranks, n, seed, device="cpu", lo=-1.0, hi=1.0):
    g = _gen(seed, device)
    out = []
    for _ in range(nranks):
        t = torch.rand(n, generator=g, device=device, dtype=torch.float32)
        out.append(t * (hi - lo) + lo)
    return out


def normal_f32(nranks, n, seed, std=1.0, device="cpu"):
    g = _gen(seed, device)
    return [torch.randn(n, generator=g, device=device, dtype=torch.float32)
            * std for _ in range(nranks)]


def normal_with_outliers_f32(nranks, n, seed, std, p_out=0.01, factor=50.0,
                             device="cpu"):
    """N(0, std) draws; each element independently becomes an outlier with
    probability p_out, its value multiplied by `factor`."""
    g = _gen(seed, device)
    out = []
    for _ in range(nranks):
        x = torch.randn(n, generator=g, device=device, dtype=torch.float32)
        m = torch.rand(n, generator=g, device=device) < p_out
        x = x * std
        x = torch.where(m, x * factor, x)
        out.append(x)
    return out


def uniform_i32(nranks, n, seed, lo, hi, device="cpu"):
    """Integers uniform on [lo, hi] inclusive."""
    g = _gen(seed, device)
    return [torch.randint(lo, hi + 1, (n,), generator=g, device=device,
                          dtype=torch.int32) for _ in range(nranks)]


def random_bits(nranks, n, seed, dtype, device="cpu"):
    """Uniformly random raw codes (uint8 / int16 views) for codec tests."""
    g = _gen(seed, device)
    if dtype == torch.uint8:
        return [torch.randint(0, 256, (n,), generator=g, device=device,
                              dtype=torch.uint8) for _ in range(nranks)]
    return [torch.randint(-32768, 32768, (n,), generator=g, device=device,
                          dtype=torch.int16) for _ in range(nranks)]


# Raw bit patterns of special values: quiet and signalling NaNs of both
# signs with and without payload, infinities, signed zeros, the largest
# finite magnitudes (whose sums overflow) and the smallest subnormals.
F32_SPECIAL_BITS = (0x7FC00000, 0xFFC00001, 0x7F800001, 0xFFA00000,
                    0x7F800000, 0xFF800000, 0x00000000, 0x80000000,
                    0x7F7FFFFF, 0xFF7FFFFF, 0x00000001, 0x80000001)
BF16_SPECIAL_CODES = (0x7FC0, 0xFFC1, 0x7F81, 0xFFA0, 0x7F80, 0xFF80,
                      0x0000, 0x8000, 0x7F7F, 0xFF7F, 0x0001, 0x8001)


def bf16_codes(nranks, n, seed, exp_lo=112, exp_hi=135, device="cpu"):
    """Random bfloat16 codes (int16 views): random sign and 7 fraction
    bits, biased exponent uniform on [exp_lo, exp_hi] (finite normals)."""
    g = _gen(seed, device)
    out = []
    for _ in range(nranks):
        sign = torch.randint(0, 2, (n,), generator=g, device=device,
                             dtype=torch.int32)
        ex = torch.randint(exp_lo, exp_hi + 1, (n,), generator=g,
                           device=device, dtype=torch.int32)
        fr = torch.randint(0, 128, (n,), generator=g, device=device,
                           dtype=torch.int32)
        code = (sign << 15) | (ex << 7) | fr
        out.append(torch.where(code >= 32768, code - 65536, code)
                   .to(torch.int16))
    return out


def plant_specials(codes, seed, specials, density=0.05, zero_cols=0.02):
    """Copies of the raw-bit tensors `codes` (int32 or int16 views, one per
    rank) in which each element is independently replaced, with
    probability `density`, by a pattern drawn from `specials`, and a
    fraction `zero_cols` of the element positions hold +0 or -0 (drawn per
    rank) in every rank."""
    g = _gen(seed, codes[0].device)
    n = codes[0].numel()
    bits = 32 if codes[0].dtype == torch.int32 else 16
    pats = torch.tensor([v - (1 << bits) if v >= 1 << (bits - 1) else v
                         for v in specials], dtype=codes[0].dtype,
                        device=codes[0].device)
    zcol = torch.rand(n, generator=g, device=codes[0].device) < zero_cols
    neg0 = torch.tensor(-(1 << (bits - 1)), dtype=codes[0].dtype,
                        device=codes[0].device)
    out = []
    for c in codes:
        hit = torch.rand(n, generator=g, device=c.device) < density
        pick = torch.randint(0, len(specials), (n,), generator=g,
                             device=c.device)
        v = torch.where(hit, pats[pick], c)
        zsign = torch.rand(n, generator=g, device=c.device) < 0.5
        zero = torch.where(zsign, neg0, torch.zeros_like(neg0))
        out.append(torch.where(zcol, zero, v))
    return out


def permutation(n, seed):
    return np.random.default_rng(int(seed)).permutation(int(n))


def log_uniform_bytes(nbuckets, lo_bytes, hi_bytes, seed):
    """Bucket sizes S_b = exp(U(ln lo, ln hi)) bytes, floored to integers."""
    rng = np.random.default_rng(int(seed))
    u = rng.uniform(math.log(lo_bytes), math.log(hi_bytes), size=nbuckets)
    return [int(math.floor(math.exp(v))) for v in u]


def batched_bf16_counts(seed=None, nbuckets=64, lo=1 << 16, hi=1 << 26):
    """Element counts of the batched BF16 workload: floor(S_b / 2)."""
    seed = seed_for(3) if seed is None else seed
    return [b // 2 for b in log_uniform_bytes(nbuckets, lo, hi, seed)]


def fp8_bucket_counts(seed=None, nbuckets=128, total=1 << 30,
                      lo=1 << 16, hi=1 << 26, block=256):
    """Counts of the FP8 workload: log-uniform weights on [lo, hi], scaled to
    `total` elements, each floored to a multiple of `block`, remainder to the
    last bucket."""
    seed = seed_for(5) if seed is None else seed
    rng = np.random.default_rng(int(seed))
    w = np.exp(rng.uniform(math.log(lo), math.log(hi), size=nbuckets))
    raw = w / w.sum() * total
    counts = [int(c) // block * block for c in raw]
    counts[-1] += total - sum(counts)
    return counts
