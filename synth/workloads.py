"""The benchmark workloads as data: frame shapes, sample counts, window radii, seeds.

Every workload uses the recipe of :mod:`synth` with seed ``seed`` for the frames and
``seed + 1000`` for the 4096-spp reference, lambda from seed 99 on a 20 x 20 grid, and
max_lag 8.
"""

from typing import List, NamedTuple


class FrameSpec(NamedTuple):
    W: int
    H: int
    S: int
    radius: int
    seed: int
    frame: int = 0
    fp16_features: bool = False


N_REGIONS = 20
MAX_LAG = 8
LAMBDA_SEED = 99
REFERENCE_SPP = 4096

# 128 x 128, 16 spp, constant noise sigma 0.1, 7 x 7 window, forward only
SMALL = FrameSpec(128, 128, 16, 3, seed=1)
# 1920 x 1080, 64 spp, per-pixel noise scale in [0.02, 0.5], 11 x 11 window (forward; and
# forward + backward against the reference)
HD = FrameSpec(1920, 1080, 64, 5, seed=2)
# 3840 x 2160, 256 spp, FP16-stored features, 15 x 15 window, forward + backward
UHD = FrameSpec(3840, 2160, 256, 7, seed=5, fp16_features=True)

# 32 frames of uneven size and sample count in one batch, 11 x 11 window, forward + backward
LADDER = [(256, 256), (512, 512), (640, 480), (800, 600), (1024, 576), (1280, 720), (1600, 900),
          (1920, 1080), (2048, 1152)]
LADDER_SPP = [4, 16, 64, 256]


def batch32(seed: int = 4) -> List[FrameSpec]:
    """Frame i: shape LADDER[(5 i + 2) mod 9], spp LADDER_SPP[i mod 4], frame counter i."""
    out = []
    for i in range(32):
        W, H = LADDER[(5 * i + 2) % len(LADDER)]
        out.append(FrameSpec(W, H, LADDER_SPP[i % len(LADDER_SPP)], 5, seed=seed, frame=i))
    return out


def sample_bytes(spec: FrameSpec) -> int:
    """Bytes of the sample planes of one frame: 3 fp32 radiance + 7 feature planes."""
    return spec.W * spec.H * spec.S * (3 * 4 + 7 * (2 if spec.fp16_features else 4))


# Quadtree partitions (Sec. 6.1-6.3 with the parameters of Sec. 8.1: M_split = 5000,
# M_refine = 1e7): the forest grows over `rounds` refinements, each after a batch of
# `grow_points` lookups (batch 0 of the point recipe, the chains' stationary distribution
# sampled once and revisited), then `lookup_points` lookups (batch 1) are timed.
# 2-D: one tree over the screen; 4-D: one tree per cell of the 20 x 20 screen grid.
QUADTREE_2D = dict(n_roots=1, capacity=1 << 16, m_split=5000, grow_points=10_000_000, rounds=8,
                   lookup_points=1 << 24, seed=31)
QUADTREE_4D = dict(n_roots=N_REGIONS * N_REGIONS, capacity=1 << 16, m_split=5000, grow_points=10_000_000,
                   rounds=8, lookup_points=1 << 24, seed=32)
