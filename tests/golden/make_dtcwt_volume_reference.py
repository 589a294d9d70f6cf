"""Write the FP64 oracle's reference for the DT-CWT shrinkage step on a volume
large enough that the library runs its first level's lateral passes with the
register-window kernels (512 depth x 128 x 128, 2 levels, tau = 0.2).

Input: CN(0, 1) samples from numpy's generator (seed 97), rounded to complex64
(the library's input); the oracle works on those values in FP64.  Stored: z at
2^14 seeded voxels, the norms of its 16 x 16 x 64 (y, x, depth) blocks, a
2^14-bucket CountSketch and ||z|| (refstats.py).  Only the oracle, the seeded
generators and the summary helpers are used.

Run: python tests/golden/make_dtcwt_volume_reference.py   (about 2 minutes)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
import synth  # noqa: E402
import refstats  # noqa: E402

OUT = os.path.join(HERE, "dtcwt_volume_512x128x128.npz")
SHAPE = (1, 128, 128, 512)      # [batch][n_y][n_x][n_depth]
TAU, LEVELS = 0.2, 2
BLOCK = (16, 16, 64)
SAMPLES, SAMPLE_SEED = 1 << 14, 31
SKETCH_BUCKETS, SKETCH_SEED = 1 << 14, 37


def inputs() -> np.ndarray:
    """The seeded input as the library receives it (complex64)."""
    return synth.complex_normal(np.random.default_rng(97), SHAPE).astype(np.complex64)


def main():
    v = inputs().astype(np.complex128)
    z = O.prox_dtcwt(v, TAU, (3, 2, 1), LEVELS)
    idx = refstats.sample_index(z.size, SAMPLES, SAMPLE_SEED)
    np.savez_compressed(
        OUT, tau=TAU, levels=LEVELS, block=np.array(BLOCK), sample_count=SAMPLES, sample_seed=SAMPLE_SEED,
        sketch_buckets=SKETCH_BUCKETS, sketch_seed=SKETCH_SEED,
        zs=z.reshape(-1)[idx], blocks=refstats.block_norms(z, BLOCK),
        sketch=refstats.count_sketch(z, SKETCH_BUCKETS, SKETCH_SEED),
        znorm=float(np.linalg.norm(z.reshape(-1))), vnorm=float(np.linalg.norm(v.reshape(-1))))
    print(f"wrote {OUT}: ||z|| = {np.linalg.norm(z.reshape(-1)):.6f}, ||v|| = {np.linalg.norm(v.reshape(-1)):.6f}")


if __name__ == "__main__":
    main()
