"""Write the FP64 oracle's reference for the full-size B-scan TV reconstruction.

Workload: 2048 spectral pixels x 1000 A-scans, 500 scatterers + 3 layers
(seed 1), exactly half the pixels of each A-scan kept, 1% noise, isotropic TV
with lambda = 0.005 lambda_max, 10 FGP steps, 100 FISTA iterations, step
1 / (1.05 L) from a 50-step power iteration.  Only the oracle, the seeded
generators and the summary helpers are used.  Stores lambda, delta, the
objective history, ||z^100||, z^100 at 2^18 seeded pixels and on the image
border (first and last A-scan, first and last depth row), the norms of its
40 x 64 (lateral x depth) tiles and a 2^16-bucket CountSketch of it
(refstats.py).

Run: python tests/golden/make_bscan_tv_reference.py [threads]
(about 10 minutes on one core)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
import synth  # noqa: E402
import refstats  # noqa: E402

OUT = os.path.join(HERE, "bscan_2048x1000_tv100.npz")
BLOCK = (40, 64)              # (lateral, depth) tile edges of the stored tile norms
SAMPLES, SAMPLE_SEED = 1 << 18, 13
SKETCH_BUCKETS, SKETCH_SEED = 1 << 16, 17


def inputs():
    """The workload's seeded inputs (shared with the GPU test)."""
    pr = synth.preset("bscan_2048x1000_tv")
    g = O.Geometry(**pr["geom"])
    rng = np.random.default_rng(1)
    x_true = synth.scatterers(rng, O.img_shape(g), pr["scatterers"])
    x_true[0, 0] += synth.layers(rng, g.n_depth, g.n_x, pr["layers"])
    mask = synth.mask_random_exact(rng, (1, g.n_x), g.n_k, g.n_k // 2)
    noise = synth.standard_normal(rng, O.meas_shape(g))
    return pr, g, x_true, mask, noise


def measurements(pr, g, x_true, mask, noise):
    """y = s . (Phi x_true + 1% noise), rounded to the float32 the library takes."""
    y = synth.noisy(O.forward(x_true, g, mask), noise, mask, pr["noise"])
    return y.astype(np.float32)


def border(z):
    """z^K on the image border: first and last A-scan, first and last depth row."""
    im = z[0, 0]
    return np.concatenate([im[0], im[-1], im[:, 0], im[:, -1]])


def main():
    if len(sys.argv) > 1:
        O.set_workers(int(sys.argv[1]))
    t0 = time.time()
    pr, g, x_true, mask, noise = inputs()
    y32 = measurements(pr, g, x_true, mask, noise)
    y = y32.astype(np.float64)
    lam = pr["lam"] * O.lambda_max(y, g, mask)
    L = O.lipschitz(g, mask, iters=50, seed=0)
    delta = O.step_size(L)
    print(f"lambda {lam:.6g}  L {L:.6g}  ({time.time() - t0:.0f} s)", flush=True)
    z, hist = O.fista(y, g, mask, O.PEN_TV, lam, delta, pr["iters"], tv_inner=10)
    idx = refstats.sample_index(z.size, SAMPLES, SAMPLE_SEED)
    np.savez(OUT, lam=lam, L=L, delta=delta, hist=hist, ynorm=np.linalg.norm(y),
             sample_count=SAMPLES, sample_seed=SAMPLE_SEED, sketch_buckets=SKETCH_BUCKETS,
             sketch_seed=SKETCH_SEED, block=np.array(BLOCK), znorm=np.linalg.norm(z),
             zs=z.reshape(-1)[idx].astype(np.complex64), border=border(z),
             blocks=refstats.block_norms(z[0, 0], BLOCK),
             sketch=refstats.count_sketch(z, SKETCH_BUCKETS, SKETCH_SEED).astype(np.complex64))
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
