"""Write the FP64 oracle's reference for the full-size volume reconstruction.

Workload: 2048 spectral pixels x 256 x 256 A-scans (2-D lateral transform),
5000 on-grid scatterers in a smooth random background (seed 2), every pixel
observed, 3-level 3-D Haar l1 with lambda = 0.01 lambda_max, 50 FISTA
iterations, step 1 / (1.05 L) from a 50-step power iteration; once with 1%
noise and once noise-free.  Only the oracle, the seeded generators and the
summary helpers are used.

Stored per run (prefix "noisy_" / "clean_"): lambda, the objective history,
||z^50||, z^50 at 2^16 seeded voxels, the norms of its 64 x 16 x 16 blocks and
a 2^16-bucket CountSketch of it (refstats.py); plus L, delta and the norms of
the float32 measurements the library is given.

Run: python tests/golden/make_volume_haar_reference.py [threads]
(about 4 hours with 8 threads; ~25 GB of host memory)
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

OUT = os.path.join(HERE, "volume_2048x256x256_haar50.npz")
PRESET = "volume_2048x256x256_haar"
BLOCK = (16, 16, 64)          # (y, x, depth) block edges of the stored block norms
SAMPLES, SAMPLE_SEED = 1 << 16, 23
SKETCH_BUCKETS, SKETCH_SEED = 1 << 16, 29


def inputs():
    """The workload's seeded inputs (shared with the GPU test): the specimen
    (complex128, (1, 256, 256, 2048)) and the unit noise (float64)."""
    pr = synth.preset(PRESET)
    g = O.Geometry(**pr["geom"])
    rng = np.random.default_rng(2)
    shape = O.img_shape(g)
    x = synth.scatterers(rng, shape, pr["scatterers"])
    # background RMS: 5% of the mean scatterer amplitude (U(0.5, 1) -> 0.75)
    x[0] += synth.smooth_field_coarse(rng, shape[1:], 16, pr["field"] * 0.75)
    noise = synth.standard_normal(rng, O.meas_shape(g))
    return pr, g, x, noise


def measurements(pr, g, x, noise):
    """(noisy, clean) float32 measurements: Phi x + 1% noise, and Phi x."""
    yc = O.forward(x, g)
    yn = synth.noisy(yc, noise, None, pr["noise"]).astype(np.float32)
    return yn, yc.astype(np.float32)


def summarise(z, prefix):
    idx = refstats.sample_index(z.size, SAMPLES, SAMPLE_SEED)
    return {prefix + "znorm": float(np.linalg.norm(z.reshape(-1))),
            prefix + "zs": z.reshape(-1)[idx].astype(np.complex64),
            prefix + "blocks": refstats.block_norms(z[0], BLOCK),
            prefix + "sketch": refstats.count_sketch(z, SKETCH_BUCKETS, SKETCH_SEED).astype(np.complex64)}


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    O.set_workers(threads)
    t0 = time.time()
    pr, g, x, noise = inputs()
    yn, yc = measurements(pr, g, x, noise)
    del x, noise
    print(f"measurements ({time.time() - t0:.0f} s)", flush=True)
    L = O.lipschitz(g, None, iters=50, seed=0)
    delta = O.step_size(L)
    out = dict(L=L, delta=delta, iters=pr["iters"], sample_count=SAMPLES, sample_seed=SAMPLE_SEED,
               sketch_buckets=SKETCH_BUCKETS, sketch_seed=SKETCH_SEED, block=np.array(BLOCK))
    print(f"L {L:.8g} ({time.time() - t0:.0f} s)", flush=True)
    for tag, y32 in (("noisy_", yn), ("clean_", yc)):
        y = y32.astype(np.float64)
        out[tag + "ynorm"] = float(np.linalg.norm(y))
        lam = pr["lam"] * O.lambda_max(y, g)
        z, hist = O.fista(y, g, None, O.PEN_HAAR, lam, delta, pr["iters"], haar_levels=3)
        out[tag + "lam"] = lam
        out[tag + "hist"] = hist
        out.update(summarise(z, tag))
        np.savez(OUT, **out)
        print(f"{tag} done: lambda {lam:.6g}, objective {hist[0]:.6g} -> {hist[-1]:.6g} "
              f"({time.time() - t0:.0f} s)", flush=True)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
