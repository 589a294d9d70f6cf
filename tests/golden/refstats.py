"""Summaries of a large reconstruction that a stored reference can hold and a
test can recompute from a candidate image of the same shape.

* sample_index: seeded flat positions (without replacement) for an
  element-by-element comparison.
* block_norms: the L2 norm of every block of a regular tiling of the image
  (localised errors, e.g. at seams or borders, show up in one block).
* count_sketch: a CountSketch of the flattened image, c[b] = sum over the
  elements i hashed to bucket b of sign(i) z_i.  It is linear, so
  ||sketch(z1) - sketch(z2)|| estimates ||z1 - z2|| over the whole image
  (the squared norm is unbiased with a relative standard deviation of at most
  sqrt(2 / buckets), 0.55% for 2^16 buckets).

Test infrastructure: holds no arithmetic of the reconstruction method.
"""
import numpy as np

SKETCH_CHUNK = 1 << 22


def sample_index(n: int, count: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(n, size=count, replace=False))


def block_norms(z: np.ndarray, block) -> np.ndarray:
    """z: (..., A, B[, C]) image; block: the block edge along each of the last
    len(block) axes (each must divide the axis).  Returns the per-block L2
    norms, shape (..., A/a, B/b[, C/c])."""
    z = np.asarray(z)
    nd = len(block)
    lead = z.shape[:-nd]
    shp = list(lead)
    for s, b in zip(z.shape[-nd:], block):
        assert s % b == 0, "block must divide the image"
        shp += [s // b, b]
    a = np.abs(z.reshape(shp)).astype(np.float64) ** 2
    axes = tuple(len(lead) + 2 * i + 1 for i in range(nd))
    return np.sqrt(a.sum(axis=axes))


def count_sketch(z: np.ndarray, buckets: int, seed: int) -> np.ndarray:
    """CountSketch of z.ravel() into `buckets` complex bins (hashes and signs
    drawn per fixed-size chunk from numpy's seeded generator)."""
    flat = np.asarray(z).reshape(-1)
    out = np.zeros(buckets, dtype=np.complex128)
    for c, a in enumerate(range(0, flat.size, SKETCH_CHUNK)):
        b = min(flat.size, a + SKETCH_CHUNK)
        rng = np.random.default_rng([seed, c])
        h = rng.integers(0, buckets, size=b - a)
        s = rng.integers(0, 2, size=b - a).astype(np.float64) * 2.0 - 1.0
        v = flat[a:b].astype(np.complex128)
        out += np.bincount(h, weights=s * v.real, minlength=buckets)
        out += 1j * np.bincount(h, weights=s * v.imag, minlength=buckets)
    return out


def compare(z: np.ndarray, ref: dict, prefix: str, block) -> dict:
    """Relative errors of candidate z against the stored summaries
    ref[prefix + 'zs' | 'blocks' | 'sketch' | 'znorm'] (positions from
    ref['sample_seed'] / ref['sample_count'], sketch from ref['sketch_seed'])."""
    z = np.asarray(z)
    idx = sample_index(z.size, int(ref["sample_count"]), int(ref["sample_seed"]))
    zs = z.reshape(-1)[idx].astype(np.complex128)
    ref_zs = ref[prefix + "zs"].astype(np.complex128)
    bn = block_norms(z, block)
    ref_bn = ref[prefix + "blocks"]
    sk = count_sketch(z, int(ref["sketch_buckets"]), int(ref["sketch_seed"]))
    ref_sk = ref[prefix + "sketch"].astype(np.complex128)
    zn = float(np.linalg.norm(z.reshape(-1).astype(np.complex128)))
    return {
        "samples": float(np.linalg.norm(zs - ref_zs) / np.linalg.norm(ref_zs)),
        "samples_max": float(np.max(np.abs(zs - ref_zs)) / np.max(np.abs(ref_zs))),
        # per-block norm error relative to the block's own norm, floored at 1%
        # of the RMS block norm (blocks the penalty has nearly emptied)
        "blocks": float(np.max(np.abs(bn - ref_bn) / np.maximum(ref_bn, 0.01 * np.sqrt(np.mean(ref_bn ** 2))))),
        "whole_sketch": float(np.linalg.norm(sk - ref_sk) / float(ref[prefix + "znorm"])),
        "norm": abs(zn - float(ref[prefix + "znorm"])) / float(ref[prefix + "znorm"]),
    }
