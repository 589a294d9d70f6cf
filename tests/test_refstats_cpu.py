"""The summaries that stand in for full-size stored references
(tests/golden/refstats.py): the CountSketch estimates the L2 norm of a
difference over the whole image, including an error confined to one tile,
and the block norms localise it."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import refstats  # noqa: E402


def _img(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_sketch_is_linear_and_estimates_the_difference_norm():
    rng = np.random.default_rng(3)
    a, b = _img(rng, (1000, 2048)), _img(rng, (1000, 2048))
    sa = refstats.count_sketch(a, 1 << 16, 17)
    sb = refstats.count_sketch(b, 1 << 16, 17)
    np.testing.assert_allclose(refstats.count_sketch(a + 2 * b, 1 << 16, 17), sa + 2 * sb, atol=1e-9)
    d = 1e-6 * b
    est = np.linalg.norm(refstats.count_sketch(a + d, 1 << 16, 17) - sa) / np.linalg.norm(d)
    assert abs(est - 1) < 0.03


def test_localised_error_seen_by_sketch_and_blocks():
    rng = np.random.default_rng(4)
    z = _img(rng, (1000, 2048))
    e = np.zeros_like(z)
    e[400:440, 1024:1088] = 1e-3 * _img(rng, (40, 64))       # one 40 x 64 tile
    est = np.linalg.norm(refstats.count_sketch(e, 1 << 16, 17)) / np.linalg.norm(e)
    assert 0.9 < est < 1.1
    bz, bze = refstats.block_norms(z, (40, 64)), refstats.block_norms(z + e, (40, 64))
    changed = np.argwhere(np.abs(bze - bz) > 1e-9 * bz)
    assert changed.tolist() == [[10, 16]]


def test_compare_reports_zero_for_the_reference_itself():
    rng = np.random.default_rng(5)
    z = _img(rng, (64, 256))
    ref = {"sample_count": 512, "sample_seed": 1, "sketch_buckets": 1024, "sketch_seed": 2}
    idx = refstats.sample_index(z.size, 512, 1)
    ref.update(zs=z.reshape(-1)[idx], blocks=refstats.block_norms(z, (16, 64)),
               sketch=refstats.count_sketch(z, 1024, 2), znorm=np.linalg.norm(z))
    err = refstats.compare(z, ref, "", (16, 64))
    assert max(err.values()) < 1e-14
    err = refstats.compare(z * (1 + 1e-5), ref, "", (16, 64))
    sk = err.pop("whole_sketch")          # an estimate: 1024 buckets -> ~4% spread
    assert all(abs(v - 1e-5) < 1e-7 for v in err.values())
    assert abs(sk - 1e-5) < 2e-6
