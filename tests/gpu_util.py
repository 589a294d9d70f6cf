"""Helpers shared by the GPU tests: seeded inputs in both precisions."""
import sys

import numpy as np

import oracle as O
import synth


def flush(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def both_geoms(**kw):
    """(oracle Geometry, library Geometry) with the same fields."""
    import paper_2108_01438_amd as P
    return O.Geometry(**kw), P.Geometry(**kw)


def rand_image(rng, shape):
    x = synth.complex_normal(rng, shape).astype(np.complex64)
    return x, x.astype(np.complex128)


def rand_meas(rng, shape):
    r = rng.standard_normal(shape).astype(np.float32)
    return r, r.astype(np.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()
