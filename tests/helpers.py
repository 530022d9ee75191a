"""Shared test-side constructors (inputs only; no method arithmetic)."""
import numpy as np

from paper_2603_23891_amd import synth


def flat_tree(mean, scale, quat, opacity, sh, sh_degree=None):
    """Every Gaussian its own root leaf (no hierarchy)."""
    mean = np.asarray(mean, np.float32).reshape(-1, 3)
    n = mean.shape[0]
    sh = np.asarray(sh, np.float32).reshape(n, -1, 3)
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[sh.shape[1]] if sh_degree is None else sh_degree
    return synth.Tree(mean=mean.T.copy(), scale=np.asarray(scale, np.float32).reshape(n, 3).T.copy(),
                      quat=np.asarray(quat, np.float32).reshape(n, 4).T.copy(),
                      opacity=np.asarray(opacity, np.float32).reshape(n), sh=sh,
                      parent=np.full(n, -1, np.int32), flags=np.ones(n, np.uint8), sh_degree=deg,
                      n_internal_span=0, max_depth=0, level_sizes=[n])


def random_flat(rng, n, cam, depth=(3.0, 30.0), log_s=(-1.5, 0.7), sh_degree=3):
    """n random Gaussians inside the camera's view."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    z = rng.uniform(*depth, n)
    x = rng.uniform(-0.5, 0.5, n) * z * (cam.width / cam.fx)
    y = rng.uniform(-0.5, 0.5, n) * z * (cam.height / cam.fy)
    pc = np.stack([x, y, z], 1)
    mean = (pc - np.asarray(cam.t, np.float64)) @ R  # R^T (pc - t)
    scale = np.exp(rng.normal(log_s[0], log_s[1], (n, 3)))
    q = rng.standard_normal((n, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = 1.0 / (1.0 + np.exp(-rng.normal(0, 1.5, n)))
    K = (sh_degree + 1) ** 2
    sh = rng.normal(0, 0.3, (n, K, 3))
    return flat_tree(mean, scale, q, op, sh, sh_degree)


def splat_array(rows):
    """Build an oracle splat array from dicts (missing fields are zero)."""
    import oracle
    a = np.zeros(len(rows), oracle.SPLAT_DTYPE)
    for i, r in enumerate(rows):
        for k, v in r.items():
            a[i][k] = v
    return a
