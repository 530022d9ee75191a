"""Independent float64 geometry used to pin the oracle.

Rotation matrices come from scipy (not from a quaternion formula), the
pinhole Jacobian from central differences of the projection map (not from
its closed form), and eigenvalues from numpy.linalg. Nothing here is shared
with the oracle or the HIP path.
"""
import numpy as np
from scipy.spatial.transform import Rotation


def world_to_cam(cam):
    return np.asarray(cam.R, np.float64).reshape(3, 3), np.asarray(cam.t, np.float64)


def project(cam, pc):
    return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])


def sigma3d(scale, quat_wxyz):
    rot = Rotation.from_quat([quat_wxyz[1], quat_wxyz[2], quat_wxyz[3], quat_wxyz[0]]).as_matrix()
    return rot @ np.diag(np.asarray(scale, np.float64) ** 2) @ rot.T


def gaussian2d(tree, cam, i):
    """(pc, uv, Sigma_2D incl. 0.3 dilation) for node i, float64."""
    W, t = world_to_cam(cam)
    mu = tree.mean[:, i].astype(np.float64)
    pc = W @ mu + t
    S = sigma3d(tree.scale[:, i].astype(np.float64), tree.quat[:, i].astype(np.float64))
    h = 1e-4 * abs(pc[2])
    J = np.stack([(project(cam, pc + h * e) - project(cam, pc - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    S2 = J @ W @ S @ W.T @ J.T + 0.3 * np.eye(2)
    return pc, project(cam, pc), S2


def radius3(tree, cam, i):
    _, _, S2 = gaussian2d(tree, cam, i)
    return 3.0 * np.sqrt(np.linalg.eigvalsh(S2).max())


def in_frustum(tree, cam, i):
    W, t = world_to_cam(cam)
    pc = W @ tree.mean[:, i].astype(np.float64) + t
    return pc[2] > cam.znear and abs(pc[0]) <= cam.kx * pc[2] and abs(pc[1]) <= cam.ky * pc[2], pc
