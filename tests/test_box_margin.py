"""The filter's block skip is exact: a block whose box the float32 box test
(the filter's, emulated here in numpy float32 with the same operations in the
same order, no contraction) calls outside a view holds no point that the
per-node float32 frustum test (transform, then z > znear, |x| <= kx z,
|y| <= ky z) lets through. Checked on boxes placed against each frustum
plane, from far inside to far outside, with their corners and random interior
points, for fly-through cameras and a camera at the origin."""
import numpy as np

from paper_2603_23891_amd import synth

f32 = np.float32


def in_frustum32(cam, P):
    R = np.asarray(cam.R, f32).reshape(9)
    t = np.asarray(cam.t, f32)
    mx, my, mz = P[:, 0], P[:, 1], P[:, 2]
    x = ((R[0] * mx + R[1] * my) + R[2] * mz) + t[0]
    y = ((R[3] * mx + R[4] * my) + R[5] * mz) + t[1]
    z = ((R[6] * mx + R[7] * my) + R[8] * mz) + t[2]
    return (z > f32(cam.znear)) & (np.abs(x) <= f32(cam.kx) * z) & (np.abs(y) <= f32(cam.ky) * z)


MARGIN = 1e-5  # the filter's relative margin


def box_outside32(cam, lo, hi):
    with np.errstate(invalid="ignore"):
        return _box_outside32(cam, lo, hi)


def _box_outside32(cam, lo, hi):
    R = np.asarray(cam.R, f32).reshape(9)
    t = np.asarray(cam.t, f32)
    kx, ky, zn = f32(cam.kx), f32(cam.ky), f32(cam.znear)
    h5 = f32(0.5)
    cx, cy, cz = h5 * (lo[:, 0] + hi[:, 0]), h5 * (lo[:, 1] + hi[:, 1]), h5 * (lo[:, 2] + hi[:, 2])
    hx, hy, hz = h5 * (hi[:, 0] - lo[:, 0]), h5 * (hi[:, 1] - lo[:, 1]), h5 * (hi[:, 2] - lo[:, 2])
    S = ((np.abs(cx) + np.abs(cy)) + np.abs(cz)) + ((hx + hy) + hz) + ((np.abs(t[0]) + np.abs(t[1])) + np.abs(t[2]))

    def lmin(a0, a1, a2, b):
        return (((a0 * cx + a1 * cy) + a2 * cz) + b) - ((np.abs(a0) * hx + np.abs(a1) * hy) + np.abs(a2) * hz)

    one, e = f32(1.0), f32(MARGIN)
    mx, my, mz = e * (one + kx) * S, e * (one + ky) * S, e * S
    out = lmin(-R[6], -R[7], -R[8], zn - t[2]) > mz
    out |= lmin(R[0] - kx * R[6], R[1] - kx * R[7], R[2] - kx * R[8], t[0] - kx * t[2]) > mx
    out |= lmin(-R[0] - kx * R[6], -R[1] - kx * R[7], -R[2] - kx * R[8], -t[0] - kx * t[2]) > mx
    out |= lmin(R[3] - ky * R[6], R[4] - ky * R[7], R[5] - ky * R[8], t[1] - ky * t[2]) > my
    out |= lmin(-R[3] - ky * R[6], -R[4] - ky * R[7], -R[5] - ky * R[8], -t[1] - ky * t[2]) > my
    return out


def boxes_against_planes(cam, rng, n):
    """Boxes with a face against one frustum plane: a point on a side plane
    (or the near plane) at a random depth, and a world-axis-aligned box (half-
    extents 1e-4 to 20 world units) placed so that its nearest point lies at
    a signed gap from the plane along the plane's outward normal: within
    float32 rounding of it for a third of the boxes (|gap| from 1e-7 to 1e-3),
    up to 10 units otherwise, inside or outside."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    zs = rng.uniform(0.3, 800.0, n)
    side = rng.integers(0, 5, n)
    u = rng.uniform(-1, 1, n)
    x = np.where(side == 0, cam.kx * zs, np.where(side == 1, -cam.kx * zs, u * cam.kx * zs))
    y = np.where(side == 2, cam.ky * zs, np.where(side == 3, -cam.ky * zs, u * cam.ky * zs))
    z = np.where(side == 4, cam.znear, zs)
    n_cam = np.zeros((n, 3))
    n_cam[side == 0] = (1, 0, -cam.kx)
    n_cam[side == 1] = (-1, 0, -cam.kx)
    n_cam[side == 2] = (0, 1, -cam.ky)
    n_cam[side == 3] = (0, -1, -cam.ky)
    n_cam[side == 4] = (0, 0, -1)
    n_cam /= np.linalg.norm(n_cam, axis=1, keepdims=True)
    n_world = n_cam @ R  # R^T n
    half = 10.0 ** rng.uniform(-4, np.log10(20.0), (n, 3))
    support = (np.abs(n_world) * half).sum(1)
    tight = rng.uniform(0, 1, n) < 1 / 3
    gap = rng.choice([-1, 1], n) * np.where(tight, 10.0 ** rng.uniform(-7, -3, n), 10.0 ** rng.uniform(-3, 1, n))
    pw = (np.stack([x, y, z], 1) - t) @ R + n_world * (support + gap)[:, None]
    return (pw - half).astype(f32), (pw + half).astype(f32)


def check(cam, lo, hi, rng, n_inner=64):
    out = box_outside32(cam, lo, hi)
    idx = np.nonzero(out)[0]
    assert idx.size > 0
    for b in idx:
        corners = np.array([[lo[b, 0] if i & 1 else hi[b, 0], lo[b, 1] if i & 2 else hi[b, 1],
                             lo[b, 2] if i & 4 else hi[b, 2]] for i in range(8)], f32)
        inner = (lo[b] + (hi[b] - lo[b]) * rng.uniform(0, 1, (n_inner, 3))).astype(f32)
        inner = np.clip(inner, lo[b], hi[b])
        pts = np.concatenate([corners, inner])
        assert not in_frustum32(cam, pts).any(), (b, lo[b], hi[b])
    return out.mean()


def test_skipped_boxes_hold_no_point_that_passes():
    rng = np.random.default_rng(7)
    cams = [synth.city20m_frames(64)[k] for k in (0, 13, 32, 51)]
    cams.append(synth.make_camera(np.eye(3), (0.0, 0.0, 0.0), 640, 480))
    fractions = []
    for cam in cams:
        lo, hi = boxes_against_planes(cam, rng, 4000)
        fractions.append(check(cam, lo, hi, rng))
    # the boxes straddle the planes: a good share is skipped, a good share not
    assert all(0.1 < f < 0.9 for f in fractions), fractions


def test_boxes_far_inside_are_never_skipped_and_far_outside_always():
    rng = np.random.default_rng(8)
    cam = synth.city20m_frames(64)[5]
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    z = rng.uniform(5.0, 500.0, 2000)
    pc = np.stack([rng.uniform(-0.5, 0.5, 2000) * cam.kx * z, rng.uniform(-0.5, 0.5, 2000) * cam.ky * z, z], 1)
    pw = (pc - t) @ R
    h = np.full((2000, 3), 0.1)
    assert not box_outside32(cam, (pw - h).astype(f32), (pw + h).astype(f32)).any()
    behind = (np.stack([pc[:, 0], pc[:, 1], -z], 1) - t) @ R
    assert box_outside32(cam, (behind - h).astype(f32), (behind + h).astype(f32)).all()
    nan = np.full((4, 3), np.nan, f32)
    inf = np.array([[-np.inf, 0, 0]] * 4, f32)
    assert not box_outside32(cam, nan, nan).any()
    assert not box_outside32(cam, inf, -inf).any()
