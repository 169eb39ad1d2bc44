"""Small hand-built scenes shared by the oracle pins (inputs only)."""
import numpy as np

import scenegen as sg


def axis_camera(width=9, height=9, f=10.0):
    """Camera at the origin looking down +z (R = I, t = 0), principal point at the
    image centre, so a Gaussian on the z axis projects onto (W/2, H/2)."""
    return sg.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f,
                     width / 2.0, height / 2.0, width, height)


def gaussians(means, log_scale, opacities, quats=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    ls = np.broadcast_to(np.asarray(log_scale, np.float32), (n, 3)).copy() \
        if np.ndim(log_scale) <= 1 else np.asarray(log_scale, np.float32)
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)) if quats is None \
        else np.asarray(quats, np.float32)
    return sg.Gaussians(means, ls, q, np.asarray(opacities, np.float32).reshape(n))


def views_for(cams, maps, code_idx, code_val, m):
    base = [0]
    for mp in maps:
        base.append(base[-1] + int(mp.max()) + 1)
    return sg.Views(list(cams), list(maps), np.asarray(base, np.int64),
                    np.asarray(code_idx, np.int32), np.asarray(code_val, np.float32), m)


def small_scene(seed, n=40, res=(16, 12), n_views=2, m=8, k=3, sites=3, iso=False, holes=0):
    """A tiny anisotropic scene in the unit cube seen from a circle of radius 3."""
    g = sg.make_gaussians(seed, n, (0.5, 0.5, 0.5), -3.2, 0.4, iso, "uniform")
    cams = sg.circle_cameras(n_views, 3.0, res[0], res[1], 60.0)
    v = sg.make_views(seed + 7, cams, sites, m, k, hole_sites=holes)
    return g, v
