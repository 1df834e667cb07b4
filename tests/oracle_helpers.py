"""Small builders for hand-made scenes used by the oracle pins."""
import numpy as np

import synth


def scene_from(means, scales, quats=None, opac=None, rgb=None, sh=None, degree=0):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    scales = np.asarray(scales, np.float32).reshape(n, 3)
    if quats is None:
        quats = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    quats = np.asarray(quats, np.float32).reshape(n, 4)
    if opac is None:
        opac = np.full(n, 0.5, np.float32)
    opac = np.asarray(opac, np.float32).reshape(n)
    k = (degree + 1) ** 2
    if sh is None:
        sh = np.zeros((n, k, 3), np.float32)
        if rgb is not None:
            # Degree-0 coefficient giving colour rgb: (rgb - 0.5) * 2 sqrt(pi).
            sh[:, 0, :] = (np.asarray(rgb, np.float64).reshape(n, 3) - 0.5) * 2.0 * np.sqrt(np.pi)
    sh = np.asarray(sh, np.float32).reshape(n, k, 3)
    return synth.Scene(means, scales, quats, opac, sh, degree)


def view(w=64, h=64, f=64.0, R=None, t=None, cx=None, cy=None):
    v = synth.identity_view(w, h, f, f)
    if cx is not None:
        v.cx = cx
    if cy is not None:
        v.cy = cy
    if R is not None:
        v.R = np.asarray(R, np.float32)
    if t is not None:
        v.t = np.asarray(t, np.float32)
    return v


def rotation_wxyz(q):
    """Rotation matrix of a (w, x, y, z) quaternion through scipy (x, y, z, w)."""
    from scipy.spatial.transform import Rotation
    q = np.asarray(q, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def pixel_index(v, px, py):
    return np.asarray(py, np.int64) * v.width + np.asarray(px, np.int64)
