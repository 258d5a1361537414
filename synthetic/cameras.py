"""Pinhole cameras producing primary rays r(t) = o + t d.

Rays are plain inputs to the renderer: one origin and one unit direction per
pixel, pixel centres at +0.5, square pixels, row-major order (row 0 at the top
of the image). Directions are computed in float64, normalised, then rounded to
float32.
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Camera:
    eye: np.ndarray      # [3]
    target: np.ndarray   # [3]
    up: np.ndarray       # [3]
    width: int
    height: int
    fov_y_deg: float = 60.0


def look_at_camera(eye, target, up, width, height, fov_y_deg=60.0):
    return Camera(np.asarray(eye, np.float64), np.asarray(target, np.float64),
                  np.asarray(up, np.float64), int(width), int(height), float(fov_y_deg))


def pinhole_rays(cam: Camera):
    """Return (origin[h*w,3], dir[h*w,3]) float32 arrays for one camera."""
    fwd = cam.target - cam.eye
    fwd = fwd / np.linalg.norm(fwd)
    right = np.cross(fwd, cam.up)
    right = right / np.linalg.norm(right)
    up = np.cross(right, fwd)
    tan_h = np.tan(np.deg2rad(cam.fov_y_deg) * 0.5)
    aspect = cam.width / cam.height
    xs = (2.0 * (np.arange(cam.width) + 0.5) / cam.width - 1.0) * tan_h * aspect
    ys = (1.0 - 2.0 * (np.arange(cam.height) + 0.5) / cam.height) * tan_h
    X, Y = np.meshgrid(xs, ys)  # [h, w]
    d = fwd[None, None, :] + X[..., None] * right[None, None, :] + Y[..., None] * up[None, None, :]
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    d = d.reshape(-1, 3)
    o = np.broadcast_to(cam.eye, d.shape)
    return (np.ascontiguousarray(o.astype(np.float32)),
            np.ascontiguousarray(d.astype(np.float32)))


def fibonacci_cameras(n, radius, resolutions, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), fov_y_deg=60.0):
    """n cameras at Fibonacci-sphere points of the given radius, looking at target."""
    cams = []
    golden = np.pi * (3.0 - np.sqrt(5.0))
    for i in range(n):
        z = 1.0 - 2.0 * (i + 0.5) / n
        r = np.sqrt(max(0.0, 1.0 - z * z))
        phi = golden * i
        eye = radius * np.array([r * np.cos(phi), r * np.sin(phi), z])
        upv = np.asarray(up, np.float64)
        # keep the view direction away from the up vector
        if abs(np.dot(eye / np.linalg.norm(eye), upv)) > 0.95:
            upv = np.array([0.0, 1.0, 0.0])
        w, h = resolutions[i]
        cams.append(look_at_camera(eye, target, upv, w, h, fov_y_deg))
    return cams


def circle_cameras(n, radius, height, resolution, target=(0.0, 0.0, 0.5), fov_y_deg=60.0):
    """n cameras evenly spaced on a horizontal circle, up = +z."""
    cams = []
    for i in range(n):
        a = 2.0 * np.pi * i / n + 0.25 * np.pi
        eye = np.array([radius * np.cos(a), radius * np.sin(a), height])
        cams.append(look_at_camera(eye, target, (0.0, 0.0, 1.0), resolution[0], resolution[1], fov_y_deg))
    return cams


def concat_rays(cams):
    """Rays of several cameras back to back, plus the per-view table."""
    os, ds, views = [], [], []
    off = 0
    for c in cams:
        o, d = pinhole_rays(c)
        os.append(o)
        ds.append(d)
        views.append((off, c.width, c.height))
        off += o.shape[0]
    return (np.ascontiguousarray(np.concatenate(os)), np.ascontiguousarray(np.concatenate(ds)),
            np.asarray(views, dtype=np.int64))
