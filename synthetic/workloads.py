"""The five measured workloads: scene, cameras and (for the mixed one) a mesh.

Each entry builds lazily because the large scenes take a few seconds to draw.
"""

import numpy as np

from . import scenes, cameras
from .mesh import glass_mesh, mirror_mesh


def _w1():
    sc = scenes.scene_config1()
    cams = [cameras.look_at_camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 64, 64)]
    return dict(name="plain-fwd-1k-64x64", scene=sc, cams=cams)


def _w2():
    sc = scenes.scene_config2()
    cams = [cameras.look_at_camera((0, 0, -4), (0, 0, 0), (0, 1, 0), 800, 800)]
    return dict(name="fwd-bwd-100k-800x800", scene=sc, cams=cams,
                target=scenes.jittered_target(sc, seed=2, sigma=0.01))


def _w3():
    sc = scenes.scene_config3()
    res = [(800, 800)] * 4 + [(400, 300)] * 4
    cams = cameras.fibonacci_cameras(8, 4.0, res)
    return dict(name="batch-300k-8views", scene=sc, cams=cams)


def _w4():
    sc = scenes.scene_config4()
    cams = [cameras.look_at_camera((0, -7, 3.5), (0, 0, 0.5), (0, 0, 1), 1920, 1080)]
    return dict(name="scene-1M-1920x1080", scene=sc, cams=cams)


def _w5():
    sc = scenes.scene_config5()
    cams = cameras.circle_cameras(4, 6.0, 3.0, (1024, 768))
    return dict(name="mesh-500k-4x1024x768", scene=sc, cams=cams, mesh=mirror_mesh(),
                light=np.array([2.0, -2.0, 5.0]))


def _w6():
    sc = scenes.scene_config5()
    cams = cameras.circle_cameras(4, 6.0, 3.0, (1024, 768))
    return dict(name="glass-500k-4x1024x768", scene=sc, cams=cams, mesh=glass_mesh(), bounces=3,
                light=np.array([2.0, -2.0, 5.0]))


WORKLOADS = {1: _w1, 2: _w2, 3: _w3, 4: _w4, 5: _w5, 6: _w6}


def workload(k):
    return WORKLOADS[k]()
