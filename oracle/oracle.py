"""ctypes wrapper of the FP64 CPU oracle (rs_oracle.c, rs_oracle_bvh.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark; never by the product path. Builds its shared
library with gcc on first use (or via build()).
"""

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("rs_oracle.c", "rs_oracle_bvh.c", "rs_oracle_mesh.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Defaults (the paper fixes none): Q = chi^2(3) 0.99 quantile, eps1 = 1e-4, K_max = 512.
Q_DEFAULT = 11.3449
EPS1_DEFAULT = 1e-4
KMAX_DEFAULT = 512


def build(force=True):
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared", "-fPIC",
           "-Wall", "-o", _LIB_PATH + ".tmp"] + _SRCS + ["-lm"]
    if force or not os.path.exists(_LIB_PATH) or any(os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SRCS):
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("Q", C.c_double), ("eps1", C.c_double), ("t_min", C.c_double), ("max_hits", C.c_int64),
                ("bg", C.c_double * 3), ("zero_colour", C.c_int32)]


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("rgb", C.c_void_p)]


class _Rays(C.Structure):
    _fields_ = [("n", C.c_int64), ("origin", C.c_void_p), ("dir", C.c_void_p), ("t_max", C.c_void_p),
                ("bg", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        # RS_ORACLE_LIB names another build of the same sources (the sanitizer test's)
        path = os.environ.get("RS_ORACLE_LIB")
        if not path:
            build(force=False)
        L = C.CDLL(path or _LIB_PATH)
        P = C.c_void_p
        L.orc_version.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_rotation.argtypes = [P, P]
        L.orc_rotation_derivs.argtypes = [P, P]
        L.orc_intersect.argtypes = [P, C.c_int64, P, P, C.c_double, C.c_double, P, P]
        L.orc_intersect.restype = C.c_int
        L.orc_ray_hits.argtypes = [P, P, C.c_int64, P, C.c_int64, P, P, P, P]
        L.orc_ray_hits.restype = C.c_int64
        L.orc_render_fwd.argtypes = [P, P, P, P, P, P, C.c_int]
        L.orc_render_lists.argtypes = [P, P, P, C.c_int64, P, P, C.c_int]
        L.orc_render_bwd.argtypes = [P, P, P, P, P, P, P, P, P, P, C.c_int]
        L.orc_render_bwd_paper.argtypes = [P, P, P, C.c_double, P, P, P, P, P, P, P, P, C.c_int]
        L.orc_ray_dC_dalpha.argtypes = [P, P, C.c_int64, P, C.c_int64, P]
        L.orc_ray_dC_dalpha.restype = C.c_int64
        L.orc_ray_alternatives.argtypes = [P, P, C.c_int64, P, C.c_double, C.c_double, C.c_double, C.c_int,
                                           C.c_int64, P]
        L.orc_ray_alternatives.restype = C.c_int64
        L.orc_alternatives_batch.argtypes = [P, P, P, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int64, P, P,
                                             C.c_int]
        L.orc_morton_codes.argtypes = [C.c_int64, P, P, P, P]
        L.orc_sort_codes.argtypes = [C.c_int64, P, P, P]
        L.orc_radix_tree.argtypes = [C.c_int64, P, P, P]
        L.orc_leaf_boxes.argtypes = [C.c_int64, P, P, P, C.c_float, P, P]
        L.orc_ploc.argtypes = [C.c_int64, P, P, P]
        L.orc_ploc.restype = C.c_int64
        L.orc_ploc_cap.argtypes = [C.c_int64]
        L.orc_ploc_cap.restype = C.c_int64
        L.orc_mesh_closest.argtypes = [C.c_int64, P, P, C.c_int64, P, P, C.c_double, P, P, C.c_double, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c32(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


class Params:
    """Renderer knobs of the paper (Q, K_max, eps1) plus background and t_min."""

    def __init__(self, Q=Q_DEFAULT, eps1=EPS1_DEFAULT, t_min=0.0, max_hits=KMAX_DEFAULT, bg=(0.0, 0.0, 0.0),
                 zero_colour=False):
        self.Q, self.eps1, self.t_min, self.max_hits = float(Q), float(eps1), float(t_min), int(max_hits)
        self.bg = tuple(float(x) for x in bg)
        self.zero_colour = bool(zero_colour)

    def c(self):
        p = _Params()
        p.Q, p.eps1, p.t_min, p.max_hits = self.Q, self.eps1, self.t_min, self.max_hits
        for k in range(3):
            p.bg[k] = self.bg[k]
        p.zero_colour = int(self.zero_colour)
        return p


class _Bound:
    """Keeps numpy arrays alive while their pointers sit in ctypes structs."""

    def __init__(self, scene, origin, direction, t_max=None, bg=None):
        self.keep = [_c32(a) for a in scene.arrays()]
        self.sc = _Scene(scene.n, *[_ptr(a) for a in self.keep])
        self.o = _c32(origin).reshape(-1, 3)
        self.d = _c32(direction).reshape(-1, 3)
        self.tm = None if t_max is None else np.ascontiguousarray(t_max, dtype=np.float64)
        self.bg = None if bg is None else np.ascontiguousarray(bg, dtype=np.float64).reshape(-1, 3)
        self.rays = _Rays(self.o.shape[0], _ptr(self.o), _ptr(self.d), _ptr(self.tm), _ptr(self.bg))


def render_fwd(scene, origin, direction, params=None, t_max=None, bg=None, threads=0):
    """Returns (rgb[n,3] f64, T_final[n] f64, L[n] int64)."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max, bg)
    n = b.o.shape[0]
    out = np.zeros((n, 3), np.float64)
    T = np.zeros(n, np.float64)
    L = np.zeros(n, np.int64)
    p = params.c()
    lib().orc_render_fwd(C.byref(b.sc), C.byref(b.rays), C.byref(p), _ptr(out), _ptr(T), _ptr(L), int(threads))
    return out, T, L


def render_lists(scene, origin, direction, params=None, cap=512, t_max=None, bg=None, threads=0):
    """The composited hits of every ray in compositing order: (ids[n, cap] int64
    with -1 after the first min(L, cap), L[n] int64)."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max, bg)
    n = b.o.shape[0]
    ids = np.zeros((n, max(int(cap), 1)), np.int64)
    L = np.zeros(n, np.int64)
    p = params.c()
    lib().orc_render_lists(C.byref(b.sc), C.byref(b.rays), C.byref(p), int(max(cap, 1)), _ptr(ids), _ptr(L),
                           int(threads))
    return ids, L


def render_bwd(scene, origin, direction, grad_rgb, params=None, t_max=None, bg=None, threads=0, want_bg=False):
    """Gradients of sum <grad_rgb, C> w.r.t. mean, scale, quat, opacity, rgb (FP64)."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max, bg)
    n = scene.n
    g = np.ascontiguousarray(grad_rgb, dtype=np.float64).reshape(-1, 3)
    dm = np.zeros((n, 3)); ds = np.zeros((n, 3)); dq = np.zeros((n, 4)); do = np.zeros(n); dc = np.zeros((n, 3))
    dbg = np.zeros((b.o.shape[0], 3)) if want_bg else None
    p = params.c()
    lib().orc_render_bwd(C.byref(b.sc), C.byref(b.rays), C.byref(p), _ptr(g), _ptr(dm), _ptr(ds), _ptr(dq),
                         _ptr(do), _ptr(dc), _ptr(dbg), int(threads))
    grads = dict(mean=dm, scale=ds, quat=dq, opacity=do, rgb=dc)
    if want_bg:
        grads["bg"] = dbg
    return grads


def render_bwd_paper(scene, origin, direction, grad_rgb, params=None, eps2=1e-4, t_max=None, bg=None, threads=0):
    """The paper's backward variant with the second threshold eps2 (see
    orc_render_bwd_paper). Returns (grads, extra[n] second-phase hits per ray,
    near[n] rays with an eps2 decision within rounding)."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max, bg)
    n = scene.n
    g = np.ascontiguousarray(grad_rgb, dtype=np.float64).reshape(-1, 3)
    dm = np.zeros((n, 3)); ds = np.zeros((n, 3)); dq = np.zeros((n, 4)); do = np.zeros(n); dc = np.zeros((n, 3))
    nr = b.o.shape[0]
    extra = np.zeros(nr, np.int32)
    near = np.zeros(nr, np.int32)
    p = params.c()
    lib().orc_render_bwd_paper(C.byref(b.sc), C.byref(b.rays), C.byref(p), float(eps2), _ptr(g), _ptr(dm),
                               _ptr(ds), _ptr(dq), _ptr(do), _ptr(dc), _ptr(extra), _ptr(near), int(threads))
    return dict(mean=dm, scale=ds, quat=dq, opacity=do, rgb=dc), extra, near.astype(bool)


def ray_hits(scene, origin, direction, k, params=None, t_max=None, cap=1 << 16):
    """Sorted hit list of ray k: (idx, t1, h2, alpha)."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max)
    idx = np.zeros(cap, np.int64); t1 = np.zeros(cap); h2 = np.zeros(cap); al = np.zeros(cap)
    p = params.c()
    n = lib().orc_ray_hits(C.byref(b.sc), C.byref(b.rays), int(k), C.byref(p), cap, _ptr(idx), _ptr(t1), _ptr(h2),
                           _ptr(al))
    n = min(n, cap)
    return idx[:n], t1[:n], h2[:n], al[:n]


def ray_dC_dalpha(scene, origin, direction, k, params=None, cap=1 << 14):
    params = params or Params()
    b = _Bound(scene, origin, direction)
    out = np.zeros((cap, 3))
    p = params.c()
    L = lib().orc_ray_dC_dalpha(C.byref(b.sc), C.byref(b.rays), int(k), C.byref(p), cap, _ptr(out))
    return out[:min(L, cap)]


def ray_alternatives(scene, origin, direction, k, params=None, dh=1e-5, dt=1e-6, dT=1e-3, max_events=3,
                     t_max=None, bg=None, cap=64):
    """Colours the ray may legitimately take under rounding-level decisions;
    None when more than max_events such events occur."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max, bg)
    out = np.zeros((cap, 3))
    p = params.c()
    n = lib().orc_ray_alternatives(C.byref(b.sc), C.byref(b.rays), int(k), C.byref(p), float(dh), float(dt),
                                   float(dT), int(max_events), cap, _ptr(out))
    if n < 0:
        return None
    return out[:min(n, cap)]


def alternatives_batch(scene, origin, direction, params=None, dh=1e-4, dt=5e-6, dT=1e-3, max_events=3,
                       t_max=None, bg=None, cap=16, threads=0):
    """Per ray: (count[n], colours[n, cap, 3]); count -1 marks an unresolved ray."""
    params = params or Params()
    b = _Bound(scene, origin, direction, t_max, bg)
    n = b.o.shape[0]
    cnt = np.zeros(n, np.int64)
    out = np.zeros((n, cap, 3))
    p = params.c()
    lib().orc_alternatives_batch(C.byref(b.sc), C.byref(b.rays), C.byref(p), float(dh), float(dt), float(dT),
                                 int(max_events), int(cap), _ptr(cnt), _ptr(out), int(threads))
    return cnt, out


def compare_with_alternatives(gpu_rgb, ref_rgb, scene, origin, direction, params=None, tol=1e-4, t_max=None,
                              bg=None, **win):
    """Parity protocol: a ray passes when |gpu - oracle| <= tol per channel, or
    when its colour is within tol of one of the oracle's rounding-level
    alternatives. Returns a dict of counts and the worst error after the protocol."""
    # up to 8 events (256 alternatives) per pixel: dense scenes put several near-tied
    # pairs on one ray
    win.setdefault("max_events", 8)
    win.setdefault("cap", 256)
    gpu = np.asarray(gpu_rgb, np.float64).reshape(-1, 3)
    ref = np.asarray(ref_rgb, np.float64).reshape(-1, 3)
    err = np.abs(gpu - ref).max(axis=1)
    bad = np.nonzero(err > tol)[0]
    resolved = 0
    unresolved = []
    worst = float(err[err <= tol].max()) if np.any(err <= tol) else 0.0
    if len(bad):
        o = np.asarray(origin, np.float32).reshape(-1, 3)[bad]
        d = np.asarray(direction, np.float32).reshape(-1, 3)[bad]
        tm = None if t_max is None else np.asarray(t_max, np.float64)[bad]
        bgs = None if bg is None else np.asarray(bg, np.float64).reshape(-1, 3)[bad]
        cnt, alts = alternatives_batch(scene, o, d, params, t_max=tm, bg=bgs, **win)
        for j, k in enumerate(bad):
            if cnt[j] > 0:
                e = np.abs(alts[j, :min(cnt[j], alts.shape[1])] - gpu[k]).max(axis=1).min()
                if e <= tol:
                    resolved += 1
                    continue
            unresolved.append(int(k))
    return dict(n=len(gpu), within=int(len(gpu) - len(bad)), resolved=resolved, unresolved=unresolved,
                max_err=float(err.max()) if len(err) else 0.0, worst_ok=worst)


def intersect(scene, i, o, d, Q=Q_DEFAULT, t_min=0.0):
    """(hit, t1, h2) of ray (o, d) against Gaussian i."""
    b = _Bound(scene, np.zeros((1, 3)), np.ones((1, 3)))
    o = np.ascontiguousarray(o, np.float32)
    d = np.ascontiguousarray(d, np.float32)
    t1 = C.c_double(); h2 = C.c_double()
    hit = lib().orc_intersect(C.byref(b.sc), int(i), _ptr(o), _ptr(d), float(Q), float(t_min), C.byref(t1),
                              C.byref(h2))
    return bool(hit), t1.value, h2.value


def rotation(q):
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    lib().orc_rotation(_ptr(q), _ptr(R))
    return R.reshape(3, 3)


def rotation_derivs(q):
    q = np.ascontiguousarray(q, np.float64)
    D = np.zeros(36)
    lib().orc_rotation_derivs(_ptr(q), _ptr(D))
    return D.reshape(4, 3, 3)


def morton_codes(mean):
    m = np.ascontiguousarray(mean, np.float32)
    n = m.shape[0]
    codes = np.zeros(n, np.uint32)
    lo = np.zeros(3, np.float32); hi = np.zeros(3, np.float32)
    lib().orc_morton_codes(n, _ptr(m), _ptr(codes), _ptr(lo), _ptr(hi))
    return codes, lo, hi


def sort_codes(codes):
    codes = np.ascontiguousarray(codes, np.uint32)
    n = codes.shape[0]
    s = np.zeros(n, np.uint32); perm = np.zeros(n, np.int32)
    lib().orc_sort_codes(n, _ptr(codes), _ptr(s), _ptr(perm))
    return s, perm


def radix_tree(sorted_codes):
    """(child[n-1, 2] int32, leaf[n-1, 2] bool) of the unique binary radix tree."""
    s = np.ascontiguousarray(sorted_codes, np.uint32)
    n = s.shape[0]
    m = max(n - 1, 0)
    child = np.zeros((max(m, 1), 2), np.int32); leaf = np.zeros((max(m, 1), 2), np.int32)
    lib().orc_radix_tree(n, _ptr(s), _ptr(child), _ptr(leaf))
    return child[:m], leaf[:m].astype(bool)


def leaf_boxes(mean, scale, quat, perm, Q=Q_DEFAULT):
    """Bit-exact leaf boxes [n, 6] (lo xyz, hi xyz) in sorted order (row j: Gaussian perm[j])."""
    m = np.ascontiguousarray(mean, np.float32)
    s = np.ascontiguousarray(scale, np.float32)
    q = np.ascontiguousarray(quat, np.float32)
    pm = np.ascontiguousarray(perm, np.int32)
    n = m.shape[0]
    out = np.zeros((max(n, 1), 6), np.float32)
    lib().orc_leaf_boxes(n, _ptr(m), _ptr(s), _ptr(q), float(Q), _ptr(pm), _ptr(out))
    return out[:n]


def ploc(leaf_boxes):
    """PLOC tree over sorted leaf boxes: (child[n-1, 2] refs (< 0: leaf ~j), boxes[n-1, 2, 6], iterations)."""
    lb = np.ascontiguousarray(leaf_boxes, np.float32)
    n = lb.shape[0]
    m = max(n - 1, 1)
    child = np.zeros((m, 2), np.int32)
    boxes = np.zeros((m, 2, 6), np.float32)
    it = lib().orc_ploc(n, _ptr(lb), _ptr(child), _ptr(boxes))
    return child[:max(n - 1, 0)], boxes[:max(n - 1, 0)], int(it)


def ploc_cap(n):
    return int(lib().orc_ploc_cap(int(n)))


def mesh_closest(verts, tris, origin, direction, t_eps=1e-9, edge=0.0, want_amb=False):
    """Brute-force FP64 closest triangle hit per ray: (t[n] (inf = miss), tri[n] (-1 = miss)[, amb[n]])."""
    v = np.ascontiguousarray(verts, np.float32)
    t = np.ascontiguousarray(tris, np.int32)
    o = np.ascontiguousarray(origin, np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(direction, np.float64).reshape(-1, 3)
    n = o.shape[0]
    th = np.zeros(n); tri = np.zeros(n, np.int64)
    amb = np.zeros(n, np.int32)
    lib().orc_mesh_closest(t.shape[0], _ptr(v), _ptr(t), n, _ptr(o), _ptr(d), float(t_eps), _ptr(th), _ptr(tri),
                           float(edge), _ptr(amb))
    if want_amb:
        return th, tri, amb.astype(bool)
    return th, tri
