"""Persistent cache of autotuned launch shapes.

A JSON file maps a key to the fastest forward and adjoint launch shapes
(hit-buffer size kbuf, persistent grid or not, packet tile width) that
rs_autotune found for it. The key hashes the GPU architecture, the built
library, the workload's shape (Gaussian and ray counts, the view table, mesh
size) and the parameters that change the work (Q, eps1, max_hits, t_min,
hit_list, the colour and gradient-variant flags). A launch shape changes the
time of a render, never a rendered value, so a stale entry can only cost time;
rebuilding the library or moving to another GPU architecture gives new keys.
Host bookkeeping for callers of rs_autotune, not part of the rendering path.
"""

import hashlib
import json
import os
import tempfile

# flags that select the work (zero colour, paper gradient); RS_PERSISTENT is a shape, and
# RS_COUNTERS only instruments
_WORK_FLAGS = (1 << 2) | (1 << 4) | (1 << 0) | (1 << 5)
_SHAPE_FLAG = 1 << 1


def library_digest(path):
    """SHA-256 of the built library's bytes (a rebuild invalidates its entries)."""
    h = hashlib.sha256()
    with open(path, "rb") as f:
        for block in iter(lambda: f.read(1 << 20), b""):
            h.update(block)
    return h.hexdigest()


def make_key(arch, library, n_gauss, n_rays, views, params, extra=None):
    """Stable key of one tuning problem. `views` is the (offset, width, height) table (or
    None), `params` an object with the fields of rs_params, `extra` any other JSON-able
    description of the workload (mesh size, bounce count)."""
    desc = dict(arch=str(arch), library=str(library), n_gauss=int(n_gauss), n_rays=int(n_rays),
                views=[[int(x) for x in v] for v in (views or [])],
                Q=float(params.Q), eps1=float(params.eps1), max_hits=int(params.max_hits),
                t_min=float(params.t_min), hit_list=int(params.hit_list), eps2=float(params.eps2),
                stack_depth=int(params.stack_depth), flags=int(params.flags) & _WORK_FLAGS,
                extra=extra)
    text = json.dumps(desc, sort_keys=True, separators=(",", ":"))
    return hashlib.sha256(text.encode()).hexdigest()


def shape_of(params):
    return dict(kbuf=int(params.kbuf), persistent=bool(int(params.flags) & _SHAPE_FLAG),
                tile_width=int(params.tile_width))


def apply_shape(params, shape):
    """A copy of `params` with the launch shape of a cache entry."""
    import dataclasses
    flags = (int(params.flags) & ~_SHAPE_FLAG) | (_SHAPE_FLAG if shape["persistent"] else 0)
    return dataclasses.replace(params, kbuf=int(shape["kbuf"]), tile_width=int(shape["tile_width"]), flags=flags)


class TuneCache:
    """The cache file: read once, rewritten whole (through a temporary file and a rename) on
    every store. An unreadable or malformed file reads as empty."""

    def __init__(self, path):
        self.path = path
        self.entries = {}
        try:
            with open(path) as f:
                data = json.load(f)
            if isinstance(data, dict) and isinstance(data.get("entries"), dict):
                self.entries = {k: v for k, v in data["entries"].items() if _valid(v)}
        except (OSError, ValueError):
            self.entries = {}

    def get(self, key):
        """(forward shape, adjoint shape) or None."""
        e = self.entries.get(key)
        return (e["fwd"], e["bwd"]) if e is not None else None

    def put(self, key, fwd_params, bwd_params, note=None):
        self.entries[key] = dict(fwd=shape_of(fwd_params), bwd=shape_of(bwd_params), note=note)
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(prefix=".tune_", dir=d)
        try:
            with os.fdopen(fd, "w") as f:
                json.dump(dict(version=1, entries=self.entries), f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise


def _valid(e):
    try:
        for side in ("fwd", "bwd"):
            s = e[side]
            if int(s["kbuf"]) not in (0, 8, 16, 24, 32, 48) or int(s["tile_width"]) not in (0, 4, 8, 16, 32):
                return False
            bool(s["persistent"])
        return True
    except (KeyError, TypeError, ValueError):
        return False
