"""The autotune cache (host bookkeeping): stable keys that change with what changes the
work or the build, entries that round-trip through the file, and bad files read as empty."""

import json
import os

from paper_2501_19196_amd import tune_cache as TC
from paper_2501_19196_amd.renderer import Params


def _key(**kw):
    base = dict(arch="gfx950", library="abc", n_gauss=1000, n_rays=4096, views=[(0, 64, 64)], params=Params(hit_list=64))
    base.update(kw)
    return TC.make_key(base["arch"], base["library"], base["n_gauss"], base["n_rays"], base["views"], base["params"])


def test_key_is_stable_and_ignores_launch_shape_and_background():
    k = _key()
    assert k == _key()
    # the launch shape and the background change no work
    assert k == _key(params=Params(hit_list=64, kbuf=32, tile_width=16, flags=2, bg=(1, 1, 1)))
    # instrumentation does not either
    assert k == _key(params=Params(hit_list=64, flags=8))


def test_key_changes_with_work_build_and_architecture():
    k = _key()
    others = [_key(arch="gfx942"), _key(library="abd"), _key(n_gauss=1001), _key(n_rays=4097),
              _key(views=[(0, 32, 128)]), _key(params=Params(hit_list=0)), _key(params=Params(hit_list=64, eps1=0.0)),
              _key(params=Params(hit_list=64, max_hits=8)), _key(params=Params(hit_list=64, flags=4)),
              _key(params=Params(hit_list=64, flags=16)), _key(params=Params(hit_list=64, Q=9.0))]
    assert len({k, *others}) == len(others) + 1


def test_round_trip_and_bad_files(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = TC.TuneCache(path)
    assert c.get("k") is None
    pf = Params(kbuf=48, tile_width=8)
    pb = Params(kbuf=32, tile_width=16, flags=2 | 16)
    c.put("k", pf, pb, note="test")
    c2 = TC.TuneCache(path)
    f, b = c2.get("k")
    assert f == dict(kbuf=48, persistent=False, tile_width=8)
    assert b == dict(kbuf=32, persistent=True, tile_width=16)
    q = TC.apply_shape(Params(hit_list=64, flags=16), b)
    assert (q.kbuf, q.tile_width, q.flags, q.hit_list) == (32, 16, 16 | 2, 64)
    q = TC.apply_shape(Params(flags=2 | 4), f)
    assert q.flags == 4
    assert not [n for n in os.listdir(tmp_path / "sub") if n.startswith(".tune_")]
    # malformed files and entries read as empty
    with open(path, "w") as fh:
        fh.write("{not json")
    assert TC.TuneCache(path).entries == {}
    with open(path, "w") as fh:
        json.dump(dict(version=1, entries=dict(a=dict(fwd=dict(kbuf=40, persistent=0, tile_width=8),
                                                      bwd=dict(kbuf=8, persistent=0, tile_width=8)),
                                               b=dict(fwd=dict(kbuf=8, persistent=1, tile_width=4),
                                                      bwd=dict(kbuf=16, persistent=0, tile_width=32)))), fh)
    c3 = TC.TuneCache(path)
    assert c3.get("a") is None and c3.get("b") is not None


def test_library_digest(tmp_path):
    p = tmp_path / "lib.so"
    p.write_bytes(b"x" * 3_000_000)
    d1 = TC.library_digest(str(p))
    p.write_bytes(b"x" * 2_999_999 + b"y")
    assert d1 != TC.library_digest(str(p)) and len(d1) == 64
