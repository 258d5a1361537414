"""The C-ABI library loads, exports every symbol include/raysplats.h declares,
and rejects invalid arguments synchronously (no GPU needed: these paths return
before any HIP call)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "raysplats.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2501_19196_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    declared = _declared()
    assert len(declared) >= 9
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(L.EXPORTS) == declared


def test_struct_layouts_match_header(L, tmp_path):
    """Every ctypes struct of the binding has the C compiler's size and field
    offsets for the header's struct (a small C program reads them)."""
    structs = [L.rs_gaussians, L.rs_view, L.rs_rays, L.rs_params, L.rs_grads, L.rs_bvh, L.rs_mesh, L.rs_shading,
               L.rs_tune, L.rs_loss_params]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "raysplats.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in st._fields_:
            # a trailing underscore marks a C name that is a Python keyword
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0].rstrip("_")}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for st in structs:
        name = st.__name__
        assert got[(name, "size")] == C.sizeof(st), name
        for f in st._fields_:
            assert got[(name, f[0])] == getattr(st, f[0]).offset, (name, f[0])


def test_defaults_and_strings(L):
    lib = L.lib()
    p = L.rs_params()
    lib.rs_default_params(C.byref(p))
    assert abs(p.Q - 11.3449) < 1e-5 and abs(p.eps1 - 1e-4) < 1e-9 and p.max_hits == 512 and p.flags == 0
    for code in range(0, -9, -1):
        assert lib.rs_status_string(code)
    assert b"unknown" not in lib.rs_status_string(L.RS_ERR_LIST_POOL)
    # final colour/T, then (256-byte aligned) the adjoint's start: 16 bytes per ray each
    assert lib.rs_ray_state_bytes(10, None) == 256 + 160
    q = L.rs_params()
    lib.rs_default_params(C.byref(q))
    q.hit_list = 8
    # then the list bookkeeping (16 bytes per ray) and the pool: a 256-byte header, the
    # chunk links, the chunk fills and whole chunks of 512 slots x 4 bytes (80 slots -> one
    # chunk)
    assert lib.rs_ray_state_bytes(10, C.byref(q)) == 512 + 256 + 256 + 256 + 256 + 512 * 4
    q.hit_list = 100
    n = 100000
    chunks = (n * 100 + 511) // 512
    head = (n * 16 + 255) // 256 * 256
    assert lib.rs_ray_state_bytes(n, C.byref(q)) == 3 * head + 256 + 2 * ((chunks * 4 + 255) // 256 * 256) + chunks * 2048
    a, b = lib.rs_bvh_workspace_bytes(1000), lib.rs_bvh_workspace_bytes(100000)
    assert 0 < a < b and b % 256 == 0


def test_invalid_arguments_are_rejected(L):
    lib = L.lib()
    p = L.rs_params()
    lib.rs_default_params(C.byref(p))
    out = L.rs_bvh()
    g = L.rs_gaussians(10, None, None, None, None, None)  # null arrays
    assert lib.rs_build_bvh(C.byref(g), C.byref(p), C.c_void_p(256), 1 << 20, C.byref(out), None) == \
        L.RS_ERR_INVALID_ARG
    g = L.rs_gaussians(-1, None, None, None, None, None)
    assert lib.rs_build_bvh(C.byref(g), C.byref(p), C.c_void_p(256), 1 << 20, C.byref(out), None) == \
        L.RS_ERR_INVALID_ARG
    # workspace too small (fake, never dereferenced, aligned pointers)
    fake = C.c_void_p(1 << 20)
    g = L.rs_gaussians(1000, fake, fake, fake, fake, fake)
    assert lib.rs_build_bvh(C.byref(g), C.byref(p), fake, 100, C.byref(out), None) == L.RS_ERR_WORKSPACE
    # bad knobs
    for field, val in (("Q", 0.0), ("eps1", -1.0), ("max_hits", -3), ("kbuf", 12), ("stack_depth", 65),
                       ("flags", 1 << 9), ("t_min", -1.0), ("tile_width", 12), ("hit_list", -1),
                       ("hit_list", 5000)):
        q = L.rs_params()
        lib.rs_default_params(C.byref(q))
        setattr(q, field, val)
        assert lib.rs_build_bvh(C.byref(g), C.byref(q), fake, 1 << 30, C.byref(out), None) == L.RS_ERR_INVALID_ARG
    # the paper's gradient variant needs stored lists, a finite K_max and eps2 in [0, 1]
    for hit_list, max_hits, eps2 in ((0, 512, 1e-4), (512, 0, 1e-4), (512, 512, 2.0), (512, 512, -0.5)):
        q = L.rs_params()
        lib.rs_default_params(C.byref(q))
        q.flags, q.hit_list, q.max_hits, q.eps2 = L.RS_PAPER_GRADIENT, hit_list, max_hits, eps2
        assert lib.rs_build_bvh(C.byref(g), C.byref(q), fake, 1 << 30, C.byref(out), None) == L.RS_ERR_INVALID_ARG
    # an uninitialised descriptor is rejected by the render calls
    r = L.rs_rays(4, fake, fake, None, None, 0, None)
    assert lib.rs_render_fwd(C.byref(L.rs_bvh()), C.byref(g), C.byref(r), C.byref(p), fake, None, None) == \
        L.RS_ERR_INVALID_ARG
    # views must tile the rays exactly
    views = (L.rs_view * 1)()
    views[0].ray_offset, views[0].width, views[0].height = 0, 3, 3
    r = L.rs_rays(10, fake, fake, None, None, 1, C.cast(views, C.POINTER(L.rs_view)))
    assert lib.rs_render_fwd(C.byref(L.rs_bvh()), C.byref(g), C.byref(r), C.byref(p), fake, None, None) == \
        L.RS_ERR_INVALID_ARG


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2501_19196_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).lower() or f == "__init__.py", f
