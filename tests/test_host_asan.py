"""Host-side AddressSanitizer run of the C ABI's argument and workspace paths (CPU only).

vs_api.cpp is compiled again with AddressSanitizer on its host code only (`-Xarch_host`; the
device code of every kernel object is the ordinary build's), linked with the other objects of
the ordinary build into a separate library, and driven in a child process with the sanitizer
runtime preloaded: the grid and parameter validation of vs_workspace_bytes (every transform
length, every rejection), the host-side rejections of vs_init, the null-state calls, the
allocation-free entry point's size check and the launch-shape setter. None of these touch a
GPU. The child fails on the first sanitizer report."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2601_05031_amd")

CHILD = r'''
import ctypes, math, sys
sys.path.insert(0, sys.argv[2])
from paper_2601_05031_amd import vs as V
V.LIB_PATH = sys.argv[1]
import paper_2601_05031_amd as P
L = P.lib()

def code_of(fn):
    try:
        fn()
        return 0
    except V.VsError as e:
        return e.code

# every transform length along x and z, and the size rejections
for axis in (0, 2):
    for n in range(1, 600):
        g = [16, 8, 16, 1.0]
        g[axis] = n
        assert code_of(lambda: P.workspace_bytes(tuple(g), P.make_params())) in (0, V.VS_E_UNSUPPORTED)
for grid, code in [((128, 2, 128, 1.0), V.VS_E_ARG), ((128, 16, 128, 0.0), V.VS_E_ARG),
                   ((4, 2049, 512, 1.0), V.VS_E_ARG), ((512, 4097, 512, 1.0), V.VS_E_ARG)]:
    assert code_of(lambda: P.workspace_bytes(grid, P.make_params())) == code, grid
for kw in (dict(eta=0.0), dict(eps=0.0), dict(rtol=0.0), dict(max_cycles=17), dict(rho=math.nan),
           dict(rho=1.0), dict(precision="fp32_refined"), dict(model="cahn_hilliard", sigma=0.0)):
    code_of(lambda: P.workspace_bytes((32, 32, 32, 1.0), P.make_params(**kw)))
# vs_init: rejections before any device call
g = V.VsGrid(32, 32, 32, 1.0)
w = V.VsWalls(V.VS_POISEUILLE, 0.05, 0.0)
p = P.make_params()
st = ctypes.c_void_p(0)
assert L.vs_init(ctypes.byref(g), ctypes.byref(w), ctypes.byref(p), None, ctypes.c_void_p(256),
                 1 << 30, None, ctypes.byref(st)) == V.VS_E_ARG
assert L.vs_init(ctypes.byref(g), ctypes.byref(w), ctypes.byref(p), ctypes.c_void_p(4096),
                 ctypes.c_void_p(4100), 1 << 30, None, ctypes.byref(st)) == V.VS_E_WORKSPACE
assert L.vs_init(ctypes.byref(g), ctypes.byref(w), ctypes.byref(p), ctypes.c_void_p(4096),
                 ctypes.c_void_p(4096), 1024, None, ctypes.byref(st)) == V.VS_E_WORKSPACE
w2 = V.VsWalls(7, 0.0, 0.0)
assert L.vs_init(ctypes.byref(g), ctypes.byref(w2), ctypes.byref(p), ctypes.c_void_p(4096),
                 ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(st)) == V.VS_E_ARG
# null states
assert L.vs_step(None, 1e-3, 1) == V.VS_E_STATE
assert L.vs_grad_step(None, 1e-3, None, None, None) == V.VS_E_STATE
off = ctypes.c_size_t(0)
assert L.vs_field_offset(None, 0, ctypes.byref(off)) == V.VS_E_STATE
out = (ctypes.c_double * 6)()
assert L.vs_diagnostics(None, None, out) == V.VS_E_STATE
b = ctypes.c_void_p(0)
assert L.vs_batch_create(None, 0, None, 1, ctypes.byref(b)) == V.VS_E_ARG
L.vs_batch_destroy(None)
L.vs_destroy(None)
for k in range(L.vs_profile_count()):
    assert L.vs_profile_name(k)
# the allocation-free entry point's size check
gb = V.VsGrid(256, 256, 256, 1.0)
assert L.vs_poisson_solve_noalloc(ctypes.byref(gb), ctypes.c_void_p(8), ctypes.c_void_p(8), 1e-10, 1,
                                  None, None, None) == V.VS_E_WORKSPACE
# launch shapes: accepted and rejected
P.set_launch_shapes((32, 32, 32, 1.0), dict(adv_slab=4, va_maxb=1024, res_maxb=1024, seg_alt=0,
                                            mu_kind=0, mu_ni=8, plane=0))
assert code_of(lambda: P.set_launch_shapes((32, 32, 32, 1.0), dict(adv_slab=0, va_maxb=1024,
               res_maxb=1024, seg_alt=0, mu_kind=0, mu_ni=8, plane=0))) == V.VS_E_ARG
assert L.vs_last_error()
print("asan ok", flush=True)
'''


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_paths_are_clean_under_address_sanitizer(tmp_path):
    from paper_2601_05031_amd import build as B

    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rt = _asan_runtime()
    objs = [os.path.join(PKG, "_build", os.path.splitext(s)[0] + ".o") for s in B.SOURCES
            if s != "vs_api.cpp"]
    if not os.path.exists(hipcc) or rt is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc, the sanitizer runtime and the objects of the ordinary build")
    cflags = [f for f in B.HIPFLAGS if f not in ("-shared", "-Wall", "-Wno-unused-function")]
    api = str(tmp_path / "vs_api_asan.o")
    so = str(tmp_path / "libvs_asan.so")
    subprocess.run([hipcc, *cflags, "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fno-omit-frame-pointer", "-c", "-o", api, os.path.join(PKG, "csrc", "vs_api.cpp")],
                   check=True, capture_output=True, timeout=600)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                    "-fsanitize=address", "-o", so, *objs, api], check=True, capture_output=True,
                   timeout=600)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD, so, ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "asan ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
