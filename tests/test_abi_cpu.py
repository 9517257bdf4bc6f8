"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
validates arguments before touching a device, and its host-side steps (the
circular trajectories and the double-precision ray setup behind the sample
count) agree exactly with the oracle. No compute call needs a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gjp():
    import paper_1609_00958_amd as m
    return m


def _declared_functions():
    with open(os.path.join(ROOT, "include", "gjp.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(gjp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(gjp):
    from paper_1609_00958_amd import _lib
    declared = _declared_functions()
    assert len(declared) >= 12
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(_lib.EXPORTS)


def test_error_paths_without_gpu(gjp):
    from paper_1609_00958_amd import _lib
    L = _lib.lib()
    views = np.zeros((2, 12))
    views[:, 6] = 1.0
    views[:, 10] = 1.0

    def desc(**kw):
        d = _lib.GeometryDesc()
        for k in range(3):
            d.vol_shape[k] = kw.get("shape", (8, 8, 8))[k]
            d.voxel_size[k] = kw.get("vs", 1.0)
        d.n_views, d.n_u, d.n_v = kw.get("n_views", 2), kw.get("n_u", 4), kw.get("n_v", 4)
        d.beam = kw.get("beam", 0)
        v = kw.get("views", views)
        d.views = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if v is not None else None
        d.weight = kw.get("weight", 0)
        d.flags = kw.get("flags", 0)
        return d, v

    h = ctypes.c_void_p()
    for kw in ({"shape": (0, 8, 8)}, {"shape": (8, -1, 8)}, {"shape": (8, 8, 40000)},
               {"vs": 0.0}, {"n_views": 0}, {"n_u": 0}, {"beam": 7}, {"weight": 3},
               {"flags": 2}, {"views": None}):
        d, keep = desc(**kw)
        st = L.gjp_create_geometry(ctypes.byref(d), ctypes.byref(h))
        assert st == _lib.GJP_EINVAL, kw
        assert L.gjp_last_error().decode()
    bad = views.copy()
    bad[1, 4] = np.nan
    d, keep = desc(views=bad)
    assert L.gjp_create_geometry(ctypes.byref(d), ctypes.byref(h)) == _lib.GJP_EINVAL
    assert b"non-finite" in L.gjp_last_error()
    assert L.gjp_create_geometry(None, ctypes.byref(h)) == _lib.GJP_EINVAL
    # projection calls reject null / bad arguments before any GPU work
    d, keep = desc()
    assert L.gjp_create_geometry(ctypes.byref(d), ctypes.byref(h)) == _lib.GJP_OK
    assert L.gjp_forward_project(h, None, 0, None, None) == _lib.GJP_EINVAL
    assert L.gjp_forward_project(h, 16, 9, 16, None) == _lib.GJP_EINVAL
    assert L.gjp_forward_project(None, 16, 0, 16, None) == _lib.GJP_EINVAL
    assert L.gjp_forward_project(h, 18, 0, 16, None) == _lib.GJP_EINVAL  # misaligned
    assert L.gjp_forward_project_naive(h, None, 0, None, None) == _lib.GJP_EINVAL
    assert L.gjp_forward_project_naive(h, 16, 9, 16, None) == _lib.GJP_EINVAL
    assert L.gjp_forward_project_naive(None, 16, 0, 16, None) == _lib.GJP_EINVAL
    assert L.gjp_back_project(h, None, 16, None) == _lib.GJP_EINVAL
    # launch configuration: host-only validation
    assert L.gjp_set_forward_tile(h, 0, 64, 8, 4) == _lib.GJP_OK
    assert L.gjp_set_forward_tile(h, 2, 16, 1, 2) == _lib.GJP_OK
    for args in ((0, 48, 8, 4), (0, 64, 0, 4), (0, 64, 65, 4), (0, 64, 8, 3), (5, 64, 8, 4)):
        assert L.gjp_set_forward_tile(h, *args) == _lib.GJP_EINVAL, args
    assert L.gjp_set_forward_tile(None, 0, 64, 8, 4) == _lib.GJP_EINVAL
    # two rays per lane (128-wide tiles) exist for 16-bit storage only
    assert L.gjp_set_forward_tile(h, 1, 128, 8, 2) == _lib.GJP_OK
    assert L.gjp_set_forward_tile(h, 0, 128, 8, 2) == _lib.GJP_EINVAL
    assert L.gjp_forward_project_batched(0, None, None, None, None, None) == _lib.GJP_EINVAL
    cnt = ctypes.c_uint64()
    assert L.gjp_count_samples(None, ctypes.byref(cnt)) == _lib.GJP_EINVAL
    assert L.gjp_views_circular_cone(0, 1.0, 2.0, 1.0, 1.0, 4, 4, None) == _lib.GJP_EINVAL
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert L.gjp_timing_read(b"forward", ctypes.byref(ms), ctypes.byref(n)) == _lib.GJP_OK
    assert L.gjp_destroy_geometry(h) == _lib.GJP_OK
    assert L.gjp_destroy_geometry(None) == _lib.GJP_OK
    with pytest.raises(gjp.GJPError):
        gjp.views_parallel(3, 1.0, 1.0, -1, 4)


@pytest.mark.parametrize("n_views", [7, 64, 180, 360, 720, 1440])
def test_trajectories_bitwise_equal_to_oracle(gjp, oracle_mod, n_views):
    for args in ((256.0, 512.0, 2.0, 2.0, 64, 64), (1024.0, 1536.0, 1.0, 1.0, 384, 384),
                 (2048.0, 3072.0, 1.0, 1.0, 768, 768)):
        a = gjp.views_circular_cone(n_views, *args)
        b = oracle_mod.views_circular_cone(n_views, *args)
        assert np.array_equal(a, b)
    a = gjp.views_parallel(n_views, 1.25, 0.75, 64, 32)
    b = oracle_mod.views_parallel(n_views, 1.25, 0.75, 64, 32)
    assert np.array_equal(a, b)


def test_sample_count_equals_oracle_configs(gjp, oracle_mod):
    # the host pass runs the kernels' double-precision setup; the oracle counts
    # its own loop (Algorithm 1 with the in-volume test on every plane)
    for name in ("c1",):
        cfg = workloads.config(name)
        G = gjp.Geometry.from_config(cfg)
        assert G.count_samples() == oracle_mod.count_samples(oracle_mod.geometry_for(cfg))
    small = [
        workloads.WorkloadConfig("p", (20, 24, 18), 30, 40, 28, beam="parallel", pitch_u=0.9,
                                 pitch_v=0.8),
        workloads.WorkloadConfig("c", (32, 32, 32), 24, 50, 50, beam="cone", sod=60.0,
                                 sdd=130.0, pitch_u=1.3, pitch_v=1.3),
    ]
    for cfg in small:
        G = gjp.Geometry.from_config(cfg)
        assert G.count_samples() == oracle_mod.count_samples(oracle_mod.geometry_for(cfg))


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_sample_count_equals_oracle_random_geometry(gjp, oracle_mod, beam):
    shape = (13, 17, 11)
    n_views, n_u, n_v = 40, 21, 19
    if beam == "cone":
        views = workloads.random_cone_views(61, n_views, shape, n_u, n_v)
        b = oracle_mod.CONE
    else:
        views = workloads.random_parallel_views(61, n_views, shape, n_u, n_v)
        b = oracle_mod.PARALLEL
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam)
    og = oracle_mod.Geometry(shape, views, n_u, n_v, beam=b)
    assert G.count_samples() == oracle_mod.count_samples(og)


def test_sample_count_anisotropic_voxels(gjp, oracle_mod):
    shape = (16, 12, 20)
    vs = (0.7, 1.3, 0.9)
    ctr = (1.5, -2.0, 0.25)
    views = workloads.random_cone_views(62, 12, shape, 15, 17, voxel_size=vs)
    views[:, 0:3] += ctr
    views[:, 3:6] += ctr
    G = gjp.Geometry(shape, views, 15, 17, voxel_size=vs, center=ctr)
    og = oracle_mod.Geometry(shape, views, 15, 17, voxel_size=vs, center=ctr)
    assert G.count_samples() == oracle_mod.count_samples(og)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_sample_count_with_cylinder_clipping(gjp, oracle_mod, beam):
    # the kernels' range setup (analytic chord + exact end predicate) against
    # the oracle's per-plane test; non-square cross-section, random rays
    shape = (19, 14, 11)
    n_views, n_u, n_v = 36, 23, 17
    if beam == "cone":
        views = workloads.random_cone_views(63, n_views, shape, n_u, n_v)
        b = oracle_mod.CONE
    else:
        views = workloads.random_parallel_views(63, n_views, shape, n_u, n_v)
        b = oracle_mod.PARALLEL
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, clip_cylinder=True)
    og = oracle_mod.Geometry(shape, views, n_u, n_v, beam=b, clip_cylinder=True)
    n_clip = G.count_samples()
    assert n_clip == oracle_mod.count_samples(og)
    assert n_clip < gjp.Geometry(shape, views, n_u, n_v, beam=beam).count_samples()


def test_sample_count_with_cylinder_clipping_circular(gjp, oracle_mod):
    for cfg in (workloads.WorkloadConfig("k", (32, 32, 24), 40, 48, 36, beam="cone", sod=150.0,
                                         sdd=300.0, pitch_u=1.5, pitch_v=1.5,
                                         clip_cylinder=True),
                workloads.WorkloadConfig("q", (30, 26, 10), 33, 40, 12, beam="parallel",
                                         pitch_u=0.9, pitch_v=1.1, clip_cylinder=True)):
        G = gjp.Geometry.from_config(cfg)
        assert G.count_samples() == oracle_mod.count_samples(oracle_mod.geometry_for(cfg))


def test_binding_rejects_non_float32_outputs(gjp):
    """The batched kernel and the autotuner write float32 sinograms: an output
    of another dtype (half the bytes) is refused before anything is launched."""
    import torch
    G = gjp.Geometry.circular_cone((8, 8, 8), 4, 6, 6, 40.0, 60.0)
    vol = torch.zeros(G.shape)
    bad = torch.zeros(G.sino_shape, dtype=torch.bfloat16)
    with pytest.raises(TypeError):
        gjp.forward_batched([vol], [G], [bad])
    with pytest.raises(TypeError):
        gjp.autotune(vol, G, bad)
    with pytest.raises(TypeError):
        gjp.forward_batched([vol.to(torch.float64)], [G])


_ENOMEM_SCRIPT = r"""
import ctypes, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1609_00958_amd import _lib  # constants and the descriptor layout only
L = ctypes.CDLL(_lib.LIB_PATH)
L.gjp_last_error.restype = ctypes.c_char_p
n_views = (1 << 20) - 1
views = np.zeros((n_views, 12))
views[:, 6] = 1.0
views[:, 10] = 1.0
d = _lib.GeometryDesc()
for k in range(3):
    d.vol_shape[k] = 8
    d.voxel_size[k] = 1.0
d.n_views, d.n_u, d.n_v = n_views, 1, 1
d.views = views.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
# the geometry keeps about 250 MB of host copies of the views; leave 64 MB
vm = int(open("/proc/self/status").read().split("VmSize:")[1].split()[0]) * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (64 << 20), vm + (64 << 20)))
h = ctypes.c_void_p()
st = L.gjp_create_geometry(ctypes.byref(d), ctypes.byref(h))
print(st, L.gjp_last_error().decode(), h.value)
"""


def test_host_allocation_failure_reports_enomem(tmp_path):
    """A host allocation that fails (address space capped in a child process)
    comes back as GJP_ENOMEM with a message, and no handle."""
    import subprocess
    import sys
    from paper_1609_00958_amd import _lib
    script = tmp_path / "enomem.py"
    script.write_text(_ENOMEM_SCRIPT)
    r = subprocess.run([sys.executable, str(script), ROOT], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    status, rest = r.stdout.strip().split(" ", 1)
    assert int(status) == _lib.GJP_ENOMEM, r.stdout
    assert "allocation" in rest and rest.endswith("None"), r.stdout


def test_forward_tile_query_and_reset(gjp):
    """Host-only launch configuration: set, query, forget (default 64 / 8 / 4)."""
    import torch
    G = gjp.Geometry.circular_cone((12, 10, 14), 5, 9, 11, 60.0, 90.0)
    assert gjp.get_forward_tile(G, torch.float32) == (64, 8, 4)
    gjp.set_forward_tile(G, torch.float32, 32, 5, 2)
    gjp.set_forward_tile(G, torch.bfloat16, 128, 16, 2)
    assert gjp.get_forward_tile(G, torch.float32) == (32, 5, 2)
    assert gjp.get_forward_tile(G, torch.bfloat16) == (128, 16, 2)
    # the key is the shape signature: a second handle of the same shape shares it
    G2 = gjp.Geometry.circular_cone((12, 10, 14), 5, 9, 11, 70.0, 95.0)
    assert gjp.get_forward_tile(G2, torch.float32) == (32, 5, 2)
    gjp.reset_forward_tile(G, torch.float32)
    assert gjp.get_forward_tile(G, torch.float32) == (64, 8, 4)
    assert gjp.get_forward_tile(G, torch.bfloat16) == (128, 16, 2)
    from paper_1609_00958_amd import _lib
    L = _lib.lib()
    i = ctypes.c_int32()
    assert L.gjp_get_forward_tile(None, 0, ctypes.byref(i), ctypes.byref(i),
                                  ctypes.byref(i)) == _lib.GJP_EINVAL
    assert L.gjp_get_forward_tile(G.handle, 5, ctypes.byref(i), ctypes.byref(i),
                                  ctypes.byref(i)) == _lib.GJP_EINVAL
