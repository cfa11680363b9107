"""The entry point that allocates nothing (evrt_trace_rays_noalloc) against
the allocating ray-query entry point (evrt_trace_rays): identical hits and
any-hit flags, bit for bit, on two calls in a row (the second with fewer
rays), with the rays staged in the library's static scratch array."""
import ctypes
import sys

import numpy as np
import pytest

import paper_2408_07996_amd as ev
from paper_2408_07996_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _rays(sc_tris, rng, n):
    o = rng.uniform(-3.0, 3.0, size=(n, 3)).astype(np.float32)
    tgt = sc_tris[rng.integers(0, len(sc_tris), n)]
    d = np.where(rng.random((n, 1)) < 0.6, tgt - o, rng.normal(size=(n, 3)))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tmin = np.full((n, 1), 1e-4, np.float32)
    tmax = np.where(rng.random((n, 1)) < 0.3, rng.uniform(0.5, 5.0, (n, 1)), np.inf).astype(np.float32)
    skip = np.where(rng.random(n) < 0.2, rng.integers(0, 50, n), ev.NO_PRIM).astype(np.uint32)
    return np.concatenate([o, tmin, d, tmax], axis=1), skip


@pytest.fixture(scope="module")
def rend():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    r = ev.Renderer(0)
    yield r
    r.close()


def _noalloc(rend, t, rays_d, skip_d, any_hit):
    import torch
    n = rays_d.shape[0]
    prim = torch.full((n,), -7, dtype=torch.int32, device=rays_d.device)
    tt = None if any_hit else torch.full((n,), -1.0, dtype=torch.float32, device=rays_d.device)
    rend.trace_rays_noalloc(t, rays_d, skip_d, any_hit, tt, prim)
    torch.cuda.synchronize()
    return prim.cpu().numpy(), (None if tt is None else tt.cpu().numpy())


def test_noalloc_trace_matches_allocating_entry(rend):
    import torch
    sc = scenes.triangle_soup(400, seed=3, moving=True)
    rend.set_scene(sc)
    verts = sc.xyz.astype(np.float32)
    rng = np.random.default_rng(11)
    for t in (0.0, 1.0):
        # The allocating call makes the scene at t resident; then two no-alloc
        # calls in a row, the second with fewer rays.
        for n in (5000, 1200):
            rays, skip = _rays(verts, rng, n)
            _say(f"noalloc t={t} n={n}")
            t_ref, p_ref = rend.trace_rays(t, rays, skip)
            a_ref = rend.trace_rays(t, rays, skip, any_hit=True)
            rays_d = torch.as_tensor(rays).cuda().contiguous()
            skip_d = torch.as_tensor(skip.view(np.int32)).cuda()
            p, tt = _noalloc(rend, t, rays_d, skip_d, False)
            np.testing.assert_array_equal(p, p_ref.cpu().numpy())
            np.testing.assert_array_equal(tt.view(np.uint32), t_ref.cpu().numpy().view(np.uint32))
            a, _ = _noalloc(rend, t, rays_d, skip_d, True)
            np.testing.assert_array_equal(a, a_ref.cpu().numpy())
            # without a skip array
            p2, tt2 = _noalloc(rend, t, rays_d, None, False)
            t_ref2, p_ref2 = rend.trace_rays(t, rays)
            np.testing.assert_array_equal(p2, p_ref2.cpu().numpy())
            np.testing.assert_array_equal(tt2.view(np.uint32), t_ref2.cpu().numpy().view(np.uint32))


def test_noalloc_errors_and_static_geometry(rend):
    import torch
    L = ev.load_library()
    sc = scenes.triangle_soup(300, seed=4, moving=True)
    rend.set_scene(sc)
    rays, skip = _rays(sc.xyz.astype(np.float32), np.random.default_rng(5), 64)
    rays_d = torch.as_tensor(rays).cuda().contiguous()
    prim = torch.empty(64, dtype=torch.int32, device="cuda")
    tt = torch.empty(64, dtype=torch.float32, device="cuda")
    # Moving geometry at a time never traced: nothing resident, nothing built.
    rc = L.evrt_trace_rays_noalloc(rend._h, 0.5, 64, ctypes.c_void_p(rays_d.data_ptr()), None, 0,
                                   ctypes.c_void_p(tt.data_ptr()), ctypes.c_void_p(prim.data_ptr()), None)
    assert rc == ev.EVRT_E_STATE, L.evrt_last_error(rend._h)
    # Above the limit: refused on the host before any device work.
    rc = L.evrt_trace_rays_noalloc(rend._h, 0.5, (1 << 20) + 1,
                                   ctypes.c_void_p(rays_d.data_ptr()), None, 0, ctypes.c_void_p(tt.data_ptr()),
                                   ctypes.c_void_p(prim.data_ptr()), None)
    assert rc == ev.EVRT_E_INVALID and b"maximum" in L.evrt_last_error(rend._h)
    # Static geometry: any resident instant serves a new time.
    st = scenes.triangle_soup(300, seed=6, moving=False)
    rend.set_scene(st)
    rays, skip = _rays(st.xyz.astype(np.float32), np.random.default_rng(8), 3000)
    t_ref, p_ref = rend.trace_rays(0.0, rays, skip)
    rays_d = torch.as_tensor(rays).cuda().contiguous()
    skip_d = torch.as_tensor(skip.view(np.int32)).cuda()
    p, t_out = _noalloc(rend, 0.75, rays_d, skip_d, False)
    np.testing.assert_array_equal(p, p_ref.cpu().numpy())
    np.testing.assert_array_equal(t_out.view(np.uint32), t_ref.cpu().numpy().view(np.uint32))
