"""Streams, caller workspaces and caller-side graph capture of the force entry point.

The library runs asynchronously on the caller's stream; with a caller workspace it
enqueues nothing but kernel launches, so a caller can record it into a HIP graph and
run independent evaluations on several streams at once.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_astro_ph_0703100_amd import _lib, api, ics

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def system(n, seed):
    pos, _, mass = ics.plummer(n, seed=seed, velocities=False)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(DEV)
    m = torch.from_numpy(mass.astype(np.float32)).to(DEV)
    return p, m


def workspace(n, **kw):
    need = _lib.nbody_workspace_size(n, api.make_opts(**kw))
    return torch.empty(need // 4, dtype=torch.float32, device=DEV)


def test_two_streams_with_their_own_workspaces():
    n, eps = 20000, 0.01
    (pa, ma), (pb, mb) = system(n, 81), system(n, 82)
    ref_a = api.force(pa, ma, eps)
    ref_b = api.force(pb, mb, eps)
    torch.cuda.synchronize()
    wa, wb = workspace(n), workspace(n)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        out_a = api.force(pa, ma, eps, workspace=wa)
    with torch.cuda.stream(sb):
        out_b = api.force(pb, mb, eps, workspace=wb)
    torch.cuda.synchronize()
    for got, ref in ((out_a, ref_a), (out_b, ref_b)):
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])


def test_caller_graph_capture_replays_match_eager():
    n, eps = 6000, 0.02
    p, m = system(n, 83)
    ws = workspace(n)
    acc = torch.empty((3, n), dtype=torch.float64, device=DEV)
    pot = torch.empty(n, dtype=torch.float64, device=DEV)
    ref_acc, ref_pot = api.force(p, m, eps)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # one eager call on the capture stream first
        api.force(p, m, eps, out=(acc, pot), workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        api.force(p, m, eps, out=(acc, pot), workspace=ws)
    for r in range(3):
        acc.zero_()
        pot.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(acc, ref_acc) and torch.equal(pot, ref_pot), r
        # unrelated eager work between replays
        _ = (p * 2.0).sum().item()
    # The captured graph reads the arrays it was recorded with: new positions, new forces.
    p.mul_(2.0)
    g.replay()
    torch.cuda.synchronize()
    acc_direct, _ = api.force(p, m, eps)
    torch.cuda.synchronize()
    assert torch.equal(acc, acc_direct)
    assert not torch.equal(acc, ref_acc)


def test_graph_creation_refuses_a_capturing_stream():
    # The library's own graphs capture on a private stream; asked to build one on a stream
    # the caller is already capturing, it returns NBODY_ECAPTURE and launches nothing, and
    # the caller's capture stays valid.
    n, eps = 4096, 0.02
    p, m = system(n, 84)
    x = p.double().contiguous()
    v = torch.zeros_like(x)
    acc = torch.empty((3, n), dtype=torch.float64, device=DEV)
    ones = torch.ones(16, device=DEV)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ones.add_(1.0)
        h = ctypes.c_void_p()
        st = _lib.load().nbody_graph_create_leapfrog(
            n, x.data_ptr(), v.data_ptr(), m.data_ptr(), eps, 1.0 / 256, 1, acc.data_ptr(),
            None, None, s.cuda_stream, ctypes.byref(h))
    assert st == _lib.NBODY_ECAPTURE and h.value is None
    g.replay()
    torch.cuda.synchronize()
    assert torch.all(ones == 2.0)


def test_capture_without_a_workspace_is_refused():
    # Recording a call that would use the library's own scratch cache is refused with
    # NBODY_ECAPTURE (a later, larger call could reallocate that cache under the graph);
    # nothing is enqueued and the caller's capture stays valid.  (The grid engine keeps
    # partial sums in scratch; the FP64-position paths need scratch with either engine.)
    n, eps = 4096, 0.02
    grid = dict(jlanes=1)
    p, m = system(n, 85)
    x64 = p.double().contiguous()
    g_acc = torch.ones((3, n), dtype=torch.float64, device=DEV)
    api.force(p, m, eps)  # the cache exists and is large enough: still refused
    acc = torch.empty((3, n), dtype=torch.float64, device=DEV)
    gx = torch.empty((3, n), dtype=torch.float64, device=DEV)
    ones = torch.ones(16, device=DEV)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ones.add_(1.0)
        st = _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), None,
                                 api.make_opts(**grid), s.cuda_stream, check=False)
        msg = _lib.nbody_last_error()
        st64 = _lib.nbody_force_f64(n, x64.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), None,
                                    api.make_opts(), s.cuda_stream, check=False)
        stv = _lib.nbody_force_vjp(n, p.data_ptr(), m.data_ptr(), eps, g_acc.data_ptr(), None,
                                   gx.data_ptr(), None, api.make_opts(**grid), s.cuda_stream,
                                   check=False)
    assert st == _lib.NBODY_ECAPTURE and "workspace" in msg, (st, msg)
    assert st64 == _lib.NBODY_ECAPTURE and stv == _lib.NBODY_ECAPTURE
    g.replay()
    torch.cuda.synchronize()
    assert torch.all(ones == 2.0)


def test_split_engine_captures_without_a_workspace():
    # The split engine on FP32 positions uses no scratch at all, so a capture needs no
    # workspace; every replay (with eager work between them) matches the eager result.
    n, eps = 3000, 0.02
    p, m = system(n, 86)
    shape = dict(ipl=1, jtile=512, jlanes=64)
    ref_a, ref_p = api.force(p, m, eps, **shape)
    acc = torch.empty((3, n), dtype=torch.float64, device=DEV)
    pot = torch.empty(n, dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        st = _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(),
                                 pot.data_ptr(), api.make_opts(**shape), s.cuda_stream,
                                 check=False)
    assert st == _lib.NBODY_OK, _lib.nbody_last_error()
    for _ in range(3):
        acc.zero_()
        pot.zero_()
        g.replay()
        api.force(p, m, 2 * eps)  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(acc, ref_a) and torch.equal(pot, ref_p)

