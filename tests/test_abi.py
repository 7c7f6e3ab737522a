"""C-ABI contract checks that run without a GPU.

The library must load, export every function ``include/nbody.h`` declares, and
reject invalid arguments before it touches the device.  No kernel is launched.
"""
import ctypes
import os
import re

import pytest

from paper_astro_ph_0703100_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*NBODY_API\s+(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(nbody_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("nbody_force", "nbody_force_ex", "nbody_force_f64", "nbody_last_error",
                     "nbody_workspace_size", "nbody_opts_default"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, "binding lacks " + name


def test_opts_layout_and_defaults():
    o = _lib.nbody_opts_default()
    assert o.precision == _lib.NBODY_COMP
    assert o.centre == _lib.NBODY_CENTRE_SYSTEM
    assert o.self_pot == 0 and o.ipl == 0 and o.jtile == 0 and o.nseg == 0 and o.jlanes == 0
    assert o.symmetric == 0
    assert not o.workspace and o.workspace_bytes == 0
    # eight int32 fields, a pointer and a size_t (the header's layout)
    assert ctypes.sizeof(_lib.nbody_opts) == 48
    assert _lib.nbody_opts.symmetric.offset == 28
    assert _lib.nbody_opts.workspace.offset == 32
    assert _lib.nbody_version().startswith("nbody")


FAKE = 0x1000  # a non-NULL address that must never be dereferenced (validation fails first)


@pytest.mark.parametrize("args,what", [
    ((-1, FAKE, FAKE, 0.1, FAKE, None), "negative n"),
    ((1 << 31, FAKE, FAKE, 0.1, FAKE, None), "n too large"),
    ((10, None, FAKE, 0.1, FAKE, None), "NULL pos"),
    ((10, FAKE, None, 0.1, FAKE, None), "NULL mass"),
    ((10, FAKE, FAKE, 0.1, None, None), "NULL acc"),
    ((10, FAKE, FAKE, 0.0, FAKE, None), "eps = 0"),
    ((10, FAKE, FAKE, -1.0, FAKE, None), "eps < 0"),
    ((10, FAKE, FAKE, float("nan"), FAKE, None), "eps NaN"),
    ((10, FAKE, FAKE, float("inf"), FAKE, None), "eps Inf"),
    ((10, FAKE, FAKE, 1e-30, FAKE, None), "eps^2 underflows"),
    ((10, FAKE + 2, FAKE, 0.1, FAKE, None), "misaligned pos"),
    ((10, FAKE, FAKE, 0.1, FAKE + 4, None), "misaligned acc"),
])
def test_force_rejects_invalid_arguments(args, what):
    st = _lib.nbody_force(*args, None, check=False)
    assert st == _lib.NBODY_EINVAL, what
    assert _lib.nbody_last_error() != ""


@pytest.mark.parametrize("args,what", [
    ((-1, FAKE, None, 10, FAKE, FAKE, 0.1, FAKE, None), "negative ni"),
    ((10, FAKE, None, -1, FAKE, FAKE, 0.1, FAKE, None), "negative nj"),
    ((10, FAKE, None, 1 << 31, FAKE, FAKE, 0.1, FAKE, None), "nj too large"),
    ((10, None, None, 10, FAKE, FAKE, 0.1, FAKE, None), "NULL pos_i"),
    ((10, FAKE, None, 10, None, FAKE, 0.1, FAKE, None), "NULL pos_j"),
    ((10, FAKE, None, 10, FAKE, None, 0.1, FAKE, None), "NULL mass_j"),
    ((10, FAKE, None, 10, FAKE, FAKE, 0.1, None, None), "NULL acc"),
    ((10, FAKE, None, 10, FAKE, FAKE, -1.0, FAKE, None), "eps < 0"),
    ((10, FAKE, None, 10, FAKE, FAKE, float("nan"), FAKE, None), "eps NaN"),
    ((10, FAKE, None, 10, FAKE, FAKE, 1e-30, FAKE, None), "eps^2 underflows"),
    ((10, FAKE, FAKE + 2, 10, FAKE, FAKE, 0.1, FAKE, None), "misaligned eps_i"),
    ((10, FAKE, None, 10, FAKE, FAKE, 0.1, FAKE, FAKE + 4), "misaligned pot"),
])
def test_force_ij_rejects_invalid_arguments(args, what):
    st = _lib.nbody_force_ij(*args, None, None, check=False)
    assert st == _lib.NBODY_EINVAL, what
    assert _lib.nbody_last_error() != ""


@pytest.mark.parametrize("args,what", [
    ((-1, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None), "negative n"),
    ((10, FAKE, None, FAKE, 0.1, FAKE, FAKE, None), "NULL vel"),
    ((10, FAKE, FAKE, FAKE, 0.1, FAKE, None, None), "NULL jerk"),
    ((10, FAKE, FAKE, None, 0.1, FAKE, FAKE, None), "NULL mass"),
    ((10, FAKE, FAKE, FAKE, 0.0, FAKE, FAKE, None), "eps = 0"),
    ((10, FAKE, FAKE + 2, FAKE, 0.1, FAKE, FAKE, None), "misaligned vel"),
    ((10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE + 4, None), "misaligned jerk"),
])
@pytest.mark.parametrize("entry", ["nbody_force_jerk", "nbody_force_jerk_f64"])
def test_force_jerk_rejects_invalid_arguments(entry, args, what):
    st = getattr(_lib, entry)(*args, None, None, check=False)
    assert st == _lib.NBODY_EINVAL, what


# nbody_force_jerk_ij(ni, pos_i, vel_i, nj, pos_j, vel_j, mass_j, eps, acc, jerk, pot, ...)
@pytest.mark.parametrize("args,what", [
    ((-1, FAKE, FAKE, 10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None), "negative ni"),
    ((10, FAKE, FAKE, 1 << 31, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None), "nj too large"),
    ((10, FAKE, None, 10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None), "NULL vel_i"),
    ((10, FAKE, FAKE, 10, FAKE, None, FAKE, 0.1, FAKE, FAKE, None), "NULL vel_j"),
    ((10, FAKE, FAKE, 10, FAKE, FAKE, None, 0.1, FAKE, FAKE, None), "NULL mass_j"),
    ((10, FAKE, FAKE, 10, FAKE, FAKE, FAKE, 0.1, FAKE, None, None), "NULL jerk"),
    ((10, FAKE, FAKE, 10, FAKE, FAKE, FAKE, -1.0, FAKE, FAKE, None), "eps < 0"),
    ((10, FAKE, FAKE, 10, FAKE, FAKE, FAKE, float("inf"), FAKE, FAKE, None), "eps inf"),
    ((10, FAKE, FAKE + 2, 10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None), "misaligned vel_i"),
    ((10, FAKE, FAKE, 10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, FAKE + 4), "misaligned pot"),
])
def test_force_jerk_ij_rejects_invalid_arguments(args, what):
    st = _lib.nbody_force_jerk_ij(*args, None, None, check=False)
    assert st == _lib.NBODY_EINVAL, what
    assert _lib.nbody_last_error() != ""


def test_force_jerk_ij_empty_i_set_and_options():
    assert _lib.nbody_force_jerk_ij(0, None, None, 10, FAKE, FAKE, FAKE, 0.0, None, None, None,
                                    None, None, check=False) == _lib.NBODY_OK
    o = _lib.nbody_opts_default()
    o.jtile = 100
    assert _lib.nbody_force_jerk_ij(10, FAKE, FAKE, 10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None,
                                    o, None, check=False) == _lib.NBODY_EINVAL
    assert _lib.nbody_workspace_size_jerk_ij(0, 10, None) == 0
    assert _lib.nbody_workspace_size_jerk_ij(1000, 5000, None) > 0


def test_force_jerk_options():
    o = _lib.nbody_opts_default()
    o.centre = 7
    assert _lib.nbody_force_jerk_f64(10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None, o, None,
                                     check=False) == _lib.NBODY_EINVAL
    assert _lib.nbody_force_jerk(0, None, None, None, 0.1, None, None, None, None, None,
                                 check=False) == _lib.NBODY_OK


def test_force_ij_empty_i_set_is_a_no_op():
    # ni = 0 returns before any device call; eps = 0 is legal for separate sets.
    assert _lib.nbody_force_ij(0, None, None, 10, FAKE, FAKE, 0.0, None, None, None, None,
                               check=False) == _lib.NBODY_OK
    o = _lib.nbody_opts_default()
    o.ipl = 3
    assert _lib.nbody_force_ij(10, FAKE, None, 10, FAKE, FAKE, 0.1, FAKE, None, o, None,
                               check=False) == _lib.NBODY_EINVAL


@pytest.mark.parametrize("field,value", [
    ("precision", 3), ("precision", -1), ("self_pot", 2), ("centre", 5),
    ("ipl", 3), ("jtile", 100), ("nseg", -2), ("nseg", 100000),
    ("jlanes", -1), ("jlanes", 3), ("jlanes", 4), ("jlanes", 128),
    ("symmetric", -1), ("symmetric", 3),
])
def test_force_ex_rejects_bad_options(field, value):
    o = _lib.nbody_opts_default()
    setattr(o, field, value)
    st = _lib.nbody_force_ex(4096, FAKE, FAKE, 0.1, FAKE, FAKE, o, None, check=False)
    assert st == _lib.NBODY_EINVAL, (field, value, _lib.nbody_last_error())


@pytest.mark.parametrize("ipl,jtile,nseg,jlanes", [
    (4, 512, 0, 16), (1, 64, 0, 16), (1, 2048, 0, 16), (1, 512, 3, 16)])
def test_force_ex_rejects_bad_split_shapes(ipl, jtile, nseg, jlanes):
    o = _lib.nbody_opts_default()
    o.ipl, o.jtile, o.nseg, o.jlanes = ipl, jtile, nseg, jlanes
    st = _lib.nbody_force_ex(4096, FAKE, FAKE, 0.1, FAKE, FAKE, o, None, check=False)
    assert st == _lib.NBODY_EINVAL, _lib.nbody_last_error()


@pytest.mark.parametrize("ipl,jtile,nseg,jlanes", [
    (8, 128, 0, 0), (3, 64, 0, 0), (1, 256, 0, 0), (1, 32, 0, 0), (1, 128, 0, 16),
    (2, 128, 5000, 0)])
def test_force_ex_rejects_bad_symmetric_shapes(ipl, jtile, nseg, jlanes):
    o = _lib.nbody_opts_default()
    o.ipl, o.jtile, o.nseg, o.jlanes, o.symmetric = ipl, jtile, nseg, jlanes, 2
    st = _lib.nbody_force_ex(4096, FAKE, FAKE, 0.1, FAKE, FAKE, o, None, check=False)
    assert st == _lib.NBODY_EINVAL, _lib.nbody_last_error()


def test_symmetric_engine_refused_where_not_built():
    """symmetric = 2 where there is no symmetric kernel (separate sets, force-jerk, the
    adjoint, tile centres, batched plans): NBODY_EUNSUPPORTED before anything is
    enqueued."""
    o = _lib.nbody_opts_default()
    o.symmetric = 2
    assert _lib.nbody_force_ij(10, FAKE, None, 10, FAKE, FAKE, 0.1, FAKE, None, o, None,
                               check=False) == _lib.NBODY_EUNSUPPORTED
    assert _lib.nbody_force_jerk(10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None, o, None,
                                 check=False) == _lib.NBODY_EUNSUPPORTED
    assert _lib.nbody_force_vjp(10, FAKE, FAKE, 0.1, FAKE, None, FAKE, None, o, None,
                                check=False) == _lib.NBODY_EUNSUPPORTED
    o.centre = _lib.NBODY_CENTRE_TILE
    assert _lib.nbody_force_f64(10, FAKE, FAKE, 0.1, FAKE, None, o, None,
                                check=False) == _lib.NBODY_EUNSUPPORTED
    o.centre = _lib.NBODY_CENTRE_SYSTEM
    arr = (ctypes.c_int64 * 3)(0, 5, 9)
    h = ctypes.c_void_p()
    assert _lib.load().nbody_plan_create_batched(2, arr, ctypes.byref(o), ctypes.byref(h)) == \
        _lib.NBODY_EUNSUPPORTED
    assert h.value is None


def test_symmetric_workspace_size():
    """The symmetric engine's scratch: i-side partials per work-item segment plus the
    j-side sums of every block row but the last, each row only for the particles after
    it, FP64 (PLAIN: FP32)."""
    o = _lib.nbody_opts_default()
    o.symmetric, o.ipl, o.jtile, o.nseg = 2, 1, 128, 4
    n = 5000  # block rows of 512: 10 rows, npad 5120; row 0 has 36 tiles -> 9 per item
    nb, bi, npad, segs = 10, 512, 5120, 4
    jwords = 4 * bi * nb * (nb - 1) // 2  # rows of 9, 8, ..., 1 blocks of bi
    # (the FP64-position path adds FP32 positions and the centre partials)
    extra = 3 * 4 * n + 8192 + 768
    want = segs * 8 * npad * 4 + jwords * 8
    got = _lib.nbody_workspace_size(n, o)
    assert want <= got <= want + extra
    o.precision = _lib.NBODY_PLAIN
    want = segs * 4 * npad * 4 + jwords * 4
    got = _lib.nbody_workspace_size(n, o)
    assert want <= got <= want + extra


def test_split_engine_refused_where_not_built():
    """jlanes > 1 on entry points without split-engine kernels: NBODY_EUNSUPPORTED before
    anything is enqueued (separate sets, force-jerk, tile centres, batched plans)."""
    o = _lib.nbody_opts_default()
    o.jlanes = 16
    assert _lib.nbody_force_ij(10, FAKE, None, 10, FAKE, FAKE, 0.1, FAKE, None, o, None,
                               check=False) == _lib.NBODY_EUNSUPPORTED
    assert _lib.nbody_force_jerk(10, FAKE, FAKE, FAKE, 0.1, FAKE, FAKE, None, o, None,
                                 check=False) == _lib.NBODY_EUNSUPPORTED
    o.centre = _lib.NBODY_CENTRE_TILE
    assert _lib.nbody_force_f64(10, FAKE, FAKE, 0.1, FAKE, None, o, None,
                                check=False) == _lib.NBODY_EUNSUPPORTED
    o.centre = _lib.NBODY_CENTRE_SYSTEM
    arr = (ctypes.c_int64 * 3)(0, 5, 9)
    h = ctypes.c_void_p()
    assert _lib.load().nbody_plan_create_batched(2, arr, ctypes.byref(o), ctypes.byref(h)) == \
        _lib.NBODY_EUNSUPPORTED
    assert h.value is None


def test_force_f64_rejects_misaligned_and_bad_args():
    o = _lib.nbody_opts_default()
    assert _lib.nbody_force_f64(10, FAKE + 4, FAKE, 0.1, FAKE, None, o, None,
                                check=False) == _lib.NBODY_EINVAL
    assert _lib.nbody_force_f64(10, None, FAKE, 0.1, FAKE, None, o, None,
                                check=False) == _lib.NBODY_EINVAL


def test_workspace_too_small_is_rejected_before_launch():
    o = _lib.nbody_opts_default()
    o.workspace = FAKE * 256
    o.workspace_bytes = 16
    st = _lib.nbody_force_ex(100000, FAKE, FAKE, 0.1, FAKE, None, o, None, check=False)
    assert st == _lib.NBODY_EINVAL
    assert "workspace" in _lib.nbody_last_error()


def test_workspace_size_grows_with_n_and_mode():
    o = _lib.nbody_opts_default()
    assert _lib.nbody_workspace_size(0, o) == 0
    a = _lib.nbody_workspace_size(1000, o)
    b = _lib.nbody_workspace_size(100000, o)
    assert 0 < a < b
    o.precision = _lib.NBODY_PLAIN
    assert _lib.nbody_workspace_size(100000, o) < b


def test_vjp_and_adjoint_workspace_sizes():
    o = _lib.nbody_opts_default()
    assert _lib.nbody_workspace_size_vjp(0, o) == 0
    assert _lib.nbody_workspace_size_adjoint(-5, o) == 0
    for n in (100, 16384, 131072):
        v = _lib.nbody_workspace_size_vjp(n, o)
        a = _lib.nbody_workspace_size_adjoint(n, o)
        assert v > 0 and a == v + 3 * 8 * n
    # The adjoint's own launch shape: the grid engine's j-split sets the VJP size.
    o.jlanes, o.nseg = 1, 8
    few = _lib.nbody_workspace_size_vjp(16384, o)
    o.nseg = 64
    assert few < _lib.nbody_workspace_size_vjp(16384, o)
    o.jlanes, o.nseg = 0, 0
    o.ipl = 3
    assert _lib.nbody_workspace_size_vjp(16384, o) == 0


def test_adjoint_rejects_a_too_small_workspace():
    o = _lib.nbody_opts_default()
    need = _lib.nbody_workspace_size_adjoint(1000, o)
    o.workspace = FAKE * 256
    o.workspace_bytes = need - 1
    st = _lib.nbody_leapfrog_adjoint(1000, FAKE, FAKE, 0.1, 0.01, 3, FAKE, FAKE, None, o, None,
                                     check=False)
    assert st == _lib.NBODY_EINVAL and "workspace" in _lib.nbody_last_error()


def test_zero_particles_is_a_noop_without_device_access():
    # n = 0 returns before any HIP call, even with NULL arrays.
    assert _lib.nbody_force(0, None, None, 0.1, None, None, None, check=False) == _lib.NBODY_OK


def test_leapfrog_rejects_invalid_arguments():
    o = _lib.nbody_opts_default()
    ok = (100, FAKE, FAKE, FAKE, 0.1, 0.01, 2, FAKE, None, None, 0, o, None)

    def call(**kw):
        names = ["n", "x", "v", "m", "eps", "dt", "nsteps", "acc", "pot", "traj", "flags", "opts",
                 "stream"]
        args = dict(zip(names, ok))
        args.update(kw)
        return _lib.nbody_leapfrog(*[args[k] for k in names], check=False)

    assert call(nsteps=-1) == _lib.NBODY_EINVAL
    assert call(dt=float("inf")) == _lib.NBODY_EINVAL
    assert call(dt=float("nan")) == _lib.NBODY_EINVAL
    assert call(v=None) == _lib.NBODY_EINVAL
    assert call(flags=4) == _lib.NBODY_EINVAL
    assert call(eps=0.0) == _lib.NBODY_EINVAL
    assert call(x=FAKE + 4) == _lib.NBODY_EINVAL
    assert call(pot=FAKE + 4) == _lib.NBODY_EINVAL
    assert call(traj=FAKE + 4) == _lib.NBODY_EINVAL
    assert call(n=0, x=None, v=None, m=None, acc=None) == _lib.NBODY_OK


def test_graph_create_rejects_invalid_arguments():
    import ctypes
    o = _lib.nbody_opts_default()
    h = ctypes.c_void_p()
    lib = _lib.load()
    st = lib.nbody_graph_create_leapfrog(0, None, None, None, 0.1, 0.01, 1, None, None,
                                         ctypes.byref(o), None, ctypes.byref(h))
    assert st == _lib.NBODY_EINVAL and not h.value
    st = lib.nbody_graph_create_leapfrog(100, FAKE, FAKE, FAKE, 0.1, 0.01, -3, FAKE, None,
                                         ctypes.byref(o), None, ctypes.byref(h))
    assert st == _lib.NBODY_EINVAL
    assert lib.nbody_graph_launch(None, None) == _lib.NBODY_EINVAL
    lib.nbody_graph_destroy(None)


def test_vjp_and_adjoint_reject_invalid_arguments():
    o = _lib.nbody_opts_default()
    for f in (_lib.nbody_force_vjp, _lib.nbody_force_vjp_f64):
        assert f(-1, FAKE, FAKE, 0.1, FAKE, None, FAKE, None, o, None, check=False) == _lib.NBODY_EINVAL
        assert f(10, FAKE, FAKE, 0.1, None, None, FAKE, None, o, None, check=False) == _lib.NBODY_EINVAL
        assert f(10, FAKE, FAKE, 0.1, FAKE, None, None, None, o, None, check=False) == _lib.NBODY_EINVAL
        assert f(10, FAKE, FAKE, -0.1, FAKE, None, FAKE, None, o, None, check=False) == _lib.NBODY_EINVAL
        assert f(10, FAKE, FAKE, 0.1, FAKE + 4, None, FAKE, None, o, None, check=False) == _lib.NBODY_EINVAL
        assert f(0, None, None, 0.1, None, None, None, None, o, None, check=False) == _lib.NBODY_OK
    adj = _lib.nbody_leapfrog_adjoint
    # Zero steps: the cotangents pass through unchanged, nothing is enqueued (the fake
    # pointers are never touched).
    assert adj(10, FAKE, FAKE, 0.1, 0.01, 0, FAKE, FAKE, FAKE, o, None, check=False) == _lib.NBODY_OK
    assert adj(10, FAKE, FAKE, 0.1, 0.01, -1, FAKE, FAKE, None, o, None, check=False) == _lib.NBODY_EINVAL
    assert adj(10, FAKE, FAKE, 0.1, float("nan"), 2, FAKE, FAKE, None, o, None, check=False) == _lib.NBODY_EINVAL
    assert adj(10, FAKE, FAKE, 0.1, 0.01, 2, FAKE, None, None, o, None, check=False) == _lib.NBODY_EINVAL
    assert adj(0, None, None, 0.1, 0.01, 2, None, None, None, o, None, check=False) == _lib.NBODY_OK


@pytest.mark.parametrize("nsys,offsets,opt,status,what", [
    (-1, [0], {}, "NBODY_EINVAL", "negative nsys"),
    (2, [1, 5, 9], {}, "NBODY_EINVAL", "offsets[0] != 0"),
    (3, [0, 5, 4, 9], {}, "NBODY_EINVAL", "decreasing offsets"),
    (1, [0, 1 << 31], {}, "NBODY_EINVAL", "too many particles"),
    (2, [0, 5, 9], {"precision": 4}, "NBODY_EINVAL", "bad precision"),
    (2, [0, 5, 9], {"ipl": 3}, "NBODY_EINVAL", "bad ipl"),
    (2, [0, 5, 9], {"jtile": 32}, "NBODY_EINVAL", "bad jtile"),
    (2, [0, 5, 9], {"centre": 2}, "NBODY_EUNSUPPORTED", "tile centres"),
    (2, [0, 5, 9], {"self_pot": 1}, "NBODY_EUNSUPPORTED", "self term kept"),
])
def test_batched_plan_rejects_bad_offsets_and_options(nsys, offsets, opt, status, what):
    # Checked on the host before any device call; the plan handle stays NULL.
    o = _lib.nbody_opts_default()
    for k, v in opt.items():
        setattr(o, k, v)
    arr = (ctypes.c_int64 * max(1, len(offsets)))(*offsets)
    h = ctypes.c_void_p(12345)
    st = _lib.load().nbody_plan_create_batched(nsys, arr, ctypes.byref(o), ctypes.byref(h))
    assert st == getattr(_lib, status), what
    assert h.value is None, what
    assert _lib.nbody_last_error() != ""


def test_batched_plan_rejects_a_caller_workspace():
    o = _lib.nbody_opts_default()
    o.workspace = FAKE
    o.workspace_bytes = 1 << 20
    arr = (ctypes.c_int64 * 3)(0, 5, 9)
    h = ctypes.c_void_p()
    assert _lib.load().nbody_plan_create_batched(2, arr, ctypes.byref(o), ctypes.byref(h)) == \
        _lib.NBODY_EINVAL
    assert _lib.load().nbody_plan_create_batched(2, arr, None, None) == _lib.NBODY_EINVAL


def test_tuning_table_roundtrip(tmp_path):
    _lib.nbody_tune_reset()
    base = _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 131072)
    assert base[0] in (1, 2, 4, 8) and base[1] in (64, 128, 256, 512)
    _lib.nbody_tune_set(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 131072, 8, 512, 12)
    _lib.nbody_tune_set(_lib.NBODY_KERNEL_VJP, _lib.NBODY_PLAIN, 5000, 1, 64, 3)
    _lib.nbody_tune_set(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_FP64RED, 3000, 2, 1024, 0, 32)
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 131072) == (8, 512, 12, 1, 0)
    # Same size bucket (floor(log2 n) = 17), other precision untouched.
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 200000) == (8, 512, 12, 1, 0)
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_PLAIN, 131072) == base
    path = tmp_path / "t.json"
    _lib.nbody_tune_save(path)
    assert '"jlanes": 32' in path.read_text()
    _lib.nbody_tune_reset()
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 131072) == base
    _lib.nbody_tune_load(path)
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 131072) == (8, 512, 12, 1, 0)
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_VJP, _lib.NBODY_PLAIN, 4096) == (1, 64, 3, 1, 0)
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_FP64RED, 2048) == (2, 1024, 0, 32, 0)
    # A file without "jlanes" keys (the earlier format) loads as grid-engine shapes.
    old = tmp_path / "old.json"
    old.write_text('{"entries": [{"kernel": 0, "precision": 2, "bucket": 12, "ipl": 2, '
                   '"jtile": 128, "nseg": 5}]}')
    _lib.nbody_tune_load(old)
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 4096) == (2, 128, 5, 1, 0)
    _lib.nbody_tune_reset()
    # Workspace sizing follows the table.
    o = _lib.nbody_opts_default()
    w0 = _lib.nbody_workspace_size(131072, o)
    _lib.nbody_tune_set(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 131072, 4, 256, 32)
    assert _lib.nbody_workspace_size(131072, o) > w0
    # A split-engine shape keeps its partial sums in registers: the FP64-position path
    # then needs only the FP32 positions and the centre partials.
    _lib.nbody_tune_set(_lib.NBODY_KERNEL_FORCE, _lib.NBODY_COMP, 4096, 1, 512, 0, 16)
    ws = _lib.nbody_workspace_size(4096, o)
    assert 4096 * 12 <= ws <= 4096 * 12 + 16384
    o.centre = _lib.NBODY_CENTRE_TILE  # the tile-centre path runs the grid engine
    assert _lib.nbody_workspace_size(4096, o) > ws
    _lib.nbody_tune_reset()
    if os.path.exists(_lib.TUNING_PATH):
        _lib.nbody_tune_load(_lib.TUNING_PATH)


def test_tuning_rejects_bad_entries(tmp_path):
    raw = _lib.load().nbody_tune_set

    def bad(k, p, n, ipl, jt, nseg, jl, sym=0):
        return raw(k, p, n, ipl, jt, nseg, jl, sym)

    assert bad(0, 2, 1000, 3, 256, 0, 1) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 4, 100, 0, 1) == _lib.NBODY_EINVAL
    assert bad(5, 2, 1000, 4, 256, 0, 1) == _lib.NBODY_EINVAL
    assert bad(0, 2, 0, 4, 256, 0, 1) == _lib.NBODY_EINVAL
    # split-engine entries: jlanes 8..64, ipl 1 or 2, jtile 256..1024 (adjoint <= 512),
    # nseg 0, force and adjoint only
    assert bad(0, 2, 1000, 1, 512, 0, 4) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 4, 512, 0, 16) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 1, 128, 0, 16) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 1, 512, 8, 16) == _lib.NBODY_EINVAL
    assert bad(1, 2, 1000, 1, 1024, 0, 16) == _lib.NBODY_EINVAL
    assert bad(2, 2, 1000, 1, 512, 0, 16) == _lib.NBODY_EINVAL
    assert bad(3, 2, 1000, 1, 512, 0, 16) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 1, 512, 0, 0) == _lib.NBODY_EINVAL
    # symmetric-engine entries: force only, jlanes 1, ipl 1, 2 or 4, jtile 64 or 128
    assert bad(0, 2, 1000, 4, 128, 0, 1, 1) == _lib.NBODY_OK
    assert bad(1, 2, 1000, 1, 128, 0, 1, 1) == _lib.NBODY_EINVAL
    assert bad(3, 2, 1000, 1, 128, 0, 1, 1) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 8, 128, 0, 1, 1) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 1, 256, 0, 1, 1) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 1, 128, 0, 16, 1) == _lib.NBODY_EINVAL
    assert bad(0, 2, 1000, 1, 128, 0, 1, 2) == _lib.NBODY_EINVAL
    _lib.nbody_tune_reset()
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [{"kernel": 0, "precision": 2, "bucket": 17, "ipl": 3, '
                   '"jtile": 256, "nseg": 0}]}')
    assert _lib.load().nbody_tune_load(str(bad).encode()) == _lib.NBODY_EINVAL
    assert _lib.load().nbody_tune_load(str(tmp_path / "missing.json").encode()) == _lib.NBODY_EINVAL


def test_tuning_file_with_a_bad_entry_changes_nothing(tmp_path):
    # A valid entry followed by an invalid one: the load fails and leaves the table as it was.
    _lib.nbody_tune_reset()
    before = _lib.nbody_tune_get(_lib.NBODY_KERNEL_JERK, _lib.NBODY_COMP, 4096)
    mixed = tmp_path / "mixed.json"
    mixed.write_text('{"entries": [{"kernel": 3, "precision": 2, "bucket": 12, "ipl": 8, '
                     '"jtile": 512, "nseg": 7}, {"kernel": 3, "precision": 2, "bucket": 13, '
                     '"ipl": 1, "jtile": 100, "nseg": 0}]}')
    assert _lib.load().nbody_tune_load(str(mixed).encode()) == _lib.NBODY_EINVAL
    assert _lib.nbody_tune_get(_lib.NBODY_KERNEL_JERK, _lib.NBODY_COMP, 4096) == before
    _lib.nbody_tune_reset()
    if os.path.exists(_lib.TUNING_PATH):
        _lib.nbody_tune_load(_lib.TUNING_PATH)


def test_noalloc_rejects_a_workspace_and_sizes_beyond_its_array():
    o = _lib.nbody_opts_default()
    o.workspace = FAKE * 256
    o.workspace_bytes = 1 << 20
    assert _lib.nbody_force_noalloc(1000, FAKE, FAKE, 0.1, FAKE, FAKE, o, None,
                                    check=False) == _lib.NBODY_EINVAL
    # 2^28 particles need 32 B of compensated partial sums each even with one j-segment:
    # far beyond the static array; refused before anything touches the device.
    assert _lib.nbody_force_noalloc(1 << 28, FAKE, FAKE, 0.1, FAKE, FAKE, None, None,
                                    check=False) == _lib.NBODY_EINVAL
    assert "static scratch" in _lib.nbody_last_error()
    # an explicit j-split whose partial sums do not fit is refused, not shortened
    o = _lib.nbody_opts_default()
    o.jlanes, o.nseg = 1, 1024
    assert _lib.nbody_force_noalloc(131072, FAKE, FAKE, 0.1, FAKE, FAKE, o, None,
                                    check=False) == _lib.NBODY_EINVAL
    assert _lib.nbody_force_noalloc(0, None, None, 0.1, None, None, None, None) == _lib.NBODY_OK
