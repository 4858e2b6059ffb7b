"""The C-ABI library loads and exports every symbol include/lbm.h declares,
and rejects bad arguments before any device work (no GPU needed)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1904_11386_amd", "liblbm.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="liblbm.so not built")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(LIB)
    names = declared_symbols()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_observables" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1904_11386_amd import binding
    assert sorted(binding.EXPORTS) == declared_symbols()


def test_workspace_bytes_and_validation():
    from paper_1904_11386_amd import binding as B
    p = B.make_params(32, 32, 32)
    n0 = B.workspace_bytes(p, 0, 0)
    n1 = B.workspace_bytes(p, 642, 1280)
    assert n1 > n0 >= 32 ** 3 * (2 * 19 * 4 * 2)
    p2 = B.make_params(32, 32, 32, n_slots=2)
    assert B.workspace_bytes(p2, 0, 0) > n0
    lib = B.load()
    out = C.c_int64()
    for bad in (dict(tau=(0.5, 1.0)), dict(G=-1.0), dict(walls=3), dict(precision=7), dict(stream_policy=3),
                dict(zchunk=12), dict(zchunk=72), dict(ring_len=4, precision=B.LBM_FP16),
                dict(rep_eps=-0.1), dict(rep_eps=float("nan")), dict(rep_eps=0.5, rep_d0=0.0),
                dict(rep_eps=0.5, rep_d0=2.5), dict(walls=2, ring_len=4),
                dict(walls=-1)):
        pb = B.make_params(16, 16, 16, **bad)
        assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_EINVAL
        assert lib.lbm_last_error(None)
    pb = B.make_params(3, 16, 16)
    assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_EINVAL
    for bad in (dict(psi_kind=2), dict(psi_kind=-1)):
        pb = B.make_params(16, 16, 16, **bad)
        assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_EINVAL
    # the repulsion's cut-off only matters when it is on; the largest allowed is 2
    for good in (dict(rep_eps=0.0, rep_d0=5.0), dict(rep_eps=0.5, rep_d0=2.0), dict(rep_eps=0.5, ring_len=4),
                 dict(psi_kind=1), dict(psi_kind=1, ring_len=4), dict(walls=2), dict(walls=1),
                 dict(walls=2, precision=B.LBM_FP16)):
        pb = B.make_params(16, 16, 16, **good)
        assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_OK
    # the bounce-back coupling: FP32, periodic, no checkpoints, adjoint or
    # repulsion; positive node mass, non-negative C0
    for bad in (dict(coupling=2), dict(coupling=-1), dict(coupling=1, precision=B.LBM_FP16),
                dict(coupling=1, walls=1), dict(coupling=1, walls=2), dict(coupling=1, n_slots=1),
                dict(coupling=1, ring_len=4), dict(coupling=1, rep_eps=0.5), dict(coupling=1, node_mass=0.0),
                dict(coupling=1, node_mass=float("inf")), dict(coupling=1, mass_c0=-1.0)):
        pb = B.make_params(16, 16, 16, **bad)
        assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_EINVAL, bad
    # one lattice pass: FP32 storage, periodic, the immersed boundary, no adjoint ring
    for bad in (dict(lattice_passes=3), dict(lattice_passes=-1), dict(lattice_passes=1, precision=B.LBM_FP16),
                dict(lattice_passes=1, walls=1), dict(lattice_passes=1, walls=2),
                dict(lattice_passes=1, coupling=1), dict(lattice_passes=1, ring_len=4)):
        pb = B.make_params(16, 16, 16, **bad)
        assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_EINVAL, bad
    for good in (dict(lattice_passes=1), dict(lattice_passes=1, psi_kind=1), dict(lattice_passes=2, walls=1),
                 dict(lattice_passes=0, precision=B.LBM_FP16), dict(lattice_passes=0, coupling=1)):
        pb = B.make_params(16, 16, 16, **good)
        assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_OK, good
    pb = B.make_params(16, 16, 16, coupling=1)
    assert lib.lbm_workspace_bytes(C.byref(pb), 162, 320, C.byref(out)) == B.LBM_OK
    n_bb = out.value
    pb = B.make_params(16, 16, 16)
    assert lib.lbm_workspace_bytes(C.byref(pb), 162, 320, C.byref(out)) == B.LBM_OK
    assert n_bb > out.value
    # more than 2^30 nodes cannot be addressed with 32-bit offsets
    pb = B.make_params(1024, 1024, 1025)
    assert lib.lbm_workspace_bytes(C.byref(pb), 0, 0, C.byref(out)) == B.LBM_EINVAL
    # init rejects a bad tau before touching the (bogus) workspace pointer
    pb = B.make_params(16, 16, 16, tau=(0.4, 1.0))
    r = np.ones(16 ** 3, np.float32)
    ctx = C.c_void_p()
    rc = lib.lbm_init(C.byref(pb), r.ctypes.data_as(C.POINTER(C.c_float)), r.ctypes.data_as(C.POINTER(C.c_float)),
                      C.c_void_p(256), 1 << 30, 0, 0, None, C.byref(ctx))
    assert rc == B.LBM_EINVAL and not ctx.value
    # negative initial density is rejected before device work
    pb = B.make_params(16, 16, 16)
    rneg = r.copy()
    rneg[5] = -1.0
    rc = lib.lbm_init(C.byref(pb), rneg.ctypes.data_as(C.POINTER(C.c_float)), r.ctypes.data_as(C.POINTER(C.c_float)),
                      C.c_void_p(256), 1 << 40, 0, 0, None, C.byref(ctx))
    assert rc == B.LBM_EINVAL
    # a workspace smaller than the query is LBM_ENOMEM
    rc = lib.lbm_init(C.byref(pb), r.ctypes.data_as(C.POINTER(C.c_float)), r.ctypes.data_as(C.POINTER(C.c_float)),
                      C.c_void_p(256), 1024, 0, 0, None, C.byref(ctx))
    assert rc == B.LBM_ENOMEM


def test_no_cpu_fallback_when_library_missing(tmp_path):
    from paper_1904_11386_amd import binding as B
    with pytest.raises(RuntimeError, match="not built"):
        B.load(str(tmp_path / "liblbm.so"))


def test_every_entry_point_rejects_a_null_context():
    """Each call that takes a context returns LBM_EINVAL for NULL before it
    touches anything (no device work), and destroying NULL is a no-op."""
    from paper_1904_11386_amd import binding as B
    lib = B.load()
    null = None
    calls = {
        "lbm_capsules_add": (null, 0, None, None, None, None, None, None, None, None, None),
        "lbm_capsules_bending": (null, 0, 0, None),
        "lbm_capsules_velocity": (null, 0, 0, None, 0),
        "lbm_debug_labels": (null, None),
        "lbm_get_node_velocities": (null, None),
        "lbm_reference_relax": (null, 1, 0.01, 1.0, 0.0, 0.05),
        "lbm_step": (null, 1),
        "lbm_step_timed": (null, 1, None),
        "lbm_observables": (null, None, None),
        "lbm_observables_noalloc": (null, None, None),
        "lbm_get_fields": (null, None, None, None),
        "lbm_get_nodes": (null, None),
        "lbm_get_node_forces": (null, None),
        "lbm_get_spread": (null, None, None),
        "lbm_debug_bins": (null, None, None),
        "lbm_state_save": (null, 0),
        "lbm_state_load": (null, 0),
        "lbm_adjoint_forward": (null, 1, 1, 0, 0, None),
        "lbm_adjoint_backward": (null, None),
        "lbm_adjoint_seed": (null, 0, 0),
        "lbm_adjoint_record": (null, 1),
        "lbm_adjoint_step": (null, 0),
        "lbm_adjoint_grads": (null, None),
    }
    # every context call is listed (the size query, init and the two
    # context-free calls aside)
    free = {"lbm_workspace_bytes", "lbm_init", "lbm_destroy", "lbm_last_error"}
    assert sorted(set(calls) | free) == declared_symbols()
    for name, args in calls.items():
        assert getattr(lib, name)(*args) == B.LBM_EINVAL, name
    lib.lbm_destroy(None)
    assert lib.lbm_last_error(None) is not None

