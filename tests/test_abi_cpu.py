"""The C-ABI library loads and exports every function include/kappa.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

import paper_0910_2004_amd as K


def test_header_declares_the_boundary():
    names = K.declared_functions()
    for required in ["kappa_validate", "kappa_rate", "kappa_match", "kappa_contract",
                     "kappa_coarsen", "kappa_project", "kappa_cut_balance", "kappa_uncoarsen",
                     "kappa_hierarchy_levels", "kappa_hierarchy_level", "kappa_hierarchy_free",
                     "kappa_initial_partition", "kappa_status_str"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(os.path.join(os.path.dirname(K.__file__), "libkappa.so")):
        pytest.fail("libkappa.so is not built (run __graft_entry__.build())")
    L = K.lib()
    missing = [n for n in K.declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version():
    L = K.lib()
    for st in range(0, -7, -1):
        s = L.kappa_status_str(st).decode()
        assert s and s != "unknown status"
    assert L.kappa_status_str(5).decode() == "unknown status"
    assert b"gfx950" in L.kappa_version()


def test_null_arguments_rejected_without_gpu_work():
    L = K.lib()
    # every entry point checks its arguments before touching the device
    assert L.kappa_validate(None, None) == K.E_ARG
    assert L.kappa_coarsen(None, None, None, None) == K.E_ARG
    assert L.kappa_hierarchy_levels(None) == 0
    assert L.kappa_hierarchy_level(None, 0, None, None, None) == K.E_ARG
    assert L.kappa_initial_partition(10, 0, 1, None, None) == K.E_ARG
    assert L.kappa_initial_partition(10, 5000, 1, None, None) == K.E_ARG
    g = K._lib.c_graph(-1, 0, None, None, None, None)
    assert L.kappa_validate(ctypes.byref(g), None) == K.E_ARG
    assert L.kappa_rate(ctypes.byref(g), 0, None, None, None) == K.E_ARG
    g = K._lib.c_graph(4, 6, None, None, None, None)
    assert L.kappa_match(ctypes.byref(g), 0, 1, None, None, None, None) == K.E_ARG
    g = K._lib.c_graph(0, 0, ctypes.c_void_p(8), None, None, None)
    assert L.kappa_rate(ctypes.byref(g), 7, None, None, None) == K.E_ARG
    # two-phase matcher: block sizes outside [0, 11] and a bad graph
    for bb in (-1, 12):
        assert L.kappa_match_two_phase(ctypes.byref(g), 0, 1, bb, None, None, None, None) == K.E_ARG
    g = K._lib.c_graph(4, 6, None, None, None, None)
    assert L.kappa_match_two_phase(ctypes.byref(g), 0, 1, 4, None, None, None, None) == K.E_ARG
    # refinement: missing parameters, k outside [1, 256], bad presets, a bad graph
    g = K._lib.c_graph(0, 0, ctypes.c_void_p(8), None, None, None)
    p = K.refine_params("fast")
    assert L.kappa_refine(ctypes.byref(g), None, 4, 3, 100, None, None, None) == K.E_ARG
    for k in (0, 257):
        assert L.kappa_refine(ctypes.byref(g), None, k, 3, 100, ctypes.byref(p), None, None) == K.E_ARG
    for over in (dict(alpha_den=0), dict(depth=-1), dict(max_local=0), dict(max_global=-1),
                 dict(stop_after=0)):
        bad = K.refine_params("fast", **over)
        assert L.kappa_refine(ctypes.byref(g), None, 4, 3, 100, ctypes.byref(bad), None,
                              None) == K.E_ARG, over
    assert L.kappa_refine(ctypes.byref(g), None, 4, 3, 0, ctypes.byref(p), None, None) == K.E_ARG
    g = K._lib.c_graph(4, 6, None, None, None, None)
    assert L.kappa_refine(ctypes.byref(g), None, 4, 3, 100, ctypes.byref(p), None, None) == K.E_ARG
    assert L.kappa_uncoarsen_refined(None, 4, 1, 3, 100, ctypes.byref(p), None, None, None,
                                     None) == K.E_ARG
    L.kappa_hierarchy_free(None)


def test_library_binds_torchs_hip_runtime():
    """Loading the library first (before any torch call) still leaves one HIP
    runtime in the process: the one torch carries."""
    import subprocess
    import sys
    code = ("import os, sys; sys.path.insert(0, %r); import paper_0910_2004_amd as K; K.lib(); "
            "m = open('/proc/self/maps').read().splitlines(); "
            "print(sorted(set(l.split()[-1] for l in m if 'libamdhip64' in l)))"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1 and "torch" in libs[0], libs


def test_noalloc_cut_balance_checks_before_device_work():
    """The allocation-free cut/balance rejects bad arguments and graphs whose
    scratch would exceed its fixed device array before any HIP call (the
    pointers below are never dereferenced)."""
    L = K.lib()
    fake = ctypes.c_void_p(8)
    res = K._lib.c_cut()
    assert L.kappa_cut_balance_noalloc(None, fake, 2, 3, 100, None, ctypes.byref(res), None) == K.E_ARG
    g = K._lib.c_graph(10, 20, fake, fake, fake, fake)
    assert L.kappa_cut_balance_noalloc(ctypes.byref(g), fake, 0, 3, 100, None, ctypes.byref(res),
                                       None) == K.E_ARG
    assert L.kappa_cut_balance_noalloc(ctypes.byref(g), None, 2, 3, 100, None, ctypes.byref(res),
                                       None) == K.E_ARG
    assert L.kappa_cut_balance_noalloc(ctypes.byref(g), fake, 2, 3, 100, None, None, None) == K.E_ARG
    # one int32 of scratch per 2048 entries: 2^31 entries need 4 MiB, beyond the 2 MiB array
    big = K._lib.c_graph(1 << 20, 1 << 31, fake, fake, fake, fake)
    assert L.kappa_cut_balance_noalloc(ctypes.byref(big), fake, 4096, 3, 100, None,
                                       ctypes.byref(res), None) == K.E_CAPACITY
