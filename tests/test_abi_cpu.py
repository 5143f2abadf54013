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


DEFAULT_TUNING = {"bin_small_max": 16, "tail_max": 128, "finish_max": 4096, "finish_max_big": 64,
                  "row_small_max": 64, "scan_one_block_max": 16384, "rounds_base": 3,
                  "rounds_n0": 2048, "rounds_growth": 8, "rounds_cap": 8}


def test_tuning_table_set_get_and_ranges():
    saved = K.tuning_get()
    try:
        K.tuning_set(DEFAULT_TUNING)
        assert K.tuning_get() == DEFAULT_TUNING
        K.tuning_set(tail_max=0, row_small_max=8, rounds_base=1, rounds_cap=1)
        t = K.tuning_get()
        assert (t["tail_max"], t["row_small_max"], t["rounds_base"], t["rounds_cap"]) == (0, 8, 1, 1)
        for bad in ({"bin_small_max": 17}, {"bin_small_max": 0}, {"row_small_max": 65},
                    {"row_small_max": 1}, {"tail_max": 4097}, {"rounds_growth": 1},
                    {"rounds_base": 4, "rounds_cap": 3}, {"scan_one_block_max": -1}):
            before = K.tuning_get()
            with pytest.raises(K.KappaError) as e:
                K.tuning_set(bad)
            assert e.value.status == K.E_RANGE and K.tuning_get() == before   # unchanged
        assert K.lib().kappa_tuning_set(None) == K.E_ARG
        assert K.lib().kappa_tuning_get(None) == K.E_ARG
    finally:
        K.tuning_set(saved)


def test_tuning_table_files(tmp_path):
    saved = K.tuning_get()
    try:
        K.tuning_set(DEFAULT_TUNING)
        good = tmp_path / "t.txt"
        good.write_text("# measured table\n\ntail_max 256   # comment\nrounds_n0 4096\n")
        K.tuning_load(str(good))
        t = K.tuning_get()
        assert t["tail_max"] == 256 and t["rounds_n0"] == 4096
        assert t["finish_max"] == DEFAULT_TUNING["finish_max"]   # fields not named are kept
        for text, status in (("no_such_field 3\n", K.E_ARG), ("tail_max\n", K.E_ARG),
                             ("tail_max 3 4\n", K.E_ARG), ("tail_max x\n", K.E_ARG),
                             ("tail_max 999999\n", K.E_RANGE)):
            bad = tmp_path / "bad.txt"
            bad.write_text(text)
            before = K.tuning_get()
            with pytest.raises(K.KappaError) as e:
                K.tuning_load(str(bad))
            assert e.value.status == status, text
            assert K.tuning_get() == before
        with pytest.raises(K.KappaError):
            K.tuning_load(str(tmp_path / "missing.txt"))
    finally:
        K.tuning_set(saved)


def test_tuning_table_read_at_load(tmp_path):
    """A fresh process reads the table named by KAPPA_TUNING when the library
    loads, and keeps the compiled defaults with KAPPA_TUNING=none."""
    import json
    import subprocess
    import sys
    f = tmp_path / "t.txt"
    f.write_text("finish_max 1000\nbin_small_max 8\n")
    code = ("import json, paper_0910_2004_amd as K; print(json.dumps(K.tuning_get()))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(K.__file__)))
    for env, want in ((str(f), dict(DEFAULT_TUNING, finish_max=1000, bin_small_max=8)),
                      ("none", DEFAULT_TUNING)):
        out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True,
                             text=True, env=dict(os.environ, KAPPA_TUNING=env), timeout=300)
        assert out.returncode == 0, out.stderr
        assert json.loads(out.stdout.strip().splitlines()[-1]) == want
