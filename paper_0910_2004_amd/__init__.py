"""MI355X (gfx950) coarsening hierarchy of a multilevel graph partitioner.

The computation lives in libkappa.so (hand-written HIP kernels behind the C
ABI of include/kappa.h); this package is its Python binding.  Importing it
does not touch the GPU; the first call loads the library and raises if it is
missing (there is no CPU fallback).
"""
from ._lib import (  # noqa: F401
    Batch, DeviceGraph, Hierarchy, KappaError, Server, LevelView, RATINGS, EXPANSION_STAR2, INNER_OUTER, WEIGHT,
    EXPANSION, EXPANSION_STAR, STOP_NONE, STOP_SIZE, STOP_EMPTY, STOP_STALL, STOP_MAXLEVEL,
    OK, E_ARG, E_GRAPH, E_RANGE, E_NOMEM, E_CAPACITY, E_HIP,
    declared_functions, lib, status_str, union_csr,
    kappa_validate, kappa_rate, kappa_match, kappa_match_two_phase, kappa_rcb_order, kappa_relabel,
    kappa_contract, kappa_coarsen, kappa_coarsen_batch, kappa_coarsen_graphs,
    kappa_initial_partition, kappa_project, kappa_cut_balance, kappa_cut_balance_noalloc,
    kappa_uncoarsen, kappa_cache_release,
    kappa_refine, kappa_uncoarsen_refined, refine_params, REFINE_PRESETS, REFINE_K_MAX,
    graphs_enable, tail_enable, persistent_enable, arena_first, use_torch_allocator, profile_enable, profile_reset, profile_read,
    tuning_get, tuning_set, tuning_load, TUNING_FIELDS,
)
