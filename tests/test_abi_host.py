"""C ABI checks that need no GPU: the library loads, exports every function
the header declares, and its host-side logic (edge colouring, instance
validation, footprint, status strings) behaves as documented."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.colouring import misra_gries
from synthetic import instance_from_edges, random_regular_instance, random_tree_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def g():
    from paper_2409_12240_amd import gtqa
    if not os.path.exists(gtqa.LIB_PATH):
        from paper_2409_12240_amd.build import build
        build()
    gtqa.load_library()
    return gtqa


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "gtqa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gtqa_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_function_is_exported(g):
    lib = C.CDLL(g.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared) <= set(g.EXPORTED) | {"gtqa_default_options"}


def test_colouring_is_bit_exact_with_oracle(g):
    for seed in range(12):
        for n in (16, 100, 1000):
            inst = random_regular_instance(77 * seed + n, n)
            a = g.gtqa_colour_edges(n, inst.edges).astype(np.int64)
            b = misra_gries(n, inst.edges).astype(np.int64)
            assert np.array_equal(a, b)
    tree = random_tree_instance(4, 50)
    assert np.array_equal(g.gtqa_colour_edges(50, tree.edges).astype(np.int64),
                          misra_gries(50, tree.edges).astype(np.int64))


def _init_rc(g, inst, colour=None, **opts):
    lib = g.load_library()
    ci = g._Instance(inst, colour)
    o = g.make_options(**opts)
    h = C.c_void_p()
    rc = lib.gtqa_init_state(C.byref(ci.c), C.byref(o), C.byref(h))
    if rc == 0:
        lib.gtqa_free_state(h)
    return rc


def test_invalid_graphs_are_rejected_before_device_work(g):
    # degree 4
    star = instance_from_edges(5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    assert _init_rc(g, star) == g.GTQA_ERR_GRAPH
    # isolated vertex
    iso = instance_from_edges(4, [(0, 1), (1, 2)])
    assert _init_rc(g, iso) == g.GTQA_ERR_GRAPH
    # unsorted edge list
    inst = random_regular_instance(1, 16)
    bad = instance_from_edges(16, inst.edges.tolist())
    bad.edges = bad.edges[::-1].copy()
    assert _init_rc(g, bad) == g.GTQA_ERR_GRAPH
    # improper colouring supplied
    col = np.zeros(inst.n_edges, dtype=np.uint8)
    assert _init_rc(g, inst, colour=col) == g.GTQA_ERR_GRAPH
    # NaN coupling
    nan = instance_from_edges(16, inst.edges.tolist(), J=np.where(np.arange(24) == 3, np.nan, 0.5))
    assert _init_rc(g, nan) == g.GTQA_ERR_NUMERIC


def test_unsupported_chi_and_bad_options(g):
    inst = random_regular_instance(2, 16)
    assert _init_rc(g, inst, chi=3) == g.GTQA_ERR_UNSUPPORTED
    assert _init_rc(g, inst, bp_max_sweeps=0) == g.GTQA_ERR_ARG


def test_footprint_and_strings(g):
    f4 = g.gtqa_footprint_bytes(1000, 1500, 4, g.GTQA_FP64)
    f4m = g.gtqa_footprint_bytes(1000, 1500, 4, g.GTQA_MIXED)
    f8 = g.gtqa_footprint_bytes(1000, 1500, 8, g.GTQA_FP64)
    assert 0 < f4m < f4 < f8
    # the site tensors alone: 1000 * 2 * 4^3 * 16 bytes
    assert f4 > 1000 * 2 * 64 * 16
    lib = g.load_library()
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8, 99):
        assert lib.gtqa_strerror(code)
    assert g.gtqa_version().startswith("gtqa")


def test_measured_traffic_is_null_for_other_sources(tmp_path, monkeypatch):
    import bench
    assert bench.measured_traffic("simple_update", 4, "mixed", 12345) is None
    # a record is valid only for the kernel source it was measured on
    monkeypatch.setattr(bench, "_source_sha", lambda: "0" * 64)
    assert bench.measured_traffic("simple_update", 4, "mixed", 96000) is None
    assert bench.measured_valu_busy("simple_update", 4, "mixed") is None


def test_measured_traffic_weights_alternative_kernels(tmp_path, monkeypatch):
    # a stage launch runs one of its main kernels, plus any companion launch:
    # the traffic per stage launch is the call-weighted sum
    import json
    import bench
    sha = "1" * 64
    rec = {"kernels": [
        {"stage": "bp_sweep", "chi": 4, "precision": "mixed", "items_per_launch": 96000, "source_sha256": sha,
         "traffic_bytes_per_launch": 300, "calls": 30, "companion": False},
        {"stage": "bp_sweep", "chi": 4, "precision": "mixed", "items_per_launch": 96000, "source_sha256": sha,
         "traffic_bytes_per_launch": 500, "calls": 10, "companion": False},
        {"stage": "simple_update", "chi": 4, "precision": "mixed", "items_per_launch": 96000,
         "source_sha256": sha, "traffic_bytes_per_launch": 1000, "calls": 40, "companion": False},
        {"stage": "simple_update", "chi": 4, "precision": "mixed", "items_per_launch": 96000,
         "source_sha256": sha, "traffic_bytes_per_launch": 8, "calls": 40, "companion": True},
    ]}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(bench, "_source_sha", lambda: sha)
    assert bench.measured_traffic("bp_sweep", 4, "mixed", 96000) == 350
    assert bench.measured_traffic("simple_update", 4, "mixed", 96000) == 1008
    assert bench.measured_traffic("gauge_apply", 4, "mixed", 96000) is None


def test_profile_companion_kernels():
    # kernels that run beside their stage's main launch (their traffic adds
    # up) against alternatives (weighted by calls)
    from paper_2409_12240_amd.rocprof_summary import is_companion
    assert is_companion("void gtqa::k_simple_update<4, float, 4, true>(gtqa::DevPool, int const*, int)")
    assert not is_companion("void gtqa::k_simple_update<4, float, 4, false>(gtqa::DevPool, int const*, int)")
    assert is_companion("void gtqa::k16_su_core<16, float>(gtqa::DevPool, int const*, int)")
    assert is_companion("void gtqa::k16_su_apply<16, float>(gtqa::DevPool, int const*, int)")
    assert not is_companion("void gtqa::k16_su_qr<16, float>(gtqa::DevPool, int const*, int)")
    assert not is_companion("void gtqa::k_bp_class<4, float, true, false, true>(gtqa::DevPool, "
                            "HIP_vector_type<int, 4u> const*, int, int, int const*)")


def test_tuning_knobs(g):
    old = g.get_tuning()
    try:
        g.set_tuning("xcd_contiguous", 1)
        g.set_tuning("su_edges_per_wave_chi4", 2)
        g.set_tuning("canon_lanes_chi4", 8)
        assert g.get_tuning() == {"su_edges_per_wave_chi4": 2, "xcd_contiguous": 1, "canon_lanes_chi4": 8}
        lib = g.load_library()
        assert lib.gtqa_set_tuning(0, 3) == g.GTQA_ERR_ARG
        assert lib.gtqa_set_tuning(1, 2) == g.GTQA_ERR_ARG
        assert lib.gtqa_set_tuning(2, 6) == g.GTQA_ERR_ARG
        assert lib.gtqa_set_tuning(7, 0) == g.GTQA_ERR_ARG
    finally:
        for k, v in old.items():
            g.set_tuning(k, v)


def test_spectral_bipartition_matches_oracle(g):
    from oracle import entropy as H
    # the weakly joined halves and random 3-regular graphs: the same side
    # (the Fiedler order decides it; eigenvalue ties would not)
    a = random_regular_instance(7, 20)
    b = random_regular_instance(8, 20)
    ea = [tuple(x) for x in a.edges.tolist()]
    eb = [tuple(x) for x in b.edges.tolist()]
    (u1, v1), (u2, v2) = ea.pop(0), eb.pop(0)
    edges = sorted((min(u, v), max(u, v)) for u, v in ea + [(u + 20, v + 20) for u, v in eb]
                   + [(u1, u2 + 20), (v1, v2 + 20)])
    side, cut = g.spectral_bipartition(40, np.array(edges))
    assert np.array_equal(side, H.spectral_bipartition(40, edges)) and cut == 2
    for seed, n in ((1, 16), (2, 100), (3, 250), (1000, 1000)):
        inst = random_regular_instance(seed, n)
        side, cut = g.spectral_bipartition(n, inst.edges)
        ref = H.spectral_bipartition(n, inst.edges)
        assert np.array_equal(side, ref), (seed, n)
        assert cut == len(H.cut_edges(inst.edges, ref))
