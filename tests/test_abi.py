"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/gsl_lpa.h declares, rejects bad arguments before any
device work, and computes the convergence limit exactly as the literal
dN / N <= tau test of Alg. 3."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsl_lpa.h")


def _lib():
    import paper_2403_01261_amd as gsl
    if not os.path.exists(gsl.LIB_PATH):
        pytest.skip("libgsl_lpa.so not built")
    return gsl, gsl.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for required in ("gsl_lpa", "gsl_split", "gsl_modularity"):
        assert required in names


def test_library_exports_every_declared_symbol():
    _, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_are_reported_without_device_work():
    gsl, lib = _lib()
    assert lib.gsl_lpa(None, None, None, -1, 20, 0.05, None) == gsl.GSL_EINVAL
    assert b"out of range" in lib.gsl_last_error()
    assert lib.gsl_lpa(None, None, None, 5, -1, 0.05, None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa(None, None, None, 5, 20, 1.5, None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa(None, None, None, 5, 20, float("nan"), None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa(None, None, None, 1 << 31, 20, 0.05, None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa(None, None, None, 0, 20, 0.05, None) == gsl.GSL_OK  # n = 0: no-op
    assert lib.gsl_lpa_f32(None, None, None, -1, 20, 0.05, None, None, None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa_f32(None, None, None, 0, 20, 0.05, None, None, None) == gsl.GSL_OK
    assert lib.gsl_lpa_f32(None, None, None, 5, 20, 2.0, None, None, None) == gsl.GSL_EINVAL
    assert lib.gsl_split(None, None, 0, None, None) == gsl.GSL_OK
    assert lib.gsl_split(None, None, 3, None, None) == gsl.GSL_EINVAL
    assert lib.gsl_modularity(None, None, None, 0, None, None) == gsl.GSL_EINVAL
    q = ctypes.c_double(7.0)
    assert lib.gsl_modularity(None, None, None, 0, None, ctypes.byref(q)) == gsl.GSL_OK
    assert q.value == 0.0


def test_batched_argument_errors_without_device_work():
    gsl, lib = _lib()
    assert lib.gsl_lpa_batched(-1, None, None, None, None, None, 20, 0.05, None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa_batched(0, None, None, None, None, None, 20, 0.05, None) == gsl.GSL_OK
    assert lib.gsl_lpa_batched(3, None, None, None, None, None, -1, 0.05, None) == gsl.GSL_EINVAL
    assert lib.gsl_lpa_batched(3, None, None, None, None, None, 20, -0.5, None) == gsl.GSL_EINVAL
    G = 3
    tab = (gsl._Graph * G)()
    iters = (ctypes.c_int32 * G)(7, 7, 7)
    # only empty graphs: nothing to do, every sweep count is 0
    assert lib.gsl_lpa_graphs(None, G, tab, 20, 0.05, None, None, iters, None) == gsl.GSL_OK
    assert list(iters) == [0, 0, 0]
    tab[1].n = -2
    assert lib.gsl_lpa_graphs(None, G, tab, 20, 0.05, None, None, iters, None) == gsl.GSL_EINVAL
    assert b"n out of range" in lib.gsl_last_error()
    tab[1].n = 4  # offsets / labels_out missing
    assert lib.gsl_lpa_graphs(None, G, tab, 20, 0.05, None, None, iters, None) == gsl.GSL_EINVAL
    tab[1].n = 1 << 30
    tab[2].n = 1 << 30
    tab[1].offsets = tab[2].offsets = 8
    tab[1].labels_out = tab[2].labels_out = 8
    assert lib.gsl_lpa_graphs(None, G, tab, 20, 0.05, None, None, iters, None) == gsl.GSL_EINVAL
    assert b"total vertex count" in lib.gsl_last_error()
    assert lib.gsl_lpa_graphs(None, 1, None, 20, 0.05, None, None, None, None) == gsl.GSL_EINVAL
    assert lib.gsl_context_create(None) == gsl.GSL_EINVAL
    assert lib.gsl_context_set_stream(None, None) == gsl.GSL_EINVAL
    lib.gsl_context_destroy(None)
    assert ctypes.sizeof(gsl._Graph) == 40
    assert lib.gsl_check_graph(None, None, -1) == gsl.GSL_EINVAL
    assert lib.gsl_check_graph(None, None, 0) == gsl.GSL_OK
    assert lib.gsl_check_graph(None, None, 4) == gsl.GSL_EINVAL
    cnt = ctypes.c_int64(5)
    assert lib.gsl_disconnected(None, None, 0, None, None, ctypes.byref(cnt)) == gsl.GSL_OK
    assert cnt.value == 0
    assert lib.gsl_disconnected(None, None, -3, None, None, None) == gsl.GSL_EINVAL
    assert lib.gsl_disconnected(None, None, 3, None, None, None) == gsl.GSL_EINVAL
    r = ctypes.c_int32(9)
    assert lib.gsl_split_ex(None, None, 0, None, None, 0, ctypes.byref(r), None) == gsl.GSL_OK
    assert r.value == 0
    assert lib.gsl_split_ex(None, None, 0, None, None, 7, None, None) == gsl.GSL_EINVAL
    assert lib.gsl_split_ex(None, None, 4, None, None, 1, None, None) == gsl.GSL_EINVAL


def _literal_limit(n, tol):
    ks = [k for k in range(n + 1) if k / n <= tol] if n > 0 else [0]
    return max(ks) if ks else -1


def test_convergence_limit_matches_literal_predicate():
    gsl, _ = _lib()
    rng = np.random.default_rng(0)
    for n in list(range(1, 60)) + [10_000, 24_000_000 // 1000]:
        tols = [0.0, 0.05, 1 / 3, 0.5, 1.0, 1 / n, 2 / n, 0.1 + 1e-17] + list(rng.random(5))
        for tol in tols:
            if not 0.0 <= tol <= 1.0:
                assert gsl.gsl_convergence_limit(n, tol) == -1
                continue
            assert gsl.gsl_convergence_limit(n, tol) == _literal_limit(n, tol), (n, tol)
    assert gsl.gsl_convergence_limit(10_000, 0.05) == 500
    assert gsl.gsl_convergence_limit(0, 0.05) == 0
    assert gsl.gsl_convergence_limit(10, -0.1) == -1


def test_convergence_limit_large_n_boundaries():
    gsl, _ = _lib()
    for n in (4_194_304, 24_000_000, 67_108_864, (1 << 31) - 1):
        for tol in (0.05, 0.1, 1 / 3, 0.0, 1.0):
            k = gsl.gsl_convergence_limit(n, tol)
            assert k / n <= tol
            assert k == n or not ((k + 1) / n <= tol)


def test_default_tiers_match_the_tuner_and_any_variant_serves_any_level():
    """gsl_set_tiers / gsl_get_tiers are host-only: the library's default
    table is the autotuner's first starting point, and a thread-per-vertex
    variant may serve a later level (bounds only need to fit capacities)."""
    gsl, _ = _lib()
    from paper_2403_01261_amd import tune
    try:
        gsl.gsl_set_tiers(None)
        assert gsl.gsl_get_tiers() == tune.DEFAULT_LEVELS
        gsl.gsl_set_tiers(tune.FINE_LEVELS)
        assert gsl.gsl_get_tiers() == tune.FINE_LEVELS
        with pytest.raises(gsl.GslError):
            gsl.gsl_set_tiers([(8, 0), (64, 16), (128, 8), (512, 9), (2048, 11), (4096, 13), (4096, 13)])
    finally:
        gsl.gsl_set_tiers(None)


def test_variant_menu_matches_the_tuner_tests():
    """gsl_tier_variant (host-only) reports the menu the autotuner's CPU tests
    model: same order, lanes per vertex and capacities."""
    gsl, _ = _lib()
    from tests.test_tune import VARIANTS
    menu = gsl.gsl_tier_variants()
    assert len(menu) == len(VARIANTS)
    for a, b in zip(menu, VARIANTS):
        assert (a["group"], a["capacity"]) == (b["group"], b["capacity"])
