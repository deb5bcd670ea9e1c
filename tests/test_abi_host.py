"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
declared symbol, sizes follow the closed forms, and errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import made as omade
from oracle import slater_condon as osc
from paper_2506_07430_amd import elocal, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "elocal.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(elocal_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = elocal.lib()
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(elocal.exported_symbols())


@pytest.mark.parametrize("n,widths", [(8, (32,)), (24, (128, 128)), (40, (256, 256, 256)), (60, (256, 256, 256))])
def test_num_params_closed_form(n, widths):
    assert elocal.num_params(n, widths) == omade.num_params(n, widths) == synth.num_params(n, widths)


def test_num_params_rejects_bad_shapes():
    w = (ctypes.c_int * 1)(32)
    assert elocal.lib().elocal_num_params(1, 1, w) == -1
    assert elocal.lib().elocal_num_params(65, 1, w) == -1
    assert elocal.lib().elocal_num_params(8, 0, w) == -1


def test_create_without_device_reports_device_error():
    if os.environ.get("HIP_VISIBLE_DEVICES", None) != "" and _has_gpu():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = elocal.lib().elocal_create(np.zeros(4).ctypes.data, np.zeros(16).ctypes.data, 2, 1, 1, ctypes.byref(h))
    assert st == 5
    assert b"device" in elocal.lib().elocal_last_error()


def test_invalid_arguments_before_device_checks():
    L = elocal.lib()
    h = ctypes.c_void_p()
    assert L.elocal_create(None, None, 8, 4, 4, ctypes.byref(h)) == 1
    assert L.elocal_create(np.zeros(1).ctypes.data, np.zeros(1).ctypes.data, 1, 1, 1, ctypes.byref(h)) == 6
    assert L.elocal_create(np.zeros(4).ctypes.data, np.zeros(16).ctypes.data, 2, 3, 1, ctypes.byref(h)) == 1
    assert L.elocal_num_connected(None) == -1
    assert L.elocal_words(None) == -1
    assert L.elocal_workspace_bytes(None, None, 10, 0) == 0
    assert b"null" in L.elocal_last_error()
    assert L.elocal_stats(None, None, None, 0, None) == 1
    assert L.elocal_destroy(None) == 1


def test_closed_form_counts_match_oracle_enumeration():
    for n, na, nb in [(8, 4, 4), (24, 12, 12), (40, 14, 14), (60, 26, 26), (64, 32, 32), (33, 0, 33)]:
        va, vb = n - na, n - nb
        C = 1 + na * va + nb * vb + na * (na - 1) // 2 * va * (va - 1) // 2 \
            + nb * (nb - 1) // 2 * vb * (vb - 1) // 2 + na * va * nb * vb
        assert C == osc.num_connected(n, na, nb)
        assert C < 2 ** 32


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_autotune_search_and_cache_on_host(tmp_path):
    """The coordinate search and the JSON cache (no GPU): the search starts at the built-in
    shape, walks each dimension with the others held at the best so far, stops at the
    budget; the cache round-trips and keeps other entries."""
    from paper_2506_07430_amd import autotune
    cost = {"cols": {0: 3.0, 1: 3.0, 2: 2.0}, "waves": {0: 0.0, 8: 1.0}, "groups": {0: 0.5, 4: 0.0, 16: 0.7},
            "grid": {0: 0.2, 512: 0.0}}

    def timed(shape):
        return 10.0 + sum(cost[k][shape[k]] for k in cost)

    table = autotune._search({"cols": [0, 1, 2], "waves": [0, 8], "groups": [0, 4, 16], "grid": [0, 512]}, timed, 1e9)
    best = min(table, key=lambda r: r["ms"])
    assert table[0]["shape"] == {"grid": 0, "groups": 0, "waves": 0, "cols": 0}
    assert best["shape"] == {"grid": 512, "groups": 4, "waves": 0, "cols": 2}
    assert len({tuple(sorted(r["shape"].items())) for r in table}) == len(table)
    short = autotune._search({"cols": [0, 1, 2], "waves": [0, 8]}, timed, 0.0)
    assert len(short) == 1
    path = str(tmp_path / "c.json")
    autotune.store_cache("a", {"shape": {"grid": 1}}, path)
    autotune.store_cache("b", {"shape": {"grid": 2}}, path)
    assert autotune.load_cache(path) == {"a": {"shape": {"grid": 1}}, "b": {"shape": {"grid": 2}}}
