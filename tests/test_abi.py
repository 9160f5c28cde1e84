"""The C-ABI library loads and exports every function include/simrank.h declares, and the
ctypes structures match the C layout (sizes and offsets compiled from the header by gcc).
No GPU work is launched."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simrank.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", text)
    skip = {"if", "while", "for", "switch", "return", "sizeof"}
    decl = set()
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                         text, flags=re.M):
        if m.group(1) not in skip:
            decl.add(m.group(1))
    assert decl and decl <= set(names)
    return sorted(decl)


def lib():
    from paper_1711_00121_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported():
    L = lib()
    names = declared_functions()
    assert "init_simrank" in names and "backward" in names and "apply_batch" in names
    for name in names:
        assert hasattr(L, name), name
    from paper_1711_00121_amd import _lib
    assert set(_lib.SIGNATURES) == set(names)


def test_default_config_and_strerror():
    from paper_1711_00121_amd import _lib
    L = lib()
    cfg = _lib.sr_config()
    assert L.sr_default_config(ctypes.byref(cfg)) == 0
    assert cfg.C == 0.6 and cfg.K == 15 and cfg.K_ps == 30 and cfg.prune == 1
    assert cfg.init_tol == 1e-15 and cfg.batch_chunk == 0 and cfg.split_rows == 8192
    assert cfg.profile == 0 and cfg.graphs == 1 and cfg.tile_skip == 1 and cfg.block_store == 0
    assert L.sr_strerror(-3) == b"edge exists"
    assert L.sr_default_config(None) == _lib.SR_EINVAL


def test_null_context_arguments_are_rejected_without_gpu():
    from paper_1711_00121_amd import _lib
    L = lib()
    assert L.apply_edge_update(None, 0, 1, 1, None) == _lib.SR_EINVAL
    assert L.sr_destroy(None) == _lib.SR_OK
    assert L.init_simrank(None, 10, 0, None, None, None, None, None, None) == _lib.SR_EINVAL
    assert L.init_simrank_tree(None, 10, 0, None, None, None, None, None) == _lib.SR_EINVAL
    assert L.sr_get_config(None, None) == _lib.SR_EINVAL


def test_chunk_bound_is_refused_before_any_gpu_work():
    """batch_chunk above 65,535 (one grid row per deferred block in the per-pass kernels) and a
    tile_skip other than 0 or 1 are validation errors of the configuration, reported before the
    device is touched."""
    import ctypes as C
    import numpy as np
    from paper_1711_00121_amd import _lib
    L = lib()
    cfg = _lib.sr_config()
    assert L.sr_default_config(C.byref(cfg)) == _lib.SR_OK
    src = np.asarray([0, 1], dtype=np.int32)
    dst = np.asarray([1, 2], dtype=np.int32)
    for field, bad in (("batch_chunk", 65536), ("tile_skip", 2), ("tile_skip", -1)):
        assert L.sr_default_config(C.byref(cfg)) == _lib.SR_OK
        setattr(cfg, field, bad)
        h = C.c_void_p()
        st = L.init_simrank(C.byref(h), 3, 2, src.ctypes.data_as(C.POINTER(C.c_int32)),
                            dst.ctypes.data_as(C.POINTER(C.c_int32)), None, C.byref(cfg), None,
                            None)
        assert st == _lib.SR_EINVAL and not h.value, (field, bad)


def test_device_bytes_without_contexts():
    """No context allocates on a host without a GPU: the library holds nothing."""
    from paper_1711_00121_amd import device_bytes
    assert device_bytes() == (0, 0)
    assert device_bytes(reset_peak=True) == (0, 0)


def test_struct_layout_matches_header():
    from paper_1711_00121_amd import _lib
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "simrank.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("sr_config %zu\n", sizeof(sr_config));
  printf("sr_update_stats %zu\n", sizeof(sr_update_stats));
  printf("sr_batch_stats %zu\n", sizeof(sr_batch_stats));
  F(sr_config, node_cap) F(sr_config, init_tol) F(sr_config, fused_batch)
  F(sr_config, split_rows) F(sr_config, profile)
  F(sr_update_stats, bound) F(sr_batch_stats, pairs) F(sr_batch_stats, fused_passes)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        r = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("gcc unavailable: " + r.stderr)
        out = subprocess.run([exe], capture_output=True, text=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    assert int(got["sr_config"]) == ctypes.sizeof(_lib.sr_config)
    assert int(got["sr_update_stats"]) == ctypes.sizeof(_lib.sr_update_stats)
    assert int(got["sr_batch_stats"]) == ctypes.sizeof(_lib.sr_batch_stats)
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(getattr(_lib, t), f).offset == int(val), key


def test_simrank_pairs_refuses_other_weights_before_any_gpu_work():
    """SimRankPairs checks the weights against the context's before touching the device."""
    import numpy as np
    import torch

    from paper_1711_00121_amd import simrank_pairs

    class Ctx:
        m0 = 4
        weights = np.array([1.0, 2.0, 0.5, 1.5])

    with pytest.raises(ValueError):
        simrank_pairs(torch.tensor([1.0, 2.0, 0.5, 1.25], dtype=torch.float64), Ctx(), [0], [1])
    with pytest.raises(ValueError):
        simrank_pairs(torch.ones(3, dtype=torch.float64), Ctx(), [0], [1])

    class Unweighted:
        m0 = 3
        weights = None

    with pytest.raises(ValueError):
        simrank_pairs(torch.tensor([1.0, 1.0, 2.0], dtype=torch.float64), Unweighted(), [0],
                      [1])
