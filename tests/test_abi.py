"""The C-ABI library loads and exports every symbol its headers declare;
host-side argument checks work without a device."""
import ctypes
import glob
import os
import re

import pytest

from paper_1606_07550_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(tricc_\w+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = N.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), f"{name} declared but not exported"


def test_binding_covers_header():
    assert set(declared_functions()) <= set(N._SIGS) | set(getattr(N, "_EXTRA_SIGS", {}))


def test_status_strings():
    for s in range(7):
        assert N.status_str(s)
    assert N.status_str(99) == "unknown status"


def test_default_tuning_is_consistent():
    from paper_1606_07550_amd import default_tuning, variant_capacity, variant_count
    t = default_tuning()
    assert variant_count() >= 6
    for b in range(N.NUM_BINS - 1):
        assert variant_capacity(t.bin_variant[b]) >= t.bin_limit[b]
    # the last bin is unbounded: its default variant accepts any out-degree
    assert variant_capacity(t.bin_variant[N.NUM_BINS - 1]) >= 2 ** 31 - 1
    assert variant_capacity(-1) == -1 and variant_capacity(variant_count()) == -1


def test_workspace_size_checks():
    from paper_1606_07550_amd import workspace_size
    a = workspace_size(1000, 10_000)
    b = workspace_size(2000, 10_000)
    c = workspace_size(1000, 20_000)
    assert 0 < a < b and a < c
    assert workspace_size(0, 0) > 0
    with pytest.raises(N.TriccError) as e:
        workspace_size(-1, 10)
    assert e.value.status == N.TRICC_EINVAL
    with pytest.raises(N.TriccError) as e:
        workspace_size(10, (1 << 30) + 1)
    assert e.value.status == N.TRICC_EOVERFLOW


def test_build_rejects_bad_arguments_before_device_work():
    L = N.lib()
    h = ctypes.c_void_p()
    # null out pointer
    assert L.tricc_graph_build(4, 0, None, None, None, 0, None, None, None) == N.TRICC_EINVAL
    # negative n
    assert L.tricc_graph_build(-3, 0, None, None, None, 0, None, None, ctypes.byref(h)) == N.TRICC_EINVAL
    # missing edge arrays
    assert L.tricc_graph_build(4, 5, None, None, ctypes.c_void_p(256), 1 << 20, None, None,
                               ctypes.byref(h)) == N.TRICC_EINVAL
    # workspace too small
    assert L.tricc_graph_build(4, 0, None, None, ctypes.c_void_p(256), 16, None, None,
                               ctypes.byref(h)) == N.TRICC_ENOMEM
    assert "workspace" in N.last_error()
    # bad tuning
    t = N.Tuning()
    L.tricc_default_tuning(ctypes.byref(t))
    t.bin_variant[2] = 999
    assert L.tricc_graph_build(4, 0, None, None, ctypes.c_void_p(256), 1 << 20, ctypes.byref(t), None,
                               ctypes.byref(h)) == N.TRICC_EINVAL
    assert not h.value


@pytest.mark.parametrize("args", [
    (0, 10, 0.57, 0.19, 0.19, 0.05, 0.1),       # scale below 1
    (31, 10, 0.57, 0.19, 0.19, 0.05, 0.1),      # scale above 30
    (5, -1, 0.57, 0.19, 0.19, 0.05, 0.1),       # negative edge count
    (5, 10, -0.1, 0.5, 0.3, 0.3, 0.1),          # negative weight
    (5, 10, float("inf"), 0.5, 0.3, 0.3, 0.1),  # weight not finite
    (5, 10, 0.0, 0.0, 0.0, 0.0, 0.1),           # weights sum to zero
    (5, 10, 0.57, 0.19, 0.19, 0.05, 1.5),       # noise above 1
    (5, 10, 0.57, 0.19, 0.19, 0.05, float("nan")),
    (5, 10, 0.57, 0.19, 0.19, 0.05, 0.1),       # null outputs with m > 0
])
def test_generator_rejects_bad_arguments_before_device_work(args):
    assert N.lib().tricc_gen_rmat(*args, 0, None, None, None, None) == N.TRICC_EINVAL
    assert N.last_error()


def test_k4_rejects_null_arguments():
    L = N.lib()
    assert L.tricc_graph_count_k4(None, ctypes.c_void_p(256), None) == N.TRICC_EINVAL


def test_min_side_variants_and_tuning_check():
    from paper_1606_07550_amd import default_tuning, variant_count
    L = N.lib()
    ms = [v for v in range(variant_count()) if L.tricc_variant_min_side(v)]
    assert ms == list(range(0, 8)) + list(range(10, 27))
    t = default_tuning()
    assert t.min_side == 1 and all(L.tricc_variant_min_side(t.bin_variant[b]) for b in range(N.NUM_BINS - 1))
    bad = default_tuning()
    bad.bin_variant[1] = 8  # the global fallback has no in-list side
    h = ctypes.c_void_p()
    assert L.tricc_graph_build(4, 0, None, None, ctypes.c_void_p(256), 1 << 30, ctypes.byref(bad), None,
                               ctypes.byref(h)) == N.TRICC_EINVAL
    assert "min_side" in N.last_error()
    bad.min_side = 0
    L.tricc_default_tuning(ctypes.byref(t))


def test_noalloc_limits_are_checked_before_device_work():
    L = N.lib()
    P_ = ctypes.c_void_p(256)
    assert L.tricc_count_noalloc(65537, 0, None, None, P_, P_, P_, P_, None) == N.TRICC_EOVERFLOW
    assert L.tricc_count_noalloc(10, (1 << 20) + 1, P_, P_, P_, P_, P_, P_, None) == N.TRICC_EOVERFLOW
    assert L.tricc_count_noalloc(-1, 0, None, None, P_, P_, P_, P_, None) == N.TRICC_EINVAL
    assert L.tricc_count_noalloc(10, 5, None, None, P_, P_, P_, P_, None) == N.TRICC_EINVAL
    assert L.tricc_count_noalloc(10, 0, None, None, None, P_, P_, P_, None) == N.TRICC_EINVAL
    # the largest graph the fixed array takes fits it
    from paper_1606_07550_amd.graph import workspace_size
    assert workspace_size(65536, 1 << 20) <= 32 << 20
