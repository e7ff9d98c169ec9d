"""C-ABI library checks that need no GPU: it loads, exports every entry point
declared in include/*.h, and its host front-end (layout graph of Sec. 2.1)
agrees with the oracle's."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(mpld_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_2303_14335_amd import _ffi
    lib = ctypes.CDLL(_ffi.LIB_PATH)
    decl = declared_functions()
    assert len(decl) >= 20
    missing = [n for n in decl if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for every one of them
    assert set(decl) <= set(_ffi.SIGNATURES)


def test_abi_version_and_error_strings():
    import paper_2303_14335_amd as mp
    assert mp.mpld_abi_version() == 3
    lib = mp._lib
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.mpld_error_string(code)
    assert lib.mpld_error_string(-99) == b"unknown error code"


@pytest.mark.parametrize("n,side,dmin,split,seed", [(300, 3000, 80, 0, 0), (3000, 9000, 120, 120, 1),
                                                    (5000, 6000, 100, 0, 2), (20000, 30000, 80, 0, 3),
                                                    # sparse: the grid cells grow; dense: crowded cells
                                                    (2000, 400000, 80, 0, 4), (6000, 4500, 150, 100, 5),
                                                    # several scan threads and stitch pairs
                                                    (40000, 40000, 100, 90, 6)])
def test_front_end_graph_matches_oracle(n, side, dmin, split, seed):
    import paper_2303_14335_amd as mp
    rects, _ = workload.generate(n, side, seed)
    g = mp.mpld_build_graph(rects, dmin, split)
    ref = oracle.build_graph(rects, dmin, split)
    assert g.num_nodes == ref.num_nodes
    assert np.array_equal(g.ce, ref.ce)
    assert np.array_equal(g.se, ref.se)


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_front_end_graph_matches_oracle_full_configs(cfg):
    """The host graph builder (several scan threads) against the oracle's
    own builder at the full sizes of the 200k-rect and 40k-rect workloads."""
    import paper_2303_14335_amd as mp
    from workload.configs import CONFIGS
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    ref = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    assert g.num_nodes == ref.num_nodes
    assert np.array_equal(g.ce, ref.ce)
    assert np.array_equal(g.se, ref.se)
    assert len(ref.ce) > 100000


def test_front_end_rejects_bad_boxes():
    import paper_2303_14335_amd as mp
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_build_graph(np.array([[10, 0, 5, 20]]), 80)
    assert e.value.code == -1


def test_front_end_empty_layout():
    import paper_2303_14335_amd as mp
    g = mp.mpld_build_graph(np.zeros((0, 4), np.int32), 80)
    assert g.num_nodes == 0 and len(g.ce) == 0


def test_no_device_is_a_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_2303_14335_amd as mp
    with pytest.raises(mp.MpldError) as e:
        mp.Context(0, use_torch=False)
    assert e.value.code == -3


def test_measurement_entry_points_reject_bad_arguments_before_any_device_call():
    # argument checks come first, so these hold with no GPU: a NULL context
    # or output is MPLD_E_INVALID, with the reason in the last error
    import paper_2303_14335_amd as mp
    lib = mp._lib
    out = ctypes.c_double()
    for fn in (lib.mpld_measure_launch_floor, lib.mpld_measure_touch_floor):
        assert fn(None, 868, 256, 10, ctypes.byref(out)) == -1
        assert b"NULL" in lib.mpld_last_error()
        assert fn(None, 868, 256, 10, None) == -1
    assert lib.mpld_measure_lds_read_rate(None, 16, 100, ctypes.byref(out), None) == -1
