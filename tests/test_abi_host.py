"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates configurations without touching a GPU."""
import os
import re

import numpy as np
import pytest

import paper_2105_05821_amd as sn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "simnet.h")).read()
    return set(re.findall(r"^SIMNET_API\s+[\w\s\*]*?\b(\w+)\s*\(", text, re.M))


def test_header_and_binding_agree():
    assert declared_symbols() == set(sn.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = sn.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_peak_probe_library_loads():
    """The measurement probes (bench.py --peaks) are a library of their own
    with the two documented entry points; argument checks run on the host."""
    import ctypes as C
    L = C.CDLL(os.path.join(ROOT, "paper_2105_05821_amd", "libsimnet_peaks.so"))
    ms = C.c_float(0.0)
    assert L.peaks_mfma(7, 1, 1, None, None, None, C.byref(ms)) == -1  # bad form
    assert L.peaks_hbm(None, None, C.c_int64(16), 0, 1, 1, None, C.byref(ms)) == -1


def good(n_sub=4, n_instr=1000, feat_ptr=0x1000):
    cfg = sn.make_config(50, 111, (47, 48, 49))
    s, l, w = sn.partition(n_instr, n_sub, 256)
    return cfg, sn.make_trace(feat_ptr, n_instr, s, l, w)


def test_validate_accepts_good_config():
    cfg, tr = good()
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_OK


@pytest.mark.parametrize("field,value", [("n_out", 4), ("n_out", 1), ("retire_width", 0),
                                         ("retire_width", 17), ("col_res", 50), ("col_exe", 47),
                                         ("lat_max", 0), ("prec", 7), ("n_slot", 1)])
def test_validate_rejects_bad_config(field, value):
    cfg, tr = good()
    setattr(cfg, field, value)
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_EINVAL


def test_validate_store_latency_config():
    """n_out = 3 (store latencies) needs a store flag column in range and
    lat_max <= 65535; with n_out = 2 store_col is ignored."""
    cfg, tr = good()
    cfg.store_col = 77
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_OK
    cfg.n_out = 3
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_EINVAL
    cfg.store_col = 2
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_OK
    cfg.lat_max = 65536
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_EINVAL


def test_validate_rejects_bad_trace():
    cfg, _ = good()
    s, l, w = sn.partition(1000, 4, 256)
    assert sn.sim_validate_config(cfg, sn.make_trace(None, 1000, s, l, w)) == sn.SIM_EINVAL
    bad_len = l.copy(); bad_len[2] = 0
    assert sn.sim_validate_config(cfg, sn.make_trace(0x1000, 1000, s, bad_len, w)) == sn.SIM_EINVAL
    bad_warm = w.copy(); bad_warm[1] = s[1] + 1
    assert sn.sim_validate_config(cfg, sn.make_trace(0x1000, 1000, s, l, bad_warm)) == sn.SIM_EINVAL
    over = l.copy(); over[-1] += 1
    assert sn.sim_validate_config(cfg, sn.make_trace(0x1000, 1000, s, over, w)) == sn.SIM_EINVAL
    assert sn.sim_validate_config(cfg, sn.make_trace(0x1000, 1 << 31, s, l, w)) == sn.SIM_EINVAL


def test_partition_matches_oracle(oracle_lib):
    """sim_partition (library, host) against the oracle's partition."""
    for N, K, wm in [(1_000_000, 4096, 256), (10, 3, 0), (1000, 7, 300), (5, 5, 2),
                     (748_000_123, 20_000, 256), (1, 1, 9)]:
        a = sn.partition(N, K, wm)
        b = oracle_lib.partition(N, K, wm)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_partition_rejects_bad_arguments():
    for N, K, wm in [(10, 0, 0), (3, 4, 0), (10, 2, -1), (0, 1, 0)]:
        with pytest.raises(ValueError):
            sn.partition(N, K, wm)
    z = np.zeros(2, np.int64)
    assert sn.lib().sim_partition(10, 2, 0, None, z.ctypes.data, z.ctypes.data) == sn.SIM_EINVAL


def test_product_does_not_import_oracle():
    """The product package must not reach the oracle or any CPU fallback."""
    src_dir = os.path.join(ROOT, "paper_2105_05821_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "simnet_oracle" not in text, f


def test_validate_dependency_flag_config():
    """col_dep: 5 columns inside the window, not over a dynamic column, and
    the trace's addresses given."""
    cfg, tr = good()
    cfg.col_dep = 42
    assert sn.sim_validate_config(cfg, tr) == sn.SIM_EINVAL  # no addresses
    s, l, w = sn.partition(100_000, 64, 256)
    tr2 = sn.make_trace(0x1000, 100_000, s, l, w, mem_ptr=0x2000)
    assert sn.sim_validate_config(cfg, tr2) == sn.SIM_OK
    cfg.col_dep = 46                                     # 46..50: past the window
    assert sn.sim_validate_config(cfg, tr2) == sn.SIM_EINVAL
    cfg.col_dep = 44                                     # 44..48 covers residence (47)
    assert sn.sim_validate_config(cfg, tr2) == sn.SIM_EINVAL


def test_noalloc_limit_matches_header():
    text = open(os.path.join(ROOT, "include", "simnet.h")).read()
    m = re.search(r"#define\s+SIM_NOALLOC_MAX_B\s+(\d+)", text)
    assert m and int(m.group(1)) == sn.NOALLOC_MAX_B
