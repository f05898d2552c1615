"""Host-side checks of the C ABI library (no GPU needed): it loads, it
exports every function declared in include/peps_env.h, and its error paths
that need no device behave."""
import ctypes as C
import os
import re

import pytest

from paper_1311_6696_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "peps_env.h")).read()
    return sorted(set(re.findall(r"^\s*(?:peps_status|void|const char\*)\s+(peps_\w+)\s*\(", text, re.M)))


def test_header_lists_the_abi():
    names = declared_functions()
    for n in ("peps_env_boundary", "peps_cluster_env", "peps_expect", "peps_ctx_create", "peps_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libpepsenv.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(binding.SYMBOLS)


def test_null_arguments_are_rejected_without_a_device():
    lib = binding.load()
    lib.peps_env_free(None)
    lib.peps_ctx_destroy(None)
    assert lib.peps_env_info(None, None, None, None, None, None) == -1
    assert b"must not be NULL" in lib.peps_last_error()
    assert lib.peps_expect(None, None, 0, None) == -1
    assert lib.peps_env_boundary(None, None, 0, None, None) == -1
    assert lib.peps_cluster_env(None, None, 0, None, 0, None, None) == -1
    assert lib.peps_ctx_graphs(None, 1) == -1
    assert lib.peps_ctx_autotune(None, 1) == -1
    assert lib.peps_ctx_stats(None, None, None, None, None) == -1
    assert lib.peps_qr(None, None, 0) == -1
    assert lib.peps_site_env(None, None, 0, None) == -1
    assert lib.peps_bond_env(None, None, 0, None) == -1
    assert lib.peps_boundary_overlap(None, None, 0) == -1
    assert lib.peps_bond_fit(None, None, 0, None) == -1


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(OSError):
        binding.load(str(tmp_path / "nope.so"))


def test_struct_layouts_match_header():
    # sizes of the records shared with C (x86-64 ABI)
    assert C.sizeof(binding.State) == 4 * 3 + 4 + 8 + 8
    assert C.sizeof(binding.Opts) == 4 * 4 + 8 + 2 * 4 + 8
    assert C.sizeof(binding.Window) == 7 * 4
    assert C.sizeof(binding.Result) == 5 * 8
    assert C.sizeof(binding.SiteReq) == 8 + 4 * 4 + 3 * 8   # r, c, dir and padding
    assert C.sizeof(binding.BondReq) == 8 + 4 * 4 + 3 * 8
    assert C.sizeof(binding.OverlapReq) == 2 * 8 + 2 * 4 + 3 * 8
    assert C.sizeof(binding.FitReq) == 8 + 4 * 4 + 7 * 8


def test_statistics_table_size_matches_header():
    """The binding's statistics arrays have the size the header declares
    (the library writes that many entries)."""
    text = open(os.path.join(ROOT, "include", "peps_env.h")).read()
    n = int(re.search(r"#define PEPS_N_STATS (\d+)", text).group(1))
    assert binding.N_STATS == n
    assert len(binding.TILES) * 6 == n


def test_option_flags_match_header():
    text = open(os.path.join(ROOT, "include", "peps_env.h")).read()
    assert binding.OPTS_PER_STATE == int(re.search(r"#define PEPS_OPTS_PER_STATE (\d+)", text).group(1))
    assert binding.OPTS_COLUMNS == int(re.search(r"#define PEPS_OPTS_COLUMNS (\d+)", text).group(1))
    assert binding.OPTS_STRICT == int(re.search(r"#define PEPS_OPTS_STRICT (\d+)", text).group(1))
    flags = (binding.OPTS_PER_STATE, binding.OPTS_COLUMNS, binding.OPTS_STRICT)
    assert all(a & b == 0 for i, a in enumerate(flags) for b in flags[i + 1:])


def test_status_codes_match_header():
    text = open(os.path.join(ROOT, "include", "peps_env.h")).read()
    for code, name in binding.STATUS.items():
        if code:
            assert int(re.search(r"PEPS_ERR_%s = (-\d+)" % name, text).group(1)) == code, name
