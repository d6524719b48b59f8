"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no compute calls)."""
import ctypes

import pytest

from paper_2210_08580_amd import binding


def test_header_declares_the_pipeline():
    syms = binding.header_symbols()
    for s in ("fds_ctx_create", "fds_assemble", "fds_filter", "fds_compress", "fds_factor",
              "fds_rhs_planewave", "fds_solve", "fds_sync", "fds_last_error", "fds_op_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    import os
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libfds.so not built")
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [s for s in binding.header_symbols() if not hasattr(L, s)]
    assert not missing, missing
    # the binding's signature table covers the whole header
    assert set(binding.header_symbols()) <= set(binding._SIGS)


def test_last_error_is_empty_string_initially():
    import os
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libfds.so not built")
    assert isinstance(binding.lib().fds_last_error(), bytes)
