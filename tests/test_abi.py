"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no compute calls)."""
import ctypes
import os

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


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror of a header struct has the C compiler's size and field
    offsets (compiles the header with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [getattr(binding, n) for n in ("fds_allocator", "fds_asm_opts", "fds_filter_opts", "fds_compress_opts",
                                             "fds_solve_opts", "fds_problem", "fds_batch_opts", "fds_solve_stats")]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fds.h"', "int main(void) {"]
    for st in structs:
        nm = st.__name__
        lines.append(f'printf("{nm} %zu\\n", sizeof({nm}));')
        for f in st._fields_:
            lines.append(f'printf("{nm}.{f[0]} %zu\\n", offsetof({nm}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.dirname(binding.HEADER)
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for st in structs:
        nm = st.__name__
        assert int(got[nm]) == ctypes.sizeof(st), nm
        for f in st._fields_:
            assert int(got[f"{nm}.{f[0]}"]) == getattr(st, f[0]).offset, (nm, f[0])
