"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/bsw.h declares, and reports the absence of a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bsw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsw_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("bsw_ctx_create", "bsw_ctx_destroy", "bsw_extend_batch",
                 "bsw_extend_batch_device", "bsw_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1907_12931_amd import bsw
    lib = bsw.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.bsw_abi_version() == 1


def test_no_gpu_gives_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1907_12931_amd import bsw
    with pytest.raises(bsw.BswError) as ei:
        bsw.Context()
    assert ei.value.code == bsw.EDEVICE


def test_params_layout():
    from paper_1907_12931_amd import bsw
    import oracle
    assert ctypes.sizeof(bsw.Params) == 56 == ctypes.sizeof(oracle.Params)
    assert bsw.RESULT_DTYPE.itemsize == 24 and bsw.DIAG_DTYPE.itemsize == 16


def test_server_without_gpu_gives_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1907_12931_amd import bsw, synth
    with pytest.raises(bsw.BswError) as ei:
        bsw.Server([synth.BWA_DEFAULT])
    assert ei.value.code == bsw.EDEVICE


def test_struct_layouts_match_header():
    """The binding's ctypes mirrors have the header's sizes and offsets."""
    from paper_1907_12931_amd import bsw
    assert ctypes.sizeof(bsw.ServerOpts) == 32
    assert bsw.ServerOpts.max_batch_pairs.offset == 8
    assert ctypes.sizeof(bsw.ServerReport) == 6 * 8 + 9 * 8
    assert bsw.CtxOpts.no_graph.offset == 32


def test_seed_layouts_match_header(tmp_path):
    """bsw_seed / bsw_seed_result as a C compiler lays them out equal the
    binding's and the reference's record types, field by field."""
    from paper_1907_12931_amd import bsw, synth
    from oracle import seeds as oseeds
    src = tmp_path / "lay.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "bsw.h"\n'
                   'int main(void) {\n'
                   '  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(bsw_seed),'
                   ' offsetof(bsw_seed, read), offsetof(bsw_seed, qb), offsetof(bsw_seed, qe),'
                   ' offsetof(bsw_seed, h0), offsetof(bsw_seed, rb));\n'
                   '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(bsw_seed_result),'
                   ' offsetof(bsw_seed_result, score), offsetof(bsw_seed_result, qbeg),'
                   ' offsetof(bsw_seed_result, qend), offsetof(bsw_seed_result, how),'
                   ' offsetof(bsw_seed_result, rbeg), offsetof(bsw_seed_result, rend));\n'
                   '  return 0;\n}\n')
    exe = tmp_path / "lay"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True,
                           text=True).stdout.split("\n")
    seed = [int(x) for x in lines[0].split()]
    res = [int(x) for x in lines[1].split()]
    for dt in (bsw.SEED_DTYPE, synth.SEED_FIELDS, oseeds.SEED_DTYPE):
        assert [dt.itemsize] + [dt.fields[f][1] for f in dt.names] == seed
    for dt in (bsw.SEED_RESULT_DTYPE, oseeds.SEED_RESULT_DTYPE):
        assert [dt.itemsize] + [dt.fields[f][1] for f in dt.names] == res
    assert (bsw.END_LOCAL, bsw.END_READ, bsw.END_NONE) == (
        oseeds.LOCAL, oseeds.READ_END, oseeds.NONE)
