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


def test_index_layouts_match_header(tmp_path):
    """bsw_sa_interval, bsw_fm_entry, bsw_fm_meta, bsw_bi_interval and
    bsw_smem as a C compiler lays them out equal the binding's types."""
    import subprocess
    from paper_1907_12931_amd import bsw, synth
    src = tmp_path / "lay2.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "bsw.h"\nint main(void) {\n'
        '  printf("%zu %zu %zu\\n", sizeof(bsw_sa_interval), offsetof(bsw_sa_interval, k),'
        ' offsetof(bsw_sa_interval, s));\n'
        '  printf("%zu %zu %zu %zu\\n", sizeof(bsw_fm_entry), offsetof(bsw_fm_entry, count),'
        ' offsetof(bsw_fm_entry, bwt), offsetof(bsw_fm_entry, pad_));\n'
        '  printf("%zu %zu %zu %zu %zu\\n", sizeof(bsw_fm_meta), offsetof(bsw_fm_meta, rows),'
        ' offsetof(bsw_fm_meta, C), offsetof(bsw_fm_meta, primary), offsetof(bsw_fm_meta, entries));\n'
        '  printf("%zu %zu %zu %zu %zu\\n", sizeof(bsw_bi_interval), offsetof(bsw_bi_interval, k),'
        ' offsetof(bsw_bi_interval, l), offsetof(bsw_bi_interval, s), offsetof(bsw_bi_interval, matched));\n'
        '  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(bsw_smem), offsetof(bsw_smem, start),'
        ' offsetof(bsw_smem, end), offsetof(bsw_smem, k), offsetof(bsw_smem, l), offsetof(bsw_smem, s));\n'
        '  return 0;\n}\n')
    exe = tmp_path / "lay2"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    rows = [[int(v) for v in line.split()] for line in
            subprocess.run([str(exe)], check=True, capture_output=True,
                           text=True).stdout.strip().split("\n")]

    def lay(dt, names):
        return [dt.itemsize] + [dt.fields[f][1] for f in names]

    assert rows[0] == lay(bsw.SA_INTERVAL_DTYPE, ("k", "s")) == lay(synth.SA_INTERVAL, ("k", "s"))
    assert rows[1] == lay(bsw.FM_ENTRY_DTYPE, ("count", "bwt", "pad_"))
    assert rows[2] == [ctypes.sizeof(bsw.FmMeta), bsw.FmMeta.rows.offset, bsw.FmMeta.C.offset,
                       bsw.FmMeta.primary.offset, bsw.FmMeta.entries.offset]
    assert rows[3] == lay(bsw.BI_INTERVAL_DTYPE, ("k", "l", "s", "matched"))
    assert rows[4] == lay(bsw.SMEM_DTYPE, ("start", "end", "k", "l", "s"))
