"""CPU checks of the C-ABI library: it loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcstedc.h")
LIB = os.path.join(ROOT, "paper_2008_01990_amd", "libdcstedc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(dc_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dc_stedc", "dc_stedc_ex", "dc_stedc_workspace", "dc_stedc_batched",
                     "dc_merge_update", "dc_stedc_backward", "dc_secular",
                     "dc_last_info", "dc_strerror"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_the_header():
    from paper_2008_01990_amd import dcstedc
    bound = {s[0] for s in dcstedc.SIGNATURES}
    assert set(declared_functions()) <= bound


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks_need_no_gpu():
    # Bad arguments are rejected on the host before anything touches a device.
    from paper_2008_01990_amd import dcstedc
    lib = dcstedc.load()
    assert lib.dc_stedc(-1, None, None, None, 1, None) == -1
    assert lib.dc_stedc(4, None, None, None, 4, None) == -2
    assert lib.dc_merge_update(-1, 1, None, 1, None, None, None, None, None, None, 1,
                               0.0, 0, None) == -1
    assert lib.dc_secular(0, None, None, 1.0, None, None, None, None, None, 0, None) == -1
    # block-size limits of the low-rank merge: 2048 with merge nodes (org
    # given), 4096 with plain column nodes; checked before any device work
    fake = ctypes.c_void_p(256)
    assert lib.dc_merge_update(8192, 8192, fake, 8192, fake, fake, fake, fake, fake, fake,
                               8192, 1e-10, 4096, None) == -13
    assert lib.dc_merge_update(8192, 8192, fake, 8192, fake, None, fake, fake, fake, fake,
                               8192, 1e-10, 8192, None) == -13
    assert lib.dc_merge_lowrank_ranks(8192, fake, fake, fake, fake, fake, 1e-10, 4096, 0,
                                      fake, None) == -8
    # the adjoint's caller-workspace form: status word, then workspace alignment
    # and size, all before any device work
    assert lib.dc_stedc_backward_workspace(-1, 0) == 0
    need = lib.dc_stedc_backward_workspace(4, 1)
    assert need > 0
    assert lib.dc_stedc_backward_ex(4, fake, fake, 4, None, fake, 4, fake, fake, fake, need,
                                    None, None) == -12
    assert lib.dc_stedc_backward_ex(4, fake, fake, 4, None, fake, 4, fake, fake,
                                    ctypes.c_void_p(264), need, fake, None) == -10
    assert lib.dc_stedc_backward_ex(4, fake, fake, 4, None, fake, 4, fake, fake, fake,
                                    need - 1, fake, None) == -11
    assert lib.dc_merge_lowrank_ranks(8192, fake, None, fake, fake, fake, 1e-10, 1024, -1,
                                      fake, None) == -9
    assert lib.dc_autotune(-1, None) == -1
    assert lib.dc_strerror(0) == b"success"
    # return codes and status words have separate decoders: a positive
    # return code is a HIP error, a positive status a non-convergence
    assert b"converge" not in lib.dc_strerror(1)
    assert b"converge" in lib.dc_status_string(1)
    assert b"non-finite" in lib.dc_status_string(-1000)
    assert b"equal eigenvalues" in lib.dc_status_string(-2000)
    o = dcstedc.DcOpts()
    lib.dc_opts_default(ctypes.byref(o))
    assert o.leaf == 32 and o.lr_tol == 0.0
    # tile variants are 0 (automatic) .. 5; others are invalid options
    for bad in (-1, 6):
        o.gemm_tile = bad
        assert lib.dc_stedc_workspace(64, ctypes.byref(o)) == 0
    # measured tuning: a negative count, and a forced tile (nothing to tune)
    assert lib.dc_autotune_batched(-1, None, None, None, None, None, None, 0, fake,
                                   None, None) == -1
    n1 = (ctypes.c_int * 1)(64)
    ptrs = (ctypes.c_void_p * 1)(256)
    o.gemm_tile = 3
    assert lib.dc_autotune_batched(1, n1, ptrs, ptrs, ptrs, n1, None, 0, fake,
                                   ctypes.byref(o), None) == -10
    assert lib.dc_autotune_levels(-1, None, 32, None, 0) == -1
    # the tuned low-rank pair: bad counts and missing outputs are rejected
    bo, ko = ctypes.c_int(0), ctypes.c_int(0)
    assert lib.dc_autotune_lowrank(-1, None, 32, ctypes.byref(bo), ctypes.byref(ko)) == -1
    assert lib.dc_autotune_lowrank(1, None, 32, ctypes.byref(bo), ctypes.byref(ko)) == -1
    assert lib.dc_autotune_lowrank(1, n1, 32, None, ctypes.byref(ko)) == -1
    assert lib.dc_autotune_lowrank(1, n1, 32, ctypes.byref(bo), None) == -1


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"),
                    reason="HIP headers not installed")
def test_binding_structs_match_the_header(tmp_path):
    # The ctypes mirrors of dc_opts and dc_merge_stat against the C compiler's
    # layout of the header's structs: size and every field's offset.
    import shutil
    import subprocess
    from paper_2008_01990_amd import dcstedc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dcstedc.h"',
             "int main(void) {"]
    expect = []
    for cname, cls in (("dc_opts", dcstedc.DcOpts), ("dc_merge_stat", dcstedc.MergeStat)):
        lines.append(f'    printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for field, _ in cls._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({cname}, {field}));')
            expect.append(getattr(cls, field).offset)
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == expect
