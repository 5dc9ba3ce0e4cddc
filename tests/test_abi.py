"""The C-ABI library loads and exports every entry point include/bnc.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bnc.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bnc_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for k in ("d", "dd", "td", "qd"):
        assert f"bnc_getrf_{k}" in names and f"bnc_getrs_{k}" in names
    for n in ("bnc_refine", "bnc_refine_workspace_size", "bnc_residual", "bnc_mw_apply", "bnc_getrf_ozaki",
              "bnc_refine_batched", "bnc_refine_batched_graph", "bnc_getrf_workspace_size",
              "bnc_getrs_workspace_size", "bnc_residual_workspace_size"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2107_12550_amd.bnc import lib_path
    L = ctypes.CDLL(lib_path)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_entry_points():
    import paper_2107_12550_amd as P
    L = P.lib()
    assert L.bnc_version().decode().startswith("bnc")
    assert L.bnc_status_string(0) == b"converged"
    # workspace grows with n and K; invalid arguments give 0
    assert L.bnc_refine_workspace_size(128, 3) > 3 * 128 * 128 * 8
    assert L.bnc_refine_workspace_size(0, 3) == 0
    assert L.bnc_refine_workspace_size(128, 5) == 0
    # argument errors are reported before anything touches the device
    rc = L.bnc_getrf_td(-1, None, 1, 1, None, None, None, 0, None)
    assert rc == -1
    rc = L.bnc_getrf_td(8, None, 8, 64, None, None, None, 0, None)
    assert rc == -2
    assert b"NULL" in L.bnc_last_error()


def test_workspace_queries():
    """Every stand-alone call takes its scratch from the caller: the size
    queries grow with n and K, cover the split form's slices, give 0 for
    n = 0 and for arguments out of range, and a call whose workspace is
    missing or too small is refused before anything is launched."""
    import paper_2107_12550_amd as P
    L = P.lib()
    for K in (1, 2, 3, 4):
        a, b = P.getrf_workspace_size(K, 1024), P.getrf_workspace_size(K, 2048)
        assert 0 < a < b
        assert P.getrf_workspace_size(K, 2048, 5) >= b + 3 * 12 * 64 * 2048 * 8
        assert P.getrf_workspace_size(K, 0) == 0
        assert 0 < P.getrs_workspace_size(K, 100) < P.getrs_workspace_size(K, 200)
        assert P.getrs_workspace_size(K, 0) == 0
    assert P.getrf_workspace_size(2, 4096) < P.getrf_workspace_size(4, 4096)
    assert P.getrf_workspace_size(5, 64) == 0 and P.getrf_workspace_size(2, 64, 13) == 0
    assert P.getrf_workspace_size(2, 16385) == 0 and P.getrs_workspace_size(0, 8) == 0
    assert 0 < P.residual_workspace_size(64) < P.residual_workspace_size(128)
    assert P.residual_workspace_size(0) == 0
    # batched slots: K planes of NT^2 plus K of NT per workgroup, after a 256-byte queue counter
    L.bnc_refine_batched_workspace_size.restype = ctypes.c_size_t
    for K, nt in ((3, 256), (2, 512), (4, 64)):
        assert L.bnc_refine_batched_workspace_size(K, 10, nt) == 10 * (K * nt * nt + K * nt) * 8 + 256
    assert L.bnc_refine_batched_workspace_size(3, 10, 0) == L.bnc_refine_batched_workspace_size(3, 10, 256)
    assert L.bnc_refine_batched_workspace_size(3, 10, 100) == 0
    assert L.bnc_refine_batched_workspace_size(5, 10, 256) == 0
    assert L.bnc_features_workspace_size(4) == 256 + 4 * 512 * 512 * 8
    # pointers are never dereferenced on these paths: fake non-NULL addresses
    A, ip, inf = 1 << 20, 2 << 20, 3 << 20
    need = P.getrf_workspace_size(3, 8)
    assert L.bnc_getrf_td(8, A, 8, 64, ip, inf, None, need, None) == -7
    assert L.bnc_getrf_td(8, A, 8, 64, ip, inf, 4 << 20, need - 1, None) == P.BNC_ERR_WORKSPACE
    assert L.bnc_getrf_ozaki(2, 5, 8, A, 8, 64, ip, inf, 4 << 20, P.getrf_workspace_size(2, 8), None) == \
        P.BNC_ERR_WORKSPACE
    need = P.getrs_workspace_size(2, 8)
    assert L.bnc_getrs_dd(8, 1, A, 8, 64, ip, A, 8, 8, None, None, need, None) == -11
    assert L.bnc_getrs_dd(8, 1, A, 8, 64, ip, A, 8, 8, None, 4 << 20, need - 1, None) == P.BNC_ERR_WORKSPACE
    assert L.bnc_residual(8, 1, 4, A, 8, 64, A, 8, A, 8, A, 8, inf, None, 0, None) == -14
    assert L.bnc_residual(8, 1, 4, A, 8, 64, A, 8, A, 8, A, 8, inf, 4 << 20, 16, None) == P.BNC_ERR_WORKSPACE
    assert L.bnc_residual(8, 1, 5, A, 8, 64, A, 8, A, 8, A, 8, inf, 4 << 20, 1 << 30, None) == -3
    # n = 0 needs no workspace and launches nothing
    assert L.bnc_getrs_qd(0, 1, None, 1, 0, None, None, 1, 1, None, None, 0, None) == 0
    assert L.bnc_test_force_timeout(4) == -1 and L.bnc_test_force_timeout(0) == 0


def test_ozaki_rejects_bad_slices_before_touching_the_device():
    import paper_2107_12550_amd as P
    L = P.lib()
    assert L.bnc_getrf_ozaki(3, 0, 4, None, 4, 16, None, None, None, 0, None) == -2
    assert L.bnc_getrf_ozaki(3, 13, 4, None, 4, 16, None, None, None, 0, None) == -2
    assert L.bnc_getrf_ozaki(5, 8, 4, None, 4, 16, None, None, None, 0, None) == -1
    # argument positions continue from n = 3
    assert L.bnc_getrf_ozaki(3, 8, -1, None, 4, 16, None, None, None, 0, None) == -3


def test_slice_width_agrees_with_the_oracle():
    """The library's slice width (its own closed form) equals the oracle's
    (every group summed out) for every factor length and slice count."""
    import oracle as O
    import paper_2107_12550_amd as P
    for K in (1, 2, 3, 4):
        for s in range(1, 13):
            assert P.oz_beta(K, s) == O.oz_beta(K, s), (K, s)
    assert P.lib().bnc_oz_beta(2, 0) == -1
    assert P.lib().bnc_oz_beta(5, 4) == -1
    assert P.lib().bnc_oz_beta(2, 13) == -1


def test_gemm_rejects_bad_arguments_before_touching_the_device():
    import paper_2107_12550_amd as P
    L = P.lib()
    assert L.bnc_gemm_td(-1, 1, 1, None, 1, 1, None, 1, 1, None, 1, 1, None) == -1
    assert L.bnc_gemm_td(4, 4, 4, None, 4, 16, None, 4, 16, None, 4, 16, None) == -4
    assert L.bnc_gemm_td(4, 4, 4, 8, 3, 16, 8, 4, 16, 8, 4, 16, None) == -5
    assert L.bnc_gemm_td(4, 4, 4, 8, 4, 15, 8, 4, 16, 8, 4, 16, None) == -6
    assert L.bnc_gemm_qd(4, 4, 4, 8, 4, 16, 8, 4, 16, 8, 4, 15, None) == -12
    assert L.bnc_gemm_d(3, 2, 0, None, 3, 0, None, 1, 2, 8, 3, 6, None) == 0  # k = 0: nothing to do


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the C layout of include/bnc.h
    (sizes and field offsets as gcc lays them out)."""
    import subprocess

    from paper_2107_12550_amd import bnc
    structs = {"bnc_refine_opts": bnc.RefineOpts, "bnc_refine_result": bnc.RefineResult,
               "bnc_batch_result": bnc.BatchResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bnc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
