"""The C ABI library loads and exports every entry point include/sellcs.h
declares; argument checks that happen on the host return the documented
status codes. No kernel is launched here."""
import ctypes
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sellcs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    names = re.findall(r"^\s*(?:sell_status|const\s+char\s*\*)\s*(sell_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1307_6209_amd import sellcs
    if not os.path.exists(sellcs.LIB_PATH):
        from paper_1307_6209_amd import _build
        _build.build()
    return sellcs.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["sell_build", "sell_spmv", "sell_spmmv", "sell_export", "sell_info", "sell_destroy",
                 "sell_batch_create", "sell_batch_create_persistent", "sell_batch_spmv", "sell_batch_destroy",
                 "sell_autotune", "sell_batch_autotune",
                 "sell_probe_bandwidth", "sell_status_string", "sell_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_the_header():
    from paper_1307_6209_amd import sellcs
    assert sorted(sellcs.SIGNATURES) == declared_functions()


def test_status_strings(L):
    for code, name in enumerate(["SELL_OK", "SELL_ERR_INVALID_ARG", "SELL_ERR_BAD_CRS", "SELL_ERR_OOM",
                                 "SELL_ERR_UNSUPPORTED", "SELL_ERR_HIP"]):
        assert L.sell_status_string(code).decode() == name


def test_host_side_argument_errors(L):
    from paper_1307_6209_amd import sellcs
    h = ctypes.c_void_p()
    assert L.sell_build(None, 32, 1, None, None, ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    assert b"null" in L.sell_last_error()
    # pointers are not dereferenced before the arguments are checked
    A = sellcs.SellCrs(10, 10, 0, ctypes.c_void_p(8), None, None)
    for C in [0, 3, 256, -4]:
        assert L.sell_build(ctypes.byref(A), C, 1, None, None, ctypes.byref(h)) == sellcs.SELL_ERR_UNSUPPORTED
    assert L.sell_build(ctypes.byref(A), 32, 0, None, None, ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    Aneg = sellcs.SellCrs(-1, 10, 0, ctypes.c_void_p(8), None, None)
    assert L.sell_build(ctypes.byref(Aneg), 32, 1, None, None, ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    Abig = sellcs.SellCrs(2**31, 10, 0, ctypes.c_void_p(8), None, None)
    assert L.sell_build(ctypes.byref(Abig), 32, 1, None, None, ctypes.byref(h)) == sellcs.SELL_ERR_UNSUPPORTED
    f64_val_f32_acc = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=1)  # FP64 values need FP64 accumulation
    assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(f64_val_f32_acc), None,
                        ctypes.byref(h)) == sellcs.SELL_ERR_UNSUPPORTED
    for u in (5, 12, 32):
        badu = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, unroll=u)
        assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(badu), None,
                            ctypes.byref(h)) == sellcs.SELL_ERR_UNSUPPORTED
    for C, vec in [(128, 2), (2, 4), (32, 3)]:
        badv = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, vec=vec)
        assert L.sell_build(ctypes.byref(A), C, 1, ctypes.byref(badv), None,
                            ctypes.byref(h)) == sellcs.SELL_ERR_UNSUPPORTED
    for xw in (-2, 2):
        badx = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, xwindow=xw)
        assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(badx), None,
                            ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    for g in (-1, 2, 16):
        badg = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, xwindow_chunks=g)
        assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(badg), None,
                            ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    for r in (-1, 2):
        badr = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, row_lengths=r)
        assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(badr), None,
                            ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    for C in (1, 4, 128):  # row lengths are kept for C in 8..64 only
        rl = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, row_lengths=1)
        assert L.sell_build(ctypes.byref(A), C, 1, ctypes.byref(rl), None,
                            ctypes.byref(h)) == sellcs.SELL_ERR_UNSUPPORTED
    assert L.sell_spmv(None, None, None, None) == sellcs.SELL_ERR_INVALID_ARG
    assert L.sell_spmmv(None, None, None, 4, None) == sellcs.SELL_ERR_INVALID_ARG
    assert L.sell_batch_create(None, 0, ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    assert L.sell_batch_create_persistent(None, 0, ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG
    bt = sellcs.SellBatchTuned()
    sig = (ctypes.c_int64 * 1)()
    assert L.sell_batch_autotune(None, 1, None, None, ctypes.byref(bt), sig) == sellcs.SELL_ERR_INVALID_ARG
    crs = (sellcs.SellCrs * 1)()
    assert L.sell_batch_autotune(crs, 0, None, None, ctypes.byref(bt), sig) == sellcs.SELL_ERR_INVALID_ARG
    assert L.sell_batch_autotune(crs, 1, None, None, None, sig) == sellcs.SELL_ERR_INVALID_ARG
    g = ctypes.c_double()
    assert L.sell_probe_bandwidth(10, 1 << 30, 1, None, ctypes.byref(g)) == sellcs.SELL_ERR_INVALID_ARG
    assert L.sell_autotune(None, 1, None, None, None) == sellcs.SELL_ERR_INVALID_ARG
    assert L.sell_destroy(None) == sellcs.SELL_OK
    assert L.sell_batch_destroy(None) == sellcs.SELL_OK


def test_allocator_failure_is_reported_before_any_device_work(L):
    """An allocator callback that returns NULL yields SELL_ERR_OOM; the
    library asks it before launching anything, so this runs without a GPU."""
    from paper_1307_6209_amd import sellcs
    calls = []
    alloc = sellcs.ALLOC_FN(lambda n, ctx: calls.append(n) or None)
    free = sellcs.FREE_FN(lambda p, ctx: None)
    al = sellcs.SellAllocator(ctypes.cast(alloc, ctypes.c_void_p), ctypes.cast(free, ctypes.c_void_p), None)
    o = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, alloc=ctypes.pointer(al))
    A = sellcs.SellCrs(10, 10, 0, ctypes.c_void_p(8), None, None)
    h = ctypes.c_void_p()
    assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(o), None, ctypes.byref(h)) == sellcs.SELL_ERR_OOM
    assert calls and not h.value
    half = sellcs.SellAllocator(ctypes.cast(alloc, ctypes.c_void_p), None, None)
    o2 = sellcs.SellBuildOpts(val_dtype=0, acc_dtype=0, alloc=ctypes.pointer(half))
    assert L.sell_build(ctypes.byref(A), 32, 1, ctypes.byref(o2), None, ctypes.byref(h)) == sellcs.SELL_ERR_INVALID_ARG


def test_library_binds_to_torchs_hip_runtime():
    """Loading the library through the binding maps one HIP runtime (torch's):
    a second runtime in the process does not share device state with torch,
    and every allocation through it fails."""
    import subprocess
    code = ("from paper_1307_6209_amd import sellcs; sellcs.lib(); "
            "import json; print(json.dumps(sellcs.hip_runtimes()))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    import json
    rts = json.loads(out.stdout.strip().splitlines()[-1])
    assert len(rts) == 1, rts


def test_every_dtype_combination_is_compiled(L):
    """The build compiles the instantiation source once per DtypeCombo
    enumerator, under the launcher suffixes dispatch.hip declares, and the
    library defines every combination's launchers (a missing one would only
    show as an unresolved symbol at its first call)."""
    import shutil
    import subprocess
    from paper_1307_6209_amd import _build, sellcs
    csrc = os.path.join(ROOT, "paper_1307_6209_amd", "csrc")
    enum = re.search(r"enum DtypeCombo \{(.*?)\};", open(os.path.join(csrc, "sell_internal.h")).read(), re.S).group(1)
    combos = re.findall(r"(COMBO_\w+)\s*=", enum)
    declared = re.findall(r"^SELL_DECL\((\w+)\)", open(os.path.join(csrc, "dispatch.hip")).read(), re.M)
    built = [dict(d[2:].split("=") for d in defs) for src, defs, _ in _build.units()
             if os.path.basename(src) == _build.COMBO_SRC]
    assert sorted(b["SELL_COMBO"] for b in built) == sorted(combos)
    assert sorted(b["SELL_LC"] for b in built) == sorted(declared)
    if shutil.which("nm") is None:
        pytest.skip("nm is not available")
    syms = subprocess.run(["nm", "-C", "--defined-only", sellcs.LIB_PATH], capture_output=True, text=True,
                          check=True).stdout
    for lc in declared:
        for fn in ("launch_spmv_", "launch_spmv_xw_", "launch_batch_", "batch_waves_per_cu_"):
            assert "sell::%s%s(" % (fn, lc) in syms, fn + lc
