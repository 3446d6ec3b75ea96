"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-side validation rejects bad input with the
documented status codes before touching a device."""
import os
import re

import numpy as np
import pytest

import paper_2604_22092_amd as fs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "fs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_documented_api():
    decl = declared_symbols()
    for name in ["fs_graph_create", "fs_sim_create", "fs_step", "fs_counts", "fs_history",
                 "fs_get_state", "fs_set_state", "fs_sim_seed"]:
        assert name in decl
    assert sorted(fs.EXPORTS) == decl


def test_library_exports_every_declared_symbol():
    L = fs.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    L = fs.lib()
    assert L.fs_status_string(0) == b"FS_OK"
    assert L.fs_status_string(2) == b"FS_ERR_INVALID_CSR"
    assert L.fs_status_string(5) == b"FS_ERR_BUSY"
    assert "gfx950" in fs.fs_version()


@pytest.mark.parametrize("rp,ci,msg", [
    ([1, 2, 2], [0, 1], "row_ptr[0]"),
    ([0, 2, 1], [1, 0], "decreases"),
    ([0, 1, 2], [1, 2], "out of range"),
    ([0, 1, 2], [-1, 0], "out of range"),
])
def test_invalid_csr_rejected(rp, ci, msg):
    with pytest.raises(fs.FsError) as ei:
        fs.fs_graph_create(np.array(rp), np.array(ci))
    assert ei.value.status == 2 and msg in str(ei.value)


def test_invalid_n_rejected():
    L = fs.lib()
    import ctypes
    h = ctypes.c_void_p()
    assert L.fs_graph_create(0, None, None, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert L.fs_graph_create(1, None, None, None, ctypes.byref(h)) == 1
    assert b"row_ptr" in L.fs_last_error()


def test_null_handles_rejected():
    L = fs.lib()
    assert L.fs_step(None, 1) == 1
    assert L.fs_sync(None) == 1
    assert L.fs_sim_destroy(None) == 1
    assert L.fs_graph_destroy(None) == 1
    assert L.fs_counts(None, 0, None) == 1
    assert L.fs_sim_seed_noalloc(None, 0, 0, None, 1) == 1
    assert L.fs_sim_autotune(None, None, None) == 1
    assert L.fs_sim_get_variant(None, None) == 1
    assert L.fs_sim_get_column_bits(None, None) == 1


def test_seed_noalloc_limit_matches_the_header():
    txt = open(os.path.join(ROOT, "include", "fs.h")).read()
    m = re.search(r"#define FS_SEED_NOALLOC_MAX (\d+)", txt)
    assert m and int(m.group(1)) == fs.FS_SEED_NOALLOC_MAX


def test_bad_hazard_parameters_rejected_on_host():
    # parameter validation happens before any device work
    for spec in [("weibull", 0.5, 3.0), ("lognormal", 0.0, 0.0), ("erlang", 0, 1.0),
                 ("erlang", 3, -1.0), ("exp", -1.0)]:
        with pytest.raises(fs.FsError) as ei:
            fs.fs_eval_hazard(spec, np.array([1.0], np.float32))
        assert ei.value.status == 1


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2604_22092_amd import _capi
    monkeypatch.setattr(_capi, "_lib", None)
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _capi.lib()


def test_batch_and_server_host_validation():
    import ctypes
    L = fs.lib()
    h = ctypes.c_void_p()
    assert L.fs_batch_create(7, None, ctypes.byref(h)) == 1 and h.value is None
    for bad in [fs.fs_server_params(0, 0, 0, 9, 0, None),     # unknown storage
                fs.fs_server_params(-1, 0, 0, 0, 0, None),    # negative budget
                fs.fs_server_params(0, -2, 0, 0, 0, None)]:   # negative slot limit
        assert L.fs_server_create(ctypes.byref(bad), ctypes.byref(h)) == 1 and h.value is None
    assert L.fs_server_create(None, ctypes.byref(h)) == 1
    assert L.fs_batch_step(None, 1) == 1
    assert L.fs_batch_add(None, None) == 1
    rid = ctypes.c_int64()
    assert L.fs_server_submit(None, None, ctypes.byref(rid)) == 1
    assert L.fs_server_stats(None, None) == 1
    assert b"NULL" in L.fs_last_error()


def test_bad_shedding_parameters_rejected_on_host():
    ages = np.array([1.0], np.float32)
    for shed in [("density", ("weibull", 0.5, 3.0), 1.0), ("hazard", ("lognormal", 0.0, -1.0), 1.0),
                 ("density", ("exp", 1.0), -2.0), ("density", ("exp", 1.0), float("inf"))]:
        with pytest.raises(fs.FsError) as ei:
            fs.fs_eval_shedding(shed, ages)
        assert ei.value.status == 1
    import ctypes
    d = fs.make_dist(("exp", 1.0))
    out = np.zeros(1, np.float32)
    assert fs.lib().fs_eval_shedding(ctypes.byref(d), 0, 1.0, 0, 1.0, 1, ages.ctypes.data,
                                     out.ctypes.data) == 1   # the constant form has no profile


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and field offsets of the ABI structs as a C compiler lays them
    out from include/fs.h, against the binding's ctypes mirrors."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"fs_dist": fs.fs_dist, "fs_sim_params": fs.fs_sim_params,
               "fs_server_params": fs.fs_server_params, "fs_request": fs.fs_request,
               "fs_request_info": fs.fs_request_info, "fs_markov_params": fs.fs_markov_params,
               "fs_tune_params": fs.fs_tune_params, "fs_tune_result": fs.fs_tune_result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fs.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])


def test_markov_host_validation():
    import ctypes
    L = fs.lib()
    h = ctypes.c_void_p()
    p = fs.fs_markov_params()
    assert L.fs_markov_create(None, ctypes.byref(p), ctypes.byref(h)) == 1 and h.value is None
    assert L.fs_markov_step(None, 1) == 1
    assert L.fs_markov_sync(None) == 1
    assert L.fs_markov_destroy(None) == 1
    assert L.fs_markov_get_state(None, None, None, None, None) == 1


def test_allocator_hook_arguments():
    import ctypes
    L = fs.lib()
    assert L.fs_set_allocator(None, None, None) == 0
    cb = fs._capi._ALLOC_FN(lambda n, c: None)
    assert L.fs_set_allocator(ctypes.cast(cb, ctypes.c_void_p), None, None) == 1
    assert b"both" in L.fs_last_error()
