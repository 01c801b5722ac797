"""The C ABI: the built library loads and exports every entry point that
include/sss.h declares.  No GPU needed (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "sss.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sss_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("sss_csr_spmv", "sss_csr_spmv_plan_create", "sss_csr_spmv_execute", "sss_plan_destroy"):
        assert s in syms


def test_header_is_plain_c_and_links(tmp_path):
    """include/sss.h is valid C99 on its own (no C++ or HIP types leak into
    the boundary), and a C program using it links against libsss.so."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(
        '#include "sss.h"\n'
        "int spmv_many(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *col,\n"
        "              const double *val, const double *x, double *y, void *stream, int calls) {\n"
        "  sss_plan_opts opts = {0};\n"
        "  opts.mode = SSS_MODE_FIXED;\n"
        "  opts.bind_rows = 1;\n"
        "  sss_plan plan = NULL;\n"
        "  int rc = sss_csr_spmv_plan_create(m, n, nnz, rp, SSS_F64, &opts, stream, &plan);\n"
        "  for (int k = 0; rc == SSS_OK && k < calls; ++k)\n"
        "    rc = sss_csr_spmv_execute(plan, rp, col, val, x, y, stream);\n"
        "  sss_plan_destroy(plan);\n"
        "  return rc;\n"
        "}\n"
        "int main(void) { return sss_status_string(SSS_OK) ? 0 : 1; }\n")
    lib_dir = os.path.join(ROOT, "paper_1504_06474_amd")
    out = tmp_path / "use"
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), str(src), "-L", lib_dir, "-lsss",
                        f"-Wl,-rpath,{lib_dir}", "-o", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_symbol():
    from paper_1504_06474_amd import sss
    L = sss.lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_status_strings_and_version():
    from paper_1504_06474_amd import sss
    L = sss.lib()
    assert L.sss_csr_spmv_cache_clear() == 0  # nothing cached: no device call
    assert L.sss_status_string(0) == b"ok"
    assert L.sss_status_string(-5) == b"malformed CSR matrix"
    assert b"gfx950" in L.sss_version()


def test_host_side_argument_checks():
    """Plan creation rejects bad sizes and parameters before any device call."""
    from paper_1504_06474_amd import sss
    L = sss.lib()
    h = ctypes.c_void_p()
    bad = sss.PlanOpts(sss.MODE_FIXED, 5, 1, 1, 0)  # W = 5 is not built
    assert L.sss_csr_spmv_plan_create(10, 10, 10, None, 0, ctypes.byref(bad), None, ctypes.byref(h)) == -2
    assert L.sss_csr_spmv_plan_create(-1, 10, 10, None, 0, None, None, ctypes.byref(h)) == -1
    assert L.sss_csr_spmv_plan_create(10, 10, 10, None, 7, None, None, ctypes.byref(h)) == -2
    bad_s = sss.PlanOpts(sss.MODE_FIXED, 8, 0, 9, 0)  # B = 9 out of range
    assert L.sss_csr_spmv_plan_create(10, 10, 10, None, 0, ctypes.byref(bad_s), None, ctypes.byref(h)) == -1
    assert L.sss_csr_spmv_execute(None, None, None, None, None, None, None) == -1
    grid = sss.MODE_GRID if hasattr(sss, "MODE_GRID") else 1
    opts = sss.PlanOpts(grid, 0, 0, 0, 0)  # GRID needs the matrix: its own call
    assert L.sss_csr_spmv_plan_create(10, 10, 10, None, 0, ctypes.byref(opts), None, ctypes.byref(h)) == -2
    assert L.sss_csr_spmv_plan_create_grid(10, 10, 10, None, None, None, None, None, 0, 5, None, None) == -1
    # reps < 1 is rejected before any device call
    assert L.sss_csr_spmv_plan_create_grid(10, 10, 10, None, None, None, None, None, 0, 0, None,
                                           ctypes.byref(h)) == -1
    assert h.value is None
    assert L.sss_batch_plan_create_grid(1, None, 0, 3, None, None, None, ctypes.byref(h)) == -1
    assert L.sss_batch_plan_create_grid(0, None, 0, 0, None, None, None, ctypes.byref(h)) == -1
    assert L.sss_csr_rowwise(-1, 1, 0, None, None, None, None, None, 0, 1, None) == -1
    assert L.sss_csr_rowwise(10, 10, 10, None, None, None, None, None, 0, 3, None) == -2
    assert L.sss_csr_rowwise(10, 10, 10, None, None, None, None, None, 0, 128, None) == -2
    assert L.sss_csr_rowwise(0, 0, 0, None, None, None, None, None, 0, 64, None) == 0
    assert L.sss_csr_rowwise(10, 10, 10, None, None, None, None, None, 0, 64, None) == -1
    assert L.sss_csr_rowwise(2147479552, 10, 10, None, None, None, None, None, 0, 64, None) == -1
    big = 2147479551  # SSS_MAX_INDEX
    assert L.sss_csr_spmv_plan_create(big + 1, 10, 10, None, 0, None, None, ctypes.byref(h)) == -1
    assert L.sss_csr_spmv_plan_create(10, 10, big + 1, None, 0, None, None, ctypes.byref(h)) == -1
    assert L.sss_csr_spmv_plan_create(10, big + 1, 10, None, 0, None, None, ctypes.byref(h)) == -1
    assert "#define SSS_MAX_INDEX 2147479551" in open(os.path.join(ROOT, "include", "sss.h")).read()
    # calls on a NULL plan are rejected before any device call
    assert L.sss_batch_execute(None, None) == -1
    assert L.sss_batch_graph_launch(None, None) == -1
    assert L.sss_batch_floor_probe(None, None, 1, None) == -1
    assert L.sss_floor_probe(None, None, None, None, None, 1, None) == -1
    assert L.sss_csr_spmv_stage1(None, None, None, None, None, None, None) == -1
    assert L.sss_csr_spmv_stage2(None, None, None, None) == -1
    assert L.sss_csr_spmv_stage2_host(None, None, None) == -1
    n = ctypes.c_int64()
    assert L.sss_plan_dirty_list(None, None, 0, ctypes.byref(n)) == -1
    # the probe's row part: a bad row count, or rows without y (pointers
    # that are never dereferenced: the checks come first)
    fake = ctypes.c_void_p(256)
    assert L.sss_gather_probe_rows(fake, None, fake, 10, 10, 0, 0, 1, 4, 0, fake, 1 << 20, ctypes.byref(n), None,
                                   fake, -1, fake, None) == -1
    assert L.sss_gather_probe_rows(fake, None, fake, 10, 10, 0, 0, 1, 4, 0, fake, 1 << 20, ctypes.byref(n), None,
                                   fake, 5, None, None) == -1
    # CG and the plan's shape: NULL plans and outputs are rejected before any device call
    assert L.sss_plan_shape(None, None, None, None, None) == -1
    assert L.sss_cg_start(None, *([None] * 9), None) == -1
    assert L.sss_cg_iterate(None, *([None] * 8), 1, None) == -1
    size = ctypes.c_size_t()
    assert L.sss_cg_workspace_size(None) == -1
    assert L.sss_cg_workspace_size(ctypes.byref(size)) == 0 and size.value % 8 == 0 and size.value >= 24
    assert L.sss_plan_destroy(None) == 0


def test_workspace_size_host_side():
    """Workspace sizes are host arithmetic (no device): FIXED mode the
    layout of its (W, S), growing with nnz; SELECTOR mode at least every
    grid class's; bad arguments rejected."""
    from paper_1504_06474_amd import sss
    L = sss.lib()
    b = ctypes.c_size_t()
    sizes = {}
    for W in (4, 8, 16):
        for S in (1, 2, 4, 8):
            o = sss.PlanOpts(sss.MODE_FIXED, W, S, 0, 0)
            assert L.sss_csr_spmv_plan_workspace_size(10 ** 6, 10 ** 6, 2 * 10 ** 7, 0, ctypes.byref(o),
                                                      ctypes.byref(b)) == 0
            sizes[W, S] = b.value
            nb = -(-2 * 10 ** 7 // (S * W * 64))
            # dirty mask, speculator (S per bunch), synchronizer index and value, tail
            assert b.value >= nb * (4 + 16 * S + 4 + 8 + 8)
    o = sss.PlanOpts(sss.MODE_SELECTOR, 0, 0, 0, 0)
    assert L.sss_csr_spmv_plan_workspace_size(10 ** 6, 10 ** 6, 2 * 10 ** 7, 0, ctypes.byref(o), ctypes.byref(b)) == 0
    assert b.value == max(sizes.values())
    o = sss.PlanOpts(sss.MODE_FIXED, 8, 5, 0, 0, 1)  # bind_rows adds a first row per bunch
    assert L.sss_csr_spmv_plan_workspace_size(10 ** 6, 10 ** 6, 2 * 10 ** 7, 0, ctypes.byref(o), ctypes.byref(b)) == 0
    bound = b.value
    o = sss.PlanOpts(sss.MODE_FIXED, 8, 5, 0, 0, 0)
    assert L.sss_csr_spmv_plan_workspace_size(10 ** 6, 10 ** 6, 2 * 10 ** 7, 0, ctypes.byref(o), ctypes.byref(b)) == 0
    assert bound > b.value
    assert L.sss_csr_spmv_plan_workspace_size(-1, 1, 1, 0, None, ctypes.byref(b)) == -1
    assert L.sss_csr_spmv_plan_workspace_size(1, 1, 1, 0, None, None) == -1
    assert L.sss_csr_spmv_plan_workspace_size(1, 1, 1, 9, None, ctypes.byref(b)) == -2
    bad = sss.PlanOpts(sss.MODE_FIXED, 5, 1, 0, 0)
    assert L.sss_csr_spmv_plan_workspace_size(1, 1, 1, 0, ctypes.byref(bad), ctypes.byref(b)) == -2
    # a workspace pointer with no size, or a size with no pointer
    h = ctypes.c_void_p()
    o = sss.PlanOpts(sss.MODE_FIXED, 8, 5, 0, 0, 0, 0, None, 64)
    assert L.sss_csr_spmv_plan_create(10, 10, 10, None, 0, ctypes.byref(o), None, ctypes.byref(h)) == -1
