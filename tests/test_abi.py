"""The C ABI: the built library loads without a GPU and exports every entry
point declared in include/lbpf.h; the Python binding names the same set."""
import ctypes
import os
import re

import pytest

from paper_1602_07483_amd import lbpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lbpf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(lbpf_[a-z0-9_]+)\s*\(",
                      text, flags=re.M)


def test_header_declares_entry_points():
    syms = declared_symbols()
    assert "lbpf_create" in syms and "lbpf_step" in syms and "lbpf_read" in syms
    assert len(syms) == len(set(syms))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(lbpf.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    assert sorted(declared_symbols()) == sorted(lbpf.SYMBOLS)


def test_status_codes_match_header():
    text = open(os.path.join(ROOT, "include", "lbpf.h")).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"(LBPF_E[A-Z]+|LBPF_OK)\s*=\s*(-?\d+)", text))
    assert codes == {"LBPF_OK": lbpf.LBPF_OK, "LBPF_EINVAL": lbpf.LBPF_EINVAL, "LBPF_ENOMEM": lbpf.LBPF_ENOMEM,
                     "LBPF_EDEVICE": lbpf.LBPF_EDEVICE, "LBPF_EUNSTABLE": lbpf.LBPF_EUNSTABLE,
                     "LBPF_ESTATE": lbpf.LBPF_ESTATE, "LBPF_EIO": lbpf.LBPF_EIO}


def test_storage_bytes_and_invalid_arguments_without_gpu():
    L = lbpf.lib()
    # the autotune cache refuses a missing context before any device call
    hit, best = ctypes.c_int32(7), ctypes.c_double()
    assert L.lbpf_autotune_cached(None, 2, b"/nonexistent/cache", ctypes.byref(hit),
                                  ctypes.byref(best)) == lbpf.LBPF_EINVAL
    assert [L.lbpf_storage_bytes(s) for s in (0, 1, 2, 3, 9)] == [4, 2, 2, 8, 0]
    # argument validation happens before any device call
    g = lbpf.lbpf_grid()
    g.nx, g.ny, g.nz, g.lattice, g.storage = 8, 8, 8, 17, 0
    p = lbpf.lbpf_params()
    p.dx = p.dt = p.W0 = p.tau0 = 1.0
    p.k = 0.15
    h = ctypes.c_void_p()
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"lattice" in L.lbpf_last_error(None)
    g.lattice = 19
    p.k = 1.5
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    p.k = 0.15
    g.nx = 0
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert not h.value
    assert L.lbpf_bench_copy(None, None, 16, None) == lbpf.LBPF_EINVAL
    # the allocation-free reduction validates before any device call
    c3 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    okp = ctypes.c_void_p(16)
    for args in ((None, okp, okp, 0, 4, 4, 4, 0.15, 1.0), (okp, okp, okp, 2, 4, 4, 4, 0.15, 1.0),
                 (okp, okp, okp, 0, 0, 4, 4, 0.15, 1.0), (okp, okp, okp, 0, 4096, 4096, 4096, 0.15, 1.0),
                 (okp, okp, okp, 0, 4, 4, 4, 1.5, 1.0), (okp, okp, okp, 0, 4, 4, 4, 0.15, 0.0)):
        assert L.lbpf_reduce_fields_noalloc(*args, c3, okp, None) == lbpf.LBPF_EINVAL
    assert b"noalloc" in L.lbpf_last_error(None)
    for bad in ((3, 16, 0, 0, 16), (0, 3, 0, 0, 16), (2, 16, 0, -1, 16), (2, 16, 0, 0, 12)):
        assert L.lbpf_bench_bandwidth(bad[0], bad[1], bad[2], bad[3], None, None, bad[4],
                                      None) == lbpf.LBPF_EINVAL
    assert L.lbpf_destroy(None) == lbpf.LBPF_OK
    # batched domains take the single-domain lattices; checked before any device call
    g.nx, g.lattice = 8, 17
    grids = (lbpf.lbpf_grid * 1)(g)
    params = (lbpf.lbpf_params * 1)(p)
    assert L.lbpf_batch_create(1, grids, params, None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"D3Q7, D3Q15 or D3Q19" in L.lbpf_batch_last_error(None)
    # an imposed velocity must be finite, and batches carry none
    g.lattice = 19
    p.vel[0] = float("nan")
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"velocity" in L.lbpf_last_error(None)
    p.vel[0] = 0.01
    grids = (lbpf.lbpf_grid * 1)(g)
    params = (lbpf.lbpf_params * 1)(p)
    assert L.lbpf_batch_create(1, grids, params, None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"advective velocity" in L.lbpf_batch_last_error(None)
    assert not h.value
    # skip_U: 0 or 1, only for a pure substance, never in a batch
    p.vel[0] = 0.0
    p.Mcinf = 1.0
    p.skip_U = 2
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    p.skip_U = 1
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"Mcinf" in L.lbpf_last_error(None)
    p.Mcinf = 0.0
    grids = (lbpf.lbpf_grid * 1)(g)
    params = (lbpf.lbpf_params * 1)(p)
    assert L.lbpf_batch_create(1, grids, params, None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"solve U and theta" in L.lbpf_batch_last_error(None)
    assert not h.value
    # skip_theta: 0 or 1, not with skip_U, not with an advective velocity
    p.skip_U = 0
    p.skip_theta = 2
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    p.skip_theta, p.skip_U = 1, 1
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"nothing to solve" in L.lbpf_last_error(None)
    p.skip_U, p.vel[2] = 0, 0.5
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"heat equation" in L.lbpf_last_error(None)
    assert not h.value
    # separate lattice of U and theta: 0 or a lattice; single contexts only
    p.skip_theta, p.vel[2] = 0, 0.0
    g.lattice_ut = 17
    assert L.lbpf_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"lattice_ut" in L.lbpf_last_error(None)
    grids = (lbpf.lbpf_grid * 1)(g)
    params = (lbpf.lbpf_params * 1)(p)
    assert L.lbpf_batch_create(1, grids, params, None, ctypes.byref(h)) == lbpf.LBPF_EINVAL
    assert b"lattice_ut" in L.lbpf_batch_last_error(None) + L.lbpf_last_error(None)
    assert not h.value


# C names of the binding's fields where they differ ("lambda" is a Python keyword)
_C_NAME = {"lam": "lambda"}


@pytest.mark.parametrize("struct", [lbpf.lbpf_grid, lbpf.lbpf_params, lbpf.lbpf_reductions])
def test_struct_layout_matches_header(struct, tmp_path):
    """The binding's ctypes structures have the header's size and the same
    offset for every field, as the C compiler lays them out."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    name = struct.__name__
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lbpf.h"', 'int main(void) {',
             '    printf("size %%zu\\n", sizeof(%s));' % name]
    for fname, _ in struct._fields_:
        c = _C_NAME.get(fname, fname)
        lines.append('    printf("%s %%zu\\n", offsetof(%s, %s));' % (fname, name, c))
    lines += ['    return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), "-o", str(exe), str(src)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    assert int(got["size"]) == ctypes.sizeof(struct)
    for fname, _ in struct._fields_:
        assert int(got[fname]) == getattr(struct, fname).offset, fname


def test_kernel_build_id_is_a_stable_digest_of_the_kernel_sources():
    """The build passes a digest of the kernel sources to the host runtime,
    which keys persisted autotuner results by it: 16 hex digits, the same
    on every call for the same sources."""
    from paper_1602_07483_amd.build import kernel_build_id, units
    k = kernel_build_id()
    assert len(k) == 16 and all(ch in "0123456789abcdef" for ch in k)
    assert kernel_build_id() == k
    lbpf_unit = [u for u in units() if u[0] == "lbpf.o"][0]
    assert '-DLBPF_KERNEL_BUILD="%s"' % k in lbpf_unit[2]
