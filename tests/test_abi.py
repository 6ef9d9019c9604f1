"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/transec_gpu.h declares, and rejects bad host arguments before
touching a device."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pkg():
    import paper_1606_01139_amd as p
    from paper_1606_01139_amd import build
    if not os.path.exists(build.library_path()):
        build.build(verbose=False)
    p.load()
    return p


def _header_functions():
    src = open(os.path.join(ROOT, "include", "transec_gpu.h")).read()
    return sorted(set(re.findall(r"\b(tsg_[a-z_]+)\s*\(", src)))


def test_header_declares_what_binding_lists(pkg):
    assert sorted(pkg.EXPORTS) == _header_functions()


def test_library_exports_every_declared_symbol(pkg):
    lib = pkg.load()
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_default_opts(pkg):
    o = pkg.default_opts()
    assert o.tol == 1e-8 and o.block == 2 and o.precision == pkg.FP64 and o.max_restarts > 0
    assert o.bulk_tol == 1e-5 and o.select == pkg.SELECT_NEAREST


@pytest.mark.parametrize("bad", ["nan_V", "inf_V", "neg_width", "zero_h", "radius7", "neg_amp", "zero_nx"])
def test_build_rejects_bad_arguments(pkg, bad):
    nx = ny = nz = 4
    V = np.zeros(nx * ny * nz)
    ab = [0.5, 2.0, 0.0, 0.5, 2.0, 1.5]
    h, R = 0.5, 6
    if bad == "nan_V":
        V[5] = np.nan
    elif bad == "inf_V":
        V[0] = np.inf
    elif bad == "neg_width":
        ab[1] = -1.0
    elif bad == "zero_h":
        h = 0.0
    elif bad == "radius7":
        R = 7
    elif bad == "neg_amp":
        ab[3] = -0.1
    elif bad == "zero_nx":
        nx = 0
        V = np.zeros(ny * nz)
    with pytest.raises(pkg.TsgError) as e:
        pkg.Operator(nx, ny, nz, h, V, ab, fd_radius=R)
    assert e.value.status == 1  # TSG_EINVAL


def test_null_context_calls_fail_cleanly(pkg):
    import ctypes as C
    lib = pkg.load()
    n = C.c_int32()
    assert lib.tsg_get_eigenvalues(None, None, 0, C.byref(n)) == 1
    assert lib.tsg_transmission(None, None, 0, None) == 1
    assert lib.tsg_combine(None, 0, None, None) == 1
    assert b"NULL" in lib.tsg_last_error(None) or len(lib.tsg_last_error(None)) > 0
    lib.tsg_destroy(None)  # NULL-safe


def test_no_device_reports_edevice(pkg):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pkg.TsgError) as e:
        pkg.Operator(4, 4, 4, 0.5, np.zeros(64), [0.5, 2.0, 0.0, 0.5, 2.0, 1.5])
    assert e.value.status == 5  # TSG_EDEVICE: no CPU fallback exists


def test_tuning_file_round_trip_and_rejections(pkg, tmp_path):
    """tsg_load_tuning parses the autotuner's JSON on the host (no device
    needed) and refuses malformed or invalid entries."""
    from paper_1606_01139_amd.binding import load_tuning, TsgError, TSG_EINVAL
    good = tmp_path / "t.json"
    good.write_text('{"stencil": [\n {"nx": 7, "ny": 5, "nz": 9, "cols": 3, "elem": 16, "radius": 6, "tx": 32, '
                    '"yb": 2, "zchunk": 16, "us": 1.5},\n {"nx": 7, "ny": 5, "nz": 9, "cols": 3, "elem": 8, '
                    '"radius": 6, "tx": 16, "yb": 1, "zchunk": 9, "xcd": 1, "nt": 256, "cb": 2, "us": 1.0}]}\n')
    assert load_tuning(str(good)) == 2
    # launches find their entry by complex element size: 16 bytes for
    # complex128, 8 for complex64; other keys fall back to the built-in rule
    from paper_1606_01139_amd.binding import stencil_geometry, C128, C64
    assert stencil_geometry(7, 5, 9, 3, C128) == {"tx": 32, "yb": 2, "zchunk": 9, "xcd": 0, "nt": 512, "cb": 1,
                                                  "tuned": True}
    assert stencil_geometry(7, 5, 9, 3, C64) == {"tx": 16, "yb": 1, "zchunk": 9, "xcd": 1, "nt": 256, "cb": 2,
                                                 "tuned": True}
    assert not stencil_geometry(7, 5, 9, 4, C128)["tuned"]
    assert not stencil_geometry(7, 5, 9, 3, C128, radius=4)["tuned"]
    with pytest.raises(TsgError):
        stencil_geometry(7, 5, 9, 0, C128)
    bad = tmp_path / "b.json"
    bad.write_text('{"stencil": [{"nx": 7, "ny": 5, "nz": 9, "cols": 3, "elem": 16, "radius": 6, "tx": 48, '
                   '"yb": 1, "zchunk": 16, "us": 1.0}]}')
    with pytest.raises(TsgError) as e:
        load_tuning(str(bad))
    assert e.value.status == TSG_EINVAL
    # an unknown order flag, an unsupported block size, a 64-wide tile on
    # 256 threads (its radius-6 halo exceeds three cells per thread), and two
    # columns per thread for complex128 (only complex64 has that kernel)
    for extra in ('"xcd": 2', '"nt": 384', '"tx": 64, "nt": 256', '"cb": 2', '"cb": 3'):
        f = tmp_path / "x.json"
        body = '"nx": 7, "ny": 5, "nz": 9, "cols": 3, "elem": 16, "radius": 6, "yb": 1, "zchunk": 16, "us": 1.0'
        if '"tx"' not in extra:
            body += ', "tx": 32'
        f.write_text('{"stencil": [{%s, %s}]}' % (body, extra))
        with pytest.raises(TsgError):
            load_tuning(str(f))
    worse = tmp_path / "w.json"
    worse.write_text('{"stencil": [{"nx": 7}]}')
    with pytest.raises(TsgError):
        load_tuning(str(worse))
    with pytest.raises(TsgError):
        load_tuning(str(tmp_path / "missing.json"))
