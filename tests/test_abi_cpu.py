"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rmdf.h declares, and rejects bad arguments before it
touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(rmdf_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def L():
    from paper_1408_3526_amd import binding
    if not os.path.exists(binding.SO_PATH):
        from paper_1408_3526_amd import build
        build.build()
    return binding.lib()


def test_exports_every_declared_symbol(L):
    names = _header_functions()
    assert "rmdf_create" in names and "rmdf_push_frame" in names
    for n in sorted(names):
        assert hasattr(L, n), n
    from paper_1408_3526_amd import binding
    assert set(binding.exported_names()) <= names


def test_params_default(L):
    from paper_1408_3526_amd import binding
    p = binding.rmdf_params_default()
    assert (p.Bx, p.By, p.delay_x, p.delay_y, p.delay_t) == (-1, -1, -1, -1, -1)
    assert p.alpha < 0 and p.velocity_mode == 0 and abs(p.conf_threshold - 0.9) < 1e-7


def _create(L, H=32, W=32, M=(8, 8, 4), gx=(0.0, 1.0), gy=(0.0,), params=None, out=True):
    from paper_1408_3526_amd import binding
    gxa = np.asarray(gx, np.float32)
    gya = np.asarray(gy, np.float32)
    ctx = ctypes.c_void_p()
    st = L.rmdf_create(H, W, M[0], M[1], M[2], gxa.ctypes.data, len(gxa), gya.ctypes.data, len(gya),
                       None if params is None else ctypes.byref(params), None,
                       ctypes.byref(ctx) if out else None)
    msg = L.rmdf_last_error(None).decode()
    if st == 0:
        L.rmdf_destroy(ctx)
    del binding
    return st, msg


@pytest.mark.parametrize("kw", [dict(H=0), dict(W=-3), dict(H=65536), dict(M=(1, 8, 4)), dict(gx=()),
                                dict(gx=(np.nan,)), dict(gy=(0.0, np.inf)), dict(gy=tuple(range(40))),
                                dict(out=False)])
def test_create_rejects_invalid(L, kw):
    st, msg = _create(L, **kw)
    assert st == -1 and msg


def test_create_rejects_bad_params(L):
    from paper_1408_3526_amd import binding
    for field, val in [("Bx", 4), ("By", 9), ("delay_t", 4), ("delay_x", 8), ("alpha", 1.0), ("tile_rows", -1),
                       ("conf_threshold", float("nan")), ("conf_threshold", -0.1), ("conf_threshold", 1.5),
                       ("conf_threshold", float("inf"))]:
        p = binding.rmdf_params_default()
        setattr(p, field, val)
        st, msg = _create(L, params=p)
        assert st == -1, (field, st, msg)


def test_unsupported_shape(L):
    st, msg = _create(L, M=(6, 6, 3))
    assert st == -5 and "compiled" in msg


def test_null_context_calls(L):
    assert L.rmdf_push_frame(None, None) == -1
    assert L.rmdf_output(None, None) == -1
    assert L.rmdf_velocity(None, None, None) == -1
    assert L.rmdf_spectrum_noalloc(None, 0, None, None, None) == -1
    assert L.rmdf_push_frames(None, 2, None, None) == -1
    assert L.rmdf_state_bytes(None, None) == -1
    assert L.rmdf_save_state(None, None, 0) == -1
    assert L.rmdf_load_state(None, None, 0) == -1
    assert L.rmdf_destroy(None) == 0


def test_noalloc_limit_matches_header():
    from paper_1408_3526_amd import binding
    txt = open(os.path.join(ROOT, "include", "rmdf.h")).read()
    m = re.search(r"RMDF_SPECTRUM_NOALLOC_MAX\s*=\s*(\d+)", txt)
    assert m and int(m.group(1)) == binding.SPECTRUM_NOALLOC_MAX


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be present")
def test_no_device_reports_device_error(L):
    st, msg = _create(L)
    assert st == -3, (st, msg)


def test_hbm_probe_rejects_bad_arguments(L):
    # checked before any launch: unknown kind, missing buffers, sizes that are
    # not a positive multiple of 16 bytes, misaligned pointers, no workgroups
    assert L.rmdf_hbm_probe(3, 16, 16, 1024, 4, 0, None) == -1
    assert L.rmdf_hbm_probe(2, None, 16, 1024, 4, 0, None) == -1
    assert L.rmdf_hbm_probe(1, None, None, 1024, 4, 0, None) == -1
    assert L.rmdf_hbm_probe(2, 16, 16, 1000, 4, 0, None) == -1
    assert L.rmdf_hbm_probe(2, 16, 16, 0, 4, 0, None) == -1
    assert L.rmdf_hbm_probe(2, 16, 24, 1024, 4, 0, None) == -1
    assert L.rmdf_hbm_probe(2, 16, 16, 1024, 0, 0, None) == -1

def test_header_is_plain_c_and_links(L, tmp_path):
    """include/rmdf.h compiles as strict C99, and a C program links against
    the library and gets argument errors back through the ABI without a GPU."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    from paper_1408_3526_amd import binding
    src = tmp_path / "abi.c"
    src.write_text(r"""
#include <stdio.h>
#include "rmdf.h"
int main(void) {
  rmdf_params p;
  rmdf_ctx *ctx = 0;
  const float g[3] = {-1.f, 0.f, 1.f};
  rmdf_params_default(&p);
  rmdf_status bad = rmdf_create(0, 16, 8, 8, 4, g, 3, g, 3, &p, 0, &ctx);
  rmdf_status nul = rmdf_push_frame(0, 0);
  printf("%d %d %d %s\n", (int)bad, (int)nul, ctx == 0, rmdf_last_error(0)[0] ? "msg" : "nomsg");
  return 0;
}
""")
    exe = tmp_path / "abi"
    libdir = os.path.dirname(binding.SO_PATH)
    subprocess.check_call([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                           str(src), "-L", libdir, "-lrmdf", "-Wl,-rpath," + libdir, "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120).stdout.split()
    assert out == [str(binding.RMDF_E_INVAL), str(binding.RMDF_E_INVAL), "1", "msg"], out
