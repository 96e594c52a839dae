"""The C-ABI library loads and exports every function include/lbmgls.h
declares, and the binding's struct layout matches the header (CPU only: no
compute call is made)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmgls.h")


def _lib():
    from paper_2311_05097_amd import lbmgls
    if not os.path.exists(lbmgls.LIB_PATH):
        from paper_2311_05097_amd import build
        build.build()
    return lbmgls


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lbm_create", "lbm_step", "lbm_read", "lbm_mass", "lbm_energy", "lbm_destroy",
                 "lbm_batch_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lbmgls = _lib()
    L = ctypes.CDLL(lbmgls.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(lbmgls.EXPORTED) == declared_functions()


def test_params_layout_matches_header(tmp_path):
    lbmgls = _lib()
    fields = [f for f, _ in lbmgls.LbmParams._fields_]
    src = tmp_path / "lay.c"
    body = "\n".join(f'printf("{f} %zu\\n", offsetof(lbm_params, {f}));' for f in fields)
    src.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "lbmgls.h"\n'
                   f'int main(void){{printf("size %zu\\n", sizeof(lbm_params));{body}return 0;}}\n')
    exe = tmp_path / "lay"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    assert int(out["size"]) == ctypes.sizeof(lbmgls.LbmParams)
    for f in fields:
        assert int(out[f]) == getattr(lbmgls.LbmParams, f).offset, f


def test_workspace_size_and_validation_host_only():
    lbmgls = _lib()
    from paper_2311_05097_amd import workloads as W
    w = W.config1()
    n32 = lbmgls.workspace_bytes(w.params, "fp32")
    n64 = lbmgls.workspace_bytes(w.params, "fp64")
    n16 = lbmgls.workspace_bytes(w.params, "fp16dev")
    assert n16 < n32 < n64
    N = 64 * 64
    assert n32 >= 2 * 18 * 4 * N + 2 * 5 * 4 * N + 3 * 4 * N
    with pytest.raises(lbmgls.LbmError):
        lbmgls.workspace_bytes(dict(w.params, nx=4), "fp32")
    with pytest.raises(lbmgls.LbmError):
        lbmgls.workspace_bytes(dict(w.params, d0=1.2), "fp32")
    # walls change no buffer; any value but 0 and 1 is rejected
    assert lbmgls.workspace_bytes(dict(w.params, bounce_y=1), "fp32") == n32
    with pytest.raises(lbmgls.LbmError):
        lbmgls.workspace_bytes(dict(w.params, bounce_y=2), "fp32")


def test_binding_shares_torchs_hip_runtime():
    """Loading the library through the binding must not bring a second HIP
    runtime into the process: torch ships its own, and a library bound to a
    different runtime cannot use torch's streams, events or device context."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2311_05097_amd import lbmgls\n"
        "lbmgls.lib()\n"
        "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
        "print(len(maps))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


HEADER3 = os.path.join(ROOT, "include", "lbmgls3d.h")


def declared_functions_3d():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER3).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(lbm3_[a-z_]+)\s*\(", text)))


def test_library_exports_every_3d_symbol():
    lbmgls = _lib()
    L = ctypes.CDLL(lbmgls.LIB_PATH)
    names = declared_functions_3d()
    for must in ("lbm3_create", "lbm3_step", "lbm3_read", "lbm3_mass", "lbm3_energy", "lbm3_destroy"):
        assert must in names
    assert not [n for n in names if not hasattr(L, n)]
    assert sorted(lbmgls.EXPORTED_3D) == names


def test_3d_params_layout_matches_header(tmp_path):
    lbmgls = _lib()
    fields = [f for f, _ in lbmgls.Lbm3Params._fields_]
    src = tmp_path / "lay3.c"
    body = "\n".join(f'printf("{f} %zu\\n", offsetof(lbm3_params, {f}));' for f in fields)
    src.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "lbmgls3d.h"\n'
                   f'int main(void){{printf("size %zu\\n", sizeof(lbm3_params));{body}return 0;}}\n')
    exe = tmp_path / "lay3"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    assert int(out["size"]) == ctypes.sizeof(lbmgls.Lbm3Params)
    for f in fields:
        assert int(out[f]) == getattr(lbmgls.Lbm3Params, f).offset, f


def test_3d_workspace_size_and_validation_host_only():
    lbmgls = _lib()
    L = lbmgls.lib()

    def nbytes(**kw):
        p = dict(nx=16, ny=12, nz=10)
        p.update(kw)
        storage = p.pop("storage", "fp64")
        return L.lbm3_workspace_bytes(ctypes.byref(lbmgls.make_params3(p, storage)))

    n64, n32 = nbytes(), nbytes(storage="fp32")
    N = 16 * 12 * 10
    assert n32 < n64 and n32 >= (2 * 30 * 4 + 2 * 7 * 4 + (3 + 1 + 1 + 3 + 5) * 8) * N
    for bad in (dict(nz=2), dict(d0=0.5), dict(tau_phi=0.5), dict(storage="fp16dev"), dict(s3=2.0),
                dict(rho2=0.0), dict(solid_eps=0.0)):
        assert nbytes(**bad) == 0, bad
        assert L.lbm3_last_error().decode()


def test_grid_size_limits_host_only():
    """Node indices are 32-bit: the largest grids below 2^31 nodes are sized,
    the first above it is refused (2-D FP64 step and smoothing; 3-D); FP32 and
    16-bit planes are addressed by 32-bit byte offsets, which holds them to
    2^30 nodes."""
    lbmgls = _lib()
    from paper_2311_05097_amd import workloads as W
    L = lbmgls.lib()
    p = W.config1().params
    assert lbmgls.workspace_bytes(dict(p, nx=46340, ny=46340), "fp64") > 2 * 18 * 8 * 46340 ** 2
    with pytest.raises(lbmgls.LbmError):
        lbmgls.workspace_bytes(dict(p, nx=46341, ny=46341), "fp64")
    for st in ("fp32", "fp16dev", "bf16dev"):
        assert lbmgls.workspace_bytes(dict(p, nx=32768, ny=32768), st) > 2 * 17 * 2 * 32768 ** 2
        for nx, ny in ((32769, 32768), (46340, 46340)):
            with pytest.raises(lbmgls.LbmError, match="2\\^30"):
                lbmgls.workspace_bytes(dict(p, nx=nx, ny=ny), st)
    assert L.lbm_smooth_workspace_bytes(46340, 46340) > 0
    assert L.lbm_smooth_workspace_bytes(46341, 46341) == 0

    def nbytes3(n):
        return L.lbm3_workspace_bytes(ctypes.byref(lbmgls.make_params3(dict(nx=n, ny=n, nz=n), "fp32")))

    assert nbytes3(1290) > 2 * 30 * 4 * 1290 ** 3
    assert nbytes3(1291) == 0 and b"2^31" in L.lbm3_last_error()
