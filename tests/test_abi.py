"""Host-side checks of the C ABI library (no GPU compute)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsfit.h")


@pytest.fixture(scope="module")
def libpath():
    from paper_2601_22026_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2601_22026_amd import build
        build.build(verbose=False)
    return _abi.LIB_PATH


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["gsf_forward", "gsf_backward", "gsf_loss_l1", "gsf_adam", "gsf_step_capture",
                 "gsf_step_replay", "gsf_plan_create", "gsf_debug_copy", "gsf_autotune"]:
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    L = ct.CDLL(libpath)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    from paper_2601_22026_amd import _abi
    assert sorted(_abi.EXPORTED) == _declared_functions()


def test_struct_layouts():
    from paper_2601_22026_amd import _abi
    assert ct.sizeof(_abi.gsf_camera) == 128
    assert _abi.gsf_camera.width.offset == 100
    assert ct.sizeof(_abi.gsf_plan_desc) == 56


def test_struct_layouts_match_the_c_header(tmp_path):
    """sizeof / offsetof of every ABI struct field, as a C compiler lays out
    include/gsfit.h, equal the ctypes mirrors of the binding."""
    import shutil
    import subprocess
    from paper_2601_22026_amd import _abi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gsf_camera": _abi.gsf_camera, "gsf_plan_desc": _abi.gsf_plan_desc,
               "gsf_step_args": _abi.gsf_step_args, "gsf_tune_space": _abi.gsf_tune_space,
               "gsf_tune_result": _abi.gsf_tune_result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsfit.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ct.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2601_22026_amd import _abi
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(_abi.GsfError):
        _abi.lib()


def test_camera_packing_roundtrip():
    import numpy as np

    import paper_2601_22026_amd as gs
    import synth
    cam = synth.look_at_camera([1.0, 2.0, -2.0], width=33, height=17, bg=(0.1, 0.2, 0.3))
    raw = gs.pack_cameras([cam])
    f = np.frombuffer(raw, dtype=np.float32)
    i = np.frombuffer(raw, dtype=np.int32)
    np.testing.assert_array_equal(f[:12].reshape(3, 4)[:, :3], cam.R)
    np.testing.assert_array_equal(f[:12].reshape(3, 4)[:, 3], cam.t)
    np.testing.assert_array_equal(f[12:15], cam.campos)
    assert (f[15], f[16], f[17], f[18]) == (np.float32(cam.fx), np.float32(cam.fy),
                                            np.float32(cam.cx), np.float32(cam.cy))
    np.testing.assert_array_equal(f[22:25], cam.bg)
    assert (i[25], i[26]) == (33, 17) and (i[27:] == 0).all()
