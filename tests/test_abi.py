"""The C-ABI library loads and exports every entry point include/*.h declares
(no GPU needed: only symbol lookup and the argument checks that fail before any HIP call)."""
import ctypes
import os
import re

import pytest

import paper_2104_06165_amd as pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phimvs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("phimvs_create", "phimvs_set_views", "phimvs_patchmatch", "phimvs_eval_cost",
                     "phimvs_step", "phimvs_get_state", "phimvs_set_state", "phimvs_init_planes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pm.LIB_PATH)
    names = _declared()
    assert names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pm.EXPORTS)


def test_default_params_and_null_context_errors():
    p = pm.default_params()
    assert p.top_k == 0 and p.bilateral and p.sigma_color == 12.0 and p.eps_var == 1e-4 and p.seed == 0x5EED
    assert p.tap_radius == 0 and p.lanes == 0 and p.score_all == 0
    L = pm.lib()
    # calls on a null context fail with PHIMVS_E_ARG instead of crashing
    assert L.phimvs_prepare(None, 0, None, 0, 7, 1, None) == -1
    assert L.phimvs_step(None, 1, 0, 1, 1) == -1
    assert L.phimvs_set_views(None, 2, None, None, None, None, None) == -1
    assert L.phimvs_last_error(None) == b"null context"
    out = ctypes.c_void_p()
    rc = L.phimvs_create(ctypes.byref(out), -1, None)
    assert rc in (-3,)  # no such device
    assert L.phimvs_net_param_count() == 9 * 5 * 32 + 32 + 3 * (9 * 32 * 32 + 32) + 9 * 32 * 4 + 4
    assert L.phimvs_net_forward(None, 1, 4, 4, None, None) == -1
    assert L.phimvs_net_adam(None, 1e-3, 0.9, 0.999, 1e-8) == -1
    assert L.phimvs_net_last_error(None) == b"null network"
    assert L.phimvs_net_create(ctypes.byref(out), -1, None) == -3


def test_params_layout_matches_the_header(tmp_path):
    """The binding's phimvs_params mirrors the header's struct field by field (offsets
    and size as the C compiler lays them out)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f[0] for f in pm._Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"phimvs.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(phimvs_params));\n" +
                   "".join(f"  printf(\"%zu\\n\", offsetof(phimvs_params, {f}));\n" for f in fields) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(pm._Params)
    assert got[1:] == [getattr(pm._Params, f).offset for f in fields]
