"""The C-ABI library builds for gfx950, loads without a GPU and exports every
function that include/inla_dense.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "inla_dense.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(inla_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2311_08050_amd import binding, build
    if not os.path.exists(binding.LIBPATH):
        build.build()
    return binding.LIBPATH


def test_header_declares_the_hot_path_calls():
    f = declared_functions()
    for name in ("inla_logdet", "inla_constrained_mode", "inla_laplace_eval", "inla_marginal_var"):
        assert name in f


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing


def test_binding_export_list_matches_header():
    from paper_2311_08050_amd import binding
    assert sorted(binding.EXPORTS) == declared_functions()


def test_struct_layouts(tmp_path):
    """Every struct the binding passes has the size and field offsets the C
    compiler gives the header's declaration."""
    import subprocess

    from paper_2311_08050_amd import binding
    pairs = [("inla_model", binding.Model), ("inla_opts", binding.Opts), ("inla_result", binding.Result),
             ("inla_kstats", binding.KStats), ("inla_theta_opts", binding.ThetaOpts),
             ("inla_pinv_prior", binding.PinvPriorStruct)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = []
    for _, cls in pairs:
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, fname).offset for fname, _ in cls._fields_]
    assert got == want


def test_version_string(libpath):
    lib = ctypes.CDLL(libpath)
    lib.inla_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.inla_version()


def test_no_oracle_in_product_path():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2311_08050_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn


def _zero_args(params):
    """NULL for every pointer (and callback), zero for every scalar, typed from
    the declaration's parameter list."""
    out = []
    for p in [q.strip() for q in params.split(",") if q.strip() and q.strip() != "void"]:
        if "*" in p or p.split()[0].endswith("_fn"):
            out.append(ctypes.c_void_p(None))
        elif "double" in p:
            out.append(ctypes.c_double(0.0))
        elif "float" in p:
            out.append(ctypes.c_float(0.0))
        elif "int64_t" in p:
            out.append(ctypes.c_int64(0))
        else:
            out.append(ctypes.c_int32(0))
    return out


def test_null_first_argument_is_an_error_not_a_crash(libpath):
    """Every int-returning entry point called with a NULL handle (or network,
    or output handle) and zero sizes returns -1 without touching a device; the
    two destroy calls accept NULL and return 0."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    lib = ctypes.CDLL(libpath)
    seen = 0
    for m in re.finditer(r"\n\s*int\s+(inla_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src):
        name, params = m.group(1), " ".join(m.group(2).split())
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        want = 0 if name in ("inla_destroy", "inla_mlp_destroy") else -1
        assert f(*_zero_args(params)) == want, name
        seen += 1
    assert seen == len(declared_functions()) - 1   # all but inla_version
