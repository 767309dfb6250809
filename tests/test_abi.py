"""The C-ABI library loads and exports every function include/md.h declares
(no compute calls: runs without a GPU).  Also checks the binding's struct
layouts against the header's field lists."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(md_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libmd():
    from paper_1411_3019_amd import build as B
    if B.stale():
        B.build()
    return C.CDLL(B.LIB)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("md_create", "md_set_surface", "md_set_particles", "md_step", "md_get_state",
                     "md_pool_create", "md_pool_admit", "md_pool_run", "md_pool_fetch"):
        assert required in names


def test_every_declared_symbol_is_exported(libmd):
    missing = [n for n in _declared_functions() if not hasattr(libmd, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_1411_3019_amd import md
    assert sorted(md.SYMBOLS) == _declared_functions()


def _struct_fields(name):
    text = open(HEADER).read()
    m = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            tok = part.strip().split()[-1].lstrip("*")
            fields.append(re.sub(r"\[.*\]", "", tok))
    return fields


@pytest.mark.parametrize("cname,pyname", [("md_params", "_Params"), ("md_diag", "_Diag"),
                                          ("md_job_desc", "_JobDesc"), ("md_model", "_Model")])
def test_struct_layout_matches_header(cname, pyname):
    from paper_1411_3019_amd import md
    assert [f for f, _ in getattr(md, pyname)._fields_] == _struct_fields(cname)


def test_struct_sizes_match_the_c_compiler(tmp_path):
    """sizeof of each ABI struct as the host C compiler lays it out equals the
    ctypes structure's size."""
    import shutil
    import subprocess
    from paper_1411_3019_amd import md
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = [("md_params", "_Params"), ("md_diag", "_Diag"), ("md_job_desc", "_JobDesc"), ("md_model", "_Model"),
             ("md_stats", "_Stats")]
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "md.h"\nint main(void) {\n'
                   + "".join(f'  printf("%zu\\n", sizeof({c}));\n' for c, _ in pairs) + "  return 0;\n}\n")
    exe = tmp_path / "sz"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert sizes == [C.sizeof(getattr(md, p)) for _, p in pairs]


def test_strerror_without_gpu(libmd):
    libmd.md_strerror.restype = C.c_char_p
    assert libmd.md_strerror(-4) == b"RATTLE Newton iteration did not converge"
    assert libmd.md_strerror(0) == b"ok"
