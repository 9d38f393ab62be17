"""The C ABI without a GPU: the header compiles as C and C++, and the built
library exports every function the header declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pirrt.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pirrt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2003_04920_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2003_04920_amd import build
        build.build()
    return binding.LIB_PATH


def test_header_compiles_as_c_and_cpp(tmp_path):
    src = tmp_path / "use.c"
    src.write_text('#include "pirrt.h"\nint main(void){pirrt_config c; return pirrt_config_init(&c);}\n')
    for compiler, std in (("gcc", "-std=c99"), ("g++", "-std=c++11")):
        subprocess.run([compiler, std, "-fsyntax-only", "-Wall", "-Werror", "-I" + os.path.dirname(HEADER),
                        "-x", "c" if compiler == "gcc" else "c++", str(src)], check=True)


def test_library_exports_every_declared_function(lib_path):
    names = declared()
    assert len(names) >= 14
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2003_04920_amd import binding
    assert sorted(binding.EXPORTS) == names


def test_host_only_entry_points(lib_path):
    from paper_2003_04920_amd import binding
    lib = binding.load()
    assert lib.pirrt_strerror(0) == b"success"
    assert lib.pirrt_strerror(-1) == b"invalid argument"
    cfg = binding.pirrt_config()
    assert lib.pirrt_config_init(ctypes.byref(cfg)) == 0 and cfg.device == -1
    assert lib.pirrt_config_init(None) == -1
    assert lib.pirrt_graph_destroy(None) == 0
    assert lib.pirrt_num_vertices(None) == -1


def test_product_path_has_no_fallback():
    """The binding refuses to run without the built library (no CPU fallback)."""
    from paper_2003_04920_amd import binding
    with pytest.raises(RuntimeError):
        binding.load(os.path.join(ROOT, "does-not-exist", "libpirrt.so"))
    pkg = os.path.join(ROOT, "paper_2003_04920_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "pirrt_oracle" not in text and "liboracle" not in text, f
